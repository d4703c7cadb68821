// Mixed-precision tile Cholesky (paper Section 2.1, Fig. 1(d): off-diagonal
// tiles held in single or half precision, diagonal tiles in double).
//
// Storage: diagonal tiles FP64; off-diagonal tile (i, j) in a 4-byte slot per
// entry, as FP32 (tag 0) or as BF16 in the first half of the slot (tag 1).
// Step k of the factorisation:
//   1. the column-k tiles below the diagonal are widened into an FP64 panel
//      buffer, the panel is factored by the FP64 kernels and written back,
//      rounded to nearest even into each tile's precision;
//   2. diagonal targets A_jj -= A_jk A_jk^T run on FP64 MFMA from the FP64
//      panel buffer (k_chol_update with diag_only);
//   3. off-diagonal targets A_ij -= A_ik A_jk^T run on FP32 MFMA with FP32
//      accumulation; BF16 operands are widened exactly, BF16 targets rounded
//      back to nearest even.
// The solves read the stored tiles and accumulate in FP64; log det Sigma and
// z^T Sigma^-1 z are FP64 sums.
#include <float.h>

#include "common.h"
#include "launch.h"

namespace exg {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float* off32(const TileMat& M, int64_t i, int64_t j) {
  return (float*)M.off + off_index(i, j, M.NT) * M.ts * M.ts;
}

// ---------------------------------------------------------- tile geometry
// box[4 k + 0..3] = min x, max x, min y, max y over the real points of tile k
__global__ __launch_bounds__(256) void k_tile_bbox(const double* __restrict__ xs, const double* __restrict__ ys,
                                                   int64_t ts, int64_t nreal, double* __restrict__ box) {
  __shared__ double red[4][256];
  const int64_t k = blockIdx.x;
  const int t = threadIdx.x;
  double a = DBL_MAX, b = -DBL_MAX, c = DBL_MAX, d = -DBL_MAX;
  for (int64_t q = t; q < ts; q += 256) {
    const int64_t g = k * ts + q;
    if (g >= nreal) break;
    a = fmin(a, xs[g]);
    b = fmax(b, xs[g]);
    c = fmin(c, ys[g]);
    d = fmax(d, ys[g]);
  }
  red[0][t] = a;
  red[1][t] = b;
  red[2][t] = c;
  red[3][t] = d;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      red[0][t] = fmin(red[0][t], red[0][t + s]);
      red[1][t] = fmax(red[1][t], red[1][t + s]);
      red[2][t] = fmin(red[2][t], red[2][t + s]);
      red[3][t] = fmax(red[3][t], red[3][t + s]);
    }
    __syncthreads();
  }
  if (t < 4) box[4 * k + t] = red[t][0];
}

// --------------------------------------------------------- panel staging
// pbuf tile q = tile (k + 1 + q, k) widened to FP64
__global__ void k_panel_gather(TileMat M, int64_t k, const uint8_t* __restrict__ tag, double* __restrict__ pbuf,
                               int64_t count) {
  const int64_t tt = M.ts * M.ts;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count * tt) return;
  const int64_t q = e / tt, o = e % tt;
  const int64_t idx = off_index(k + 1 + q, k, M.NT);
  const float* src = (const float*)M.off + idx * tt;
  pbuf[e] = tag[idx] ? (double)bf16_to_f32(((const uint16_t*)src)[o]) : (double)src[o];
}

// tile (k + 1 + q, k) = pbuf tile q rounded to nearest even in its precision
__global__ void k_panel_scatter(TileMat M, int64_t k, const uint8_t* __restrict__ tag, const double* __restrict__ pbuf,
                                int64_t count) {
  const int64_t tt = M.ts * M.ts;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count * tt) return;
  const int64_t q = e / tt, o = e % tt;
  const int64_t idx = off_index(k + 1 + q, k, M.NT);
  float* dst = (float*)M.off + idx * tt;
  const float f = (float)pbuf[e];
  if (tag[idx])
    ((uint16_t*)dst)[o] = f32_to_bf16(f);
  else
    dst[o] = f;
}

// ------------------------------------------------ FP32 MFMA trailing update
constexpr int FBK = 32;        // k-depth of one LDS stage
constexpr int FLDP = BLK + 4;  // padded LDS row (floats)
constexpr int FLDS = 2 * 2 * FBK * FLDP;

__device__ __forceinline__ v4f mfma32(float x, float y, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
}

// C_ij -= A_ik A_jk^T for the off-diagonal targets k < j < i < NT.
// v_mfma_f32_16x16x4f32: operand X lane l holds X[l % 16][l / 16], operand Y
// holds Y[l / 16][l % 16], D = X Y has lane l, register r at D[4 (l/16) + r][l % 16].
__global__ __launch_bounds__(256, 2) void k_update_lp(TileMat M, const uint8_t* __restrict__ tag, int T, int64_t k,
                                                      int64_t nreal, int64_t nb) {
  __shared__ float sm[FLDS];
  const int64_t ts = M.ts, tt = ts * ts;
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const int64_t p = b / (T * T);
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  int64_t a, c;
  tri_decode(p, &a, &c);  // c <= a
  const int64_t i = k + 2 + a, j = k + 1 + c;
  if (i * ts + u * BLK >= nreal) return;  // padded rows: update is zero
  const int64_t ia = off_index(i, k, M.NT), ib = off_index(j, k, M.NT), ic = off_index(i, j, M.NT);
  const bool abf = tag[ia] != 0, bbf = tag[ib] != 0, cbf = tag[ic] != 0;
  const float* A = (const float*)M.off + ia * tt;
  const float* B = (const float*)M.off + ib * tt;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wr = w >> 1, wc = w & 1;
  float* sA = sm;
  float* sB = sm + 2 * FBK * FLDP;
  // raw 16-byte chunks of a stage: FP32 tiles use 4 chunks of 4 values per
  // thread, BF16 tiles 2 chunks of 8 values
  u4 ra0[4], rb0[4], ra1[4], rb1[4];
  auto gl = [&](const float* X, bool bf, int rowoff, int k0, u4 (&r)[4]) {
    if (!bf) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int idx = t + 256 * s, kk = idx >> 5, m4 = idx & 31;
        r[s] = *(const u4*)(X + rowoff + 4 * m4 + (int64_t)(k0 + kk) * ts);
      }
    } else {
      const uint16_t* Xh = (const uint16_t*)X;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int idx = t + 256 * s, kk = idx >> 4, m8 = idx & 15;
        r[s] = *(const u4*)(Xh + rowoff + 8 * m8 + (int64_t)(k0 + kk) * ts);
      }
    }
  };
  auto st = [&](float* S, bool bf, u4 (&r)[4]) {
    if (!bf) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int idx = t + 256 * s, kk = idx >> 5, m4 = idx & 31;
        *(u4*)(S + kk * FLDP + 4 * m4) = r[s];
      }
    } else {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int idx = t + 256 * s, kk = idx >> 4, m8 = idx & 15;
        u4 lo, hi;
        lo.x = r[s].x << 16;
        lo.y = r[s].x & 0xffff0000u;
        lo.z = r[s].y << 16;
        lo.w = r[s].y & 0xffff0000u;
        hi.x = r[s].z << 16;
        hi.y = r[s].z & 0xffff0000u;
        hi.z = r[s].w << 16;
        hi.w = r[s].w & 0xffff0000u;
        *(u4*)(S + kk * FLDP + 8 * m8) = lo;
        *(u4*)(S + kk * FLDP + 8 * m8 + 4) = hi;
      }
    }
  };
  v4f acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = (v4f){0.f, 0.f, 0.f, 0.f};
  auto compute = [&](int cur) {
    const float* sa = sA + cur * FBK * FLDP + wr * 64 + (lane & 15);
    const float* sb = sB + cur * FBK * FLDP + wc * 64 + (lane & 15);
#pragma unroll
    for (int kk = 0; kk < FBK; kk += 4) {
      const int ko = (kk + (lane >> 4)) * FLDP;
      float af[4], bf[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) af[x] = sa[ko + 16 * x];
#pragma unroll
      for (int y = 0; y < 4; ++y) bf[y] = sb[ko + 16 * y];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = mfma32(bf[y], af[x], acc[x][y]);
    }
  };
  const int ra = u * BLK, rb = v * BLK;
  const int nst = (int)(ts / FBK);  // even
  gl(A, abf, ra, 0, ra0);
  gl(B, bbf, rb, 0, rb0);
  gl(A, abf, ra, FBK, ra1);
  gl(B, bbf, rb, FBK, rb1);
  st(sA, abf, ra0);
  st(sB, bbf, rb0);
  __syncthreads();
  for (int s = 0; s < nst; s += 2) {
    if (s + 2 < nst) {
      gl(A, abf, ra, (s + 2) * FBK, ra0);
      gl(B, bbf, rb, (s + 2) * FBK, rb0);
    }
    compute(0);
    st(sA + FBK * FLDP, abf, ra1);
    st(sB + FBK * FLDP, bbf, rb1);
    __syncthreads();
    if (s + 3 < nst) {
      gl(A, abf, ra, (s + 3) * FBK, ra1);
      gl(B, bbf, rb, (s + 3) * FBK, rb1);
    }
    compute(1);
    if (s + 2 < nst) {
      st(sA, abf, ra0);
      st(sB, bbf, rb0);
    }
    __syncthreads();
  }
  // C(m, n) -= acc: m = wr*64 + 16x + (lane & 15), n = wc*64 + 16y + 4 (lane >> 4) + r
  float* C = (float*)M.off + ic * tt + u * BLK + (int64_t)v * BLK * ts;
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int m = wr * 64 + 16 * x + (lane & 15);
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = wc * 64 + 16 * y + 4 * (lane >> 4) + r;
        const int64_t o = m + (int64_t)n * ts;
        if (!cbf) {
          C[o] -= acc[x][y][r];
        } else {
          uint16_t* Ch = (uint16_t*)C;
          Ch[o] = f32_to_bf16(bf16_to_f32(Ch[o]) - acc[x][y][r]);
        }
      }
  }
}

// ------------------------------------------------- solves on mixed tiles
// rhs_i -= L_ik y_k for the 128-row blocks g0 <= g < gmax below tile k
__global__ __launch_bounds__(256) void k_gemv_fwd_lp(TileMat M, const uint8_t* __restrict__ tag, int64_t k,
                                                     int64_t g0, const double* __restrict__ yk,
                                                     double* __restrict__ rhs) {
  extern __shared__ double sy[];  // ts + 256
  const int64_t ts = M.ts;
  double* red = sy + ts;
  const int T = (int)(ts / BLK);
  const int64_t g = g0 + blockIdx.x;
  const int64_t i = g / T;
  const int u = (int)(g % T);
  const int t = threadIdx.x;
  for (int q = t; q < ts; q += 256) sy[q] = yk[q];
  __syncthreads();
  const int64_t idx = off_index(i, k, M.NT);
  const float* L = (const float*)M.off + idx * ts * ts;
  const int r = t & 127, h = t >> 7;
  double s = 0.0;
  if (tag[idx]) {
    const uint16_t* Lh = (const uint16_t*)L + u * BLK + r;
    for (int64_t q = h; q < ts; q += 2) s += (double)bf16_to_f32(Lh[q * ts]) * sy[q];
  } else {
    const float* Lf = L + u * BLK + r;
    for (int64_t q = h; q < ts; q += 2) s += (double)Lf[q * ts] * sy[q];
  }
  red[t] = s;
  __syncthreads();
  if (h == 0) rhs[i * ts + u * BLK + r] -= red[r] + red[r + 128];
}

// ---------------------------------------------------------------- launchers
void launch_tile_bbox(const double* xs, const double* ys, int64_t ts, int64_t NT, int64_t nreal, double* box,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_tile_bbox, dim3((unsigned)NT), dim3(256), 0, s, xs, ys, ts, nreal, box);
}

void launch_panel_gather(const TileMat& M, int64_t k, const uint8_t* tag, double* pbuf, hipStream_t s) {
  const int64_t count = M.NT - k - 1;
  if (count <= 0) return;
  const int64_t n = count * M.ts * M.ts;
  hipLaunchKernelGGL(k_panel_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, M, k, tag, pbuf, count);
}

void launch_panel_scatter(const TileMat& M, int64_t k, const uint8_t* tag, const double* pbuf, hipStream_t s) {
  const int64_t count = M.NT - k - 1;
  if (count <= 0) return;
  const int64_t n = count * M.ts * M.ts;
  hipLaunchKernelGGL(k_panel_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, M, k, tag, pbuf, count);
}

void launch_update_lp(const TileMat& M, const uint8_t* tag, int64_t k, int64_t nreal, hipStream_t s) {
  const int T = (int)(M.ts / BLK);
  const int64_t m = M.NT - k - 2;  // strictly-lower pairs among the m + 1 trailing tiles
  if (m <= 0) return;
  const int64_t nblk = m * (m + 1) / 2 * T * T;
  hipLaunchKernelGGL(k_update_lp, dim3((unsigned)nblk), dim3(256), 0, s, M, tag, T, k, nreal, nblk);
}

void launch_trsv_fwd_lp(const TileMat& M, const uint8_t* tag, const double* Xd, int64_t nreal, double* rhs,
                        double* y, hipStream_t s) {
  const int64_t ts = M.ts, NT = M.NT;
  const int T = (int)(ts / BLK);
  const size_t shm = (size_t)(ts + 256) * sizeof(double);
  const int64_t gmax = (nreal + BLK - 1) / BLK;
  for (int64_t k = 0; k < NT; ++k) {
    launch_diag_apply_n(Xd + k * ts * ts, ts, rhs + k * ts, y + k * ts, s);
    const int64_t g0 = (k + 1) * T;
    if (gmax > g0)
      hipLaunchKernelGGL(k_gemv_fwd_lp, dim3((unsigned)(gmax - g0)), dim3(256), shm, s, M, tag, k, g0, y + k * ts,
                         rhs);
  }
}

}  // namespace exg
