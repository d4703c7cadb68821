// Mixed-precision tile Cholesky (paper Section 2.1, Fig. 1(d): off-diagonal
// tiles held in single or half precision, diagonal tiles in double).
//
// Storage: diagonal tiles FP64; off-diagonal tile (i, j) in a 4-byte slot per
// entry, as FP32 (tag 0) or as BF16 in the first half of the slot (tag 1).
// Step k of the factorisation:
//   1. the column-k tiles below the diagonal are widened into an FP64 panel
//      buffer, the panel is factored by the FP64 kernels and written back,
//      rounded to nearest even into each tile's precision and, for the
//      update, to FP32 in a panel copy;
//   2. diagonal targets A_jj -= A_jk A_jk^T run on FP64 MFMA from the FP64
//      panel buffer (k_chol_update with diag_only);
//   3. off-diagonal targets A_ij -= A_ik A_jk^T run on FP32 MFMA with FP32
//      accumulation from the FP32 panel copy; BF16 targets are widened
//      exactly and rounded back to nearest even.
// The solves read the stored tiles and accumulate in FP64; log det Sigma and
// z^T Sigma^-1 z are FP64 sums.
#include <float.h>

#include "common.h"
#include "launch.h"

namespace exg {


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

// tile (k + 1 + q, k) = pbuf tile q rounded to nearest even in its precision;
// p32 tile q = pbuf tile q rounded to FP32 (the operands of the FP32 update)
__global__ void k_panel_scatter(TileMat M, int64_t k, const uint8_t* __restrict__ tag, const double* __restrict__ pbuf,
                                float* __restrict__ p32, int64_t count) {
  const int64_t tt = M.ts * M.ts;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count * tt) return;
  const int64_t q = e / tt, o = e % tt;
  const int64_t idx = off_index(k + 1 + q, k, M.NT);
  float* dst = (float*)M.off + idx * tt;
  const float f = (float)pbuf[e];
  p32[e] = f;
  if (tag[idx])
    ((uint16_t*)dst)[o] = f32_to_bf16(f);
  else
    dst[o] = f;
}

// ------------------------------------------------ FP32 MFMA trailing update
constexpr int FBK = 16;        // k-depth of one LDS stage
constexpr int FLDP = BLK + 4;  // padded LDS row (floats)
constexpr int FLDS = 2 * 2 * FBK * FLDP;

typedef float v16f __attribute__((ext_vector_type(16)));

__device__ __forceinline__ v16f mfma32x32(float x, float y, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, c, 0, 0, 0);
}

// C_ij -= L_ik L_jk^T for the off-diagonal targets k < j < i < NT, with the
// operands taken from the FP32 rounding of the FP64 panel (p32 tile q holds
// L_{k+1+q, k}), so that a BF16-stored panel tile never feeds its rounding
// error into targets near the diagonal.  One 256-thread block computes one
// 128 x 128 block of a target tile; wave (wr, wc) owns its 64 x 64 quarter as
// 2 x 2 products on v_mfma_f32_32x32x2f32.  That instruction takes operand X
// lane l as X[l % 32][l / 32] and Y lane l as Y[l / 32][l % 32]; D = X Y has
// lane l, register r at D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
__global__ __launch_bounds__(256, 2) void k_update_lp(TileMat M, const uint8_t* __restrict__ tag,
                                                      const float* __restrict__ p32, int T, int64_t k,
                                                      int64_t nreal, int64_t nb, int mode, int64_t off) {
  __shared__ float sm[FLDS];
  const int64_t ts = M.ts, tt = ts * ts;
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const int64_t p = b / (T * T);
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  int64_t a, c;
  pair_map(mode, off, p, &a, &c);  // c <= a
  const int64_t i = k + 2 + a, j = k + 1 + c;
  if (i * ts + u * BLK >= nreal) return;  // padded rows: update is zero
  const float* A = p32 + (a + 1) * tt + u * BLK;
  const float* B = p32 + c * tt + v * BLK;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wr = w >> 1, wc = w & 1;
  typedef float f4 __attribute__((ext_vector_type(4)));
  constexpr int NL = FBK * BLK / 4 / 256;  // float4 loads per thread per operand and stage
  f4 ra0[NL], rb0[NL], ra1[NL], rb1[NL];
  float* sA = sm;
  float* sB = sm + 2 * FBK * FLDP;
  auto gload = [&](int k0, f4 (&ra)[NL], f4 (&rb)[NL]) {
#pragma unroll
    for (int s = 0; s < NL; ++s) {
      const int idx = t + 256 * s, kk = idx >> 5, m4 = idx & 31;
      ra[s] = *(const f4*)(A + 4 * m4 + (int64_t)(k0 + kk) * ts);
      rb[s] = *(const f4*)(B + 4 * m4 + (int64_t)(k0 + kk) * ts);
    }
  };
  auto sstore = [&](int buf, f4 (&ra)[NL], f4 (&rb)[NL]) {
#pragma unroll
    for (int s = 0; s < NL; ++s) {
      const int idx = t + 256 * s, kk = idx >> 5, m4 = idx & 31;
      *(f4*)(sA + buf * FBK * FLDP + kk * FLDP + 4 * m4) = ra[s];
      *(f4*)(sB + buf * FBK * FLDP + kk * FLDP + 4 * m4) = rb[s];
    }
  };
  v16f acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[x][y][r] = 0.f;
  auto compute = [&](int cur) {
    const float* sa = sA + cur * FBK * FLDP + wr * 64 + (lane & 31);
    const float* sb = sB + cur * FBK * FLDP + wc * 64 + (lane & 31);
#pragma unroll
    for (int kk = 0; kk < FBK; kk += 2) {
      const int ko = (kk + (lane >> 5)) * FLDP;
      float af[2], bf[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) af[x] = sa[ko + 32 * x];
#pragma unroll
      for (int y = 0; y < 2; ++y) bf[y] = sb[ko + 32 * y];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = mfma32x32(bf[y], af[x], acc[x][y]);
    }
  };
  // global loads run two stages ahead of the MFMAs (two register sets)
  const int nst = (int)(ts / FBK);  // even
  gload(0, ra0, rb0);
  gload(FBK, ra1, rb1);
  sstore(0, ra0, rb0);
  __syncthreads();
  for (int s = 0; s < nst; s += 2) {
    if (s + 2 < nst) gload((s + 2) * FBK, ra0, rb0);
    compute(0);
    sstore(1, ra1, rb1);
    __syncthreads();
    if (s + 3 < nst) gload((s + 3) * FBK, ra1, rb1);
    compute(1);
    if (s + 2 < nst) sstore(0, ra0, rb0);
    __syncthreads();
  }
  // C(m, n) -= acc: m = wr*64 + 32x + lane % 32, n = wc*64 + 32y + 8 (r/4) + 4 (lane/32) + r % 4
  const int64_t ic = off_index(i, j, M.NT);
  const bool cbf = tag[ic] != 0;
  float* C = (float*)M.off + ic * tt + u * BLK + (int64_t)v * BLK * ts;
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int m = wr * 64 + 32 * x + (lane & 31);
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int n = wc * 64 + 32 * y + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
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

void launch_panel_scatter(const TileMat& M, int64_t k, const uint8_t* tag, const double* pbuf, float* p32,
                          hipStream_t s) {
  const int64_t count = M.NT - k - 1;
  if (count <= 0) return;
  const int64_t n = count * M.ts * M.ts;
  hipLaunchKernelGGL(k_panel_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, M, k, tag, pbuf, p32,
                     count);
}

void launch_update_lp(const TileMat& M, const uint8_t* tag, const float* p32, int64_t k, int64_t nreal, int part,
                      hipStream_t s) {
  const int T = (int)(M.ts / BLK);
  const int64_t m = M.NT - k - 2;  // strictly-lower pairs among the m + 1 trailing tiles
  if (m <= 0) return;
  int mode = PAIRS_TRI;
  int64_t off = 0, npairs = m * (m + 1) / 2;
  if (part == UPD_FIRST_COLUMN) {
    mode = PAIRS_COL, npairs = m;
  } else if (part == UPD_REST) {
    off = 1, npairs = (m - 1) * m / 2;
  }
  if (npairs <= 0) return;
  const int64_t nblk = npairs * T * T;
  hipLaunchKernelGGL(k_update_lp, dim3((unsigned)nblk), dim3(256), 0, s, M, tag, p32, T, k, nreal, nblk, mode, off);
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
