// Latency-bound pieces of the likelihood path:
//   * location ordering (bounding box, Morton keys, bitonic sort, gather);
//   * Cholesky + inverse of one 128 x 128 diagonal block held in LDS;
//   * the tile-by-tile forward and backward triangular solves;
//   * deterministic reductions for log det Sigma, z^T Sigma^-1 z, l(theta) and
//     the gradient partial sums;
//   * small fills and copies.
#include <float.h>

#include "common.h"
#include "launch.h"

namespace exg {

// ------------------------------------------------------------------ ordering
// box[0..3] = min x, max x, min y, max y; box[4] = number of non-finite
// values among x, y (and z when given)
__global__ __launch_bounds__(1024) void k_bbox(const double* __restrict__ x, const double* __restrict__ y,
                                               const double* __restrict__ z, int64_t n, double* __restrict__ box) {
  __shared__ double red[5][1024];
  double mnx = DBL_MAX, mxx = -DBL_MAX, mny = DBL_MAX, mxy = -DBL_MAX, bad = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double a = x[i], b = y[i];
    const double c = z ? z[i] : 0.0;
    if (!(fabs(a) <= DBL_MAX) || !(fabs(b) <= DBL_MAX) || !(fabs(c) <= DBL_MAX)) bad += 1.0;
    mnx = fmin(mnx, a);
    mxx = fmax(mxx, a);
    mny = fmin(mny, b);
    mxy = fmax(mxy, b);
  }
  const int t = threadIdx.x;
  red[0][t] = mnx;
  red[1][t] = mxx;
  red[2][t] = mny;
  red[3][t] = mxy;
  red[4][t] = bad;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (t < s) {
      red[0][t] = fmin(red[0][t], red[0][t + s]);
      red[1][t] = fmax(red[1][t], red[1][t + s]);
      red[2][t] = fmin(red[2][t], red[2][t + s]);
      red[3][t] = fmax(red[3][t], red[3][t + s]);
      red[4][t] += red[4][t + s];
    }
    __syncthreads();
  }
  if (t < 5) box[t] = red[t][0];
}

__device__ __forceinline__ uint32_t spread16(uint32_t v) {
  v &= 0xffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

// key = Morton code of the 16-bit quantised location (high 32 bits) and the
// caller index (low 32 bits), so keys are distinct and the order is unique.
__global__ void k_morton(const double* __restrict__ x, const double* __restrict__ y, int64_t n, int64_t P,
                         const double* __restrict__ box, uint64_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  if (i >= n) {
    keys[i] = ~(uint64_t)0;
    return;
  }
  const double wx = box[1] - box[0], wy = box[3] - box[2];
  const double sx = wx > 0 ? 65535.999 / wx : 0.0, sy = wy > 0 ? 65535.999 / wy : 0.0;
  const uint32_t qx = (uint32_t)((x[i] - box[0]) * sx), qy = (uint32_t)((y[i] - box[2]) * sy);
  const uint32_t code = spread16(qx) | (spread16(qy) << 1);
  keys[i] = ((uint64_t)code << 32) | (uint64_t)i;
}

// one compare-exchange step of the bitonic network over the whole array
__global__ void k_bitonic_global(uint64_t* __restrict__ keys, int64_t P, int64_t j, int64_t k) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const int64_t l = i ^ j;
  if (l <= i) return;
  const uint64_t a = keys[i], b = keys[l];
  const bool up = (i & k) == 0;
  if ((a > b) == up) {
    keys[i] = b;
    keys[l] = a;
  }
}

// the steps j = jmax..1 of stage k on chunks of 2048 keys in LDS; with
// kfrom = 2 it runs every stage k <= 2048 (a full sort of each chunk)
__global__ __launch_bounds__(1024) void k_bitonic_local(uint64_t* __restrict__ keys, int64_t kfrom, int64_t kto,
                                                         int64_t jmax) {
  __shared__ uint64_t s[2048];
  const int64_t base = (int64_t)blockIdx.x * 2048;
  const int t = threadIdx.x;
  s[t] = keys[base + t];
  s[t + 1024] = keys[base + t + 1024];
  __syncthreads();
  for (int64_t k = kfrom; k <= kto; k <<= 1) {
    for (int64_t j = (k == kfrom ? jmax : k >> 1); j > 0; j >>= 1) {
      // thread t handles the pair (i, i ^ j) with i having bit j clear
      const int64_t lo = ((t / j) * 2 * j) + (t % j);
      const int64_t hi = lo + j;
      const bool up = ((base + lo) & k) == 0;
      const uint64_t a = s[lo], b = s[hi];
      if ((a > b) == up) {
        s[lo] = b;
        s[hi] = a;
      }
      __syncthreads();
    }
  }
  keys[base + t] = s[t];
  keys[base + t + 1024] = s[t + 1024];
}

// sorted, zero-padded copies of x, y, z and the permutation (sorted -> caller)
__global__ void k_gather(const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
                         int64_t n, int64_t npad, const uint64_t* __restrict__ keys, double* __restrict__ xs,
                         double* __restrict__ ys, double* __restrict__ zs, int32_t* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  if (i < n) {
    const int64_t src = (int64_t)(keys[i] & 0xffffffffu);
    perm[i] = (int32_t)src;
    xs[i] = x[src];
    ys[i] = y[src];
    if (zs) zs[i] = z ? z[src] : 0.0;
  } else {
    perm[i] = -1;
    xs[i] = 0.0;
    ys[i] = 0.0;
    if (zs) zs[i] = 0.0;
  }
}

// out[perm[i]] = v[i] for i < n
__global__ void k_scatter(const double* __restrict__ v, const int32_t* __restrict__ perm, int64_t n,
                          double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[perm[i]] = v[i];
}

// ------------------------------------------------ diagonal 128-block factor
// Cholesky of one 128 x 128 block and the inverse of its factor, in LDS.
//   factor (right-looking, one barrier per column): at step j every thread
//   reads d = S_jj, updates S_cr -= S_jr S_jc / d for j < c <= r, and writes
//   L_rj = S_jr / sqrt(d) into the free upper slot (column r, row j).
//   inverse: X = L^-1 by rows, T_ij -= (L_im / L_mm) T_mj for i > m >= j with
//   unit T_mm, then X_ij = T_ij / L_ii (one barrier per row).
// Writes L (zeros above the diagonal) over the block, X to dinv (ld 128), the
// block's sum of 2 ln L_jj to *ldpart and the first failing global column
// (1-based) to *info with an atomic minimum.
__global__ __launch_bounds__(1024) void k_potrf_blk(double* __restrict__ A, int64_t lda, double* __restrict__ dinv,
                                                    double* __restrict__ ldpart, unsigned long long* __restrict__ info,
                                                    int64_t col0) {
  __shared__ double S[BLK * (BLK + 1)];
  __shared__ double dg[BLK];
  constexpr int P = BLK + 1;
  const int t = threadIdx.x;
  for (int e = t; e < BLK * BLK; e += 1024) {
    const int c = e >> 7, r = e & 127;
    if (r >= c) S[c * P + r] = A[r + (int64_t)c * lda];
  }
  __syncthreads();
  const int r = t & 127, g = t >> 7;
  for (int j = 0; j < BLK; ++j) {
    const double d = S[j * P + j];
    const double sd = sqrt(d);
    if (t == 0) {
      dg[j] = sd;
      if (!(d > 0.0) || !(d <= DBL_MAX)) atomicMin(info, (unsigned long long)(col0 + j + 1));
    }
    if (r > j) {
      const double sjr = S[j * P + r];
      if (g == 0) S[r * P + j] = sjr / sd;
      const double f = sjr / d;
      for (int c = j + 1 + g; c <= r; c += 8) S[c * P + r] -= f * S[j * P + c];
    }
    __syncthreads();
  }
  // inverse: strictly lower part of S holds T, initialised to 0
  for (int e = t; e < BLK * BLK; e += 1024) {
    const int c = e >> 7, rr = e & 127;
    if (rr > c) S[c * P + rr] = 0.0;
  }
  __syncthreads();
  for (int m = 0; m < BLK - 1; ++m) {
    if (r > m) {
      const double lim = S[r * P + m] / dg[m];
      for (int j = g; j <= m; j += 8) {
        const double tmj = (j == m) ? 1.0 : S[j * P + m];
        S[j * P + r] -= lim * tmj;
      }
    }
    __syncthreads();
  }
  for (int e = t; e < BLK * BLK; e += 1024) {
    const int c = e >> 7, rr = e & 127;
    double lv, xv;
    if (rr > c) {
      lv = S[rr * P + c];
      xv = S[c * P + rr] / dg[rr];
    } else if (rr == c) {
      lv = dg[rr];
      xv = 1.0 / dg[rr];
    } else {
      lv = 0.0;
      xv = 0.0;
    }
    A[rr + (int64_t)c * lda] = lv;
    dinv[rr + c * BLK] = xv;
  }
  if (t == 0) {
    double s = 0.0;
    for (int j = 0; j < BLK; ++j) s += 2.0 * log(dg[j]);
    *ldpart = s;
  }
}

// ------------------------------------------------------- triangular solves
// y_k = L_kk^-1 b_k on one diagonal tile, b_k = yv[k ts .. k ts + ts) on entry.
// Block c: y_c = Dinv_c b_c, then b_c' -= L_kk[c', c] y_c for c' > c.
__global__ __launch_bounds__(256) void k_trsv_fwd_diag(const double* __restrict__ Lkk, int64_t ts,
                                                       const double* __restrict__ dinv, double* __restrict__ yk) {
  extern __shared__ double sb[];  // ts doubles + 256 scratch
  double* red = sb + ts;
  const int t = threadIdx.x, T = (int)(ts / BLK);
  for (int i = t; i < ts; i += 256) sb[i] = yk[i];
  __syncthreads();
  const int r = t & 127, h = t >> 7;
  for (int c = 0; c < T; ++c) {
    const double* D = dinv + (int64_t)c * BLK * BLK;
    double s = 0.0;
    for (int k = h; k < BLK; k += 2) s += D[r + k * BLK] * sb[c * BLK + k];
    red[t] = s;
    __syncthreads();
    if (h == 0) sb[c * BLK + r] = red[r] + red[r + 128];
    __syncthreads();
    // rows below block c inside this tile
    for (int64_t row = (int64_t)(c + 1) * BLK + t; row < ts; row += 256) {
      double a = 0.0;
      const double* Lc = Lkk + row + (int64_t)c * BLK * ts;
      for (int k = 0; k < BLK; ++k) a += Lc[(int64_t)k * ts] * sb[c * BLK + k];
      sb[row] -= a;
    }
    __syncthreads();
  }
  for (int i = t; i < ts; i += 256) yk[i] = sb[i];
}

// yv_i -= L_ik y_k for the 128-row blocks g0 <= g < g1 below tile k.
__global__ __launch_bounds__(256) void k_gemv_fwd(const double* __restrict__ tiles, int64_t ts, int64_t k,
                                                  int64_t g0, double* __restrict__ yv) {
  extern __shared__ double sy[];  // ts + 256
  double* red = sy + ts;
  const int T = (int)(ts / BLK);
  const int64_t g = g0 + blockIdx.x;
  const int64_t i = g / T;
  const int u = (int)(g % T);
  const int t = threadIdx.x;
  for (int q = t; q < ts; q += 256) sy[q] = yv[k * ts + q];
  __syncthreads();
  const double* L = tiles + (tri(i) + k) * ts * ts + u * BLK;
  const int r = t & 127, h = t >> 7;
  double s = 0.0;
  for (int64_t q = h; q < ts; q += 2) s += L[r + q * ts] * sy[q];
  red[t] = s;
  __syncthreads();
  if (h == 0) yv[i * ts + u * BLK + r] -= red[r] + red[r + 128];
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// rhs_j -= L_kj^T a_k for the 128-column blocks c0 <= c < c1 (columns of tiles j < k).
__global__ __launch_bounds__(256) void k_gemv_bwd(const double* __restrict__ tiles, int64_t ts, int64_t k,
                                                  const double* __restrict__ ak, double* __restrict__ rhs) {
  const int T = (int)(ts / BLK);
  const int64_t cb = blockIdx.x;  // column block over tiles j < k
  const int64_t j = cb / T;
  const int v = (int)(cb % T);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double* L = tiles + (tri(k) + j) * ts * ts;
  for (int n = w; n < BLK; n += 4) {
    const int64_t col = (int64_t)v * BLK + n;
    const double* Lc = L + col * ts;
    double s = 0.0;
    for (int64_t r = lane; r < ts; r += 64) s += Lc[r] * ak[r];
    s = wave_sum(s);
    if (lane == 0) rhs[j * ts + col] -= s;
  }
}

// a_k = L_kk^-T b_k on one diagonal tile, b_k = rhs[k ts ..) on entry, result in place.
// Block c descending: a_c = Dinv_c^T b_c, then b_c' -= L_kk[c, c']^T a_c for c' < c.
__global__ __launch_bounds__(256) void k_trsv_bwd_diag(const double* __restrict__ Lkk, int64_t ts,
                                                       const double* __restrict__ dinv, double* __restrict__ bk) {
  extern __shared__ double sb[];  // ts
  const int t = threadIdx.x, T = (int)(ts / BLK);
  const int lane = t & 63, w = t >> 6;
  for (int i = t; i < ts; i += 256) sb[i] = bk[i];
  __syncthreads();
  for (int c = T - 1; c >= 0; --c) {
    const double* D = dinv + (int64_t)c * BLK * BLK;
    // a_c[n] = sum_k D[k, n] b_c[k]: column n of D
    double outv[BLK / 4];
#pragma unroll
    for (int q = 0; q < BLK / 4; ++q) {
      const int n = w + 4 * q;
      double s = 0.0;
      for (int kk = lane; kk < BLK; kk += 64) s += D[kk + n * BLK] * sb[c * BLK + kk];
      outv[q] = wave_sum(s);
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < BLK / 4; ++q) sb[c * BLK + w + 4 * q] = outv[q];
    }
    __syncthreads();
    // b_c'[n] -= sum_r L(c*128 + r, c'*128 + n) a_c[r] for columns before block c
    for (int64_t col = w; col < (int64_t)c * BLK; col += 4) {
      const double* Lc = Lkk + (int64_t)c * BLK + col * ts;
      double s = 0.0;
      for (int rr = lane; rr < BLK; rr += 64) s += Lc[rr] * sb[c * BLK + rr];
      s = wave_sum(s);
      if (lane == 0) sb[col] -= s;
    }
    __syncthreads();
  }
  for (int i = t; i < ts; i += 256) bk[i] = sb[i];
}


// w = L e on the lower tiles (diagonal tiles read below their diagonal only);
// one 128-row block per workgroup
__global__ __launch_bounds__(256) void k_trmv_lower(const double* __restrict__ tiles, int64_t ts,
                                                    const double* __restrict__ e, double* __restrict__ w) {
  __shared__ double red[256];
  const int T = (int)(ts / BLK);
  const int64_t g = blockIdx.x;
  const int64_t i = g / T;
  const int u = (int)(g % T);
  const int t = threadIdx.x, r = t & 127, h = t >> 7;
  const int64_t row = u * BLK + r;
  double s = 0.0;
  for (int64_t j = 0; j <= i; ++j) {
    const double* L = tiles + (tri(i) + j) * ts * ts + row;
    const double* ej = e + j * ts;
    const int64_t qmax = (j == i) ? row : ts - 1;
    for (int64_t q = h; q <= qmax; q += 2) s += L[q * ts] * ej[q];
  }
  red[t] = s;
  __syncthreads();
  if (h == 0) w[i * ts + row] = red[r] + red[r + 128];
}

// ------------------------------------------------------------- reductions
// out[0] = l, out[1] = log det, out[2] = y^T y  (eq. 2 with the true n)
__global__ __launch_bounds__(256) void k_finalize_loglik(const double* __restrict__ yv, int64_t n,
                                                         const double* __restrict__ ldpart, int64_t nld,
                                                         double* __restrict__ out) {
  __shared__ double red[2 * 256];
  double v[2] = {0.0, 0.0};
  for (int64_t i = threadIdx.x; i < n; i += 256) v[0] += yv[i] * yv[i];
  for (int64_t i = threadIdx.x; i < nld; i += 256) v[1] += ldpart[i];
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    const double q = v[0], ld = v[1];
    out[0] = -0.5 * ((double)n * 1.8378770664093454836 + ld + q);
    out[1] = ld;
    out[2] = q;
  }
}

// out[0..2] = sum over parts of part[3 p + k]
__global__ __launch_bounds__(256) void k_finalize_grad(const double* __restrict__ part, int64_t nparts,
                                                       double* __restrict__ out) {
  __shared__ double red[3 * 256];
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t p = threadIdx.x; p < nparts; p += 256) {
    v[0] += part[3 * p];
    v[1] += part[3 * p + 1];
    v[2] += part[3 * p + 2];
  }
  block_sum<3>(v, red);
  if (threadIdx.x == 0) {
    out[0] = v[0];
    out[1] = v[1];
    out[2] = v[2];
  }
}

// ------------------------------------------------------------ fills/copies
__global__ void k_fill_u64(unsigned long long* p, unsigned long long v) { *p = v; }

__global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_copy_f64(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// dst[k] = lower part of diagonal tile k (zeros above the diagonal), k < NT
__global__ void k_copy_diag_lower(double* __restrict__ dst, const double* __restrict__ tiles, int64_t ts, int64_t NT) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tt = ts * ts;
  if (e >= NT * tt) return;
  const int64_t k = e / tt, q = e % tt;
  const int64_t r = q % ts, c = q / ts;
  dst[e] = (r >= c) ? tiles[(tri(k) + k) * tt + q] : 0.0;
}

// dst[k] block (c, c) = dinv[k][c] for every diagonal tile k
__global__ void k_put_dinv(double* __restrict__ dst, const double* __restrict__ dinv, int64_t ts, int64_t NT, int c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NT * BLK * BLK) return;
  const int T = (int)(ts / BLK);
  const int64_t k = e / (BLK * BLK), q = e % (BLK * BLK);
  const int r = (int)(q % BLK), cc = (int)(q / BLK);
  dst[k * ts * ts + (int64_t)c * BLK + r + ((int64_t)c * BLK + cc) * ts] = dinv[(k * T + c) * BLK * BLK + q];
}

// diagonal tile k of the tile matrix = src (ts x ts)
__global__ void k_put_diag_tile(double* __restrict__ tiles, const double* __restrict__ src, int64_t ts, int64_t k) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ts * ts) tiles[(tri(k) + k) * ts * ts + e] = src[e];
}

// ------------------------------------------------------------- launchers
static inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_sort_locations(const double* x, const double* y, const double* z, int64_t n, int64_t npad, int64_t P,
                           double* box, uint64_t* keys, double* xs, double* ys, double* zs, int32_t* perm,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_bbox, dim3(1), dim3(1024), 0, s, x, y, z, n, box);
  hipLaunchKernelGGL(k_morton, dim3(nb(P, 256)), dim3(256), 0, s, x, y, n, P, box, keys);
  // P is a power of two >= 2048
  hipLaunchKernelGGL(k_bitonic_local, dim3((unsigned)(P / 2048)), dim3(1024), 0, s, keys, (int64_t)2, (int64_t)2048,
                     (int64_t)1);
  for (int64_t k = 4096; k <= P; k <<= 1) {
    int64_t j = k >> 1;
    for (; j >= 2048; j >>= 1)
      hipLaunchKernelGGL(k_bitonic_global, dim3(nb(P, 256)), dim3(256), 0, s, keys, P, j, k);
    hipLaunchKernelGGL(k_bitonic_local, dim3((unsigned)(P / 2048)), dim3(1024), 0, s, keys, k, k, j);
  }
  hipLaunchKernelGGL(k_gather, dim3(nb(npad, 256)), dim3(256), 0, s, x, y, z, n, npad, keys, xs, ys, zs, perm);
}

void launch_scatter(const double* v, const int32_t* perm, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter, dim3(nb(n, 256)), dim3(256), 0, s, v, perm, n, out);
}

void launch_potrf_blk(double* A, int64_t lda, double* dinv, double* ldpart, unsigned long long* info, int64_t col0,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_potrf_blk, dim3(1), dim3(1024), 0, s, A, lda, dinv, ldpart, info, col0);
}

void launch_trsv_fwd(const double* tiles, int64_t ts, int64_t NT, int64_t nreal, const double* dinv, double* yv,
                     hipStream_t s) {
  const int T = (int)(ts / BLK);
  const size_t shm = (size_t)(ts + 256) * sizeof(double);
  const int64_t gmax = (nreal + BLK - 1) / BLK;  // row blocks holding real rows
  for (int64_t k = 0; k < NT; ++k) {
    const double* Lkk = tiles + (k * (k + 1) / 2 + k) * ts * ts;
    hipLaunchKernelGGL(k_trsv_fwd_diag, dim3(1), dim3(256), shm, s, Lkk, ts, dinv + k * T * BLK * BLK, yv + k * ts);
    const int64_t g0 = (k + 1) * T;
    if (gmax > g0)
      hipLaunchKernelGGL(k_gemv_fwd, dim3((unsigned)(gmax - g0)), dim3(256), shm, s, tiles, ts, k, g0, yv);
  }
}

void launch_trsv_bwd(const double* tiles, int64_t ts, int64_t NT, const double* dinv, double* av, hipStream_t s) {
  const int T = (int)(ts / BLK);
  const size_t shm = (size_t)ts * sizeof(double);
  for (int64_t k = NT - 1; k >= 0; --k) {
    const double* Lkk = tiles + (k * (k + 1) / 2 + k) * ts * ts;
    hipLaunchKernelGGL(k_trsv_bwd_diag, dim3(1), dim3(256), shm, s, Lkk, ts, dinv + k * T * BLK * BLK, av + k * ts);
    if (k > 0) hipLaunchKernelGGL(k_gemv_bwd, dim3((unsigned)(k * T)), dim3(256), 0, s, tiles, ts, k, av + k * ts, av);
  }
}

void launch_trmv_lower(const double* tiles, int64_t ts, int64_t NT, int64_t nreal, const double* e, double* w,
                       hipStream_t s) {
  const int64_t gmax = (nreal + BLK - 1) / BLK;
  (void)NT;
  hipLaunchKernelGGL(k_trmv_lower, dim3((unsigned)gmax), dim3(256), 0, s, tiles, ts, e, w);
}

void launch_finalize_loglik(const double* yv, int64_t n, const double* ldpart, int64_t nld, double* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_loglik, dim3(1), dim3(256), 0, s, yv, n, ldpart, nld, out);
}

void launch_finalize_grad(const double* part, int64_t nparts, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_grad, dim3(1), dim3(256), 0, s, part, nparts, out);
}

void launch_fill_info(unsigned long long* info, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, s, info, ~0ull);
}

void launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_f64, dim3(nb(n, 256)), dim3(256), 0, s, p, n, v);
}

void launch_copy(double* dst, const double* src, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_copy_f64, dim3(nb(n, 256)), dim3(256), 0, s, dst, src, n);
}

void launch_copy_diag_lower(double* dst, const double* tiles, int64_t ts, int64_t NT, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_diag_lower, dim3(nb(NT * ts * ts, 256)), dim3(256), 0, s, dst, tiles, ts, NT);
}

void launch_put_dinv(double* dst, const double* dinv, int64_t ts, int64_t NT, int c, hipStream_t s) {
  hipLaunchKernelGGL(k_put_dinv, dim3(nb(NT * BLK * BLK, 256)), dim3(256), 0, s, dst, dinv, ts, NT, c);
}

void launch_put_diag_tile(double* tiles, const double* src, int64_t ts, int64_t k, hipStream_t s) {
  hipLaunchKernelGGL(k_put_diag_tile, dim3(nb(ts * ts, 256)), dim3(256), 0, s, tiles, src, ts, k);
}

}  // namespace exg
