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
#include "solve.h"

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

// sqrt(d) and 1 / sqrt(d) from the hardware reciprocal square root and two
// Newton steps (each doubles the correct bits: y <- y + y (1 - d y^2) / 2),
// then one Newton step on the square root itself (s <- s + (d - s^2) / (2 s));
// within an ulp or two of the correctly rounded values, without the long
// correctly rounded sequences on the factorisation's serial path.
__device__ __forceinline__ void sqrt_and_rsqrt(double d, double* sq, double* rsq) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  const double s0 = d * y;
  *sq = fma(0.5 * y, fma(-s0, s0, d), s0);
  *rsq = y;
}

// ------------------------------------------------ diagonal 128-block factor
// Cholesky of one 128 x 128 block and the inverse of its factor.
// 256 threads; thread (tr, tc) = (t % 16, t / 16) holds the 64 entries
// (tr + 16 p, tc + 16 q) in registers.
//   factor (right-looking, one barrier per column): the owners of column j
//   publish it to LDS, then every thread applies A_rc -= A_rj A_cj / A_jj to
//   its entries with r, c > j and the owners keep L_rj = A_rj / sqrt(A_jj).
//   inverse: L goes to LDS; with T = unit lower triangular, rows m = 0..127:
//   the owners of row m publish it and T_ij -= (L_im / L_mm) T_mj for i > m >= j;
//   then X = L^-1 has X_ij = T_ij / L_ii.
// Writes L (zeros above the diagonal) over the block, X to dinv (ld 128), the
// block's sum of 2 ln L_jj to *ldpart and the first failing global column
// (1-based) to *info with an atomic minimum.
__global__ __launch_bounds__(256) void k_potrf_blk(double* __restrict__ A, int64_t lda, double* __restrict__ dinv,
                                                   double* __restrict__ ldpart, unsigned long long* __restrict__ info,
                                                   int64_t col0) {
  // L packed by columns (lower triangle only): L_rc at lcol(c) + r - c.  The
  // block needs 69 KB of LDS, so it fits on a CU beside one trailing-update
  // block and the lookahead panel is not starved by the update.
  __shared__ double Ls[BLK * (BLK + 1) / 2];
  __shared__ double pub[2][BLK];  // published column (factor) / row (inverse)
  __shared__ double dg[BLK];      // L_jj
  __shared__ double idg[BLK];     // 1 / L_jj
  const int t = threadIdx.x, tr = t & 15, tc = t >> 4;
  double a[8][8];
#pragma unroll
  for (int p = 0; p < 8; ++p)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r = tr + 16 * p, c = tc + 16 * q;
      a[p][q] = (r >= c) ? A[r + (int64_t)c * lda] : 0.0;
    }
  // j = 16 qj + jj: the block index qj is a compile-time constant in each
  // unrolled copy, so the owners address their registers statically
#pragma unroll
  for (int qj = 0; qj < 8; ++qj) {
#pragma unroll 1
    for (int jj = 0; jj < 16; ++jj) {
      const int j = 16 * qj + jj;
      const int buf = j & 1;
      if (tc == jj) {
#pragma unroll
        for (int p = 0; p < 8; ++p) {
          const int r = tr + 16 * p;
          if (r >= j) pub[buf][r] = a[p][qj];
        }
      }
      __syncthreads();
      const double d = pub[buf][j];
      double sd, isd;
      sqrt_and_rsqrt(d, &sd, &isd);
      if (t == 0) {
        dg[j] = sd;
        idg[j] = isd;
        if (!(d > 0.0) || !(d <= DBL_MAX)) atomicMin(info, (unsigned long long)(col0 + j + 1));
      }
      const double id = isd * isd;
      double lr[8], lc[8];
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const int r = tr + 16 * p;
        lr[p] = (r > j) ? pub[buf][r] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int c = tc + 16 * q;
        lc[q] = (c > j) ? pub[buf][c] * id : 0.0;
      }
#pragma unroll
      for (int q = qj; q < 8; ++q) {
        // lower blocks only: the upper ones are never read
#pragma unroll
        for (int p = q; p < 8; ++p) a[p][q] -= lr[p] * lc[q];
      }
      if (tc == jj) {
#pragma unroll
        for (int p = qj; p < 8; ++p) {
          const int r = tr + 16 * p;
          if (r > j) a[p][qj] = pub[buf][r] * isd;
          else if (r == j) a[p][qj] = sd;
        }
      }
    }
  }
  // L to LDS and to the block (zeros above the diagonal)
#pragma unroll
  for (int p = 0; p < 8; ++p)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r = tr + 16 * p, c = tc + 16 * q;
      const double lv = (r >= c) ? a[p][q] : 0.0;
      if (r >= c) Ls[c * BLK - c * (c - 1) / 2 + r - c] = lv;
      A[r + (int64_t)c * lda] = lv;
      a[p][q] = 0.0;  // now T, strictly lower part
    }
  __syncthreads();
#pragma unroll
  for (int pm = 0; pm < 8; ++pm) {
#pragma unroll 1
    for (int mm = 0; mm < 16; ++mm) {
      const int m = 16 * pm + mm;
      if (m == BLK - 1) break;
      const int buf = m & 1;
      if (tr == mm) {
#pragma unroll
        for (int q = 0; q <= pm; ++q) {
          const int c = tc + 16 * q;
          if (c < m) pub[buf][c] = a[pm][q];
        }
        if (tc == 0) pub[buf][m] = 1.0;
      }
      __syncthreads();
      const double inv_lmm = idg[m];
      double li[8], tm[8];
#pragma unroll
      for (int p = pm; p < 8; ++p) {
        const int r = tr + 16 * p;
        li[p] = (r > m) ? Ls[m * BLK - m * (m - 1) / 2 + r - m] * inv_lmm : 0.0;
      }
#pragma unroll
      for (int q = 0; q <= pm; ++q) {
        const int c = tc + 16 * q;
        tm[q] = (c <= m) ? pub[buf][c] : 0.0;
      }
#pragma unroll
      for (int p = pm; p < 8; ++p)
#pragma unroll
        for (int q = 0; q <= pm; ++q) a[p][q] -= li[p] * tm[q];
    }
  }
#pragma unroll
  for (int p = 0; p < 8; ++p)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r = tr + 16 * p, c = tc + 16 * q;
      const double il = idg[r];
      dinv[r + c * BLK] = (r > c) ? a[p][q] * il : ((r == c) ? il : 0.0);
    }
  // 2 sum ln L_jj: one logarithm per thread, fixed-order block sum (pub is
  // free once every thread has left the inverse loop)
  __syncthreads();
  double lg[1] = {t < BLK ? 2.0 * log(dg[t]) : 0.0};
  block_sum<1>(lg, &pub[0][0]);
  if (t == 0) *ldpart = lg[0];
}

// ------------------------------------------------------- triangular solves
// rhs_i -= L_ik y_k for the 128-row blocks g0 <= g < gmax below tile k.
__global__ __launch_bounds__(SOLVE_THREADS) void k_gemv_fwd(TileMat M, int64_t k, int64_t g0,
                                                           const double* __restrict__ yk, double* __restrict__ rhs) {
  const int64_t ts = M.ts;
  extern __shared__ double sy[];  // ts + SOLVE_THREADS
  double* red = sy + ts;
  const int T = (int)(ts / BLK);
  const int64_t g = g0 + blockIdx.x;
  const int64_t i = g / T;
  const int u = (int)(g % T);
  const int t = threadIdx.x;
  for (int q = t; q < ts; q += SOLVE_THREADS) sy[q] = yk[q];
  __syncthreads();
  const double* L = tptr(M, i, k) + u * BLK;
  const double s = slab_rowdot([=](int r, int c) { return L[r + (int64_t)c * ts]; }, sy, (int)ts, red);
  if (t < BLK) rhs[i * ts + u * BLK + t] -= s;
}

// out = X b on one diagonal tile, X lower triangular (explicit inverse);
// one 128-row block per workgroup
__global__ __launch_bounds__(SOLVE_THREADS) void k_diag_apply_n(const double* __restrict__ X, int64_t ts,
                                                               const double* __restrict__ b,
                                                               double* __restrict__ out) {
  __shared__ double sb[4096];  // ts <= 4096
  __shared__ double red[SOLVE_THREADS];
  const int rb = blockIdx.x, t = threadIdx.x;
  const int cmax = (rb + 1) * BLK;  // X(row, c) = 0 for c >= cmax
  for (int q = t; q < cmax; q += SOLVE_THREADS) sb[q] = b[q];
  __syncthreads();
  const double* Xr = X + rb * BLK;
  const double s = slab_rowdot([=](int r, int c) { return Xr[r + (int64_t)c * ts]; }, sb, cmax, red);
  if (t < BLK) out[rb * BLK + t] = s;
}

// out = X^T b on one diagonal tile, X lower triangular; one 128-column block
// per workgroup, eight columns per wave (lanes run down the columns)
__global__ __launch_bounds__(SOLVE_THREADS) void k_diag_apply_t(const double* __restrict__ X, int64_t ts,
                                                               const double* __restrict__ b,
                                                               double* __restrict__ out) {
  const int64_t col0 = (int64_t)blockIdx.x * BLK + 8 * (threadIdx.x >> 6);
  double s[8];
  wave_coldot8([=](int64_t r, int64_t c) { return X[r + c * ts]; }, b, col0, true, ts, s);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) out[col0 + e] = s[e];
  }
}

// rhs_j -= L_kj^T a_k over the 128-column blocks of the tiles j < k (one
// block per workgroup)
__global__ __launch_bounds__(SOLVE_THREADS) void k_gemv_bwd(TileMat M, int64_t k, const double* __restrict__ ak,
                                                           double* __restrict__ rhs) {
  const int64_t ts = M.ts;
  const int T = (int)(ts / BLK);
  const int64_t cb = blockIdx.x;
  const int64_t j = cb / T;
  const int64_t col0 = (cb % T) * BLK + 8 * (threadIdx.x >> 6);
  const double* L = tptr(M, k, j);
  double s[8];
  wave_coldot8([=](int64_t r, int64_t c) { return L[r + c * ts]; }, ak, col0, false, ts, s);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) rhs[j * ts + col0 + e] -= s[e];
  }
}

// w = L e on the lower tiles (diagonal tiles read below their diagonal only);
// one 128-row block per workgroup
__global__ __launch_bounds__(256) void k_trmv_lower(TileMat M, const double* __restrict__ e, double* __restrict__ w) {
  const int64_t ts = M.ts;
  __shared__ double red[256];
  const int T = (int)(ts / BLK);
  const int64_t g = blockIdx.x;
  const int64_t i = g / T;
  const int u = (int)(g % T);
  const int t = threadIdx.x, r = t & 127, h = t >> 7;
  const int64_t row = u * BLK + r;
  double s = 0.0;
  for (int64_t j = 0; j <= i; ++j) {
    const double* L = tptr(M, i, j) + row;
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

// eq. (2) from log det Sigma (sum of ldpart) and the quadratic form
// z^T Sigma^-1 z = z^T a with a = Sigma^-1 z (refined solve)
__global__ __launch_bounds__(256) void k_finalize_loglik_za(const double* __restrict__ zs, const double* __restrict__ av,
                                                            int64_t n, const double* __restrict__ ldpart, int64_t nld,
                                                            double* __restrict__ out) {
  __shared__ double red[2 * 256];
  double v[2] = {0.0, 0.0};
  for (int64_t i = threadIdx.x; i < n; i += 256) v[0] += zs[i] * av[i];
  for (int64_t i = threadIdx.x; i < nld; i += 256) v[1] += ldpart[i];
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    const double q = v[0], ld = v[1];
    out[0] = -0.5 * ((double)n * 1.8378770664093454836 + ld + q);
    out[1] = ld;
    out[2] = q;
  }
}

// y = a + d
__global__ void k_add2_f64(double* __restrict__ y, const double* __restrict__ a, const double* __restrict__ d,
                           int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] + d[i];
}

// Refinement bookkeeping on the device (no host round trip): nrm[0] holds
// the squared norm of the accepted residual.  init: nrm[0] = |r|^2.  trial:
// flag = |r_try|^2 < nrm[0], and then nrm[0] = |r_try|^2.
__global__ __launch_bounds__(1024) void k_resid_norm(const double* __restrict__ r, int64_t n, double* __restrict__ nrm,
                                                     int trial) {
  __shared__ double red[1024];
  double v[1] = {0.0};
  for (int64_t i = threadIdx.x; i < n; i += 1024) v[0] += r[i] * r[i];
  block_sum<1>(v, red);
  if (threadIdx.x == 0) {
    if (!trial) {
      nrm[0] = v[0];
    } else {
      const bool better = v[0] < nrm[0];
      nrm[1] = better ? 1.0 : 0.0;
      if (better) nrm[0] = v[0];
    }
  }
}

// accept the trial step when the flag is set: a <- a_try, r <- r_try
__global__ void k_refine_select(double* __restrict__ a, const double* __restrict__ a_try, double* __restrict__ r,
                                const double* __restrict__ r_try, const double* __restrict__ nrm, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && nrm[1] != 0.0) {
    a[i] = a_try[i];
    r[i] = r_try[i];
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

__global__ void k_copy_f64(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// dst[k] = lower part of diagonal tile k (zeros above the diagonal), k < NT
__global__ void k_copy_diag_lower(double* __restrict__ dst, const double* __restrict__ diag, int64_t ts, int64_t NT) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tt = ts * ts;
  if (e >= NT * tt) return;
  const int64_t k = e / tt, q = e % tt;
  const int64_t r = q % ts, c = q / ts;
  dst[e] = (r >= c) ? diag[k * tt + q] : 0.0;
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
  hipLaunchKernelGGL(k_potrf_blk, dim3(1), dim3(256), 0, s, A, lda, dinv, ldpart, info, col0);
}

void launch_trsv_fwd(const TileMat& M, const double* Xd, int64_t nreal, double* rhs, double* y, hipStream_t s) {
  const int64_t ts = M.ts, NT = M.NT;
  const int T = (int)(ts / BLK);
  const size_t shm = (size_t)(ts + SOLVE_THREADS) * sizeof(double);
  const int64_t gmax = (nreal + BLK - 1) / BLK;  // row blocks holding real rows
  for (int64_t k = 0; k < NT; ++k) {
    launch_diag_apply_n(Xd + k * ts * ts, ts, rhs + k * ts, y + k * ts, s);
    const int64_t g0 = (k + 1) * T;
    if (gmax > g0)
      hipLaunchKernelGGL(k_gemv_fwd, dim3((unsigned)(gmax - g0)), dim3(SOLVE_THREADS), shm, s, M, k, g0, y + k * ts,
                         rhs);
  }
}

void launch_diag_apply_n(const double* Xk, int64_t ts, const double* b, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_apply_n, dim3((unsigned)(ts / BLK)), dim3(SOLVE_THREADS), 0, s, Xk, ts, b, out);
}

void launch_diag_apply_t(const double* Xk, int64_t ts, const double* b, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_apply_t, dim3((unsigned)(ts / BLK)), dim3(SOLVE_THREADS), 0, s, Xk, ts, b, out);
}

void launch_trsv_bwd(const TileMat& M, const double* Xd, double* rhs, double* a, hipStream_t s) {
  const int64_t ts = M.ts, NT = M.NT;
  const int T = (int)(ts / BLK);
  for (int64_t k = NT - 1; k >= 0; --k) {
    launch_diag_apply_t(Xd + k * ts * ts, ts, rhs + k * ts, a + k * ts, s);
    if (k > 0)
      hipLaunchKernelGGL(k_gemv_bwd, dim3((unsigned)(k * T)), dim3(SOLVE_THREADS), 0, s, M, k, a + k * ts, rhs);
  }
}

void launch_trmv_lower(const TileMat& M, int64_t nreal, const double* e, double* w, hipStream_t s) {
  const int64_t gmax = (nreal + BLK - 1) / BLK;
  hipLaunchKernelGGL(k_trmv_lower, dim3((unsigned)gmax), dim3(256), 0, s, M, e, w);
}

void launch_finalize_loglik(const double* yv, int64_t n, const double* ldpart, int64_t nld, double* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_loglik, dim3(1), dim3(256), 0, s, yv, n, ldpart, nld, out);
}

void launch_finalize_loglik_za(const double* zs, const double* av, int64_t n, const double* ldpart, int64_t nld,
                               double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_loglik_za, dim3(1), dim3(256), 0, s, zs, av, n, ldpart, nld, out);
}

void launch_add2(double* y, const double* a, const double* d, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_add2_f64, dim3(nb(n, 256)), dim3(256), 0, s, y, a, d, n);
}

void launch_resid_norm(const double* r, int64_t n, double* nrm, int trial, hipStream_t s) {
  hipLaunchKernelGGL(k_resid_norm, dim3(1), dim3(1024), 0, s, r, n, nrm, trial);
}

void launch_refine_select(double* a, const double* a_try, double* r, const double* r_try, const double* nrm,
                          int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_refine_select, dim3(nb(n, 256)), dim3(256), 0, s, a, a_try, r, r_try, nrm, n);
}

void launch_finalize_grad(const double* part, int64_t nparts, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_grad, dim3(1), dim3(256), 0, s, part, nparts, out);
}

void launch_fill_info(unsigned long long* info, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, s, info, ~0ull);
}

void launch_copy(double* dst, const double* src, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_copy_f64, dim3(nb(n, 256)), dim3(256), 0, s, dst, src, n);
}

void launch_copy_diag_lower(double* dst, const double* diag, int64_t ts, int64_t NT, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_diag_lower, dim3(nb(NT * ts * ts, 256)), dim3(256), 0, s, dst, diag, ts, NT);
}

void launch_put_dinv(double* dst, const double* dinv, int64_t ts, int64_t NT, int c, hipStream_t s) {
  hipLaunchKernelGGL(k_put_dinv, dim3(nb(NT * BLK * BLK, 256)), dim3(256), 0, s, dst, dinv, ts, NT, c);
}


}  // namespace exg
