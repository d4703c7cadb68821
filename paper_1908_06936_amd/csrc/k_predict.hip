// Kriging (the conditional distribution of the Gaussian field given the data,
// paper Sections 4 and 5): at new locations s_i,
//   mean_i = c_i^T Sigma^-1 z = c_i^T a,            a = L^-T L^-1 z,
//   mse_i  = sigma^2 - |L^-1 c_i|^2,                c_i = (Sigma(s_i, s_j))_j,
// after the Cholesky factorisation of the observed covariance.  The mean is
// one fused pass over (new, observed) pairs that regenerates c_i on the fly;
// the variance needs V = L^-1 C for a block of new points, a tile forward
// substitution with many right-hand sides on FP64 MFMA.
#include "common.h"
#include "launch.h"
#include "matern_dev.h"

namespace exg {

// mean[i] = sum_j Sigma(new_i, obs_j) a_j over the real observed points; one
// 256-thread workgroup per new point, fixed-order reduction.
__global__ __launch_bounds__(256) void k_krige_mean(const double* __restrict__ xs, const double* __restrict__ ys,
                                                    const double* __restrict__ av, int64_t nreal,
                                                    const double* __restrict__ xn, const double* __restrict__ yn,
                                                    int64_t m, const double* __restrict__ qt,
                                                    const double* __restrict__ cst, double* __restrict__ mean) {
  __shared__ double red[256];
  const int64_t i = blockIdx.x;
  if (i >= m) return;
  const double px = xn[i], py = yn[i];
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < nreal; j += 256) {
    s += matern_value(loc_dist(px, py, xs[j], ys[j], cst), cst, qt) * av[j];
  }
  double v[1] = {s};
  block_sum<1>(v, red);
  if (threadIdx.x == 0) mean[i] = v[0];
}

// C[j + c ldc] = Sigma(obs_j, new_{c0 + c}) for rows j < npad (zero on the
// padded rows), columns c < ncols (zero for c0 + c >= m)
__global__ __launch_bounds__(256) void k_gen_cross(const double* __restrict__ xs, const double* __restrict__ ys,
                                                   int64_t nreal, int64_t npad, const double* __restrict__ xn,
                                                   const double* __restrict__ yn, int64_t m, int64_t c0,
                                                   int64_t ncols, const double* __restrict__ qt,
                                                   const double* __restrict__ cst, double* __restrict__ C,
                                                   int64_t ldc) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (j >= npad || c >= ncols) return;
  double v = 0.0;
  if (j < nreal && c0 + c < m) {
    v = matern_value(loc_dist(xs[j], ys[j], xn[c0 + c], yn[c0 + c], cst), cst, qt);
  }
  C[j + c * ldc] = v;
}

// V_k = X_kk C_k on the 128-row blocks u of tile row k, columns in 128-wide
// blocks cb; X_kk lower triangular, so the k range stops at (u + 1) 128.
__global__ __launch_bounds__(256, 2) void k_trsm_diag(const double* __restrict__ Xk, int64_t ts,
                                                      const double* __restrict__ Ck, double* __restrict__ Vk,
                                                      int64_t ld, int T) {
  __shared__ double sm[GEMM_LDS];
  const int u = (int)(blockIdx.x % T);
  const int64_t cb = blockIdx.x / T;
  v4d acc[4][4];
  acc_zero(acc);
  // Aop(m, q) = X[u*128 + m, q], Bop(n, q) = C[q, cb*128 + n]
  gemm_blk<false, true, true>(Xk + u * BLK, ts, Ck + cb * BLK * ld, ld, (u + 1) * BLK, acc, sm);
  acc_store(Vk + u * BLK + cb * BLK * ld, ld, acc, 1.0, false);
}

// C_i -= L_ik V_k for the tiles i > k with real rows, 128 x 128 blocks
// (i, u, cb); g0 = first global 128-row block below tile k.
__global__ __launch_bounds__(256, 2) void k_trsm_update(TileMat M, int64_t k, int64_t g0,
                                                        const double* __restrict__ Vk, double* __restrict__ C,
                                                        int64_t ld, int T, int64_t nrb) {
  __shared__ double sm[GEMM_LDS];
  const int64_t ts = M.ts;
  const int64_t g = g0 + blockIdx.x % nrb;
  const int64_t cb = blockIdx.x / nrb;
  const int64_t i = g / T;
  const int u = (int)(g % T);
  v4d acc[4][4];
  acc_zero(acc);
  // Aop(m, q) = L_ik[u*128 + m, q], Bop(n, q) = V_k[q, cb*128 + n]
  gemm_blk<false, true, true>(tptr(M, i, k) + u * BLK, ts, Vk + cb * BLK * ld, ld, (int)ts, acc, sm);
  acc_store(C + i * ts + u * BLK + cb * BLK * ld, ld, acc, -1.0, true);
}

// mse[c0 + c] = sigma^2 - sum_j V[j, c]^2, one workgroup per column
__global__ __launch_bounds__(256) void k_col_mse(const double* __restrict__ V, int64_t ld, int64_t nrows,
                                                 int64_t m, int64_t c0, const double* __restrict__ cst,
                                                 double* __restrict__ mse) {
  __shared__ double red[256];
  const int64_t c = blockIdx.x;
  if (c0 + c >= m) return;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < nrows; j += 256) {
    const double v = V[j + c * ld];
    s += v * v;
  }
  double v[1] = {s};
  block_sum<1>(v, red);
  if (threadIdx.x == 0) mse[c0 + c] = cst[C_S2] - v[0];
}

// ---------------------------------------------------------------- launchers
void launch_krige_mean(const double* xs, const double* ys, const double* av, int64_t nreal, const double* xn,
                       const double* yn, int64_t m, const double* qt, const double* cst, double* mean, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_krige_mean, dim3((unsigned)m), dim3(256), 0, s, xs, ys, av, nreal, xn, yn, m, qt, cst, mean);
}

void launch_krige_mse(const TileMat& M, const double* Xd, const double* xs, const double* ys, int64_t nreal,
                      const double* xn, const double* yn, int64_t m, int64_t c0, int64_t ncols, const double* qt,
                      const double* cst, double* C, double* V, double* mse, hipStream_t s) {
  const int64_t ts = M.ts, NT = M.NT, npad = NT * ts, ld = npad;
  const int T = (int)(ts / BLK);
  const int64_t ncb = ncols / BLK;  // ncols is a multiple of 128
  hipLaunchKernelGGL(k_gen_cross, dim3((unsigned)((npad + 255) / 256), (unsigned)ncols), dim3(256), 0, s, xs, ys,
                     nreal, npad, xn, yn, m, c0, ncols, qt, cst, C, ld);
  const int64_t gmax = (nreal + BLK - 1) / BLK;  // 128-row blocks holding real rows
  for (int64_t k = 0; k < NT; ++k) {
    hipLaunchKernelGGL(k_trsm_diag, dim3((unsigned)(T * ncb)), dim3(256), 0, s, Xd + k * ts * ts, ts, C + k * ts,
                       V + k * ts, ld, T);
    const int64_t g0 = (k + 1) * T;
    if (gmax > g0) {
      const int64_t nrb = gmax - g0;
      hipLaunchKernelGGL(k_trsm_update, dim3((unsigned)(nrb * ncb)), dim3(256), 0, s, M, k, g0,
                         (const double*)(V + k * ts), C, ld, T, nrb);
    }
  }
  hipLaunchKernelGGL(k_col_mse, dim3((unsigned)ncols), dim3(256), 0, s, (const double*)V, ld, npad, m, c0, cst, mse);
}

}  // namespace exg
