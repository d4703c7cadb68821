// Epilogue of the fused LAUUM + score contraction: for one 128 x 128 block of
// W = Sigma^-1 held in the MFMA accumulators, regenerate dSigma_m (eq. (3)
// differentiated in sigma^2, beta and nu) for the block's entries and form
//   g_m = sum over i >= j of (w_ij / 2) (a_i a_j - W_ij) dSigma_m(i, j),
// w = 2 below the diagonal and 1 on it, a = Sigma^-1 z; padded rows and
// columns and entries above the diagonal contribute nothing.  The block's
// three sums go to out[0..2] (a fixed-order reduction, no atomics).
#pragma once

#include "common.h"
#include "gemm32.h"
#include "matern_dev.h"

namespace exg {

__device__ __forceinline__ void contract_entry(int64_t gi, int64_t gj, double xi, double yi, double ai, double wv,
                                               const double* __restrict__ xs, const double* __restrict__ ys,
                                               const double* __restrict__ av, const double* __restrict__ qt,
                                               const double* __restrict__ cst, double (&g3)[3]) {
  const double wgt = (gi == gj) ? 0.5 : 1.0;  // (w / 2) with w = 1 or 2
  const double f = wgt * (ai * av[gj] - wv);
  double d0, d1, d2;
  matern_grad(loc_dist(xi, yi, xs[gj], ys[gj], cst), cst, qt, &d0, &d1, &d2);
  g3[0] += f * d0;
  g3[1] += f * d1;
  g3[2] += f * d2;
}

// FP64 accumulators in the layout of gemm_core (rows m = wr*64 + 16 i +
// (lane & 15), columns n = wc*64 + 16 j + 4 r + (lane >> 4)); row0 / col0 are
// the global indices of the block's first row and column.  The 16 values of
// one row group go through thread-private LDS slots so that the loop over
// them indexes at run time without forcing the accumulators out of registers.
__device__ __forceinline__ void contract_block64(const v4d (&acc)[4][4], int64_t row0, int64_t col0, int64_t nreal,
                                                 const double* __restrict__ xs, const double* __restrict__ ys,
                                                 const double* __restrict__ av, const double* __restrict__ qt,
                                                 const double* __restrict__ cst, double* sm /* >= 16 x 256 */,
                                                 double* out) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  double g3[3] = {0.0, 0.0, 0.0};
  double* fb = sm;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) fb[(j * 4 + r) * GEMM_THREADS + t] = acc[i][j][r];
    const int64_t gi = row0 + wr * 64 + 16 * i + (lane & 15);
    if (gi >= nreal) continue;
    const double xi = xs[gi], yi = ys[gi], ai = av[gi];
    for (int e = 0; e < 16; ++e) {
      const int j = e >> 2, r = e & 3;
      const int64_t gj = col0 + wc * 64 + 16 * j + 4 * r + (lane >> 4);
      if (gj >= nreal || gj > gi) continue;
      contract_entry(gi, gj, xi, yi, ai, fb[e * GEMM_THREADS + t], xs, ys, av, qt, cst, g3);
    }
  }
  __syncthreads();
  block_sum<3>(g3, sm);
  if (t == 0) {
    out[0] = g3[0];
    out[1] = g3[1];
    out[2] = g3[2];
  }
}

// FP32 accumulators in the layout of gemm32 (rows m = wr*64 + 32 x +
// (lane & 31), columns n = wc*64 + 32 y + 8 (r / 4) + 4 (lane / 32) + r % 4),
// contracted in FP64 like contract_block64.
__device__ __forceinline__ void contract_block32(const v16f (&acc)[2][2], int64_t row0, int64_t col0, int64_t nreal,
                                                 const double* __restrict__ xs, const double* __restrict__ ys,
                                                 const double* __restrict__ av, const double* __restrict__ qt,
                                                 const double* __restrict__ cst, float* sm /* >= 32 x 256 */,
                                                 double* out) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  double g3[3] = {0.0, 0.0, 0.0};
  float* fb = sm;
#pragma unroll
  for (int x = 0; x < 2; ++x) {
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 16; ++r) fb[(y * 16 + r) * GEMM_THREADS + t] = acc[x][y][r];
    const int64_t gi = row0 + wr * 64 + 32 * x + (lane & 31);
    if (gi >= nreal) continue;
    const double xi = xs[gi], yi = ys[gi], ai = av[gi];
    for (int e = 0; e < 32; ++e) {
      const int y = e >> 4, r = e & 15;
      const int64_t gj = col0 + wc * 64 + 32 * y + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (gj >= nreal || gj > gi) continue;
      contract_entry(gi, gj, xi, yi, ai, (double)fb[e * GEMM_THREADS + t], xs, ys, av, qt, cst, g3);
    }
  }
  __syncthreads();
  block_sum<3>(g3, (double*)sm);
  if (t == 0) {
    out[0] = g3[0];
    out[1] = g3[1];
    out[2] = g3[2];
  }
}

}  // namespace exg
