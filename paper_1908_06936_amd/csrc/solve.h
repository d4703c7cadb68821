// Building blocks of the tile triangular solves: matrix-vector products over
// one 128-row or 128-column slab of a column-major ts x ts tile, 1024 threads
// per workgroup so that enough loads are in flight to stream the tile.
// Elements are read through a loader ld(row, col) that returns FP64 (FP64
// tiles, or FP32 / BF16 tiles widened exactly); sums are FP64 in a fixed order.
#pragma once

#include "common.h"

namespace exg {

constexpr int SOLVE_THREADS = 1024;

// rows r = t % 128 of a slab: sum_{c < cmax} ld(r, c) v[c] (v in LDS, cmax a
// multiple of 32).  Eight thread groups h = t / 128 take the columns
// c = h (mod 8); their sums meet in red (1024 doubles).  The result is valid
// in the threads with h = 0.
template <class LD>
__device__ __forceinline__ double slab_rowdot(LD ld, const double* v, int cmax, double* red) {
  const int t = threadIdx.x, r = t & 127, h = t >> 7;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int c = h; c < cmax; c += 32) {
    s0 += ld(r, c) * v[c];
    s1 += ld(r, c + 8) * v[c + 8];
    s2 += ld(r, c + 16) * v[c + 16];
    s3 += ld(r, c + 24) * v[c + 24];
  }
  red[t] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  double s = 0.0;
  if (h == 0) {
#pragma unroll
    for (int g = 0; g < 8; ++g) s += red[g * 128 + r];
  }
  return s;
}

// columns col0 + e, e < 8, of a tile, one wave: s[e] = sum_{r >= rlo(e)} ld(r, col0 + e) v[r]
// over the rows r < ts, rlo(e) = col0 + e when tri (lower triangle only), else 0.
// Lanes run down the column (coalesced); every lane receives the sums.
template <class LD>
__device__ __forceinline__ void wave_coldot8(LD ld, const double* __restrict__ v, int64_t col0, bool tri, int64_t ts,
                                             double (&s)[8]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int e = 0; e < 8; ++e) s[e] = 0.0;
  const int64_t r0 = tri ? (col0 & ~(int64_t)63) : 0;
  for (int64_t rb = r0; rb < ts; rb += 64) {
    const int64_t r = rb + lane;
    const double vr = v[r];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const double x = (!tri || r >= col0 + e) ? ld(r, col0 + e) : 0.0;
      s[e] += x * vr;
    }
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) s[e] = wave_sum(s[e]);
}

}  // namespace exg
