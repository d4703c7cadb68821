// Fisher information of theta (exact_fisher in the paper's API table):
//   I_jk = tr(Sigma^-1 dSigma_j Sigma^-1 dSigma_k) / 2
//        = <B_j, B_k> / 2,   B_j = X dSigma_j X^T,   X = L^-1,
// with <.,.> the Frobenius product of the symmetric B's.  For sigma^2,
// dSigma = Sigma / sigma^2 gives B = I / sigma^2, so I_ss = n / (2 sigma^4) and
// I_sk = tr(B_k) / (2 sigma^2); the (beta, nu) block needs B_beta and B_nu
// (with a nugget tau^2, dSigma_sigma2 = (Sigma - tau^2 I) / sigma^2 and B_sigma2
// is formed like the other two).  Each B_j lives in ONE buffer of lower
// tiles (n^2 / 2 doubles), built in two sweeps over chunks of tile columns:
//   1. G_j = dSigma_j is regenerated for the chunk's tile rows into a strip
//      (G symmetric: the strip holds G(J, K) for the chunk's J and every K),
//      and M(I, J) = sum_{K <= I} X(I, K) G(K, J) is written for I >= J into
//      the lower tiles (B = M X^T needs only M's lower tiles);
//   2. in place, chunks in descending order: B(I, J) = sum_{K <= J} M(I, K)
//      X(J, K)^T reads only columns K <= J, which no later chunk overwrites;
//      the chunk's results are staged in the strip and copied back.
// The products run on FP64 MFMA through the shared block core; one streaming
// pass over the lower tiles forms the traces and Frobenius products.
// Lower-tile layout: tile (I, J), I >= J, at low_index(I, J) ts^2, packed by
// tile columns (diagonal included), each tile column-major.
#include "common.h"
#include "launch.h"
#include "matern_dev.h"

namespace exg {

__host__ __device__ __forceinline__ int64_t low_index(int64_t I, int64_t J, int64_t NT) {
  return J * NT - J * (J - 1) / 2 + (I - J);
}

__device__ __forceinline__ double* low_tile(double* B, int64_t I, int64_t J, int64_t NT, int64_t ts) {
  return B + low_index(I, J, NT) * ts * ts;
}

// strip tile (jj, K) = G(J0 + jj, K) for K < NT: ts x ts, rows the points of
// tile J0 + jj, columns those of tile K, at (jj NT + K) ts^2; zero on padding
__global__ __launch_bounds__(256) void k_gen_dstrip(double* __restrict__ S, int comp, int T, int64_t NT, int64_t ts,
                                                    int64_t J0, int64_t W, int64_t nreal,
                                                    const double* __restrict__ xs, const double* __restrict__ ys,
                                                    const double* __restrict__ qt, const double* __restrict__ cst) {
  const int64_t b = blockIdx.x;
  const int64_t tile = b / (T * T);
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  const int64_t jj = tile / NT, K = tile % NT;
  if (jj >= W || J0 + jj >= NT) return;
  const int r = threadIdx.x & 127, c0 = threadIdx.x >> 7;
  const int64_t gi = (J0 + jj) * ts + u * BLK + r;
  double* out = S + (jj * NT + K) * ts * ts + u * BLK + r + (int64_t)v * BLK * ts;
  const bool ipad = gi >= nreal;
  const double xi = ipad ? 0.0 : xs[gi], yi = ipad ? 0.0 : ys[gi];
  for (int c = c0; c < BLK; c += 2) {
    const int64_t gj = K * ts + v * BLK + c;
    double val = 0.0;
    if (!ipad && gj < nreal) {
      double d0, d1, d2;
      matern_grad(loc_dist(xi, yi, xs[gj], ys[gj], cst), cst, qt, &d0, &d1, &d2);
      val = comp == 0 ? d0 : (comp == 1 ? d1 : d2);
    }
    out[(int64_t)c * ts] = val;
  }
}

// tile pair q of a chunk -> (jj, I): chunk columns J0 .. J0 + W - 1, rows
// I >= J0 + jj, heaviest (largest I) first within each column
__device__ __forceinline__ bool chunk_pair(int64_t q, int64_t NT, int64_t J0, int64_t W, int64_t* jj, int64_t* I) {
  for (int64_t c = 0; c < W && J0 + c < NT; ++c) {
    const int64_t cnt = NT - (J0 + c);
    if (q < cnt) {
      *jj = c;
      *I = NT - 1 - q;
      return true;
    }
    q -= cnt;
  }
  return false;
}

// sweep 1: M(I, J) = sum_{K <= I} X(I, K) G(K, J) for the chunk's J and I >= J
// into the lower tiles of Bm.  G(K, J)[k, n] = strip(jj, K)[n + k ts], so both
// operands are read along their contiguous row index; X(I, I) is lower
// triangular, so the range stops after the block's own 128 columns of tile I.
__global__ __launch_bounds__(256, 2) void k_fisher_xg(TileMat X, const double* __restrict__ S, double* __restrict__ Bm,
                                                      int T, int64_t J0, int64_t W, int64_t nreal, int64_t nb) {
  __shared__ double sm[GEMM_LDS];
  const int64_t ts = X.ts, NT = X.NT;
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  int64_t jj, I;
  if (!chunk_pair(b / (T * T), NT, J0, W, &jj, &I)) return;
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  const int64_t J = J0 + jj;
  v4d acc[4][4];
  acc_zero(acc);
  if (I * ts + u * BLK < nreal && J * ts + v * BLK < nreal) {
    auto ap = [=](int k0) -> const double* { return tptr(X, I, k0 / ts) + u * BLK + (int64_t)(k0 % ts) * ts; };
    auto bp = [=](int k0) -> const double* {
      return S + (jj * NT + k0 / ts) * ts * ts + v * BLK + (int64_t)(k0 % ts) * ts;
    };
    gemm_core<false, false>(ap, ts, bp, ts, (int)(I * ts + (u + 1) * BLK), acc, sm);
  }
  acc_store(low_tile(Bm, I, J, NT, ts) + u * BLK + (int64_t)v * BLK * ts, ts, acc, 1.0, false);
}

// sweep 2: B(I, J) = sum_{K <= J} M(I, K) X(J, K)^T for the chunk's J, I >= J
// (blocks v <= u on the diagonal tile), M read from the lower tiles of Bm,
// the result staged in stage tile (jj, I) at (jj NT + I) ts^2.  X(J, J) is
// lower triangular: its columns beyond the block's own 128 are zero.
__global__ __launch_bounds__(256, 2) void k_fisher_mxt(TileMat X, const double* __restrict__ Bm,
                                                       double* __restrict__ stage, int T, int64_t J0, int64_t W,
                                                       int64_t nreal, int64_t nb) {
  __shared__ double sm[GEMM_LDS];
  const int64_t ts = X.ts, NT = X.NT;
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  int64_t jj, I;
  if (!chunk_pair(b / (T * T), NT, J0, W, &jj, &I)) return;
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  const int64_t J = J0 + jj;
  if ((I == J && u < v) || I * ts + u * BLK >= nreal || J * ts + v * BLK >= nreal) return;
  v4d acc[4][4];
  acc_zero(acc);
  auto ap = [=](int k0) -> const double* {
    return low_tile((double*)Bm, I, k0 / ts, NT, ts) + u * BLK + (int64_t)(k0 % ts) * ts;
  };
  auto bp = [=](int k0) -> const double* { return tptr(X, J, k0 / ts) + v * BLK + (int64_t)(k0 % ts) * ts; };
  gemm_core<false, false>(ap, ts, bp, ts, (int)(J * ts + (v + 1) * BLK), acc, sm);
  acc_store(stage + (jj * NT + I) * ts * ts + u * BLK + (int64_t)v * BLK * ts, ts, acc, 1.0, false);
}

// lower tile (I, J0 + jj) of Bm <- stage tile (jj, I) for I >= J0 + jj; the
// blocks of a diagonal tile above its diagonal carry no value and are never read
__global__ void k_fisher_unstage(const double* __restrict__ stage, double* __restrict__ Bm, int64_t NT, int64_t ts,
                                 int64_t J0, int64_t W) {
  const int64_t tt = ts * ts;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= W * NT * tt) return;
  const int64_t t = e / tt, o = e % tt;
  const int64_t jj = t / NT, I = t % NT, J = J0 + jj;
  if (J >= NT || I < J) return;
  Bm[low_index(I, J, NT) * tt + o] = stage[e];
}

// B(I, J) block (u, v) of the lower tiles (blocks v <= u on the diagonal tiles)
// for the streaming pass; false for blocks above the diagonal or in the padding
__device__ __forceinline__ bool fisher_lower_block(int64_t b, int T, int64_t ts, int64_t nreal, int64_t* I,
                                                   int64_t* J, int* u, int* v) {
  const int64_t p = b / (T * T);
  const int sub = (int)(b % (T * T));
  *u = sub / T;
  *v = sub % T;
  tri_decode(p, I, J);
  return !((*I == *J && *u < *v) || *I * ts + *u * BLK >= nreal || *J * ts + *v * BLK >= nreal);
}

// Per lower block of the symmetric B_0 = B_sigma2 (Bs, null: B_0 = I / sigma2,
// handled in the finalisation), B_1 = B_beta (Bb) and B_2 = B_nu (Bn): the
// block's terms of tr B_0, tr B_1, tr B_2, <B_0, B_0>, <B_1, B_1>, <B_2, B_2>,
// <B_0, B_1>, <B_0, B_2>, <B_1, B_2> (weight 2 off the diagonal by symmetry)
// into part[9 b ..]; padded rows and columns of B are zero, so whole blocks
// are summed.
constexpr int FP = 9;
__global__ __launch_bounds__(256) void k_fisher_dot(const double* __restrict__ Bs, const double* __restrict__ Bb,
                                                    const double* __restrict__ Bn, double* __restrict__ part, int T,
                                                    int64_t NT, int64_t ts, int64_t nreal, int64_t nb) {
  __shared__ double red[FP * 256];
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  int64_t I, J;
  int u, v;
  double s[FP];
#pragma unroll
  for (int q = 0; q < FP; ++q) s[q] = 0.0;
  if (fisher_lower_block(b, T, ts, nreal, &I, &J, &u, &v)) {
    const int64_t off = low_index(I, J, NT) * ts * ts + u * BLK + (int64_t)v * BLK * ts;
    const bool diag = I == J && u == v;
    const double w = diag ? 1.0 : 2.0;
    for (int e = threadIdx.x; e < BLK * BLK; e += 256) {
      const int m = e & (BLK - 1), n = e >> 7;
      const int64_t q = off + m + (int64_t)n * ts;
      const double p0 = Bs ? Bs[q] : 0.0, p1 = Bb[q], p2 = Bn[q];
      if (diag && m == n) {
        s[0] += p0;
        s[1] += p1;
        s[2] += p2;
      }
      s[3] += w * p0 * p0;
      s[4] += w * p1 * p1;
      s[5] += w * p2 * p2;
      s[6] += w * p0 * p1;
      s[7] += w * p0 * p2;
      s[8] += w * p1 * p2;
    }
  }
  block_sum<FP>(s, red);
  if (threadIdx.x < FP) part[FP * b + threadIdx.x] = s[threadIdx.x];
}

// I (row-major 3 x 3) from the partial sums; one workgroup, fixed-order sums.
// has_s0 = 0: B_0 = I / sigma2, so <B_0, B_0> = n / sigma2^2 and
// <B_0, B_k> = tr B_k / sigma2.
__global__ __launch_bounds__(256) void k_fisher_finalize(const double* __restrict__ part, int64_t nb,
                                                         const double* __restrict__ cst, int64_t nreal, int has_s0,
                                                         double* __restrict__ out) {
  __shared__ double red[FP * 256];
  double v[FP];
#pragma unroll
  for (int q = 0; q < FP; ++q) v[q] = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += 256) {
#pragma unroll
    for (int q = 0; q < FP; ++q) v[q] += part[FP * b + q];
  }
  block_sum<FP>(v, red);
  if (threadIdx.x == 0) {
    const double s2 = cst[C_S2];
    if (!has_s0) {
      v[3] = (double)nreal / (s2 * s2);
      v[6] = v[1] / s2;
      v[7] = v[2] / s2;
    }
    out[0] = 0.5 * v[3];
    out[1] = out[3] = 0.5 * v[6];
    out[2] = out[6] = 0.5 * v[7];
    out[4] = 0.5 * v[4];
    out[5] = out[7] = 0.5 * v[8];
    out[8] = 0.5 * v[5];
  }
}

// ---------------------------------------------------------------- launchers
int64_t fisher_part_blocks(int64_t ts, int64_t NT) {
  const int64_t T = ts / BLK;
  return NT * (NT + 1) / 2 * T * T;
}

int64_t fisher_chunk_tiles(int64_t NT) { return NT < 8 ? NT : (NT + 7) / 8; }

size_t fisher_strip_doubles(int64_t ts, int64_t NT) { return (size_t)fisher_chunk_tiles(NT) * NT * ts * ts; }

// one parameter's B = X dSigma_comp X^T (comp 0: sigma2, 1: beta, 2: nu) into
// the lower tiles of Bm, through the strip S (fisher_strip_doubles)
void launch_fisher_param(const TileMat& X, int comp, int64_t nreal, const double* xs, const double* ys,
                         const double* qt, const double* cst, double* S, double* Bm, hipStream_t s) {
  const int64_t ts = X.ts, NT = X.NT;
  const int T = (int)(ts / BLK);
  const int64_t W = fisher_chunk_tiles(NT), tt = ts * ts;
  auto pairs = [&](int64_t J0) {
    int64_t q = 0;
    for (int64_t c = 0; c < W && J0 + c < NT; ++c) q += NT - (J0 + c);
    return q;
  };
  for (int64_t J0 = 0; J0 < NT; J0 += W) {
    hipLaunchKernelGGL(k_gen_dstrip, dim3((unsigned)(W * NT * T * T)), dim3(256), 0, s, S, comp, T, NT, ts, J0, W,
                       nreal, xs, ys, qt, cst);
    const int64_t nb = pairs(J0) * T * T;
    hipLaunchKernelGGL(k_fisher_xg, dim3((unsigned)nb), dim3(256), 0, s, X, (const double*)S, Bm, T, J0, W, nreal, nb);
  }
  for (int64_t J0 = (NT - 1) / W * W; J0 >= 0; J0 -= W) {
    const int64_t nb = pairs(J0) * T * T;
    hipLaunchKernelGGL(k_fisher_mxt, dim3((unsigned)nb), dim3(256), 0, s, X, (const double*)Bm, S, T, J0, W, nreal,
                       nb);
    hipLaunchKernelGGL(k_fisher_unstage, dim3((unsigned)((W * NT * tt + 255) / 256)), dim3(256), 0, s,
                       (const double*)S, Bm, NT, ts, J0, W);
  }
}

void launch_fisher_reduce(const double* Bs, const double* Bb, const double* Bn, int64_t ts, int64_t NT, int64_t nreal,
                          const double* cst, double* part, double* out, hipStream_t s) {
  const int T = (int)(ts / BLK);
  const int64_t nl = fisher_part_blocks(ts, NT);
  hipLaunchKernelGGL(k_fisher_dot, dim3((unsigned)nl), dim3(256), 0, s, Bs, Bb, Bn, part, T, NT, ts, nreal, nl);
  hipLaunchKernelGGL(k_fisher_finalize, dim3(1), dim3(256), 0, s, (const double*)part, nl, cst, nreal, Bs ? 1 : 0,
                     out);
}

}  // namespace exg
