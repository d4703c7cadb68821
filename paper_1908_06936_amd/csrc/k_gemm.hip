// FP64 MFMA kernels of the tile algorithms.  Every kernel maps one 256-thread
// workgroup to 128 x 128 output blocks and calls the shared gemm_blk core.
//
// Cholesky (tile algorithm of Buttari, Langou, Kurzak & Dongarra, Parallel
// Computing 35, 2009, right-looking over tile columns; the paper relies on it
// through its tile library, Section 2.2):
//   panel k: a left-looking sweep over the 128-wide sub-columns c of tile
//   column k: update, factor the 128 x 128 diagonal block (k_potrf_blk),
//   then multiply the blocks below by its inverse (TRSM);
//   trailing update: A_ij -= A_ik A_jk^T for k < j <= i (SYRK on i = j).
//
// Inverse L^-1 (tile TRTRI, in place, step k): A_ik <- -A_ik X_kk (i > k);
// A_ij += A_ik A_kj (i > k > j); A_kj <- X_kk A_kj (j < k); A_kk <- X_kk, with
// X_kk the inverse of the diagonal tile, itself built from the 128-block
// inverses by the same four steps on 128-blocks.
//
// Fused LAUUM and score contraction: W = L^-T L^-1 = Sigma^-1 block by block,
// W_IJ = sum_{K >= I} X_KI^T X_KJ, contracted at once with
//   (a_i a_j / 2 - W_ij / 2) dSigma_m(i, j),  a = Sigma^-1 z,
// so W is never stored.
#include "common.h"
#include "contract.h"
#include "launch.h"

namespace exg {

// -------------------------------------------------------------- Cholesky
// trailing update of step k over the tiles (i, j), k < j <= i < NT
// below: the FP64 tiles (k+1, k), ..., (NT-1, k) of column k, contiguous.
// Mixed precision runs it only on its FP64 targets: the diagonal tiles
// (PAIRS_DIAG) and the FP64 band tiles, given as a list of (i, j) entries
// off, off + 1, ... (PAIRS_LIST; stored in the band pool).
__global__ __launch_bounds__(256, 2) void k_chol_update(TileMat M, const double* __restrict__ below, int T, int64_t k,
                                                        int64_t nreal, int64_t nb, int mode, int64_t off,
                                                        const int32_t* __restrict__ li,
                                                        const int32_t* __restrict__ lj) {
  __shared__ double sm[GEMM_LDS];
  const int64_t ts = M.ts;
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const int64_t p = b / (T * T);
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  int64_t a, c;
  if (mode == PAIRS_LIST) {
    a = li[off + p] - k - 1;
    c = lj[off + p] - k - 1;
  } else {
    pair_map(mode, off, p, &a, &c);
  }
  const int64_t i = k + 1 + a, j = k + 1 + c;
  if (i == j && u < v) return;
  if (i * ts + u * BLK >= nreal || j * ts + v * BLK >= nreal) return;  // padding: update is zero
  const double* A = below + a * ts * ts + u * BLK;
  const double* B = below + c * ts * ts + v * BLK;
  double* C = ((i == j || !M.pool) ? tptr(M, i, j) : band64(M, off_index(i, j, M.NT))) + u * BLK +
              (int64_t)v * BLK * ts;
  v4d acc[4][4];
  acc_zero(acc);
  gemm_blk<false, false, true>(A, ts, B, ts, (int)ts, acc, sm);
  acc_store(C, ts, acc, -1.0, true);
}

// panel k, sub-column c: rows g0 + blockIdx.x (128-row blocks, global index)
//   C = A[g, c] -= A[g, 0:c] A[(k,c), 0:c]^T
// The panel of column k is the diagonal tile Dk followed by the contiguous
// FP64 tiles `below`; row block g (global index) lies in tile i = g / T.
__device__ __forceinline__ double* panel_tile(double* Dk, double* below, int64_t i, int64_t k, int64_t ts) {
  return i == k ? Dk : below + (i - k - 1) * ts * ts;
}

__global__ __launch_bounds__(256, 2) void k_panel_update(double* __restrict__ Dk, double* __restrict__ below,
                                                         int64_t ts, int T, int64_t k, int c, int64_t g0) {
  __shared__ double sm[GEMM_LDS];
  const int64_t g = g0 + blockIdx.x;
  const int64_t i = g / T;
  const int u = (int)(g % T);
  double* P = panel_tile(Dk, below, i, k, ts) + u * BLK;
  const double* D = Dk + c * BLK;
  v4d acc[4][4];
  acc_zero(acc);
  gemm_blk<false, false, true>(P, ts, D, ts, c * BLK, acc, sm);
  acc_store(P + (int64_t)c * BLK * ts, ts, acc, -1.0, true);
}

// panel k, sub-column c: C = A[g, c] Dinv_c^T for the blocks below the diagonal
// block (in place: each workgroup reads only the block it overwrites)
__global__ __launch_bounds__(256, 2) void k_panel_trsm(double* __restrict__ Dk, double* __restrict__ below, int64_t ts,
                                                       int T, int64_t k, int c, int64_t g0,
                                                       const double* __restrict__ dinv) {
  __shared__ double sm[GEMM_LDS];
  const int64_t g = g0 + blockIdx.x;
  const int64_t i = g / T;
  const int u = (int)(g % T);
  double* C = panel_tile(Dk, below, i, k, ts) + u * BLK + (int64_t)c * BLK * ts;
  v4d acc[4][4];
  acc_zero(acc);
  gemm_blk<false, false>(C, ts, dinv, BLK, BLK, acc, sm);
  acc_store(C, ts, acc, 1.0, false);
}

// ------------------------------------------- inverses of the diagonal tiles
// All NT diagonal tiles at once, on copies Xd[k] (ts x ts) that start as the
// lower part of L_kk; step c of the 128-block algorithm.
// right: X[r, c] <- -X[r, c] Dinv_c for r > c
__global__ __launch_bounds__(256, 2) void k_dinv_right(double* __restrict__ Xd, const double* __restrict__ dinv,
                                                       int64_t ts, int T, int c) {
  __shared__ double sm[GEMM_LDS];
  const int nr = T - 1 - c;
  const int64_t k = blockIdx.x / nr;
  const int r = c + 1 + (int)(blockIdx.x % nr);
  double* C = Xd + k * ts * ts + r * BLK + (int64_t)c * BLK * ts;
  const double* D = dinv + (k * T + c) * BLK * BLK;
  v4d acc[4][4];
  acc_zero(acc);
  gemm_blk<false, true>(C, ts, D, BLK, BLK, acc, sm);  // Bop(n, q) = D(q, n)
  acc_store(C, ts, acc, -1.0, false);
}

// gemm: X[r, b] += X[r, c] X[c, b] for r > c > b
__global__ __launch_bounds__(256, 2) void k_dinv_gemm(double* __restrict__ Xd, int64_t ts, int T, int c) {
  __shared__ double sm[GEMM_LDS];
  const int nr = T - 1 - c;
  const int per = nr * c;
  const int64_t k = blockIdx.x / per;
  const int q = (int)(blockIdx.x % per);
  const int r = c + 1 + q / c, bb = q % c;
  double* X = Xd + k * ts * ts;
  v4d acc[4][4];
  acc_zero(acc);
  gemm_blk<false, true>(X + r * BLK + (int64_t)c * BLK * ts, ts, X + c * BLK + (int64_t)bb * BLK * ts, ts, BLK, acc,
                        sm);
  acc_store(X + r * BLK + (int64_t)bb * BLK * ts, ts, acc, 1.0, true);
}

// left: X[c, b] <- Dinv_c X[c, b] for b < c (in place)
__global__ __launch_bounds__(256, 2) void k_dinv_left(double* __restrict__ Xd, const double* __restrict__ dinv,
                                                      int64_t ts, int T, int c) {
  __shared__ double sm[GEMM_LDS];
  const int64_t k = blockIdx.x / c;
  const int bb = (int)(blockIdx.x % c);
  double* C = Xd + k * ts * ts + c * BLK + (int64_t)bb * BLK * ts;
  const double* D = dinv + (k * T + c) * BLK * BLK;
  v4d acc[4][4];
  acc_zero(acc);
  gemm_blk<false, true>(D, BLK, C, ts, BLK, acc, sm);  // Aop(m, q) = D(m, q), Bop(n, q) = C(q, n)
  acc_store(C, ts, acc, 1.0, false);
}

// --------------------------------------------------------- tile TRTRI step k
// P_i = -A_ik X_kk for i > k, into the buffer P (tile i - k - 1); one block
// (u, v) per workgroup, k range restricted to the non-zero rows v*128.. of the
// lower-triangular X_kk.
__global__ __launch_bounds__(256, 2) void k_tri_right(TileMat M, const double* __restrict__ Xk, double* __restrict__ P,
                                                      int T, int64_t k, int64_t nreal, int64_t nb) {
  const int64_t ts = M.ts;
  __shared__ double sm[GEMM_LDS];
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const int64_t i = k + 1 + b / (T * T);
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  const int64_t off = (int64_t)v * BLK * ts;
  const double* A = tptr(M, i, k) + u * BLK + off;
  double* C = P + (i - k - 1) * ts * ts + u * BLK + off;
  v4d acc[4][4];
  acc_zero(acc);
  // padded rows of L^-1 are zero: store zeros (the buffer is copied back whole)
  if (i * ts + u * BLK < nreal) gemm_blk<false, true>(A, ts, Xk + v * BLK + off, ts, (int)(ts - v * BLK), acc, sm);
  acc_store(C, ts, acc, -1.0, false);
}

// A_ij += P_i A_kj for k < i < NT, 0 <= j < k (P_i = the new A_ik)
__global__ __launch_bounds__(256, 2) void k_tri_gemm(TileMat M, const double* __restrict__ P, int T, int64_t k,
                                                     int64_t nreal, int64_t nb) {
  const int64_t ts = M.ts;
  __shared__ double sm[GEMM_LDS];
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const int64_t p = b / (T * T);
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  const int64_t i = k + 1 + p / k, j = p % k;
  if (i * ts + u * BLK >= nreal) return;
  const double* A = P + (i - k - 1) * ts * ts + u * BLK;
  const double* B = tptr(M, k, j) + (int64_t)v * BLK * ts;
  double* C = tptr(M, i, j) + u * BLK + (int64_t)v * BLK * ts;
  v4d acc[4][4];
  acc_zero(acc);
  gemm_blk<false, true>(A, ts, B, ts, (int)ts, acc, sm);
  acc_store(C, ts, acc, 1.0, true);
}

// R_j = X_kk A_kj for j < k, into the buffer P (tile j); k range restricted
// to the non-zero columns ..(u+1)*128 of row block u of X_kk.
__global__ __launch_bounds__(256, 2) void k_tri_left(TileMat M, const double* __restrict__ Xk, double* __restrict__ P,
                                                     int T, int64_t k, int64_t nb) {
  const int64_t ts = M.ts;
  __shared__ double sm[GEMM_LDS];
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const int64_t j = b / (T * T);
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  const int64_t off = (int64_t)v * BLK * ts;
  const double* B = tptr(M, k, j) + off;
  double* C = P + j * ts * ts + u * BLK + off;
  v4d acc[4][4];
  acc_zero(acc);
  gemm_blk<false, true>(Xk + u * BLK, ts, B, ts, (u + 1) * BLK, acc, sm);
  acc_store(C, ts, acc, 1.0, false);
}

// tile (i0 + q, jcol) or (irow, j0 + q) <- P tile q, q < count (column or row run)
__global__ void k_copy_back(TileMat M, const double* __restrict__ P, int64_t count, int64_t i0, int64_t j0,
                            int column) {
  const int64_t tt = M.ts * M.ts;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count * tt) return;
  const int64_t q = e / tt, o = e % tt;
  const int64_t i = column ? i0 + q : i0, j = column ? j0 : j0 + q;
  tptr(M, i, j)[o] = P[e];
}

// ------------------------------------------ tile transposition
// Every lower tile of the tile matrix transposed in place, so that the columns
// of X = L^-1 become contiguous rows for the LAUUM below (both of its operands
// are then read along their contiguous index).  One workgroup swaps the 64 x 64
// blocks (a, b) and (b, a), a <= b, of one tile through LDS.
constexpr int TB = 64;
__global__ __launch_bounds__(256) void k_transpose_tiles(TileMat M, int64_t npt, int64_t nb) {
  __shared__ double s1[TB][TB + 1];
  __shared__ double s2[TB][TB + 1];
  const int64_t g = blockIdx.x;
  if (g >= nb) return;
  const int64_t ts = M.ts;
  int64_t I, J, bq, aq;
  tri_decode(g / npt, &I, &J);
  tri_decode(g % npt, &bq, &aq);  // aq <= bq
  double* T = tptr(M, I, J);
  const int64_t ra = aq * TB, rb = bq * TB;
  for (int e = threadIdx.x; e < TB * TB; e += 256) {
    const int r = e & (TB - 1), c = e >> 6;
    s1[c][r] = T[(ra + r) + (rb + c) * ts];
    if (aq != bq) s2[c][r] = T[(rb + r) + (ra + c) * ts];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TB * TB; e += 256) {
    const int r = e & (TB - 1), c = e >> 6;
    if (aq != bq) {
      T[(ra + r) + (rb + c) * ts] = s2[r][c];
      T[(rb + r) + (ra + c) * ts] = s1[r][c];
    } else {
      T[(ra + r) + (ra + c) * ts] = s1[r][c];
    }
  }
}

// ------------------------------------------ fused LAUUM + score contraction
// Block (I, J, u, v) of W = X^T X with X = L^-1 (lower tiles, in place of L,
// each tile transposed by k_transpose_tiles),
// followed by g_m += sum (w_ij (a_i a_j - W_ij) / 2) dSigma_m(i, j) over its
// entries, w = 2 below the diagonal, 1 on it, 0 above and on padding.
// part[3 b + m] receives the block's sums (zeros for skipped blocks).
__global__ __launch_bounds__(256, 2) void k_lauum_contract(TileMat M, int T, int64_t nreal,
                                                           const double* __restrict__ xs,
                                                           const double* __restrict__ ys, const double* __restrict__ av,
                                                           const double* __restrict__ qt,
                                                           const double* __restrict__ cst, double* __restrict__ part,
                                                           int64_t nb) {
  __shared__ double sm[GEMM_LDS];
  const int64_t ts = M.ts, NT = M.NT;
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const int64_t p = b / (T * T);
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  int64_t I, J;
  tri_decode(p, &I, &J);
  // DST: dSigma is zero outside the tile band, so are those blocks' terms
  if ((I == J && u < v) || I * ts + u * BLK >= nreal || J * ts + v * BLK >= nreal || (M.dst > 0 && I - J >= M.dst)) {
    if (threadIdx.x < 3) part[3 * b + threadIdx.x] = 0.0;
    return;
  }
  v4d acc[4][4];
  acc_zero(acc);
  // One virtual k range over the tiles K = I, ..., NT-1 of tile columns I and
  // J: first rows r0.. of tile row I (X_II is lower triangular, so rows above
  // u*128 of its column block u are zero), then every row of the tiles below.
  // Transposed tiles: X(K, I)[k, m] sits at k ts + m of tile (K, I).  The
  // off-diagonal tiles of one tile column are stored one after another, so
  // row kk of the stack (K, I), K > I, is at kk ts of the stack's first tile
  // ((kk / ts) ts^2 + (kk % ts) ts = kk ts): no division per stage.
  const int64_t r0 = (int64_t)u * BLK, c0 = (int64_t)v * BLK;
  const int64_t L0 = ts - r0;
  const double* XdI = M.diag + I * ts * ts;
  const double* XbI = I + 1 < NT ? (const double*)M.off + off_index(I + 1, I, NT) * ts * ts : XdI;
  auto ap = [=](int k0) -> const double* {
    return k0 < L0 ? XdI + r0 + (r0 + k0) * ts : XbI + r0 + (int64_t)(k0 - L0) * ts;
  };
  // I > J: the tiles (I, J), (I + 1, J), ... are one stack as well
  const double* XJ = I == J ? XbI : tptr(M, I, J);
  auto bp = [=](int k0) -> const double* {
    if (I > J) return XJ + c0 + (r0 + k0) * ts;
    return k0 < L0 ? XdI + c0 + (r0 + k0) * ts : XbI + c0 + (int64_t)(k0 - L0) * ts;
  };
  gemm_core<false, false, true>(ap, ts, bp, ts, (int)(L0 + (NT - 1 - I) * ts), acc, sm);
  contract_block64(acc, I * ts + r0, J * ts + c0, nreal, xs, ys, av, qt, cst, sm, part + 3 * b);
}

// ------------------------------------------------------------- launchers
void launch_chol_update(const TileMat& M, const double* below, int64_t k, int64_t nreal, bool diag_only, int part,
                        hipStream_t s) {
  const int T = (int)(M.ts / BLK);
  int64_t m = M.NT - k - 1;  // trailing tiles
  if (M.dst > 0 && m > M.dst - 1) m = M.dst - 1;  // DST: L_ik = 0 for i - k >= dst
  if (m <= 0) return;
  int mode;
  int64_t off, npairs;
  if (diag_only) {
    mode = PAIRS_DIAG;
    off = part == UPD_REST ? 1 : 0;
    npairs = part == UPD_ALL ? m : part == UPD_FIRST_COLUMN ? 1 : m - 1;
  } else if (part == UPD_ALL) {
    mode = PAIRS_TRI, off = 0, npairs = m * (m + 1) / 2;
  } else if (part == UPD_FIRST_COLUMN) {
    mode = PAIRS_COL, off = 0, npairs = m;
  } else {
    mode = PAIRS_TRI, off = 1, npairs = (m - 1) * m / 2;
  }
  if (npairs <= 0) return;
  const int64_t nblk = npairs * T * T;
  hipLaunchKernelGGL(k_chol_update, dim3((unsigned)nblk), dim3(256), 0, s, M, below, T, k, nreal, nblk,
                     mode, off, (const int32_t*)nullptr, (const int32_t*)nullptr);
}

void launch_band_update(const TileMat& M, const double* below, int64_t k, int64_t nreal, const int32_t* li,
                        const int32_t* lj, int64_t e0, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  const int T = (int)(M.ts / BLK);
  const int64_t nblk = count * T * T;
  hipLaunchKernelGGL(k_chol_update, dim3((unsigned)nblk), dim3(256), 0, s, M, below, T, k, nreal, nblk,
                     (int)PAIRS_LIST, e0, li, lj);
}

void launch_panel(double* Dk, double* below, int64_t ts, int64_t NT, int64_t k, int64_t nreal, double* dinv_k,
                  double* ldpart_k, unsigned long long* info, hipStream_t s) {
  const int T = (int)(ts / BLK);
  const int64_t gmax = (nreal + BLK - 1) / BLK;  // blocks holding real rows
  (void)NT;
  for (int c = 0; c < T; ++c) {
    const int64_t gd = k * T + c;  // global index of the diagonal block
    if (c > 0 && gmax > gd)
      hipLaunchKernelGGL(k_panel_update, dim3((unsigned)(gmax - gd)), dim3(256), 0, s, Dk, below, ts, T, k, c, gd);
    double* Dblk = Dk + c * BLK + (int64_t)c * BLK * ts;
    launch_potrf_blk(Dblk, ts, dinv_k + (int64_t)c * BLK * BLK, ldpart_k + c, info, gd * BLK, s);
    if (gmax > gd + 1)
      hipLaunchKernelGGL(k_panel_trsm, dim3((unsigned)(gmax - gd - 1)), dim3(256), 0, s, Dk, below, ts, T, k, c,
                         gd + 1, dinv_k + (int64_t)c * BLK * BLK);
  }
}

void launch_diag_inverses(double* Xd, const double* diag, const double* dinv, int64_t ts, int64_t NT, hipStream_t s) {
  const int T = (int)(ts / BLK);
  launch_copy_diag_lower(Xd, diag, ts, NT, s);
  for (int c = 0; c < T; ++c) {
    if (T - 1 - c > 0)
      hipLaunchKernelGGL(k_dinv_right, dim3((unsigned)(NT * (T - 1 - c))), dim3(256), 0, s, Xd, dinv, ts, T, c);
    if (T - 1 - c > 0 && c > 0)
      hipLaunchKernelGGL(k_dinv_gemm, dim3((unsigned)(NT * (T - 1 - c) * c)), dim3(256), 0, s, Xd, ts, T, c);
    if (c > 0) hipLaunchKernelGGL(k_dinv_left, dim3((unsigned)(NT * c)), dim3(256), 0, s, Xd, dinv, ts, T, c);
    launch_put_dinv(Xd, dinv, ts, NT, c, s);
  }
}

// Step k of the in-place tile inverse X = L^-1 (after this step rows 0..k of
// X are final), in two halves for two streams.  The first half (P_i = -A_ik
// X_kk into P, then column k <- P) reads only column k of L and X_kk, which no
// earlier step writes, so step k + 1's first half can run beside step k's
// second half (A_ij += P_i A_kj left of column k, row k <- X_kk A_kj, the
// diagonal tile <- X_kk) when the two use different staging buffers.
void launch_trtri_right(const TileMat& M, const double* Xk, double* P, int64_t k, int64_t nreal, hipStream_t s) {
  const int64_t ts = M.ts, NT = M.NT;
  const int T = (int)(ts / BLK);
  const int64_t nbelow = NT - k - 1;
  if (nbelow <= 0) return;
  const int64_t nr = nbelow * T * T;
  hipLaunchKernelGGL(k_tri_right, dim3((unsigned)nr), dim3(256), 0, s, M, Xk, P, T, k, nreal, nr);
  hipLaunchKernelGGL(k_copy_back, dim3((unsigned)((nbelow * ts * ts + 255) / 256)), dim3(256), 0, s, M, P, nbelow,
                     k + 1, k, 1);
}

void launch_trtri_rest(const TileMat& M, const double* Xk, double* P, int64_t k, int64_t nreal, hipStream_t s) {
  const int64_t ts = M.ts, NT = M.NT;
  const int T = (int)(ts / BLK);
  const int64_t tt = ts * ts;
  const int64_t nbelow = NT - k - 1;
  if (nbelow > 0 && k > 0) {
    const int64_t ng = nbelow * k * T * T;
    hipLaunchKernelGGL(k_tri_gemm, dim3((unsigned)ng), dim3(256), 0, s, M, P, T, k, nreal, ng);
  }
  if (k > 0) {
    const int64_t nl = k * T * T;
    hipLaunchKernelGGL(k_tri_left, dim3((unsigned)nl), dim3(256), 0, s, M, Xk, P, T, k, nl);
    hipLaunchKernelGGL(k_copy_back, dim3((unsigned)((k * tt + 255) / 256)), dim3(256), 0, s, M, P, k, k, (int64_t)0,
                       0);
  }
  launch_copy(M.diag + k * tt, Xk, tt, s);
}

int64_t lauum_blocks(int64_t ts, int64_t NT) {
  const int64_t T = ts / BLK;
  return NT * (NT + 1) / 2 * T * T;
}

void launch_lauum_contract(const TileMat& M, int64_t nreal, const double* xs, const double* ys, const double* av,
                           const double* qt, const double* cst, double* part, hipStream_t s) {
  const int T = (int)(M.ts / BLK);
  const int64_t t64 = M.ts / TB, npt = t64 * (t64 + 1) / 2, ntr = M.NT * (M.NT + 1) / 2 * npt;
  hipLaunchKernelGGL(k_transpose_tiles, dim3((unsigned)ntr), dim3(256), 0, s, M, npt, ntr);
  const int64_t nb = lauum_blocks(M.ts, M.NT);
  hipLaunchKernelGGL(k_lauum_contract, dim3((unsigned)nb), dim3(256), 0, s, M, T, nreal, xs, ys, av, qt, cst, part,
                     nb);
}

}  // namespace exg
