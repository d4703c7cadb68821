// Host-side launchers of the device kernels (one per kernel family).  All
// pointers are device pointers; every launch goes on the given stream.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace exg {


// k_matern.hip
// doubles of the per-theta table array (quadrature nodes + Chebyshev tables)
int64_t quad_table_doubles();
void launch_quad_table(const double theta[3], int metric, double nugget, double* qt, double* cst, hipStream_t s);
void launch_gen_tiles(const TileMat& M, int64_t nreal, const double* xs, const double* ys, const double* qt,
                      const double* cst, const uint8_t* tag, hipStream_t s);
void launch_gen_dense(double* cov, int64_t ldc, int64_t n, const double* x, const double* y, const double* qt,
                      const double* cst, hipStream_t s);
// r = z - Sigma a in FP64 (Sigma regenerated), sorted order, zero on padding
void launch_sigma_residual(const double* xs, const double* ys, const double* zs, const double* av, int64_t nreal,
                           int64_t npad, const double* qt, const double* cst, double* r, hipStream_t s);

// k_small.hip
void launch_sort_locations(const double* x, const double* y, const double* z, int64_t n, int64_t npad, int64_t P,
                           double* box, uint64_t* keys, double* xs, double* ys, double* zs, int32_t* perm,
                           hipStream_t s);
void launch_scatter(const double* v, const int32_t* perm, int64_t n, double* out, hipStream_t s);
void launch_potrf_blk(double* A, int64_t lda, double* dinv, double* ldpart, unsigned long long* info, int64_t col0,
                      hipStream_t s);
void launch_trsv_fwd(const TileMat& M, const double* Xd, int64_t nreal, double* rhs, double* y, hipStream_t s);
void launch_trsv_bwd(const TileMat& M, const double* Xd, double* rhs, double* a, hipStream_t s);
void launch_trmv_lower(const TileMat& M, int64_t nreal, const double* e, double* w, hipStream_t s);
void launch_finalize_loglik(const double* yv, int64_t n, const double* ldpart, int64_t nld, double* out,
                            hipStream_t s);
void launch_finalize_grad(const double* part, int64_t nparts, double* out, hipStream_t s);
// eq. (2) with the quadratic form z^T a (a = Sigma^-1 z)
void launch_finalize_loglik_za(const double* zs, const double* av, int64_t n, const double* ldpart, int64_t nld,
                               double* out, hipStream_t s);
// refinement steps on the device: y = a + d; nrm[0] = |r|^2 (trial = 0) or
// nrm[1] = (|r|^2 < nrm[0]) with nrm[0] lowered then (trial = 1); the select
// takes a_try, r_try when nrm[1] is set
void launch_add2(double* y, const double* a, const double* d, int64_t n, hipStream_t s);
void launch_resid_norm(const double* r, int64_t n, double* nrm, int trial, hipStream_t s);
void launch_refine_select(double* a, const double* a_try, double* r, const double* r_try, const double* nrm,
                          int64_t n, hipStream_t s);
void launch_fill_info(unsigned long long* info, hipStream_t s);
void launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);
void launch_copy_diag_lower(double* dst, const double* diag, int64_t ts, int64_t NT, hipStream_t s);
void launch_put_dinv(double* dst, const double* dinv, int64_t ts, int64_t NT, int c, hipStream_t s);

void launch_diag_apply_n(const double* Xk, int64_t ts, const double* b, double* out, hipStream_t s);
void launch_diag_apply_t(const double* Xk, int64_t ts, const double* b, double* out, hipStream_t s);

// k_mixed.hip
void launch_tile_bbox(const double* xs, const double* ys, int64_t ts, int64_t NT, int64_t nreal, double* box,
                      hipStream_t s);
// dmin[off_index(i, j)]: smallest distance between the real points of location
// blocks i > j (sorted, planar); corr: the correlation at that distance
void launch_tile_dmin(const double* xs, const double* ys, int64_t ts, int64_t NT, int64_t nreal, double* dmin,
                      hipStream_t s);
void launch_tile_corr(const double* dmin, int64_t NT, const double* qt, const double* cst, double* corr,
                      hipStream_t s);
void launch_panel_gather(const TileMat& M, int64_t k, const uint8_t* tag, double* pbuf, hipStream_t s);
void launch_panel_scatter(const TileMat& M, int64_t k, const uint8_t* tag, const double* pbuf, float* p32,
                          hipStream_t s);
// BF16 copy of the FP64 panel of step k, each tile transposed (k contiguous)
void launch_panel_bf16t(const TileMat& M, int64_t k, const double* pbuf, uint16_t* pbt, hipStream_t s);
// skip_bf16: BF16 targets are left to launch_update_bf16
void launch_update_lp(const TileMat& M, const uint8_t* tag, const float* p32, const uint16_t* pbt, int64_t k,
                      int64_t nreal, int part, bool skip_bf16, hipStream_t s);
// step k of the mixed update for the BF16 targets (li[e], lj[e]), e0 <= e <
// e0 + count, on 256 x 256 blocks (ts a multiple of 256); pbt: the BF16 panel
// copy of step k (tiles transposed)
void launch_update_bf16(const TileMat& M, const int32_t* li, const int32_t* lj, int64_t e0, int64_t count,
                        const uint16_t* pbt, int64_t k, int64_t nreal, hipStream_t s);
void launch_trsv_bwd_lp(const TileMat& M, const uint8_t* tag, const double* Xd, double* rhs, double* a,
                        hipStream_t s);
// one step of the mixed inverse (FP32 off-diagonal tiles of L^-1, FP32 buffer P)
// The FP64 band tiles of the mixed factor: device lists li / lj (tile (li[e],
// lj[e]), column-major order, pool slot e) and rl (list entries in row-major
// order), with host arrays of the first entry of each tile column (cfirst,
// into li / lj) and of each tile row (rfirst, into rl), NT + 1 each.
struct BandLists {
  const int32_t* li;
  const int32_t* lj;
  const int32_t* rl;
  const int64_t* cfirst;
  const int64_t* rfirst;
};
// step k of the mixed inverse (P: FP32 staging, Q: FP64 staging of the band
// tiles, each (NT - 1) ts^2 elements)
void launch_trtri_right_lp(const TileMat& M, const uint8_t* tag, const double* Xk, float* P, double* Q,
                           const BandLists& bl, int64_t k, int64_t nreal, hipStream_t s);
void launch_trtri_rest_lp(const TileMat& M, const uint8_t* tag, const double* Xk, float* P, double* Q,
                          const BandLists& bl, int64_t k, int64_t nreal, hipStream_t s);
// mixed fused LAUUM + contraction; returns the number of partial triples
int64_t launch_lauum_contract_lp(const TileMat& M, const uint8_t* tag, int64_t nreal, const double* xs,
                                 const double* ys, const double* av, const double* qt, const double* cst,
                                 const int32_t* li, const int32_t* lj, int64_t nband, double* part, hipStream_t s);
void launch_trsv_fwd_lp(const TileMat& M, const uint8_t* tag, const double* Xd, int64_t nreal, double* rhs,
                        double* y, hipStream_t s);

// k_gemm.hip
// trailing update of step k (diag_only: only the diagonal targets); part is
// an UpdatePart: all targets, the first trailing column, or the rest
void launch_chol_update(const TileMat& M, const double* below, int64_t k, int64_t nreal, bool diag_only, int part,
                        hipStream_t s);
// mixed precision: FP64 update of the band tiles (li[e], lj[e]), e0 <= e < e0 + count
void launch_band_update(const TileMat& M, const double* below, int64_t k, int64_t nreal, const int32_t* li,
                        const int32_t* lj, int64_t e0, int64_t count, hipStream_t s);
void launch_panel(double* Dk, double* below, int64_t ts, int64_t NT, int64_t k, int64_t nreal, double* dinv_k,
                  double* ldpart_k, unsigned long long* info, hipStream_t s);
void launch_diag_inverses(double* Xd, const double* diag, const double* dinv, int64_t ts, int64_t NT, hipStream_t s);
// the step's two halves: P_k and column k (any stream), then the rest
void launch_trtri_right(const TileMat& M, const double* Xk, double* P, int64_t k, int64_t nreal, hipStream_t s);
void launch_trtri_rest(const TileMat& M, const double* Xk, double* P, int64_t k, int64_t nreal, hipStream_t s);
int64_t lauum_blocks(int64_t ts, int64_t NT);
void launch_lauum_contract(const TileMat& M, int64_t nreal, const double* xs, const double* ys, const double* av,
                           const double* qt, const double* cst, double* part, hipStream_t s);

// k_predict.hip
void launch_krige_mean(const double* xs, const double* ys, const double* av, int64_t nreal, const double* xn,
                       const double* yn, int64_t m, const double* qt, const double* cst, double* mean, hipStream_t s);
// variance of new points c0 .. c0 + ncols - 1 (ncols a multiple of 128; C, V: npad x ncols, ld npad)
void launch_krige_mse(const TileMat& M, const double* Xd, const double* xs, const double* ys, int64_t nreal,
                      const double* xn, const double* yn, int64_t m, int64_t c0, int64_t ncols, const double* qt,
                      const double* cst, double* C, double* V, double* mse, hipStream_t s);

// k_fisher.hip (X: the tile matrix holding L^-1; B's: lower tiles packed by
// tile columns, n^2 / 2 doubles each)
int64_t fisher_part_blocks(int64_t ts, int64_t NT);
// doubles of the strip shared by the regenerated derivative rows and the staging
size_t fisher_strip_doubles(int64_t ts, int64_t NT);
void launch_fisher_param(const TileMat& X, int comp, int64_t nreal, const double* xs, const double* ys,
                         const double* qt, const double* cst, double* S, double* Bm, hipStream_t s);
// Bs: B_sigma2 or null (B_sigma2 = I / sigma2); part: 9 fisher_part_blocks
// doubles; out: 9 doubles (device)
void launch_fisher_reduce(const double* Bs, const double* Bb, const double* Bn, int64_t ts, int64_t NT, int64_t nreal,
                          const double* cst, double* part, double* out, hipStream_t s);

}  // namespace exg
