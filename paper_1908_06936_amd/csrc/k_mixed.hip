// Mixed-precision tile Cholesky (paper Section 2.1, Fig. 1(d): off-diagonal
// tiles held in single or half precision, diagonal tiles in double).
//
// Storage: diagonal tiles FP64; off-diagonal tile (i, j) in a 4-byte slot per
// entry, as FP32 (tag 0) or as BF16 in the first half of the slot (tag 1), or,
// for the FP64 band near the diagonal (tag 2), in a pool of FP64 tiles.
// Step k of the factorisation:
//   1. the column-k tiles below the diagonal are widened into an FP64 panel
//      buffer, the panel is factored by the FP64 kernels and written back,
//      rounded to nearest even into each tile's precision and, for the
//      update, to FP32 (and BF16, transposed) in panel copies;
//   2. diagonal and FP64 band targets A_ij -= A_ik A_jk^T run on FP64 MFMA
//      from the FP64 panel buffer (k_chol_update);
//   3. FP32 targets run on FP32 MFMA with FP32 accumulation from the FP32
//      panel copy (k_update_lp); BF16 targets on BF16 MFMA with FP32
//      accumulation from the BF16 copy, widened exactly and rounded back to
//      nearest even (k_update_bf16 in k_bf16.hip, or k_update_lp).
// The solves read the stored tiles and accumulate in FP64; log det Sigma and
// z^T Sigma^-1 z are FP64 sums.  The inverse factor and the fused LAUUM for
// the score follow the same precision map (below).
#include <float.h>

#include "common.h"
#include "contract.h"
#include "gemm32.h"
#include "launch.h"
#include "matern_dev.h"
#include "solve.h"

namespace exg {


__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return bf16_bits_to_f32(h); }
__device__ __forceinline__ uint16_t f32_to_bf16(float f) { return f32_to_bf16_rne(f); }

// C(m, n) += alpha acc over one 128 x 128 block of the off-diagonal tile
// whose slot starts at `tile` (in-tile element offset o0 of the block's first
// entry, leading dimension ld): FP32 tiles in place, BF16 tiles (first half of
// the slot) widened, updated and rounded to nearest even.  The 16 values of
// one accumulator are loaded before any is stored, so that the loads are not
// waited for one by one.
__device__ __forceinline__ void acc32_update(void* tile, bool bf, int64_t o0, int64_t ld, const v16f (&acc)[2][2],
                                             float alpha) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int m = wr * 64 + 32 * x + (lane & 31);
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int64_t ob = o0 + m + (int64_t)(wc * 64 + 32 * y + 4 * (lane >> 5)) * ld;
      if (!bf) {
        float* C = (float*)tile + ob;
        float old[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) old[r] = C[(int64_t)(8 * (r >> 2) + (r & 3)) * ld];
#pragma unroll
        for (int r = 0; r < 16; ++r) C[(int64_t)(8 * (r >> 2) + (r & 3)) * ld] = old[r] + alpha * acc[x][y][r];
      } else {
        uint16_t* Ch = (uint16_t*)tile + ob;
        uint16_t old[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) old[r] = Ch[(int64_t)(8 * (r >> 2) + (r & 3)) * ld];
#pragma unroll
        for (int r = 0; r < 16; ++r)
          Ch[(int64_t)(8 * (r >> 2) + (r & 3)) * ld] = f32_to_bf16(bf16_to_f32(old[r]) + alpha * acc[x][y][r]);
      }
    }
  }
}

// C(m, n) = alpha acc into a 128 x 128 block of an FP32 array
__device__ __forceinline__ void acc32_store(float* C, int64_t ld, const v16f (&acc)[2][2], float alpha) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int m = wr * 64 + 32 * x + (lane & 31);
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int n = wc * 64 + 32 * y + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        C[m + (int64_t)n * ld] = alpha * acc[x][y][r];
      }
  }
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

// dmin[off_index(i, j)] = the smallest distance between a real point of
// location block i and one of block j, i > j (planar coordinates): one
// workgroup per tile pair, block j's points staged in LDS, a min-reduction.
// It depends on the sorted locations only, so an estimation computes it once.
__global__ __launch_bounds__(256) void k_tile_dmin(const double* __restrict__ xs, const double* __restrict__ ys,
                                                   int64_t ts, int64_t NT, int64_t nreal, double* __restrict__ dmin) {
  extern __shared__ double sp[];  // 2 ts: block j's x then y
  __shared__ double red[256];
  const int64_t p = blockIdx.x;
  int64_t a, b;
  tri_decode(p, &a, &b);  // b <= a < NT - 1
  const int64_t i = a + 1, j = b;
  const int t = threadIdx.x;
  const int64_t nj = nreal - j * ts < ts ? nreal - j * ts : ts;
  const int64_t ni = nreal - i * ts < ts ? nreal - i * ts : ts;
  for (int64_t q = t; q < nj; q += 256) {
    sp[q] = xs[j * ts + q];
    sp[ts + q] = ys[j * ts + q];
  }
  __syncthreads();
  double m = DBL_MAX;
  for (int64_t q = t; q < ni; q += 256) {
    const double px = xs[i * ts + q], py = ys[i * ts + q];
    for (int64_t r = 0; r < nj; ++r) {
      const double dx = px - sp[r], dy = py - sp[ts + r];
      m = fmin(m, dx * dx + dy * dy);
    }
  }
  red[t] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) red[t] = fmin(red[t], red[t + s]);
    __syncthreads();
  }
  if (t == 0) dmin[off_index(i, j, NT)] = sqrt(red[0]);
}

// corr[q] = the Matern correlation at distance dmin[q] for every off-diagonal
// tile: the largest |Sigma_ab| / sigma^2 of the tile, since the correlation
// decreases with distance
__global__ __launch_bounds__(256) void k_tile_corr(const double* __restrict__ dmin, int64_t noff,
                                                   const double* __restrict__ qt, const double* __restrict__ cst,
                                                   double* __restrict__ corr) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= noff) return;
  corr[q] = matern_value(dmin[q], cst, qt) / cst[C_S2];
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
  const int tg = tag[idx];
  pbuf[e] = tg == TAG_F64 ? band64(M, idx)[o]
                          : (tg == TAG_BF16 ? (double)bf16_to_f32(((const uint16_t*)src)[o]) : (double)src[o]);
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
  const int tg = tag[idx];
  if (tg == TAG_F64)
    band64(M, idx)[o] = pbuf[e];
  else if (tg == TAG_BF16)
    ((uint16_t*)dst)[o] = f32_to_bf16(f);
  else
    dst[o] = f;
}

// pbt tile q = pbuf tile q rounded to BF16 (nearest even, through FP32) and
// transposed, so that the BF16 update reads its operands k contiguous:
// element (m, kk) of tile q at pbt[q ts^2 + m ts + kk].  One 64 x 64 block
// per workgroup, transposed through LDS.
__global__ __launch_bounds__(256) void k_panel_bf16t(const double* __restrict__ pbuf, uint16_t* __restrict__ pbt,
                                                     int64_t ts, int64_t count) {
  __shared__ uint16_t sb[64][66];
  const int64_t nb = ts / 64;
  const int64_t b = blockIdx.x;
  if (b >= count * nb * nb) return;
  const int64_t q = b / (nb * nb), r = b % (nb * nb);
  const int64_t m0 = (r % nb) * 64, k0 = (r / nb) * 64;
  const double* src = pbuf + q * ts * ts;
  uint16_t* dst = pbt + q * ts * ts;
  const int t = threadIdx.x;
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int m = t & 63, kk = (t >> 6) + 4 * p;
    sb[kk][m] = f32_to_bf16((float)src[(m0 + m) + (k0 + kk) * ts]);
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int kk = t & 63, m = (t >> 6) + 4 * p;
    dst[(m0 + m) * ts + k0 + kk] = sb[kk][m];
  }
}

// ------------------------------------------- low-precision trailing update
// C_ij -= L_ik L_jk^T for the off-diagonal targets k < j < i < NT.  FP32
// targets run on FP32 MFMA with operands rounded to FP32 from the FP64 panel
// (p32 tile q holds L_{k+1+q, k}), so that a BF16-stored panel tile never
// feeds its rounding error into targets near the diagonal; BF16 targets run
// on BF16 MFMA with FP32 accumulation from the BF16 transposed panel copy pbt
// (null when the step has no BF16 targets); FP64 band targets are skipped.  One 256-thread block computes
// one 128 x 128 block of a target tile.
__global__ __launch_bounds__(256, 2) void k_update_lp(TileMat M, const uint8_t* __restrict__ tag,
                                                      const float* __restrict__ p32,
                                                      const uint16_t* __restrict__ pbt, int T, int64_t k,
                                                      int64_t nreal, int64_t nb, int mode, int64_t off,
                                                      int skip_bf16) {
  constexpr int SMB = G32_LDS * 4 > GB_LDS_BYTES ? G32_LDS * 4 : GB_LDS_BYTES;
  __shared__ __attribute__((aligned(16))) char smraw[SMB];
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
  const int64_t ic = off_index(i, j, M.NT);
  const int tg = tag[ic];
  if (tg == TAG_F64) return;  // FP64 band target: updated by the FP64 kernel
  if (tg == TAG_BF16 && skip_bf16) return;  // on the 256 x 256 BF16 kernel
  float* C = (float*)M.off + ic * tt;
  if (tg == TAG_BF16 && pbt) {
    v4f acc[4][4];
    accb_zero(acc);
    const uint16_t* A = pbt + (a + 1) * tt + (int64_t)u * BLK * ts;
    const uint16_t* B = pbt + c * tt + (int64_t)v * BLK * ts;
    gemm_bf16([=](int k0) { return A + k0; }, ts, [=](int k0) { return B + k0; }, ts, (int)ts, acc,
              (uint16_t*)smraw);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wr = w >> 1, wc = w & 1;
    uint16_t* Ch = (uint16_t*)C + u * BLK + (int64_t)v * BLK * ts;
    // the 16 values of one row group are loaded before any is stored
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int m = wr * 64 + 16 * x + (lane & 15);
      uint16_t old[4][4];
#pragma unroll
      for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) old[y][r] = Ch[m + (int64_t)(wc * 64 + 16 * y + 4 * (lane >> 4) + r) * ts];
#pragma unroll
      for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          Ch[m + (int64_t)(wc * 64 + 16 * y + 4 * (lane >> 4) + r) * ts] =
              f32_to_bf16(bf16_to_f32(old[y][r]) - acc[x][y][r]);
    }
  } else {
    v16f acc[2][2];
    acc32_zero(acc);
    gemm32_blk<SRC_F32, false, SRC_F32, false>(p32 + (a + 1) * tt + u * BLK, ts, p32 + c * tt + v * BLK, ts, (int)ts,
                                                acc, (float*)smraw);
    acc32_update(C, tg == TAG_BF16, u * BLK + (int64_t)v * BLK * ts, ts, acc, -1.f);
  }
}

// ------------------------------------------------- solves on mixed tiles
// rhs_i -= L_ik y_k for the 128-row blocks g0 <= g < gmax below tile k,
// reading FP32 or BF16 tiles and accumulating in FP64
__global__ __launch_bounds__(SOLVE_THREADS) void k_gemv_fwd_lp(TileMat M, const uint8_t* __restrict__ tag, int64_t k,
                                                              int64_t g0, const double* __restrict__ yk,
                                                              double* __restrict__ rhs) {
  extern __shared__ double sy[];  // ts + SOLVE_THREADS
  const int64_t ts = M.ts;
  double* red = sy + ts;
  const int T = (int)(ts / BLK);
  const int64_t g = g0 + blockIdx.x;
  const int64_t i = g / T;
  const int u = (int)(g % T);
  const int t = threadIdx.x;
  for (int q = t; q < ts; q += SOLVE_THREADS) sy[q] = yk[q];
  __syncthreads();
  const int64_t idx = off_index(i, k, M.NT);
  const float* L = (const float*)M.off + idx * ts * ts;
  const int tg = tag[idx];
  double s;
  if (tg == TAG_F64) {
    const double* Ld = band64(M, idx) + u * BLK;
    s = slab_rowdot([=](int r, int c) { return Ld[r + (int64_t)c * ts]; }, sy, (int)ts, red);
  } else if (tg == TAG_BF16) {
    const uint16_t* Lh = (const uint16_t*)L + u * BLK;
    s = slab_rowdot([=](int r, int c) { return (double)bf16_to_f32(Lh[r + (int64_t)c * ts]); }, sy, (int)ts, red);
  } else {
    const float* Lf = L + u * BLK;
    s = slab_rowdot([=](int r, int c) { return (double)Lf[r + (int64_t)c * ts]; }, sy, (int)ts, red);
  }
  if (t < BLK) rhs[i * ts + u * BLK + t] -= s;
}

// rhs_j -= L_kj^T a_k over the 128-column blocks of the tiles j < k (one block
// per workgroup), reading FP32 or BF16 tiles and accumulating in FP64
__global__ __launch_bounds__(SOLVE_THREADS) void k_gemv_bwd_lp(TileMat M, const uint8_t* __restrict__ tag, int64_t k,
                                                              const double* __restrict__ ak,
                                                              double* __restrict__ rhs) {
  const int64_t ts = M.ts;
  const int T = (int)(ts / BLK);
  const int64_t cb = blockIdx.x;
  const int64_t j = cb / T;
  const int64_t col0 = (cb % T) * BLK + 8 * (threadIdx.x >> 6);
  const int64_t idx = off_index(k, j, M.NT);
  const float* L = (const float*)M.off + idx * ts * ts;
  const int tg = tag[idx];
  double s[8];
  if (tg == TAG_F64) {
    const double* Ld = band64(M, idx);
    wave_coldot8([=](int64_t r, int64_t c) { return Ld[r + c * ts]; }, ak, col0, false, ts, s);
  } else if (tg == TAG_BF16) {
    const uint16_t* Lh = (const uint16_t*)L;
    wave_coldot8([=](int64_t r, int64_t c) { return (double)bf16_to_f32(Lh[r + c * ts]); }, ak, col0, false, ts, s);
  } else {
    wave_coldot8([=](int64_t r, int64_t c) { return (double)L[r + c * ts]; }, ak, col0, false, ts, s);
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) rhs[j * ts + col0 + e] -= s[e];
  }
}

// ------------------------------------- FP64 MFMA core over mixed operands
// gemm_core's block product (same lane layout, stages, double buffering and
// order of the products) for operands whose element type changes along k:
// aptr(k0) / bptr(k0) return the address of Op(0, k0) for one BK-deep stage
// and whether the elements there are FP64 or FP32 (uniform over the
// workgroup; FP32 widened exactly at the LDS store).  One instantiation covers
// every mix, which keeps a kernel with several tile precisions to one copy of
// the k loop.
struct MixPtr {
  const void* p;
  bool f64;
};

template <bool AKC, bool BKC, class AP, class BP>
__device__ __forceinline__ void gemm_core_mix(AP aptr, int64_t lda, BP bptr, int64_t ldb, int K, v4d (&acc)[4][4],
                                              double* sm) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  double* sA = sm;
  double* sB = sm + 2 * BK * LDP;
  // a register set: four element pairs per operand, raw (two doubles, or two
  // floats in the first 8 bytes) and the element type of the stage
  typedef uint32_t e4 __attribute__((ext_vector_type(4)));
  typedef uint32_t e2 __attribute__((ext_vector_type(2)));
  struct Set {
    e4 a[4], b[4];
    bool fa, fb;
  };
  Set r0, r1;
  // element offsets of the thread's pairs within a stage (fixed for the whole
  // k range); each stage's base address is the same in every lane and is held
  // in scalar registers, the byte offset is the element offset shifted by the
  // stage's element size (127 ld + 15 elements must stay below 2^29)
  uint32_t ea[4], eb[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int idx = t + GEMM_THREADS * s;
    ea[s] = (uint32_t)(AKC ? 2 * (idx & 7) + (int64_t)(idx >> 3) * lda : 2 * (idx & 63) + (int64_t)(idx >> 6) * lda);
    eb[s] = (uint32_t)(BKC ? 2 * (idx & 7) + (int64_t)(idx >> 3) * ldb : 2 * (idx & 63) + (int64_t)(idx >> 6) * ldb);
  }
  typedef __attribute__((address_space(1))) const e4 g4;
  typedef __attribute__((address_space(1))) const e2 g2;
  auto gload = [&](int k0, Set& r) {
    const MixPtr A = aptr(k0), B = bptr(k0);
    gbyte* pa = uniform_base(A.p);
    gbyte* pb = uniform_base(B.p);
    r.fa = A.f64;
    r.fb = B.f64;
    if (A.f64) {
#pragma unroll
      for (int s = 0; s < 4; ++s) r.a[s] = *(g4*)(pa + (ea[s] << 3));
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const e2 f = *(g2*)(pa + (ea[s] << 2));
        r.a[s].x = f.x, r.a[s].y = f.y;
      }
    }
    if (B.f64) {
#pragma unroll
      for (int s = 0; s < 4; ++s) r.b[s] = *(g4*)(pb + (eb[s] << 3));
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const e2 f = *(g2*)(pb + (eb[s] << 2));
        r.b[s].x = f.x, r.b[s].y = f.y;
      }
    }
  };
  auto widen = [](const e4& u, bool f64) -> d2 {
    if (f64) return (d2){__hiloint2double((int)u.y, (int)u.x), __hiloint2double((int)u.w, (int)u.z)};
    return (d2){(double)__uint_as_float(u.x), (double)__uint_as_float(u.y)};
  };
  auto put = [&](double* S, bool kc, int idx, d2 v) {
    if (!kc) {
      *(d2*)(S + (idx >> 6) * LDP + 2 * (idx & 63)) = v;
    } else {
      const int m = idx >> 3, kp = idx & 7;
      S[(2 * kp) * LDP + m] = v.x;
      S[(2 * kp + 1) * LDP + m] = v.y;
    }
  };
  auto sstore = [&](int buf, const Set& r) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int idx = t + GEMM_THREADS * s;
      put(sA + buf * BK * LDP, AKC, idx, widen(r.a[s], r.fa));
      put(sB + buf * BK * LDP, BKC, idx, widen(r.b[s], r.fb));
    }
  };
  auto compute = [&](int cur) {
    const double* a = sA + cur * BK * LDP + wr * 64 + (lane & 15);
    const double* b = sB + cur * BK * LDP + wc * 64 + (lane & 15);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int ko = (kk + (lane >> 4)) * LDP;
      double af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = a[ko + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = b[ko + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma64(bf[j], af[i], acc[i][j]);
    }
  };
  const int nst = K / BK;  // even
  gload(0, r0);
  gload(BK, r1);
  sstore(0, r0);
  __syncthreads();
  for (int st = 0; st < nst; st += 2) {
    if (st + 2 < nst) gload((st + 2) * BK, r0);
    compute(0);
    sstore(1, r1);
    __syncthreads();
    if (st + 3 < nst) gload((st + 3) * BK, r1);
    compute(1);
    if (st + 2 < nst) sstore(0, r0);
    __syncthreads();
  }
}

// ------------------------------------------------ mixed tile TRTRI, step k
// The same four steps as the FP64 inverse.  L^-1 follows the precision map of
// the factor: a tile of the FP64 band (tag FP64) stays FP64 in its pool slot,
// every product into it runs on FP64 MFMA (FP32 operands widened exactly), and
// its FP32 rounding is kept in the tile's 4-byte slot for the FP32 readers of
// the finished inverse; every other off-diagonal tile is FP32 (the 4-byte
// slots take FP32 whatever the tile's tag was: a tile is read through its tag
// only as an untouched factor tile, in the first step below, and is FP32 from
// then on) with its products on FP32 MFMA.  The band tiles carry the largest
// entries of L^-1, and their FP32 sums were the main error of the score's
// trace term.  The FP32 kernels below skip band targets; the *_band kernels
// take them, staging in the FP64 buffer Q (same tile positions as P) and
// writing the FP32 rounding into P, so that P stays complete for the FP32
// readers.
// P_i = -L_ik X_kk for i > k into the FP32 buffer P (tile i - k - 1); k range
// restricted to the non-zero rows v*128.. of the lower-triangular X_kk.
__global__ __launch_bounds__(256, 2) void k_tri_right_lp(TileMat M, const uint8_t* __restrict__ tag,
                                                         const double* __restrict__ Xk, float* __restrict__ P, int T,
                                                         int64_t k, int64_t nreal, int64_t nb) {
  __shared__ float sm[G32_LDS];
  const int64_t ts = M.ts, tt = ts * ts;
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const int64_t i = k + 1 + b / (T * T);
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  const int64_t off = (int64_t)v * BLK * ts;
  const int64_t idx = off_index(i, k, M.NT);
  const int tg = tag[idx];
  if (tg == TAG_F64) return;  // k_tri_right_band
  float* C = P + (i - k - 1) * tt + u * BLK + off;
  v16f acc[2][2];
  acc32_zero(acc);
  // padded rows of L^-1 are zero: store zeros (the buffer is copied back whole)
  if (i * ts + u * BLK < nreal) {
    const float* A = (const float*)M.off + idx * tt;
    const double* B = Xk + v * BLK + off;
    const int K = (int)(ts - v * BLK);
    if (tg == TAG_BF16)
      gemm32_blk<SRC_BF16, false, SRC_F64, true>((const uint16_t*)A + u * BLK + off, ts, B, ts, K, acc, sm);
    else
      gemm32_blk<SRC_F32, false, SRC_F64, true>(A + u * BLK + off, ts, B, ts, K, acc, sm);
  }
  acc32_store(C, ts, acc, -1.f);
}

// A_ij += P_i A_kj for k < i < NT, 0 <= j < k (P_i = the new A_ik), FP32
// targets; A_kj of a band tile is read from its FP64 slot
__global__ __launch_bounds__(256, 2) void k_tri_gemm_lp(TileMat M, const uint8_t* __restrict__ tag,
                                                        const float* __restrict__ P, int T, int64_t k, int64_t nreal,
                                                        int64_t nb) {
  __shared__ float sm[G32_LDS];
  const int64_t ts = M.ts, tt = ts * ts;
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const int64_t p = b / (T * T);
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  const int64_t i = k + 1 + p / k, j = p % k;
  if (i * ts + u * BLK >= nreal || tag[off_index(i, j, M.NT)] == TAG_F64) return;
  v16f acc[2][2];
  acc32_zero(acc);
  const float* A = P + (i - k - 1) * tt + u * BLK;
  const int64_t kj = off_index(k, j, M.NT), ob = (int64_t)v * BLK * ts;
  if (tag[kj] == TAG_F64)
    gemm32_blk<SRC_F32, false, SRC_F64, true>(A, ts, band64(M, kj) + ob, ts, (int)ts, acc, sm);
  else
    gemm32_blk<SRC_F32, false, SRC_F32, true>(A, ts, off32(M, k, j) + ob, ts, (int)ts, acc, sm);
  acc32_update(off32(M, i, j), false, u * BLK + ob, ts, acc, 1.f);
}

// R_j = X_kk A_kj for j < k into the FP32 buffer P (tile j); k range
// restricted to the non-zero columns ..(u+1)*128 of row block u of X_kk.
// Band tiles (k, j) are left to k_tri_left_band.
__global__ __launch_bounds__(256, 2) void k_tri_left_lp(TileMat M, const uint8_t* __restrict__ tag,
                                                        const double* __restrict__ Xk, float* __restrict__ P, int T,
                                                        int64_t k, int64_t nb) {
  __shared__ float sm[G32_LDS];
  const int64_t ts = M.ts, tt = ts * ts;
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const int64_t j = b / (T * T);
  if (tag[off_index(k, j, M.NT)] == TAG_F64) return;
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  const int64_t off = (int64_t)v * BLK * ts;
  v16f acc[2][2];
  acc32_zero(acc);
  gemm32_blk<SRC_F64, false, SRC_F32, true>(Xk + u * BLK, ts, off32(M, k, j) + off, ts, (u + 1) * BLK, acc, sm);
  acc32_store(P + j * tt + u * BLK + off, ts, acc, 1.f);
}

// C = alpha acc into a 128 x 128 block of an FP64 array and its FP32 rounding
// into the same place of an FP32 array (acc_store's lane assignment)
__device__ __forceinline__ void acc_store_pair(double* C, float* C32, int64_t ldc, const v4d (&acc)[4][4],
                                               double alpha) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = wr * 64 + 16 * i + (lane & 15);
    const int64_t o = m + (int64_t)(wc * 64 + (lane >> 4)) * ldc;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double v = alpha * acc[i][j][r];
        const int64_t e = o + (int64_t)(16 * j + 4 * r) * ldc;
        C[e] = v;
        C32[e] = (float)v;
      }
  }
}

// Band tiles of column k: P_i = -L_ik X_kk on FP64 MFMA for the list entries
// e0 + q (tile (li[e0 + q], k)), into Q and its FP32 rounding into P.
__global__ __launch_bounds__(256, 2) void k_tri_right_band(TileMat M, const double* __restrict__ Xk,
                                                           double* __restrict__ Q, float* __restrict__ P,
                                                           const int32_t* __restrict__ li, int64_t e0, int T,
                                                           int64_t k, int64_t nreal, int64_t nb) {
  __shared__ double sm[GEMM_LDS];
  const int64_t ts = M.ts, tt = ts * ts;
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const int64_t i = li[e0 + b / (T * T)];
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  const int64_t off = (int64_t)v * BLK * ts, o = (i - k - 1) * tt + u * BLK + off;
  v4d acc[4][4];
  acc_zero(acc);
  if (i * ts + u * BLK < nreal)
    gemm_blk<false, true, true>(band64(M, off_index(i, k, M.NT)) + u * BLK + off, ts, Xk + v * BLK + off, ts,
                          (int)(ts - v * BLK), acc, sm);
  acc_store_pair(Q + o, P + o, ts, acc, -1.0);
}

// Band targets of step k: A_ij += P_i A_kj for the list entries e < e1 (the
// band tiles of columns j < k) with li[e] > k, on FP64 MFMA; P_i from Q where
// (i, k) is a band tile, else from P, and A_kj from the FP64 slot where (k, j)
// is a band tile, else from the FP32 slot.
__global__ __launch_bounds__(256, 2) void k_tri_gemm_band(TileMat M, const uint8_t* __restrict__ tag,
                                                          const double* __restrict__ Q, const float* __restrict__ P,
                                                          const int32_t* __restrict__ li,
                                                          const int32_t* __restrict__ lj, int T, int64_t k,
                                                          int64_t nreal, int64_t nb) {
  __shared__ double sm[GEMM_LDS];
  const int64_t ts = M.ts, tt = ts * ts, NT = M.NT;
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const int64_t e = b / (T * T);
  const int64_t i = li[e], j = lj[e];
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  if (i <= k || i * ts + u * BLK >= nreal) return;
  v4d acc[4][4];
  acc_zero(acc);
  const int64_t oa = (i - k - 1) * tt + u * BLK, ob = (int64_t)v * BLK * ts;
  const int64_t kj = off_index(k, j, NT);
  const bool a64 = tag[off_index(i, k, NT)] == TAG_F64, b64 = tag[kj] == TAG_F64;
  // byte addresses and log2 of the element size of both operands
  const char* A = a64 ? (const char*)(Q + oa) : (const char*)(P + oa);
  const char* B = b64 ? (const char*)(band64(M, kj) + ob) : (const char*)(off32(M, k, j) + ob);
  const int sa = a64 ? 3 : 2, sb = b64 ? 3 : 2;
  gemm_core_mix<false, true>([=](int k0) { return MixPtr{A + (((int64_t)k0 * ts) << sa), a64}; }, ts,
                             [=](int k0) { return MixPtr{B + ((int64_t)k0 << sb), b64}; }, ts, (int)ts, acc, sm);
  acc_store(band64(M, off_index(i, j, NT)) + u * BLK + ob, ts, acc, 1.0, true);
}

// Band tiles of row k: R_j = X_kk A_kj on FP64 MFMA for the row-list entries
// rl[r0 + q] (tile (k, lj[.])), into Q and its FP32 rounding into P (tile j).
__global__ __launch_bounds__(256, 2) void k_tri_left_band(TileMat M, const double* __restrict__ Xk,
                                                          double* __restrict__ Q, float* __restrict__ P,
                                                          const int32_t* __restrict__ lj,
                                                          const int32_t* __restrict__ rl, int64_t r0, int T,
                                                          int64_t k, int64_t nb) {
  __shared__ double sm[GEMM_LDS];
  const int64_t ts = M.ts, tt = ts * ts;
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const int64_t j = lj[rl[r0 + b / (T * T)]];
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  const int64_t off = (int64_t)v * BLK * ts, o = j * tt + u * BLK + off;
  v4d acc[4][4];
  acc_zero(acc);
  gemm_blk<false, true>(Xk + u * BLK, ts, band64(M, off_index(k, j, M.NT)) + off, ts, (u + 1) * BLK, acc, sm);
  acc_store_pair(Q + o, P + o, ts, acc, 1.0);
}

// FP64 slots of band tiles <- Q: column mode, tiles (li[e0 + q], k) from Q tile
// li - k - 1; row mode, tiles (k, lj[rl[e0 + q]]) from Q tile lj; q < count
__global__ void k_copy_back_band(TileMat M, const double* __restrict__ Q, const int32_t* __restrict__ li,
                                 const int32_t* __restrict__ lj, const int32_t* __restrict__ rl, int64_t e0,
                                 int64_t count, int64_t k, int column) {
  const int64_t tt = M.ts * M.ts;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count * tt) return;
  const int64_t q = e / tt, o = e % tt;
  int64_t i, j, src;
  if (column) {
    i = li[e0 + q], j = k, src = i - k - 1;
  } else {
    i = k, j = lj[rl[e0 + q]], src = j;
  }
  band64(M, off_index(i, j, M.NT))[o] = Q[src * tt + o];
}

// FP32 tile (i0 + q, jcol) or (irow, j0 + q) <- P tile q, q < count
__global__ void k_copy_back_lp(TileMat M, const float* __restrict__ P, int64_t count, int64_t i0, int64_t j0,
                               int column) {
  const int64_t tt = M.ts * M.ts;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count * tt) return;
  const int64_t q = e / tt, o = e % tt;
  const int64_t i = column ? i0 + q : i0, j = column ? j0 : j0 + q;
  off32(M, i, j)[o] = P[e];
}

// ------------------------------------------ tile transposition (mixed)
// Every lower tile of X = L^-1 in mixed storage (FP64 diagonal tiles, FP32
// off-diagonal slots, FP64 band slots) transposed in place, as the FP64 path
// does, so that both LAUUM operands are read along their contiguous index.
// One workgroup swaps the 64 x 64 blocks (a, b) and (b, a), a <= b, of one
// tile through LDS.
template <typename E>
__device__ __forceinline__ void swap_blocks64(E* T, int64_t ts, int64_t ra, int64_t rb, bool same, E (*s1)[65],
                                              E (*s2)[65]) {
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e & 63, c = e >> 6;
    s1[c][r] = T[(ra + r) + (rb + c) * ts];
    if (!same) s2[c][r] = T[(rb + r) + (ra + c) * ts];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e & 63, c = e >> 6;
    if (!same) {
      T[(ra + r) + (rb + c) * ts] = s2[r][c];
      T[(rb + r) + (ra + c) * ts] = s1[r][c];
    } else {
      T[(ra + r) + (ra + c) * ts] = s1[r][c];
    }
  }
}

// blocks g < nlow: the lower tiles in tile order; g >= nlow: the band pool slots
__global__ __launch_bounds__(256) void k_transpose_tiles_lp(TileMat M, int64_t npt, int64_t nlow, int64_t nb) {
  __shared__ double d1[64][65], d2[64][65];
  const int64_t g = blockIdx.x;
  if (g >= nb) return;
  int64_t I, J, bq, aq;
  tri_decode(g % npt, &bq, &aq);  // aq <= bq
  if (g >= nlow) {
    swap_blocks64<double>(M.pool + (g - nlow) / npt * M.ts * M.ts, M.ts, aq * 64, bq * 64, aq == bq, d1, d2);
    return;
  }
  tri_decode(g / npt, &I, &J);
  if (I == J)
    swap_blocks64<double>(M.diag + I * M.ts * M.ts, M.ts, aq * 64, bq * 64, aq == bq, d1, d2);
  else
    swap_blocks64<float>(off32(M, I, J), M.ts, aq * 64, bq * 64, aq == bq, (float(*)[65])d1, (float(*)[65])d2);
}

// ------------------------------------ mixed fused LAUUM + score contraction
// X = L^-1 has FP64 diagonal tiles and FP32 off-diagonal tiles, every tile
// transposed by k_transpose_tiles_lp: the stored T(K, I) holds X(K, I)^T, so
// X(K, I)[k, m] = T(K, I)[m + k ts] and both operands of
// W_IJ = sum_K X_KI^T X_KJ are read along their contiguous index.  W follows the precision map of Sigma: blocks W_IJ of FP32 and BF16
// tiles run on FP32 MFMA with FP32 accumulation; diagonal blocks W_II and the
// blocks of FP64 band tiles run on FP64 MFMA (FP32 tiles widened exactly),
// where the entries of dSigma are largest.  The contraction is FP64 in both.
// FP32 kernel: pair p -> (a, c), c <= a, I = a + 1 > J = c; band tiles skipped.
__global__ __launch_bounds__(256, 2) void k_lauum_contract_lp(TileMat M, const uint8_t* __restrict__ tag, int T,
                                                              int64_t nreal, const double* __restrict__ xs,
                                                              const double* __restrict__ ys,
                                                              const double* __restrict__ av,
                                                              const double* __restrict__ qt,
                                                              const double* __restrict__ cst,
                                                              double* __restrict__ part, int64_t nb) {
  __shared__ float sm[G32_LDS];
  const int64_t ts = M.ts, NT = M.NT;
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const int64_t p = b / (T * T);
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  int64_t a, c;
  tri_decode(p, &a, &c);
  const int64_t I = a + 1, J = c;
  if (tag[off_index(I, J, NT)] == TAG_F64 || I * ts + u * BLK >= nreal || J * ts + v * BLK >= nreal) {
    if (threadIdx.x < 3) part[3 * b + threadIdx.x] = 0.0;
    return;
  }
  v16f acc[2][2];
  acc32_zero(acc);
  const int64_t r0 = (int64_t)u * BLK, c0 = (int64_t)v * BLK;
  // K = I: rows r0.. of the lower-triangular X_II against the same rows of X_IJ
  gemm32_blk<SRC_F64, false, SRC_F32, false>(M.diag + I * ts * ts + r0 + r0 * ts, ts, off32(M, I, J) + c0 + r0 * ts,
                                             ts, (int)(ts - r0), acc, sm);
  // K = I + 1 .. NT - 1: every row of the tiles below
  if (I + 1 < NT) {
    // the slots of one tile column are consecutive: row k0 of the stack of
    // tiles (I + 1.., C) is at k0 ts of its first tile
    const float* XI = off32(M, I + 1, I);
    const float* XJ = off32(M, I + 1, J);
    auto ap = [=](int k0) -> const float* { return XI + r0 + (int64_t)k0 * ts; };
    auto bp = [=](int k0) -> const float* { return XJ + c0 + (int64_t)k0 * ts; };
    gemm32<SRC_F32, false, SRC_F32, false>(ap, ts, bp, ts, (int)((NT - 1 - I) * ts), acc, sm);
  }
  contract_block32(acc, I * ts + r0, J * ts + c0, nreal, xs, ys, av, qt, cst, sm, part + 3 * b);
}

// FP64 kernel: block (I, J, u, v) with (I, J) = the diagonal tile p for
// p < NT, else band tile (li, lj)[p - NT]; v <= u on the diagonal.  X tiles
// of the band are read from their FP64 slots, the others from their FP32
// slots (widened), over runs of tiles K with the same pair of precisions.
__global__ __launch_bounds__(256, 2) void k_lauum_f64_lp(TileMat M, const uint8_t* __restrict__ tag, int T,
                                                         int64_t nreal, const double* __restrict__ xs,
                                                         const double* __restrict__ ys,
                                                         const double* __restrict__ av,
                                                         const double* __restrict__ qt,
                                                         const double* __restrict__ cst, double* __restrict__ part,
                                                         int64_t nb, const int32_t* __restrict__ li,
                                                         const int32_t* __restrict__ lj) {
  __shared__ double sm[GEMM_LDS];
  const int64_t ts = M.ts, NT = M.NT;
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const int64_t p = b / (T * T);
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  const int64_t I = p < NT ? p : li[p - NT], J = p < NT ? p : lj[p - NT];
  if ((I == J && u < v) || I * ts + u * BLK >= nreal || J * ts + v * BLK >= nreal) {
    if (threadIdx.x < 3) part[3 * b + threadIdx.x] = 0.0;
    return;
  }
  v4d acc[4][4];
  acc_zero(acc);
  const int64_t r0 = (int64_t)u * BLK, c0 = (int64_t)v * BLK;
  const double* XII = M.diag + I * ts * ts;
  const double* XIJ = I == J ? XII : band64(M, off_index(I, J, NT));
  gemm_blk<false, false, true>(XII + r0 + r0 * ts, ts, XIJ + c0 + r0 * ts, ts, (int)(ts - r0), acc, sm);
  // K = I + 1 .. NT - 1: each stage lies in one tile K, read in that tile's precision
  if (I + 1 < NT) {
    const UDiv dts(ts);  // k0 < npad, npad ts < 2^32
    auto op = [=](int k0, int64_t C, int64_t c) {
      const int64_t q = dts.q((uint32_t)k0);
      const int64_t idx = off_index(I + 1, C, NT) + q, o = c + (k0 - q * ts) * ts;
      if (tag[idx] == TAG_F64) return MixPtr{band64(M, idx) + o, true};
      return MixPtr{(const float*)M.off + idx * ts * ts + o, false};
    };
    gemm_core_mix<false, false>([=](int k0) { return op(k0, I, r0); }, ts, [=](int k0) { return op(k0, J, c0); }, ts,
                                (int)((NT - 1 - I) * ts), acc, sm);
  }
  contract_block64(acc, I * ts + r0, J * ts + c0, nreal, xs, ys, av, qt, cst, sm, part + 3 * b);
}

// ---------------------------------------------------------------- launchers
void launch_tile_bbox(const double* xs, const double* ys, int64_t ts, int64_t NT, int64_t nreal, double* box,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_tile_bbox, dim3((unsigned)NT), dim3(256), 0, s, xs, ys, ts, nreal, box);
}

void launch_tile_dmin(const double* xs, const double* ys, int64_t ts, int64_t NT, int64_t nreal, double* dmin,
                      hipStream_t s) {
  const int64_t noff = NT * (NT - 1) / 2;
  if (noff <= 0) return;
  hipLaunchKernelGGL(k_tile_dmin, dim3((unsigned)noff), dim3(256), (size_t)(2 * ts * sizeof(double)), s, xs, ys, ts,
                     NT, nreal, dmin);
}

void launch_tile_corr(const double* dmin, int64_t NT, const double* qt, const double* cst, double* corr,
                      hipStream_t s) {
  const int64_t noff = NT * (NT - 1) / 2;
  if (noff <= 0) return;
  hipLaunchKernelGGL(k_tile_corr, dim3((unsigned)((noff + 255) / 256)), dim3(256), 0, s, dmin, noff, qt, cst, corr);
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

void launch_panel_bf16t(const TileMat& M, int64_t k, const double* pbuf, uint16_t* pbt, hipStream_t s) {
  const int64_t count = M.NT - k - 1;
  if (count <= 0) return;
  const int64_t nb = M.ts / 64;
  hipLaunchKernelGGL(k_panel_bf16t, dim3((unsigned)(count * nb * nb)), dim3(256), 0, s, pbuf, pbt, M.ts, count);
}

void launch_update_lp(const TileMat& M, const uint8_t* tag, const float* p32, const uint16_t* pbt, int64_t k,
                      int64_t nreal, int part, bool skip_bf16, hipStream_t s) {
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
  hipLaunchKernelGGL(k_update_lp, dim3((unsigned)nblk), dim3(256), 0, s, M, tag, p32, pbt, T, k, nreal, nblk, mode,
                     off, (int)skip_bf16);
}

void launch_trsv_fwd_lp(const TileMat& M, const uint8_t* tag, const double* Xd, int64_t nreal, double* rhs,
                        double* y, hipStream_t s) {
  const int64_t ts = M.ts, NT = M.NT;
  const int T = (int)(ts / BLK);
  const size_t shm = (size_t)(ts + SOLVE_THREADS) * sizeof(double);
  const int64_t gmax = (nreal + BLK - 1) / BLK;
  for (int64_t k = 0; k < NT; ++k) {
    launch_diag_apply_n(Xd + k * ts * ts, ts, rhs + k * ts, y + k * ts, s);
    const int64_t g0 = (k + 1) * T;
    if (gmax > g0)
      hipLaunchKernelGGL(k_gemv_fwd_lp, dim3((unsigned)(gmax - g0)), dim3(SOLVE_THREADS), shm, s, M, tag, k, g0,
                         y + k * ts, rhs);
  }
}

void launch_trsv_bwd_lp(const TileMat& M, const uint8_t* tag, const double* Xd, double* rhs, double* a,
                        hipStream_t s) {
  const int64_t ts = M.ts, NT = M.NT;
  const int T = (int)(ts / BLK);
  for (int64_t k = NT - 1; k >= 0; --k) {
    launch_diag_apply_t(Xd + k * ts * ts, ts, rhs + k * ts, a + k * ts, s);
    if (k > 0)
      hipLaunchKernelGGL(k_gemv_bwd_lp, dim3((unsigned)(k * T)), dim3(SOLVE_THREADS), 0, s, M, tag, k, a + k * ts,
                         rhs);
  }
}

// the step's two halves for two streams, as launch_trtri_right / _rest
void launch_trtri_right_lp(const TileMat& M, const uint8_t* tag, const double* Xk, float* P, double* Q,
                           const BandLists& bl, int64_t k, int64_t nreal, hipStream_t s) {
  const int64_t ts = M.ts, NT = M.NT, tt = ts * ts;
  const int T = (int)(ts / BLK);
  const int64_t nbelow = NT - k - 1;
  if (nbelow <= 0) return;
  const int64_t nr = nbelow * T * T;
  hipLaunchKernelGGL(k_tri_right_lp, dim3((unsigned)nr), dim3(256), 0, s, M, tag, Xk, P, T, k, nreal, nr);
  const int64_t e0 = bl.cfirst[k], ne = bl.cfirst[k + 1] - e0;  // band tiles of column k
  if (ne > 0) {
    const int64_t nbb = ne * T * T;
    hipLaunchKernelGGL(k_tri_right_band, dim3((unsigned)nbb), dim3(256), 0, s, M, Xk, Q, P, bl.li, e0, T, k, nreal,
                       nbb);
  }
  hipLaunchKernelGGL(k_copy_back_lp, dim3((unsigned)((nbelow * tt + 255) / 256)), dim3(256), 0, s, M, P, nbelow,
                     k + 1, k, 1);
  if (ne > 0)
    hipLaunchKernelGGL(k_copy_back_band, dim3((unsigned)((ne * tt + 255) / 256)), dim3(256), 0, s, M, Q, bl.li,
                       bl.lj, bl.rl, e0, ne, k, 1);
}

void launch_trtri_rest_lp(const TileMat& M, const uint8_t* tag, const double* Xk, float* P, double* Q,
                          const BandLists& bl, int64_t k, int64_t nreal, hipStream_t s) {
  const int64_t ts = M.ts, NT = M.NT;
  const int T = (int)(ts / BLK);
  const int64_t tt = ts * ts;
  const int64_t nbelow = NT - k - 1;
  if (nbelow > 0 && k > 0) {
    const int64_t ng = nbelow * k * T * T;
    hipLaunchKernelGGL(k_tri_gemm_lp, dim3((unsigned)ng), dim3(256), 0, s, M, tag, P, T, k, nreal, ng);
    const int64_t nbg = bl.cfirst[k] * T * T;  // band tiles of columns < k (those with rows > k are targets)
    if (nbg > 0)
      hipLaunchKernelGGL(k_tri_gemm_band, dim3((unsigned)nbg), dim3(256), 0, s, M, tag, Q, P, bl.li, bl.lj, T, k,
                         nreal, nbg);
  }
  if (k > 0) {
    const int64_t nl = k * T * T;
    hipLaunchKernelGGL(k_tri_left_lp, dim3((unsigned)nl), dim3(256), 0, s, M, tag, Xk, P, T, k, nl);
    const int64_t r0 = bl.rfirst[k], nrow = bl.rfirst[k + 1] - r0;  // band tiles of row k
    if (nrow > 0) {
      const int64_t nbl = nrow * T * T;
      hipLaunchKernelGGL(k_tri_left_band, dim3((unsigned)nbl), dim3(256), 0, s, M, Xk, Q, P, bl.lj, bl.rl, r0, T, k,
                         nbl);
    }
    hipLaunchKernelGGL(k_copy_back_lp, dim3((unsigned)((k * tt + 255) / 256)), dim3(256), 0, s, M, P, k, k,
                       (int64_t)0, 0);
    if (nrow > 0)
      hipLaunchKernelGGL(k_copy_back_band, dim3((unsigned)((nrow * tt + 255) / 256)), dim3(256), 0, s, M, Q, bl.li,
                         bl.lj, bl.rl, r0, nrow, k, 0);
  }
  launch_copy(M.diag + k * tt, Xk, tt, s);
}

// part: lauum_blocks(ts, NT) + nband T^2 triples, the FP32 blocks first;
// returns the number of triples written
int64_t launch_lauum_contract_lp(const TileMat& M, const uint8_t* tag, int64_t nreal, const double* xs,
                                 const double* ys, const double* av, const double* qt, const double* cst,
                                 const int32_t* li, const int32_t* lj, int64_t nband, double* part, hipStream_t s) {
  const int T = (int)(M.ts / BLK);
  const int64_t NT = M.NT;
  const int64_t nb_off = NT * (NT - 1) / 2 * T * T, nb64 = (NT + nband) * T * T;
  const int64_t t64 = M.ts / 64, npt = t64 * (t64 + 1) / 2, nlow = NT * (NT + 1) / 2 * npt,
                ntr = nlow + nband * npt;
  hipLaunchKernelGGL(k_transpose_tiles_lp, dim3((unsigned)ntr), dim3(256), 0, s, M, npt, nlow, ntr);
  if (nb_off > 0)
    hipLaunchKernelGGL(k_lauum_contract_lp, dim3((unsigned)nb_off), dim3(256), 0, s, M, tag, T, nreal, xs, ys, av, qt,
                       cst, part, nb_off);
  hipLaunchKernelGGL(k_lauum_f64_lp, dim3((unsigned)nb64), dim3(256), 0, s, M, tag, T, nreal, xs, ys, av, qt, cst,
                     part + 3 * nb_off, nb64, li, lj);
  return nb_off + nb64;
}

}  // namespace exg
