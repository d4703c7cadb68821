// BF16 targets of the mixed-precision trailing update (paper Section 2.1,
// Fig. 1(d): the far off-diagonal tiles in half precision), on a wide block:
// one 512-thread workgroup computes a 256 x 256 block of a BF16 target tile,
//   A_ij -= A_ik A_jk^T   (the BF16 roundings of the FP64 panel, FP32 sums,
//                          the target widened and rounded back to BF16).
// The eight waves form a 2 x 4 grid, each owning 128 x 64 of the block (8 x 4
// tiles of v_mfma_f32_16x16x32_bf16, 128 accumulators per lane), two waves
// per SIMD.  Against a 128 x 128 block the workgroup reads half the operand
// bytes per flop and pays its prologue and the target's read-modify-write
// once per four times the work.  The products run in the same order as on
// the 128 x 128 block (k ascending in 32-deep MFMA steps for every output), so
// both give the same bits.
#include "common.h"
#include "gemm32.h"
#include "launch.h"

namespace exg {

constexpr int WB = 256;               // output block edge
constexpr int WB_BK = 32;             // k-depth of one stage: 64 bytes of a row
constexpr int WB_STAGE = WB * WB_BK;  // BF16 values per operand and stage

// LDS position of the 16-byte chunk c (k = 8c .. 8c + 7) of row m: chunk
// c ^ ((m >> 2) & 3) of a 64-byte row, so that the 16 rows one 16-lane group
// reads (or the 4 x 4 chunks it writes) fall in 16 distinct groups of 4 banks
__device__ __forceinline__ int wb_off(int m, int c) { return m * WB_BK + 8 * (c ^ ((m >> 2) & 3)); }

// acc += sum_{k < K} Aop(m, k) Bop(n, k) over a 256 x 256 block; BF16 operands
// stored k contiguous, Aop(m, k0 + q) = aptr(k0)[q + m lda] (likewise B), K a
// multiple of 2 WB_BK, rows 16-byte aligned.  With wr = wave / 4 and
// wc = wave % 4, acc[x][y] register r holds output row
// m = wr*128 + 16 x + (lane & 15) and column n = wc*64 + 16 y + 4 (lane >> 4) + r.
// Ends with a barrier.
template <class AP, class BP>
__device__ __forceinline__ void gemm_bf16_wide(AP aptr, int64_t lda, BP bptr, int64_t ldb, int K, v4f (&acc)[8][4],
                                               uint16_t* sm) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 2, wc = w & 3;
  uint16_t* sA = sm;
  uint16_t* sB = sm + 2 * WB_STAGE;
  // two register sets: the global loads run two stages ahead of the MFMAs
  u4 ra0[2], rb0[2], ra1[2], rb1[2];
  auto gload = [&](int k0, u4 (&ra)[2], u4 (&rb)[2]) {
    const uint16_t* A = aptr(k0);
    const uint16_t* B = bptr(k0);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int idx = t + 512 * s, m = idx >> 2, c = idx & 3;
      ra[s] = *(const u4*)(A + 8 * c + (int64_t)m * lda);
      rb[s] = *(const u4*)(B + 8 * c + (int64_t)m * ldb);
    }
  };
  auto sstore = [&](int buf, const u4 (&ra)[2], const u4 (&rb)[2]) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int idx = t + 512 * s, m = idx >> 2, c = idx & 3;
      *(u4*)(sA + buf * WB_STAGE + wb_off(m, c)) = ra[s];
      *(u4*)(sB + buf * WB_STAGE + wb_off(m, c)) = rb[s];
    }
  };
  auto compute = [&](int cur) {
    const uint16_t* sa = sA + cur * WB_STAGE;
    const uint16_t* sb = sB + cur * WB_STAGE;
    const int c = lane >> 4;
    v8bf af[8], bf[4];
#pragma unroll
    for (int x = 0; x < 8; ++x) af[x] = *(const v8bf*)(sa + wb_off(wr * 128 + 16 * x + (lane & 15), c));
#pragma unroll
    for (int y = 0; y < 4; ++y) bf[y] = *(const v8bf*)(sb + wb_off(wc * 64 + 16 * y + (lane & 15), c));
#pragma unroll
    for (int x = 0; x < 8; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = mfma_bf16(bf[y], af[x], acc[x][y]);
  };
  const int nst = K / WB_BK;  // even
  gload(0, ra0, rb0);
  gload(WB_BK, ra1, rb1);
  sstore(0, ra0, rb0);
  __syncthreads();
  for (int s = 0; s < nst; s += 2) {
    if (s + 2 < nst) gload((s + 2) * WB_BK, ra0, rb0);
    compute(0);
    sstore(1, ra1, rb1);
    __syncthreads();
    if (s + 3 < nst) gload((s + 3) * WB_BK, ra1, rb1);
    compute(1);
    if (s + 2 < nst) sstore(0, ra0, rb0);
    __syncthreads();
  }
}

// Step k, BF16 targets (li[e], lj[e]) for the list entries e0 <= e < e0 +
// nb / TW^2 (TW = ts / 256 blocks per tile edge); A_ik and A_jk are the BF16
// panel copy's tiles i - k - 1 and j - k - 1, transposed (k contiguous).
__global__ __launch_bounds__(512, 1) void k_update_bf16(TileMat M, const int32_t* __restrict__ li,
                                                        const int32_t* __restrict__ lj, int64_t e0,
                                                        const uint16_t* __restrict__ pbt, int64_t k, int64_t nreal,
                                                        int TW, int64_t nb) {
  __shared__ __attribute__((aligned(16))) uint16_t sm[4 * WB_STAGE];  // 64 KB: 2 operands x 2 stages
  const int64_t ts = M.ts, tt = ts * ts;
  // each XCD takes a contiguous range of the blocks: the TW^2 blocks of one
  // target tile read the same TW row blocks of each operand
  const int64_t b = xcd_block(nb);
  if (b < 0) return;
  const int64_t e = e0 + b / (TW * TW);
  const int sub = (int)(b % (TW * TW));
  const int u = sub / TW, v = sub % TW;
  const int64_t i = li[e], j = lj[e];
  if (i * ts + (int64_t)u * WB >= nreal) return;  // padded rows: the update is zero
  v4f acc[8][4];
#pragma unroll
  for (int x = 0; x < 8; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = (v4f){0.f, 0.f, 0.f, 0.f};
  const uint16_t* A = pbt + (i - k - 1) * tt + (int64_t)u * WB * ts;
  const uint16_t* B = pbt + (j - k - 1) * tt + (int64_t)v * WB * ts;
  gemm_bf16_wide([=](int k0) { return A + k0; }, ts, [=](int k0) { return B + k0; }, ts, (int)ts, acc, sm);
  // the target: BF16 values in the first half of the tile's 4-byte slots
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wr = w >> 2, wc = w & 3;
  uint16_t* C = (uint16_t*)((float*)M.off + off_index(i, j, M.NT) * tt) + (int64_t)u * WB + (int64_t)v * WB * ts;
  // two row groups per batch: their 32 values are loaded before any is stored
#pragma unroll
  for (int x0 = 0; x0 < 8; x0 += 2) {
    uint16_t old[2][4][4];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          old[q][y][r] = C[wr * 128 + 16 * (x0 + q) + (lane & 15) + (int64_t)(wc * 64 + 16 * y + 4 * (lane >> 4) + r) * ts];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          C[wr * 128 + 16 * (x0 + q) + (lane & 15) + (int64_t)(wc * 64 + 16 * y + 4 * (lane >> 4) + r) * ts] =
              f32_to_bf16_rne(bf16_bits_to_f32(old[q][y][r]) - acc[x0 + q][y][r]);
  }
}

void launch_update_bf16(const TileMat& M, const int32_t* li, const int32_t* lj, int64_t e0, int64_t count,
                        const uint16_t* pbt, int64_t k, int64_t nreal, hipStream_t s) {
  if (count <= 0) return;
  const int TW = (int)(M.ts / WB);
  const int64_t nb = count * TW * TW;
  hipLaunchKernelGGL(k_update_bf16, dim3((unsigned)((nb + 7) / 8 * 8)), dim3(512), 0, s, M, li, lj, e0, pbt, k, nreal,
                     TW, nb);
}

}  // namespace exg
