// Device-side building blocks shared by the HIP kernels of the library.
//
// Layout conventions
//   * The n x n covariance is padded to npad = NT * ts and stored as its lower
//     tiles only, each a ts x ts column-major block (leading dimension ts):
//     the NT diagonal tiles in one FP64 array (tile k at k ts^2), the
//     off-diagonal tiles (i, j), i > j, column by column in a second array
//     (slot off_index(i, j) ts^2; FP64, or 4-byte slots in mixed precision).
//     Padding: Sigma_pp = 1 on padded diagonal entries, 0 elsewhere, which
//     adds nothing to log det Sigma or to z^T Sigma^-1 z (padded z = 0).
//   * Every dense product is cut into 128 x 128 output blocks, one per
//     256-thread workgroup (4 wave64s in a 2 x 2 arrangement, each owning a
//     64 x 64 sub-block = 4 x 4 MFMA tiles of 16 x 16).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace exg {

constexpr int BLK = 128;        // output block edge
constexpr int BK = 16;          // k-depth of one LDS stage
constexpr int LDP = BLK + 2;    // padded LDS row length (doubles)
constexpr int GEMM_THREADS = 256;
constexpr int GEMM_LDS = 2 * 2 * BK * LDP;  // doubles: 2 operands x 2 stages

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float fl2 __attribute__((ext_vector_type(2)));

// two consecutive operand elements held between the global load and the LDS
// store of the FP64 core; FP32 sources are widened (exactly) at the store
template <typename T>
struct Pair2;
// bytes in the global address space (loads through it are global, not flat)
typedef __attribute__((address_space(1))) const char gbyte;

template <>
struct Pair2<double> {
  d2 v;
  __device__ __forceinline__ void load(const double* p) { v = *(const d2*)p; }
  __device__ __forceinline__ void load_g(gbyte* p) { v = *(__attribute__((address_space(1))) const d2*)p; }
  __device__ __forceinline__ d2 get() const { return v; }
};
template <>
struct Pair2<float> {
  fl2 v;
  __device__ __forceinline__ void load(const float* p) { v = *(const fl2*)p; }
  __device__ __forceinline__ void load_g(gbyte* p) { v = *(__attribute__((address_space(1))) const fl2*)p; }
  __device__ __forceinline__ d2 get() const { return (d2){(double)v.x, (double)v.y}; }
};

__device__ __forceinline__ int64_t tri(int64_t i) { return i * (i + 1) / 2; }

// Quotient a / d for a run of a values against one divisor d >= 2 without a
// division per call: q(a) is the high half of a m, m = floor(2^32 / d) + 1.
// With m d = 2^32 + e, 0 < e <= d, a m / 2^32 = a / d + a e / (d 2^32), and the
// added term stays below 1 / d while a d < 2^32, so q(a) = floor(a / d) exactly.
struct UDiv {
  uint32_t m;
  __device__ __forceinline__ explicit UDiv(int64_t d) : m((uint32_t)(0x100000000ull / (uint64_t)d + 1)) {}
  __device__ __forceinline__ uint32_t q(uint32_t a) const { return __umulhi(a, m); }
};



// The tile matrix: the NT diagonal tiles in one FP64 array, the off-diagonal
// tiles (i > j) in a second array packed by tile columns, so that the tiles
// below the diagonal of one column are contiguous:
//   off_index(i, j) = j (NT - 1) - j (j - 1) / 2 + (i - j - 1).
// Every tile is ts x ts, column-major (leading dimension ts).  In FP64 mode the
// off-diagonal array holds doubles; in mixed precision it holds 4-byte slots
// (FP32 values, or BF16 values in the first half of the slot).
struct TileMat {
  double* diag;
  void* off;
  int64_t ts, NT;
  // mixed precision only: FP64 band tiles live in a pool of FP64 tiles;
  // pidx[off_index(i, j)] is the pool slot of tile (i, j) (-1: not a band tile)
  double* pool = nullptr;
  const int32_t* pidx = nullptr;
  // diagonal-super-tile approximation: tiles (i, j) with i - j >= dst are
  // zero and stay zero (no fill-in outside a tile band); 0 = exact
  int64_t dst = 0;
};

// precision tag of an off-diagonal tile in mixed precision
enum TileTag { TAG_F32 = 0, TAG_BF16 = 1, TAG_F64 = 2 };

// FP64 band tile with off-diagonal index idx (mixed precision)
__device__ __forceinline__ double* band64(const TileMat& M, int64_t idx) {
  return M.pool + (int64_t)M.pidx[idx] * M.ts * M.ts;
}

__host__ __device__ __forceinline__ int64_t off_index(int64_t i, int64_t j, int64_t NT) {
  return j * (NT - 1) - j * (j - 1) / 2 + (i - j - 1);
}

// FP64 tile (i, j), i >= j, of an all-FP64 tile matrix
__device__ __forceinline__ double* tptr(const TileMat& M, int64_t i, int64_t j) {
  return (i == j) ? M.diag + i * M.ts * M.ts : (double*)M.off + off_index(i, j, M.NT) * M.ts * M.ts;
}

// Decode p in [0, m(m+1)/2) into (a, b), 0 <= b <= a < m, a ascending with p.
__device__ __forceinline__ void tri_decode(int64_t p, int64_t* a, int64_t* b) {
  int64_t r = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
  while (tri(r + 1) <= p) ++r;
  while (tri(r) > p) --r;
  *a = r;
  *b = p - tri(r);
}

// Which (target row, target column) tile pairs of step k one update launch
// covers.  Pairs are offsets (a, c), c <= a, below the step's first trailing
// tile; the first trailing column (c = 0) is updated apart from the rest so
// that the next panel can be factored while the rest of the update runs.
enum UpdatePart { UPD_ALL = 0, UPD_FIRST_COLUMN = 1, UPD_REST = 2 };
enum PairMap { PAIRS_TRI = 0, PAIRS_DIAG = 1, PAIRS_COL = 2, PAIRS_LIST = 3 };

// pair group p -> (a, c): PAIRS_TRI the p-th lower pair shifted by off on
// both sides, PAIRS_DIAG a = c = p + off, PAIRS_COL a = p + off and c = 0
__device__ __forceinline__ void pair_map(int mode, int64_t off, int64_t p, int64_t* a, int64_t* c) {
  if (mode == PAIRS_DIAG) {
    *a = *c = p + off;
  } else if (mode == PAIRS_COL) {
    *a = p + off;
    *c = 0;
  } else {
    tri_decode(p, a, c);
    *a += off;
    *c += off;
  }
}

// v_mfma_f64_16x16x4f64 lane layout (checked on gfx950):
//   operand X (first):  lane l holds X[l % 16][l / 16]      (16 x 4)
//   operand Y (second): lane l holds Y[l / 16][l % 16]      (4 x 16)
//   result D = X Y:     lane l, register r holds D[4 r + l / 16][l % 16]
__device__ __forceinline__ v4d mfma64(double x, double y, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
}

// A pointer that every lane of the workgroup holds, moved to scalar registers
// (the caller guarantees that it is the same in every lane).
__device__ __forceinline__ gbyte* uniform_base(const void* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (gbyte*)(((uint64_t)hi << 32) | lo);
}

// One 128 x 128 block of  sum_k Aop(m, k) Bop(n, k)  accumulated into acc,
// over a virtual k range [0, K) that may run across several tiles.
//   aptr(k0) returns the address of Aop(0, k0) for a stage starting at k0;
//   within a stage (BK consecutive k):
//     Aop(m, k0 + q) = aptr(k0)[m + q * lda]   (AKC = false, m contiguous)
//                    = aptr(k0)[q + m * lda]   (AKC = true,  k contiguous)
//   bptr / Bop(n, k) likewise with ldb, BKC.
// The operands may be FP64 or FP32 (aptr / bptr return const double* or
// const float*; FP32 values are widened exactly).  K must be a multiple of
// 2 BK; every pair of elements read must be aligned to its size.  acc[i][j] holds output rows m = wr*64 + 16 i + (lane & 15) and
// columns n = wc*64 + 16 j + 4 r + (lane >> 4), r = 0..3 (wr = wave >> 1,
// wc = wave & 1); with this assignment the lanes of one store instruction
// write 16 consecutive rows of a column-major output.
// SB = true: each stage's operand addresses are aptr(k0) / bptr(k0), which must
// then be the same in every lane, held in scalar registers plus one 32-bit byte
// offset per thread and load (so 127 lda + 15 elements must stay below 4 GiB);
// this frees about 14 vector registers.  SB = false: 64-bit vector addresses.
template <bool AKC, bool BKC, bool SB = false, class AP, class BP>
__device__ __forceinline__ void gemm_core(AP aptr, int64_t lda, BP bptr, int64_t ldb, int K, v4d (&acc)[4][4],
                                          double* sm) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  double* sA = sm;
  double* sB = sm + 2 * BK * LDP;
  using TA = std::remove_cv_t<std::remove_pointer_t<decltype(aptr(0))>>;
  using TB = std::remove_cv_t<std::remove_pointer_t<decltype(bptr(0))>>;
  // two register sets: the global loads run two stages ahead of the MFMAs
  Pair2<TA> ra0[4], ra1[4];
  Pair2<TB> rb0[4], rb1[4];
  uint32_t oa[4], ob[4];  // SB: byte offsets of the thread's pairs within a stage
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int idx = t + GEMM_THREADS * s;
    oa[s] = (uint32_t)(sizeof(TA) * (AKC ? 2 * (idx & 7) + (int64_t)(idx >> 3) * lda
                                         : 2 * (idx & 63) + (int64_t)(idx >> 6) * lda));
    ob[s] = (uint32_t)(sizeof(TB) * (BKC ? 2 * (idx & 7) + (int64_t)(idx >> 3) * ldb
                                         : 2 * (idx & 63) + (int64_t)(idx >> 6) * ldb));
  }
  auto gload = [&](int k0, Pair2<TA> (&ra)[4], Pair2<TB> (&rb)[4]) {
    if constexpr (SB) {
      gbyte* A = uniform_base(aptr(k0));
      gbyte* B = uniform_base(bptr(k0));
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        ra[s].load_g(A + oa[s]);
        rb[s].load_g(B + ob[s]);
      }
      return;
    }
    const TA* A = aptr(k0);
    const TB* B = bptr(k0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int idx = t + GEMM_THREADS * s;
      if (!AKC) {
        const int kk = idx >> 6, m2 = idx & 63;
        ra[s].load(A + 2 * m2 + (int64_t)kk * lda);
      } else {
        const int m = idx >> 3, kp = idx & 7;
        ra[s].load(A + 2 * kp + (int64_t)m * lda);
      }
      if (!BKC) {
        const int kk = idx >> 6, n2 = idx & 63;
        rb[s].load(B + 2 * n2 + (int64_t)kk * ldb);
      } else {
        const int n = idx >> 3, kp = idx & 7;
        rb[s].load(B + 2 * kp + (int64_t)n * ldb);
      }
    }
  };
  auto sstore = [&](int buf, const Pair2<TA> (&ra)[4], const Pair2<TB> (&rb)[4]) {
    double* a = sA + buf * BK * LDP;
    double* b = sB + buf * BK * LDP;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int idx = t + GEMM_THREADS * s;
      const d2 va = ra[s].get(), vb = rb[s].get();
      if (!AKC) {
        const int kk = idx >> 6, m2 = idx & 63;
        *(d2*)(a + kk * LDP + 2 * m2) = va;
      } else {
        const int m = idx >> 3, kp = idx & 7;
        a[(2 * kp) * LDP + m] = va.x;
        a[(2 * kp + 1) * LDP + m] = va.y;
      }
      if (!BKC) {
        const int kk = idx >> 6, n2 = idx & 63;
        *(d2*)(b + kk * LDP + 2 * n2) = vb;
      } else {
        const int n = idx >> 3, kp = idx & 7;
        b[(2 * kp) * LDP + n] = vb.x;
        b[(2 * kp + 1) * LDP + n] = vb.y;
      }
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
  const int nst = K / BK;  // even: every K here is a multiple of 128
  gload(0, ra0, rb0);
  gload(BK, ra1, rb1);
  sstore(0, ra0, rb0);
  __syncthreads();
  for (int st = 0; st < nst; st += 2) {
    // stage st from LDS buffer 0; stage st+1 waits in set 1; fetch st+2 into set 0
    if (st + 2 < nst) gload((st + 2) * BK, ra0, rb0);
    compute(0);
    sstore(1, ra1, rb1);
    __syncthreads();
    // stage st+1 from LDS buffer 1; stage st+2 waits in set 0; fetch st+3 into set 1
    if (st + 3 < nst) gload((st + 3) * BK, ra1, rb1);
    compute(1);
    if (st + 2 < nst) sstore(0, ra0, rb0);
    __syncthreads();
  }
}

// gemm_core over one contiguous operand pair:
//   Aop(m, k) = A[m + k lda] (AKC = false) or A[k + m lda] (AKC = true), same for B.
template <bool AKC, bool BKC, bool SB = false>
__device__ __forceinline__ void gemm_blk(const double* __restrict__ A, int64_t lda, const double* __restrict__ B,
                                         int64_t ldb, int K, v4d (&acc)[4][4], double* sm) {
  auto ap = [=](int k0) { return AKC ? A + k0 : A + (int64_t)k0 * lda; };
  auto bp = [=](int k0) { return BKC ? B + k0 : B + (int64_t)k0 * ldb; };
  gemm_core<AKC, BKC, SB>(ap, lda, bp, ldb, K, acc, sm);
}

// Workgroups are dispatched to the 8 XCDs in turn (workgroup b to XCD b mod 8),
// each XCD with its own L2.  xcd_block maps the dispatch index to a logical
// block so that XCD x runs the contiguous logical range [x nb8, (x + 1) nb8),
// nb8 = ceil(nb / 8): the blocks resident on one XCD at a time are neighbours
// in the launch's block order and reuse each other's operand reads in that
// XCD's L2 (used by the BF16 update, whose blocks are bound by operand reads;
// the FP64 trailing update ran 3.5% slower with it while it halved the bytes
// fetched past L2).  The grid must have 8 nb8 workgroups; -1 for the spare ones.
__device__ __forceinline__ int64_t xcd_block(int64_t nb) {
  const int64_t nb8 = (nb + 7) / 8;
  const int64_t b = (int64_t)(blockIdx.x % 8) * nb8 + blockIdx.x / 8;
  return b < nb ? b : -1;
}

__device__ __forceinline__ void acc_zero(v4d (&acc)[4][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};
}

// C(m, n) = beta * C(m, n) + alpha * acc  on a column-major 128 x 128 block.
// With beta = 1 the 16 values of one accumulator row group are all loaded
// before any is stored: the compiler cannot tell that the computed addresses
// differ, and would otherwise wait for each load's round trip in turn.
__device__ __forceinline__ void acc_store(double* C, int64_t ldc, const v4d (&acc)[4][4], double alpha, bool beta1) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = wr * 64 + 16 * i + (lane & 15);
    double* p = C + m + (int64_t)(wc * 64 + (lane >> 4)) * ldc;
    double old[4][4];
    if (beta1) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) old[j][r] = p[(int64_t)(16 * j + 4 * r) * ldc];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double v = alpha * acc[i][j][r];
        p[(int64_t)(16 * j + 4 * r) * ldc] = beta1 ? old[j][r] + v : v;
      }
  }
}

// Block-wide sum of NV doubles per thread in a fixed order (deterministic).
// sum over the 64 lanes of a wave (every lane receives the total)
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red /* NV * blockDim */) {
  const int t = threadIdx.x, nt = blockDim.x;
#pragma unroll
  for (int q = 0; q < NV; ++q) red[q * nt + t] = v[q];
  __syncthreads();
  for (int s = nt >> 1; s > 0; s >>= 1) {
    if (t < s) {
#pragma unroll
      for (int q = 0; q < NV; ++q) red[q * nt + t] += red[q * nt + t + s];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = red[q * nt];
  __syncthreads();
}

}  // namespace exg
