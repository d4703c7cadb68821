// Low-precision MFMA block cores for the mixed-precision kernels: one
// 128 x 128 block of  sum_k Aop(m, k) Bop(n, k)  accumulated in FP32,
//   gemm32:    on v_mfma_f32_32x32x2f32, operands read from FP32, FP64
//              (rounded to nearest FP32) or BF16 (widened exactly) tiles and
//              staged through LDS as FP32;
//   gemm_bf16: on v_mfma_f32_16x16x32_bf16, BF16 operands stored with k
//              contiguous, staged through LDS as they are.
#pragma once

#include "common.h"

namespace exg {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

constexpr int G32_BK = 16;                           // k-depth of one LDS stage
constexpr int G32_LDP = BLK + 4;                     // padded LDS row (floats)
constexpr int G32_LDS = 2 * 2 * G32_BK * G32_LDP;   // floats: 2 operands x 2 stages

enum SrcKind { SRC_F32 = 0, SRC_F64 = 1, SRC_BF16 = 2 };

__device__ __forceinline__ float bf16_bits_to_f32(uint32_t h16) { return __uint_as_float(h16 << 16); }

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// v_mfma_f32_32x32x2f32 (checked on gfx950): operand X lane l holds
// X[l % 32][l / 32], operand Y lane l holds Y[l / 32][l % 32]; D = X Y has
// lane l, register r at D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
__device__ __forceinline__ v16f mfma32x32(float x, float y, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, c, 0, 0, 0);
}

// One operand's share of a stage (G32_BK k values x 128 rows) for one thread,
// held in registers between the global load and the LDS store.  p points at
// Op(0, k0); KC = false: Op(m, k0 + q) = p[m + q ld]; KC = true: p[q + m ld].
template <int SK, bool KC>
struct Stage32;

template <>
struct Stage32<SRC_F32, false> {
  f4 r[2];
  __device__ __forceinline__ void load(const void* p, int64_t ld, int t) {
    const float* a = (const float*)p;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int idx = t + 256 * s, kk = idx >> 5, m4 = idx & 31;
      r[s] = *(const f4*)(a + 4 * m4 + (int64_t)kk * ld);
    }
  }
  __device__ __forceinline__ void store(float* S, int t) const {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int idx = t + 256 * s, kk = idx >> 5, m4 = idx & 31;
      *(f4*)(S + kk * G32_LDP + 4 * m4) = r[s];
    }
  }
};

template <>
struct Stage32<SRC_F32, true> {
  f4 r[2];
  __device__ __forceinline__ void load(const void* p, int64_t ld, int t) {
    const float* a = (const float*)p;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int idx = t + 256 * s, m = idx >> 2, k4 = idx & 3;
      r[s] = *(const f4*)(a + 4 * k4 + (int64_t)m * ld);
    }
  }
  __device__ __forceinline__ void store(float* S, int t) const {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int idx = t + 256 * s, m = idx >> 2, k4 = idx & 3;
#pragma unroll
      for (int e = 0; e < 4; ++e) S[(4 * k4 + e) * G32_LDP + m] = r[s][e];
    }
  }
};

template <>
struct Stage32<SRC_F64, false> {
  d2 r[4];
  __device__ __forceinline__ void load(const void* p, int64_t ld, int t) {
    const double* a = (const double*)p;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int idx = t + 256 * s, kk = idx >> 6, m2 = idx & 63;
      r[s] = *(const d2*)(a + 2 * m2 + (int64_t)kk * ld);
    }
  }
  __device__ __forceinline__ void store(float* S, int t) const {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int idx = t + 256 * s, kk = idx >> 6, m2 = idx & 63;
      f2 v;
      v.x = (float)r[s].x;
      v.y = (float)r[s].y;
      *(f2*)(S + kk * G32_LDP + 2 * m2) = v;
    }
  }
};

template <>
struct Stage32<SRC_F64, true> {
  d2 r[4];
  __device__ __forceinline__ void load(const void* p, int64_t ld, int t) {
    const double* a = (const double*)p;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int idx = t + 256 * s, m = idx >> 3, k2 = idx & 7;
      r[s] = *(const d2*)(a + 2 * k2 + (int64_t)m * ld);
    }
  }
  __device__ __forceinline__ void store(float* S, int t) const {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int idx = t + 256 * s, m = idx >> 3, k2 = idx & 7;
      S[(2 * k2) * G32_LDP + m] = (float)r[s].x;
      S[(2 * k2 + 1) * G32_LDP + m] = (float)r[s].y;
    }
  }
};

template <>
struct Stage32<SRC_BF16, false> {
  u4 r;
  __device__ __forceinline__ void load(const void* p, int64_t ld, int t) {
    const uint16_t* a = (const uint16_t*)p;
    const int kk = t >> 4, m8 = t & 15;
    r = *(const u4*)(a + 8 * m8 + (int64_t)kk * ld);
  }
  __device__ __forceinline__ void store(float* S, int t) const {
    const int kk = t >> 4, m8 = t & 15;
    f4 lo, hi;
    lo.x = __uint_as_float(r.x << 16);
    lo.y = __uint_as_float(r.x & 0xffff0000u);
    lo.z = __uint_as_float(r.y << 16);
    lo.w = __uint_as_float(r.y & 0xffff0000u);
    hi.x = __uint_as_float(r.z << 16);
    hi.y = __uint_as_float(r.z & 0xffff0000u);
    hi.z = __uint_as_float(r.w << 16);
    hi.w = __uint_as_float(r.w & 0xffff0000u);
    *(f4*)(S + kk * G32_LDP + 8 * m8) = lo;
    *(f4*)(S + kk * G32_LDP + 8 * m8 + 4) = hi;
  }
};

__device__ __forceinline__ void acc32_zero(v16f (&acc)[2][2]) {
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[x][y][r] = 0.f;
}

// acc += sum over the virtual k range [0, K) of Aop(m, k) Bop(n, k).
//   aptr(k0) / bptr(k0) return the address of Op(0, k0) for a stage starting
//   at k0 (SA / SB: element kind, AKC / BKC: k contiguous or m contiguous).
// K must be a multiple of 2 G32_BK; 16-byte loads must be aligned.  acc[x][y]
// register r holds output row m = wr*64 + 32 x + (lane & 31) and column
// n = wc*64 + 32 y + 8 (r / 4) + 4 (lane / 32) + r % 4 (wr = wave / 2,
// wc = wave % 2).  Ends with a barrier, so sm may be reused at once.
template <int SA, bool AKC, int SB, bool BKC, class AP, class BP>
__device__ __forceinline__ void gemm32(AP aptr, int64_t lda, BP bptr, int64_t ldb, int K, v16f (&acc)[2][2],
                                       float* sm) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  float* sA = sm;
  float* sB = sm + 2 * G32_BK * G32_LDP;
  // two register sets: the global loads run two stages ahead of the MFMAs
  Stage32<SA, AKC> a0, a1;
  Stage32<SB, BKC> b0, b1;
  auto compute = [&](int cur) {
    const float* sa = sA + cur * G32_BK * G32_LDP + wr * 64 + (lane & 31);
    const float* sb = sB + cur * G32_BK * G32_LDP + wc * 64 + (lane & 31);
#pragma unroll
    for (int kk = 0; kk < G32_BK; kk += 2) {
      const int ko = (kk + (lane >> 5)) * G32_LDP;
      float af[2], bf[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) af[x] = sa[ko + 32 * x];
#pragma unroll
      for (int y = 0; y < 2; ++y) bf[y] = sb[ko + 32 * y];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = mfma32x32(bf[y], af[x], acc[x][y]);
    }
  };
  const int nst = K / G32_BK;  // even
  a0.load(aptr(0), lda, t);
  b0.load(bptr(0), ldb, t);
  a1.load(aptr(G32_BK), lda, t);
  b1.load(bptr(G32_BK), ldb, t);
  a0.store(sA, t);
  b0.store(sB, t);
  __syncthreads();
  for (int s = 0; s < nst; s += 2) {
    if (s + 2 < nst) {
      a0.load(aptr((s + 2) * G32_BK), lda, t);
      b0.load(bptr((s + 2) * G32_BK), ldb, t);
    }
    compute(0);
    a1.store(sA + G32_BK * G32_LDP, t);
    b1.store(sB + G32_BK * G32_LDP, t);
    __syncthreads();
    if (s + 3 < nst) {
      a1.load(aptr((s + 3) * G32_BK), lda, t);
      b1.load(bptr((s + 3) * G32_BK), ldb, t);
    }
    compute(1);
    if (s + 2 < nst) {
      a0.store(sA, t);
      b0.store(sB, t);
    }
    __syncthreads();
  }
}

// plain-pointer form: Op(0, k0) = base + k0 * (KC ? 1 : ld)
template <int SA, bool AKC, int SB, bool BKC, typename TA, typename TB>
__device__ __forceinline__ void gemm32_blk(const TA* A, int64_t lda, const TB* B, int64_t ldb, int K,
                                           v16f (&acc)[2][2], float* sm) {
  gemm32<SA, AKC, SB, BKC>([=](int k0) { return A + (AKC ? (int64_t)k0 : (int64_t)k0 * lda); }, lda,
                           [=](int k0) { return B + (BKC ? (int64_t)k0 : (int64_t)k0 * ldb); }, ldb, K, acc, sm);
}

// ---------------------------------------------------------------- BF16 core
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int GB_BK = 32;                             // k-depth of one stage
constexpr int GB_LDK = GB_BK + 8;                     // padded LDS row (BF16): 80 bytes
constexpr int GB_LDS_BYTES = 2 * 2 * BLK * GB_LDK * 2;  // 2 operands x 2 stages

// v_mfma_f32_16x16x32_bf16 (checked on gfx950): operand X lane l holds
// X[l % 16][8 (l / 16) + e], operand Y lane l holds Y[8 (l / 16) + e][l % 16],
// e < 8; D = X Y has lane l, register r at D[4 (l / 16) + r][l % 16].
__device__ __forceinline__ v4f mfma_bf16(v8bf x, v8bf y, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
}

__device__ __forceinline__ void accb_zero(v4f (&acc)[4][4]) {
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = (v4f){0.f, 0.f, 0.f, 0.f};
}

// acc += sum_{k < K} Aop(m, k) Bop(n, k) with BF16 operands stored k
// contiguous: Aop(m, k0 + q) = aptr(k0)[q + m lda] (likewise B); K a multiple
// of 2 GB_BK, rows 16-byte aligned.  acc[x][y] register r holds output row
// m = wr*64 + 16 x + (lane & 15) and column n = wc*64 + 16 y + 4 (lane >> 4) + r.
// Ends with a barrier.
template <class AP, class BP>
__device__ __forceinline__ void gemm_bf16(AP aptr, int64_t lda, BP bptr, int64_t ldb, int K, v4f (&acc)[4][4],
                                          uint16_t* sm) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  uint16_t* sA = sm;
  uint16_t* sB = sm + 2 * BLK * GB_LDK;
  u4 ra0[2], rb0[2], ra1[2], rb1[2];
  auto gload = [&](int k0, u4 (&ra)[2], u4 (&rb)[2]) {
    const uint16_t* A = aptr(k0);
    const uint16_t* B = bptr(k0);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int idx = t + 256 * s, m = idx >> 2, k8 = idx & 3;
      ra[s] = *(const u4*)(A + 8 * k8 + (int64_t)m * lda);
      rb[s] = *(const u4*)(B + 8 * k8 + (int64_t)m * ldb);
    }
  };
  auto sstore = [&](int buf, const u4 (&ra)[2], const u4 (&rb)[2]) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int idx = t + 256 * s, m = idx >> 2, k8 = idx & 3;
      *(u4*)(sA + buf * BLK * GB_LDK + m * GB_LDK + 8 * k8) = ra[s];
      *(u4*)(sB + buf * BLK * GB_LDK + m * GB_LDK + 8 * k8) = rb[s];
    }
  };
  auto compute = [&](int cur) {
    const uint16_t* sa = sA + cur * BLK * GB_LDK + (wr * 64 + (lane & 15)) * GB_LDK + 8 * (lane >> 4);
    const uint16_t* sb = sB + cur * BLK * GB_LDK + (wc * 64 + (lane & 15)) * GB_LDK + 8 * (lane >> 4);
    v8bf af[4], bf[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) af[x] = *(const v8bf*)(sa + 16 * x * GB_LDK);
#pragma unroll
    for (int y = 0; y < 4; ++y) bf[y] = *(const v8bf*)(sb + 16 * y * GB_LDK);
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = mfma_bf16(bf[y], af[x], acc[x][y]);
  };
  const int nst = K / GB_BK;  // even
  gload(0, ra0, rb0);
  gload(GB_BK, ra1, rb1);
  sstore(0, ra0, rb0);
  __syncthreads();
  for (int s = 0; s < nst; s += 2) {
    if (s + 2 < nst) gload((s + 2) * GB_BK, ra0, rb0);
    compute(0);
    sstore(1, ra1, rb1);
    __syncthreads();
    if (s + 3 < nst) gload((s + 3) * GB_BK, ra1, rb1);
    compute(1);
    if (s + 2 < nst) sstore(0, ra0, rb0);
    __syncthreads();
  }
}

}  // namespace exg
