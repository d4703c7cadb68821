// Covariance generation (paper eq. 3) on the device: per-theta quadrature
// tables, the packed lower-tile matrix used by the factorisation, and a dense
// n x n matrix in the caller's order (used to check generation entry by entry).
#include "common.h"
#include "launch.h"
#include "matern_dev.h"

namespace exg {

// psi(z), z > 0: shift with psi(z) = psi(z + 1) - 1/z until z >= 12, then
// psi(z) ~ ln z - 1/(2z) - sum_k B_2k / (2k z^2k)  (DLMF 5.5.2, 5.11.2).
__device__ double dev_digamma(double z) {
  double acc = 0.0;
  while (z < 12.0) {
    acc -= 1.0 / z;
    z += 1.0;
  }
  const double iz2 = 1.0 / (z * z);
  const double s =
      iz2 * (1.0 / 12 - iz2 * (1.0 / 120 - iz2 * (1.0 / 252 - iz2 * (1.0 / 240 - iz2 * (1.0 / 132 - iz2 * (691.0 / 32760))))));
  return acc + log(z) - 0.5 / z - s;
}

// One thread per (bucket m, node k): node t = k h_m, weights of the three
// integrands including the trapezoidal end weight h/2 at t = 0.
__global__ void k_quad_table(double s2, double beta, double nu, double metric, double nugget,
                             double* __restrict__ qt, double* __restrict__ cst) {
  const int m = blockIdx.x, k = threadIdx.x;
  const double h = 0.1 * exp2(-0.5 * m);
  const double t = k * h;
  const double sh = sinh(0.5 * t);
  const double w = (k == 0) ? 0.5 * h : h;
  double* q = qt + ((int64_t)m * QNK + k) * QW;
  q[0] = 2.0 * sh * sh;  // cosh t - 1 without cancellation
  q[1] = t;
  q[2] = w * cosh(nu * t);
  q[3] = w * cosh((nu - 1.0) * t);
  q[4] = w * t * sinh(nu * t);
  if (m == 0 && k == 0) {
    const double c = exp((1.0 - nu) * 0.69314718055994530942 - lgamma(nu));
    cst[C_S2] = s2;
    cst[C_BETA] = beta;
    cst[C_NU] = nu;
    cst[C_C] = c;
    cst[C_PSI] = dev_digamma(nu);
    cst[C_S2C] = s2 * c;
    cst[C_METRIC] = metric;
    cst[C_NUG] = nugget;
  }
}

// Tables of u0, u1, u2 on segment blockIdx.x of ln x (see matern_dev.h): the
// functions at the 13 Chebyshev points by the quadrature; stored per function
// are its value at the segment centre (the middle point, t = 0) and the
// Chebyshev coefficients of ln(u / u_centre), c_k = (2/N) sum_j d_j
// cos(pi k (j + 1/2) / N), whose magnitudes stay small.  Runs after
// k_quad_table.
__global__ __launch_bounds__(64) void k_cheb_table(double* __restrict__ qt, const double* __restrict__ cst) {
  __shared__ double fv[3][CH_N];
  const int seg = blockIdx.x, j = threadIdx.x;
  const double nu = cst[C_NU];
  if (j < CH_N) {
    const double tj = cos(3.14159265358979323846 * (j + 0.5) / CH_N);
    const double x = exp(CH_SLO + (seg + 0.5 * (tj + 1.0)) * CH_DS);
    double t0, t1, t2;
    quad_k3(qt, x, nu, &t0, &t1, &t2);
    const double xn = pow(x, nu);
    fv[0][j] = xn * t0;
    fv[1][j] = xn * x * t1;
    fv[2][j] = xn * t2;
  }
  __syncthreads();
  if (j < 3 * 16) {
    const int f = j >> 4, k = j & 15;
    double c = 0.0;
    if (k < CH_N) {
      for (int q = 0; q < CH_N; ++q)
        c += log(fv[f][q] / fv[f][CH_MID]) * cos(3.14159265358979323846 * k * (q + 0.5) / CH_N);
      c *= 2.0 / CH_N;
    } else if (k == CH_N) {
      c = fv[f][CH_MID];
    }
    qt[QT_CHEB_OFF + seg * CH_STRIDE + f * 16 + k] = c;
  }
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Lower tiles of the padded covariance.  One 256-thread block per 128 x 128
// block (u, v) of tile (I, J); blocks above the diagonal of a diagonal tile
// are not needed by any later step and are skipped.  Mixed precision (tag !=
// NULL): diagonal tiles FP64, off-diagonal tiles FP32 (tag 0) or BF16 (tag 1),
// each rounded to nearest even from the FP64 value, or FP64 in the band pool
// (tag 2).
__global__ __launch_bounds__(256) void k_gen_tiles(TileMat M, int T, int64_t nreal, const double* __restrict__ xs,
                                                   const double* __restrict__ ys, const double* __restrict__ qt,
                                                   const double* __restrict__ cst, const uint8_t* __restrict__ tag,
                                                   int64_t tile_first) {
  const int64_t ts = M.ts;
  const int64_t b = blockIdx.x;
  const int64_t p = tile_first + b / (T * T);
  const int sub = (int)(b % (T * T));
  const int u = sub / T, v = sub % T;
  int64_t I, J;
  tri_decode(p, &I, &J);
  if (I == J && u < v) return;
  const int r = threadIdx.x & 127, c0 = threadIdx.x >> 7;
  const int64_t gi = I * ts + u * BLK + r;
  const bool ipad = gi >= nreal;
  const double xi = ipad ? 0.0 : xs[gi], yi = ipad ? 0.0 : ys[gi];
  const int64_t o = (u * BLK + r) + (int64_t)(v * BLK) * ts;  // element offset in the tile
  // 0: FP64, 1: FP32, 2: BF16
  const int64_t idx = I == J ? 0 : off_index(I, J, M.NT);
  const int tg = (!tag || I == J) ? -1 : tag[idx];
  const int kind = (tg < 0 || tg == TAG_F64) ? 0 : (tg == TAG_BF16 ? 2 : 1);
  double* out64 = nullptr;
  float* out32 = nullptr;
  uint16_t* out16 = nullptr;
  if (kind == 0) {
    out64 = (tg == TAG_F64 ? band64(M, idx) : tptr(M, I, J)) + o;
  } else if (kind == 1) {
    out32 = (float*)M.off + off_index(I, J, M.NT) * ts * ts + o;
  } else {
    out16 = (uint16_t*)((float*)M.off + off_index(I, J, M.NT) * ts * ts) + o;
  }
  const bool zero_tile = M.dst > 0 && I - J >= M.dst;  // outside the DST band
  for (int c = c0; c < BLK; c += 2) {
    const int64_t gj = J * ts + v * BLK + c;
    double val;
    if (zero_tile) {
      val = 0.0;
    } else if (ipad || gj >= nreal) {
      val = (gi == gj) ? 1.0 : 0.0;
    } else {
      val = matern_value(loc_dist(xi, yi, xs[gj], ys[gj], cst), cst, qt);
      if (gi == gj) val += cst[C_NUG];  // the observation's own noise
    }
    const int64_t e = (int64_t)c * ts;
    if (kind == 0) out64[e] = val;
    else if (kind == 1) out32[e] = (float)val;
    else out16[e] = f32_to_bf16_rne((float)val);
  }
}

// cov[i + j ldc] = Sigma(s_i, s_j) in the caller's order.
__global__ __launch_bounds__(256) void k_gen_dense(double* __restrict__ cov, int64_t ldc, int64_t n,
                                                   const double* __restrict__ x, const double* __restrict__ y,
                                                   const double* __restrict__ qt, const double* __restrict__ cst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i], yi = y[i];
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
    cov[i + j * ldc] = matern_value(loc_dist(xi, yi, x[j], y[j], cst), cst, qt) + (i == j ? cst[C_NUG] : 0.0);
  }
}

int64_t quad_table_doubles() { return QT_TOTAL; }

// qt: QT_TOTAL doubles (quadrature nodes, then the Chebyshev tables)
void launch_quad_table(const double theta[3], int metric, double nugget, double* qt, double* cst, hipStream_t s) {
  hipLaunchKernelGGL(k_quad_table, dim3(QNB), dim3(QNK), 0, s, theta[0], theta[1], theta[2], (double)metric, nugget,
                     qt, cst);
  hipLaunchKernelGGL(k_cheb_table, dim3(CH_NSEG), dim3(64), 0, s, qt, (const double*)cst);
}

void launch_gen_tiles(const TileMat& M, int64_t nreal, const double* xs, const double* ys, const double* qt,
                      const double* cst, const uint8_t* tag, hipStream_t s) {
  const int64_t ts = M.ts, NT = M.NT;
  const int T = (int)(ts / BLK);
  const int64_t ntile = NT * (NT + 1) / 2;
  // keep each launch's grid below 2^31 blocks
  const int64_t per = (int64_t)1 << 24;
  for (int64_t f = 0; f < ntile; f += per) {
    const int64_t cnt = (ntile - f < per) ? ntile - f : per;
    hipLaunchKernelGGL(k_gen_tiles, dim3((unsigned)(cnt * T * T)), dim3(256), 0, s, M, T, nreal, xs, ys, qt, cst, tag,
                       f);
  }
}

// r_i = z_i - sum_j Sigma_ij a_j over the real points (Sigma regenerated in
// FP64, the nugget on the diagonal), r_i = 0 on padded rows; one 256-thread
// workgroup per row, fixed-order reduction.  The residual of a solve done
// through a lower-precision factor.
__global__ __launch_bounds__(256) void k_sigma_residual(const double* __restrict__ xs, const double* __restrict__ ys,
                                                        const double* __restrict__ zs, const double* __restrict__ av,
                                                        int64_t nreal, int64_t npad, const double* __restrict__ qt,
                                                        const double* __restrict__ cst, double* __restrict__ r) {
  __shared__ double red[256];
  const int64_t i = blockIdx.x;
  if (i >= npad) return;
  if (i >= nreal) {
    if (threadIdx.x == 0) r[i] = 0.0;
    return;
  }
  const double px = xs[i], py = ys[i];
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < nreal; j += 256)
    s += matern_value(loc_dist(px, py, xs[j], ys[j], cst), cst, qt) * av[j];
  double v[1] = {s};
  block_sum<1>(v, red);
  if (threadIdx.x == 0) r[i] = zs[i] - (v[0] + cst[C_NUG] * av[i]);
}

void launch_sigma_residual(const double* xs, const double* ys, const double* zs, const double* av, int64_t nreal,
                           int64_t npad, const double* qt, const double* cst, double* r, hipStream_t s) {
  hipLaunchKernelGGL(k_sigma_residual, dim3((unsigned)npad), dim3(256), 0, s, xs, ys, zs, av, nreal, npad, qt, cst, r);
}

void launch_gen_dense(double* cov, int64_t ldc, int64_t n, const double* x, const double* y, const double* qt,
                      const double* cst, hipStream_t s) {
  const unsigned gx = (unsigned)((n + 255) / 256);
  const unsigned gy = (unsigned)(n < 8192 ? n : 8192);
  hipLaunchKernelGGL(k_gen_dense, dim3(gx, gy), dim3(256), 0, s, cov, ldc, n, x, y, qt, cst);
}

}  // namespace exg
