// Host side of the C ABI: context, workspace plan, the step schedule of the
// likelihood / gradient pipeline and the entry points declared in exageo.h.
#include "exageo.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdarg>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "launch.h"
#include "mle.h"
#include "noalloc.h"

namespace {

constexpr int64_t BLKH = 128;
constexpr int NEV = 512;                     // profiling events

struct Plan {
  int64_t n = 0, ts = 0, NT = 0, T = 0, npad = 0, P = 0;
  bool grad = false;
  bool mixed = false;
  size_t off_diag = 0, off_offt = 0, off_xd = 0, off_dinv = 0, off_ld = 0, off_xs = 0, off_ys = 0, off_zs = 0, off_yv = 0,
         off_av = 0, off_perm = 0, off_keys = 0, off_box = 0, off_qt = 0, off_cst = 0, off_part = 0, off_out = 0,
         off_info = 0, off_tmp = 0, off_y = 0, off_alpha = 0, off_ptmp = 0, off_pbuf = 0, off_p32 = 0, off_pbt = 0, off_tag = 0,
         off_tbox = 0, off_pool = 0, off_pidx = 0, off_bli = 0, off_blj = 0, off_brl = 0, off_b16i = 0, off_b16j = 0, off_corr = 0, off_rtry = 0,
         off_rnrm = 0, off_fb = 0, off_fstrip = 0, off_fpart = 0, off_fout = 0, off_dmin = 0;
  size_t ptmp_doubles = 0;  // FP64 staging of the inverse (also the kriging blocks)
  int nfisher = 0;          // derivative matrices held for the Fisher information (0, 2 or 3)
  int64_t pool_cap = 0;  // mixed precision: FP64 band tiles the pool can hold
  int64_t dst = 0;       // DST tile band (0: exact)
  size_t bytes = 0;
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// want_grad: 0 = l, 1 = l and its gradient, 2 = also the Fisher information
// (two derivative matrices), 3 = the Fisher information with a nugget (three)
Plan make_plan(int64_t n, int64_t ts, int want_grad, int precision = EXAGEO_FP64) {
  Plan p;
  p.n = n;
  p.ts = ts;
  p.NT = (n + ts - 1) / ts;
  p.T = ts / BLKH;
  p.npad = p.NT * ts;
  p.P = 2048;
  while (p.P < p.npad) p.P <<= 1;
  p.grad = want_grad != 0;
  p.mixed = precision == EXAGEO_MIXED;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t tt = (size_t)ts * ts;
  p.off_diag = take((size_t)p.NT * tt * 8);
  const size_t noff = (size_t)std::max<int64_t>(1, p.NT * (p.NT - 1) / 2);
  p.off_offt = take(noff * tt * (p.mixed ? 4 : 8));
  if (p.mixed) {
    // two halves each: the panel of step k + 1 is built while step k's update reads step k's
    p.off_pbuf = take(2 * (size_t)std::max<int64_t>(1, p.NT - 1) * tt * 8);
    p.off_p32 = take(2 * (size_t)std::max<int64_t>(1, p.NT - 1) * tt * 4);
    p.off_pbt = take(2 * (size_t)std::max<int64_t>(1, p.NT - 1) * tt * 2);
    p.off_tag = take(noff);
    p.off_tbox = take((size_t)p.NT * 4 * 8);
    // FP64 tiles of the precision map: up to half of the off-diagonal tiles
    // (at least 4 per tile column), so that the mixed workspace stays about
    // the size of the FP64 one
    p.pool_cap = std::min<int64_t>((int64_t)noff, std::max<int64_t>(4 * p.NT, ((int64_t)noff + 1) / 2));
    p.off_corr = take(noff * 8);
    p.off_dmin = take(noff * 8);  // smallest point distance of every off-diagonal tile
    p.off_rtry = take((size_t)p.npad * 8);  // trial residual of the refinement
    p.off_rnrm = take(4 * 8);
    p.off_pool = take((size_t)std::max<int64_t>(1, p.pool_cap) * tt * 8);
    p.off_pidx = take(noff * 4);
    p.off_bli = take((size_t)std::max<int64_t>(1, p.pool_cap) * 4);
    p.off_blj = take((size_t)std::max<int64_t>(1, p.pool_cap) * 4);
    p.off_brl = take((size_t)std::max<int64_t>(1, p.pool_cap) * 4);  // band list entries by tile rows
    p.off_b16i = take(noff * 4);  // BF16 tiles, column-major list
    p.off_b16j = take(noff * 4);
  }
  p.off_xd = take((size_t)p.NT * tt * 8);
  // FP64 inverse: FP64 staging buffer (the mixed inverse stages in the FP32 panel copy)
  // (two halves: consecutive TRTRI steps stage on different streams); kriging
  // uses it for its blocks of at least 128 new points (2 npad 128 doubles)
  if (p.grad && !p.mixed) {
    p.ptmp_doubles = std::max(2 * (size_t)std::max<int64_t>(1, p.NT - 1) * tt, 2 * (size_t)p.npad * BLKH);
    p.off_ptmp = take(p.ptmp_doubles * 8);
  }
  p.off_dinv = take((size_t)p.NT * p.T * BLKH * BLKH * 8);
  p.off_ld = take((size_t)p.NT * p.T * 8);
  p.off_xs = take((size_t)p.npad * 8);
  p.off_ys = take((size_t)p.npad * 8);
  p.off_zs = take((size_t)p.npad * 8);
  p.off_yv = take((size_t)p.npad * 8);
  p.off_av = take((size_t)p.npad * 8);
  p.off_tmp = take((size_t)p.npad * 8);
  p.off_y = take((size_t)p.npad * 8);
  p.off_alpha = take((size_t)p.npad * 8);
  p.off_perm = take((size_t)p.npad * 4);
  p.off_keys = take((size_t)p.P * 8);
  p.off_box = take(8 * 8);
  p.off_qt = take((size_t)exg::quad_table_doubles() * 8);
  p.off_cst = take(8 * 8);
  p.off_part = take((size_t)(p.grad ? exg::lauum_blocks(ts, p.NT) + p.pool_cap * p.T * p.T : 1) * 3 * 8);
  p.off_out = take(16 * 8);
  p.off_info = take(8);
  if (want_grad >= 2 && !p.mixed) {
    // Fisher information: one buffer of lower tiles per derivative matrix, a
    // strip of tile rows shared by the regenerated derivatives and the staging
    p.nfisher = want_grad == 3 ? 3 : 2;
    const size_t low = (size_t)p.NT * (p.NT + 1) / 2 * tt;
    p.off_fb = take((size_t)p.nfisher * low * 8);
    p.off_fstrip = take(exg::fisher_strip_doubles(ts, p.NT) * 8);
    p.off_fpart = take((size_t)exg::fisher_part_blocks(ts, p.NT) * 9 * 8);
    p.off_fout = take(16 * 8);
  }
  p.bytes = o;
  return p;
}

}  // namespace

enum { POLICY_CORRELATION = 0, POLICY_DISTANCE = 1 };
constexpr double kDefaultRho64 = 0.3;
constexpr double kDefaultRho16 = 1e-4;
constexpr int kDefaultRefine = 1;

struct exageo_ctx {
  int device = 0;
  int64_t ts = 768;
  hipStream_t stream = nullptr;
  // mixed-precision map: by correlation bound (default) or by distance bands
  int policy = POLICY_CORRELATION;
  double rho64 = kDefaultRho64;   // FP64 when the tile's correlation bound is >= rho64
  double rho16 = kDefaultRho16;   // BF16 when it (and its updates' bound) is < rho16
  double band_factor = 3.0;     // distance policy: BF16 at or beyond band_factor * beta
  double fp64_band_factor = 0.0;  // distance policy: FP64 below fp64_band_factor * beta
  int refine = kDefaultRefine;    // FP64 refinement steps of Sigma^-1 z through the mixed factor
  int64_t dst_band = 0;           // DST approximation of loglik / loglik_grad / mle (0: exact)
  int metric = EXAGEO_EUCLIDEAN;  // distance between locations
  double nugget = 0.0;            // tau^2 added to the diagonal
  bool verbose = false;           // exageo_mle prints one line per evaluation
  bool profiling = false;
  std::string err;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  // device address of this device's fixed scratch array (allocation-free
  // entry point), looked up when the context is created
  void* scratch = nullptr;
  // pinned host staging for results
  double* hres = nullptr;
  // current plan and sorted-location cache key (only valid inside one call or an MLE run)
  Plan plan;
  // mixed precision: tile bounding boxes of the sorted locations (host copy)
  // and pinned staging for the per-tile precision tags
  std::vector<double> tbox;
  uint8_t* htag = nullptr;
  size_t htag_bytes = 0;
  double* hcorr = nullptr;  // pinned: correlation bound per off-diagonal tile
  size_t hcorr_words = 0;
  // FP64 band: pool slot per off-diagonal tile, band list (column-major
  // order) and the first list entry of each tile column, all host copies
  int32_t* hband = nullptr;  // pinned: pidx (noff) then li, lj, rl (pool_cap each)
  size_t hband_words = 0;
  std::vector<int64_t> bfirst;
  // the same list by tile rows: rl[r] = list entry, rfirst[i] = first r of row i
  std::vector<int64_t> brfirst;
  // BF16 tiles in column-major order and the first entry of each tile column
  std::vector<int64_t> b16first;
  int bf16_block = 256;  // output block edge of the BF16 update (256 when ts allows, else 128)
  // side stream (default priority) for the lookahead panel, and its events
  hipStream_t side = nullptr;
  hipEvent_t ev_col = nullptr, ev_panel = nullptr;
  // profiling
  hipEvent_t ev[NEV];
  int nev_created = 0;
  double timings[24] = {0};
};

namespace {

exageo_status fail(exageo_ctx* c, exageo_status st, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
exageo_status fail(exageo_ctx* c, exageo_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

// Largest n the kernels' index arithmetic allows at tile size ts: the GEMM
// cores take 32-bit per-thread byte offsets (up to 127 rows of a leading
// dimension npad, 127 * 8 npad < 2^32) and the mixed LAUUM divides k < npad by
// ts through a reciprocal that is exact while npad ts < 2^32.  Device memory
// holds n far below either bound (4.2 million at tile 768).
bool n_fits(int64_t n, int64_t ts) {
  if (n > (int64_t)INT32_MAX) return false;
  const int64_t npad = (n + ts - 1) / ts * ts;
  return npad < ((int64_t)1 << 32) / std::max<int64_t>(ts, 127 * 8);
}

#define HIPCHK(c, expr)                                                                               \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess) return fail((c), EXAGEO_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

bool theta_ok(const double* th) {
  if (!th) return false;
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(th[k]) || !(th[k] > 0.0)) return false;
  return th[2] <= 15.0;
}

exageo_status set_device(exageo_ctx* c) {
  HIPCHK(c, hipSetDevice(c->device));
  return EXAGEO_OK;
}

// make sure the workspace holds plan p
exageo_status ensure_ws(exageo_ctx* c, const Plan& p) {
  if (c->ws && c->ws_bytes >= p.bytes) return EXAGEO_OK;
  if (c->ws && !c->ws_owned)
    return fail(c, EXAGEO_ENOMEM, "workspace of %zu bytes is smaller than the %zu bytes needed", c->ws_bytes,
                p.bytes);
  if (c->ws) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipFree(c->ws));
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  void* ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, p.bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, EXAGEO_ENOMEM, "hipMalloc(%zu) failed: %s", p.bytes, hipGetErrorString(e));
  }
  c->ws = (char*)ptr;
  c->ws_bytes = p.bytes;
  c->ws_owned = true;
  return EXAGEO_OK;
}

template <typename T>
T* at(exageo_ctx* c, size_t off) {
  return reinterpret_cast<T*>(c->ws + off);
}

void rec(exageo_ctx* c, int i) {
  if (c->profiling && i < c->nev_created) (void)hipEventRecord(c->ev[i], c->stream);
}

float ev_ms(exageo_ctx* c, int a, int b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, c->ev[a], c->ev[b]) != hipSuccess) return 0.f;
  return ms;
}

// ---------------------------------------------------------------- pipeline
// Event slots: 0 start, 1 after ordering, 2 after generation, 3 after
// Cholesky, 4 after solve+reduce, 5 after gradient, 6.. pairs around the
// trailing-update launches.
constexpr int EV_UPD0 = 8;

exageo_status prepare_locations(exageo_ctx* c, const Plan& p, const double* x, const double* y, const double* z) {
  exg::launch_sort_locations(x, y, z, p.n, p.npad, p.P, at<double>(c, p.off_box), at<uint64_t>(c, p.off_keys),
                             at<double>(c, p.off_xs), at<double>(c, p.off_ys), at<double>(c, p.off_zs),
                             at<int32_t>(c, p.off_perm), c->stream);
  HIPCHK(c, hipGetLastError());
  if (p.mixed) {
    // bounding boxes of the location blocks of the tiles, for the precision map
    exg::launch_tile_bbox(at<double>(c, p.off_xs), at<double>(c, p.off_ys), p.ts, p.NT, p.n,
                          at<double>(c, p.off_tbox), c->stream);
    if (c->metric == EXAGEO_EUCLIDEAN)
      exg::launch_tile_dmin(at<double>(c, p.off_xs), at<double>(c, p.off_ys), p.ts, p.NT, p.n,
                            at<double>(c, p.off_dmin), c->stream);
    c->tbox.assign((size_t)p.NT * 4, 0.0);
    HIPCHK(c, hipMemcpyAsync(c->tbox.data(), at<double>(c, p.off_tbox), (size_t)p.NT * 4 * 8, hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return EXAGEO_OK;
}

// Precision of every off-diagonal tile (TAG_F32, TAG_BF16 or TAG_F64) and the
// FP64 pool slots, from the tile bounding boxes of the sorted locations.
//   correlation policy: c_ij = correlation at the smallest distance between
//     the points of location blocks i and j (the tile's largest |Sigma_ab| /
//     sigma^2); FP64 when c_ij >= rho64, BF16 when c_ij < rho16 and every
//     update it receives is small too (max over k < j of c_ik c_jk < rho16:
//     the BF16 update multiplies BF16 roundings of L_ik and L_jk), FP32
//     otherwise;
//   distance policy: BF16 when the box distance is >= band_factor * beta,
//     FP64 when it is below fp64_band_factor * beta.
// FP64 candidates beyond the pool's capacity stay FP32, the most correlated
// (closest) first.  With great-circle distances (no planar boxes) every
// off-diagonal tile is FP32.  Returns the BF16 and FP64 fractions.
exageo_status upload_tags(exageo_ctx* c, const Plan& p, const double theta[3], double* frac_bf16, double* frac_fp64) {
  const size_t noff = (size_t)std::max<int64_t>(1, p.NT * (p.NT - 1) / 2);
  const size_t words = 3 * noff + 3 * (size_t)std::max<int64_t>(1, p.pool_cap);
  if (c->htag_bytes < noff) {
    if (c->htag) HIPCHK(c, hipHostFree(c->htag));
    c->htag = nullptr;
    HIPCHK(c, hipHostMalloc((void**)&c->htag, noff));
    c->htag_bytes = noff;
  }
  if (c->hband_words < words) {
    if (c->hband) HIPCHK(c, hipHostFree(c->hband));
    c->hband = nullptr;
    HIPCHK(c, hipHostMalloc((void**)&c->hband, words * 4));
    c->hband_words = words;
  }
  const bool planar = c->metric == EXAGEO_EUCLIDEAN;
  const bool by_corr = c->policy == POLICY_CORRELATION;
  if (planar && by_corr && p.NT > 1) {
    if (c->hcorr_words < noff) {
      if (c->hcorr) HIPCHK(c, hipHostFree(c->hcorr));
      c->hcorr = nullptr;
      HIPCHK(c, hipHostMalloc((void**)&c->hcorr, noff * 8));
      c->hcorr_words = noff;
    }
    exg::launch_tile_corr(at<double>(c, p.off_dmin), p.NT, at<double>(c, p.off_qt), at<double>(c, p.off_cst),
                          at<double>(c, p.off_corr), c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(c->hcorr, at<double>(c, p.off_corr), noff * 8, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));  // previous upload consumed, correlations here
  const double band16 = c->band_factor * theta[1], band64 = c->fp64_band_factor * theta[1];
  int32_t* pidx = c->hband;
  int32_t* li = c->hband + noff;
  int32_t* lj = li + std::max<int64_t>(1, p.pool_cap);
  // candidates for FP64: (closeness key, off index), smallest key first
  std::vector<std::pair<double, int64_t>> cand;
  int64_t nbf = 0, ntot = 0;
  for (int64_t j = 0; j < p.NT; ++j) {
    const double* bj = &c->tbox[4 * j];
    for (int64_t i = j + 1; i < p.NT; ++i) {
      const int64_t idx = exg::off_index(i, j, p.NT);
      pidx[idx] = -1;
      ++ntot;
      c->htag[idx] = exg::TAG_F32;
      if (!planar) continue;
      if (by_corr) {
        const double cij = c->hcorr[idx];
        if (cij >= c->rho64) {
          cand.emplace_back(-cij, idx);
        } else if (cij < c->rho16) {
          double u = 0.0;
          for (int64_t k = 0; k < j && u < c->rho16; ++k)
            u = std::max(u, c->hcorr[exg::off_index(i, k, p.NT)] * c->hcorr[exg::off_index(j, k, p.NT)]);
          if (u < c->rho16) c->htag[idx] = exg::TAG_BF16;
        }
      } else {
        const double* bi = &c->tbox[4 * i];
        const double dx = std::max(0.0, std::max(bi[0] - bj[1], bj[0] - bi[1]));
        const double dy = std::max(0.0, std::max(bi[2] - bj[3], bj[2] - bi[3]));
        const double d = std::sqrt(dx * dx + dy * dy);
        if (c->band_factor > 0.0 && d >= band16) c->htag[idx] = exg::TAG_BF16;
        else if (d < band64) cand.emplace_back(d, idx);
      }
    }
  }
  if ((int64_t)cand.size() > p.pool_cap) {
    std::stable_sort(cand.begin(), cand.end(),
                     [](const std::pair<double, int64_t>& u, const std::pair<double, int64_t>& v) {
                       return u.first < v.first;
                     });
    cand.resize((size_t)p.pool_cap);
  }
  for (const auto& e : cand) c->htag[e.second] = exg::TAG_F64;
  // band list in column-major tile order; pool slots follow the list
  c->bfirst.assign((size_t)p.NT + 1, 0);
  int64_t nb64 = 0;
  for (int64_t j = 0; j < p.NT; ++j) {
    c->bfirst[j] = nb64;
    for (int64_t i = j + 1; i < p.NT; ++i) {
      const int64_t idx = exg::off_index(i, j, p.NT);
      if (c->htag[idx] == exg::TAG_F64) {
        pidx[idx] = (int32_t)nb64;
        li[nb64] = (int32_t)i;
        lj[nb64] = (int32_t)j;
        ++nb64;
      } else if (c->htag[idx] == exg::TAG_BF16) {
        ++nbf;
      }
    }
  }
  c->bfirst[p.NT] = nb64;
  // row order: count per row, prefix sums, then entries in column order within a row
  int32_t* rl = lj + std::max<int64_t>(1, p.pool_cap);
  c->brfirst.assign((size_t)p.NT + 1, 0);
  for (int64_t e = 0; e < nb64; ++e) ++c->brfirst[(size_t)li[e] + 1];
  for (int64_t i = 0; i < p.NT; ++i) c->brfirst[(size_t)i + 1] += c->brfirst[(size_t)i];
  {
    std::vector<int64_t> fill(c->brfirst.begin(), c->brfirst.end() - 1);
    for (int64_t e = 0; e < nb64; ++e) rl[fill[(size_t)li[e]]++] = (int32_t)e;
  }
  if (p.NT == 1) {
    c->htag[0] = exg::TAG_F32;
    pidx[0] = -1;
  }
  // BF16 list (column-major tile order)
  int32_t* b16i = rl + std::max<int64_t>(1, p.pool_cap);
  int32_t* b16j = b16i + noff;
  c->b16first.assign((size_t)p.NT + 1, 0);
  int64_t n16 = 0;
  for (int64_t j = 0; j < p.NT; ++j) {
    c->b16first[(size_t)j] = n16;
    for (int64_t i = j + 1; i < p.NT; ++i)
      if (c->htag[exg::off_index(i, j, p.NT)] == exg::TAG_BF16) {
        b16i[n16] = (int32_t)i;
        b16j[n16] = (int32_t)j;
        ++n16;
      }
  }
  c->b16first[(size_t)p.NT] = n16;
  HIPCHK(c, hipMemcpyAsync(at<uint8_t>(c, p.off_tag), c->htag, noff, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(at<int32_t>(c, p.off_pidx), pidx, noff * 4, hipMemcpyHostToDevice, c->stream));
  if (nb64 > 0) {
    HIPCHK(c, hipMemcpyAsync(at<int32_t>(c, p.off_bli), li, (size_t)nb64 * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(at<int32_t>(c, p.off_blj), lj, (size_t)nb64 * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(at<int32_t>(c, p.off_brl), rl, (size_t)nb64 * 4, hipMemcpyHostToDevice, c->stream));
  }
  if (n16 > 0) {
    HIPCHK(c, hipMemcpyAsync(at<int32_t>(c, p.off_b16i), b16i, (size_t)n16 * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(at<int32_t>(c, p.off_b16j), b16j, (size_t)n16 * 4, hipMemcpyHostToDevice, c->stream));
  }
  *frac_bf16 = ntot ? (double)nbf / (double)ntot : 0.0;
  *frac_fp64 = ntot ? (double)nb64 / (double)ntot : 0.0;
  return EXAGEO_OK;
}

exg::TileMat tilemat(exageo_ctx* c, const Plan& p) {
  exg::TileMat M;
  M.diag = at<double>(c, p.off_diag);
  M.off = at<void>(c, p.off_offt);
  M.ts = p.ts;
  M.NT = p.NT;
  if (p.mixed) {
    M.pool = at<double>(c, p.off_pool);
    M.pidx = at<int32_t>(c, p.off_pidx);
  }
  M.dst = p.dst;
  return M;
}

// FP64 tiles (k+1, k), ..., (NT-1, k): contiguous in the column-packed layout
double* below_fp64(const exg::TileMat& M, int64_t k) {
  return (double*)M.off + exg::off_index(k + 1, k, M.NT) * M.ts * M.ts;
}

// Sigma(theta) tiles and their Cholesky factor in place.
exageo_status factorize(exageo_ctx* c, const Plan& p, const double theta[3]) {
  const exg::TileMat M = tilemat(c, p);
  const int64_t tt = p.ts * p.ts;
  const uint8_t* tag = nullptr;
  c->timings[10] = p.mixed ? EXAGEO_MIXED : EXAGEO_FP64;
  c->timings[11] = 0.0;
  c->timings[12] = 0.0;
  c->timings[14] = 0.0;
  exg::launch_quad_table(theta, c->metric, c->nugget, at<double>(c, p.off_qt), at<double>(c, p.off_cst), c->stream);
  if (p.mixed) {
    double fbf = 0.0, f64 = 0.0;
    exageo_status st = upload_tags(c, p, theta, &fbf, &f64);
    if (st) return st;
    tag = at<uint8_t>(c, p.off_tag);
    c->timings[11] = fbf;
    c->timings[12] = p.NT > 1 ? 1.0 - fbf - f64 : 0.0;
    c->timings[14] = f64;
  }
  exg::launch_fill_info(at<unsigned long long>(c, p.off_info), c->stream);
  exg::launch_gen_tiles(M, p.n, at<double>(c, p.off_xs), at<double>(c, p.off_ys), at<double>(c, p.off_qt),
                        at<double>(c, p.off_cst), tag, c->stream);
  rec(c, 2);
  double upd_flops = 0.0;
  double flops_by[3] = {0.0, 0.0, 0.0};  // FP32, BF16, FP64 targets
  int nupd = 0;
  // Lookahead of one panel: step k first updates the first trailing column
  // (k + 1) on the main stream; the side stream then factors panel k + 1
  // while the main stream runs the rest of step k's update.  In mixed
  // precision the FP64 panel buffer and its FP32 copy alternate between two
  // halves so that panel k + 1 never overwrites the operands of step k.
  hipStream_t S = c->stream, S2 = c->side;
  const bool any_bf16 = p.mixed && c->timings[11] > 0.0;
  const int32_t* bli = p.mixed ? at<int32_t>(c, p.off_bli) : nullptr;
  const int32_t* blj = p.mixed ? at<int32_t>(c, p.off_blj) : nullptr;
  // BF16 targets on 256 x 256 blocks when the tile edge allows
  const bool wide16 = any_bf16 && c->bf16_block == 256 && p.ts % 256 == 0;
  const int32_t* b16i = p.mixed ? at<int32_t>(c, p.off_b16i) : nullptr;
  const int32_t* b16j = p.mixed ? at<int32_t>(c, p.off_b16j) : nullptr;
  const size_t phalf = (size_t)std::max<int64_t>(1, p.NT - 1) * tt;
  auto panel = [&](int64_t k, hipStream_t s) -> double* {
    double* below = nullptr;
    if (k + 1 < p.NT) {
      if (p.mixed) {
        below = at<double>(c, p.off_pbuf) + (k & 1) * phalf;
        exg::launch_panel_gather(M, k, tag, below, s);
      } else {
        below = below_fp64(M, k);
      }
    }
    // DST: the rows below the band are zero and are left alone
    const int64_t prow = p.dst > 0 ? std::min<int64_t>(p.n, (k + p.dst) * p.ts) : p.n;
    exg::launch_panel(M.diag + k * tt, below, p.ts, p.NT, k, prow, at<double>(c, p.off_dinv) + k * p.T * BLKH * BLKH,
                      at<double>(c, p.off_ld) + k * p.T, at<unsigned long long>(c, p.off_info), s);
    if (p.mixed && k + 1 < p.NT) {
      exg::launch_panel_scatter(M, k, tag, below, at<float>(c, p.off_p32) + (k & 1) * phalf, s);
      if (any_bf16) exg::launch_panel_bf16t(M, k, below, at<uint16_t>(c, p.off_pbt) + (k & 1) * phalf, s);
    }
    return below;
  };
  double* below = panel(0, S);
  for (int64_t k = 0; k + 1 < p.NT; ++k) {
    float* p32 = p.mixed ? at<float>(c, p.off_p32) + (k & 1) * phalf : nullptr;
    const uint16_t* pbt = p.mixed && any_bf16 ? at<uint16_t>(c, p.off_pbt) + (k & 1) * phalf : nullptr;
    const int slot = EV_UPD0 + 2 * (int)k;
    if (slot + 1 < c->nev_created) rec(c, slot);
    exg::launch_chol_update(M, below, k, p.n, p.mixed, exg::UPD_FIRST_COLUMN, S);
    if (p.mixed) {
      const int64_t e0 = c->bfirst[k + 1], e1 = c->bfirst[k + 2];
      exg::launch_band_update(M, below, k, p.n, bli, blj, e0, e1 - e0, S);
      exg::launch_update_lp(M, tag, p32, pbt, k, p.n, exg::UPD_FIRST_COLUMN, wide16, S);
      if (wide16) {
        const int64_t f0 = c->b16first[k + 1], f1 = c->b16first[k + 2];
        exg::launch_update_bf16(M, b16i, b16j, f0, f1 - f0, pbt, k, p.n, S);
      }
    }
    HIPCHK(c, hipEventRecord(c->ev_col, S));
    HIPCHK(c, hipStreamWaitEvent(S2, c->ev_col, 0));
    double* next = panel(k + 1, S2);
    HIPCHK(c, hipEventRecord(c->ev_panel, S2));
    exg::launch_chol_update(M, below, k, p.n, p.mixed, exg::UPD_REST, S);
    if (p.mixed) {
      const int64_t e0 = c->bfirst[k + 2], e1 = c->bfirst[p.NT];
      exg::launch_band_update(M, below, k, p.n, bli, blj, e0, e1 - e0, S);
      exg::launch_update_lp(M, tag, p32, pbt, k, p.n, exg::UPD_REST, wide16, S);
      if (wide16) {
        const int64_t f0 = c->b16first[k + 2], f1 = c->b16first[p.NT];
        exg::launch_update_bf16(M, b16i, b16j, f0, f1 - f0, pbt, k, p.n, S);
      }
    }
    if (slot + 1 < c->nev_created) rec(c, slot + 1);
    HIPCHK(c, hipStreamWaitEvent(S, c->ev_panel, 0));
    below = next;
    {
      const int64_t mt = p.dst > 0 ? std::min<int64_t>(p.NT - k - 1, p.dst - 1) : p.NT - k - 1;
      nupd += mt >= 2 ? 2 : (mt == 1 ? 1 : 0);  // launches of k_chol_update in this step
    }
    // algorithmic flops of this update over the real rows, by target precision
    const int64_t iend = p.dst > 0 ? std::min<int64_t>(p.NT, k + p.dst) : p.NT;  // DST: rows in the band
    for (int64_t j = k + 1; j < iend; ++j) {
      const double rj = (double)std::min<int64_t>(p.ts, p.n - j * p.ts);
      upd_flops += rj * (rj + 1.0) * (double)p.ts;  // SYRK
      flops_by[2] += rj * (rj + 1.0) * (double)p.ts;
      for (int64_t i = j + 1; i < iend; ++i) {
        const double ri = (double)std::min<int64_t>(p.ts, p.n - i * p.ts);
        const double f = 2.0 * ri * rj * (double)p.ts;
        upd_flops += f;
        const int tg = p.mixed ? c->htag[exg::off_index(i, j, p.NT)] : (int)exg::TAG_F64;
        flops_by[tg == exg::TAG_F64 ? 2 : (tg == exg::TAG_BF16 ? 1 : 0)] += f;
      }
    }
  }
  HIPCHK(c, hipGetLastError());
  rec(c, 3);
  c->timings[5] = upd_flops;
  c->timings[15] = flops_by[0];
  c->timings[16] = flops_by[1];
  c->timings[17] = flops_by[2];
  c->timings[9] = nupd;
  c->timings[13] = (double)std::max<int64_t>(0, p.NT - 1);
  return EXAGEO_OK;
}

// y = L^-1 z with the explicit inverses of the diagonal tiles, then eq. (2).
// Mixed precision with refinement steps: a = Sigma^-1 z through the mixed
// factor (forward and backward solves) and its residual r = z - Sigma a with
// Sigma regenerated in FP64; each step tries a + (mixed factor)^-1 r and keeps
// it only if its residual is smaller (a step that does not contract, as when
// the mixed factor is too far from Sigma, is not taken).  The quadratic form
// is z^T a, so when the steps converge only log det Sigma carries the mixed
// error.  Everything stays on the device (no host round trip per step).
exageo_status solve_reduce(exageo_ctx* c, const Plan& p) {
  double* rhs = at<double>(c, p.off_yv);
  double* y = at<double>(c, p.off_y);
  const exg::TileMat M = tilemat(c, p);
  double* Xd = at<double>(c, p.off_xd);
  exg::launch_diag_inverses(Xd, M.diag, at<double>(c, p.off_dinv), p.ts, p.NT, c->stream);
  exg::launch_copy(rhs, at<double>(c, p.off_zs), p.npad, c->stream);
  c->timings[21] = 0.0;
  if (p.mixed) {
    const uint8_t* tag = at<uint8_t>(c, p.off_tag);
    exg::launch_trsv_fwd_lp(M, tag, Xd, p.n, rhs, y, c->stream);
    if (c->refine > 0) {
      double* av = at<double>(c, p.off_alpha);  // accepted a
      double* at_ = at<double>(c, p.off_y);      // trial a (y is not needed any more)
      double* r = at<double>(c, p.off_yv);       // accepted residual
      double* rt = at<double>(c, p.off_rtry);    // trial residual
      double* w = at<double>(c, p.off_tmp);
      double* d = at<double>(c, p.off_av);
      double* nrm = at<double>(c, p.off_rnrm);
      const double* zs = at<double>(c, p.off_zs);
      const double *xs = at<double>(c, p.off_xs), *ys = at<double>(c, p.off_ys);
      const double *qt = at<double>(c, p.off_qt), *cst = at<double>(c, p.off_cst);
      exg::launch_copy(w, y, p.npad, c->stream);
      exg::launch_trsv_bwd_lp(M, tag, Xd, w, av, c->stream);
      exg::launch_sigma_residual(xs, ys, zs, av, p.n, p.npad, qt, cst, r, c->stream);
      exg::launch_resid_norm(r, p.npad, nrm, 0, c->stream);
      for (int it = 0; it < c->refine; ++it) {
        exg::launch_copy(rt, r, p.npad, c->stream);  // the forward solve consumes its right-hand side
        exg::launch_trsv_fwd_lp(M, tag, Xd, p.n, rt, w, c->stream);
        exg::launch_trsv_bwd_lp(M, tag, Xd, w, d, c->stream);
        exg::launch_add2(at_, av, d, p.npad, c->stream);
        exg::launch_sigma_residual(xs, ys, zs, at_, p.n, p.npad, qt, cst, rt, c->stream);
        exg::launch_resid_norm(rt, p.npad, nrm, 1, c->stream);
        exg::launch_refine_select(av, at_, r, rt, nrm, p.npad, c->stream);
      }
      exg::launch_finalize_loglik_za(zs, av, p.n, at<double>(c, p.off_ld), p.NT * p.T, at<double>(c, p.off_out),
                                     c->stream);
      c->timings[21] = c->refine;
      HIPCHK(c, hipGetLastError());
      rec(c, 4);
      return EXAGEO_OK;
    }
  } else {
    exg::launch_trsv_fwd(M, Xd, p.n, rhs, y, c->stream);
  }
  exg::launch_finalize_loglik(y, p.n, at<double>(c, p.off_ld), p.NT * p.T, at<double>(c, p.off_out), c->stream);
  HIPCHK(c, hipGetLastError());
  rec(c, 4);
  return EXAGEO_OK;
}

// X = L^-1 in place: step k + 1's first half (P = -L_ik X_kk into the other
// staging half, column k + 1 written back) runs on the side stream beside
// step k's second half on the main stream.  ev_col = "first half of the next
// step done"; ev_panel = "the main stream has finished every earlier step".
template <class Right, class Rest>
exageo_status trtri_two_streams(exageo_ctx* c, int64_t NT, Right right, Rest rest) {
  hipStream_t S = c->stream, S2 = c->side;
  HIPCHK(c, hipEventRecord(c->ev_panel, S));
  HIPCHK(c, hipStreamWaitEvent(S2, c->ev_panel, 0));
  right(0, S2);
  HIPCHK(c, hipEventRecord(c->ev_col, S2));
  for (int64_t k = 0; k < NT; ++k) {
    HIPCHK(c, hipStreamWaitEvent(S, c->ev_col, 0));
    if (k + 1 < NT) {
      HIPCHK(c, hipEventRecord(c->ev_panel, S));
      HIPCHK(c, hipStreamWaitEvent(S2, c->ev_panel, 0));
      right(k + 1, S2);
      HIPCHK(c, hipEventRecord(c->ev_col, S2));
    }
    rest(k, S);
  }
  return EXAGEO_OK;
}

exageo_status gradient(exageo_ctx* c, const Plan& p) {
  const exg::TileMat M = tilemat(c, p);
  double* rhs = at<double>(c, p.off_av);
  double* av = at<double>(c, p.off_alpha);
  double* Xd = at<double>(c, p.off_xd);
  int64_t nparts = exg::lauum_blocks(p.ts, p.NT);  // partial triples of the contraction
  const int64_t tt = p.ts * p.ts, half = std::max<int64_t>(1, p.NT - 1) * tt;
  // a = Sigma^-1 z = L^-T y (already there, refined, in mixed precision with
  // refinement steps)
  exg::launch_copy(rhs, at<double>(c, p.off_y), p.npad, c->stream);
  exageo_status st;
  if (p.mixed) {
    // mixed precision: the same steps with the off-diagonal tiles of L^-1 in
    // FP64 on the factor's FP64 band and FP32 elsewhere (staged in the two
    // halves of the FP32 panel copy and of the FP64 panel buffer)
    const uint8_t* tag = at<uint8_t>(c, p.off_tag);
    float* P32 = at<float>(c, p.off_p32);
    double* Q64 = at<double>(c, p.off_pbuf);
    const exg::BandLists bl{at<int32_t>(c, p.off_bli), at<int32_t>(c, p.off_blj), at<int32_t>(c, p.off_brl),
                            c->bfirst.data(), c->brfirst.data()};
    if (c->refine <= 0) exg::launch_trsv_bwd_lp(M, tag, Xd, rhs, av, c->stream);
    st = trtri_two_streams(
        c, p.NT,
        [&](int64_t k, hipStream_t s) {
          exg::launch_trtri_right_lp(M, tag, Xd + k * tt, P32 + (k & 1) * half, Q64 + (k & 1) * half, bl, k, p.n, s);
        },
        [&](int64_t k, hipStream_t s) {
          exg::launch_trtri_rest_lp(M, tag, Xd + k * tt, P32 + (k & 1) * half, Q64 + (k & 1) * half, bl, k, p.n, s);
        });
    if (st) return st;
    nparts = exg::launch_lauum_contract_lp(M, tag, p.n, at<double>(c, p.off_xs), at<double>(c, p.off_ys), av,
                                           at<double>(c, p.off_qt), at<double>(c, p.off_cst),
                                           at<int32_t>(c, p.off_bli), at<int32_t>(c, p.off_blj), c->bfirst[p.NT],
                                           at<double>(c, p.off_part), c->stream);
  } else {
    exg::launch_trsv_bwd(M, Xd, rhs, av, c->stream);
    // L^-1 in place, then the fused LAUUM + contraction
    double* P64 = at<double>(c, p.off_ptmp);
    st = trtri_two_streams(
        c, p.NT,
        [&](int64_t k, hipStream_t s) { exg::launch_trtri_right(M, Xd + k * tt, P64 + (k & 1) * half, k, p.n, s); },
        [&](int64_t k, hipStream_t s) { exg::launch_trtri_rest(M, Xd + k * tt, P64 + (k & 1) * half, k, p.n, s); });
    if (st) return st;
    exg::launch_lauum_contract(M, p.n, at<double>(c, p.off_xs), at<double>(c, p.off_ys), av,
                               at<double>(c, p.off_qt), at<double>(c, p.off_cst), at<double>(c, p.off_part),
                               c->stream);
  }
  exg::launch_finalize_grad(at<double>(c, p.off_part), nparts, at<double>(c, p.off_out) + 3, c->stream);
  HIPCHK(c, hipGetLastError());
  rec(c, 5);
  return EXAGEO_OK;
}

// copy out[0..5] and info to the host and wait
exageo_status fetch(exageo_ctx* c, const Plan& p, double* out6, int64_t* info_sorted, double* box_flag) {
  HIPCHK(c, hipMemcpyAsync(c->hres, at<double>(c, p.off_out), 6 * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->hres + 6, at<double>(c, p.off_info), 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->hres + 7, at<double>(c, p.off_box), 5 * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  memcpy(out6, c->hres, 6 * 8);
  uint64_t inf;
  memcpy(&inf, c->hres + 6, 8);
  *info_sorted = (inf == ~(uint64_t)0) ? 0 : (int64_t)inf;
  if (box_flag) memcpy(box_flag, c->hres + 7, 5 * 8);
  return EXAGEO_OK;
}

// caller index + 1 of the sorted column `col1` (1-based)
int64_t caller_column(exageo_ctx* c, const Plan& p, int64_t col1) {
  if (col1 <= 0 || col1 > p.n) return col1;
  int32_t src = -1;
  if (hipMemcpy(&src, at<int32_t>(c, p.off_perm) + (col1 - 1), 4, hipMemcpyDeviceToHost) != hipSuccess) return col1;
  return (int64_t)src + 1;
}

void finish_timings(exageo_ctx* c, const Plan& p, bool grad) {
  if (!c->profiling) return;
  (void)hipEventSynchronize(c->ev[grad ? 5 : 4]);
  c->timings[0] = ev_ms(c, 0, grad ? 5 : 4);
  c->timings[1] = ev_ms(c, 0, 1);
  c->timings[2] = ev_ms(c, 1, 2);
  c->timings[3] = ev_ms(c, 2, 3);
  double upd = 0.0;
  for (int i = 0; i < (int)c->timings[13]; ++i) {
    const int slot = EV_UPD0 + 2 * i;
    if (slot + 1 < c->nev_created) upd += ev_ms(c, slot, slot + 1);
  }
  c->timings[4] = upd;
  c->timings[6] = ev_ms(c, 3, 4);
  c->timings[7] = grad ? ev_ms(c, 4, 5) : 0.0;
  const double n = (double)p.n;
  c->timings[8] = n * n * n / 3.0 + n * n / 2.0 + n / 6.0;
}

// box[4] counts non-finite values among x, y and z
bool inputs_finite(const double box[5]) { return box[4] == 0.0; }

}  // namespace

// ===================================================================== ABI
extern "C" {

exageo_status exageo_create(exageo_ctx** out, int device, int64_t ts, void* hip_stream) {
  if (!out) return EXAGEO_EINVAL;
  *out = nullptr;
  if (ts < BLKH || ts % BLKH != 0 || ts > 4096) return EXAGEO_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return EXAGEO_EINVAL;
  exageo_ctx* c = new exageo_ctx();
  c->device = device;
  c->ts = ts;
  c->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess || hipHostMalloc((void**)&c->hres, 64 * sizeof(double)) != hipSuccess ||
      hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_col, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_panel, hipEventDisableTiming) != hipSuccess ||
      exg::scratch_address(device, &c->scratch) != hipSuccess) {
    exageo_destroy(c);
    return EXAGEO_EDEVICE;
  }
  *out = c;
  return EXAGEO_OK;
}

void exageo_destroy(exageo_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->ws && c->ws_owned) (void)hipFree(c->ws);
  if (c->hres) (void)hipHostFree(c->hres);
  if (c->htag) (void)hipHostFree(c->htag);
  if (c->hcorr) (void)hipHostFree(c->hcorr);
  if (c->hband) (void)hipHostFree(c->hband);
  for (int i = 0; i < c->nev_created; ++i) (void)hipEventDestroy(c->ev[i]);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  if (c->ev_col) (void)hipEventDestroy(c->ev_col);
  if (c->ev_panel) (void)hipEventDestroy(c->ev_panel);
  delete c;
}

exageo_status exageo_set_stream(exageo_ctx* c, void* hip_stream) {
  if (!c) return EXAGEO_EINVAL;
  c->stream = (hipStream_t)hip_stream;
  return EXAGEO_OK;
}

size_t exageo_workspace_bytes(int64_t n, int64_t ts, int precision, int want_grad) {
  if (n < 1 || ts < BLKH || ts % BLKH != 0 || want_grad < 0 || want_grad > 3) return 0;
  if (precision != EXAGEO_FP64 && precision != EXAGEO_MIXED) return 0;
  return make_plan(n, ts, want_grad, precision).bytes;
}

exageo_status exageo_set_workspace(exageo_ctx* c, void* dev_ptr, size_t bytes) {
  if (!c) return EXAGEO_EINVAL;
  if (set_device(c) != EXAGEO_OK) return EXAGEO_EDEVICE;
  if (c->ws && c->ws_owned) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipFree(c->ws));
  }
  c->ws = (char*)dev_ptr;
  c->ws_bytes = dev_ptr ? bytes : 0;
  c->ws_owned = false;
  return EXAGEO_OK;
}

exageo_status exageo_set_distance(exageo_ctx* c, int metric) {
  if (!c || (metric != EXAGEO_EUCLIDEAN && metric != EXAGEO_GREAT_CIRCLE)) return EXAGEO_EINVAL;
  c->metric = metric;
  return EXAGEO_OK;
}

exageo_status exageo_set_verbose(exageo_ctx* c, int on) {
  if (!c) return EXAGEO_EINVAL;
  c->verbose = on != 0;
  return EXAGEO_OK;
}

exageo_status exageo_set_nugget(exageo_ctx* c, double tau2) {
  if (!c || !(tau2 >= 0.0) || !std::isfinite(tau2)) return EXAGEO_EINVAL;
  c->nugget = tau2;
  return EXAGEO_OK;
}

exageo_status exageo_set_dst_band(exageo_ctx* c, int64_t band) {
  if (!c || band < 0) return EXAGEO_EINVAL;
  c->dst_band = band;
  return EXAGEO_OK;
}

exageo_status exageo_set_mixed_fp64_band(exageo_ctx* c, double fp64_band_factor) {
  if (!c || !(fp64_band_factor >= 0.0) || !std::isfinite(fp64_band_factor)) return EXAGEO_EINVAL;
  c->fp64_band_factor = fp64_band_factor;
  c->policy = POLICY_DISTANCE;
  return EXAGEO_OK;
}

exageo_status exageo_set_mixed_policy(exageo_ctx* c, double band_factor) {
  if (!c || !(band_factor >= 0.0) || !std::isfinite(band_factor)) return EXAGEO_EINVAL;
  c->band_factor = band_factor;
  c->policy = POLICY_DISTANCE;
  return EXAGEO_OK;
}

exageo_status exageo_set_mixed_correlation(exageo_ctx* c, double fp64_at_or_above, double bf16_below) {
  if (!c || !std::isfinite(fp64_at_or_above) || !std::isfinite(bf16_below) || !(bf16_below >= 0.0) ||
      !(fp64_at_or_above >= bf16_below))
    return EXAGEO_EINVAL;
  c->rho64 = fp64_at_or_above;
  c->rho16 = bf16_below;
  c->policy = POLICY_CORRELATION;
  return EXAGEO_OK;
}

exageo_status exageo_set_mixed_refinement(exageo_ctx* c, int steps) {
  if (!c || steps < 0 || steps > 8) return EXAGEO_EINVAL;
  c->refine = steps;
  return EXAGEO_OK;
}

exageo_status exageo_set_mixed_bf16_block(exageo_ctx* c, int edge) {
  if (!c || (edge != 128 && edge != 256)) return EXAGEO_EINVAL;
  c->bf16_block = edge;
  return EXAGEO_OK;
}

const char* exageo_last_error(const exageo_ctx* c) { return c ? c->err.c_str() : "null context"; }

exageo_status exageo_set_profiling(exageo_ctx* c, int on) {
  if (!c) return EXAGEO_EINVAL;
  c->profiling = on != 0;
  if (c->profiling && c->nev_created == 0) {
    if (set_device(c) != EXAGEO_OK) return EXAGEO_EDEVICE;
    for (int i = 0; i < NEV; ++i) {
      if (hipEventCreate(&c->ev[i]) != hipSuccess) break;
      c->nev_created = i + 1;
    }
  }
  return EXAGEO_OK;
}

int exageo_get_timings(const exageo_ctx* c, double* out, int nmax) {
  if (!c || !out) return 0;
  int m = nmax < 24 ? nmax : 24;
  for (int i = 0; i < m; ++i) out[i] = c->timings[i];
  return m;
}

exageo_status exageo_matern_cov(exageo_ctx* c, int64_t n, const double* x, const double* y, const double theta[3],
                                double* cov, int64_t ldc) {
  if (!c) return EXAGEO_EINVAL;
  c->err.clear();
  if (n < 1 || !x || !y || !cov || ldc < n || !theta_ok(theta))
    return fail(c, EXAGEO_EINVAL, "matern_cov: invalid argument");
  if (set_device(c) != EXAGEO_OK) return EXAGEO_EDEVICE;
  Plan p = make_plan(1, c->ts, 0);
  exageo_status st = ensure_ws(c, p);
  if (st) return st;
  exg::launch_quad_table(theta, c->metric, c->nugget, at<double>(c, p.off_qt), at<double>(c, p.off_cst), c->stream);
  exg::launch_gen_dense(cov, ldc, n, x, y, at<double>(c, p.off_qt), at<double>(c, p.off_cst), c->stream);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return EXAGEO_OK;
}

// evaluation at theta on locations already sorted into the workspace
static exageo_status eval_sorted(exageo_ctx* c, const Plan& p, const double theta[3], bool want_grad, double* loglik,
                                 double* grad, int64_t* info, bool check_box) {
  exageo_status st = factorize(c, p, theta);
  if (st) return st;
  st = solve_reduce(c, p);
  if (st) return st;
  double out[6], box[5];
  int64_t inf = 0;
  st = fetch(c, p, out, &inf, box);
  if (st) return st;
  if (check_box && !inputs_finite(box)) return fail(c, EXAGEO_EINVAL, "non-finite location or observation");
  if (inf != 0 || !std::isfinite(out[0])) {
    if (inf == 0) {
      // no non-positive pivot: the non-finite value comes from z
      return fail(c, EXAGEO_EINVAL, "non-finite likelihood (non-finite observations?)");
    }
    if (loglik) *loglik = -INFINITY;
    if (info) *info = caller_column(c, p, inf);
    finish_timings(c, p, false);
    return fail(c, EXAGEO_ENOTPD, "covariance not positive definite at column %lld", (long long)inf);
  }
  if (loglik) *loglik = out[0];
  if (info) *info = 0;
  c->timings[19] = out[1];
  c->timings[20] = out[2];
  if (!want_grad) {
    finish_timings(c, p, false);
    return EXAGEO_OK;
  }
  st = gradient(c, p);
  if (st) return st;
  st = fetch(c, p, out, &inf, nullptr);
  if (st) return st;
  if (grad) {
    grad[0] = out[3];
    grad[1] = out[4];
    grad[2] = out[5];
  }
  finish_timings(c, p, true);
  return EXAGEO_OK;
}

static exageo_status loglik_common(exageo_ctx* c, int64_t n, const double* x, const double* y, const double* z,
                                   const double theta[3], int precision, double* loglik, double* grad, int64_t* info,
                                   bool want_grad) {
  if (!c) return EXAGEO_EINVAL;
  c->err.clear();
  if (info) *info = 0;
  if (n < 1 || !x || !y || !z || !theta_ok(theta) || !loglik || (want_grad && !grad))
    return fail(c, EXAGEO_EINVAL, "loglik: invalid argument");
  if (precision != EXAGEO_FP64 && precision != EXAGEO_MIXED) return fail(c, EXAGEO_EINVAL, "unknown precision");
  if (!n_fits(n, c->ts)) return fail(c, EXAGEO_EINVAL, "n too large for tile size %lld", (long long)c->ts);
  if (set_device(c) != EXAGEO_OK) return EXAGEO_EDEVICE;
  if (precision == EXAGEO_MIXED && c->dst_band > 0)
    return fail(c, EXAGEO_EINVAL, "the DST approximation runs in FP64 only");
  Plan p = make_plan(n, c->ts, want_grad, precision);
  p.dst = c->dst_band;
  exageo_status st = ensure_ws(c, p);
  if (st) return st;
  c->plan = p;
  std::memset(c->timings, 0, sizeof c->timings);
  rec(c, 0);
  st = prepare_locations(c, p, x, y, z);
  if (st) return st;
  rec(c, 1);
  return eval_sorted(c, p, theta, want_grad, loglik, grad, info, true);
}

exageo_status exageo_loglik(exageo_ctx* c, int64_t n, const double* x, const double* y, const double* z,
                            const double theta[3], int precision, double* loglik, int64_t* info) {
  return loglik_common(c, n, x, y, z, theta, precision, loglik, nullptr, info, false);
}

exageo_status exageo_loglik_grad(exageo_ctx* c, int64_t n, const double* x, const double* y, const double* z,
                                 const double theta[3], int precision, double* loglik, double grad[3],
                                 int64_t* info) {
  return loglik_common(c, n, x, y, z, theta, precision, loglik, grad, info, true);
}

exageo_status exageo_loglik_grad_noalloc(exageo_ctx* c, int64_t n, const double* x, const double* y,
                                         const double* z, const double theta[3], double* loglik, double grad[3],
                                         int64_t* info) {
  if (!c) return EXAGEO_EINVAL;
  c->err.clear();
  if (info) *info = 0;
  if (n < 1 || !x || !y || !z || !theta_ok(theta) || !loglik)
    return fail(c, EXAGEO_EINVAL, "loglik_grad_noalloc: invalid argument");
  if (!c->scratch) return fail(c, EXAGEO_EDEVICE, "loglik_grad_noalloc: no scratch address for this device");
  const bool want_grad = grad != nullptr;
  const size_t need = make_plan(n, c->ts, want_grad, EXAGEO_FP64).bytes;
  if (need > exg::kScratchBytes)
    return fail(c, EXAGEO_ENOMEM,
                "loglik_grad_noalloc: n = %lld with tile %lld needs %zu bytes, above the %zu-byte fixed scratch",
                (long long)n, (long long)c->ts, need, exg::kScratchBytes);
  // run the ordinary pipeline on the fixed scratch: it fits, so nothing is
  // allocated; the context's own workspace is restored afterwards
  char* ws = c->ws;
  const size_t ws_bytes = c->ws_bytes;
  const bool ws_owned = c->ws_owned;
  c->ws = (char*)c->scratch;
  c->ws_bytes = exg::kScratchBytes;
  c->ws_owned = false;
  const exageo_status st = loglik_common(c, n, x, y, z, theta, EXAGEO_FP64, loglik, grad, info, want_grad);
  c->ws = ws;
  c->ws_bytes = ws_bytes;
  c->ws_owned = ws_owned;
  return st;
}

exageo_status exageo_simulate(exageo_ctx* c, int64_t n, const double* x, const double* y, const double theta[3],
                              const double* e, double* z, int64_t* info) {
  if (!c) return EXAGEO_EINVAL;
  c->err.clear();
  if (info) *info = 0;
  if (n < 1 || !x || !y || !e || !z || !theta_ok(theta)) return fail(c, EXAGEO_EINVAL, "simulate: invalid argument");
  if (!n_fits(n, c->ts)) return fail(c, EXAGEO_EINVAL, "n too large for tile size %lld", (long long)c->ts);
  if (set_device(c) != EXAGEO_OK) return EXAGEO_EDEVICE;
  Plan p = make_plan(n, c->ts, 0);
  exageo_status st = ensure_ws(c, p);
  if (st) return st;
  // sorted copy of e goes to zs
  st = prepare_locations(c, p, x, y, e);
  if (st) return st;
  st = factorize(c, p, theta);
  if (st) return st;
  double* w = at<double>(c, p.off_tmp);
  exg::launch_trmv_lower(tilemat(c, p), p.n, at<double>(c, p.off_zs), w, c->stream);
  exg::launch_scatter(w, at<int32_t>(c, p.off_perm), p.n, z, c->stream);
  HIPCHK(c, hipGetLastError());
  double out[6], box[5];
  int64_t inf = 0;
  exg::launch_finalize_loglik(w, p.n, at<double>(c, p.off_ld), p.NT * p.T, at<double>(c, p.off_out), c->stream);
  st = fetch(c, p, out, &inf, box);
  if (st) return st;
  if (!inputs_finite(box)) return fail(c, EXAGEO_EINVAL, "non-finite location or draw");
  if (inf != 0) {
    if (info) *info = caller_column(c, p, inf);
    return fail(c, EXAGEO_ENOTPD, "covariance not positive definite at column %lld", (long long)inf);
  }
  return EXAGEO_OK;
}

exageo_status exageo_mle(exageo_ctx* c, int64_t n, const double* x, const double* y, const double* z,
                         const double lb[3], const double ub[3], const double* theta0, double tol, int max_iters,
                         int method, int precision, double theta_hat[3], double* loglik_hat,
                         exageo_mle_stats* stats) {
  if (!c) return EXAGEO_EINVAL;
  c->err.clear();
  if (n < 1 || !x || !y || !z || !lb || !ub || !theta_hat || !loglik_hat || !(tol >= 0.0) || max_iters < 0)
    return fail(c, EXAGEO_EINVAL, "mle: invalid argument");
  if (method != EXAGEO_DFO && method != EXAGEO_LBFGSB && method != EXAGEO_LBFGSB_FP64_FINISH)
    return fail(c, EXAGEO_EINVAL, "unknown method");
  if (precision != EXAGEO_FP64 && precision != EXAGEO_MIXED) return fail(c, EXAGEO_EINVAL, "unknown precision");
  for (int k = 0; k < 3; ++k) {
    if (!theta_ok(lb) || !theta_ok(ub) || lb[k] > ub[k]) return fail(c, EXAGEO_EINVAL, "mle: bad bounds");
    if (theta0 && (!(theta0[k] >= lb[k]) || !(theta0[k] <= ub[k]))) return fail(c, EXAGEO_EINVAL, "theta0 outside bounds");
  }
  if (set_device(c) != EXAGEO_OK) return EXAGEO_EDEVICE;
  const bool want_grad = method != EXAGEO_DFO;
  if (precision == EXAGEO_MIXED && c->dst_band > 0)
    return fail(c, EXAGEO_EINVAL, "the DST approximation runs in FP64 only");
  // mixed search with an FP64 finish: both plans live in one workspace, in turn
  const bool finish64 = method == EXAGEO_LBFGSB_FP64_FINISH && precision == EXAGEO_MIXED;
  Plan p = make_plan(n, c->ts, want_grad, precision);
  p.dst = c->dst_band;
  Plan p64 = make_plan(n, c->ts, 1, EXAGEO_FP64);
  p64.dst = c->dst_band;
  exageo_status st = ensure_ws(c, finish64 && p64.bytes > p.bytes ? p64 : p);
  if (st) return st;
  c->plan = p;
  st = prepare_locations(c, p, x, y, z);
  if (st) return st;
  const Plan* cur = &p;
  const auto t0 = std::chrono::steady_clock::now();
  int64_t nev = 0, ngev = 0;
  exageo_status first_err = EXAGEO_OK;
  bool checked_box = false;
  exg::Objective obj = [&](const double th[3], bool g, double* f, double gr[3]) -> bool {
    double ll = -INFINITY;
    int64_t inf = 0;
    exageo_status s = eval_sorted(c, *cur, th, g, &ll, gr, &inf, !checked_box);
    checked_box = true;
    if (g) ++ngev;
    else ++nev;
    if (c->verbose) {
      std::fprintf(stderr, "[exageo_mle] eval %lld %s%s theta = (%.10g, %.10g, %.10g) l = %.12g%s\n",
                   (long long)(nev + ngev), cur->mixed ? "mixed" : "fp64", g ? " +grad" : "", th[0], th[1], th[2],
                   ll, s == EXAGEO_OK ? "" : " (failed)");
      std::fflush(stderr);
    }
    if (s == EXAGEO_OK) {
      *f = ll;
      return true;
    }
    if (s != EXAGEO_ENOTPD && first_err == EXAGEO_OK) first_err = s;
    *f = -INFINITY;
    return s == EXAGEO_ENOTPD;
  };
  double th0[3];
  // default start: the lower bound for the derivative-free search (the
  // paper's convention); the geometric centre of the box for the gradient
  // method, whose first step would otherwise sit on the flat face beta -> 0
  for (int k = 0; k < 3; ++k)
    th0[k] = theta0 ? theta0[k] : (method == EXAGEO_DFO ? lb[k] : std::sqrt(lb[k] * ub[k]));
  exg::MleResult res;
  int64_t nfinish = 0;
  if (method == EXAGEO_DFO) {
    res = exg::maximize_dfo(obj, lb, ub, th0, tol, max_iters);
  } else if (!finish64) {
    res = exg::maximize_lbfgsb(obj, lb, ub, th0, tol, max_iters);
  } else {
    // the mixed l carries rounding noise of the order of its error (its
    // factor is a perturbed Sigma's), which keeps the search from meeting an
    // absolute tol at large n: search in mixed precision while l still
    // improves by more than 1e-6 |l| (at most half the budget, 40 evaluations
    // when unlimited), then finish in FP64 from the best mixed point with the
    // quasi-Newton model the mixed search built (its scores are accurate), so
    // that the finish takes model steps at once; it ends after two accepted
    // steps in a row below tol
    const int cap1 = max_iters > 0 ? std::max(1, max_iters / 2) : 40;
    exg::Curvature curv;
    const exg::MleResult r1 = exg::maximize_lbfgsb(obj, lb, ub, th0, tol, cap1, 1e-6, 1, &curv);
    if (first_err != EXAGEO_OK) return first_err;
    double th1[3];
    for (int k = 0; k < 3; ++k) th1[k] = std::isfinite(r1.f) ? r1.theta[k] : th0[k];
    cur = &p64;
    c->plan = p64;
    st = prepare_locations(c, p64, x, y, z);
    if (st) return st;
    const int64_t used = nev + ngev, before = ngev;
    const int cap2 = max_iters > 0 ? (int)std::max<int64_t>(1, max_iters - used) : 0;
    res = exg::maximize_lbfgsb(obj, lb, ub, th1, tol, cap2, 0.0, curv.count > 0 ? 2 : 3, &curv);
    res.iters += r1.iters;
    nfinish = ngev - before;
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (first_err != EXAGEO_OK) return first_err;
  for (int k = 0; k < 3; ++k) theta_hat[k] = res.theta[k];
  *loglik_hat = res.f;
  if (stats) {
    stats->n_evals = nev;
    stats->n_grad_evals = ngev;
    stats->iters = res.iters;
    stats->total_s = secs;
    stats->per_eval_s = (nev + ngev) ? secs / (double)(nev + ngev) : 0.0;
    stats->status = res.converged ? EXAGEO_OK : EXAGEO_ENOCONV;
    stats->n_fp64_finish_evals = nfinish;
  }
  if (!std::isfinite(res.f)) return fail(c, EXAGEO_ENOTPD, "no feasible point found");
  return res.converged ? EXAGEO_OK : fail(c, EXAGEO_ENOCONV, "max_iters reached before tol");
}

exageo_status exageo_predict(exageo_ctx* c, int64_t n, const double* x, const double* y, const double* z,
                             const double theta[3], int64_t m, const double* xnew, const double* ynew, double* mean,
                             double* mse, int64_t* info) {
  if (!c) return EXAGEO_EINVAL;
  c->err.clear();
  if (info) *info = 0;
  if (n < 1 || !x || !y || !z || !theta_ok(theta) || m < 0 || (m > 0 && (!xnew || !ynew || !mean)))
    return fail(c, EXAGEO_EINVAL, "predict: invalid argument");
  if (!n_fits(n, c->ts) || m > (int64_t)INT32_MAX) return fail(c, EXAGEO_EINVAL, "n or m too large");
  if (set_device(c) != EXAGEO_OK) return EXAGEO_EDEVICE;
  Plan p = make_plan(n, c->ts, 1, EXAGEO_FP64);  // the gradient plan: its staging holds the kriging blocks
  exageo_status st = ensure_ws(c, p);
  if (st) return st;
  c->plan = p;
  std::memset(c->timings, 0, sizeof c->timings);
  rec(c, 0);
  st = prepare_locations(c, p, x, y, z);
  if (st) return st;
  rec(c, 1);
  double ll = 0.0;
  st = eval_sorted(c, p, theta, false, &ll, nullptr, info, true);
  if (st) return st;
  if (m == 0) return EXAGEO_OK;
  const exg::TileMat M = tilemat(c, p);
  double* Xd = at<double>(c, p.off_xd);
  double* av = at<double>(c, p.off_alpha);
  // a = Sigma^-1 z = L^-T y, then the mean in one pass over (new, observed) pairs
  exg::launch_copy(at<double>(c, p.off_av), at<double>(c, p.off_y), p.npad, c->stream);
  exg::launch_trsv_bwd(M, Xd, at<double>(c, p.off_av), av, c->stream);
  exg::launch_krige_mean(at<double>(c, p.off_xs), at<double>(c, p.off_ys), av, p.n, xnew, ynew, m,
                         at<double>(c, p.off_qt), at<double>(c, p.off_cst), mean, c->stream);
  if (mse) {
    // blocks of up to 512 new points (as many as the staging buffer holds, at
    // least 128): C = Sigma(obs, new), V = L^-1 C
    const int64_t fit = (int64_t)(p.ptmp_doubles / (2 * (size_t)p.npad)) / 128 * 128;
    const int64_t mcap = std::min<int64_t>(std::min<int64_t>(512, fit), (m + 127) / 128 * 128);
    double* Cb = at<double>(c, p.off_ptmp);
    double* Vb = Cb + (size_t)p.npad * mcap;
    for (int64_t c0 = 0; c0 < m; c0 += mcap) {
      const int64_t cols = std::min<int64_t>(mcap, (m - c0 + 127) / 128 * 128);
      exg::launch_krige_mse(M, Xd, at<double>(c, p.off_xs), at<double>(c, p.off_ys), p.n, xnew, ynew, m, c0, cols,
                            at<double>(c, p.off_qt), at<double>(c, p.off_cst), Cb, Vb, mse, c->stream);
    }
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return EXAGEO_OK;
}

exageo_status exageo_fisher(exageo_ctx* c, int64_t n, const double* x, const double* y, const double theta[3],
                            double fisher[9], int64_t* info) {
  if (!c) return EXAGEO_EINVAL;
  c->err.clear();
  if (info) *info = 0;
  if (n < 1 || !x || !y || !theta_ok(theta) || !fisher) return fail(c, EXAGEO_EINVAL, "fisher: invalid argument");
  if (!n_fits(n, c->ts)) return fail(c, EXAGEO_EINVAL, "n too large for tile size %lld", (long long)c->ts);
  if (c->dst_band > 0) return fail(c, EXAGEO_EINVAL, "the Fisher information is computed for the exact covariance only");
  if (set_device(c) != EXAGEO_OK) return EXAGEO_EDEVICE;
  const bool nug = c->nugget > 0.0;  // B_sigma2 is then not I / sigma2
  Plan p = make_plan(n, c->ts, nug ? 3 : 2, EXAGEO_FP64);
  exageo_status st = ensure_ws(c, p);
  if (st) return st;
  c->plan = p;
  std::memset(c->timings, 0, sizeof c->timings);
  rec(c, 0);
  // the observations do not enter I(theta): x stands in for them in the sort
  st = prepare_locations(c, p, x, y, x);
  if (st) return st;
  rec(c, 1);
  double ll = 0.0;
  st = eval_sorted(c, p, theta, false, &ll, nullptr, info, true);
  if (st) return st;
  const exg::TileMat M = tilemat(c, p);
  double* Xd = at<double>(c, p.off_xd);
  // L^-1 in place (the tile matrix then holds X = L^-1, lower-triangular tiles)
  {
    const int64_t tt = p.ts * p.ts, half = std::max<int64_t>(1, p.NT - 1) * tt;
    double* P64 = at<double>(c, p.off_ptmp);
    st = trtri_two_streams(
        c, p.NT,
        [&](int64_t k, hipStream_t s) { exg::launch_trtri_right(M, Xd + k * tt, P64 + (k & 1) * half, k, p.n, s); },
        [&](int64_t k, hipStream_t s) { exg::launch_trtri_rest(M, Xd + k * tt, P64 + (k & 1) * half, k, p.n, s); });
    if (st) return st;
  }
  const size_t low = (size_t)p.NT * (p.NT + 1) / 2 * (size_t)p.ts * p.ts;
  double* fb = at<double>(c, p.off_fb);
  double* Bb = fb;                       // B_beta
  double* Bn = fb + low;                 // B_nu
  double* Bs = nug ? fb + 2 * low : nullptr;  // B_sigma2
  double* strip = at<double>(c, p.off_fstrip);
  double* out = at<double>(c, p.off_fout);
  const double* xs = at<double>(c, p.off_xs);
  const double* ys = at<double>(c, p.off_ys);
  const double* qt = at<double>(c, p.off_qt);
  const double* cst = at<double>(c, p.off_cst);
  exg::launch_fisher_param(M, 1, p.n, xs, ys, qt, cst, strip, Bb, c->stream);
  exg::launch_fisher_param(M, 2, p.n, xs, ys, qt, cst, strip, Bn, c->stream);
  if (nug) exg::launch_fisher_param(M, 0, p.n, xs, ys, qt, cst, strip, Bs, c->stream);
  exg::launch_fisher_reduce(Bs, Bb, Bn, p.ts, p.NT, p.n, cst, at<double>(c, p.off_fpart), out, c->stream);
  rec(c, 5);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(c->hres, out, 9 * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  memcpy(fisher, c->hres, 9 * 8);
  if (c->profiling) {
    c->timings[0] = ev_ms(c, 0, 5);
    c->timings[7] = ev_ms(c, 4, 5);
    // MFMA flops of the two products per parameter over the R real 128-blocks:
    // X G over the lower block pairs (g, h), h <= g, each over g + 1
    // 128-columns (sum_g (g + 1)^2 = R (R + 1) (2R + 1) / 6 block products),
    // and M X^T over the same pairs with h + 1 (sum = R (R + 1) (R + 2) / 6);
    // together R (R + 1)^2 / 2
    const double R = (double)((p.n + BLKH - 1) / BLKH), b3 = 2.0 * BLKH * BLKH * BLKH;
    c->timings[18] = (nug ? 3.0 : 2.0) * b3 * (R * (R + 1.0) * (R + 1.0) / 2.0);
  }
  return EXAGEO_OK;
}

}  // extern "C"
