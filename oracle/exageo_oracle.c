/*
 * exageo_oracle.c -- plain, slow, obviously-correct FP64 reference for the
 * exact Gaussian log-likelihood of a Matern random field.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only tests/, the package smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU path.
 *
 * What it computes (ExaGeoStatR paper, Section 1):
 *   - the Matern covariance of eq. (3), with x = r / beta exactly as printed
 *     (no sqrt(2 nu) rescaling) and Sigma_ii = sigma^2 at r = 0;
 *   - the zero-mean Gaussian log-likelihood of eq. (2),
 *       l = -1/2 (n log 2 pi + log det Sigma + z^T Sigma^-1 z),
 *     through an unblocked Cholesky factor, a forward solve, 2 sum log L_ii
 *     and y^T y (the three operations the paper names for the likelihood);
 *   - the score dl/dtheta_k = 1/2 a^T dSigma_k a - 1/2 tr(Sigma^-1 dSigma_k),
 *     a = Sigma^-1 z, with Sigma^-1 formed explicitly (L^-1, then L^-T L^-1).
 *     The paper's optimiser is derivative free; this is the textbook Gaussian
 *     score (Rasmussen & Williams 2006, eq. 5.9).
 *
 * Special functions are written here from published mathematics:
 *   K_nu : Temme's series (J. Comput. Phys. 19, 1975) for x < 1.25 at order
 *          |mu| <= 1/2, with Gamma_1/Gamma_2 from the Taylor series of
 *          log Gamma(1+z) (DLMF 5.7.3); for x >= 1.25 the minimal solution of
 *          the three-term recurrence of U(nu+1/2+n, 2nu+1, 2x) (DLMF 13.3.7,
 *          10.39.6) by Miller's backward recurrence (Gautschi, SIAM Rev. 9,
 *          1967), normalised with Temme's sum  sum_n C_n U_n = (2x)^(-nu-1/2);
 *          then upward recurrence in the order (DLMF 10.29.1).
 *   dK_nu/dnu : integral of t sinh(nu t) exp(-x cosh t) over (0, inf)
 *          (DLMF 10.32.9 differentiated in nu), adaptive Gauss-Legendre with
 *          nodes computed here by Newton's method.
 *   psi  : recurrence psi(z+1) = psi(z) + 1/z and the asymptotic series
 *          (DLMF 5.5.2, 5.11.2).
 * libm supplies exp, log, sqrt, sinh, cosh, lgamma, tgamma.
 *
 * Precision: everything in double.  Build with -O2 -ffp-contract=off.  The
 * optional OpenMP pragmas only split loops whose iterations are independent
 * (each dot product keeps its order), so results are bitwise identical for any
 * thread count.
 *
 * Status codes: 0 ok, -1 invalid argument, -2 matrix not positive definite
 * (info = 1-based column of the first non-positive pivot).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOTPD (-2)

static const double OR_PI = 3.14159265358979323846;
static const double OR_EULER = 0.57721566490153286061;
static const double OR_LN2 = 0.69314718055994530942;

/* ------------------------------------------------------------------ */
/* Riemann zeta at integers k >= 2: direct sum to N-1 plus Euler-Maclaurin
 * tail  N^(1-k)/(k-1) + N^-k/2 + sum_j B_2j/(2j)! (k)_(2j-1) N^(-k-2j+1). */
static double or_zeta_int(int k) {
  const int N = 12;
  static const double B2j[6] = {1.0 / 6, -1.0 / 30, 1.0 / 42, -1.0 / 30, 5.0 / 66, -691.0 / 2730};
  double s = 0.0;
  for (int n = N - 1; n >= 1; --n) s += pow((double)n, -(double)k);
  double Nd = (double)N;
  s += pow(Nd, 1.0 - k) / (k - 1.0) + 0.5 * pow(Nd, -(double)k);
  double fact = 1.0;   /* (2j)! */
  double rising = 1.0; /* k (k+1) ... (k+2j-2) */
  for (int j = 1; j <= 6; ++j) {
    fact *= (2.0 * j - 1.0) * (2.0 * j);
    if (j == 1)
      rising = k;
    else
      rising *= (k + 2.0 * j - 3.0) * (k + 2.0 * j - 2.0);
    s += B2j[j - 1] / fact * rising * pow(Nd, -(double)k - 2.0 * j + 1.0);
  }
  return s;
}

/* log Gamma(1+mu) = -gamma mu + sum_{k>=2} (-1)^k zeta(k) mu^k / k (DLMF 5.7.3),
 * split into its even part E(mu) and odd part O(mu) = mu * O1(mu). */
static void or_lngamma1p_parts(double mu, double *E, double *O1) {
  double e = 0.0, o1 = -OR_EULER;
  double mkm1 = mu; /* mu^(k-1) for k = 2 */
  for (int k = 2; k <= 70; ++k) {
    double t = ((k % 2) ? -1.0 : 1.0) * or_zeta_int(k) / k;
    if (k % 2 == 0)
      e += t * mkm1 * mu; /* mu^k */
    else
      o1 += t * mkm1; /* mu^(k-1) */
    mkm1 *= mu;
    if (fabs(mkm1) < 1e-40) break;
  }
  *E = e;
  *O1 = o1;
}

/* sinh(v)/v, stable near 0 */
static double or_sinhc(double v) {
  if (fabs(v) < 1e-4) return 1.0 + v * v / 6.0 * (1.0 + v * v / 20.0);
  return sinh(v) / v;
}

/* Temme's series at order mu, |mu| <= 1/2, 0 < x < 1.25.
 * Returns K_mu(x) and K_{mu+1}(x). */
static void or_temme(double mu, double x, double *k0, double *k1) {
  double E, O1;
  or_lngamma1p_parts(mu, &E, &O1);
  double O = mu * O1;
  /* 1/Gamma(1 -+ mu) = exp(-E +- O):
   * Gamma_1 = (1/Gamma(1-mu) - 1/Gamma(1+mu)) / (2 mu) = e^-E sinh(O)/mu
   * Gamma_2 = (1/Gamma(1-mu) + 1/Gamma(1+mu)) / 2     = e^-E cosh(O) */
  double g1 = exp(-E) * or_sinhc(O) * O1;
  double g2 = exp(-E) * cosh(O);
  double lx = log(2.0 / x);
  double sig = mu * lx;
  double pimu = OR_PI * mu;
  double fac = (fabs(pimu) < 1e-300) ? 1.0 : pimu / sin(pimu);
  double f = fac * (cosh(sig) * g1 + or_sinhc(sig) * lx * g2);
  double p = 0.5 * exp(sig) * tgamma(1.0 + mu);  /* (x/2)^-mu Gamma(1+mu) / 2 */
  double q = 0.5 * exp(-sig) * tgamma(1.0 - mu); /* (x/2)^mu Gamma(1-mu) / 2 */
  double c = 1.0;
  double s0 = f, s1 = p;
  double d = 0.25 * x * x;
  for (int k = 1; k < 500; ++k) {
    f = (k * f + p + q) / ((double)k * k - mu * mu);
    p /= (k - mu);
    q /= (k + mu);
    c *= d / k;
    double h = p - k * f;
    s0 += c * f;
    s1 += c * h;
    if (fabs(c * f) < 1e-18 * fabs(s0) && fabs(c * h) < 1e-18 * fabs(s1)) break;
  }
  *k0 = s0;
  *k1 = 2.0 * s1 / x;
}

/* e^x K_nu(x) for x >= 1.25 (any real nu), from the minimal solution
 * u_n = U(nu+1/2+n, 2nu+1, 2x) of
 *   u_{n-1} = 2 (n + x) u_n - a_{n+1} u_{n+1},  a_m = (m - 1/2)^2 - nu^2,
 * and  sum_n C_n u_n = (2x)^(-nu-1/2),  C_0 = 1, C_{n+1} = C_n a_{n+1}/(n+1).
 * Then K_nu(x) = sqrt(pi/(2x)) e^-x / (sum_n C_n u_n / u_0). */
static double or_besselk_scaled_cf(double nu, double x) {
  enum { NTOP = 120 };
  double C[NTOP + 1];
  C[0] = 1.0;
  for (int n = 0; n < NTOP; ++n) {
    double a = (n + 0.5) * (n + 0.5) - nu * nu;
    C[n + 1] = C[n] * a / (n + 1.0);
  }
  double up1 = 0.0, u = 1.0;
  double S = C[NTOP] * u;
  for (int n = NTOP; n >= 1; --n) {
    double a = (n + 0.5) * (n + 0.5) - nu * nu;
    double um1 = 2.0 * (n + x) * u - a * up1;
    up1 = u;
    u = um1;
    S += C[n - 1] * u;
    if (fabs(u) > 1e200) {
      up1 *= 1e-200;
      u *= 1e-200;
      S *= 1e-200;
    }
  }
  return sqrt(OR_PI / (2.0 * x)) / (S / u);
}

/* e^x K_nu(x), x > 0, any real nu. */
double oracle_besselk_scaled(double nu, double x) {
  if (!(x > 0.0) || !isfinite(nu)) return NAN;
  nu = fabs(nu); /* K_{-nu} = K_nu (DLMF 10.27.3) */
  double Nf = floor(nu + 0.5);
  int N = (int)Nf;
  double mu = nu - Nf; /* in [-1/2, 1/2) */
  double k0, k1;
  if (x < 1.25) {
    or_temme(mu, x, &k0, &k1);
    double ex = exp(x);
    k0 *= ex;
    k1 *= ex;
  } else {
    k0 = or_besselk_scaled_cf(mu, x);
    k1 = or_besselk_scaled_cf(mu + 1.0, x);
  }
  if (N == 0) return k0;
  /* K_{m+1} = K_{m-1} + (2 m / x) K_m, m = mu+1, ..., mu+N-1 */
  for (int k = 1; k < N; ++k) {
    double m = mu + k;
    double k2 = k0 + 2.0 * m / x * k1;
    k0 = k1;
    k1 = k2;
  }
  return k1;
}

double oracle_besselk(double nu, double x) { return oracle_besselk_scaled(nu, x) * exp(-x); }

/* ------------------------------------------------------------------ */
/* Gauss-Legendre nodes/weights on [-1,1] by Newton's method on P_m. */
#define OR_GL_MAX 40
static void or_gauss_legendre(int m, double *xs, double *ws) {
  for (int i = 0; i < (m + 1) / 2; ++i) {
    double z = cos(OR_PI * (i + 0.75) / (m + 0.5));
    double pp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = 0.0;
      for (int j = 1; j <= m; ++j) {
        double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
      }
      pp = m * (z * p0 - p1) / (z * z - 1.0);
      double dz = p0 / pp;
      z -= dz;
      if (fabs(dz) < 1e-16) {
        /* one more pass for the final derivative */
        p0 = 1.0;
        p1 = 0.0;
        for (int j = 1; j <= m; ++j) {
          double p2 = p1;
          p1 = p0;
          p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
        }
        pp = m * (z * p0 - p1) / (z * z - 1.0);
        break;
      }
    }
    xs[i] = -z;
    xs[m - 1 - i] = z;
    ws[i] = ws[m - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

typedef struct {
  int ready;
  double x10[10], w10[10], x20[20], w20[20];
} or_gl_rules;

static or_gl_rules or_rules;

static void or_rules_init(void) {
  if (or_rules.ready) return;
  or_gauss_legendre(10, or_rules.x10, or_rules.w10);
  or_gauss_legendre(20, or_rules.x20, or_rules.w20);
  or_rules.ready = 1;
}

/* integrand of e^x dK_nu/dnu: t sinh(nu t) exp(-x (cosh t - 1)) */
static double or_dnu_integrand(double nu, double x, double t) {
  double cm1 = 2.0 * sinh(0.5 * t) * sinh(0.5 * t); /* cosh t - 1 */
  return t * sinh(nu * t) * exp(-x * cm1);
}

static double or_gl_panel(double nu, double x, double a, double b, int m, const double *xs, const double *ws) {
  double c = 0.5 * (a + b), h = 0.5 * (b - a), s = 0.0;
  for (int i = 0; i < m; ++i) s += ws[i] * or_dnu_integrand(nu, x, c + h * xs[i]);
  return s * h;
}

static double or_adapt(double nu, double x, double a, double b, double tol, int depth) {
  double g10 = or_gl_panel(nu, x, a, b, 10, or_rules.x10, or_rules.w10);
  double g20 = or_gl_panel(nu, x, a, b, 20, or_rules.x20, or_rules.w20);
  /* G20 is far more accurate than G10 on a resolved panel; the difference is
   * accepted once it is below the absolute target or the rounding level. */
  if (fabs(g20 - g10) <= tol + 1e-15 * fabs(g20) || depth > 30) return g20;
  double m = 0.5 * (a + b);
  return or_adapt(nu, x, a, m, 0.5 * tol, depth + 1) + or_adapt(nu, x, m, b, 0.5 * tol, depth + 1);
}

/* e^x dK_nu(x)/dnu = int_0^inf t sinh(nu t) exp(-x (cosh t - 1)) dt, x > 0. */
double oracle_besselk_dnu_scaled(double nu, double x) {
  or_rules_init();
  if (!(x > 0.0)) return NAN;
  double sgn = 1.0;
  if (nu < 0) { /* odd in nu */
    nu = -nu;
    sgn = -1.0;
  }
  if (nu == 0.0) return 0.0;
  /* upper limit: integrand below exp(-60) relative to its scale */
  double T = 1.0;
  while (x * 2.0 * sinh(0.5 * T) * sinh(0.5 * T) - nu * T - log(T + 1.0) < 60.0) T *= 1.25;
  /* a first pass over P panels sets the absolute tolerance */
  enum { P = 8 };
  double coarse = 0.0;
  for (int i = 0; i < P; ++i)
    coarse += or_gl_panel(nu, x, T * i / P, T * (i + 1) / P, 20, or_rules.x20, or_rules.w20);
  double tol = 1e-16 * fabs(coarse) / P;
  double s = 0.0;
  for (int i = 0; i < P; ++i) s += or_adapt(nu, x, T * i / P, T * (i + 1) / P, tol, 0);
  return sgn * s;
}

double oracle_besselk_dnu(double nu, double x) { return oracle_besselk_dnu_scaled(nu, x) * exp(-x); }

/* ------------------------------------------------------------------ */
/* psi(z) for z > 0: recurrence up to z >= 10, then
 * psi(z) ~ ln z - 1/(2z) - sum_k B_2k / (2k z^2k) (DLMF 5.5.2, 5.11.2). */
double oracle_digamma(double z) {
  if (!(z > 0.0)) return NAN;
  double acc = 0.0;
  while (z < 10.0) {
    acc -= 1.0 / z;
    z += 1.0;
  }
  static const double B2k[8] = {1.0 / 6, -1.0 / 30, 1.0 / 42, -1.0 / 30, 5.0 / 66, -691.0 / 2730, 7.0 / 6, -3617.0 / 510};
  double z2 = 1.0 / (z * z), zp = z2, s = 0.0;
  for (int k = 1; k <= 8; ++k) {
    s += B2k[k - 1] / (2.0 * k) * zp;
    zp *= z2;
  }
  return acc + log(z) - 0.5 / z - s;
}

/* ------------------------------------------------------------------ */
/* s2 * 2^(1-nu)/Gamma(nu) * x^nu * e^-x * g, with g a scaled Bessel value.
 * The product form keeps full relative accuracy at small x, where x^nu and
 * K_nu(x) are large and small in inverse proportion; the log form is used
 * only when that product could leave the double range. */
static double or_matern_scale(double s2, double nu, double x, double g) {
  if (nu <= 20.0 && x > 1e-30) return s2 * (pow(2.0, 1.0 - nu) / tgamma(nu)) * pow(x, nu) * (exp(-x) * g);
  return s2 * exp((1.0 - nu) * OR_LN2 - lgamma(nu) + nu * log(x) - x + log(g));
}

/* Matern covariance, eq. (3): sigma2 2^(1-nu)/Gamma(nu) x^nu K_nu(x), x = r/beta. */
double oracle_matern(double r, const double *theta) {
  double s2 = theta[0], beta = theta[1], nu = theta[2];
  if (r == 0.0) return s2;
  double x = r / beta;
  return or_matern_scale(s2, nu, x, oracle_besselk_scaled(nu, x));
}

/* The three partial derivatives of the Matern covariance at distance r.
 *  d/dsigma2 = C/sigma2
 *  d/dbeta   = sigma2 c x^(nu+1) K_{nu-1}(x) / beta   (DLMF 10.29.4, 10.27.3)
 *  d/dnu     = C (-ln 2 - psi(nu) + ln x) + sigma2 c x^nu dK_nu/dnu(x)
 * with c = 2^(1-nu)/Gamma(nu).  At r = 0: (1, 0, 0). */
void oracle_matern_grad(double r, const double *theta, double *d) {
  double s2 = theta[0], beta = theta[1], nu = theta[2];
  if (r == 0.0) {
    d[0] = 1.0;
    d[1] = 0.0;
    d[2] = 0.0;
    return;
  }
  double x = r / beta;
  double C = or_matern_scale(s2, nu, x, oracle_besselk_scaled(nu, x));
  d[0] = C / s2;
  d[1] = or_matern_scale(s2, nu, x, oracle_besselk_scaled(nu - 1.0, x)) * x / beta;
  double dk = oracle_besselk_dnu_scaled(nu, x);
  d[2] = C * (-OR_LN2 - oracle_digamma(nu) + log(x)) + or_matern_scale(s2, nu, x, dk);
}

static double or_dist(const double *x, const double *y, int64_t i, int64_t j) {
  double dx = x[i] - x[j], dy = y[i] - y[j];
  return sqrt(dx * dx + dy * dy);
}

static int or_theta_ok(const double *theta) {
  for (int k = 0; k < 3; ++k)
    if (!isfinite(theta[k]) || !(theta[k] > 0.0)) return 0;
  return 1;
}

/* Full n x n covariance, row-major, cov[i*n + j]. */
int oracle_matern_cov(int64_t n, const double *x, const double *y, const double *theta, double *cov) {
  if (n < 1 || !or_theta_ok(theta)) return OR_EINVAL;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) cov[i * n + j] = oracle_matern(or_dist(x, y, i, j), theta);
  return OR_OK;
}

/* Full n x n matrix of one theta-derivative of the covariance (comp 0: sigma2,
 * 1: beta, 2: nu), row-major, out[i*n + j]. */
int oracle_matern_dcov(int64_t n, const double *x, const double *y, const double *theta, int comp, double *out) {
  if (n < 1 || comp < 0 || comp > 2 || !or_theta_ok(theta)) return OR_EINVAL;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double d[3];
      oracle_matern_grad(or_dist(x, y, i, j), theta, d);
      out[i * n + j] = d[comp];
    }
  return OR_OK;
}

/* packed lower, row-major: element (i, j), j <= i, at i (i + 1) / 2 + j */
#define PK(i, j) ((size_t)(i) * ((size_t)(i) + 1) / 2 + (size_t)(j))

static void or_build_packed(int64_t n, const double *x, const double *y, const double *theta, double *A) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j <= i; ++j) A[PK(i, j)] = oracle_matern(or_dist(x, y, i, j), theta);
}

/* Unblocked left-looking Cholesky in place on packed lower storage.
 * Returns 0 or the 1-based column of the first non-positive pivot. */
static int64_t or_cholesky(int64_t n, double *A) {
  for (int64_t j = 0; j < n; ++j) {
    double *rj = A + PK(j, 0);
    double d = rj[j];
    for (int64_t k = 0; k < j; ++k) d -= rj[k] * rj[k];
    if (!(d > 0.0) || !isfinite(d)) return j + 1;
    double ljj = sqrt(d);
    rj[j] = ljj;
#pragma omp parallel for schedule(static)
    for (int64_t i = j + 1; i < n; ++i) {
      double *ri = A + PK(i, 0);
      double s = ri[j];
      for (int64_t k = 0; k < j; ++k) s -= ri[k] * rj[k];
      ri[j] = s / ljj;
    }
  }
  return 0;
}

/* y = L^-1 b, forward substitution */
static void or_forward(int64_t n, const double *L, const double *b, double *yv) {
  for (int64_t i = 0; i < n; ++i) {
    const double *ri = L + PK(i, 0);
    double s = b[i];
    for (int64_t k = 0; k < i; ++k) s -= ri[k] * yv[k];
    yv[i] = s / ri[i];
  }
}

/* a = L^-T y, backward substitution */
static void or_backward(int64_t n, const double *L, const double *yv, double *a) {
  for (int64_t i = n - 1; i >= 0; --i) {
    double s = yv[i];
    for (int64_t k = i + 1; k < n; ++k) s -= L[PK(k, i)] * a[k];
    a[i] = s / L[PK(i, i)];
  }
}

static int or_args_ok(int64_t n, const double *x, const double *y, const double *z, const double *theta) {
  if (n < 1 || !x || !y || !z || !theta || !or_theta_ok(theta)) return 0;
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(x[i]) || !isfinite(y[i]) || !isfinite(z[i])) return 0;
  return 1;
}

/* Cholesky factor (packed lower, row-major) of the Matern covariance. */
int oracle_cholesky(int64_t n, const double *x, const double *y, const double *theta, double *L, int64_t *info) {
  if (n < 1 || !or_theta_ok(theta)) return OR_EINVAL;
  or_build_packed(n, x, y, theta, L);
  int64_t inf = or_cholesky(n, L);
  if (info) *info = inf;
  return inf ? OR_ENOTPD : OR_OK;
}

/* z = L e with L the Cholesky factor of Sigma(theta): a draw of the field
 * at the given locations from standard normal draws e (paper, Example 1). */
int oracle_simulate(int64_t n, const double *x, const double *y, const double *theta, const double *e, double *z,
                    int64_t *info) {
  double *L = (double *)malloc(sizeof(double) * (size_t)PK(n, 0));
  if (!L) return OR_EINVAL;
  int st = oracle_cholesky(n, x, y, theta, L, info);
  if (st == OR_OK) {
    for (int64_t i = 0; i < n; ++i) {
      const double *ri = L + PK(i, 0);
      double s = 0.0;
      for (int64_t k = 0; k <= i; ++k) s += ri[k] * e[k];
      z[i] = s;
    }
  }
  free(L);
  return st;
}

/* l(theta), eq. (2) with mu = 0. Also returns log det Sigma and z^T Sigma^-1 z. */
int oracle_loglik(int64_t n, const double *x, const double *y, const double *z, const double *theta, double *loglik,
                  double *logdet_out, double *quad_out, int64_t *info) {
  if (info) *info = 0;
  if (!or_args_ok(n, x, y, z, theta)) return OR_EINVAL;
  double *L = (double *)malloc(sizeof(double) * (size_t)PK(n, 0));
  double *yv = (double *)malloc(sizeof(double) * (size_t)n);
  if (!L || !yv) {
    free(L);
    free(yv);
    return OR_EINVAL;
  }
  or_build_packed(n, x, y, theta, L);
  int64_t inf = or_cholesky(n, L);
  int st = OR_OK;
  if (inf) {
    if (info) *info = inf;
    if (loglik) *loglik = -INFINITY;
    st = OR_ENOTPD;
  } else {
    or_forward(n, L, z, yv);
    double logdet = 0.0, q = 0.0;
    for (int64_t i = 0; i < n; ++i) logdet += 2.0 * log(L[PK(i, i)]);
    for (int64_t i = 0; i < n; ++i) q += yv[i] * yv[i];
    if (loglik) *loglik = -0.5 * ((double)n * log(2.0 * OR_PI) + logdet + q);
    if (logdet_out) *logdet_out = logdet;
    if (quad_out) *quad_out = q;
  }
  free(L);
  free(yv);
  return st;
}

/* l(theta) and its gradient in (sigma2, beta, nu). */
int oracle_loglik_grad(int64_t n, const double *x, const double *y, const double *z, const double *theta,
                       double *loglik, double *grad, int64_t *info) {
  if (info) *info = 0;
  if (!or_args_ok(n, x, y, z, theta)) return OR_EINVAL;
  size_t np = (size_t)PK(n, 0);
  double *L = (double *)malloc(sizeof(double) * np);
  double *X = (double *)malloc(sizeof(double) * np); /* L^-1, packed lower row-major */
  double *yv = (double *)malloc(sizeof(double) * (size_t)n);
  double *a = (double *)malloc(sizeof(double) * (size_t)n);
  if (!L || !X || !yv || !a) {
    free(L);
    free(X);
    free(yv);
    free(a);
    return OR_EINVAL;
  }
  int st = OR_OK;
  or_build_packed(n, x, y, theta, L);
  int64_t inf = or_cholesky(n, L);
  if (inf) {
    if (info) *info = inf;
    if (loglik) *loglik = -INFINITY;
    st = OR_ENOTPD;
    goto done;
  }
  or_forward(n, L, z, yv);
  {
    double logdet = 0.0, q = 0.0;
    for (int64_t i = 0; i < n; ++i) logdet += 2.0 * log(L[PK(i, i)]);
    for (int64_t i = 0; i < n; ++i) q += yv[i] * yv[i];
    if (loglik) *loglik = -0.5 * ((double)n * log(2.0 * OR_PI) + logdet + q);
  }
  or_backward(n, L, yv, a);
  /* X = L^-1 by rows: X_ii = 1/L_ii and, for j < i,
   *   X_ij = -(sum_{k=j}^{i-1} L_ik X_kj) / L_ii   (k ascending). */
  memset(X, 0, sizeof(double) * np);
  for (int64_t i = 0; i < n; ++i) {
    const double *ri = L + PK(i, 0);
    double *xi = X + PK(i, 0);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < i; ++j) {
      double s = 0.0;
      for (int64_t k = j; k < i; ++k) s += ri[k] * X[PK(k, j)];
      xi[j] = -s / ri[i];
    }
    xi[i] = 1.0 / ri[i];
  }
  {
    /* W = X^T X, lower part: W_ij = sum_{k >= i} X_ki X_kj (k ascending),
     * then g_m = sum_{i,j} (a_i a_j / 2 - W_ij / 2) dSigma_m(i,j) with the
     * symmetric off-diagonal pairs counted twice. */
    double *rowsum = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *w = NULL;
#pragma omp parallel private(w)
    {
      w = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(dynamic, 4)
      for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j <= i; ++j) w[j] = 0.0;
        for (int64_t k = i; k < n; ++k) {
          const double *xk = X + PK(k, 0);
          double xki = xk[i];
          for (int64_t j = 0; j <= i; ++j) w[j] += xki * xk[j];
        }
        double r0 = 0.0, r1 = 0.0, r2 = 0.0;
        for (int64_t j = 0; j <= i; ++j) {
          double d[3];
          oracle_matern_grad(or_dist(x, y, i, j), theta, d);
          double f = (i == j ? 1.0 : 2.0) * (0.5 * a[i] * a[j] - 0.5 * w[j]);
          r0 += f * d[0];
          r1 += f * d[1];
          r2 += f * d[2];
        }
        rowsum[3 * i] = r0;
        rowsum[3 * i + 1] = r1;
        rowsum[3 * i + 2] = r2;
      }
      free(w);
    }
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      g0 += rowsum[3 * i];
      g1 += rowsum[3 * i + 1];
      g2 += rowsum[3 * i + 2];
    }
    free(rowsum);
    grad[0] = g0;
    grad[1] = g1;
    grad[2] = g2;
  }
done:
  free(L);
  free(X);
  free(yv);
  free(a);
  return st;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}
