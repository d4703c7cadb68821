// Bounded maximisation of l(theta) over theta = (sigma2, beta, nu): the outer
// loop of the paper's estimator (Section 2.2 optimisation toolbox, bounds and
// start at the lower bound as in Section 3 Example 2).  Both methods work on
// u = log theta, which makes the three parameters comparable in scale.
#include <algorithm>
#include <cmath>
#include <limits>

#include "mle.h"

namespace exg {

namespace {

constexpr int D = 3;

struct Box {
  double lo[D], hi[D];
  void clamp(double* u) const {
    for (int k = 0; k < D; ++k) u[k] = std::min(hi[k], std::max(lo[k], u[k]));
  }
};

Box log_box(const double lb[3], const double ub[3]) {
  Box b;
  for (int k = 0; k < D; ++k) {
    b.lo[k] = std::log(lb[k]);
    b.hi[k] = std::log(ub[k]);
  }
  return b;
}

void to_theta(const double* u, const double lb[3], const double ub[3], double* th) {
  for (int k = 0; k < D; ++k) th[k] = std::min(ub[k], std::max(lb[k], std::exp(u[k])));
}

}  // namespace

// ------------------------------------------------------------- Nelder-Mead
MleResult maximize_dfo(const Objective& obj, const double lb[3], const double ub[3], const double theta0[3],
                       double tol, int max_evals) {
  const Box box = log_box(lb, ub);
  MleResult res{};
  res.f = -std::numeric_limits<double>::infinity();
  int64_t nev = 0;
  bool hard = false;
  auto F = [&](const double* u) {  // value to minimise: -l
    double th[3], f = -INFINITY, g[3];
    to_theta(u, lb, ub, th);
    ++nev;
    if (!obj(th, false, &f, g)) hard = true;
    const double v = std::isfinite(f) ? -f : std::numeric_limits<double>::infinity();
    if (-v > res.f) {
      res.f = -v;
      for (int k = 0; k < D; ++k) res.theta[k] = th[k];
    }
    return v;
  };
  auto budget_left = [&]() { return max_evals <= 0 || nev < max_evals; };

  const double alpha = 1.0, gamma = 2.0, rho = 0.5, sigma = 0.5;
  int64_t it = 0;
  bool conv = false;
  double start[D];
  for (int k = 0; k < D; ++k) start[k] = std::log(theta0[k]);
  box.clamp(start);
  for (int k = 0; k < D; ++k) res.theta[k] = theta0[k];
  // A simplex can collapse onto a flat face of l (e.g. beta so small that
  // Sigma ~ sigma2 I); each converged run is therefore restarted from its best
  // vertex with a fresh simplex of half the previous size, until a restart
  // improves l by less than tol.
  double frac = 0.25;
  double prev_best = std::numeric_limits<double>::infinity();
  for (int restart = 0; restart < 12 && !hard && budget_left(); ++restart, frac *= 0.5) {
    double S[D + 1][D], fv[D + 1];
    for (int k = 0; k < D; ++k) S[0][k] = start[k];
    fv[0] = F(S[0]);
    for (int v = 1; v <= D; ++v) {
      for (int k = 0; k < D; ++k) S[v][k] = S[0][k];
      const int k = v - 1;
      double step = frac * (box.hi[k] - box.lo[k]);
      if (S[0][k] + step > box.hi[k]) step = -step;  // step into the box
      S[v][k] += step;
      box.clamp(S[v]);
      fv[v] = budget_left() ? F(S[v]) : std::numeric_limits<double>::infinity();
    }
    bool run_conv = false;
    while (!hard && budget_left()) {
      // order vertices by value (best first)
      int idx[D + 1] = {0, 1, 2, 3};
      std::sort(idx, idx + D + 1, [&](int a, int b) { return fv[a] < fv[b]; });
      double So[D + 1][D], fo[D + 1];
      for (int v = 0; v <= D; ++v) {
        fo[v] = fv[idx[v]];
        for (int k = 0; k < D; ++k) So[v][k] = S[idx[v]][k];
      }
      for (int v = 0; v <= D; ++v) {
        fv[v] = fo[v];
        for (int k = 0; k < D; ++k) S[v][k] = So[v][k];
      }
      ++it;
      if (std::isfinite(fv[D]) && std::fabs(fv[D] - fv[0]) < tol) {
        run_conv = true;
        break;
      }
      double cen[D] = {0, 0, 0};
      for (int v = 0; v < D; ++v)
        for (int k = 0; k < D; ++k) cen[k] += S[v][k] / D;
      double xr[D];
      for (int k = 0; k < D; ++k) xr[k] = cen[k] + alpha * (cen[k] - S[D][k]);
      box.clamp(xr);
      const double fr = F(xr);
      if (fr < fv[0]) {
        double xe[D];
        for (int k = 0; k < D; ++k) xe[k] = cen[k] + gamma * (xr[k] - cen[k]);
        box.clamp(xe);
        const double fe = budget_left() ? F(xe) : std::numeric_limits<double>::infinity();
        if (fe < fr) {
          for (int k = 0; k < D; ++k) S[D][k] = xe[k];
          fv[D] = fe;
        } else {
          for (int k = 0; k < D; ++k) S[D][k] = xr[k];
          fv[D] = fr;
        }
        continue;
      }
      if (fr < fv[D - 1]) {
        for (int k = 0; k < D; ++k) S[D][k] = xr[k];
        fv[D] = fr;
        continue;
      }
      // contraction: outside if the reflected point beats the worst, else inside
      double xc[D];
      const bool outside = fr < fv[D];
      for (int k = 0; k < D; ++k)
        xc[k] = outside ? cen[k] + rho * (xr[k] - cen[k]) : cen[k] + rho * (S[D][k] - cen[k]);
      box.clamp(xc);
      if (!budget_left()) break;
      const double fc = F(xc);
      if (fc < (outside ? fr : fv[D])) {
        for (int k = 0; k < D; ++k) S[D][k] = xc[k];
        fv[D] = fc;
        continue;
      }
      // shrink towards the best vertex
      for (int v = 1; v <= D && budget_left(); ++v) {
        for (int k = 0; k < D; ++k) S[v][k] = S[0][k] + sigma * (S[v][k] - S[0][k]);
        fv[v] = F(S[v]);
      }
    }
    if (!run_conv) break;  // budget or hard failure
    const double best = -res.f;
    if (prev_best - best < tol) {
      conv = true;
      break;
    }
    prev_best = best;
    for (int k = 0; k < D; ++k) start[k] = std::log(res.theta[k]);
    box.clamp(start);
  }
  res.iters = it;
  res.evals = nev;
  res.converged = conv;
  return res;
}

// ------------------------------------------------------- projected L-BFGS
MleResult maximize_lbfgsb(const Objective& obj, const double lb[3], const double ub[3], const double theta0[3],
                          double tol, int max_evals, double rtol, int patience, Curvature* curv) {
  const Box box = log_box(lb, ub);
  MleResult res{};
  res.f = -std::numeric_limits<double>::infinity();
  int64_t nev = 0;
  bool hard = false;
  // F(u) = -l(exp u), gradient dF/du_k = -theta_k dl/dtheta_k
  auto FG = [&](const double* u, double* gu) {
    double th[3], f = -INFINITY, g[3] = {0, 0, 0};
    to_theta(u, lb, ub, th);
    ++nev;
    if (!obj(th, true, &f, g)) hard = true;
    if (!std::isfinite(f)) return std::numeric_limits<double>::infinity();
    for (int k = 0; k < D; ++k) gu[k] = -th[k] * g[k];
    if (f > res.f) {
      res.f = f;
      for (int k = 0; k < D; ++k) res.theta[k] = th[k];
    }
    return -f;
  };
  auto budget_left = [&]() { return max_evals <= 0 || nev < max_evals; };
  constexpr int M = Curvature::M;
  double sm[M][D], ym[M][D], rhom[M];
  int mcount = 0, mhead = 0;
  if (curv && curv->count > 0) {
    for (int i = 0; i < M; ++i) {
      for (int k = 0; k < D; ++k) {
        sm[i][k] = curv->s[i][k];
        ym[i][k] = curv->y[i][k];
      }
      rhom[i] = curv->rho[i];
    }
    mcount = std::min(curv->count, M);
    mhead = curv->head % M;
  }

  double u[D], g[D];
  for (int k = 0; k < D; ++k) u[k] = std::log(theta0[k]);
  box.clamp(u);
  for (int k = 0; k < D; ++k) res.theta[k] = theta0[k];
  double f = FG(u, g);
  if (!std::isfinite(f)) {
    // infeasible start: move towards the box centre until a point evaluates
    for (int t = 0; t < 30 && !std::isfinite(f) && budget_left() && !hard; ++t) {
      for (int k = 0; k < D; ++k) u[k] = 0.5 * (u[k] + 0.5 * (box.lo[k] + box.hi[k]));
      f = FG(u, g);
    }
  }
  int64_t it = 0;
  int small = 0;  // consecutive accepted steps below the tolerance
  bool conv = false;
  while (std::isfinite(f) && !hard && budget_left()) {
    ++it;
    // free variables: not at a bound with the gradient pushing outward
    bool freev[D];
    for (int k = 0; k < D; ++k) {
      const bool at_lo = u[k] <= box.lo[k] && g[k] > 0;
      const bool at_hi = u[k] >= box.hi[k] && g[k] < 0;
      freev[k] = !(at_lo || at_hi) && box.hi[k] > box.lo[k];
    }
    double pg = 0.0;
    for (int k = 0; k < D; ++k)
      if (freev[k]) pg = std::max(pg, std::fabs(g[k]));
    if (pg < 1e-12 * std::max(1.0, std::fabs(f))) {
      conv = true;
      break;
    }
    // two-loop recursion on the free subspace
    double q[D], d[D], al[M];
    for (int k = 0; k < D; ++k) q[k] = freev[k] ? g[k] : 0.0;
    for (int i = 0; i < mcount; ++i) {
      const int j = (mhead - 1 - i + M) % M;
      double sq = 0.0;
      for (int k = 0; k < D; ++k) sq += freev[k] ? sm[j][k] * q[k] : 0.0;
      al[i] = rhom[j] * sq;
      for (int k = 0; k < D; ++k)
        if (freev[k]) q[k] -= al[i] * ym[j][k];
    }
    double gam = 1.0;
    if (mcount > 0) {
      const int j = (mhead - 1 + M) % M;
      double sy = 0.0, yy = 0.0;
      for (int k = 0; k < D; ++k) {
        sy += sm[j][k] * ym[j][k];
        yy += ym[j][k] * ym[j][k];
      }
      if (yy > 0) gam = sy / yy;
    } else {
      // first step: at most 0.5 in log space along the steepest descent
      const double gn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
      gam = gn > 0 ? std::min(1.0, 0.5 / gn) : 1.0;
    }
    for (int k = 0; k < D; ++k) q[k] *= gam;
    for (int i = mcount - 1; i >= 0; --i) {
      const int j = (mhead - 1 - i + M) % M;
      double yq = 0.0;
      for (int k = 0; k < D; ++k) yq += freev[k] ? ym[j][k] * q[k] : 0.0;
      const double be = rhom[j] * yq;
      for (int k = 0; k < D; ++k)
        if (freev[k]) q[k] += sm[j][k] * (al[i] - be);
    }
    double gd = 0.0;
    for (int k = 0; k < D; ++k) {
      d[k] = freev[k] ? -q[k] : 0.0;
      gd += g[k] * d[k];
    }
    if (!(gd < 0.0)) {  // not a descent direction: restart from steepest descent
      mcount = 0;
      double gn = 0.0;
      for (int k = 0; k < D; ++k) gn += freev[k] ? g[k] * g[k] : 0.0;
      gn = std::sqrt(gn);
      for (int k = 0; k < D; ++k) d[k] = freev[k] ? -g[k] * std::min(1.0, 0.5 / gn) : 0.0;
    }
    // projected backtracking line search
    double a = 1.0, un[D], gn[D], fn = std::numeric_limits<double>::infinity();
    bool accepted = false;
    for (int ls = 0; ls < 30 && budget_left() && !hard; ++ls, a *= 0.5) {
      for (int k = 0; k < D; ++k) un[k] = u[k] + a * d[k];
      box.clamp(un);
      double dec = 0.0;
      for (int k = 0; k < D; ++k) dec += g[k] * (un[k] - u[k]);
      if (dec == 0.0) break;
      fn = FG(un, gn);
      if (std::isfinite(fn) && fn <= f + 1e-4 * dec) {
        accepted = true;
        break;
      }
    }
    if (!accepted) {
      // the search stopped for lack of evaluations or at a hard failure:
      // not converged
      if (!budget_left() || hard) break;
      if (mcount > 0) {
        mcount = 0;  // retry once from steepest descent
        continue;
      }
      conv = true;  // no decrease possible along the projected gradient
      break;
    }
    double s[D], y[D], sy = 0.0;
    for (int k = 0; k < D; ++k) {
      s[k] = un[k] - u[k];
      y[k] = gn[k] - g[k];
      sy += s[k] * y[k];
    }
    if (sy > 1e-12) {
      for (int k = 0; k < D; ++k) {
        sm[mhead][k] = s[k];
        ym[mhead][k] = y[k];
      }
      rhom[mhead] = 1.0 / sy;
      mhead = (mhead + 1) % M;
      mcount = std::min(mcount + 1, M);
    }
    const double df = f - fn;
    for (int k = 0; k < D; ++k) {
      u[k] = un[k];
      g[k] = gn[k];
    }
    f = fn;
    small = df < tol + rtol * std::fabs(f) ? small + 1 : 0;
    if (small >= patience) {
      conv = true;
      break;
    }
  }
  if (curv) {
    for (int i = 0; i < M; ++i) {
      for (int k = 0; k < D; ++k) {
        curv->s[i][k] = sm[i][k];
        curv->y[i][k] = ym[i][k];
      }
      curv->rho[i] = rhom[i];
    }
    curv->count = mcount;
    curv->head = mhead;
  }
  res.iters = it;
  res.evals = nev;
  res.converged = conv;
  return res;
}

}  // namespace exg
