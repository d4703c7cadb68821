// Bounded maximisers of l(theta) used by exageo_mle (host code).
#pragma once
#include <stdint.h>

#include <functional>

namespace exg {

// Evaluates l at theta (and its gradient when want_grad).  Returns false on a
// hard failure; a non-positive-definite point returns true with f = -inf.
using Objective = std::function<bool(const double theta[3], bool want_grad, double* f, double grad[3])>;

struct MleResult {
  double theta[3];
  double f;
  int64_t iters;
  int64_t evals;
  bool converged;
};

// Nelder-Mead simplex search (Nelder & Mead, Computer Journal 7, 1965) on
// u = log theta, with every trial point clamped into [log lb, log ub].
// Stops when the spread of l over the simplex is below tol, or after
// max_evals evaluations (0 = no limit).
MleResult maximize_dfo(const Objective& f, const double lb[3], const double ub[3], const double theta0[3], double tol,
                       int max_evals);

// The curvature pairs (s, y) of the quasi-Newton model, in u = log theta.
// maximize_lbfgsb starts from the pairs in `curv` when it is given and holds
// any, and leaves its own pairs there on return, so that a second search
// (e.g. an FP64 finish after a mixed-precision search) continues with the
// model the first one built instead of a steepest-descent restart.
struct Curvature {
  static constexpr int M = 6;
  double s[M][3], y[M][3], rho[M];
  int count = 0, head = 0;
};


// Projected limited-memory BFGS on u = log theta within [log lb, log ub]:
// variables at a bound whose gradient points outward are held fixed, the
// two-loop recursion (Nocedal, Math. Comp. 35, 1980) gives the step on the free
// ones, and a projected backtracking (Armijo) line search keeps the iterate in
// the box (after the bounded L-BFGS of Byrd, Lu, Nocedal & Zhu, SIAM J. Sci.
// Comput. 16, 1995, without its generalised Cauchy point).  Stops when
// successive accepted l differ by less than tol + rtol |l| (patience times in a
// row), or after max_evals.
MleResult maximize_lbfgsb(const Objective& f, const double lb[3], const double ub[3], const double theta0[3],
                          double tol, int max_evals, double rtol = 0.0, int patience = 1, Curvature* curv = nullptr);

}  // namespace exg
