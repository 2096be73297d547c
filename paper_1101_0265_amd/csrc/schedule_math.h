// Scalar parameter recurrences of the purification schemes, FP64, shared by host set-up
// code and the on-device schedule kernel of libsnf.  Expressions keep the paper's operation
// order and are compiled without floating-point contraction, so every implementation that
// evaluates the same expressions in IEEE FP64 takes the same decisions bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace snf {
namespace sched {

// ---- Algorithm 1 (McWeeny-based fixed-mu purification) ---------------------------------

// gamma = 2 max(lambda_max - mu, mu - lambda_min)
__host__ __device__ inline double alg1_gamma(double lmin, double lmax, double mu) {
#pragma clang fp contract(off)
  const double a = lmax - mu, b = mu - lmin;
  return 2.0 * (b > a ? b : a);
}

// beta = 0.5 (1 - xi / gamma): X-space image of the level nearest mu
__host__ __device__ inline double alg1_beta0(double xi, double gamma) {
#pragma clang fp contract(off)
  return 0.5 * (1.0 - xi / gamma);
}

// alpha = 3 / sqrt(12 beta^2 - 18 beta + 9), the root alpha >= 1 of Eq. 3 for m = 1
__host__ __device__ inline double alg1_alpha(double beta) {
#pragma clang fp contract(off)
  return 3.0 / sqrt(12.0 * beta * beta - 18.0 * beta + 9.0);
}

// beta_s = alpha (beta - 0.5) + 0.5;  beta <- 3 beta_s^2 - 2 beta_s^3
__host__ __device__ inline double alg1_beta_next(double beta, double alpha) {
#pragma clang fp contract(off)
  const double bs = alpha * (beta - 0.5) + 0.5;
  return 3.0 * bs * bs - 2.0 * bs * bs * bs;
}

// ---- P_{m,m}, m odd: the higher-order fixed-mu schemes (Eqs. 2 and 3) ------------------
//
// P_{m,m} is point-symmetric about (1/2, 1/2) and P'(x) = c_m x^m (1 - x)^m with
// c_m = (2m+1)! / (m!)^2.  With x = 1/2 + v, P'(x) = c_m (1/4 - v^2)^m; integrating term by
// term from v = 0 gives P(1/2 + v) = 1/2 + v r(v^2) with
//   r_k = c_m C(m, k) (-1)^k 4^(k-m) / (2k + 1),   k = 0..m.
// For m = 1, 3, 5 each c_m C(m, k) is divisible by 2k + 1, so every r_k is an integer times a
// power of two: exact in FP64.
constexpr int kPmmMaxM = 5;

__host__ __device__ inline double pmm_r(int m, int k) {
  int64_t fact = 1;
  for (int t = 2; t <= 2 * m + 1; ++t) fact *= t;
  int64_t fm = 1;
  for (int t = 2; t <= m; ++t) fm *= t;
  const int64_t cm = fact / (fm * fm);
  int64_t binom = 1;
  for (int t = 0; t < k; ++t) binom = binom * (m - t) / (t + 1);
  const int64_t q = cm * binom / (2 * k + 1);
  double p4 = 1.0;
  for (int t = k; t < m; ++t) p4 *= 0.25;
  return (double)((k & 1) ? -q : q) * p4;
}

// r_0..r_m of pmm_r into r[] (the coefficients of the matrix evaluation)
__host__ __device__ inline void pmm_coeffs(int m, double* r) {
  for (int k = 0; k <= m; ++k) r[k] = pmm_r(m, k);
}

// ---- P_{i,j}, i and j odd: scale-and-fold about the unstable fixed point x* -------------
//
// X_0 = (mu I - F) / gamma + x* I puts mu on x*; the unoccupied part of the spectrum then
// lies in [0, a], the occupied part in [1 - a', 1].  f_i(X) = P(alpha (X - x* I) + x* I).
// Each side has its own form of Eq. 3 (the folded image of its interval end equals the image
// of its gap edge; that alpha minimises the side's new bound), and alpha is the smaller of
// the two.  The occupied side is the unoccupied side of the mirrored polynomial:
// 1 - P_{i,j}(1 - y) = P_{j,i}(y), whose fixed point is 1 - x*.
constexpr int kPijMax = 5;                 // i, j in {1, 3, 5}
constexpr int kPijQ = 2 * kPijMax + 1;     // coefficients of Q, degree i + j

// P_{i,j}(x) = x^(i+1) sum_{k=0..j} C(i+k, k) (1-x)^k, Horner's rule in y = 1 - x; accurate
// relative to its value near 0 and for x < 0 (every term positive there).
__host__ __device__ inline double pij_eval(int i, int j, double x) {
#pragma clang fp contract(off)
  const double y = 1.0 - x;
  double acc = 0.0;
  for (int k = j; k >= 0; --k) {
    int64_t c = 1;                           // C(i+k, k)
    for (int t = 1; t <= k; ++t) c = c * (i + t) / t;
    acc = acc * y + (double)c;
  }
  double xp = x;
  for (int t = 0; t < i; ++t) xp = xp * x;
  return xp * acc;
}

// The root of P(x) = x inside (0, 1): P(x) - x is negative above 0 and positive below 1 and
// P is S-shaped, so the root is unique; bisection until the bracket stops shrinking.
__host__ __device__ inline double pij_xstar(int i, int j) {
#pragma clang fp contract(off)
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 1100; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    const double g = pij_eval(i, j, mid) - mid;
    if (g == 0.0) return mid;
    if (g < 0.0) lo = mid; else hi = mid;
  }
  return lo;
}

// gamma = max((mu - lambda_min) / (1 - x*), (lambda_max - mu) / x*): the spectrum of X_0
// fills [0, 1]
__host__ __device__ inline double pij_gamma(double lmin, double lmax, double mu, double xs) {
#pragma clang fp contract(off)
  const double a = (mu - lmin) / (1.0 - xs), b = (lmax - mu) / xs;
  return a > b ? a : b;
}

// Q(v) = (P(x* + v) - x*) / v = sum_k q_k v^k, k = 0..i+j, from P' = C x^i (1-x)^j with
// C = (i+j+1)! / (i! j!): q_k = P^(k+1)(x*) / (k+1)! = C / (k+1) [v^k] (x*+v)^i (1-x*-v)^j.
__host__ __device__ inline void pij_taylor(int i, int j, double xs, double* q) {
#pragma clang fp contract(off)
  double cc = 1.0;                           // C = (i+j+1)! / (i! j!) = (i+j+1) C(i+j, i)
  for (int t = 1; t <= i; ++t) cc = cc * (double)(j + t) / (double)t;
  cc = cc * (double)(i + j + 1);
  const double xm = 1.0 - xs;
  for (int k = 0; k <= i + j; ++k) {
    double sum = 0.0;
    for (int l = 0; l <= i && l <= k; ++l) {
      const int r = k - l;
      if (r > j) continue;
      double bi = 1.0, bj = 1.0;
      for (int t = 0; t < l; ++t) bi = bi * (double)(i - t) / (double)(t + 1);
      for (int t = 0; t < r; ++t) bj = bj * (double)(j - t) / (double)(t + 1);
      double term = bi * bj;
      for (int t = 0; t < i - l; ++t) term = term * xs;
      for (int t = 0; t < j - r; ++t) term = term * xm;
      sum = (r & 1) ? sum - term : sum + term;
    }
    q[k] = cc / (double)(k + 1) * sum;
  }
}

// ---- table-driven forms for the on-device schedule ----------------------------------------
// The binomial coefficients C(i+k, k) come from a table filled once at set-up (exact integers
// in FP64), so the schedule kernel does not rebuild them with integer divisions at every
// evaluation; the arithmetic is that of pij_eval.
__host__ __device__ inline void pij_binoms(int i, int j, double* bin) {
  for (int k = 0; k <= j; ++k) {
    int64_t c = 1;                           // C(i+k, k)
    for (int t = 1; t <= k; ++t) c = c * (i + t) / t;
    bin[k] = (double)c;
  }
}

// P_{i,j}(x) = x^(i+1) sum_{k=0..j} bin[k] (1-x)^k, bin[k] = C(i+k, k): the incomplete-beta
// form, accurate relative to its value near x = 0 and for x < 0, where the scalar schedule
// evaluates it (the centred form 1/2 + v r(v^2) of P_{m,m} cancels there).
__host__ __device__ inline double pij_eval_tab(int i, int j, const double* bin, double x) {
#pragma clang fp contract(off)
  const double y = 1.0 - x;
  double acc = 0.0;
  for (int k = j; k >= 0; --k) acc = acc * y + bin[k];
  double xp = x;
  for (int t = 0; t < i; ++t) xp = xp * x;
  return xp * acc;
}

// The root alpha >= 1 of Eq. 3, P(alpha (beta - 1/2) + 1/2) = P((1 - alpha) / 2), for
// P = P_{m,m} and 0 < beta < 1/2 (bin: C(m+k, k)): G(alpha) = P((1 - alpha) / 2) -
// P(alpha (beta - 1/2) + 1/2) is -P(beta) < 0 at alpha = 1 and positive at
// alpha = 1 / (1 - 2 beta) (the scaled gap edge reaches 0); P falls on x < 0 and rises on
// [0, 1], so G increases in between and bisection (until the bracket of doubles stops
// shrinking) converges to the unique root.  Outside (0, 1/2), alpha = 1.
__host__ __device__ inline double pmm_alpha_tab(int m, const double* bin, double beta) {
#pragma clang fp contract(off)
  if (!(beta > 0.0 && beta < 0.5)) return 1.0;
  double lo = 1.0, hi = 1.0 / (1.0 - 2.0 * beta);
  for (int it = 0; it < 2200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    const double g = pij_eval_tab(m, m, bin, 0.5 * (1.0 - mid)) -
                     pij_eval_tab(m, m, bin, mid * (beta - 0.5) + 0.5);
    if (g < 0.0) lo = mid; else hi = mid;
  }
  return lo;
}

// One side's Eq. 3 for P = P_{i,j} (bin: C(i+k, k)): the root alpha >= 1 of
// P(x* (1 - alpha)) = P(x* - alpha (x* - a)), for 0 < a < x*.  The difference is -P(a) < 0
// at alpha = 1 and positive where the scaled edge reaches 0 (alpha = x* / (x* - a)); P falls
// on x < 0 and rises on [0, x*], so bisection converges to the unique root.  Outside (0, x*):
// 1.  The occupied side is this with (j, i), 1 - x* and a-bar.
__host__ __device__ inline double pij_alpha_side_tab(int i, int j, const double* bin, double xs,
                                                     double a) {
#pragma clang fp contract(off)
  if (!(a > 0.0 && a < xs)) return 1.0;
  double lo = 1.0, hi = xs / (xs - a);
  for (int it = 0; it < 2200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    const double g = pij_eval_tab(i, j, bin, xs * (1.0 - mid)) -
                     pij_eval_tab(i, j, bin, xs - mid * (xs - a));
    if (g < 0.0) lo = mid; else hi = mid;
  }
  return lo;
}

// New bound of one side: the larger image of its interval end and of its gap edge.
__host__ __device__ inline double pij_side_next_tab(int i, int j, const double* bin, double xs,
                                                    double a, double alpha) {
#pragma clang fp contract(off)
  const double u = pij_eval_tab(i, j, bin, xs * (1.0 - alpha));
  const double v = pij_eval_tab(i, j, bin, xs - alpha * (xs - a));
  return u > v ? u : v;
}

// ---- Algorithm 2 (P_{0,1} & P_{1,0} varying-mu purification) ---------------------------

// f0(lambda) = (lambda_max - lambda) / (lambda_max - lambda_min)
__host__ __device__ inline double alg2_f0(double lam, double lmin, double lmax) {
#pragma clang fp contract(off)
  return (lmax - lam) / (lmax - lmin);
}

__host__ __device__ inline bool alg2_square(double beta, double betabar) {
#pragma clang fp contract(off)
  return beta + betabar > 1.0;
}

__host__ __device__ inline double alg2_square_alpha(double beta) {
#pragma clang fp contract(off)
  return beta / (2.0 - beta);
}

// ((1 + alpha) x - alpha)^2
__host__ __device__ inline double alg2_square_map(double x, double alpha) {
#pragma clang fp contract(off)
  const double y = (1.0 + alpha) * x - alpha;
  return y * y;
}

__host__ __device__ inline double alg2_fold_alpha(double betabar) {
#pragma clang fp contract(off)
  return (1.0 - betabar) / (1.0 + betabar);
}

// 2 (1 + alpha) x - (1 + alpha)^2 x^2
__host__ __device__ inline double alg2_fold_map(double x, double alpha) {
#pragma clang fp contract(off)
  return 2.0 * (1.0 + alpha) * x - (1.0 + alpha) * (1.0 + alpha) * x * x;
}

// ---- trace-based choice of the unscaled trace-correcting scheme --------------------------

// square iff |tr(X^2) - N| < |2 tr X - tr(X^2) - N|; a tie folds
__host__ __device__ inline bool trace_square(double t1, double t2, double nocc) {
#pragma clang fp contract(off)
  return fabs(t2 - nocc) < fabs(2.0 * t1 - t2 - nocc);
}

}  // namespace sched
}  // namespace snf
