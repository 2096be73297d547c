// Scalar parameter recurrences of the purification schemes, FP64, shared by host set-up
// code and the on-device schedule kernel of libsnf.  Expressions keep the paper's operation
// order and are compiled without floating-point contraction, so every implementation that
// evaluates the same expressions in IEEE FP64 takes the same decisions bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

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
