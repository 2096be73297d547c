/*
 * snf.h -- C ABI of the scale-and-fold density-matrix purification library for MI355X.
 *
 * The library computes the density matrix D = theta(mu I - F) of a symmetric effective
 * Hamiltonian F (the problem statement in the introduction of Rubensson,
 * arXiv:1101.0265) by recursive purification, Eq. 1:
 *     X_0 = f_0(F),   X_i = f_i(X_{i-1}),  i = 1, 2, ...
 * where f_0 is linear and every f_i costs one matrix-matrix product X.X (two for
 * Algorithm 1, m + 1 for the P_{m,m} schemes, (i + j)/2 + 1 for P_{i,j}).  Eleven schemes
 * are offered:
 *
 *   SNF_SP2_TRACE   second-order trace-correcting purification, x^2 / 2x - x^2 chosen from
 *                   the trace of X (the unscaled scheme the paper compares against).
 *   SNF_TC2_BETA    Algorithm 2 with alpha = 0: same polynomials, chosen from the images
 *                   beta / beta-bar of the gap edges.
 *   SNF_SNF_VARMU   Algorithm 2: varying-mu scale-and-fold, Eqs. 4 and 5.
 *   SNF_MCWEENY     Algorithm 1 with alpha = 1: regular grand-canonical McWeeny.
 *   SNF_SNF_FIXMU   Algorithm 1: McWeeny-based fixed-mu scale-and-fold, Eqs. 2 and 3.
 *   SNF_SNF_FIXMU3  fixed-mu scale-and-fold with P_{3,3} (Eq. 2 for m = 3): alpha >= 1 is
 *                   the root of Eq. 3, found on the device by bisection; 4 products per f_i.
 *   SNF_SNF_FIXMU5  the same with P_{5,5}; 6 products per f_i.
 *   SNF_PMM3        SNF_SNF_FIXMU3 with alpha = 1 (unscaled grand-canonical P_{3,3}).
 *   SNF_PMM5        SNF_SNF_FIXMU5 with alpha = 1.
 *   The P_{m,m} schemes evaluate P_{m,m}(1/2 + v) = 1/2 + v r(v^2) (the polynomial is
 *   point-symmetric about (1/2, 1/2); r has degree m): v^2, r by Horner's rule, then v r.
 *   They take the inputs of Algorithm 1; the dense entry points run them in SNF_P_FP64
 *   only (the block-sparse path computes every scheme in FP32).
 *   SNF_SNF_FIXMU_PIJ  fixed-mu scale-and-fold with P_{i,j}, i and j odd (poly_i, poly_j in
 *                   snf_params, each 1, 3 or 5), scaled about the polynomial's unstable
 *                   fixed point x* (the remark closing the P_{m,m} paragraph before
 *                   Algorithm 1; x* != 1/2 when i != j):
 *                     X_0 = (mu I - F) / gamma + x* I,
 *                     gamma = max((mu - lambda_min) / (1 - x*), (lambda_max - mu) / x*),
 *                     f_i(X) = P_{i,j}(alpha (X - x* I) + x* I).
 *                   The unoccupied part of the spectrum lies in [0, a], the occupied part
 *                   in [1 - a', 1]; each side has its own Eq. 3 (the folded image of its
 *                   interval end equals the image of its gap edge), and alpha is the
 *                   smaller root: the largest scaling that speeds up both sides.  For
 *                   i = j this is SNF_SNF_FIXMU / SNF_SNF_FIXMU3 / SNF_SNF_FIXMU5.
 *                   Evaluation: P(x* + v) = x* + v Q(v), Q by Horner's rule in v^2 with
 *                   coefficients linear in v.  Inputs of Algorithm 1; SNF_P_FP64 only on
 *                   the dense entry points;
 *                   SNF_EINVAL for poly_i / poly_j outside {1, 3, 5} or a gap edge that
 *                   falls outside [0, 1] (xi / (2 gamma) >= min(x*, 1 - x*)).
 *   SNF_PIJ         SNF_SNF_FIXMU_PIJ with alpha = 1 (unscaled grand-canonical P_{i,j}).
 *
 * Conventions shared by every entry point:
 *  - Matrices are row-major FP64.  Only the upper triangle of F (j >= i) is read; the
 *    lower triangle is taken as its mirror, so F is symmetric by construction.
 *  - Device pointers are HIP device allocations on the current device (torch tensors on
 *    cuda:N are fine).  The library never frees or retains caller memory.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  All work is enqueued
 *    on it; calls that return results return after that work has completed.
 *  - The library owns a per-device workspace (padded copies of X, partial sums, the
 *    scalar state).  It grows on demand and is reused; calls that overlap in time on the
 *    same device from different host threads are serialised by an internal lock.
 *  - Return value: one of the SNF_* status codes below.  Negative = error, the outputs are
 *    then unspecified (except snf_result.status); snf_strerror() gives a message, and for
 *    SNF_EDEVICE the text of the last HIP error.
 */
#ifndef SNF_H
#define SNF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------------------------- */
#define SNF_OK          0   /* converged: ||X^2 - X||_F <= tol                                */
#define SNF_PENDING     1   /* serving: request not finished yet                              */
#define SNF_OK_FLOOR    2   /* stopped on stagnation above tol (precision/truncation floor)  */
#define SNF_EINVAL     -1   /* bad argument: null pointer, n <= 0, inconsistent bounds ...    */
#define SNF_ENOMEM     -2   /* device allocation failed / over the memory budget             */
#define SNF_ENOCONV    -3   /* max_iter iterations without reaching tol                       */
#define SNF_ENONFINITE -4   /* a non-finite value appeared in X (bad input or bounds)         */
#define SNF_EMIXED     -5   /* converged, but |tr D - n_occ| >= 0.5: states were mixed        */
#define SNF_EDEVICE    -6   /* a HIP runtime call failed                                      */
#define SNF_ESIZE      -7   /* snf_purify_dense_noalloc: order above SNF_NOALLOC_MAX_N         */

/* ---- schemes and precision modes ------------------------------------------------------- */
typedef enum {
  SNF_SP2_TRACE = 0,
  SNF_TC2_BETA = 1,
  SNF_SNF_VARMU = 2,
  SNF_MCWEENY = 3,
  SNF_SNF_FIXMU = 4,
  SNF_SNF_FIXMU3 = 5,
  SNF_SNF_FIXMU5 = 6,
  SNF_PMM3 = 7,
  SNF_PMM5 = 8,
  SNF_SNF_FIXMU_PIJ = 9,
  SNF_PIJ = 10
} snf_scheme;

typedef enum {
  SNF_P_FP64 = 0,        /* every product in FP64 (MFMA f64)                                   */
  SNF_P_FP32 = 1,        /* FP32 products (MFMA f32) after the FP64 phase, no refinement      */
  SNF_P_FP32_REF64 = 2,  /* FP64 phase, FP32 products, then FP64 refinement to tol             */
  SNF_P_BF16_REF64 = 3   /* FP64 phase, BF16-input/FP32-accumulate products, FP64 refinement  */
} snf_precision;

/* Branch letters recorded per iteration. */
#define SNF_BRANCH_SQUARE 0   /* P_{1,0}: X <- ((1+a) X - a I)^2           (Eq. 4)          */
#define SNF_BRANCH_FOLD   1   /* P_{0,1}: X <- 2 (1+a) X - (1+a)^2 X^2      (Eq. 5)          */
#define SNF_BRANCH_P11    2   /* P_{1,1}: X <- 3 Xs^2 - 2 Xs^3, Xs = a (X - I/2) + I/2 (Eq. 2) */
#define SNF_BRANCH_P33    3   /* P_{3,3}(Xs)                                                 */
#define SNF_BRANCH_P55    4   /* P_{5,5}(Xs)                                                 */
#define SNF_BRANCH_PIJ    5   /* P_{i,j}(a (X - x* I) + x* I)                                */

/* Flags (snf_params.flags). */
#define SNF_FLAG_TIME_PRODUCTS 1  /* bracket every product kernel with HIP events and report
                                     their summed duration in snf_result.product_ms         */
#define SNF_FLAG_TRUNC_ERROR_CONTROL 2  /* snf_purify_bsr: trunc_tau is an error budget for
                                     ||D - D_exact||_F, not a per-block threshold (below)   */
#define SNF_FLAG_SUBSPACE_NEWTON 4  /* snf_purify_dense: after the solve, one Newton step on
                                     the occupied subspace that re-references F, then FP64
                                     refinement (see snf_purify_dense)                      */

/*
 * Inputs of a purification (Algorithm 1 and the P_{m,m} schemes need lambda_min, lambda_max,
 * mu, xi; Algorithm 2
 * and its alpha = 0 form need lambda_min, lambda_max, homo, lumo; the trace scheme needs
 * lambda_min, lambda_max, n_occ).
 *  lambda_min/lambda_max: bounds of the whole spectrum of F (lambda_min <= eig <= lambda_max).
 *  homo/lumo: a lower bound of the highest occupied eigenvalue and an upper bound of the
 *             lowest unoccupied one (the gap-edge bounds the scale-and-fold scheme needs).
 *  mu, xi:    chemical potential and band gap for the fixed-mu schemes; the gap is taken
 *             as symmetric about mu.
 *  n_occ:     number of occupied states; -1 if unknown (then no trace check is made;
 *             invalid for SNF_SP2_TRACE).
 *  tol:       stop when ||X_{i-1}^2 - X_{i-1}||_F <= tol; D = X_{i-1}.
 *  max_iter:  at most this many f_i (1..SNF_LOG_MAX-1).
 *  gap_switch: precision modes: products stay FP64 while the X-space gap
 *             (beta-bar - beta) is below this value (0 = low precision from the start).
 *  lowp_floor: precision modes: leave the low-precision phase once the a-priori
 *             eigenvalue error max(beta, 1 - beta-bar) is below this value (0 = default
 *             1e-4 for FP32, 1e-2 for BF16).
 *  flags:     SNF_FLAG_* bits.
 *  poly_i, poly_j: the polynomial P_{i,j} of SNF_SNF_FIXMU_PIJ / SNF_PIJ (odd, 1..5);
 *             ignored by the other schemes.  For these two schemes the log's beta is a and
 *             its beta-bar is 1 - a' (the bounds of the two parts above).
 *  screen_tau: snf_purify_bsr only: norm screening of the block products, >= 0 (0 = off);
 *             see snf_step_bsr; for the fixed-mu schemes every product of an iteration
 *             (for A.B the block product A_IK B_KJ is left out when
 *             ||A_IK||_F ||B_KJ||_F < screen_tau: Algorithm 1's S2.X, the Horner levels W.T of
 *             P_{m,m} and T.W of P_{i,j}, their last product X.T).  Its error is not part of
 *             the budget of
 *             SNF_FLAG_TRUNC_ERROR_CONTROL; with a fixed threshold,
 *             screen_tau <= trunc_tau / 100 left the accuracy of the lattice solves
 *             unchanged.  Ignored by the dense paths.
 */
typedef struct {
  double lambda_min, lambda_max;
  double mu, xi;
  double homo, lumo;
  int64_t n_occ;
  double tol;
  int32_t max_iter;
  int32_t flags;
  double gap_switch;
  double lowp_floor;
  int32_t poly_i, poly_j;
  double screen_tau;
} snf_params;

#define SNF_LOG_MAX 256

/* One record per iteration i = 0 .. iterations (the last one is the certifying product). */
typedef struct {
  int32_t i;          /* iteration index: X_i was the input of this product                */
  int32_t branch;     /* SNF_BRANCH_* applied to X_i (-1 for the last, certifying record)  */
  int32_t precision;  /* 0 FP64, 1 FP32, 2 BF16 product for X_i^2                          */
  int32_t reserved;   /* dense: precision phase (0 FP64, 1 low precision, 2 refinement);
                         block-sparse: stored blocks of X_i                                */
  double alpha;       /* scaling parameter of the step                                     */
  double beta;        /* image of the lumo bound in X_i                                     */
  double betabar;     /* image of the homo bound in X_i                                     */
  double e;           /* ||X_i^2 - X_i||_F                                                   */
  double t1;          /* tr X_i                                                              */
  double t2;          /* ||X_i||_F^2 = tr X_i^2                                              */
} snf_log_rec;

typedef struct {
  int32_t status;         /* mirrors the return code                                    */
  int32_t iterations;     /* f_i applied; D = X_iterations                              */
  int32_t products;       /* matrix-matrix products, the certifying one included        */
  int32_t products_fp64;  /* ... of which FP64                                          */
  int32_t products_lowp;  /* ... of which FP32 or BF16                                  */
  int32_t products_newton;/* ... of which the subspace correction and its refinement    */
  double idem_err;        /* ||D^2 - D||_F (from the certifying product)                */
  double trace;           /* tr D                                                       */
  double trace_err;       /* tr D - n_occ (0 if n_occ unknown)                          */
  double alpha_last, beta_last, betabar_last;
  double device_ms;       /* f_0 through the copy-out of D, HIP events on `stream`      */
  double product_ms;      /* summed product-kernel time (SNF_FLAG_TIME_PRODUCTS); at
                             padded order <= 256 in FP64 the whole step loop is one
                             launch, and this is its duration                          */
  uint8_t branch[SNF_LOG_MAX]; /* SNF_BRANCH_* of iteration i                            */
  double flops;           /* algorithmic flops of all products: n^2 (n+1) each (only the
                             upper triangle of a symmetric product is needed); block-sparse:
                             2 b^3 per block triple (I,K,J), I <= J, of stored blocks
                             (screened triples included: the count is the pattern's)    */
  int64_t blocks;         /* block-sparse: stored blocks of D (0 for dense)             */
} snf_result;

/*
 * snf_purify_dense -- purify a dense symmetric F (Eq. 1 with the chosen scheme).
 *   F_dev:  n x n FP64, row stride ld (elements), device, read-only, upper triangle used.
 *   D_dev:  n x n FP64 output, row stride ld, device; must not alias F_dev.
 *   n >= 1, ld >= n.
 *   log/log_cap: optional (may be NULL/0) host array receiving min(iterations+1, log_cap)
 *           snf_log_rec records.
 *   out:    host struct, filled on return (required).
 * Synchronous: returns after D and the result are complete.
 *
 * SNF_FLAG_SUBSPACE_NEWTON (not in the paper, for the precision modes): low-precision
 * products leave the occupied subspace slightly rotated, and refinement by purification,
 * being a function of the iterate alone, cannot see it.  With the flag, the solve's result
 * D~ gets one Newton step that re-references F: with G = f_0(F) of Algorithm 2, W = G D~ and
 * M = D~ G D~ (FP64 products), G splits into G - V, which commutes with D~ and has D~ as its
 * projector, and the coupling V = W + W^T - 2 M; the first-order change of the projector along
 * V comes from running Algorithm 2's polynomial sequence (from the gap-edge bounds, until
 * max(beta, 1 - beta-bar) <= 1e-10) on G - V while carrying its derivative along
 * (X1 <- c2 (X X1 + X1 X) + c1 X1, one product X X1 per step, in FP32 unless precision is
 * SNF_P_FP64); D~ + X1 is then refined by trace-correcting FP64 steps to tol.  The error left
 * is of second order in the rotation.  Needs n_occ >= 0 and gap edges (homo/lumo, or
 * mu -/+ xi/2); SNF_EINVAL otherwise.  out: the solve's decisions and log; products and flops
 * include the correction; idem_err, trace and status are the refinement's.
 */
int snf_purify_dense(const double* F_dev, int64_t n, int64_t ld, const snf_params* params,
                     snf_scheme scheme, snf_precision precision, double* D_dev,
                     snf_result* out, snf_log_rec* log, int32_t log_cap, void* stream);

/*
 * snf_purify_dense_noalloc -- snf_purify_dense for callers that cannot allocate: code under
 * HIP stream capture, tight serving loops, harnesses that forbid hipMalloc.  The call makes
 * no allocation at all (no hipMalloc / hipHostMalloc / hipFree, no events, nothing from
 * torch): all device memory beyond F and D comes from a fixed array of
 * SNF_NOALLOC_SCRATCH_BYTES that the library's code object holds on every device it is loaded
 * on, until the process ends.  Same arguments, results and errors as snf_purify_dense, bit
 * for bit (the same kernels on the same decomposition), restricted to:
 *   - precision SNF_P_FP64 and the schemes other than SNF_SNF_FIXMU_PIJ / SNF_PIJ
 *     (SNF_EINVAL otherwise);
 *   - n rounded up to a multiple of 128 at most SNF_NOALLOC_MAX_N (SNF_ESIZE otherwise).
 * The first call on a device looks up the array's device address (hipGetSymbolAddress).
 * Calls on one device share the array: the library serialises them with a per-device lock
 * within the process; work enqueued by such a call must not overlap another one's (it does
 * not: the call is synchronous).  Nothing carries over between calls (every buffer is written
 * before it is read).  snf_result.device_ms comes from the device's wall clock; the
 * SNF_FLAG_TIME_PRODUCTS flag is ignored (product_ms = 0).
 */
#define SNF_NOALLOC_MAX_N 896
#define SNF_NOALLOC_SCRATCH_BYTES (26u << 20)
int snf_purify_dense_noalloc(const double* F_dev, int64_t n, int64_t ld,
                             const snf_params* params, snf_scheme scheme,
                             snf_precision precision, double* D_dev, snf_result* out,
                             snf_log_rec* log, int32_t log_cap, void* stream);

/*
 * snf_step_dense -- one purification step on a dense symmetric X, the unit of work of the
 * loop above (rows a2+a3 of the method: product and fused combination).
 *   Computes P = A.B (A, B symmetric n x n FP64, row stride ld, device; they need not
 *   commute) and
 *     Y = c2 P + c1 A + c0 I            (written to Y_dev, row stride ld)
 *   and, in FP64, sums[0] = ||P - A||_F^2, sums[1] = tr Y, sums[2] = ||Y||_F^2
 *   (host array of 3 doubles).  With A == B (the same pointer) this is one f_i of Eqs. 4-5
 *   and the idempotency check of A; P is then symmetric, only its upper triangle of tiles is
 *   computed and Y is exactly symmetric.  With A != B every tile is computed (twice the
 *   work) and Y is in general not symmetric.  Only the upper triangles of A and B are
 *   assumed to define them in neither case: both must be stored in full.
 *   precision: SNF_P_FP64 (f64 MFMA), SNF_P_FP32 (f32 MFMA on FP32-rounded copies of A and
 *   B), SNF_P_BF16_REF64 (bf16 MFMA with FP32 accumulation on BF16-rounded copies).  Y_dev
 *   must not alias A_dev or B_dev.  Synchronous.
 *   kernel_ms (optional, may be NULL): duration of the product kernel (HIP events).
 */
int snf_step_dense(const double* A_dev, const double* B_dev, int64_t n, int64_t ld,
                   double c2, double c1, double c0, snf_precision precision, double* Y_dev,
                   double* sums, double* kernel_ms, void* stream);

/* ---- block-sparse (BSR) path ----------------------------------------------------------
 * The linear-scaling regime (the sparsity paragraph of the paper: the schemes are of the
 * form of Eq. 1, so they combine with truncation of small matrix elements).  X is stored in
 * block-sparse row form with square FP32 blocks; after every step the blocks of X_new with
 * Frobenius norm below trunc_tau are dropped (block (I,J) together with (J,I); diagonal
 * blocks are always kept), so the pattern, the memory and the work follow the decay of D.
 */
typedef struct {
  int64_t n;          /* order; a multiple of b                                             */
  int32_t b;          /* block size; must be 32                                             */
  int32_t nb;         /* block rows = n / b                                                 */
  int64_t nnzb;       /* stored blocks                                                      */
  int32_t* row_ptr;   /* device, nb + 1 entries, row_ptr[0] = 0, row_ptr[nb] = nnzb         */
  int32_t* col_idx;   /* device, nnzb block-column indices, strictly ascending in each row  */
  float* val;         /* device, nnzb * b * b values, each block row-major                  */
} snf_bsr;

/*
 * snf_purify_bsr -- purify a block-sparse symmetric F.  Schemes SNF_SP2_TRACE, SNF_TC2_BETA,
 * SNF_SNF_VARMU (one product per iteration) and the fixed-mu SNF_SNF_FIXMU, SNF_MCWEENY
 * (Algorithm 1 and its alpha = 1 form: S2 = Xs^2, then S2.X, Xs = a (X - I/2) + I/2),
 * SNF_SNF_FIXMU3/5 and SNF_PMM3/5 (P_{m,m}: W = Xs'^2, Horner levels in W, then X.T; m + 1
 * products), SNF_SNF_FIXMU_PIJ and SNF_PIJ (P_{i,j}: the first product writes W and the top
 * Horner level, then the levels, then X.T; (i + j)/2 + 1 products).  A fixed-mu iteration's
 * intermediates keep every candidate block and the truncation applies to its result; these
 * schemes' error-control budget (SNF_FLAG_TRUNC_ERROR_CONTROL) applies to each iteration's
 * result, with the gap of the bounds of the iterate it produces (for P_{i,j} 1 - a - a') and
 * N from the scheme's own recurrence; screen_tau applies to every product of their
 * iterations.
 *   F:      caller-owned, device arrays; the pattern must be symmetric with every diagonal
 *           block present; only blocks (I,J) with I <= J (and the upper triangle of diagonal
 *           blocks) are read, the rest is taken as their transpose.
 *   trunc_tau: block truncation threshold (Frobenius norm), >= 0 (0 = no truncation).
 *           With SNF_FLAG_TRUNC_ERROR_CONTROL in params->flags, trunc_tau > 0 is instead a
 *           budget eps for ||D - D_exact||_F (forward-error control, which the sparsity
 *           paragraph expects the schemes to combine with): the step producing X_i drops
 *           off-diagonal block pairs of total Frobenius norm at most eps g_i / (sqrt 2 N), with
 *           g_i = beta-bar_i - beta_i the X-space gap of X_i (a perturbation E of X_i turns its
 *           occupied subspace by about ||E|| / g_i) and N the iterations the scalar recurrence
 *           predicts until max(beta, 1 - beta-bar) <= eps.  The blocks dropped are those in the
 *           lowest bins of a half-octave grid of squared block norms, floor(2 log2 ||B||_F^2)
 *           clamped to [-160, 40], while the bins' charge, 2 count_j 2^((j+1)/2) (each bin at
 *           its upper edge, mirror blocks included), stays within the step's budget squared.
 *   D_out:  receives a library-allocated snf_bsr (host struct, device arrays) holding D;
 *           release it with snf_bsr_free.  NULL on error.
 *   Stops with SNF_OK at ||X^2 - X||_F <= tol, or SNF_OK_FLOOR once the a-priori error
 *   bound max(beta, 1 - beta-bar) is below params->lowp_floor (0 = default 1e-3) and the
 *   idempotency error stopped shrinking (e_i > 0.5 e_{i-2}): the truncation floor.
 *   Synchronous; reads pattern sizes back to the host once per iteration.
 */
int snf_purify_bsr(const snf_bsr* F, const snf_params* params, snf_scheme scheme,
                   double trunc_tau, snf_bsr** D_out, snf_result* out, snf_log_rec* log,
                   int32_t log_cap, void* stream);

/*
 * snf_step_bsr -- one block-sparse step: Y = trunc_tau-truncation of (c2 X.X + c1 X + c0 I),
 * the unit of work of the loop above; sums[0] = ||X.X - X||_F^2, sums[1] = tr Y,
 * sums[2] = ||Y||_F^2 (after truncation).  X as F above; *Y_out library-allocated.
 * kernel_ms (optional): duration of the numeric product kernel.
 * screen_tau (>= 0; 0 = off): norm screening of the product, the other way to exploit the
 *   decay of the blocks that the sparsity paragraph points to: the block product
 *   X_IK X_KJ is left out of (X.X)_IJ when ||X_IK||_F ||X_KJ||_F < screen_tau (block norms
 *   of the FP32 values, in FP64).  Each term left out has Frobenius norm below screen_tau,
 *   so (X.X)_IJ moves by less than screen_tau times the number of such K.  The screened
 *   product is used both for sums[0] and for Y; the pattern of Y is still that of X.X.
 *   SNF_EINVAL for a negative or non-finite value.
 */
int snf_step_bsr(const snf_bsr* X, double c2, double c1, double c0, double trunc_tau,
                 double screen_tau, snf_bsr** Y_out, double* sums, double* kernel_ms,
                 void* stream);

/* Copy the arrays of a (library-allocated) snf_bsr into caller device buffers of sizes
   nb + 1, nnzb and nnzb * b * b; enqueued on `stream`, returns after completion. */
int snf_bsr_copy_out(const snf_bsr* src, int32_t* row_ptr, int32_t* col_idx, float* val,
                     void* stream);

/* Free a library-allocated snf_bsr (device arrays and the struct).  NULL is ignored. */
void snf_bsr_free(snf_bsr* m);

/* ---- serving: many independent purifications, continuous batching --------------------
 * A server owns one device arena of hbm_budget_bytes, a HIP stream and a scheduler thread.
 * Submitted requests wait in a FIFO queue and are admitted while a slot is free and their
 * workspace fits in the arena; admitted requests advance together, one product step per
 * grouped launch (each request keeps its own X, scalar state and partial sums on the
 * device), finished requests leave and queued ones join between steps.  A request's tile
 * decomposition and reduction order do not depend on the other requests in flight, so its
 * result is bitwise the same alone and in any mix.  Created on the current device.
 */
typedef struct snf_server snf_server;

/* hbm_budget_bytes: arena size (device memory for all in-flight requests);
   max_slots: at most this many requests in flight (1..4096).  *out receives the server. */
int snf_serve_create(size_t hbm_budget_bytes, int32_t max_slots, snf_server** out);

/* Device bytes one request of order n and this precision occupies in the arena (the schemes
   with one or two products per iteration; a P_{m,m} or P_{i,j} request, FP64 only, holds one
   more n_pad x n_pad FP64 buffer, n_pad = n rounded up to a multiple of 128). */
size_t snf_serve_request_bytes(int64_t n, snf_precision precision);

/* Queue a purification of the host n x n FP64 matrix F_host (row-major, copied before the
 * call returns, so the caller may reuse it).  D_host_out (n x n FP64, row-major) receives D
 * and must stay valid until snf_serve_poll reports completion.  Never waits for the GPU.
 * Returns SNF_OK and a ticket; SNF_EINVAL for bad arguments (checked as for
 * snf_purify_dense, so the P_{m,m} and P_{i,j} schemes are served in SNF_P_FP64 only);
 * SNF_ENOMEM if the request alone exceeds the budget. */
int snf_serve_submit(snf_server* server, const double* F_host, int64_t n,
                     const snf_params* params, snf_scheme scheme, snf_precision precision,
                     double* D_host_out, uint64_t* ticket);

/* As snf_serve_submit, for inputs already resident on the server's device: F_dev (n x n
 * FP64, row-major, device) is read when the request is admitted and must stay unchanged
 * until completion; D_dev_out (n x n FP64, row-major, device, not aliasing F_dev) receives
 * D.  No host staging and no PCIe transfer of the matrices. */
int snf_serve_submit_device(snf_server* server, const double* F_dev, int64_t n,
                            const snf_params* params, snf_scheme scheme,
                            snf_precision precision, double* D_dev_out, uint64_t* ticket);

/* SNF_PENDING while the request is queued or running; otherwise its final status, with
 * *out filled (when out is not NULL) as snf_purify_dense would fill it.  device_ms = time
 * from admission to completion.  SNF_EINVAL for an unknown ticket. */
int snf_serve_poll(snf_server* server, uint64_t ticket, snf_result* out);

/* Per-request latency in milliseconds: ms[0] queued (submit -> admit), ms[1] running
   (admit -> done), ms[2] total (submit -> done).  SNF_PENDING until done. */
int snf_serve_timing(snf_server* server, uint64_t ticket, double* ms);

/* Per-request timeline in milliseconds since snf_serve_create: t[0] submitted, t[1] admitted
 * (slot and arena memory taken), t[2] finished (the scheduler saw the stop flag of the
 * request's last step, which has completed on the device; from here its memory may be given
 * to a queued request, whose device work is stream-ordered behind this one's copy-out),
 * t[3] done (the result is complete and visible to snf_serve_poll).  t: host array of 4
 * doubles.  SNF_PENDING until done, SNF_EINVAL for an unknown ticket. */
int snf_serve_timeline(snf_server* server, uint64_t ticket, double* t);

/* Finish every queued and running request, stop the scheduler, release the arena. */
int snf_serve_destroy(snf_server* server);

/* ---- bounds of the inputs --------------------------------------------------------------
 * Both algorithms take bounds as inputs: the extremal eigenvalues of F or bounds of them, and
 * for the scaled varying-mu scheme a lower bound of the highest occupied (homo) and an upper
 * bound of the lowest unoccupied (lumo) eigenvalue (the bounds paragraph after Fig. 3, which
 * points to methods for interior eigenvalues).  Both estimators run `steps` Lanczos steps with
 * full reorthogonalisation (classical Gram-Schmidt applied twice) on the device, from
 * start_dev (n FP64 values, device; NULL = a fixed pseudo-random vector, u_i in [-1, 1) from
 * SplitMix64 of i), and diagonalise the tridiagonal on the host.  The tridiagonal is cut at
 * the first beta_j <= 1e-12 max |alpha_0..j| (an invariant subspace).  Matrices are dense
 * row-major FP64 with row stride ld, upper triangle read.  1 <= steps <= 512.  The
 * workspace (steps + 1 vectors per Lanczos chain) is kept per device.  Synchronous on
 * `stream`.
 */

/* snf_spectral_bounds -- out[0] = theta_min - r_min - pad, out[1] = theta_max + r_max + pad,
 * theta the extreme Ritz values, r their residual norms beta_k |s_k| (an eigenvalue lies
 * within r of theta), pad = 1e-13 max |theta| for rounding: outer bounds once the extreme Ritz
 * pairs belong to the extreme eigenvalues, which a small r shows.  out[2], out[3] = the
 * Gershgorin enclosure (rigorous, looser).  out: host array of 4 doubles. */
int snf_spectral_bounds(const double* F_dev, int64_t n, int64_t ld, int32_t steps,
                        const double* start_dev, double* out, void* stream);

/* snf_gap_bounds -- from D_dev, a projector onto the occupied subspace of F (the result of a
 * trace-scheme purification needs no gap bounds): the largest eigenvalue of
 * D (F - lambda_min I) D is HOMO - lambda_min and that of (I - D)(lambda_max I - F)(I - D) is
 * lambda_max - LUMO; Ritz values never exceed the largest eigenvalue, so
 * out[0] = lambda_min + theta_1 - pad <= HOMO and out[1] = lambda_max - theta_2 + pad >= LUMO
 * at any number of steps (pad = 1e-13 (lambda_max - lambda_min)); loose after few steps,
 * never inside the gap, up to a shift of second order in the subspace error of D.
 * lambda_min < lambda_max: bounds of the spectrum (for example from snf_spectral_bounds).
 * out: host array of 2 doubles. */
int snf_gap_bounds(const double* F_dev, const double* D_dev, int64_t n, int64_t ld,
                   double lambda_min, double lambda_max, int32_t steps,
                   const double* start_dev, double* out, void* stream);

/* Bytes of device workspace snf_purify_dense needs for order n (allocated on demand); the
   P_{m,m} schemes take one more n_pad x n_pad FP64 buffer (n_pad = n rounded up to 128). */
size_t snf_workspace_bytes(int64_t n, snf_precision precision);

/* Release the calling device's cached workspace (it is re-created on the next call). */
int snf_release_workspace(void);

/* Release every per-device workspace the library holds, on every device it has used:
 * device buffers, pinned host memory, HIP events (snf_release_workspace frees only the
 * calling device's dense buffers).  Call it while the HIP runtime is still up, before the
 * process exits (the Python binding registers it with atexit), so that no allocation of the
 * library is left to the runtime's own teardown.  Destroy servers first; the call must not
 * overlap other calls into the library.  The library stays usable: the next call on a device
 * sets its workspace up again.  Returns SNF_OK. */
int snf_shutdown(void);

/* Human-readable text of a status code (static storage; SNF_EDEVICE includes the last
   HIP error string seen by this thread). */
const char* snf_strerror(int status);

/* Library version string "major.minor.patch". */
const char* snf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SNF_H */
