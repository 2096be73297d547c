// Internal declarations shared by the HIP translation units of libsnf (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/snf.h"
#include "schedule_math.h"

namespace snf {

// Output tile of one workgroup of the dense product kernels, and the padding unit of
// every internal n x n buffer (so the product main loop needs no bounds checks).
constexpr int kTile = 128;
constexpr int kThreads = 256;        // threads of the bf16 product and split fix-up kernels
constexpr int kF0Blocks = 1024;      // fixed grid of the f0 / conversion kernels
constexpr int kReduceThreads = 256;

// Precision of a product.
enum : int32_t { kPrecF64 = 0, kPrecF32 = 1, kPrecBF16 = 2 };

// Phase of the precision schedule.
enum : int32_t { kPhaseHigh = 0, kPhaseLow = 1, kPhaseRefine = 2 };

// Kind of the pending product.
enum : int32_t {
  kKindSquare = 0,   // P = X.X, epilogue Y = c2 P + c1 X + c0 I, idempotency of X checked
  kKindCube = 1,     // Algorithm 1 second product: R = S2.X, Y = c2 R + c1 S2
  kKindHorner = 2,   // P_{m,m}: T <- W.T + r_k I (or the first level from W.W);
                     // P_{i,j}: T <- T.W + c1 X + c0 I
  kKindFinal = 3     // P_{m,m}: X_new = a X.T0 - (a/2) T0 + I/2;
                     // P_{i,j}: X_new = a X.T0 - a x* T0 + x* I
};

// m of a P_{m,m} scheme (3 or 5), 0 for the other schemes.
inline __host__ __device__ int scheme_pmm_m(int scheme) {
  return (scheme == SNF_SNF_FIXMU3 || scheme == SNF_PMM3) ? 3
       : (scheme == SNF_SNF_FIXMU5 || scheme == SNF_PMM5) ? 5 : 0;
}

// The P_{i,j} schemes (i, j from snf_params).
inline __host__ __device__ bool scheme_is_pij(int scheme) {
  return scheme == SNF_SNF_FIXMU_PIJ || scheme == SNF_PIJ;
}

// Matrix products one f_i costs (pi, pj: the P_{i,j} schemes' polynomial).
inline int products_per_iteration(int scheme, int pi = 0, int pj = 0) {
  const int m = scheme_pmm_m(scheme);
  if (m) return m + 1;
  if (scheme_is_pij(scheme)) return (pi + pj) / 2 + 1;
  return (scheme == SNF_MCWEENY || scheme == SNF_SNF_FIXMU) ? 2 : 1;
}

// Scalar state of one purification, resident in device memory.  Written by the host
// once (configuration), then only by the schedule kernel (one thread).
struct SnfState {
  // ---- configuration ----
  int32_t scheme;
  int32_t max_iter;
  int32_t mode;          // snf_precision
  int32_t has_nocc;
  int64_t n;
  int64_t n_occ;
  double tol, lambda_min, lambda_max, mu, xi, homo, lumo;
  double gap_switch, lowp_floor;
  // ---- evolving ----
  double beta, betabar, gamma;
  double t1, t2;          // tr X_cur, ||X_cur||_F^2
  double alpha;           // alpha of the pending iteration
  double c2, c1, c0;      // epilogue coefficients of the pending product
  double e_last;
  double e_hist[3];       // idempotency of the last three iterates (stagnation test)
  int32_t iter;           // f_i applied; X_cur = X_iter
  int32_t products, products_f64, products_lowp;
  int32_t kind;           // kKind* of the pending product
  int32_t branch;         // SNF_BRANCH_* of the pending iteration
  int32_t prec;           // kPrec* of the pending product
  int32_t phase;          // kPhase*
  int32_t stop;           // 0 while running; else 1 + index into the status table below
  int32_t status;         // final snf status code once stop != 0
  int32_t cur;            // buffer index holding X_cur
  int32_t ia, ib, ix, io; // operand / linear-term / output buffer indices of the pending product
  int32_t pmm_m;          // m of a P_{m,m} scheme, else 0
  int32_t horner_left;    // P_{m,m}: Horner products still to run in this iteration
  int32_t bw, bt;         // P_{m,m}, P_{i,j}: buffers holding W and the last Horner T
  int32_t pij_i, pij_j;   // P_{i,j} schemes: the polynomial, else 0
  double xstar;           // fixed-mu schemes: image of mu in X_0 (1/2, or x* of P_{i,j})
  double abar;            // P_{i,j}: distance of the occupied part's lower bound from 1
  double pq[sched::kPijQ];  // P_{i,j}: P(x* + v) = x* + v sum_k pq[k] v^k
  double pbin[2][sched::kPijMax + 1];   // C(i+k, k) (k <= j) and C(j+k, k) (k <= i)
  double pr[sched::kPmmMaxM + 1];       // P_{m,m}: r_0 .. r_m
  int32_t dual;           // pending product also writes Y2 = d2 P + d1 X + d0 I to x[io2]
  int32_t io2;
  double d2, d1, d0;
  int32_t want_e;         // pending product checks idempotency of its A operand
  int32_t write_lowp;     // epilogue also writes the low-precision operand copy
  int32_t nlog;
  snf_log_rec log[SNF_LOG_MAX];
};

// Buffers of one purification: three FP64 n_pad x n_pad matrices (four for the P_{m,m}
// schemes) and, for precision modes, their low-precision operand copies (FP32 or BF16, same
// indices).
struct Buffers {
  double* x[4];
  void* lp[4];
};

// ---- kernels launched by the host drivers (defined in kernels_dense.hip) ----------------
void launch_f0(const double* F, int64_t n, int64_t ld, int64_t np, SnfState* st,
               const Buffers* bufs_dev, int lowp_kind, double* partials, hipStream_t s);
void launch_schedule(SnfState* st, const double* partials, int count, int init,
                     hipStream_t s);
// Work decomposition of one product launch (see make_product_grid).
struct ProductGrid {
  int64_t np, n;       // padded and true order
  int sym;             // 1: upper-triangle tiles, mirrored output
  int dp_tiles;        // tiles computed whole, one workgroup each
  int tail_tiles;      // following tiles, each split into split_s k-slices
  int split_s;
  int partial_count;   // partial-sum slots written: dp_tiles + 16 * tail_tiles (or tiles)
  double* partials;    // [partial_count][4] FP64 sums per tile / fix-up workgroup
  double* split_buf;   // [tail_tiles * split_s][64][256] raw accumulators of the slices
};

// Split the last (tiles mod num_cus) tiles into k-slices when that tail would leave most
// compute units idle, or a single wave of fewer tiles than compute units would hold one
// workgroup per unit; split_cap = slices the split buffer holds.
ProductGrid make_product_grid(int64_t np, int64_t n, int sym, int num_cus, double* partials,
                              double* split_buf, int split_cap, int stage_depth);
// k values per stage of the deepest product variant a precision mode may run
inline int stage_depth_for(snf_precision p) {
  return p == SNF_P_BF16_REF64 ? 64 : (p == SNF_P_FP32 || p == SNF_P_FP32_REF64) ? 32 : 16;
}
constexpr int kSplitCap = 512;   // slices held by the split buffer (64*256 doubles each)

// Product of the pending step; each variant exits at once unless the state asks for its
// precision (so the host can enqueue all variants without knowing the device's choice).
void launch_product(int prec, SnfState* st, const Buffers* bufs_dev, const ProductGrid& g,
                    hipStream_t s);
// Small orders: FP64 product in 32x32 tiles of the upper triangle, k split over the four
// waves of a workgroup and summed in LDS (no split fix-up); one partial slot per tile.
constexpr int64_t kSmallMaxNp = 896;   // padded orders that take this path (FP64 mode)
struct SmallGrid {
  int64_t np, n;
  int tiles;
  double* partials;
};
SmallGrid make_small_grid(int64_t np, int64_t n, double* partials);
void launch_product_small(SnfState* st, const Buffers* bufs_dev, const SmallGrid& g,
                          hipStream_t s);
// The whole step loop of a small-order FP64 solve in one cooperative launch (one workgroup
// per 32x32 tile, a grid barrier per step); partials2 holds 2 x tiles slots.  Returns 0, or
// -1 when the runtime refuses the cooperative launch.
constexpr int64_t kPersistMaxNp = 256;
int launch_solve_small(SnfState* st, const Buffers* bufs_dev, const SmallGrid& g,
                       double* partials2, int max_steps, hipStream_t s);
// FP64 product with the second epilogue output (P_{i,j} schemes: launched beside
// launch_product(kPrecF64, ...); exactly one of the two runs, as the state asks).
void launch_product_dual(SnfState* st, const Buffers* bufs_dev, const ProductGrid& g,
                         hipStream_t s);
void launch_split_fixup(SnfState* st, const Buffers* bufs_dev, const ProductGrid& g,
                        hipStream_t s);
void launch_copy_out(const SnfState* st, const Buffers* bufs_dev, int64_t n, int64_t np,
                     double* D, int64_t ld, hipStream_t s);
// Padded copy helpers for the stand-alone step.
void launch_pad_copy(const double* src, int64_t n, int64_t ld, double* dst, int64_t np,
                     void* lp_dst, int lowp_kind, hipStream_t s);
void launch_unpad_copy(const double* src, int64_t np, int64_t n, double* dst, int64_t ld,
                       hipStream_t s);
void launch_sum_partials(const double* partials, int count, double* out3, hipStream_t s);

int num_product_tiles(int64_t np, int sym);

// ---- subspace correction (kernels_dense.hip; driven by snf_purify_dense) ----------------
// One product of the host-planned correction sequence: buffer indices into the Buffers
// table the launch uses, the product's precision, whether the epilogue writes the FP32 copy,
// and the epilogue coefficients Y = c2 P + c1 X[ix] + c0 I.
struct NewtonOp {
  int32_t ia, ib, ix, io, prec, write_lowp;
  double c2, c1, c0;
};
void launch_newton_set(SnfState* st, const NewtonOp* ops, int k, hipStream_t s);
void launch_newton_split(const double* G, const double* W, const double* M, int64_t n,
                         int64_t np, double* Xbd, float* Xbd_lp, double* X1, float* X1_lp,
                         hipStream_t s);
void launch_newton_sym(const double* Z, const double* X1, double c2, double c1, int64_t n,
                       int64_t np, double* out, float* out_lp, hipStream_t s);
void launch_newton_add(const double* Dt, const double* X1, int64_t n, int64_t np, double* out,
                       double* partials, hipStream_t s);

// Keep the text of a failed HIP call for snf_strerror(SNF_EDEVICE); returns SNF_EDEVICE.
int record_hip_error(hipError_t e, const char* what);

// Release every per-device workspace of one translation unit (device buffers, pinned host
// memory, events), each with its device current; the workspaces are set up again on their
// next use.  snf_shutdown calls all three.
void dense_release_all_devices();
void bsr_release_all_devices();
void bounds_release_all_devices();

// Host helpers of the dense driver, shared with the serving loop (api_dense.hip).
int validate(int64_t n, const snf_params* p, snf_scheme scheme, snf_precision prec);
void init_state(SnfState* s, int64_t n, const snf_params* p, snf_scheme scheme,
                snf_precision prec);
void fill_result(const SnfState* s, snf_result* out, snf_log_rec* log, int log_cap);
int lowp_bytes_for(snf_precision p);
int lowp_kind_for(snf_precision p);

// One request of a grouped launch (device array, one entry per serving slot).
struct SlotDesc {
  SnfState* st;
  Buffers* bufs;       // device
  double* partials;    // [tiles][4]
  int64_t np, n;
};

// One step of every active request: product variants selected by prec_mask (bit kPrec*, and
// kGroupedDualBit for the FP64 variant with a second output that P_{i,j} requests take),
// each request's schedule, and the stop flags gathered into stop_out[nactive] (0 while a
// request runs; 1 + the buffer index of its result once it stopped).  With s2 and
// the two events, the FP32 / BF16 product launches run on s2 beside the FP64 one on s.
// offs[a] = first workgroup of active request a (offs[nactive] = total_tiles).
constexpr int kGroupedDualBit = 1 << 8;
void launch_grouped_step(int prec_mask, const SlotDesc* slots, const int* active,
                         const int* offs, int nactive, int total_tiles, int32_t* stop_out,
                         hipStream_t s, hipStream_t s2 = nullptr, hipEvent_t fork = nullptr,
                         hipEvent_t join = nullptr);

}  // namespace snf
