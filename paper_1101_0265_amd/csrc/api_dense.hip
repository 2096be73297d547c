// Host side of the dense C ABI: validation, workspace, the launch-ahead purification loop.
//
// The loop is driven from the host but decided on the device: every product step is the
// pair (product kernel, schedule kernel); the schedule kernel writes the next step's
// coefficients, buffer indices and precision into the device-resident state, and sets a
// stop flag once ||X^2 - X||_F <= tol (or an error / iteration limit).  Kernels enqueued after
// the stop exit immediately.  The host keeps two chunks of steps in flight and reads the
// stop flag of the older chunk from pinned memory, so the GPU never waits for the host and
// at most one chunk of empty launches follows convergence.  At the smallest orders the whole
// loop is one cooperative launch instead.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <memory>
#include <mutex>
#include <vector>

#include "schedule_math.h"
#include "snf_internal.h"

namespace snf {

static thread_local char g_err_text[256];

static int dev_error(hipError_t e, const char* what) {
  snprintf(g_err_text, sizeof(g_err_text), "HIP error in %s: %s", what, hipGetErrorString(e));
  return SNF_EDEVICE;
}

int record_hip_error(hipError_t e, const char* what) { return dev_error(e, what); }

#define SNF_HIP(call)                                  \
  do {                                                 \
    hipError_t _e = (call);                            \
    if (_e != hipSuccess) return dev_error(_e, #call); \
  } while (0)

static int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// ---- per-device workspace -------------------------------------------------------------
struct Workspace {
  int64_t np = 0;          // padded order the buffers hold
  int lp_bytes = 0;        // bytes per element of the low-precision copies (0, 2, 4)
  double* x[4] = {nullptr, nullptr, nullptr, nullptr};
  void* lp[4] = {nullptr, nullptr, nullptr, nullptr};
  double* partials = nullptr;
  int partial_cap = 0;
  double* split_buf = nullptr;       // kSplitCap slices of 64*256 doubles
  int num_cus = 0;
  SnfState* state = nullptr;
  Buffers* bufs_dev = nullptr;
  SnfState* state_host = nullptr;    // pinned
  int32_t* flags_host = nullptr;     // pinned, [2] stop flags of in-flight chunks
  double* sums_dev = nullptr;
  double* sums_host = nullptr;       // pinned
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> prod_ev;
  // subspace correction: five FP64 buffers of order nnp, FP32 copies of four of them, the
  // Buffers tables and the planned product sequence on the device
  int64_t nnp = 0;
  bool nlp_on = false;
  double* nx[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  float* nlp[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  Buffers* nbufs_dev = nullptr;      // [4] tables
  NewtonOp* nops_dev = nullptr;
  int nops_cap = 0;
  std::mutex mu;
};

static std::mutex g_ws_mu;
static Workspace* g_ws[64];

static Workspace* workspace_for_current_device(int* dev_out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> g(g_ws_mu);
  if (!g_ws[dev]) g_ws[dev] = new Workspace();
  *dev_out = dev;
  return g_ws[dev];
}

static void free_buffers(Workspace* w) {
  for (int i = 0; i < 4; ++i) {
    if (w->x[i]) (void)hipFree(w->x[i]);
    if (w->lp[i]) (void)hipFree(w->lp[i]);
    w->x[i] = nullptr;
    w->lp[i] = nullptr;
  }
  w->np = 0;
  w->lp_bytes = 0;
}

// Every resource of a workspace: device buffers, pinned host memory, events.  The object
// itself stays (another thread may be waiting on its mutex) and is set up again on its next
// use.  Called with w->mu held and the workspace's device current.
static void free_newton(Workspace* w) {
  for (int i = 0; i < 5; ++i) {
    if (w->nx[i]) (void)hipFree(w->nx[i]);
    if (w->nlp[i]) (void)hipFree(w->nlp[i]);
    w->nx[i] = nullptr;
    w->nlp[i] = nullptr;
  }
  w->nnp = 0;
  w->nlp_on = false;
}

static void release_all(Workspace* w) {
  free_buffers(w);
  free_newton(w);
  if (w->nbufs_dev) (void)hipFree(w->nbufs_dev);
  w->nbufs_dev = nullptr;
  if (w->nops_dev) (void)hipFree(w->nops_dev);
  w->nops_dev = nullptr;
  w->nops_cap = 0;
  if (w->x[3]) (void)hipFree(w->x[3]);
  w->x[3] = nullptr;
  if (w->partials) (void)hipFree(w->partials);
  w->partials = nullptr;
  w->partial_cap = 0;
  if (w->split_buf) (void)hipFree(w->split_buf);
  w->split_buf = nullptr;
  if (w->state) (void)hipFree(w->state);
  w->state = nullptr;
  if (w->bufs_dev) (void)hipFree(w->bufs_dev);
  w->bufs_dev = nullptr;
  if (w->sums_dev) (void)hipFree(w->sums_dev);
  w->sums_dev = nullptr;
  if (w->state_host) (void)hipHostFree(w->state_host);
  w->state_host = nullptr;
  if (w->flags_host) (void)hipHostFree(w->flags_host);
  w->flags_host = nullptr;
  if (w->sums_host) (void)hipHostFree(w->sums_host);
  w->sums_host = nullptr;
  for (int i = 0; i < 4; ++i) {
    if (w->ev[i]) (void)hipEventDestroy(w->ev[i]);
    w->ev[i] = nullptr;
  }
  for (hipEvent_t e : w->prod_ev) (void)hipEventDestroy(e);
  w->prod_ev.clear();
  w->num_cus = 0;
}

void dense_release_all_devices() {
  int prev = 0;
  const bool restore = hipGetDevice(&prev) == hipSuccess;
  for (int dev = 0; dev < 64; ++dev) {
    Workspace* w = nullptr;
    {
      std::lock_guard<std::mutex> g(g_ws_mu);
      w = g_ws[dev];
    }
    if (!w || hipSetDevice(dev) != hipSuccess) continue;
    std::lock_guard<std::mutex> g(w->mu);
    (void)hipDeviceSynchronize();
    release_all(w);
  }
  if (restore) (void)hipSetDevice(prev);
}

// nbuf: FP64 n_pad x n_pad buffers the call needs (3, or 4 for the P_{m,m} and P_{i,j}
// schemes).
static int ensure_workspace(Workspace* w, int64_t np, int lp_bytes, int partial_need,
                            int nbuf = 3) {
  if (!w->state) {
    SNF_HIP(hipMalloc(&w->state, sizeof(SnfState)));
    SNF_HIP(hipMalloc(&w->bufs_dev, sizeof(Buffers)));
    SNF_HIP(hipHostMalloc(&w->state_host, sizeof(SnfState), hipHostMallocDefault));
    SNF_HIP(hipHostMalloc(&w->flags_host, 8 * sizeof(int32_t), hipHostMallocDefault));
    SNF_HIP(hipMalloc(&w->sums_dev, 4 * sizeof(double)));
    SNF_HIP(hipHostMalloc(&w->sums_host, 4 * sizeof(double), hipHostMallocDefault));
    for (int i = 0; i < 4; ++i) SNF_HIP(hipEventCreate(&w->ev[i]));
    int dev = 0;
    SNF_HIP(hipGetDevice(&dev));
    SNF_HIP(hipDeviceGetAttribute(&w->num_cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (hipMalloc(&w->split_buf, (size_t)kSplitCap * 64 * kThreads * sizeof(double)) !=
        hipSuccess) {
      (void)hipGetLastError();
      w->split_buf = nullptr;   // no split tail: whole tiles only
    }
  }
  if (partial_need > w->partial_cap) {
    if (w->partials) (void)hipFree(w->partials);
    w->partials = nullptr;
    const int cap = partial_need < kF0Blocks ? kF0Blocks : partial_need;
    if (hipMalloc(&w->partials, (size_t)cap * 4 * sizeof(double)) != hipSuccess) {
      w->partial_cap = 0;
      (void)hipGetLastError();
      return SNF_ENOMEM;
    }
    w->partial_cap = cap;
  }
  if (np > w->np || lp_bytes > w->lp_bytes) {
    free_buffers(w);
    const size_t elems = (size_t)np * (size_t)np;
    for (int i = 0; i < 3; ++i) {
      if (hipMalloc(&w->x[i], elems * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        free_buffers(w);
        return SNF_ENOMEM;
      }
      if (lp_bytes && hipMalloc(&w->lp[i], elems * lp_bytes) != hipSuccess) {
        (void)hipGetLastError();
        free_buffers(w);
        return SNF_ENOMEM;
      }
    }
    w->np = np;
    w->lp_bytes = lp_bytes;
  }
  if (nbuf > 3 && !w->x[3]) {
    const size_t elems = (size_t)w->np * (size_t)w->np;
    if (hipMalloc(&w->x[3], elems * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      w->x[3] = nullptr;
      return SNF_ENOMEM;
    }
  }
  return SNF_OK;
}

int lowp_bytes_for(snf_precision p) {
  switch (p) {
    case SNF_P_FP32:
    case SNF_P_FP32_REF64: return 4;
    case SNF_P_BF16_REF64: return 2;
    default: return 0;
  }
}

int lowp_kind_for(snf_precision p) {
  switch (p) {
    case SNF_P_FP32:
    case SNF_P_FP32_REF64: return kPrecF32;
    case SNF_P_BF16_REF64: return kPrecBF16;
    default: return -1;
  }
}

// Buffers of the internal loop are the workspace buffers, but their padded order can be
// larger than this call needs; the kernels use the call's np with the same base pointers,
// so a buffer of order w->np serves any np <= w->np.
static int upload_buffers(Workspace* w, hipStream_t s) {
  Buffers b;
  for (int i = 0; i < 4; ++i) {
    b.x[i] = w->x[i];
    b.lp[i] = w->lp[i];
  }
  SNF_HIP(hipMemcpyAsync(w->bufs_dev, &b, sizeof(b), hipMemcpyHostToDevice, s));
  return SNF_OK;
}

// ---- validation -------------------------------------------------------------------------
static bool finite(double v) { return isfinite(v) != 0; }

int validate(int64_t n, const snf_params* p, snf_scheme scheme, snf_precision prec) {
  if (!p || n <= 0) return SNF_EINVAL;
  if ((int)scheme < SNF_SP2_TRACE || (int)scheme > SNF_PIJ) return SNF_EINVAL;
  if ((int)prec < SNF_P_FP64 || (int)prec > SNF_P_BF16_REF64) return SNF_EINVAL;
  if (!finite(p->lambda_min) || !finite(p->lambda_max) || !(p->lambda_min < p->lambda_max))
    return SNF_EINVAL;
  if (!(p->tol > 0.0) || !finite(p->tol)) return SNF_EINVAL;
  if (p->max_iter < 1 || p->max_iter >= SNF_LOG_MAX) return SNF_EINVAL;
  if (p->n_occ >= 0 && p->n_occ > n) return SNF_EINVAL;
  const bool gap_edges = finite(p->homo) && finite(p->lumo) && p->homo < p->lumo &&
                         p->lambda_min <= p->homo && p->lumo <= p->lambda_max;
  switch (scheme) {
    case SNF_SP2_TRACE:
      if (p->n_occ < 0) return SNF_EINVAL;
      if (prec != SNF_P_FP64 && !gap_edges) return SNF_EINVAL;
      break;
    case SNF_TC2_BETA:
    case SNF_SNF_VARMU:
      if (!gap_edges) return SNF_EINVAL;
      break;
    case SNF_SNF_FIXMU_PIJ:
    case SNF_PIJ: {
      if (prec != SNF_P_FP64) return SNF_EINVAL;
      const int pi = p->poly_i, pj = p->poly_j;
      if (pi < 1 || pj < 1 || pi > sched::kPijMax || pj > sched::kPijMax || !(pi & 1) ||
          !(pj & 1))
        return SNF_EINVAL;
      if (!finite(p->mu) || !finite(p->xi) || !(p->mu > p->lambda_min) ||
          !(p->mu < p->lambda_max) || !(p->xi > 0.0))
        return SNF_EINVAL;
      const double xs = sched::pij_xstar(pi, pj);
      const double h = p->xi / (2.0 * sched::pij_gamma(p->lambda_min, p->lambda_max, p->mu, xs));
      if (!(h < xs) || !(h < 1.0 - xs)) return SNF_EINVAL;
      break;
    }
    case SNF_SNF_FIXMU3:
    case SNF_SNF_FIXMU5:
    case SNF_PMM3:
    case SNF_PMM5:
      if (prec != SNF_P_FP64) return SNF_EINVAL;
      [[fallthrough]];
    case SNF_MCWEENY:
    case SNF_SNF_FIXMU:
      if (!finite(p->mu) || !finite(p->xi) || !(p->mu > p->lambda_min) ||
          !(p->mu < p->lambda_max) || !(p->xi > 0.0))
        return SNF_EINVAL;
      if (!(p->xi < sched::alg1_gamma(p->lambda_min, p->lambda_max, p->mu))) return SNF_EINVAL;
      break;
  }
  if (p->flags & SNF_FLAG_SUBSPACE_NEWTON) {
    // the correction follows Algorithm 2's sequence between gap edges and refines by the
    // trace rule
    const bool edges = (gap_edges) ||
                       (finite(p->mu) && finite(p->xi) && p->xi > 0.0 &&
                        p->lambda_min <= p->mu - 0.5 * p->xi &&
                        p->mu + 0.5 * p->xi <= p->lambda_max);
    if (!edges || p->n_occ < 0) return SNF_EINVAL;
  }
  if (prec != SNF_P_FP64) {
    if (!finite(p->gap_switch) || p->gap_switch < 0.0 || p->gap_switch > 1.0) return SNF_EINVAL;
    if (!finite(p->lowp_floor) || p->lowp_floor < 0.0 || p->lowp_floor >= 0.5) return SNF_EINVAL;
  }
  return SNF_OK;
}

void init_state(SnfState* s, int64_t n, const snf_params* p, snf_scheme scheme,
                snf_precision prec) {
  memset(s, 0, sizeof(*s));
  s->scheme = scheme;
  s->max_iter = p->max_iter;
  s->mode = prec;
  s->has_nocc = p->n_occ >= 0;
  s->n = n;
  s->n_occ = p->n_occ;
  s->tol = p->tol;
  s->lambda_min = p->lambda_min;
  s->lambda_max = p->lambda_max;
  s->mu = p->mu;
  s->xi = p->xi;
  s->homo = p->homo;
  s->lumo = p->lumo;
  s->gap_switch = p->gap_switch;
  s->lowp_floor = p->lowp_floor > 0.0 ? p->lowp_floor : (prec == SNF_P_BF16_REF64 ? 1e-2 : 1e-4);
  s->pmm_m = scheme_pmm_m(scheme);
  s->xstar = 0.5;
  if (s->pmm_m) {
    sched::pij_binoms(s->pmm_m, s->pmm_m, s->pbin[0]);
    sched::pmm_coeffs(s->pmm_m, s->pr);
  }
  if (scheme_is_pij(scheme)) {
    sched::pij_binoms(p->poly_i, p->poly_j, s->pbin[0]);
    sched::pij_binoms(p->poly_j, p->poly_i, s->pbin[1]);
  }
  if (scheme_is_pij(scheme)) {
    // mu onto the fixed point x* of P_{i,j}; gap edges x* -/+ xi / (2 gamma)
    s->pij_i = p->poly_i;
    s->pij_j = p->poly_j;
    s->xstar = sched::pij_xstar(s->pij_i, s->pij_j);
    s->gamma = sched::pij_gamma(p->lambda_min, p->lambda_max, p->mu, s->xstar);
    const double h = p->xi / (2.0 * s->gamma);
    s->beta = s->xstar - h;
    s->abar = (1.0 - s->xstar) - h;
    s->betabar = 1.0 - s->abar;
    sched::pij_taylor(s->pij_i, s->pij_j, s->xstar, s->pq);
  } else if (scheme == SNF_MCWEENY || scheme == SNF_SNF_FIXMU || s->pmm_m) {
    s->gamma = sched::alg1_gamma(p->lambda_min, p->lambda_max, p->mu);
    s->beta = sched::alg1_beta0(p->xi, s->gamma);
    s->betabar = 1.0 - s->beta;
  } else {
    const bool edges = isfinite(p->homo) && isfinite(p->lumo);
    s->beta = edges ? sched::alg2_f0(p->lumo, p->lambda_min, p->lambda_max) : 0.0;
    s->betabar = edges ? sched::alg2_f0(p->homo, p->lambda_min, p->lambda_max) : 1.0;
  }
  s->phase = kPhaseHigh;
  s->cur = 0;
  s->e_hist[0] = s->e_hist[1] = s->e_hist[2] = INFINITY;
}

void fill_result(const SnfState* s, snf_result* out, snf_log_rec* log, int log_cap) {
  memset(out, 0, sizeof(*out));
  out->status = s->status;
  out->iterations = s->iter;
  out->products = s->products;
  out->products_fp64 = s->products_f64;
  out->products_lowp = s->products_lowp;
  out->idem_err = s->e_last;
  out->trace = s->t1;
  out->trace_err = s->has_nocc ? s->t1 - (double)s->n_occ : 0.0;
  out->alpha_last = s->alpha;
  out->beta_last = s->beta;
  out->betabar_last = s->betabar;
  const double nd = (double)s->n;
  out->flops = (double)s->products * nd * nd * (nd + 1.0);
  out->blocks = 0;
  const int nrec = s->nlog < SNF_LOG_MAX ? s->nlog : SNF_LOG_MAX;
  for (int i = 0; i < nrec && i < SNF_LOG_MAX; ++i)
    out->branch[i] = (uint8_t)(s->log[i].branch < 0 ? 255 : s->log[i].branch);
  if (log && log_cap > 0) {
    const int m = nrec < log_cap ? nrec : log_cap;
    memcpy(log, s->log, (size_t)m * sizeof(snf_log_rec));
  }
}

}  // namespace snf

using namespace snf;

extern "C" {

const char* snf_version(void) { return "0.1.0"; }

const char* snf_strerror(int status) {
  switch (status) {
    case SNF_OK: return "converged";
    case SNF_PENDING: return "pending";
    case SNF_OK_FLOOR: return "stopped at the precision/truncation floor above tol";
    case SNF_EINVAL: return "invalid argument";
    case SNF_ENOMEM: return "out of device memory or over the memory budget";
    case SNF_ENOCONV: return "no convergence within max_iter";
    case SNF_ENONFINITE: return "non-finite value in the iteration";
    case SNF_EMIXED: return "converged to a projector with the wrong occupation";
    case SNF_EDEVICE: return g_err_text[0] ? g_err_text : "HIP runtime error";
    case SNF_ESIZE: return "order above the no-allocation entry point's maximum";
    default: return "unknown status";
  }
}

size_t snf_workspace_bytes(int64_t n, snf_precision precision) {
  if (n <= 0) return 0;
  const int64_t np = round_up(n, kTile);
  const size_t elems = (size_t)np * (size_t)np;
  return elems * (3 * sizeof(double) + 3 * (size_t)lowp_bytes_for(precision)) +
         (size_t)(num_product_tiles(np, 1) + kF0Blocks) * 4 * sizeof(double) + sizeof(SnfState);
}

int snf_release_workspace(void) {
  int dev = 0;
  Workspace* w = workspace_for_current_device(&dev);
  if (!w) return SNF_EDEVICE;
  std::lock_guard<std::mutex> g(w->mu);
  free_buffers(w);
  free_newton(w);
  if (w->partials) (void)hipFree(w->partials);
  w->partials = nullptr;
  w->partial_cap = 0;
  return SNF_OK;
}

}  // extern "C"

namespace snf {
// ---- subspace correction ------------------------------------------------------------------
// After a solve, one Newton step on the occupied subspace of its result D~ that re-references
// F (not in the paper: a low-precision solve followed by refinement by purification leaves a
// rotation of the subspace that no function of the iterate can see).  With G = f_0(F) (the
// map of Algorithm 2) split with respect to D~ into the part that commutes with D~ and the
// coupling V = W + W^T - 2 M (W = G D~, M = D~ G D~), D~ is the projector of G - V, and the
// first-order change of the projector along V is obtained by running Algorithm 2's polynomial
// sequence on X_0 = G - V while carrying its derivative X1 along (X1_0 = V,
// X1 <- c2 (X X1 + X1 X) + c1 X1, X X1 from one product whose transpose is X1 X).  Then
// D = D~ + X1 is refined by trace-correcting FP64 steps to tol.  W, M and the refinement run in
// FP64; the response products in FP32 unless the solve was FP64 (their relative error only
// enters at second order).
constexpr int kNewtonMaxIter = 120;     // steps of the response recurrence at most
constexpr double kNewtonEps = 1e-10;    // ... until max(beta, 1 - beta-bar) <= this

struct NewtonStats {
  int products_f64 = 0, products_lowp = 0, launches = 0;
  double flops = 0.0;
};

static int ensure_newton(Workspace* w, int64_t np, bool lp, int nops) {
  if (np > w->nnp || (lp && !w->nlp_on)) {
    free_newton(w);
    const size_t elems = (size_t)np * (size_t)np;
    for (int i = 0; i < 5; ++i) {
      if (hipMalloc(&w->nx[i], elems * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        free_newton(w);
        return SNF_ENOMEM;
      }
      if (lp && i != 1 && hipMalloc(&w->nlp[i], elems * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        free_newton(w);
        return SNF_ENOMEM;
      }
    }
    w->nnp = np;
    w->nlp_on = lp;
  }
  if (!w->nbufs_dev) SNF_HIP(hipMalloc(&w->nbufs_dev, 4 * sizeof(Buffers)));
  if (nops > w->nops_cap) {
    if (w->nops_dev) (void)hipFree(w->nops_dev);
    w->nops_dev = nullptr;
    w->nops_cap = 0;
    SNF_HIP(hipMalloc(&w->nops_dev, (size_t)nops * sizeof(NewtonOp)));
    w->nops_cap = nops;
  }
  return SNF_OK;
}

// Gap edges of the correction's polynomial sequence: the given bounds, else mu -/+ xi / 2.
static bool newton_edges(const snf_params* p, double* homo, double* lumo) {
  if (isfinite(p->homo) && isfinite(p->lumo) && p->homo < p->lumo) {
    *homo = p->homo;
    *lumo = p->lumo;
  } else if (isfinite(p->mu) && isfinite(p->xi) && p->xi > 0.0) {
    *homo = p->mu - 0.5 * p->xi;
    *lumo = p->mu + 0.5 * p->xi;
  } else {
    return false;
  }
  return p->lambda_min <= *homo && *lumo <= p->lambda_max;
}

// (c2, c1, c0) of Algorithm 2's steps until max(beta, 1 - beta-bar) <= eps (the same FP64
// recurrence as the device schedule).
static void newton_steps(double lmin, double lmax, double homo, double lumo, double eps,
                         std::vector<double>& c) {
#pragma clang fp contract(off)
  double beta = sched::alg2_f0(lumo, lmin, lmax), betabar = sched::alg2_f0(homo, lmin, lmax);
  for (int it = 0; it < kNewtonMaxIter; ++it) {
    const double bound = beta > 1.0 - betabar ? beta : 1.0 - betabar;
    if (bound <= eps) break;
    const bool sq = sched::alg2_square(beta, betabar);
    const double a = sq ? sched::alg2_square_alpha(beta) : sched::alg2_fold_alpha(betabar);
    if (sq) {
      c.push_back((1.0 + a) * (1.0 + a));
      c.push_back(-2.0 * a * (1.0 + a));
      c.push_back(a * a);
      beta = sched::alg2_square_map(beta, a);
      betabar = sched::alg2_square_map(betabar, a);
    } else {
      c.push_back(-((1.0 + a) * (1.0 + a)));
      c.push_back(2.0 * (1.0 + a));
      c.push_back(0.0);
      beta = sched::alg2_fold_map(beta, a);
      betabar = sched::alg2_fold_map(betabar, a);
    }
  }
}

// Runs the correction on the solve's result (buffer x[cur] of the workspace) and leaves in
// w->state the state of the refinement that follows, ready for its step loop (the caller's),
// with the corrected, not yet refined D in buffer x[target], target 0 or 1 and != cur.
static int newton_correct(Workspace* w, const double* F_dev, int64_t n, int64_t ld, int64_t np,
                          const snf_params* p, snf_precision prec, int cur, int target,
                          hipStream_t s, NewtonStats* ns) {
  if ((target != 0 && target != 1) || target == cur) return SNF_EINVAL;
  double homo = 0.0, lumo = 0.0;
  if (!newton_edges(p, &homo, &lumo)) return SNF_EINVAL;
  std::vector<double> c;
  newton_steps(p->lambda_min, p->lambda_max, homo, lumo, kNewtonEps, c);
  const int N = (int)(c.size() / 3);
  const int cp = prec == SNF_P_FP64 ? kPrecF64 : kPrecF32;
  const bool lp = cp == kPrecF32;
  int rc = ensure_newton(w, np, lp, 2 + 2 * N);
  if (rc != SNF_OK) return rc;
  double* const* X = w->nx;
  float* const* L = w->nlp;
  // Buffers tables: 0 f_0 -> G; 1 W = G D~, M = D~ W; 2 / 3 the even / odd iterations
  Buffers t[4];
  memset(t, 0, sizeof(t));
  t[0].x[0] = X[0];
  t[1].x[0] = X[0];
  t[1].x[1] = w->x[cur];
  t[1].x[2] = X[1];
  t[1].x[3] = X[2];
  const int xa[2] = {3, 0}, x1a[2] = {4, 2};       // X and X1 of an even / odd iteration
  for (int par = 0; par < 2; ++par) {
    Buffers& b = t[2 + par];
    b.x[0] = X[xa[par]];
    b.x[1] = X[x1a[par]];
    b.x[2] = X[1];                                   // Z = X X1
    b.x[3] = X[xa[1 - par]];                         // the next X
    b.lp[0] = L[xa[par]];
    b.lp[1] = L[x1a[par]];
    b.lp[3] = L[xa[1 - par]];
  }
  std::vector<NewtonOp> ops;
  ops.push_back(NewtonOp{0, 1, 0, 2, kPrecF64, 0, 1.0, 0.0, 0.0});     // W = G D~
  ops.push_back(NewtonOp{1, 2, 1, 3, kPrecF64, 0, 1.0, 0.0, 0.0});     // M = D~ W
  for (int i = 0; i < N; ++i) {
    ops.push_back(NewtonOp{0, 1, 0, 2, cp, 0, 1.0, 0.0, 0.0});         // Z = X X1
    ops.push_back(NewtonOp{0, 0, 0, 3, cp, lp ? 1 : 0, c[3 * i], c[3 * i + 1], c[3 * i + 2]});
  }
  SNF_HIP(hipMemcpyAsync(w->nbufs_dev, t, sizeof(t), hipMemcpyHostToDevice, s));
  SNF_HIP(hipMemcpyAsync(w->nops_dev, ops.data(), ops.size() * sizeof(NewtonOp),
                         hipMemcpyHostToDevice, s));
  // the product kernels read the state: Algorithm 2's f_0 map, FP32 copies as FP32
  SnfState* sh = w->state_host;
  init_state(sh, n, p, SNF_SNF_VARMU, SNF_P_FP32_REF64);
  sh->homo = homo;
  sh->lumo = lumo;
  sh->cur = 0;
  SNF_HIP(hipMemcpyAsync(w->state, sh, sizeof(SnfState), hipMemcpyHostToDevice, s));
  SNF_HIP(hipStreamSynchronize(s));                  // the host staging is reused below

  const ProductGrid g0 = make_product_grid(np, n, 0, w->num_cus, w->partials, w->split_buf,
                                           kSplitCap, stage_depth_for(prec));
  const ProductGrid g1 = make_product_grid(np, n, 1, w->num_cus, w->partials, w->split_buf,
                                           kSplitCap, stage_depth_for(prec));
  const double nd = (double)n, full = 2.0 * nd * nd * nd, half = nd * nd * (nd + 1.0);
  auto product = [&](int k, int tab, const ProductGrid& g) {
    launch_newton_set(w->state, w->nops_dev, k, s);
    launch_product(ops[k].prec, w->state, w->nbufs_dev + tab, g, s);
    launch_split_fixup(w->state, w->nbufs_dev + tab, g, s);
    if (ops[k].prec == kPrecF64) ns->products_f64 += 1; else ns->products_lowp += 1;
    ns->launches += 1;
  };
  launch_f0(F_dev, n, ld, np, w->state, w->nbufs_dev + 0, -1, w->partials, s);
  product(0, 1, g0);
  product(1, 1, g1);
  ns->flops += full + half;
  launch_newton_split(X[0], X[1], X[2], n, np, X[3], L[3], X[4], L[4], s);
  for (int i = 0; i < N; ++i) {
    const int par = i & 1;
    product(2 + 2 * i, 2 + par, g0);
    launch_newton_sym(X[1], X[x1a[par]], c[3 * i], c[3 * i + 1], n, np, X[x1a[1 - par]],
                      L[x1a[1 - par]], s);
    product(3 + 2 * i, 2 + par, g1);
    ns->flops += full + half;
  }
  SNF_HIP(hipGetLastError());
  // D = D~ + X1 into the refinement's buffer, with its trace sums; then the refinement state
  launch_newton_add(w->x[cur], X[x1a[N & 1]], n, np, w->x[target], w->partials, s);
  init_state(sh, n, p, p->n_occ >= 0 ? SNF_SP2_TRACE : SNF_MCWEENY, SNF_P_FP32_REF64);
  sh->phase = kPhaseRefine;
  sh->cur = target;
  SNF_HIP(hipMemcpyAsync(w->state, sh, sizeof(SnfState), hipMemcpyHostToDevice, s));
  launch_schedule(w->state, w->partials, kF0Blocks, 1, s);
  SNF_HIP(hipGetLastError());
  SNF_HIP(hipStreamSynchronize(s));
  return SNF_OK;
}

static int purify_dense_body(const double* F_dev, int64_t n, int64_t ld,
                             const snf_params* params, snf_scheme scheme,
                             snf_precision precision, double* D_dev, snf_result* out,
                             snf_log_rec* log, int32_t log_cap, void* stream) {
  int rc = validate(n, params, scheme, precision);
  if (rc == SNF_OK && (!F_dev || !D_dev || ld < n || (const void*)F_dev == (const void*)D_dev))
    rc = SNF_EINVAL;
  if (rc != SNF_OK) {
    out->status = rc;
    return rc;
  }
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  Workspace* w = workspace_for_current_device(&dev);
  if (!w) {
    out->status = SNF_EDEVICE;
    return SNF_EDEVICE;
  }
  std::lock_guard<std::mutex> guard(w->mu);
  const int64_t np = round_up(n, kTile);
  const int sym = 1;
  const int tiles = num_product_tiles(np, sym);
  // (the subspace correction's full-grid products need a partial slot per tile of the grid)
  const int slot_tiles = (params->flags & SNF_FLAG_SUBSPACE_NEWTON) ? num_product_tiles(np, 0)
                                                                     : tiles;
  rc = ensure_workspace(w, np, lowp_bytes_for(precision), slot_tiles + 16 * kSplitCap,
                        (scheme_pmm_m(scheme) || scheme_is_pij(scheme)) ? 4 : 3);
  if (rc != SNF_OK) {
    out->status = rc;
    return rc;
  }
  const ProductGrid grid = make_product_grid(np, n, sym, w->num_cus, w->partials, w->split_buf,
                                             kSplitCap, stage_depth_for(precision));
  // A workspace of larger order is used with this call's np: the kernels index rows with
  // np, so every buffer just needs np*np elements.
  init_state(w->state_host, n, params, scheme, precision);
  const bool time_products = (params->flags & SNF_FLAG_TIME_PRODUCTS) != 0;
  const int per_it = products_per_iteration(scheme, params->poly_i, params->poly_j);
  const int max_steps = (params->max_iter + 1) * per_it + 1;
  if (time_products && (int)w->prod_ev.size() < 2 * max_steps) {
    const size_t old = w->prod_ev.size();
    w->prod_ev.resize(2 * max_steps);
    for (size_t i = old; i < w->prod_ev.size(); ++i) SNF_HIP(hipEventCreate(&w->prod_ev[i]));
  }

  rc = upload_buffers(w, s);
  if (rc != SNF_OK) return out->status = rc;
  SNF_HIP(hipMemcpyAsync(w->state, w->state_host, sizeof(SnfState), hipMemcpyHostToDevice, s));
  SNF_HIP(hipEventRecord(w->ev[0], s));
  launch_f0(F_dev, n, ld, np, w->state, w->bufs_dev, lowp_kind_for(precision), w->partials, s);
  launch_schedule(w->state, w->partials, kF0Blocks, 1, s);
  SNF_HIP(hipGetLastError());

  // Launch-ahead loop: chunks of `chunk` steps, two chunks in flight.
  const int chunk = np >= 2048 ? 2 : (np >= 1024 ? 4 : 8);
  const bool lowp = precision != SNF_P_FP64;
  const bool pij = scheme_is_pij(scheme);
  // small orders in FP64: 32x32 tiles with the k range split inside the workgroup
  const bool small = !lowp && !pij && np <= kSmallMaxNp;
  const SmallGrid sgrid = make_small_grid(np, n, w->partials);
  int enq = 0, chunks = 0, checked = 0;
  int ev_used = 0;
  bool stopped = false;
  volatile int32_t* flags = w->flags_host;
  auto enqueue_chunk = [&]() -> int {
    for (int k = 0; k < chunk && enq < max_steps; ++k, ++enq) {
      if (time_products) SNF_HIP(hipEventRecord(w->prod_ev[ev_used], s));
      if (small) {
        launch_product_small(w->state, w->bufs_dev, sgrid, s);
      } else {
        launch_product(kPrecF64, w->state, w->bufs_dev, grid, s);
        if (pij) launch_product_dual(w->state, w->bufs_dev, grid, s);
        if (lowp) launch_product(lowp_kind_for(precision), w->state, w->bufs_dev, grid, s);
        launch_split_fixup(w->state, w->bufs_dev, grid, s);
      }
      if (time_products) SNF_HIP(hipEventRecord(w->prod_ev[ev_used + 1], s));
      if (time_products) ev_used += 2;
      launch_schedule(w->state, w->partials, small ? sgrid.tiles : grid.partial_count, 0, s);
    }
    SNF_HIP(hipGetLastError());
    SNF_HIP(hipMemcpyAsync((void*)(flags + (chunks & 1)), &w->state->stop, sizeof(int32_t),
                           hipMemcpyDeviceToHost, s));
    SNF_HIP(hipEventRecord(w->ev[2 + (chunks & 1)], s));
    ++chunks;
    return SNF_OK;
  };
  // the smallest orders run the whole step loop in one cooperative launch (not the P_{m,m}
  // schemes: measured no faster inside that launch, P_{5,5} with alpha = 1 slower)
  bool persistent = false;
  if (small && np <= kPersistMaxNp && !scheme_pmm_m(scheme)) {
    if (time_products) SNF_HIP(hipEventRecord(w->prod_ev[0], s));
    persistent = launch_solve_small(w->state, w->bufs_dev, sgrid, w->partials, max_steps, s) == 0;
    if (!persistent) (void)hipGetLastError();   // not co-resident: the launch-per-step path
    else if (time_products) SNF_HIP(hipEventRecord(w->prod_ev[1], s));
    if (persistent) {
      ev_used = 2;
      stopped = true;
    }
  }
  if (!persistent) {
    rc = enqueue_chunk();
    if (rc != SNF_OK) return out->status = rc;
  }
  while (!stopped && enq < max_steps) {
    rc = enqueue_chunk();
    if (rc != SNF_OK) return out->status = rc;
    // wait for the older in-flight chunk and look at its stop flag
    SNF_HIP(hipEventSynchronize(w->ev[2 + (checked & 1)]));
    stopped = flags[checked & 1] != 0;
    ++checked;
  }
  // subspace correction of the solve's result, then its FP64 refinement
  std::unique_ptr<SnfState> main_st;
  NewtonStats ns;
  if (params->flags & SNF_FLAG_SUBSPACE_NEWTON) {
    SNF_HIP(hipMemcpyAsync(w->state_host, w->state, sizeof(SnfState), hipMemcpyDeviceToHost, s));
    SNF_HIP(hipStreamSynchronize(s));
    const int st0 = w->state_host->stop ? w->state_host->status : SNF_ENOCONV;
    if (st0 == SNF_OK || st0 == SNF_OK_FLOOR) {
      main_st.reset(new SnfState(*w->state_host));
      // the refinement ping-pongs between buffers 0 and 1 (its steps write buffer 1 - cur), so
      // the corrected D goes to the one of them that does not hold the solve's result
      const int target = main_st->cur == 0 ? 1 : 0;
      rc = newton_correct(w, F_dev, n, ld, np, params, precision, main_st->cur, target, s, &ns);
      if (rc != SNF_OK) return rc;
      bool rstop = false;
      for (int renq = 0; !rstop && renq < params->max_iter + 1;) {
        for (int k = 0; k < chunk && renq < params->max_iter + 1; ++k, ++renq) {
          launch_product(kPrecF64, w->state, w->bufs_dev, grid, s);
          launch_split_fixup(w->state, w->bufs_dev, grid, s);
          launch_schedule(w->state, w->partials, grid.partial_count, 0, s);
        }
        SNF_HIP(hipGetLastError());
        SNF_HIP(hipMemcpyAsync((void*)flags, &w->state->stop, sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
        SNF_HIP(hipStreamSynchronize(s));
        rstop = flags[0] != 0;
      }
    }
  }
  launch_copy_out(w->state, w->bufs_dev, n, np, D_dev, ld, s);
  SNF_HIP(hipGetLastError());
  SNF_HIP(hipEventRecord(w->ev[1], s));
  SNF_HIP(hipMemcpyAsync(w->state_host, w->state, sizeof(SnfState), hipMemcpyDeviceToHost, s));
  SNF_HIP(hipStreamSynchronize(s));

  const SnfState* st = main_st ? main_st.get() : w->state_host;
  int status = st->stop ? st->status : SNF_ENOCONV;
  fill_result(st, out, log, log_cap);
  if (main_st) {
    // decisions and log are the solve's; counts add the correction and the refinement; the
    // idempotency, trace and status are the refinement's
    const SnfState* r = w->state_host;
    status = r->stop ? r->status : SNF_ENOCONV;
    const double nd = (double)n;
    out->products += ns.launches + r->products;
    out->products_fp64 += ns.products_f64 + r->products_f64;
    out->products_lowp += ns.products_lowp + r->products_lowp;
    out->products_newton = ns.launches + r->products;
    out->idem_err = r->e_last;
    out->trace = r->t1;
    out->trace_err = r->has_nocc ? r->t1 - (double)r->n_occ : 0.0;
    out->flops += ns.flops + (double)r->products * nd * nd * (nd + 1.0);
  }
  out->status = status;
  float ms = 0.f;
  SNF_HIP(hipEventElapsedTime(&ms, w->ev[0], w->ev[1]));
  out->device_ms = ms;
  if (time_products && persistent) {
    // one launch ran every product and every schedule step
    float m = 0.f;
    SNF_HIP(hipEventElapsedTime(&m, w->prod_ev[0], w->prod_ev[1]));
    out->product_ms = m;
  } else if (time_products) {
    // step k of the loop ran the k-th product; steps after the stop were empty launches
    double tot = 0.0;
    const int real = st->products;
    for (int k = 0; k < real && 2 * k + 1 < ev_used; ++k) {
      float m = 0.f;
      SNF_HIP(hipEventElapsedTime(&m, w->prod_ev[2 * k], w->prod_ev[2 * k + 1]));
      tot += m;
    }
    out->product_ms = tot;
  }
  return status;
}
}  // namespace snf

extern "C" {

int snf_purify_dense(const double* F_dev, int64_t n, int64_t ld, const snf_params* params,
                     snf_scheme scheme, snf_precision precision, double* D_dev,
                     snf_result* out, snf_log_rec* log, int32_t log_cap, void* stream) {
  if (!out) return SNF_EINVAL;
  memset(out, 0, sizeof(*out));
  // every return path, HIP errors included, leaves its code in out->status
  const int rc = purify_dense_body(F_dev, n, ld, params, scheme, precision, D_dev, out, log,
                                   log_cap, stream);
  out->status = rc;
  return rc;
}

int snf_shutdown(void) {
  dense_release_all_devices();
  bsr_release_all_devices();
  bounds_release_all_devices();
  return SNF_OK;
}

int snf_step_dense(const double* A_dev, const double* B_dev, int64_t n, int64_t ld, double c2,
                   double c1, double c0, snf_precision precision, double* Y_dev, double* sums,
                   double* kernel_ms, void* stream) {
  if (!A_dev || !B_dev || !Y_dev || !sums || n <= 0 || ld < n) return SNF_EINVAL;
  if (precision != SNF_P_FP64 && precision != SNF_P_FP32 && precision != SNF_P_BF16_REF64)
    return SNF_EINVAL;
  if ((const void*)Y_dev == (const void*)A_dev || (const void*)Y_dev == (const void*)B_dev)
    return SNF_EINVAL;
  if (!isfinite(c2) || !isfinite(c1) || !isfinite(c0)) return SNF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  Workspace* w = workspace_for_current_device(&dev);
  if (!w) return SNF_EDEVICE;
  std::lock_guard<std::mutex> guard(w->mu);
  const int64_t np = round_up(n, kTile);
  // A.A is symmetric: the upper triangle of tiles, mirrored.  A.B of two symmetric operands
  // that need not commute is not: every tile, no mirror.
  const int sym = (const void*)A_dev == (const void*)B_dev ? 1 : 0;
  const int tiles = num_product_tiles(np, sym);
  int rc = ensure_workspace(w, np, lowp_bytes_for(precision), tiles + 16 * kSplitCap);
  if (rc != SNF_OK) return rc;
  const ProductGrid grid = make_product_grid(np, n, sym, w->num_cus, w->partials, w->split_buf,
                                             kSplitCap, stage_depth_for(precision));
  const int lk = lowp_kind_for(precision);
  rc = upload_buffers(w, s);
  if (rc != SNF_OK) return rc;
  SnfState* sh = w->state_host;
  memset(sh, 0, sizeof(*sh));
  sh->mode = precision;
  sh->n = n;
  sh->prec = lk < 0 ? kPrecF64 : lk;
  sh->c2 = c2;
  sh->c1 = c1;
  sh->c0 = c0;
  sh->kind = kKindSquare;
  sh->want_e = 1;
  sh->ia = 0;
  sh->ib = 1;
  sh->ix = 0;
  sh->io = 2;
  sh->write_lowp = 0;
  SNF_HIP(hipMemcpyAsync(w->state, sh, sizeof(SnfState), hipMemcpyHostToDevice, s));
  launch_pad_copy(A_dev, n, ld, w->x[0], np, w->lp[0], lk, s);
  launch_pad_copy(B_dev, n, ld, w->x[1], np, w->lp[1], lk, s);
  SNF_HIP(hipEventRecord(w->ev[0], s));
  launch_product(sh->prec, w->state, w->bufs_dev, grid, s);
  launch_split_fixup(w->state, w->bufs_dev, grid, s);
  SNF_HIP(hipEventRecord(w->ev[1], s));
  launch_sum_partials(w->partials, grid.partial_count, w->sums_dev, s);
  launch_unpad_copy(w->x[2], np, n, Y_dev, ld, s);
  SNF_HIP(hipGetLastError());
  SNF_HIP(hipMemcpyAsync(w->sums_host, w->sums_dev, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  SNF_HIP(hipStreamSynchronize(s));
  sums[0] = w->sums_host[0];
  sums[1] = w->sums_host[1];
  sums[2] = w->sums_host[2];
  if (kernel_ms) {
    float ms = 0.f;
    SNF_HIP(hipEventElapsedTime(&ms, w->ev[0], w->ev[1]));
    *kernel_ms = ms;
  }
  return SNF_OK;
}

}  // extern "C"
