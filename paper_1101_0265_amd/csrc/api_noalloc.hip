// snf_purify_dense_noalloc: the dense purification of snf_purify_dense for callers that cannot
// allocate (code under stream capture, tight serving loops, harnesses that forbid hipMalloc).
//
// Every byte of device memory beyond the caller's F and D comes from `scratch`, a file-scope
// device array of fixed size: the FP64 iterate buffers, the per-tile partial sums, the scalar
// state and the buffer table.  Its device address is taken once per device with
// hipGetSymbolAddress (the array's name in host code is a host-side stand-in, not a device
// address) and kept; every kernel argument and copy uses that address.  Host staging (the
// scalar state, the stop flag) lives in static host arrays, and the step loop reads the stop
// flag with a synchronous copy instead of pinned memory and events, so the call makes no
// allocation of any kind.  The kernels are those of snf_purify_dense (the small-order FP64
// product, its cooperative whole-solve variant, f_0, the schedule and the copy-out), launched
// in the same order on the same decomposition, so the results are the same bit for bit.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <string.h>

#include <mutex>

#include "schedule_math.h"
#include "snf_internal.h"

namespace snf {
namespace na {

constexpr int64_t kNaMaxNp = kSmallMaxNp;               // 896: the small-order FP64 path
constexpr int kNaPartialSlots = kF0Blocks;              // >= f_0's blocks and 2 x 406 tiles
constexpr size_t kNaMatrix = (size_t)kNaMaxNp * kNaMaxNp;

// Layout of the scratch array (offsets in doubles, each a multiple of 32, i.e. 256 bytes).
constexpr size_t align32(size_t v) { return (v + 31) / 32 * 32; }
constexpr size_t kOffState = 0;
constexpr size_t kOffBufs = align32(kOffState + (sizeof(SnfState) + 7) / 8);
constexpr size_t kOffClock = align32(kOffBufs + (sizeof(Buffers) + 7) / 8);
constexpr size_t kOffPartials = align32(kOffClock + 2);
constexpr size_t kOffX = align32(kOffPartials + (size_t)kNaPartialSlots * 4);
constexpr size_t kScratchDoubles = SNF_NOALLOC_SCRATCH_BYTES / 8;
static_assert(kOffX + 4 * kNaMatrix <= kScratchDoubles,
              "the layout must fit in SNF_NOALLOC_SCRATCH_BYTES");
static_assert(kNaMaxNp == SNF_NOALLOC_MAX_N, "SNF_NOALLOC_MAX_N is the padded-order limit");

}  // namespace na
}  // namespace snf

// The scratch memory of snf_purify_dense_noalloc; each device holds its own copy until the
// process ends.
static __device__ __align__(256) double scratch[snf::na::kScratchDoubles];

namespace snf {
namespace {
using namespace na;

std::mutex g_na_mu[64];
double* g_na_ptr[64];                 // device address of scratch, per device
SnfState g_na_state[64];              // host staging of the scalar state, per device
int32_t g_na_flag[64];

__global__ void na_clock_kernel(unsigned long long* out) {
  if (threadIdx.x == 0) *out = wall_clock64();
}

#define NA_HIP(call)                                       \
  do {                                                     \
    hipError_t _e = (call);                                \
    if (_e != hipSuccess) return record_hip_error(_e, #call); \
  } while (0)

int na_body(const double* F_dev, int64_t n, int64_t ld, const snf_params* params,
            snf_scheme scheme, double* D_dev, snf_result* out, snf_log_rec* log,
            int32_t log_cap, hipStream_t s, int dev) {
  double* base = g_na_ptr[dev];
  if (!base) {
    // first call on this device: the device address of this device's copy of the array
    void* p = nullptr;
    NA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return SNF_EDEVICE;
    base = (double*)p;
    g_na_ptr[dev] = base;
  }
  const int64_t np = (n + kTile - 1) / kTile * kTile;
  SnfState* st = (SnfState*)(base + kOffState);
  Buffers* bufs_dev = (Buffers*)(base + kOffBufs);
  unsigned long long* clk = (unsigned long long*)(base + kOffClock);
  double* partials = base + kOffPartials;
  // The iterate buffers hold kNaMaxNp^2 values each; the kernels index rows with this call's
  // np, and every entry of an np x np buffer is written before it is read (f_0 writes all of
  // X_0 including its zero padding, every product's epilogue all of its output), so nothing
  // left by an earlier call needs clearing.
  Buffers b;
  for (int i = 0; i < 4; ++i) {
    b.x[i] = base + kOffX + (size_t)i * kNaMatrix;
    b.lp[i] = nullptr;
  }
  SnfState* sh = &g_na_state[dev];
  init_state(sh, n, params, scheme, SNF_P_FP64);
  NA_HIP(hipMemcpyAsync(bufs_dev, &b, sizeof(b), hipMemcpyHostToDevice, s));
  NA_HIP(hipMemcpyAsync(st, sh, sizeof(SnfState), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(na_clock_kernel, dim3(1), dim3(64), 0, s, clk);
  launch_f0(F_dev, n, ld, np, st, bufs_dev, -1, partials, s);
  launch_schedule(st, partials, kF0Blocks, 1, s);
  NA_HIP(hipGetLastError());

  const int per_it = products_per_iteration(scheme, params->poly_i, params->poly_j);
  const int max_steps = (params->max_iter + 1) * per_it + 1;
  const SmallGrid sgrid = make_small_grid(np, n, partials);
  bool stopped = false;
  if (np <= kPersistMaxNp && !scheme_pmm_m(scheme)) {
    // the whole step loop in one cooperative launch, as snf_purify_dense does
    stopped = launch_solve_small(st, bufs_dev, sgrid, partials, max_steps, s) == 0;
    if (!stopped) (void)hipGetLastError();   // not co-resident: a launch per step below
  }
  const int chunk = np >= 1024 ? 4 : 8;
  int enq = 0;
  while (!stopped && enq < max_steps) {
    for (int k = 0; k < chunk && enq < max_steps; ++k, ++enq) {
      launch_product_small(st, bufs_dev, sgrid, s);
      launch_schedule(st, partials, sgrid.tiles, 0, s);
    }
    NA_HIP(hipGetLastError());
    // a synchronous read of the stop flag (no pinned staging, no events)
    NA_HIP(hipMemcpyAsync(&g_na_flag[dev], &st->stop, sizeof(int32_t), hipMemcpyDeviceToHost,
                          s));
    NA_HIP(hipStreamSynchronize(s));
    stopped = g_na_flag[dev] != 0;
  }
  launch_copy_out(st, bufs_dev, n, np, D_dev, ld, s);
  hipLaunchKernelGGL(na_clock_kernel, dim3(1), dim3(64), 0, s, clk + 1);
  NA_HIP(hipGetLastError());
  NA_HIP(hipMemcpyAsync(sh, st, sizeof(SnfState), hipMemcpyDeviceToHost, s));
  unsigned long long ticks[2] = {0, 0};
  NA_HIP(hipMemcpyAsync(ticks, clk, sizeof(ticks), hipMemcpyDeviceToHost, s));
  NA_HIP(hipStreamSynchronize(s));
  const int status = sh->stop ? sh->status : SNF_ENOCONV;
  fill_result(sh, out, log, log_cap);
  out->status = status;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
    out->device_ms = (double)(ticks[1] - ticks[0]) / (double)khz;
  return status;
}

}  // namespace
}  // namespace snf

using namespace snf;

extern "C" {

int snf_purify_dense_noalloc(const double* F_dev, int64_t n, int64_t ld,
                             const snf_params* params, snf_scheme scheme,
                             snf_precision precision, double* D_dev, snf_result* out,
                             snf_log_rec* log, int32_t log_cap, void* stream) {
  if (!out) return SNF_EINVAL;
  memset(out, 0, sizeof(*out));
  int rc = validate(n, params, scheme, precision);
  if (rc == SNF_OK && (!F_dev || !D_dev || ld < n || (const void*)F_dev == (const void*)D_dev))
    rc = SNF_EINVAL;
  if (rc == SNF_OK && (precision != SNF_P_FP64 || scheme_is_pij(scheme))) rc = SNF_EINVAL;
  if (rc == SNF_OK && (n + kTile - 1) / kTile * kTile > kNaMaxNp) rc = SNF_ESIZE;
  if (rc != SNF_OK) {
    out->status = rc;
    return rc;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    out->status = SNF_EDEVICE;
    return SNF_EDEVICE;
  }
  std::lock_guard<std::mutex> guard(g_na_mu[dev]);
  rc = na_body(F_dev, n, ld, params, scheme, D_dev, out, log, log_cap, (hipStream_t)stream,
               dev);
  out->status = rc;
  return rc;
}

}  // extern "C"
