// Serving loop: continuous batching of many independent dense purifications on one GPU.
//
// A scheduler thread owns three HIP streams and a device arena (the HBM budget).  Each loop
// turn
//   1. launches one grouped step over every started request: the product tiles of all of
//      them in one launch per precision variant (FP64 and low precision on two streams),
//      then every request's schedule, then a gather of their stop flags;
//   2. while that step runs, enqueues on the third stream the retirement of the requests
//      whose stop flag came back from the previous step (D and the result to the host,
//      arena and slot released) and admits queued requests (FIFO) while a slot is free and
//      the arena can hold the request's workspace (F in, f_0 and the initial schedule);
//   3. waits for the step and reads its stop flags.
// Nothing is allocated on the device while serving (the arena is sub-allocated), so a
// finishing request never waits on a device-wide free.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.h"
#include "snf_internal.h"

namespace snf {

using Clock = std::chrono::steady_clock;

struct ServeRequest {
  uint64_t ticket = 0;
  int64_t n = 0, np = 0;
  snf_params params;
  snf_scheme scheme;
  snf_precision prec;
  bool device_io = false;        // F and D are device buffers of the caller
  const double* F_dev = nullptr;
  double* D_dev = nullptr;
  double* D_host = nullptr;
  std::vector<double> F_pageable;   // host F when no pinned staging was free at submit
  bool pinned = false;              // pinned block [F | D | state] (host) or [state] (device)
  size_t pin_off = 0, pin_bytes = 0;
  double* F_pin = nullptr;
  double* D_pin = nullptr;
  SnfState* st_pin = nullptr;
  // submitted; admitted (slot and memory taken); finished (the scheduler read the stop flag
  // of its last step); done (result complete on the host)
  Clock::time_point t_submit, t_admit, t_finish, t_done;
  int slot = -1;
  size_t off = 0, bytes = 0;
  hipEvent_t ev = nullptr;
  bool started = false;     // admission work enqueued: takes part in the next grouped step
  bool finished = false;    // its stop flag came back: retired behind the next step
  int result_buf = 0;       // the iterate buffer holding D (from the stop flag)
  int status = SNF_PENDING;
  snf_result result;
};

struct RequestLayout {   // byte offsets of one request's workspace inside its arena block
  size_t x[4], lp[4], partials, total;
  int nbuf;              // iterate-sized buffers: 3, or 4 for the P_{m,m} and P_{i,j} schemes
};

// buffers a request of this scheme needs: X (two, ping-pong) and an intermediate (Algorithm
// 1's S2, and F at admission); the P_{m,m} and P_{i,j} iterations keep W and two Horner
// levels beside X
static int request_buffers(snf_scheme scheme) {
  return (scheme_pmm_m(scheme) || scheme_is_pij(scheme)) ? 4 : 3;
}

static RequestLayout request_layout(int64_t n, snf_precision prec, int nbuf = 3) {
  RequestLayout L;
  L.nbuf = nbuf;
  const int64_t np = (n + kTile - 1) / kTile * kTile;
  const size_t mat = (size_t)np * np * sizeof(double);
  const size_t lpb = (size_t)np * np * lowp_bytes_for(prec);
  const int tiles = num_product_tiles(np, 1);
  const size_t slots = (size_t)(tiles > kF0Blocks ? tiles : kF0Blocks);
  size_t o = 0;
  for (int i = 0; i < 4; ++i) L.x[i] = L.lp[i] = 0;
  for (int i = 0; i < nbuf; ++i) {
    L.x[i] = o;
    o += (mat + 255) & ~(size_t)255;
  }
  for (int i = 0; i < nbuf; ++i) {
    L.lp[i] = o;
    o += (lpb + 255) & ~(size_t)255;
  }
  L.partials = o;
  o += slots * 4 * sizeof(double);
  L.total = (o + 255) & ~(size_t)255;
  return L;
}

static size_t pinned_bytes(const ServeRequest* r) {
  const size_t st = (sizeof(SnfState) + 255) & ~(size_t)255;
  if (r->device_io) return st;
  const size_t mat = ((size_t)r->n * r->n * sizeof(double) + 255) & ~(size_t)255;
  return 2 * mat + st;
}

}  // namespace snf

using namespace snf;

struct snf_server {
  int device = 0;
  hipStream_t stream = nullptr;
  // second stream of a step: the FP32 product launch runs beside the FP64 one (different
  // requests), joined by events before the schedule
  hipStream_t stream2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipStream_t stream3 = nullptr;      // admissions and retirements, beside the steps
  hipEvent_t ev_adm = nullptr;        // recorded on stream3 behind the latest admissions
  hipEvent_t ev_step = nullptr;       // recorded behind a step's stop flags
  size_t budget = 0;
  int max_slots = 0;
  char* arena_base = nullptr;     // device arena (the HBM budget)
  Arena arena;
  char* pin_base = nullptr;       // pinned host staging arena
  size_t pin_size = 0;
  Arena pin_arena;
  // device tables, one entry per slot
  SnfState* states = nullptr;
  Buffers* bufs = nullptr;
  SlotDesc* slots = nullptr;
  int* index_dev = nullptr;      // [2 * max_slots + 1]: active slots, then tile offsets
  int32_t* stop_dev = nullptr;   // [max_slots]
  // pinned host staging of the tables
  SnfState* state_stage = nullptr;   // [max_slots]
  Buffers* bufs_stage = nullptr;     // [max_slots]
  SlotDesc* desc_stage = nullptr;    // [max_slots]
  int* index_stage = nullptr;        // [2 * max_slots + 1]
  int32_t* stop_stage = nullptr;     // [max_slots]
  // host bookkeeping
  std::thread thread, finisher;
  std::mutex mu;
  std::condition_variable cv, fin_cv;
  std::deque<ServeRequest*> pending;
  std::deque<ServeRequest*> finishing;
  std::vector<ServeRequest*> slot_req;
  std::unordered_map<uint64_t, ServeRequest*> by_ticket;
  std::vector<hipEvent_t> free_events;
  uint64_t next_ticket = 1;
  bool stopping = false, sched_done = false;
  int sticky_error = SNF_OK;
  Clock::time_point t_create;      // origin of snf_serve_timeline
};

namespace snf {

static void fail_all_locked(snf_server* sv, int rc) {
  sv->sticky_error = rc;
  auto fail = [&](ServeRequest* r) {
    r->status = rc;
    r->result.status = rc;
    r->t_done = Clock::now();
    if (r->t_finish < r->t_admit) r->t_finish = r->t_done;
  };
  for (ServeRequest* r : sv->slot_req)
    if (r) fail(r);
  std::fill(sv->slot_req.begin(), sv->slot_req.end(), nullptr);
  for (ServeRequest* r : sv->pending) fail(r);
  sv->pending.clear();
}

// Pinned staging for a request (caller holds the lock).  Host mode copies F in here.
static bool take_pinned_locked(snf_server* sv, ServeRequest* r) {
  size_t off = 0;
  const size_t bytes = pinned_bytes(r);
  if (!sv->pin_base || !sv->pin_arena.alloc(bytes, &off)) return false;
  r->pinned = true;
  r->pin_off = off;
  r->pin_bytes = bytes;
  char* b = sv->pin_base + off;
  if (r->device_io) {
    r->st_pin = (SnfState*)b;
  } else {
    const size_t mat = ((size_t)r->n * r->n * sizeof(double) + 255) & ~(size_t)255;
    r->F_pin = (double*)b;
    r->D_pin = (double*)(b + mat);
    r->st_pin = (SnfState*)(b + 2 * mat);
  }
  return true;
}

static hipEvent_t take_event_locked(snf_server* sv) {
  if (!sv->free_events.empty()) {
    hipEvent_t e = sv->free_events.back();
    sv->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

#define SV_HIP(call)                              \
  do {                                            \
    if ((call) != hipSuccess) return SNF_EDEVICE; \
  } while (0)

// Admission of one request into slot r->slot: tables, F into x[2] (row stride n), f_0 and
// the initial schedule -- all stream-ordered, no host waits.
static int start_request(snf_server* sv, ServeRequest* r, hipStream_t s) {
  const int k = r->slot;
  const RequestLayout L = request_layout(r->n, r->prec, request_buffers(r->scheme));
  char* base = sv->arena_base + r->off;
  Buffers& b = sv->bufs_stage[k];
  for (int i = 0; i < 4; ++i) {
    const bool have = i < L.nbuf;
    b.x[i] = have ? (double*)(base + L.x[i]) : nullptr;
    b.lp[i] = have && lowp_bytes_for(r->prec) ? (void*)(base + L.lp[i]) : nullptr;
  }
  SlotDesc& d = sv->desc_stage[k];
  d.st = sv->states + k;
  d.bufs = sv->bufs + k;
  d.partials = (double*)(base + L.partials);
  d.np = r->np;
  d.n = r->n;
  init_state(&sv->state_stage[k], r->n, &r->params, r->scheme, r->prec);
  SV_HIP(hipMemcpyAsync(sv->bufs + k, &b, sizeof(Buffers), hipMemcpyHostToDevice, s));
  SV_HIP(hipMemcpyAsync(sv->slots + k, &d, sizeof(SlotDesc), hipMemcpyHostToDevice, s));
  SV_HIP(hipMemcpyAsync(sv->states + k, &sv->state_stage[k], sizeof(SnfState),
                        hipMemcpyHostToDevice, s));
  const size_t fbytes = (size_t)r->n * r->n * sizeof(double);
  if (r->device_io)
    SV_HIP(hipMemcpyAsync(b.x[2], r->F_dev, fbytes, hipMemcpyDeviceToDevice, s));
  else
    SV_HIP(hipMemcpyAsync(b.x[2], r->F_pin, fbytes, hipMemcpyHostToDevice, s));
  launch_f0(b.x[2], r->n, r->n, r->np, sv->states + k, sv->bufs + k, lowp_kind_for(r->prec),
            d.partials, s);
  launch_schedule(sv->states + k, d.partials, kF0Blocks, 1, s);
  SV_HIP(hipGetLastError());
  return SNF_OK;
}

// Retirement of a finished request: D out (device copy, or through x[2] to the pinned D
// staging), the state to pinned memory, an event behind them; the finisher thread completes
// it on the host.  Stream order keeps a later admission into the same memory behind these.
static int retire_request(snf_server* sv, ServeRequest* r, hipStream_t s) {
  const int k = r->slot;
  const Buffers& b = sv->bufs_stage[k];
  if (r->device_io) {
    launch_copy_out(sv->states + k, sv->bufs + k, r->n, r->np, r->D_dev, r->n, s);
  } else {
    // D leaves through an iterate buffer other than the one holding it (x[2] unless D is
    // there: a P_{m,m} or P_{i,j} iteration rotates its result over all four)
    double* stage = b.x[r->result_buf == 2 ? 0 : 2];
    launch_copy_out(sv->states + k, sv->bufs + k, r->n, r->np, stage, r->n, s);
    SV_HIP(hipMemcpyAsync(r->D_pin, stage, (size_t)r->n * r->n * sizeof(double),
                          hipMemcpyDeviceToHost, s));
  }
  SV_HIP(hipMemcpyAsync(r->st_pin, sv->states + k, sizeof(SnfState), hipMemcpyDeviceToHost, s));
  SV_HIP(hipEventRecord(r->ev, s));
  SV_HIP(hipGetLastError());
  return SNF_OK;
}

static void finisher(snf_server* sv) {
  (void)hipSetDevice(sv->device);
  for (;;) {
    ServeRequest* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->fin_cv.wait(lk, [&] { return !sv->finishing.empty() || sv->sched_done; });
      if (sv->finishing.empty()) return;
      r = sv->finishing.front();
      sv->finishing.pop_front();
    }
    int status = SNF_EDEVICE;
    snf_result res;
    memset(&res, 0, sizeof(res));
    if (hipEventSynchronize(r->ev) == hipSuccess) {
      if (!r->device_io) memcpy(r->D_host, r->D_pin, (size_t)r->n * r->n * sizeof(double));
      fill_result(r->st_pin, &res, nullptr, 0);
      status = r->st_pin->stop ? r->st_pin->status : SNF_ENOCONV;
    }
    res.status = status;
    std::lock_guard<std::mutex> lk(sv->mu);
    r->result = res;
    r->status = status;
    r->t_done = Clock::now();
    sv->pin_arena.release(r->pin_off, r->pin_bytes);
    r->pinned = false;
    sv->free_events.push_back(r->ev);
    r->ev = nullptr;
    sv->cv.notify_all();   // pinned staging freed: admission may proceed
  }
}

// One iteration: launch the grouped step over the requests started earlier; while it runs,
// enqueue on a third stream the retirement of the requests whose stop flag came back from the
// previous step and the admission of pending requests into free slots (none of them is in
// the step, so both overlap its products); then wait for the step and read its stop flags.
// The next step waits for the admissions (event).  A request joins the step after the one
// during which it was admitted and is copied out during the step after its stop flag.
static void scheduler(snf_server* sv) {
  (void)hipSetDevice(sv->device);
  std::vector<ServeRequest*> admitted, finished;
  std::vector<int> active;
  bool adm_pending = false;
  for (;;) {
    int rc = SNF_OK;
    hipStream_t s = sv->stream, s3 = sv->stream3;
    if (adm_pending) {   // the step below reads the admitted requests' state and X_0
      if (hipStreamWaitEvent(s, sv->ev_adm, 0) != hipSuccess) rc = SNF_EDEVICE;
      adm_pending = false;
    }
    // 1. grouped step over every started, unfinished request
    active.clear();
    int prec_mask = 1 << kPrecF64;
    for (int i = 0; i < sv->max_slots; ++i) {   // slot_req is written by this thread only
      const ServeRequest* r = sv->slot_req[i];
      if (r && r->started && !r->finished) {
        active.push_back(i);
        if (r->prec == SNF_P_FP32 || r->prec == SNF_P_FP32_REF64) prec_mask |= 1 << kPrecF32;
        if (r->prec == SNF_P_BF16_REF64) prec_mask |= 1 << kPrecBF16;
        if (scheme_is_pij(r->scheme)) prec_mask |= kGroupedDualBit;
      }
    }
    // largest orders first: their tiles run the longest k-loops, so dispatching them first
    // lets the short tiles of small requests fill the end of the step (dispatch order only;
    // every request keeps its own tiles and reduction order)
    std::stable_sort(active.begin(), active.end(), [&](int x, int y) {
      return sv->desc_stage[x].np > sv->desc_stage[y].np;
    });
    const int na = (int)active.size();
    if (na > 0 && rc == SNF_OK) {
      int* idx = sv->index_stage;
      int total = 0;
      for (int a = 0; a < na; ++a) {
        idx[a] = active[a];
        idx[na + a] = total;
        total += num_product_tiles(sv->desc_stage[active[a]].np, 1);
      }
      idx[2 * na] = total;
      // one copy: the active slots at [0, na), the tile offsets at [na, 2 na]
      if (hipMemcpyAsync(sv->index_dev, idx, (2 * na + 1) * sizeof(int), hipMemcpyHostToDevice,
                         s) != hipSuccess)
        rc = SNF_EDEVICE;
      if (rc == SNF_OK) {
        launch_grouped_step(prec_mask, sv->slots, sv->index_dev, sv->index_dev + na, na, total,
                            sv->stop_dev, s, sv->stream2, sv->ev_fork, sv->ev_join);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(sv->stop_stage, sv->stop_dev, na * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipEventRecord(sv->ev_step, s) != hipSuccess)
          rc = SNF_EDEVICE;
      }
    }
    // 2. retire the requests finished in the previous step (their buffers are untouched by
    //    this step: they are not in it, and stopped states make every kernel exit)
    for (size_t f = 0; f < finished.size() && rc == SNF_OK; ++f) {
      ServeRequest* r = finished[f];
      rc = retire_request(sv, r, s3);
      if (rc != SNF_OK) break;
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->arena.release(r->off, r->bytes);
      sv->slot_req[r->slot] = nullptr;
      sv->finishing.push_back(r);
      sv->fin_cv.notify_one();
    }
    finished.clear();
    // 3. admission into free slots (stream order keeps it behind the retirements)
    admitted.clear();
    if (rc == SNF_OK) {
      std::unique_lock<std::mutex> lk(sv->mu);
      for (;;) {
        bool any_running = false;
        for (ServeRequest* r : sv->slot_req) any_running |= (r != nullptr);
        // FIFO on device memory; a request whose host staging is not available yet is
        // passed over (requests holding staging must be able to run and release it)
        for (size_t qi = 0; qi < sv->pending.size();) {
          int k = -1;
          for (int i = 0; i < sv->max_slots; ++i)
            if (!sv->slot_req[i]) {
              k = i;
              break;
            }
          if (k < 0) break;
          ServeRequest* r = sv->pending[qi];
          if (!r->pinned && !take_pinned_locked(sv, r)) {
            ++qi;
            continue;
          }
          size_t off = 0;
          if (!sv->arena.alloc(r->bytes, &off)) break;
          hipEvent_t ev = take_event_locked(sv);
          if (!ev) {
            sv->arena.release(off, r->bytes);
            break;
          }
          sv->pending.erase(sv->pending.begin() + qi);
          if (!r->F_pageable.empty()) {   // late pinned staging: move the host copy over
            memcpy(r->F_pin, r->F_pageable.data(), r->F_pageable.size() * sizeof(double));
            std::vector<double>().swap(r->F_pageable);
          }
          r->ev = ev;
          r->slot = k;
          r->off = off;
          r->t_admit = Clock::now();
          sv->slot_req[k] = r;
          admitted.push_back(r);
          any_running = true;
        }
        if (any_running || na > 0) break;   // work to launch, or a step to wait for
        if (sv->stopping && sv->pending.empty()) {
          sv->sched_done = true;
          sv->fin_cv.notify_all();
          return;
        }
        sv->cv.wait(lk);
      }
    }
    for (ServeRequest* r : admitted) {
      if (rc != SNF_OK) break;
      rc = start_request(sv, r, s3);
      r->started = (rc == SNF_OK);
    }
    if (rc == SNF_OK && !admitted.empty()) {
      if (hipEventRecord(sv->ev_adm, s3) != hipSuccess) rc = SNF_EDEVICE;
      adm_pending = true;
    }
    // 4. wait for the step (and the work enqueued behind it); read its stop flags
    if (rc == SNF_OK && na > 0) {
      // poll the step's event: a blocking wait would add the wake-up latency of the
      // runtime's sleep to every step
      hipError_t q;
      while ((q = hipEventQuery(sv->ev_step)) == hipErrorNotReady) std::this_thread::yield();
      if (q != hipSuccess) {
        rc = SNF_EDEVICE;
      } else {
        for (int a = 0; a < na; ++a) {
          if (!sv->stop_stage[a]) continue;
          ServeRequest* r = sv->slot_req[active[a]];
          r->finished = true;
          r->result_buf = sv->stop_stage[a] - 1;
          r->t_finish = Clock::now();
          finished.push_back(r);
        }
      }
    }
    if (rc != SNF_OK) {
      finished.clear();
      std::lock_guard<std::mutex> lk(sv->mu);
      fail_all_locked(sv, rc);
      if (sv->stopping) {
        sv->sched_done = true;
        sv->fin_cv.notify_all();
        return;
      }
    }
  }
}

static int submit_common(snf_server* sv, ServeRequest* r, uint64_t* ticket) {
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stopping || sv->sticky_error != SNF_OK) {
      const int rc = sv->stopping ? SNF_EINVAL : sv->sticky_error;
      if (r->pinned) sv->pin_arena.release(r->pin_off, r->pin_bytes);
      delete r;
      return rc;
    }
    r->ticket = sv->next_ticket++;
    sv->by_ticket[r->ticket] = r;
    sv->pending.push_back(r);
    *ticket = r->ticket;
  }
  sv->cv.notify_one();
  return SNF_OK;
}

static ServeRequest* new_request(snf_server* sv, int64_t n, const snf_params* params,
                                 snf_scheme scheme, snf_precision precision) {
  ServeRequest* r = new ServeRequest();
  r->n = n;
  r->np = (n + kTile - 1) / kTile * kTile;
  r->params = *params;
  r->scheme = scheme;
  r->prec = precision;
  r->bytes = request_layout(n, precision, request_buffers(scheme)).total;
  memset(&r->result, 0, sizeof(r->result));
  r->result.status = SNF_PENDING;
  r->t_submit = Clock::now();
  return r;
}

}  // namespace snf

extern "C" {

size_t snf_serve_request_bytes(int64_t n, snf_precision precision) {
  if (n <= 0) return 0;
  return request_layout(n, precision).total;
}

int snf_serve_create(size_t hbm_budget_bytes, int32_t max_slots, snf_server** out) {
  if (!out || hbm_budget_bytes < ((size_t)1 << 20) || max_slots < 1 || max_slots > 4096)
    return SNF_EINVAL;
  *out = nullptr;
  snf_server* sv = new snf_server();
  sv->budget = hbm_budget_bytes;
  sv->max_slots = max_slots;
  sv->t_create = Clock::now();
  sv->slot_req.assign(max_slots, nullptr);
  size_t pin = hbm_budget_bytes / 4;
  if (pin < ((size_t)64 << 20)) pin = (size_t)64 << 20;
  if (pin > ((size_t)2 << 30)) pin = (size_t)2 << 30;
  sv->pin_size = pin;
  bool ok = hipGetDevice(&sv->device) == hipSuccess &&
            hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&sv->stream2, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&sv->ev_fork, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&sv->ev_join, hipEventDisableTiming) == hipSuccess &&
            hipStreamCreateWithFlags(&sv->stream3, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&sv->ev_adm, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&sv->ev_step, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipMalloc(&sv->arena_base, hbm_budget_bytes) == hipSuccess;
  ok = ok && hipHostMalloc(&sv->pin_base, pin, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipMalloc(&sv->states, max_slots * sizeof(SnfState)) == hipSuccess &&
       hipMalloc(&sv->bufs, max_slots * sizeof(Buffers)) == hipSuccess &&
       hipMalloc(&sv->slots, max_slots * sizeof(SlotDesc)) == hipSuccess &&
       hipMalloc(&sv->index_dev, (2 * max_slots + 1) * sizeof(int)) == hipSuccess &&
       hipMalloc(&sv->stop_dev, max_slots * sizeof(int32_t)) == hipSuccess;
  ok = ok &&
       hipHostMalloc(&sv->state_stage, max_slots * sizeof(SnfState), hipHostMallocDefault) ==
           hipSuccess &&
       hipHostMalloc(&sv->bufs_stage, max_slots * sizeof(Buffers), hipHostMallocDefault) ==
           hipSuccess &&
       hipHostMalloc(&sv->desc_stage, max_slots * sizeof(SlotDesc), hipHostMallocDefault) ==
           hipSuccess &&
       hipHostMalloc(&sv->index_stage, (2 * max_slots + 1) * sizeof(int),
                     hipHostMallocDefault) == hipSuccess &&
       hipHostMalloc(&sv->stop_stage, max_slots * sizeof(int32_t), hipHostMallocDefault) ==
           hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    sv->stopping = true;
    sv->sched_done = true;
    snf_serve_destroy(sv);
    return SNF_ENOMEM;
  }
  sv->arena.init(hbm_budget_bytes);
  sv->pin_arena.init(pin);
  sv->thread = std::thread(scheduler, sv);
  sv->finisher = std::thread(finisher, sv);
  *out = sv;
  return SNF_OK;
}

int snf_serve_submit(snf_server* sv, const double* F_host, int64_t n, const snf_params* params,
                     snf_scheme scheme, snf_precision precision, double* D_host_out,
                     uint64_t* ticket) {
  if (!sv || !F_host || !D_host_out || !ticket) return SNF_EINVAL;
  int rc = validate(n, params, scheme, precision);
  if (rc != SNF_OK) return rc;
  ServeRequest* r = new_request(sv, n, params, scheme, precision);
  r->D_host = D_host_out;
  if (r->bytes > sv->budget || pinned_bytes(r) > sv->pin_size) {
    delete r;
    return SNF_ENOMEM;
  }
  bool pinned;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    pinned = take_pinned_locked(sv, r);
  }
  const size_t elems = (size_t)n * n;
  if (pinned) memcpy(r->F_pin, F_host, elems * sizeof(double));
  else r->F_pageable.assign(F_host, F_host + elems);
  return submit_common(sv, r, ticket);
}

int snf_serve_submit_device(snf_server* sv, const double* F_dev, int64_t n,
                            const snf_params* params, snf_scheme scheme,
                            snf_precision precision, double* D_dev_out, uint64_t* ticket) {
  if (!sv || !F_dev || !D_dev_out || !ticket || (const void*)F_dev == (const void*)D_dev_out)
    return SNF_EINVAL;
  int rc = validate(n, params, scheme, precision);
  if (rc != SNF_OK) return rc;
  ServeRequest* r = new_request(sv, n, params, scheme, precision);
  r->device_io = true;
  r->F_dev = F_dev;
  r->D_dev = D_dev_out;
  if (r->bytes > sv->budget) {
    delete r;
    return SNF_ENOMEM;
  }
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    (void)take_pinned_locked(sv, r);   // else taken at admission
  }
  return submit_common(sv, r, ticket);
}

int snf_serve_poll(snf_server* sv, uint64_t ticket, snf_result* out) {
  if (!sv) return SNF_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->by_ticket.find(ticket);
  if (it == sv->by_ticket.end()) return SNF_EINVAL;
  ServeRequest* r = it->second;
  if (r->status == SNF_PENDING) return SNF_PENDING;
  if (out) {
    *out = r->result;
    out->device_ms =
        std::chrono::duration<double, std::milli>(r->t_done - r->t_admit).count();
  }
  return r->status;
}

int snf_serve_timing(snf_server* sv, uint64_t ticket, double* ms) {
  if (!sv || !ms) return SNF_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->by_ticket.find(ticket);
  if (it == sv->by_ticket.end()) return SNF_EINVAL;
  ServeRequest* r = it->second;
  if (r->status == SNF_PENDING) return SNF_PENDING;
  using ms_t = std::chrono::duration<double, std::milli>;
  ms[0] = ms_t(r->t_admit - r->t_submit).count();
  ms[1] = ms_t(r->t_done - r->t_admit).count();
  ms[2] = ms_t(r->t_done - r->t_submit).count();
  return SNF_OK;
}

int snf_serve_timeline(snf_server* sv, uint64_t ticket, double* t) {
  if (!sv || !t) return SNF_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->by_ticket.find(ticket);
  if (it == sv->by_ticket.end()) return SNF_EINVAL;
  ServeRequest* r = it->second;
  if (r->status == SNF_PENDING) return SNF_PENDING;
  using ms_t = std::chrono::duration<double, std::milli>;
  t[0] = ms_t(r->t_submit - sv->t_create).count();
  t[1] = ms_t(r->t_admit - sv->t_create).count();
  t[2] = ms_t(r->t_finish - sv->t_create).count();
  t[3] = ms_t(r->t_done - sv->t_create).count();
  return SNF_OK;
}

int snf_serve_destroy(snf_server* sv) {
  if (!sv) return SNF_EINVAL;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
  }
  sv->cv.notify_all();
  if (sv->thread.joinable()) sv->thread.join();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->sched_done = true;
  }
  sv->fin_cv.notify_all();
  if (sv->finisher.joinable()) sv->finisher.join();
  if (sv->stream) (void)hipStreamSynchronize(sv->stream);
  if (sv->stream3) (void)hipStreamSynchronize(sv->stream3);
  if (sv->stream2) (void)hipStreamSynchronize(sv->stream2);
  for (auto& kv : sv->by_ticket) delete kv.second;
  for (hipEvent_t e : sv->free_events) (void)hipEventDestroy(e);
  if (sv->arena_base) (void)hipFree(sv->arena_base);
  if (sv->pin_base) (void)hipHostFree(sv->pin_base);
  if (sv->states) (void)hipFree(sv->states);
  if (sv->bufs) (void)hipFree(sv->bufs);
  if (sv->slots) (void)hipFree(sv->slots);
  if (sv->index_dev) (void)hipFree(sv->index_dev);
  if (sv->stop_dev) (void)hipFree(sv->stop_dev);
  if (sv->state_stage) (void)hipHostFree(sv->state_stage);
  if (sv->bufs_stage) (void)hipHostFree(sv->bufs_stage);
  if (sv->desc_stage) (void)hipHostFree(sv->desc_stage);
  if (sv->index_stage) (void)hipHostFree(sv->index_stage);
  if (sv->stop_stage) (void)hipHostFree(sv->stop_stage);
  if (sv->stream2) (void)hipStreamSynchronize(sv->stream2);
  if (sv->ev_fork) (void)hipEventDestroy(sv->ev_fork);
  if (sv->ev_join) (void)hipEventDestroy(sv->ev_join);
  if (sv->stream2) (void)hipStreamDestroy(sv->stream2);
  if (sv->ev_adm) (void)hipEventDestroy(sv->ev_adm);
  if (sv->ev_step) (void)hipEventDestroy(sv->ev_step);
  if (sv->stream3) (void)hipStreamDestroy(sv->stream3);
  if (sv->stream) (void)hipStreamDestroy(sv->stream);
  const int rc = sv->sticky_error;
  delete sv;
  return rc;
}

}  // extern "C"
