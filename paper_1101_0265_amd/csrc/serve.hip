// Serving loop: continuous batching of many independent dense purifications on one GPU.
//
// A scheduler thread owns a HIP stream and a device arena (the HBM budget).  Each loop turn
//   1. admits queued requests (FIFO) while a slot is free and the arena can hold the
//      request's workspace: copies F in, runs f_0 and the initial schedule for it;
//   2. launches one grouped step over every running request: the product tiles of all of
//      them in one launch per precision variant, then every request's schedule, then a
//      gather of their stop flags;
//   3. reads the stop flags back and retires the finished requests (D and the result to
//      the host, arena and slot released).
// Nothing is allocated on the device while serving (the arena is sub-allocated), so a
// finishing request never waits on a device-wide free.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "snf_internal.h"

namespace snf {

using Clock = std::chrono::steady_clock;

// First-fit sub-allocator over [0, size) with coalescing of free neighbours.
class Arena {
 public:
  void init(size_t size) {
    free_.clear();
    free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

struct ServeRequest {
  uint64_t ticket = 0;
  int64_t n = 0, np = 0;
  snf_params params;
  snf_scheme scheme;
  snf_precision prec;
  std::vector<double> F;
  double* D_host = nullptr;
  Clock::time_point t_submit, t_admit, t_done;
  int slot = -1;
  size_t off = 0, bytes = 0;
  int status = SNF_PENDING;
  snf_result result;
};

struct RequestLayout {   // byte offsets of one request's workspace inside its arena block
  size_t x[3], lp[3], partials, total;
};

static RequestLayout request_layout(int64_t n, snf_precision prec) {
  RequestLayout L;
  const int64_t np = (n + kTile - 1) / kTile * kTile;
  const size_t mat = (size_t)np * np * sizeof(double);
  const size_t lpb = (size_t)np * np * lowp_bytes_for(prec);
  const int tiles = num_product_tiles(np, 1);
  const size_t slots = (size_t)(tiles > kF0Blocks ? tiles : kF0Blocks);
  size_t o = 0;
  for (int i = 0; i < 3; ++i) {
    L.x[i] = o;
    o += (mat + 255) & ~(size_t)255;
  }
  for (int i = 0; i < 3; ++i) {
    L.lp[i] = o;
    o += (lpb + 255) & ~(size_t)255;
  }
  L.partials = o;
  o += slots * 4 * sizeof(double);
  L.total = (o + 255) & ~(size_t)255;
  return L;
}

}  // namespace snf

using namespace snf;

struct snf_server {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;
  int max_slots = 0;
  char* arena_base = nullptr;
  Arena arena;
  // device tables, one entry per slot
  SnfState* states = nullptr;
  Buffers* bufs = nullptr;
  SlotDesc* slots = nullptr;
  int* active_dev = nullptr;     // [max_slots]
  int* offs_dev = nullptr;       // [max_slots + 1]
  int32_t* stop_dev = nullptr;   // [max_slots]
  // pinned host staging
  SnfState* state_stage = nullptr;   // [max_slots]
  Buffers* bufs_stage = nullptr;     // [max_slots]
  SlotDesc* desc_stage = nullptr;    // [max_slots]
  int* index_stage = nullptr;        // [2 * max_slots + 1]
  int32_t* stop_stage = nullptr;     // [max_slots]
  // host bookkeeping
  std::thread thread;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<ServeRequest*> pending;
  std::vector<ServeRequest*> slot_req;
  std::unordered_map<uint64_t, ServeRequest*> by_ticket;
  uint64_t next_ticket = 1;
  bool stopping = false;
  int sticky_error = SNF_OK;
};

namespace snf {

static void fail_all_locked(snf_server* sv, int rc) {
  sv->sticky_error = rc;
  for (ServeRequest* r : sv->slot_req)
    if (r) {
      r->status = rc;
      r->result.status = rc;
      r->t_done = Clock::now();
    }
  std::fill(sv->slot_req.begin(), sv->slot_req.end(), nullptr);
  for (ServeRequest* r : sv->pending) {
    r->status = rc;
    r->result.status = rc;
    r->t_done = Clock::now();
  }
  sv->pending.clear();
}

#define SV_HIP(call)                          \
  do {                                        \
    if ((call) != hipSuccess) return SNF_EDEVICE; \
  } while (0)

// Stage 1 for one admitted request (stream-ordered, no host waits except the pageable F copy).
static int start_request(snf_server* sv, ServeRequest* r) {
  const int k = r->slot;
  const RequestLayout L = request_layout(r->n, r->prec);
  char* base = sv->arena_base + r->off;
  Buffers& b = sv->bufs_stage[k];
  for (int i = 0; i < 3; ++i) {
    b.x[i] = (double*)(base + L.x[i]);
    b.lp[i] = lowp_bytes_for(r->prec) ? (void*)(base + L.lp[i]) : nullptr;
  }
  SlotDesc& d = sv->desc_stage[k];
  d.st = sv->states + k;
  d.bufs = sv->bufs + k;
  d.partials = (double*)(base + L.partials);
  d.np = r->np;
  d.n = r->n;
  init_state(&sv->state_stage[k], r->n, &r->params, r->scheme, r->prec);
  hipStream_t s = sv->stream;
  SV_HIP(hipMemcpyAsync(sv->bufs + k, &b, sizeof(Buffers), hipMemcpyHostToDevice, s));
  SV_HIP(hipMemcpyAsync(sv->slots + k, &d, sizeof(SlotDesc), hipMemcpyHostToDevice, s));
  SV_HIP(hipMemcpyAsync(sv->states + k, &sv->state_stage[k], sizeof(SnfState),
                        hipMemcpyHostToDevice, s));
  // F is staged in x[2] (row stride n), read by f_0, which writes X_0 into x[0]
  SV_HIP(hipMemcpyAsync(b.x[2], r->F.data(), (size_t)r->n * r->n * sizeof(double),
                        hipMemcpyHostToDevice, s));
  launch_f0(b.x[2], r->n, r->n, r->np, sv->states + k, sv->bufs + k, lowp_kind_for(r->prec),
            d.partials, s);
  launch_schedule(sv->states + k, d.partials, kF0Blocks, 1, s);
  SV_HIP(hipGetLastError());
  r->F.clear();
  r->F.shrink_to_fit();
  return SNF_OK;
}

// Stage 3 for one finished request: D to the host, result into *res / *status (published
// to pollers by the caller, under the lock).
static int finish_request(snf_server* sv, ServeRequest* r, snf_result* res, int* status) {
  const int k = r->slot;
  hipStream_t s = sv->stream;
  SnfState* hs = &sv->state_stage[k];
  SV_HIP(hipMemcpyAsync(hs, sv->states + k, sizeof(SnfState), hipMemcpyDeviceToHost, s));
  SV_HIP(hipStreamSynchronize(s));
  const double* X = sv->bufs_stage[k].x[hs->cur];
  SV_HIP(hipMemcpy2DAsync(r->D_host, r->n * sizeof(double), X, r->np * sizeof(double),
                          r->n * sizeof(double), r->n, hipMemcpyDeviceToHost, s));
  SV_HIP(hipStreamSynchronize(s));
  fill_result(hs, res, nullptr, 0);
  *status = hs->stop ? hs->status : SNF_ENOCONV;
  res->status = *status;
  return SNF_OK;
}

static void scheduler(snf_server* sv) {
  (void)hipSetDevice(sv->device);
  std::vector<ServeRequest*> admitted;
  std::vector<int> active;
  for (;;) {
    admitted.clear();
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      for (;;) {
        bool any_running = false;
        for (ServeRequest* r : sv->slot_req) any_running |= (r != nullptr);
        while (!sv->pending.empty()) {
          int k = -1;
          for (int i = 0; i < sv->max_slots; ++i)
            if (!sv->slot_req[i]) {
              k = i;
              break;
            }
          if (k < 0) break;
          ServeRequest* r = sv->pending.front();
          size_t off = 0;
          if (!sv->arena.alloc(r->bytes, &off)) break;   // FIFO: wait for memory
          sv->pending.pop_front();
          r->slot = k;
          r->off = off;
          r->t_admit = Clock::now();
          sv->slot_req[k] = r;
          admitted.push_back(r);
          any_running = true;
        }
        if (any_running) break;
        if (sv->stopping && sv->pending.empty()) return;
        sv->cv.wait(lk);
      }
    }
    int rc = SNF_OK;
    for (ServeRequest* r : admitted)
      if ((rc = start_request(sv, r)) != SNF_OK) break;
    // grouped step over every running request
    active.clear();
    int prec_mask = 1 << kPrecF64;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      for (int i = 0; i < sv->max_slots; ++i)
        if (sv->slot_req[i]) {
          active.push_back(i);
          const snf_precision p = sv->slot_req[i]->prec;
          if (p == SNF_P_FP32 || p == SNF_P_FP32_REF64) prec_mask |= 1 << kPrecF32;
          if (p == SNF_P_BF16_REF64) prec_mask |= 1 << kPrecBF16;
        }
    }
    const int na = (int)active.size();
    if (rc == SNF_OK && na > 0) {
      int* idx = sv->index_stage;
      int total = 0;
      for (int a = 0; a < na; ++a) {
        idx[a] = active[a];
        idx[na + a] = total;
        total += num_product_tiles(sv->desc_stage[active[a]].np, 1);
      }
      idx[2 * na] = total;
      hipStream_t s = sv->stream;
      if (hipMemcpyAsync(sv->active_dev, idx, na * sizeof(int), hipMemcpyHostToDevice, s) !=
              hipSuccess ||
          hipMemcpyAsync(sv->offs_dev, idx + na, (na + 1) * sizeof(int), hipMemcpyHostToDevice,
                         s) != hipSuccess)
        rc = SNF_EDEVICE;
      if (rc == SNF_OK) {
        launch_grouped_step(prec_mask, sv->slots, sv->active_dev, sv->offs_dev, na, total,
                            sv->stop_dev, s);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(sv->stop_stage, sv->stop_dev, na * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          rc = SNF_EDEVICE;
      }
      if (rc == SNF_OK) {
        for (int a = 0; a < na && rc == SNF_OK; ++a) {
          if (!sv->stop_stage[a]) continue;
          ServeRequest* r = sv->slot_req[active[a]];
          snf_result res;
          int status = SNF_OK;
          rc = finish_request(sv, r, &res, &status);
          if (rc != SNF_OK) break;
          std::lock_guard<std::mutex> lk(sv->mu);
          r->result = res;
          r->status = status;
          r->t_done = Clock::now();
          sv->arena.release(r->off, r->bytes);
          sv->slot_req[r->slot] = nullptr;
        }
      }
    }
    if (rc != SNF_OK) {
      std::lock_guard<std::mutex> lk(sv->mu);
      fail_all_locked(sv, rc);
      if (sv->stopping) return;
    }
  }
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
  sv->slot_req.assign(max_slots, nullptr);
  bool ok = hipGetDevice(&sv->device) == hipSuccess &&
            hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipMalloc(&sv->arena_base, hbm_budget_bytes) == hipSuccess;
  ok = ok && hipMalloc(&sv->states, max_slots * sizeof(SnfState)) == hipSuccess &&
       hipMalloc(&sv->bufs, max_slots * sizeof(Buffers)) == hipSuccess &&
       hipMalloc(&sv->slots, max_slots * sizeof(SlotDesc)) == hipSuccess &&
       hipMalloc(&sv->active_dev, max_slots * sizeof(int)) == hipSuccess &&
       hipMalloc(&sv->offs_dev, (max_slots + 1) * sizeof(int)) == hipSuccess &&
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
    snf_serve_destroy(sv);
    return SNF_ENOMEM;
  }
  sv->arena.init(hbm_budget_bytes);
  sv->thread = std::thread(scheduler, sv);
  *out = sv;
  return SNF_OK;
}

int snf_serve_submit(snf_server* sv, const double* F_host, int64_t n, const snf_params* params,
                     snf_scheme scheme, snf_precision precision, double* D_host_out,
                     uint64_t* ticket) {
  if (!sv || !F_host || !D_host_out || !ticket) return SNF_EINVAL;
  int rc = validate(n, params, scheme, precision);
  if (rc != SNF_OK) return rc;
  const size_t bytes = request_layout(n, precision).total;
  if (bytes > sv->budget) return SNF_ENOMEM;
  ServeRequest* r = new ServeRequest();
  r->n = n;
  r->np = (n + kTile - 1) / kTile * kTile;
  r->params = *params;
  r->scheme = scheme;
  r->prec = precision;
  r->F.assign(F_host, F_host + (size_t)n * n);
  r->D_host = D_host_out;
  r->bytes = bytes;
  memset(&r->result, 0, sizeof(r->result));
  r->result.status = SNF_PENDING;
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stopping) {
      delete r;
      return SNF_EINVAL;
    }
    if (sv->sticky_error != SNF_OK) {
      delete r;
      return sv->sticky_error;
    }
    r->ticket = sv->next_ticket++;
    sv->by_ticket[r->ticket] = r;
    sv->pending.push_back(r);
    *ticket = r->ticket;
  }
  sv->cv.notify_one();
  return SNF_OK;
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

int snf_serve_destroy(snf_server* sv) {
  if (!sv) return SNF_EINVAL;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
  }
  sv->cv.notify_all();
  if (sv->thread.joinable()) sv->thread.join();
  if (sv->stream) (void)hipStreamSynchronize(sv->stream);
  for (auto& kv : sv->by_ticket) delete kv.second;
  if (sv->arena_base) (void)hipFree(sv->arena_base);
  if (sv->states) (void)hipFree(sv->states);
  if (sv->bufs) (void)hipFree(sv->bufs);
  if (sv->slots) (void)hipFree(sv->slots);
  if (sv->active_dev) (void)hipFree(sv->active_dev);
  if (sv->offs_dev) (void)hipFree(sv->offs_dev);
  if (sv->stop_dev) (void)hipFree(sv->stop_dev);
  if (sv->state_stage) (void)hipHostFree(sv->state_stage);
  if (sv->bufs_stage) (void)hipHostFree(sv->bufs_stage);
  if (sv->desc_stage) (void)hipHostFree(sv->desc_stage);
  if (sv->index_stage) (void)hipHostFree(sv->index_stage);
  if (sv->stop_stage) (void)hipHostFree(sv->stop_stage);
  if (sv->stream) (void)hipStreamDestroy(sv->stream);
  const int rc = sv->sticky_error;
  delete sv;
  return rc == SNF_OK ? SNF_OK : rc;
}

}  // extern "C"
