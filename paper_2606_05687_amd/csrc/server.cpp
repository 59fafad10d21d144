// Continuous-batching serving front end over the batched solve.
//
// Requests (batches of problems in caller device memory, each typically one
// simulated environment group's problems of one control tick) are queued on
// the host.  A scheduler thread packs whatever is queued into the next free
// lane as soon as one frees up (continuous batching: a launch takes every
// waiting request that fits its capacity), gathers the packed inputs into the
// lane's staging buffers on the lane's own HIP stream (one kernel over a table
// of copy descriptors for every array of every request), runs the solve there
// and scatters the outputs back the same way.  Lanes run
// concurrently, so requests that arrive while others are on the GPU are
// admitted into the next lane and their work overlaps on the device.  A
// completion thread polls each lane's event and stamps request latency
// (submit to results ready).  Optional warm start: problem i of a request with
// warm_base >= 0 starts from the iterates stored in slot warm_base + i (shifted
// by one stage) and leaves its final iterates there.
//
// Each problem is computed by the same kernels with the same per-problem
// arithmetic whatever else is in its launch, so a result is bitwise the same
// alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pinmpc.h"
#include "pinmpc_internal.h"

using namespace pinmpc;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
  int64_t ticket = 0;
  pinmpc_batch in{};
  pinmpc_out out{};
  int32_t warm_base = -1;
  Clock::time_point t_submit;
  double latency_ms = -1.0;
  bool done = false;
  int status = PINMPC_OK;
};

struct Lane {
  pinmpc_ctx ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  void* mem = nullptr;
  // staging, capacity cap problems at PINMPC_NMAX stages
  float *A, *B, *e, *x0, *u_prev, *x_ref, *u_ref, *Q, *R, *mu, *fz, *tau, *weight;
  uint8_t* contact;
  int32_t *N, *warm_idx;
  float *u, *x, *res;
  int32_t *iters, *status, *detail;
  // copy descriptors of a launch's gather and scatter (pinned host table and
  // its device copy, room for kMaxDescPerProblem per problem of capacity)
  CopyDesc* desc_host = nullptr;
  CopyDesc* desc_dev = nullptr;
  std::vector<Request*> inflight;
  bool busy = false;      // owns requests (set by the scheduler before enqueueing)
  bool launched = false;  // its event was recorded after the last enqueued work
};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Gather: up to 16 arrays per request, scatter: up to 6; a request holds at
// least one problem.
constexpr int kMaxDescPerProblem = 22;

size_t staging_bytes(int cap) {
  const size_t S = (size_t)cap * PINMPC_NMAX;
  size_t b = 0;
  auto add = [&](size_t x) { b += align256(x); };
  add(S * NX * NX * 4); add(S * NX * NU * 4); add(S * NX * 4); add((size_t)cap * NX * 4);
  add((size_t)cap * NU * 4); add(S * NX * 4); add(S * NU * 4); add((size_t)cap * NX * 4);
  add((size_t)cap * NU * 4); add((size_t)cap * 4); add((size_t)cap * 4); add((size_t)cap * 4);
  add((size_t)cap * 4); add(S * 2); add((size_t)cap * 4); add((size_t)cap * 4);
  add(S * NU * 4); add((size_t)cap * (PINMPC_NMAX + 1) * NX * 4); add((size_t)cap * PINMPC_NRES * 4);
  add((size_t)cap * 4); add((size_t)cap * 4); add((size_t)cap * 4 * 4);
  add((size_t)cap * kMaxDescPerProblem * sizeof(CopyDesc));
  return b;
}

void carve_lane(Lane& L, int cap) {
  const size_t S = (size_t)cap * PINMPC_NMAX;
  char* p = (char*)L.mem;
  auto take = [&](size_t x) { char* r = p; p += align256(x); return r; };
  L.A = (float*)take(S * NX * NX * 4);
  L.B = (float*)take(S * NX * NU * 4);
  L.e = (float*)take(S * NX * 4);
  L.x0 = (float*)take((size_t)cap * NX * 4);
  L.u_prev = (float*)take((size_t)cap * NU * 4);
  L.x_ref = (float*)take(S * NX * 4);
  L.u_ref = (float*)take(S * NU * 4);
  L.Q = (float*)take((size_t)cap * NX * 4);
  L.R = (float*)take((size_t)cap * NU * 4);
  L.mu = (float*)take((size_t)cap * 4);
  L.fz = (float*)take((size_t)cap * 4);
  L.tau = (float*)take((size_t)cap * 4);
  L.weight = (float*)take((size_t)cap * 4);
  L.contact = (uint8_t*)take(S * 2);
  L.N = (int32_t*)take((size_t)cap * 4);
  L.warm_idx = (int32_t*)take((size_t)cap * 4);
  L.u = (float*)take(S * NU * 4);
  L.x = (float*)take((size_t)cap * (PINMPC_NMAX + 1) * NX * 4);
  L.res = (float*)take((size_t)cap * PINMPC_NRES * 4);
  L.iters = (int32_t*)take((size_t)cap * 4);
  L.status = (int32_t*)take((size_t)cap * 4);
  L.detail = (int32_t*)take((size_t)cap * 4 * 4);
  L.desc_dev = (CopyDesc*)take((size_t)cap * kMaxDescPerProblem * sizeof(CopyDesc));
}

// Builds a table of copy descriptors (rows numbered consecutively).
struct Table {
  CopyDesc* d;
  int n = 0;
  uint64_t rows = 0;
  void add(const void* src, void* dst, size_t row_bytes, size_t src_pitch, size_t dst_pitch,
           size_t nrows, int op = -1, int32_t a = 0, int32_t b = 0) {
    if (nrows == 0 || row_bytes == 0) return;
    CopyDesc& c = d[n++];
    if (op < 0) {
      const bool words = (row_bytes % 4 == 0) && (src_pitch % 4 == 0) && (dst_pitch % 4 == 0) &&
                         ((uintptr_t)src % 4 == 0) && ((uintptr_t)dst % 4 == 0);
      op = words ? COPY_WORDS : COPY_BYTES;
    }
    c.src = src;
    c.dst = dst;
    c.row_bytes = (uint32_t)row_bytes;
    c.src_pitch = (uint32_t)src_pitch;
    c.dst_pitch = (uint32_t)dst_pitch;
    c.rows = (uint32_t)nrows;
    c.op = op;
    c.a = a;
    c.b = b;
    c.pad = 0;
    c.row0 = rows;
    rows += nrows;
  }
};


}  // namespace

struct pinmpc_server_s {
  int device = 0;
  int cap = 0;
  pinmpc_settings s{};
  std::vector<Lane> lanes;
  float* warm_store = nullptr;
  int32_t warm_slots = 0;
  std::mutex m;
  std::condition_variable cv_sched, cv_done;
  std::deque<Request*> queue;
  std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
  int64_t next_ticket = 1;
  bool stop = false;
  std::thread sched, completer;
  int64_t launches = 0, problems = 0;
  int error = PINMPC_OK;

  int launch(Lane& L, std::vector<Request*>& batch);
  void sched_loop();
  void done_loop();
};

int pinmpc_server_s::launch(Lane& L, std::vector<Request*>& rq) {
  hipStream_t st = L.stream;
  int n = 1, total = 0;
  bool has_e = false, has_up = false, has_ur = false, has_w = false, warm = false;
  for (Request* r : rq) {
    n = std::max(n, (int)r->in.n_max);
    total += r->in.batch;
    has_e |= r->in.e != nullptr;
    has_up |= r->in.u_prev != nullptr;
    has_ur |= r->in.u_ref != nullptr;
    has_w |= r->in.weight != nullptr;
    warm |= r->warm_base >= 0;
  }
  // gather table: every array of every request into the lane's staging,
  // stage arrays re-pitched from the request's n_max to the launch's n
  Table g{L.desc_host};
  int off = 0;
  for (Request* r : rq) {
    const pinmpc_batch& q = r->in;
    const size_t nb = (size_t)q.batch, nr = (size_t)q.n_max, o = (size_t)off;
    auto stg = [&](void* dst, const void* src, size_t elem) {
      g.add(src, (char*)dst + o * n * elem, nr * elem, nr * elem, n * elem, nb);
    };
    auto per = [&](void* dst, const void* src, size_t elem) {
      g.add(src, (char*)dst + o * elem, nb * elem, nb * elem, nb * elem, 1);
    };
    auto fill = [&](void* dst, size_t count, int32_t a, int32_t b) {
      g.add(nullptr, dst, count * 4, 0, 0, 1, COPY_FILL, a, b);
    };
    stg(L.A, q.A, NX * NX * 4);
    stg(L.B, q.Bu, NX * NU * 4);
    stg(L.x_ref, q.x_ref, NX * 4);
    stg(L.contact, q.contact, 2);
    if (has_e) {
      if (q.e) stg(L.e, q.e, NX * 4);
      else fill(L.e + o * n * NX, nb * n * NX, 0, 0);
    }
    if (has_ur) {
      if (q.u_ref) stg(L.u_ref, q.u_ref, NU * 4);
      else fill(L.u_ref + o * n * NU, nb * n * NU, 0, 0);
    }
    per(L.x0, q.x0, NX * 4);
    per(L.Q, q.Q, NX * 4);
    per(L.R, q.R, NU * 4);
    per(L.mu, q.mu, 4);
    per(L.fz, q.fz_max, 4);
    per(L.tau, q.tau_max, 4);
    if (has_up) {
      if (q.u_prev) per(L.u_prev, q.u_prev, NU * 4);
      else fill(L.u_prev + o * NU, nb * NU, 0, 0);
    }
    if (has_w) {
      if (q.weight) per(L.weight, q.weight, 4);
      else g.add(q.fz_max, L.weight + o, nb * 4, nb * 4, nb * 4, 1, COPY_HALF);
    }
    if (q.N) per(L.N, q.N, 4);
    else fill(L.N + o, nb, q.n_max, 0);
    if (warm) fill(L.warm_idx + o, nb, r->warm_base < 0 ? -1 : r->warm_base,
                   r->warm_base < 0 ? 0 : 1);
    off += q.batch;
  }
  // scatter table: the launch's outputs back into each request's buffers
  Table sc{L.desc_host + g.n};
  off = 0;
  for (Request* r : rq) {
    const pinmpc_out& d = r->out;
    const size_t nb = (size_t)r->in.batch, nr = (size_t)r->in.n_max, o = (size_t)off;
    sc.add(L.u + o * n * NU, d.u, nr * NU * 4, (size_t)n * NU * 4, nr * NU * 4, nb);
    sc.add(L.x + o * (n + 1) * NX, d.x, (nr + 1) * NX * 4, (size_t)(n + 1) * NX * 4,
           (nr + 1) * NX * 4, nb);
    if (d.res) sc.add(L.res + o * PINMPC_NRES, d.res, nb * PINMPC_NRES * 4, 0, 0, 1);
    if (d.iters) sc.add(L.iters + o, d.iters, nb * 4, 0, 0, 1);
    if (d.status) sc.add(L.status + o, d.status, nb * 4, 0, 0, 1);
    if (d.detail) sc.add(L.detail + o * 4, d.detail, nb * 16, 0, 0, 1);
    off += r->in.batch;
  }
  // the scatter rows are numbered from zero in their own table
  const size_t nd = (size_t)g.n + sc.n;
  if (hipMemcpyAsync(L.desc_dev, L.desc_host, nd * sizeof(CopyDesc), hipMemcpyHostToDevice,
                     st) != hipSuccess ||
      launch_copy_batch(L.desc_dev, g.n, g.rows, st) != hipSuccess)
    return PINMPC_EDEVICE;
  pinmpc_batch sb{};
  sb.batch = total;
  sb.n_max = n;
  sb.N = L.N;
  sb.A = L.A;
  sb.Bu = L.B;
  sb.e = has_e ? L.e : nullptr;
  sb.x0 = L.x0;
  sb.u_prev = has_up ? L.u_prev : nullptr;
  sb.x_ref = L.x_ref;
  sb.u_ref = has_ur ? L.u_ref : nullptr;
  sb.Q = L.Q;
  sb.R = L.R;
  sb.contact = L.contact;
  sb.mu = L.mu;
  sb.fz_max = L.fz;
  sb.tau_max = L.tau;
  sb.weight = has_w ? L.weight : nullptr;
  pinmpc_out so{L.u, L.x, L.res, L.iters, L.status, L.detail};
  int rc = solve_internal(L.ctx, &sb, &so, st, warm ? L.warm_idx : nullptr, warm_store);
  if (rc) return rc;
  if (launch_copy_batch(L.desc_dev + g.n, sc.n, sc.rows, st) != hipSuccess)
    return PINMPC_EDEVICE;
  if (hipEventRecord(L.ev, st) != hipSuccess) return PINMPC_EDEVICE;
  return PINMPC_OK;
}

void pinmpc_server_s::sched_loop() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(m);
  while (true) {
    Lane* free_lane = nullptr;
    cv_sched.wait(lk, [&] {
      if (stop) return true;
      if (queue.empty()) return false;
      for (auto& L : lanes)
        if (!L.busy) return true;
      return false;
    });
    if (stop) return;
    for (auto& L : lanes)
      if (!L.busy) { free_lane = &L; break; }
    std::vector<Request*> rq;
    int total = 0;
    while (!queue.empty() && total + queue.front()->in.batch <= cap) {
      total += queue.front()->in.batch;
      rq.push_back(queue.front());
      queue.pop_front();
    }
    free_lane->busy = true;
    free_lane->launched = false;
    free_lane->inflight = rq;
    lk.unlock();
    const int rc = launch(*free_lane, rq);
    lk.lock();
    // only now may the completion thread look at this lane's event: before
    // the record an earlier (or never recorded) event reads as complete
    free_lane->launched = (rc == PINMPC_OK);
    if (rc) {
      error = rc;
      for (Request* r : rq) {
        r->status = rc;
        r->done = true;
        r->latency_ms =
            std::chrono::duration<double, std::milli>(Clock::now() - r->t_submit).count();
      }
      free_lane->inflight.clear();
      free_lane->busy = false;
      cv_done.notify_all();
      continue;
    }
    ++launches;
    problems += total;
    cv_done.notify_all();
  }
}

void pinmpc_server_s::done_loop() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(m);
  while (true) {
    bool any = false;
    for (auto& L : lanes) {
      if (!L.busy || L.inflight.empty()) continue;
      any = true;
      if (!L.launched) continue;
      const hipError_t q = hipEventQuery(L.ev);
      if (q == hipErrorNotReady) continue;
      const auto now = Clock::now();
      for (Request* r : L.inflight) {
        r->status = (q == hipSuccess) ? PINMPC_OK : PINMPC_EDEVICE;
        r->latency_ms = std::chrono::duration<double, std::milli>(now - r->t_submit).count();
        r->done = true;
      }
      L.inflight.clear();
      L.busy = false;
      L.launched = false;
      cv_sched.notify_all();
      cv_done.notify_all();
    }
    if (stop && !any) return;
    if (any) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else {
      cv_done.wait_for(lk, std::chrono::milliseconds(2));
    }
  }
}

extern "C" {

int pinmpc_server_create(pinmpc_server* out, int device, const pinmpc_settings* s, int n_lanes,
                         int32_t lane_capacity, int32_t warm_slots, size_t hbm_budget_bytes) {
  if (!out || n_lanes < 1 || n_lanes > 16 || lane_capacity < 1 || warm_slots < 0)
    return PINMPC_EINVAL;
  *out = nullptr;
  pinmpc_settings set;
  pinmpc_default_settings(&set);
  if (s) set = *s;
  set.graph = 0;    // staged batches change shape launch to launch
  const size_t budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)64 << 30;
  size_t ws = 0;
  if (pinmpc_workspace_bytes(&set, lane_capacity, PINMPC_NMAX, &ws)) return PINMPC_EINVAL;
  const size_t per_lane = ws + staging_bytes(lane_capacity);
  const size_t warm_bytes = (size_t)warm_slots * PINMPC_NMAX * NSTATE * NL * 4;
  if (per_lane * n_lanes + warm_bytes > budget) return PINMPC_EBUDGET;
  if (hipSetDevice(device) != hipSuccess) return PINMPC_EDEVICE;
  auto* srv = new pinmpc_server_s;
  srv->device = device;
  srv->cap = lane_capacity;
  srv->s = set;
  srv->lanes.resize(n_lanes);
  int rc = PINMPC_OK;
  for (auto& L : srv->lanes) {
    if ((rc = pinmpc_create(&L.ctx, device, ws + 1, &set))) break;
    if ((rc = reserve_internal(L.ctx, lane_capacity, PINMPC_NMAX))) break;
    if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&L.ev, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&L.mem, staging_bytes(lane_capacity)) != hipSuccess ||
        hipHostMalloc((void**)&L.desc_host,
                      (size_t)lane_capacity * kMaxDescPerProblem * sizeof(CopyDesc),
                      hipHostMallocDefault) != hipSuccess) {
      rc = PINMPC_ENOMEM;
      break;
    }
    carve_lane(L, lane_capacity);
  }
  if (!rc && warm_slots) {
    if (hipMalloc(&srv->warm_store, warm_bytes) != hipSuccess ||
        hipMemset(srv->warm_store, 0, warm_bytes) != hipSuccess)
      rc = PINMPC_ENOMEM;
    srv->warm_slots = warm_slots;
  }
  if (rc) {
    for (auto& L : srv->lanes) {
      if (L.ctx) pinmpc_destroy(L.ctx);
      if (L.stream) (void)hipStreamDestroy(L.stream);
      if (L.ev) (void)hipEventDestroy(L.ev);
      if (L.mem) (void)hipFree(L.mem);
      if (L.desc_host) (void)hipHostFree(L.desc_host);
    }
    if (srv->warm_store) (void)hipFree(srv->warm_store);
    delete srv;
    return rc;
  }
  srv->sched = std::thread([srv] { srv->sched_loop(); });
  srv->completer = std::thread([srv] { srv->done_loop(); });
  *out = srv;
  return PINMPC_OK;
}

int pinmpc_submit(pinmpc_server s, const pinmpc_batch* req, const pinmpc_out* out,
                  int32_t warm_base, int64_t* ticket) {
  if (!s || !req || !out || !ticket) return PINMPC_EINVAL;
  if (req->batch < 1 || req->batch > s->cap || req->n_max < 1 || req->n_max > PINMPC_NMAX)
    return PINMPC_EINVAL;
  if (req->contacts != 0 && req->contacts != 2) return PINMPC_EINVAL;   // feet only
  if (!req->A || !req->Bu || !req->x0 || !req->x_ref || !req->Q || !req->R || !req->contact ||
      !req->mu || !req->fz_max || !req->tau_max || !out->u || !out->x)
    return PINMPC_EINVAL;
  if (warm_base >= 0 && (int64_t)warm_base + req->batch > s->warm_slots) return PINMPC_EINVAL;
  auto r = std::make_unique<Request>();
  r->in = *req;
  r->out = *out;
  r->warm_base = warm_base;
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(s->m);
  if (s->stop) return PINMPC_EBUSY;
  if (warm_base >= 0) {
    // a warm slot belongs to one request at a time: the solve reads the slot
    // and writes it back, so two requests in flight on one slot would race
    const int64_t lo = warm_base, hi = (int64_t)warm_base + req->batch;
    for (const auto& kv : s->reqs) {
      const Request& o = *kv.second;
      if (o.done || o.warm_base < 0) continue;
      if (lo < (int64_t)o.warm_base + o.in.batch && (int64_t)o.warm_base < hi)
        return PINMPC_EBUSY;
    }
  }
  r->ticket = s->next_ticket++;
  *ticket = r->ticket;
  s->queue.push_back(r.get());
  s->reqs[r->ticket] = std::move(r);
  s->cv_sched.notify_one();
  return PINMPC_OK;
}

int pinmpc_poll(pinmpc_server s, int64_t ticket, int* done, double* latency_ms) {
  if (!s || !done) return PINMPC_EINVAL;
  std::lock_guard<std::mutex> lk(s->m);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return PINMPC_EINVAL;
  Request* r = it->second.get();
  *done = r->done ? 1 : 0;
  if (latency_ms) *latency_ms = r->latency_ms;
  if (r->done) {
    const int st = r->status;
    s->reqs.erase(it);
    return st;
  }
  return PINMPC_OK;
}

int pinmpc_wait(pinmpc_server s, int64_t ticket, double* latency_ms) {
  if (!s) return PINMPC_EINVAL;
  std::unique_lock<std::mutex> lk(s->m);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return PINMPC_EINVAL;
  Request* r = it->second.get();
  s->cv_done.wait(lk, [&] { return r->done; });
  if (latency_ms) *latency_ms = r->latency_ms;
  const int st = r->status;
  s->reqs.erase(it);
  return st;
}

int pinmpc_server_stats(pinmpc_server s, int64_t* launches, int64_t* problems) {
  if (!s) return PINMPC_EINVAL;
  std::lock_guard<std::mutex> lk(s->m);
  if (launches) *launches = s->launches;
  if (problems) *problems = s->problems;
  return s->error;
}

namespace {

constexpr char kWarmMagic[4] = {'P', 'M', 'W', 'S'};
constexpr int32_t kWarmVersion = 1;

// Range checks shared by export and import; with the server mutex held,
// PINMPC_EBUSY when a request that is not done uses one of the slots.
int check_warm_range(pinmpc_server s, int32_t base, int32_t count, size_t bytes) {
  if (base < 0 || count < 1 || (int64_t)base + count > s->warm_slots) return PINMPC_EINVAL;
  if (bytes < PINMPC_WARM_IMAGE_BYTES(count)) return PINMPC_EINVAL;
  const int64_t lo = base, hi = (int64_t)base + count;
  for (const auto& kv : s->reqs) {
    const Request& o = *kv.second;
    if (o.done || o.warm_base < 0) continue;
    if (lo < (int64_t)o.warm_base + o.in.batch && (int64_t)o.warm_base < hi) return PINMPC_EBUSY;
  }
  return PINMPC_OK;
}

}  // namespace

int pinmpc_server_export_state(pinmpc_server s, int32_t slot_base, int32_t count,
                               void* host_buf, size_t bytes) {
  if (!s || !host_buf) return PINMPC_EINVAL;
  std::lock_guard<std::mutex> lk(s->m);
  const int rc = check_warm_range(s, slot_base, count, bytes);
  if (rc) return rc;
  char* h = (char*)host_buf;
  const int32_t hdr[3] = {kWarmVersion, count, PINMPC_NMAX};
  std::memcpy(h, kWarmMagic, 4);
  std::memcpy(h + 4, hdr, sizeof(hdr));
  const size_t slot_floats = PINMPC_WARM_SLOT_BYTES / 4;
  if (hipSetDevice(s->device) != hipSuccess ||
      hipMemcpy(h + 16, s->warm_store + (size_t)slot_base * slot_floats,
                (size_t)count * PINMPC_WARM_SLOT_BYTES, hipMemcpyDeviceToHost) != hipSuccess)
    return PINMPC_EDEVICE;
  return PINMPC_OK;
}

int pinmpc_server_import_state(pinmpc_server s, int32_t slot_base, int32_t count,
                               const void* host_buf, size_t bytes) {
  if (!s || !host_buf) return PINMPC_EINVAL;
  std::lock_guard<std::mutex> lk(s->m);
  const int rc = check_warm_range(s, slot_base, count, bytes);
  if (rc) return rc;
  const char* h = (const char*)host_buf;
  int32_t hdr[3];
  std::memcpy(hdr, h + 4, sizeof(hdr));
  if (std::memcmp(h, kWarmMagic, 4) != 0 || hdr[0] != kWarmVersion || hdr[1] != count ||
      hdr[2] != PINMPC_NMAX)
    return PINMPC_EINVAL;
  const size_t slot_floats = PINMPC_WARM_SLOT_BYTES / 4;
  if (hipSetDevice(s->device) != hipSuccess ||
      hipMemcpy(s->warm_store + (size_t)slot_base * slot_floats, h + 16,
                (size_t)count * PINMPC_WARM_SLOT_BYTES, hipMemcpyHostToDevice) != hipSuccess)
    return PINMPC_EDEVICE;
  return PINMPC_OK;
}

int pinmpc_server_destroy(pinmpc_server s) {
  if (!s) return PINMPC_EINVAL;
  {
    std::unique_lock<std::mutex> lk(s->m);
    // drain: wait for queued and running requests
    s->cv_done.wait(lk, [&] {
      if (!s->queue.empty()) return false;
      for (auto& L : s->lanes)
        if (L.busy) return false;
      return true;
    });
    s->stop = true;
  }
  s->cv_sched.notify_all();
  s->cv_done.notify_all();
  s->sched.join();
  s->completer.join();
  (void)hipSetDevice(s->device);
  for (auto& L : s->lanes) {
    (void)hipStreamSynchronize(L.stream);
    pinmpc_destroy(L.ctx);
    (void)hipStreamDestroy(L.stream);
    (void)hipEventDestroy(L.ev);
    (void)hipFree(L.mem);
    (void)hipHostFree(L.desc_host);
  }
  if (s->warm_store) (void)hipFree(s->warm_store);
  delete s;
  return PINMPC_OK;
}

}  // extern "C"
