// Host side of the C ABI: argument validation, workspace carving under the
// HBM budget, launch sequencing on the caller's stream, phase timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <algorithm>
#include <cstring>
#include <new>

#include "pinmpc.h"
#include "pinmpc_internal.h"

using namespace pinmpc;

struct GraphKey {
  pinmpc_batch in;
  pinmpc_out out;
  pinmpc_settings s;
  hipStream_t stream;
  void* mem;
};

static bool same_settings(const pinmpc_settings& a, const pinmpc_settings& b) {
  return a.rho == b.rho && a.iters == b.iters && a.accel == b.accel &&
         a.restart_eta == b.restart_eta && a.scaling == b.scaling && a.refine == b.refine &&
         a.refine_passes == b.refine_passes && a.ipm_iters == b.ipm_iters &&
         a.polish_passes == b.polish_passes && a.kkt_tol == b.kkt_tol &&
         a.precision == b.precision && a.form == b.form && a.graph == b.graph &&
         a.first_passes == b.first_passes && a.group == b.group && a.scan == b.scan;
}

static bool same_key(const GraphKey& a, const GraphKey& b) {
  return std::memcmp(&a.in, &b.in, sizeof(a.in)) == 0 &&
         std::memcmp(&a.out, &b.out, sizeof(a.out)) == 0 && same_settings(a.s, b.s) &&
         a.stream == b.stream && a.mem == b.mem;
}

struct pinmpc_ctx_s {
  int device = 0;
  size_t budget = 0;
  pinmpc_settings s{};
  void* mem = nullptr;
  size_t mem_bytes = 0;
  // phase events of the last PINMPC_STATS_RING solves (start, after setup,
  // after the sweeps, end); ev points at the current solve's set
  hipEvent_t ring[PINMPC_STATS_RING][4] = {};
  bool ring_graph[PINMPC_STATS_RING] = {};   // that solve replayed a graph
  int64_t nsolves = 0;
  hipEvent_t* ev = ring[0];
  bool have_timing = false;
  hipGraphExec_t gexec = nullptr;
  GraphKey gkey{};
  // the last solve's shape, sweep count and refinement work counter
  size_t last_stages = 0;
  int last_iters = 0;
  const unsigned long long* last_work = nullptr;
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

}  // namespace

namespace pinmpc {

// Carve (or size, when base == nullptr) the workspace for batch x n with nc
// contacts per stage.
size_t carve_workspace(char* base, int32_t batch, int32_t n, Workspace* w, int nc) {
  const size_t NU = 6 * (size_t)nc, NL = NX + NU;
  const size_t NH = NL * (NL + 1) / 2, NM = NU * (NU + 1) / 2;
  const size_t rdoubles = nc == 4 ? std::max(refine_block_doubles(n), refine_wide_block_doubles(n))
                                  : refine_block_doubles(n);
  const size_t S = (size_t)batch * n;        // stages
  const size_t Bn = (size_t)batch;
  const size_t X = (size_t)batch * (n + 1);  // state slots
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  Workspace t{};
  t.Bt = (float*)take(S * NX * NU * 4);
  t.Hp = (float*)take(S * NH * 4);
  t.Mp = (float*)take(S * NM * 4);
  t.qb = (float*)take(S * NL * 4);
  t.Abf = (uint16_t*)take(S * NX * NX * 2);
  t.Btbf = (uint16_t*)take(S * NX * NU * 2);
  t.Hbf = (uint16_t*)take(S * NH * 2);
  t.Mbf = (uint16_t*)take(S * NM * 2);
  t.sf = (float*)take(S * 4);
  t.tsc = (float*)take(Bn * 4);
  t.cur = (float*)take(S * NSTATE * NL * 4);
  t.hat = (float*)take(S * NSTATE * NL * 4);
  t.alpha = (float*)take(Bn * 4);
  t.cprev = (float*)take(Bn * 4);
  t.restarts = (int32_t*)take(Bn * 4);
  t.flags = (uint32_t*)take(Bn * 4);
  t.rblk = (double*)take(Bn * rdoubles * 8);
  t.faces = (int32_t*)take(S * 2 * 4);
  t.order = (int32_t*)take(Bn * 3 * 4);
  t.counts = (int32_t*)take(4 * 4);
  t.rlist = (int32_t*)take(Bn * 4);
  t.rcount = (int32_t*)take(4);
  t.rpass = (int32_t*)take(Bn * 4);
  t.work = (unsigned long long*)take(8);
  t.sp_aty = (float*)take(S * NL * 4);
  t.sp_du = (float*)take(S * NU * 4);
  t.sp_xi = (float*)take(S * NL * 4);
  t.sp_new = (float*)take(S * NSTATE * NL * 4);
  t.sp_ct = (float*)take(S * 4);
  t.sp_dec = (float*)take(Bn * 2 * 4);
  t.bytes = off;
  t.warm_idx = nullptr;
  t.warm_store = nullptr;
  if (w) *w = t;
  return off;
}

int check_settings(const pinmpc_settings* s) {
  if (!s) return PINMPC_EINVAL;
  if (!(s->rho > 0.f) || !std::isfinite(s->rho)) return PINMPC_EINVAL;
  if (s->iters < 0 || s->iters > 1000000) return PINMPC_EINVAL;
  if (!(s->restart_eta > 0.f && s->restart_eta <= 1.f)) return PINMPC_EINVAL;
  if (s->refine_passes < 0 || s->ipm_iters < 0 || s->polish_passes < 0) return PINMPC_EINVAL;
  if (s->refine_passes > 1000 || s->ipm_iters > 1000 || s->polish_passes > 1000)
    return PINMPC_EINVAL;
  if (!(s->kkt_tol > 0.0)) return PINMPC_EINVAL;
  if (s->precision < 0 || s->precision > 1) return PINMPC_EINVAL;
  if (s->form < -1 || s->form > 2) return PINMPC_EINVAL;
  if (s->graph < 0 || s->graph > 1) return PINMPC_EINVAL;
  if (s->first_passes < 0) return PINMPC_EINVAL;
  if (s->group != 1 && s->group != 2 && s->group != 4) return PINMPC_EINVAL;
  if (s->scan != 0 && s->scan != 2 && s->scan != 4 && s->scan != 8) return PINMPC_EINVAL;
  // a refinement needs at least one pass or interior-point iteration: the
  // outputs are the last pass's solution
  if (s->refine && s->refine_passes == 0 && s->ipm_iters == 0) return PINMPC_EINVAL;
  return PINMPC_OK;
}

int contacts_of(const pinmpc_batch* in) { return in->contacts == 4 ? 4 : 2; }

int check_batch(const pinmpc_batch* in) {
  if (!in) return PINMPC_EINVAL;
  if (in->batch < 0 || in->n_max < 1 || in->n_max > PINMPC_NMAX_LONG) return PINMPC_EINVAL;
  if (in->contacts != 0 && in->contacts != 2 && in->contacts != 4) return PINMPC_EINVAL;
  if (in->contacts == 4 && in->n_max > PINMPC_NMAX) return PINMPC_EINVAL;
  if (in->batch == 0) return PINMPC_OK;
  if (!in->A || !in->Bu || !in->x0 || !in->x_ref || !in->Q || !in->R || !in->contact ||
      !in->mu || !in->fz_max || !in->tau_max)
    return PINMPC_EINVAL;
  return PINMPC_OK;
}

Problem to_problem(const pinmpc_batch* in) {
  Problem p;
  p.batch = in->batch;
  p.n_max = in->n_max;
  p.nc = contacts_of(in);
  p.N = in->N;
  p.A = in->A;
  p.B = in->Bu;
  p.e = in->e;
  p.x0 = in->x0;
  p.u_prev = in->u_prev;
  p.x_ref = in->x_ref;
  p.u_ref = in->u_ref;
  p.Q = in->Q;
  p.R = in->R;
  p.contact = in->contact;
  p.mu = in->mu;
  p.fz_max = in->fz_max;
  p.tau_max = in->tau_max;
  p.weight = in->weight;
  return p;
}

// The fused kernel holds one problem per workgroup with one thread per
// (stage, lifted row) and that row's operators in registers: horizons up to
// 1024 / 25 = 40 stages.  Longer horizons in the fused and packed forms run all
// sweeps in one launch of the streaming kernel (iterates resident, operators
// streamed).
static bool fits_fused(int n_max) { return NL * n_max <= 1024; }

// The ADMM sweeps in the form the settings ask for.
int launch_admm_phase(const pinmpc_settings& s, const Problem& p, const Workspace& w, int iters,
                      hipStream_t st) {
  if (iters <= 0) return PINMPC_OK;
  if (p.nc != NCONTACT) {
    // four contacts: the streaming sweep kernel, one launch per sweep (form
    // 0) or all sweeps in one launch
    if (s.form == 0) {
      for (int it = 0; it < iters; ++it)
        if (launch_admm_sweep(p, w, s, 1, st) != hipSuccess) return PINMPC_EDEVICE;
    } else if (launch_admm_sweep(p, w, s, iters, st) != hipSuccess) {
      return PINMPC_EDEVICE;
    }
    return PINMPC_OK;
  }
  if (s.form == 2 || p.n_max > PINMPC_NMAX) {
    // the horizon split across workgroups: every horizon up to PINMPC_NMAX_LONG
    if (launch_admm_split(p, w, s, iters, st) != hipSuccess) return PINMPC_EDEVICE;
  } else if (s.form == -1 && p.n_max > CLASS_N[0]) {
    // pack problems by horizon class: fused kernels sized for each class,
    // the persistent streaming kernel for the longest horizons
    if (launch_classify(p, w, st) != hipSuccess) return PINMPC_EDEVICE;
    for (int cls = 0; cls < 2; ++cls)
      if (launch_admm_fused_class(p, w, s, iters, cls, st) != hipSuccess) return PINMPC_EDEVICE;
    if (p.n_max > CLASS_N[1] && launch_admm_sweep_class(p, w, s, 2, iters, st) != hipSuccess)
      return PINMPC_EDEVICE;
  } else if (s.form != 0 && fits_fused(p.n_max)) {
    if (launch_admm_fused(p, w, s, iters, st) != hipSuccess) return PINMPC_EDEVICE;
  } else if (s.form != 0) {
    if (launch_admm_sweep(p, w, s, iters, st) != hipSuccess) return PINMPC_EDEVICE;
  } else {
    for (int it = 0; it < iters; ++it)
      if (launch_admm_sweep(p, w, s, 1, st) != hipSuccess) return PINMPC_EDEVICE;
  }
  return PINMPC_OK;
}

// The FP64 refinement for the batch's contact count.
hipError_t launch_refine_any(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                             const pinmpc_out& out, hipStream_t st) {
  return p.nc == NCONTACT ? launch_refine(p, w, s, out, st) : launch_refine_wide(p, w, s, out, st);
}

}  // namespace pinmpc

namespace {

int ensure_workspace(pinmpc_ctx c, int32_t batch, int32_t n, int nc, hipStream_t st,
                     Workspace* w) {
  const size_t need = carve_workspace(nullptr, batch, n, nullptr, nc);
  if (need > c->budget) return PINMPC_EBUDGET;
  if (need > c->mem_bytes) {
    if (c->mem) {
      if (hipStreamSynchronize(st) != hipSuccess) return PINMPC_EDEVICE;
      if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
      }
      (void)hipFree(c->mem);
      c->mem = nullptr;
      c->mem_bytes = 0;
    }
    if (hipMalloc(&c->mem, need) != hipSuccess) {
      c->mem = nullptr;
      return PINMPC_ENOMEM;
    }
    c->mem_bytes = need;
  }
  carve_workspace((char*)c->mem, batch, n, w, nc);
  return PINMPC_OK;
}

int run_admm(pinmpc_ctx c, const Problem& p, const Workspace& w, int iters, hipStream_t st) {
  // the refinement adds its work to this counter (a fill kernel: graph-safe)
  if (launch_fill_i32((int32_t*)w.work, 2, 0, 0, st) != hipSuccess) return PINMPC_EDEVICE;
  c->last_stages = (size_t)p.batch * p.n_max;
  c->last_iters = iters;
  c->last_work = w.work;
  if (launch_setup(p, w, c->s, st) != hipSuccess) return PINMPC_EDEVICE;
  if (launch_admm_init(p, w, st) != hipSuccess) return PINMPC_EDEVICE;
  if (c->have_timing) (void)hipEventRecord(c->ev[1], st);
  return launch_admm_phase(c->s, p, w, iters, st);
}

}  // namespace

extern "C" {

void pinmpc_default_settings(pinmpc_settings* s) {
  if (!s) return;
  std::memset(s, 0, sizeof(*s));
  s->rho = 10.f;
  s->iters = 100;
  s->accel = 1;
  s->restart_eta = 0.999f;
  s->scaling = 1;
  s->refine = 1;
  s->refine_passes = 8;
  s->ipm_iters = 40;
  s->polish_passes = 6;
  s->kkt_tol = 1e-9;
  s->precision = 0;
  s->form = 0;
  s->graph = 1;
  s->first_passes = 4;
  s->group = 1;
  s->scan = 0;
}

int pinmpc_create(pinmpc_ctx* out, int device, size_t hbm_budget_bytes,
                  const pinmpc_settings* s) {
  if (!out) return PINMPC_EINVAL;
  *out = nullptr;
  pinmpc_settings def;
  pinmpc_default_settings(&def);
  if (!s) s = &def;
  const int rc = check_settings(s);
  if (rc) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return PINMPC_EDEVICE;
  if (hipSetDevice(device) != hipSuccess || refine_prepare() != hipSuccess)
    return PINMPC_EDEVICE;
  pinmpc_ctx c = new (std::nothrow) pinmpc_ctx_s;
  if (!c) return PINMPC_ENOMEM;
  c->device = device;
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)64 << 30;
  c->s = *s;
  c->have_timing = true;
  for (auto& set : c->ring)
    for (auto& e : set)
      if (hipEventCreate(&e) != hipSuccess) c->have_timing = false;
  *out = c;
  return PINMPC_OK;
}

int pinmpc_set_settings(pinmpc_ctx c, const pinmpc_settings* s) {
  if (!c) return PINMPC_EINVAL;
  const int rc = check_settings(s);
  if (rc) return rc;
  c->s = *s;
  return PINMPC_OK;
}

int pinmpc_workspace_bytes(const pinmpc_settings* s, int32_t batch, int32_t n_max,
                           size_t* bytes) {
  if (!bytes || batch < 0 || n_max < 1 || n_max > PINMPC_NMAX_LONG) return PINMPC_EINVAL;
  (void)s;
  *bytes = carve_workspace(nullptr, batch, n_max, nullptr);
  return PINMPC_OK;
}

int pinmpc_workspace_bytes_contacts(const pinmpc_settings* s, int32_t batch, int32_t n_max,
                                    int32_t contacts, size_t* bytes) {
  if (contacts == 0 || contacts == 2) return pinmpc_workspace_bytes(s, batch, n_max, bytes);
  if (contacts != 4 || !bytes || batch < 0 || n_max < 1 || n_max > PINMPC_NMAX)
    return PINMPC_EINVAL;
  (void)s;
  *bytes = carve_workspace(nullptr, batch, n_max, nullptr, 4);
  return PINMPC_OK;
}

}  // extern "C"

namespace pinmpc {

int solve_internal(pinmpc_ctx c, const pinmpc_batch* in, const pinmpc_out* out_in,
                   hipStream_t st, const int32_t* warm_idx, float* warm_store) {
  if (!c || !out_in) return PINMPC_EINVAL;
  pinmpc_out outv = *out_in;
  pinmpc_out* out = &outv;
  int rc = check_batch(in);
  if (rc) return rc;
  if (in->batch > 0 && (!out->u || !out->x)) return PINMPC_EINVAL;
  if (contacts_of(in) != NCONTACT && c->s.refine && c->s.ipm_iters == 0) return PINMPC_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return PINMPC_EDEVICE;
  if (in->batch == 0) return PINMPC_OK;
  Workspace w;
  rc = ensure_workspace(c, in->batch, in->n_max, contacts_of(in), st, &w);
  if (rc) return rc;
  w.warm_idx = warm_idx;
  w.warm_store = warm_store;
  const Problem p = to_problem(in);
  if (c->s.graph && !warm_idx) {
    GraphKey key;
    std::memset(&key, 0, sizeof(key));
    std::memcpy(&key.in, in, sizeof(*in));
    std::memcpy(&key.out, out, sizeof(*out));
    key.s = c->s;
    key.stream = st;
    key.mem = c->mem;
    if (!c->gexec || !same_key(key, c->gkey)) {
      if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
      }
      // capture setup -> sweeps -> refinement; only kernel launches (no
      // memset nodes), timing events stay outside the graph
      hipStream_t cap;
      if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
        return PINMPC_EDEVICE;
      const bool timing = c->have_timing;
      c->have_timing = false;
      hipGraph_t g = nullptr;
      int crc = PINMPC_OK;
      if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        crc = PINMPC_EDEVICE;
      } else {
        crc = run_admm(c, p, w, c->s.iters, cap);
        if (!crc && launch_refine_any(p, w, c->s, *out, cap) != hipSuccess) crc = PINMPC_EDEVICE;
        if (hipStreamEndCapture(cap, &g) != hipSuccess) crc = PINMPC_EDEVICE;
      }
      c->have_timing = timing;
      (void)hipStreamDestroy(cap);
      if (!crc && hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
        c->gexec = nullptr;
        crc = PINMPC_EDEVICE;
      }
      if (g) (void)hipGraphDestroy(g);
      if (crc) return crc;
      std::memcpy(&c->gkey, &key, sizeof(key));
    }
    const int slot = (int)(c->nsolves % PINMPC_STATS_RING);
    c->ev = c->ring[slot];
    c->ring_graph[slot] = true;
    if (c->have_timing) (void)hipEventRecord(c->ev[0], st);
    if (hipGraphLaunch(c->gexec, st) != hipSuccess) return PINMPC_EDEVICE;
    if (c->have_timing) (void)hipEventRecord(c->ev[3], st);
    ++c->nsolves;
    return PINMPC_OK;
  }
  const int slot = (int)(c->nsolves % PINMPC_STATS_RING);
  c->ev = c->ring[slot];
  c->ring_graph[slot] = false;
  if (c->have_timing) (void)hipEventRecord(c->ev[0], st);
  rc = run_admm(c, p, w, c->s.iters, st);
  if (rc) return rc;
  if (warm_idx && launch_warm_save(p, w, c->s.accel, st) != hipSuccess) return PINMPC_EDEVICE;
  if (c->have_timing) (void)hipEventRecord(c->ev[2], st);
  if (launch_refine_any(p, w, c->s, *out, st) != hipSuccess) return PINMPC_EDEVICE;
  if (c->have_timing) (void)hipEventRecord(c->ev[3], st);
  ++c->nsolves;
  return PINMPC_OK;
}

int solve_in_buffer(pinmpc_ctx c, const pinmpc_batch* in, const pinmpc_out* out_in,
                    hipStream_t st, void* base, size_t capacity) {
  if (!c || !out_in) return PINMPC_EINVAL;
  const pinmpc_out& out = *out_in;
  int rc = check_batch(in);
  if (rc) return rc;
  if (in->batch > 0 && (!out.u || !out.x)) return PINMPC_EINVAL;
  if (contacts_of(in) != NCONTACT && c->s.refine && c->s.ipm_iters == 0) return PINMPC_EINVAL;
  const int nc = contacts_of(in);
  if (carve_workspace(nullptr, in->batch, in->n_max, nullptr, nc) > capacity)
    return PINMPC_ETOOBIG;
  if (in->batch == 0) return PINMPC_OK;
  if (!base) return PINMPC_EINVAL;
  Workspace w;
  carve_workspace((char*)base, in->batch, in->n_max, &w, nc);
  const Problem p = to_problem(in);
  // eager launches only: instantiating a graph would allocate
  const int slot = (int)(c->nsolves % PINMPC_STATS_RING);
  c->ev = c->ring[slot];
  c->ring_graph[slot] = false;
  if (c->have_timing) (void)hipEventRecord(c->ev[0], st);
  rc = run_admm(c, p, w, c->s.iters, st);
  if (rc) return rc;
  if (c->have_timing) (void)hipEventRecord(c->ev[2], st);
  if (launch_refine_any(p, w, c->s, out, st) != hipSuccess) return PINMPC_EDEVICE;
  if (c->have_timing) (void)hipEventRecord(c->ev[3], st);
  ++c->nsolves;
  return PINMPC_OK;
}

int context_device(pinmpc_ctx c) { return c ? c->device : -1; }

int reserve_internal(pinmpc_ctx c, int32_t batch, int32_t n) {
  if (!c) return PINMPC_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return PINMPC_EDEVICE;
  Workspace w;
  return ensure_workspace(c, batch, n, NCONTACT, nullptr, &w);
}

}  // namespace pinmpc

extern "C" {

int pinmpc_solve(pinmpc_ctx c, const pinmpc_batch* in, pinmpc_out* out, void* hip_stream) {
  return pinmpc::solve_internal(c, in, out, (hipStream_t)hip_stream, nullptr, nullptr);
}

int pinmpc_admm(pinmpc_ctx c, const pinmpc_batch* in, int32_t iters, float* z_out,
                void* hip_stream) {
  if (!c || !z_out || iters < 0) return PINMPC_EINVAL;
  int rc = check_batch(in);
  if (rc) return rc;
  if (hipSetDevice(c->device) != hipSuccess) return PINMPC_EDEVICE;
  hipStream_t st = (hipStream_t)hip_stream;
  if (in->batch == 0) return PINMPC_OK;
  Workspace w;
  rc = ensure_workspace(c, in->batch, in->n_max, contacts_of(in), st, &w);
  if (rc) return rc;
  const Problem p = to_problem(in);
  const bool timing = c->have_timing;
  c->have_timing = false;
  rc = run_admm(c, p, w, iters, st);
  c->have_timing = timing;
  if (rc) return rc;
  if (launch_admm_extract(p, w, c->s.accel, z_out, st) != hipSuccess) return PINMPC_EDEVICE;
  return PINMPC_OK;
}

int pinmpc_stats_back(pinmpc_ctx c, int32_t back, double* total_ms, double* setup_ms,
                      double* admm_ms, double* refine_ms) {
  if (!c || !c->have_timing || back < 0 || back >= PINMPC_STATS_RING || back >= c->nsolves)
    return PINMPC_EINVAL;
  const int slot = (int)((c->nsolves - 1 - back) % PINMPC_STATS_RING);
  hipEvent_t* ev = c->ring[slot];
  if (hipEventSynchronize(ev[3]) != hipSuccess) return PINMPC_EDEVICE;
  if (c->ring_graph[slot]) {
    float t = 0;
    if (hipEventElapsedTime(&t, ev[0], ev[3]) != hipSuccess) return PINMPC_EDEVICE;
    if (total_ms) *total_ms = t;
    if (setup_ms) *setup_ms = -1.0;
    if (admm_ms) *admm_ms = -1.0;
    if (refine_ms) *refine_ms = -1.0;
    return PINMPC_OK;
  }
  float t01 = 0, t12 = 0, t23 = 0;
  if (hipEventElapsedTime(&t01, ev[0], ev[1]) != hipSuccess) return PINMPC_EDEVICE;
  if (hipEventElapsedTime(&t12, ev[1], ev[2]) != hipSuccess) return PINMPC_EDEVICE;
  if (hipEventElapsedTime(&t23, ev[2], ev[3]) != hipSuccess) return PINMPC_EDEVICE;
  if (setup_ms) *setup_ms = t01;
  if (admm_ms) *admm_ms = t12;
  if (refine_ms) *refine_ms = t23;
  if (total_ms) *total_ms = (double)t01 + t12 + t23;
  return PINMPC_OK;
}

int pinmpc_stats(pinmpc_ctx c, double* total_ms, double* setup_ms, double* admm_ms,
                 double* refine_ms) {
  return pinmpc_stats_back(c, 0, total_ms, setup_ms, admm_ms, refine_ms);
}

int pinmpc_stats_traffic(pinmpc_ctx c, double* bytes, double* gbytes_per_s) {
  if (!c || !c->have_timing || c->nsolves == 0 || !c->last_work) return PINMPC_EINVAL;
  hipEvent_t* ev = c->ring[(c->nsolves - 1) % PINMPC_STATS_RING];
  if (hipEventSynchronize(ev[3]) != hipSuccess) return PINMPC_EDEVICE;
  unsigned long long pass_stages = 0;
  if (hipSetDevice(c->device) != hipSuccess ||
      hipMemcpy(&pass_stages, c->last_work, sizeof(pass_stages), hipMemcpyDeviceToHost) !=
          hipSuccess)
    return PINMPC_EDEVICE;
  const double b = (double)c->last_stages *
                       (PINMPC_SETUP_BYTES + (double)c->last_iters * PINMPC_SWEEP_BYTES) +
                   (double)pass_stages * PINMPC_REFINE_BYTES;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, ev[0], ev[3]) != hipSuccess) return PINMPC_EDEVICE;
  if (bytes) *bytes = b;
  if (gbytes_per_s) *gbytes_per_s = ms > 0.f ? b / ((double)ms * 1e6) : 0.0;
  return PINMPC_OK;
}

int pinmpc_build_dynamics(const pinmpc_physics* in, float* A, float* Bu, float* e,
                          void* hip_stream) {
  if (!in || in->batch < 0 || in->n_max < 1 || in->n_max > PINMPC_NMAX_LONG) return PINMPC_EINVAL;
  if (in->model < 0 || in->model > 1) return PINMPC_EINVAL;
  if (in->batch == 0) return PINMPC_OK;
  if (!A || !Bu || !in->c_ref || !in->feet || !in->mass || !in->dt) return PINMPC_EINVAL;
  if (in->model == 0 && (!in->yaw || !in->inertia)) return PINMPC_EINVAL;
  if (in->model == 1 && !e) return PINMPC_EINVAL;
  Physics ph;
  ph.batch = in->batch;
  ph.n_max = in->n_max;
  ph.model = in->model;
  ph.N = in->N;
  ph.yaw = in->yaw;
  ph.c_ref = in->c_ref;
  ph.feet = in->feet;
  ph.mass = in->mass;
  ph.inertia = in->inertia;
  ph.dt = in->dt;
  return launch_dynamics(ph, A, Bu, e, (hipStream_t)hip_stream) == hipSuccess ? PINMPC_OK
                                                                             : PINMPC_EDEVICE;
}

static int to_store(const pinmpc_landmarks* in, LandmarkStore* st) {
  if (!in || in->envs < 0 || in->n_landmarks < 1 || in->n_landmarks > 31 || in->ring < 2 ||
      in->ticks_per_step < 1)
    return PINMPC_EINVAL;
  if (in->envs > 0 && (!in->com || !in->tag)) return PINMPC_EINVAL;
  st->envs = in->envs;
  st->n_landmarks = in->n_landmarks;
  st->ring = in->ring;
  st->ticks_per_step = in->ticks_per_step;
  st->com = in->com;
  st->tag = in->tag;
  return PINMPC_OK;
}

int pinmpc_landmarks_clear(const pinmpc_landmarks* in, const uint8_t* env_mask,
                           void* hip_stream) {
  LandmarkStore st;
  const int rc = to_store(in, &st);
  if (rc) return rc;
  return launch_landmarks_clear(st, env_mask, (hipStream_t)hip_stream) == hipSuccess
             ? PINMPC_OK
             : PINMPC_EDEVICE;
}

int pinmpc_landmarks_push(const pinmpc_landmarks* in, int32_t n_max, const int32_t* N,
                          const float* x, int32_t tick, void* hip_stream) {
  LandmarkStore st;
  const int rc = to_store(in, &st);
  if (rc) return rc;
  if (n_max < 1 || n_max > PINMPC_NMAX_LONG || tick < 0) return PINMPC_EINVAL;
  if ((int64_t)st.ring <= (int64_t)n_max * st.ticks_per_step) return PINMPC_EINVAL;
  if ((int64_t)tick + (int64_t)n_max * st.ticks_per_step > INT32_MAX) return PINMPC_EINVAL;
  if (st.envs > 0 && !x) return PINMPC_EINVAL;
  return launch_landmarks_push(st, n_max, N, x, tick, (hipStream_t)hip_stream) == hipSuccess
             ? PINMPC_OK
             : PINMPC_EDEVICE;
}

int pinmpc_landmark_reward(const pinmpc_landmarks* in, const float* com, int32_t tick,
                           const float* alpha, const float* qc, float sigma, float* reward,
                           int32_t* used, void* hip_stream) {
  LandmarkStore st;
  const int rc = to_store(in, &st);
  if (rc) return rc;
  if (tick < 0 || !(sigma > 0.f) || !std::isfinite(sigma)) return PINMPC_EINVAL;
  if (st.envs > 0 && (!com || !alpha || !qc || !reward)) return PINMPC_EINVAL;
  return launch_landmark_reward(st, com, tick, alpha, qc, sigma, reward, used,
                                (hipStream_t)hip_stream) == hipSuccess
             ? PINMPC_OK
             : PINMPC_EDEVICE;
}

int pinmpc_destroy(pinmpc_ctx c) {
  if (!c) return PINMPC_EINVAL;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->mem) (void)hipFree(c->mem);
  for (auto& set : c->ring)
    for (auto& e : set)
      if (e) (void)hipEventDestroy(e);
  delete c;
  return PINMPC_OK;
}

const char* pinmpc_strerror(int code) {
  switch (code) {
    case PINMPC_OK: return "ok";
    case PINMPC_EINVAL: return "invalid argument";
    case PINMPC_ENOMEM: return "device allocation failed";
    case PINMPC_EBUDGET: return "workspace exceeds the HBM budget";
    case PINMPC_EDEVICE: return "HIP runtime or launch error";
    case PINMPC_EBUSY: return "busy";
    case PINMPC_ETOOBIG: return "batch needs more workspace than the static scratch holds";
    default: return "unknown error";
  }
}

}  // extern "C"
