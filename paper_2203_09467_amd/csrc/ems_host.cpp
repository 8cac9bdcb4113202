// ems_host.cpp -- C ABI of the step loop: context, workspace carving, geometry,
// event slots and queue, the host iteration loop, tally readout.
//
// The host loop (paper Sec. 3.2: a step is several kernels with synchronisation
// points; events are batched to keep enough tracks in flight), per sync interval:
//   1. admit whole queued events while pool room and the energy budget allow
//      (one kernel appending primaries to the pools);
//   2. K iterations enqueued back to back, each k_iter_begin (pool sizes from the
//      previous outputs, on the device), k_transport (up to four steps per track),
//      k_interact (interactions, secondaries, room check);
//   3. one readback of the counters and the list of events that just finished.
// The step count of a track, not the iteration, keys its random numbers, so
// admission order, put-off interactions and pool size change no result.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <string>
#include <unordered_map>
#include <vector>

#include "emshower.h"
#include "ems_device.h"
#include "ems_host.h"

using namespace ems;

namespace {

thread_local std::string g_err;

ems_status fail(ems_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_OK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(EMS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kMaxPerSync = 32;
constexpr uint32_t kMaxVol = 4096;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Sequential carving of the workspace; with base == nullptr it only measures.
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off = align_up(off + n * sizeof(T));
    return p;
  }
};

struct EventInfo {
  uint32_t slot;
  uint32_t n_prim, n_gamma;  // primaries, of which photons
  double e_in;
};

}  // namespace

struct ems_ctx {
  ems_config cfg{};
  Params P{};
  Pool set{};         // all four pool buffers (see Pool)
  Pool pool[2][2]{};  // views [class: photon, charged][buffer]
  IQueue iq{};
  Queue q{};
  int cur = 0;
  uint32_t nG = 0, nC = 0;  // tracks in the current photon / charged pool
  bool tables = false, geometry = false;
  ems_physics_options opts{};
  // device regions
  double* tab_d = nullptr;
  float* tab_f = nullptr;
  double* geo_bounds = nullptr;
  int* geo_mat = nullptr;
  int* geo_bin = nullptr;
  double* e_in = nullptr;
  double* scale = nullptr;
  int64_t* stage_off = nullptr;
  uint32_t* stage_slot = nullptr;
  uint32_t* stage_id = nullptr;
  double* stage_out = nullptr;
  unsigned long long* ctr = nullptr;
  // pinned host mirror of the counters and done list
  unsigned long long* h_ctr = nullptr;
  uint64_t run_steps[3] = {0, 0, 0};  // track-steps by species since init_geometry
  uint32_t* h_done = nullptr;
  // event slots
  std::vector<uint32_t> free_slots;
  std::vector<int> slot_state;  // 0 free, 1 queued or in flight, 2 finished
  std::vector<uint32_t> slot_id;
  std::vector<double> slot_e;
  std::unordered_map<uint32_t, uint32_t> id_to_slot;
  std::deque<EventInfo> pending;
  uint32_t q_head = 0, q_count = 0;
  uint64_t pending_prims = 0;
  double e_flight = 0.0;
  // step-kernel statistics
  hipEvent_t ev[2 * kMaxPerSync] = {};
  int per_sync = 8;  // iterations per host synchronisation
  ems_kernel_stats stats{};
};

namespace {

void carve(Carver& c, const ems_config& cfg, ems_ctx* x) {
  const size_t N = cfg.pool_capacity, E = cfg.max_events, B = cfg.max_bins, Qc = cfg.queue_capacity;
  Pool set;  // four buffers per field: (photon, charged) x (parity 0, 1)
  set.x = c.take<double>(4 * N);
  set.y = c.take<double>(4 * N);
  set.z = c.take<double>(4 * N);
  set.u = c.take<double>(4 * N);
  set.v = c.take<double>(4 * N);
  set.w = c.take<double>(4 * N);
  set.T = c.take<double>(4 * N);
  set.nlam = c.take<double>(4 * N);
  set.k0 = c.take<uint32_t>(4 * N);
  set.k1 = c.take<uint32_t>(4 * N);
  set.k2 = c.take<uint32_t>(4 * N);
  set.evt = c.take<uint32_t>(4 * N);
  set.nstep = c.take<uint32_t>(4 * N);
  set.meta = c.take<uint32_t>(4 * N);
  set.src = c.take<uint32_t>(4 * N);
  IQueue iq;
  const size_t NQ = (size_t)kNumQueues * N;
  iq.x = c.take<double>(NQ);
  iq.y = c.take<double>(NQ);
  iq.z = c.take<double>(NQ);
  iq.u = c.take<double>(NQ);
  iq.v = c.take<double>(NQ);
  iq.w = c.take<double>(NQ);
  iq.T = c.take<double>(NQ);
  iq.k0 = c.take<uint32_t>(NQ);
  iq.k1 = c.take<uint32_t>(NQ);
  iq.k2 = c.take<uint32_t>(NQ);
  iq.evt = c.take<uint32_t>(NQ);
  iq.nstep = c.take<uint32_t>(NQ);
  iq.meta = c.take<uint32_t>(NQ);
  iq.src = c.take<uint32_t>(NQ);
  iq.capacity = (uint32_t)N;
  double* tab_d = c.take<double>((size_t)kMaxMat * 3 * kGrid * kQ);
  float* tab_f = c.take<float>((size_t)kMaxMat * 3 * kGrid * kQ);
  double* gb = c.take<double>(kMaxVol + 1);
  int* gm = c.take<int>(kMaxVol);
  int* gbin = c.take<int>(kMaxVol);
  unsigned long long* tally = c.take<unsigned long long>(E * B);
  unsigned long long* ledger = c.take<unsigned long long>(E * kLedger);
  int* alive = c.take<int>(E);
  double* scale = c.take<double>(E);
  double* e_in = c.take<double>(E);
  uint32_t* done = c.take<uint32_t>(E);
  unsigned long long* ctr = c.take<unsigned long long>(kNumLines * kLineWords);
  unsigned long long* esc = c.take<unsigned long long>(3 * kGrid);
  Queue q;
  q.species = c.take<int32_t>(Qc);
  q.T = c.take<double>(Qc);
  q.x = c.take<double>(Qc);
  q.y = c.take<double>(Qc);
  q.z = c.take<double>(Qc);
  q.u = c.take<double>(Qc);
  q.v = c.take<double>(Qc);
  q.w = c.take<double>(Qc);
  q.slot = c.take<uint32_t>(Qc);
  q.index = c.take<uint32_t>(Qc);
  q.event_id = c.take<uint32_t>(Qc);
  q.capacity = (uint32_t)Qc;
  int64_t* so = c.take<int64_t>(E + 1);
  uint32_t* ss = c.take<uint32_t>(E);
  uint32_t* si = c.take<uint32_t>(E);
  double* sout = c.take<double>(E * (B + 5));
  if (!x) return;
  x->set = set;
  for (int cl = 0; cl < 2; ++cl)
    for (int b = 0; b < 2; ++b) {
      const size_t o = (size_t)(2 * cl + b) * N;
      Pool& p = x->pool[cl][b];
      p.x = set.x + o;
      p.y = set.y + o;
      p.z = set.z + o;
      p.u = set.u + o;
      p.v = set.v + o;
      p.w = set.w + o;
      p.T = set.T + o;
      p.nlam = set.nlam + o;
      p.k0 = set.k0 + o;
      p.k1 = set.k1 + o;
      p.k2 = set.k2 + o;
      p.evt = set.evt + o;
      p.nstep = set.nstep + o;
      p.meta = set.meta + o;
      p.src = set.src + o;
    }
  x->iq = iq;
  x->tab_d = tab_d;
  x->tab_f = tab_f;
  x->geo_bounds = gb;
  x->geo_mat = gm;
  x->geo_bin = gbin;
  x->P.tab_d = tab_d;
  x->P.tab_f = tab_f;
  x->P.bounds = gb;
  x->P.vmat = gm;
  x->P.vbin = gbin;
  x->P.tally = tally;
  x->P.ledger = ledger;
  x->P.alive = alive;
  x->P.scale = scale;
  x->P.done = done;
  x->P.ctr = ctr;
  x->P.esc_hist = esc;
  x->scale = scale;
  x->e_in = e_in;
  x->ctr = ctr;
  x->q = q;
  x->stage_off = so;
  x->stage_slot = ss;
  x->stage_id = si;
  x->stage_out = sout;
}

bool config_ok(const ems_config* c) {
  return c && c->pool_capacity >= 64 && c->pool_capacity <= (1u << 30) && c->max_events >= 1 &&
         c->max_bins >= 1 && (uint64_t)c->max_events * c->max_bins < (1ull << 29) &&
         c->queue_capacity >= 1 && c->iterations_per_sync <= kMaxPerSync &&
         (c->precision == EMS_FP64 || c->precision == EMS_MIXED);
}

void reset_events(ems_ctx* x) {
  const uint32_t E = x->cfg.max_events;
  x->free_slots.resize(E);
  for (uint32_t i = 0; i < E; ++i) x->free_slots[i] = E - 1 - i;
  x->slot_state.assign(E, 0);
  x->slot_id.assign(E, 0);
  x->slot_e.assign(E, 0.0);
  x->id_to_slot.clear();
  x->pending.clear();
  x->q_head = 0;
  x->q_count = 0;
  x->pending_prims = 0;
  x->e_flight = 0.0;
  x->nG = x->nC = 0;
  x->cur = 0;
}

}  // namespace

extern "C" {

const char* ems_last_error(void) { return g_err.c_str(); }

size_t ems_workspace_bytes(const ems_config* cfg) {
  if (!config_ok(cfg)) return 0;
  Carver c{nullptr};
  carve(c, *cfg, nullptr);
  return c.off;
}

ems_status ems_create(const ems_config* cfg, void* d_workspace, size_t bytes, ems_ctx** out) {
  if (!out) return fail(EMS_E_ARG, "ems_create: out is null");
  *out = nullptr;
  if (!config_ok(cfg)) return fail(EMS_E_ARG, "ems_create: invalid configuration");
  if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0)
    return fail(EMS_E_ARG, "ems_create: workspace must be non-null and 256-byte aligned");
  const size_t need = ems_workspace_bytes(cfg);
  if (bytes < need)
    return fail(EMS_E_CAPACITY, "ems_create: workspace of " + std::to_string(bytes) +
                                    " bytes, need " + std::to_string(need));
  ems_ctx* x = new (std::nothrow) ems_ctx();
  if (!x) return fail(EMS_E_INTERNAL, "ems_create: out of host memory");
  x->cfg = *cfg;
  Carver c{static_cast<char*>(d_workspace)};
  carve(c, *cfg, x);
  x->P.seed = cfg->seed;
  x->P.max_events = cfg->max_events;
  hipError_t e = hipHostMalloc((void**)&x->h_ctr, kNumLines * kLineWords * sizeof(unsigned long long),
                               hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&x->h_done, (size_t)cfg->max_events * sizeof(uint32_t),
                      hipHostMallocDefault);
  if (e != hipSuccess) {
    if (x->h_ctr) (void)hipHostFree(x->h_ctr);
    delete x;
    return fail(EMS_E_HIP, std::string("ems_create: pinned host buffer: ") + hipGetErrorString(e));
  }
  x->per_sync = cfg->iterations_per_sync == 0 ? 8 : (int)cfg->iterations_per_sync;
  if (cfg->flags & EMS_FLAG_TIME_STEPS) {
    for (int j = 0; j < 2 * x->per_sync; ++j)
      if (hipEventCreate(&x->ev[j]) != hipSuccess) {
        ems_destroy(x);
        return fail(EMS_E_HIP, "ems_create: hipEventCreate failed");
      }
  }
  reset_events(x);
  *out = x;
  return EMS_OK;
}

void ems_destroy(ems_ctx* x) {
  if (!x) return;
  if (x->h_ctr) (void)hipHostFree(x->h_ctr);
  if (x->h_done) (void)hipHostFree(x->h_done);
  for (hipEvent_t e : x->ev)
    if (e) (void)hipEventDestroy(e);
  delete x;
}

ems_status init_physics_tables(ems_ctx* x, const ems_material* mats, int32_t n_mats,
                               const ems_physics_options* o, void* stream) {
  if (!x || !o || (n_mats > 0 && !mats)) return fail(EMS_E_ARG, "init_physics_tables: null argument");
  if (n_mats < 1 || n_mats > kMaxMat) return fail(EMS_E_ARG, "init_physics_tables: 1..8 materials");
  if (!(o->tracking_cut > 0.0) || !(o->step_alpha > 0.0 && o->step_alpha <= 1.0) ||
      !(o->step_rfinal > 0.0) || o->max_steps < 1)
    return fail(EMS_E_ARG, "init_physics_tables: invalid options");
  std::vector<double> tab;
  MatParams mp[kMaxMat];
  std::memset(mp, 0, sizeof(mp));
  if (ems::build_physics_tables(mats, n_mats, *o, tab, mp) != 0)
    return fail(EMS_E_ARG, "init_physics_tables: invalid material");
  std::vector<float> tabf(tab.size());
  for (size_t i = 0; i < tab.size(); ++i) tabf[i] = (float)tab[i];
  hipStream_t s = (hipStream_t)stream;
  HIP_OK(hipMemcpyAsync(x->tab_d, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(x->tab_f, tabf.data(), tabf.size() * sizeof(float), hipMemcpyHostToDevice, s));
  HIP_OK(hipStreamSynchronize(s));
  Params& P = x->P;
  P.lnE0 = std::log(1.0e-3);
  P.dlnE = std::log(1.0e8) / (kGrid - 1);
  P.inv_dlnE = 1.0 / P.dlnE;
  P.lnE0_f = (float)P.lnE0;
  P.dlnE_f = (float)P.dlnE;
  P.inv_dlnE_f = (float)P.inv_dlnE;
  for (int m = 0; m < kMaxMat; ++m) P.mat[m] = mp[m];
  P.n_mats = n_mats;
  P.tcut = o->tracking_cut;
  P.alpha = o->step_alpha;
  P.rfinal = o->step_rfinal;
  P.tcut_f = (float)P.tcut;
  P.alpha_f = (float)P.alpha;
  P.rfinal_f = (float)P.rfinal;
  P.max_steps = o->max_steps;
  P.charged_local = o->charged_local != 0;
  P.cont_loss = o->continuous_loss != 0;
  x->opts = *o;
  x->tables = true;
  x->geometry = false;
  return EMS_OK;
}

ems_status init_geometry(ems_ctx* x, const ems_geometry* g, void* stream) {
  if (!x || !g || !g->bounds || !g->material || !g->tally_bin)
    return fail(EMS_E_ARG, "init_geometry: null argument");
  if (!x->tables) return fail(EMS_E_STATE, "init_geometry: call init_physics_tables first");
  if (g->kind != EMS_GEOM_SLABS && g->kind != EMS_GEOM_CYLINDERS)
    return fail(EMS_E_ARG, "init_geometry: unknown kind");
  if (g->n_vol < 1 || (uint32_t)g->n_vol > kMaxVol) return fail(EMS_E_ARG, "init_geometry: 1..4096 volumes");
  if (g->n_bins < 1 || (uint32_t)g->n_bins > x->cfg.max_bins)
    return fail(EMS_E_ARG, "init_geometry: n_bins exceeds the configured max_bins");
  for (int i = 0; i < g->n_vol; ++i) {
    if (!(g->bounds[i + 1] > g->bounds[i])) return fail(EMS_E_ARG, "init_geometry: bounds must increase");
    if (g->material[i] < -1 || g->material[i] >= x->P.n_mats)
      return fail(EMS_E_ARG, "init_geometry: unknown material index");
    if (g->tally_bin[i] < 0 || g->tally_bin[i] >= g->n_bins)
      return fail(EMS_E_ARG, "init_geometry: tally bin out of range");
  }
  if (g->kind == EMS_GEOM_SLABS && !(g->half_x > 0 && g->half_y > 0))
    return fail(EMS_E_ARG, "init_geometry: slab half widths must be positive");
  if (g->kind == EMS_GEOM_CYLINDERS && !(g->half_z > 0 && g->bounds[0] == 0.0))
    return fail(EMS_E_ARG, "init_geometry: shells need half_z > 0 and a first radius of 0");
  if (g->bz != 0.0 && !(g->field_tol > 0.0))
    return fail(EMS_E_ARG, "init_geometry: a field needs a positive field_tol");
  hipStream_t s = (hipStream_t)stream;
  HIP_OK(hipMemcpyAsync(x->geo_bounds, g->bounds, sizeof(double) * (g->n_vol + 1), hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(x->geo_mat, g->material, sizeof(int) * g->n_vol, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(x->geo_bin, g->tally_bin, sizeof(int) * g->n_vol, hipMemcpyHostToDevice, s));
  Params& P = x->P;
  P.gkind = g->kind;
  P.nvol = g->n_vol;
  P.nbins = g->n_bins;
  P.hx = g->half_x;
  P.hy = g->half_y;
  P.hz = g->half_z;
  P.bz = g->bz;
  P.ftol = g->field_tol;
  HIP_OK(launch_zero_u64(x->ctr, kNumLines * kLineWords, s));
  x->run_steps[0] = x->run_steps[1] = x->run_steps[2] = 0;
  HIP_OK(launch_zero_u64(P.esc_hist, 3 * kGrid, s));
  HIP_OK(hipStreamSynchronize(s));
  reset_events(x);
  x->geometry = true;
  return EMS_OK;
}

}  // extern "C"

namespace {

// Submit a batch: slots, ring copy, slot initialisation.  Nothing changes on error.
ems_status submit(ems_ctx* x, const ems_event_batch* b, hipStream_t s) {
  const uint32_t ne = b->n_events;
  if (ne == 0) return EMS_OK;
  if (!b->event_ids || !b->offsets) return fail(EMS_E_ARG, "transport_events: null ids/offsets");
  if (b->offsets[0] != 0) return fail(EMS_E_ARG, "transport_events: offsets[0] must be 0");
  for (uint32_t e = 0; e < ne; ++e)
    if (b->offsets[e + 1] < b->offsets[e] + 1)
      return fail(EMS_E_ARG, "transport_events: every event needs at least one primary");
  const uint64_t n = (uint64_t)b->offsets[ne];
  if (!b->species || !b->energy || !b->pos || !b->dir)
    return fail(EMS_E_ARG, "transport_events: null primary arrays");
  if (ne > x->free_slots.size())
    return fail(EMS_E_CAPACITY, "transport_events: not enough free event slots");
  if (n + x->q_count > x->cfg.queue_capacity)
    return fail(EMS_E_CAPACITY, "transport_events: primaries exceed the queue capacity");
  for (uint32_t e = 0; e < ne; ++e) {
    if (x->id_to_slot.count(b->event_ids[e])) return fail(EMS_E_ARG, "transport_events: duplicate event id");
    if ((uint64_t)(b->offsets[e + 1] - b->offsets[e]) > x->cfg.pool_capacity / 4)
      return fail(EMS_E_CAPACITY, "transport_events: event larger than a quarter of the pool");
  }
  {
    std::vector<uint32_t> ids(b->event_ids, b->event_ids + ne);
    if (!std::is_sorted(ids.begin(), ids.end())) std::sort(ids.begin(), ids.end());
    if (std::adjacent_find(ids.begin(), ids.end()) != ids.end())
      return fail(EMS_E_ARG, "transport_events: duplicate event id in batch");
  }
  std::vector<uint32_t> slots(ne);
  for (uint32_t e = 0; e < ne; ++e) slots[e] = x->free_slots[x->free_slots.size() - 1 - e];
  HIP_OK(hipMemcpyAsync(x->stage_off, b->offsets, sizeof(int64_t) * (ne + 1), hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(x->stage_slot, slots.data(), sizeof(uint32_t) * ne, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(x->stage_id, b->event_ids, sizeof(uint32_t) * ne, hipMemcpyHostToDevice, s));
  const uint32_t tail = (x->q_head + x->q_count) % x->q.capacity;
  // validity flags of the batch's primaries: a word of the done line, unused otherwise
  unsigned long long* bad = x->ctr + kLDone * kLineWords + 1;
  HIP_OK(launch_zero_u64(bad, 1, s));
  HIP_OK(launch_enqueue(x->q, tail, x->stage_off, x->stage_slot, x->stage_id, ne, b->species,
                        b->energy, b->pos, b->dir, (uint32_t)n, bad, s));
  HIP_OK(launch_event_init(x->P, x->stage_off, x->stage_slot, b->energy, b->species, ne, x->e_in,
                           x->scale, x->stage_out, s));
  // primary energy per event (admission energy budget) and photons per event (pool sizes)
  std::vector<double> ev_e(ne);
  std::vector<int32_t> sp(n);
  HIP_OK(hipMemcpyAsync(ev_e.data(), x->stage_out, ne * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(sp.data(), b->species, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  unsigned long long badw = 0;
  HIP_OK(hipMemcpyAsync(&badw, bad, sizeof(badw), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (badw) {
    std::string m = "transport_events: invalid primaries:";
    if (badw & 1ull) m += " species not 0, 1 or 2;";
    if (badw & 2ull) m += " kinetic energy not in (0, 1e5] MeV;";
    if (badw & 4ull) m += " position not finite;";
    if (badw & 8ull) m += " direction not a unit vector;";
    return fail(EMS_E_ARG, m);
  }
  for (uint64_t r = 0; r < n; ++r)
    if (sp[r] < 0 || sp[r] > 2) return fail(EMS_E_ARG, "transport_events: species must be 0, 1 or 2");
  x->id_to_slot.reserve(x->id_to_slot.size() + ne);
  for (uint32_t e = 0; e < ne; ++e) {
    const uint32_t sl = slots[e];
    x->free_slots.pop_back();
    x->slot_state[sl] = 1;
    x->slot_id[sl] = b->event_ids[e];
    x->slot_e[sl] = ev_e[e];
    x->id_to_slot[b->event_ids[e]] = sl;
    uint32_t ng = 0;
    for (int64_t r = b->offsets[e]; r < b->offsets[e + 1]; ++r) ng += sp[r] == EMS_GAMMA;
    x->pending.push_back({sl, (uint32_t)(b->offsets[e + 1] - b->offsets[e]), ng, ev_e[e]});
  }
  x->q_count += (uint32_t)n;
  x->pending_prims += n;
  return EMS_OK;
}

// Admit queued events (whole) into the current pools.  The admission kernel runs
// after k_iter_begin has set the admission cursors to the pool sizes.
ems_status admit(ems_ctx* x, hipStream_t s, uint32_t* m_out) {
  uint32_t m = 0, mg = 0;
  const uint32_t room = x->cfg.pool_capacity / 4;  // keep room for the showers to grow
  const double budget = x->cfg.energy_budget;
  const uint32_t n_active = x->nG + x->nC;
  while (!x->pending.empty()) {
    const EventInfo& ev = x->pending.front();
    // an empty pool always takes the next event, so admission cannot stall
    const bool first = n_active + m == 0;
    if (!first && n_active + m + ev.n_prim > room) break;
    if (!first && budget > 0.0 && x->e_flight > 0.0 && x->e_flight + ev.e_in > budget) break;
    m += ev.n_prim;
    mg += ev.n_gamma;
    x->e_flight += ev.e_in;
    x->pending.pop_front();
  }
  *m_out = m;
  if (m == 0) return EMS_OK;
  HIP_OK(launch_admit(x->P, x->q, x->set, x->cfg.pool_capacity, x->cur, x->q_head, m, s));
  x->q_head = (x->q_head + m) % x->q.capacity;
  x->q_count -= m;
  x->pending_prims -= m;
  x->nG += mg;
  x->nC += m - mg;
  return EMS_OK;
}

// One sync interval: up to `iters` iterations enqueued back to back (admission
// only at its start), then one readback of the counters.  Pool sizes and queue
// sizes stay on the device between iterations.  The pool is kept within `bound`
// tracks by the interaction kernel (interactions that would not fit are put off),
// so every launch covers at most `bound` tracks: twice the pool at the start of
// the interval plus a margin, or the whole capacity when full_room is set.
struct IntervalOut {
  uint64_t stepped = 0, deferred = 0, busy = 0, peak = 0;
};

constexpr uint32_t kBoundMargin = 65536;
// steps a track may take in one transport launch while it neither interacts nor
// dies (single-step diagnostics take one)
constexpr uint32_t kStepsPerLaunch = 4;
// a pool this small cannot fill the GPU: its launches are latency bound, so each
// takes more steps per track (the tail of a run, long-lived loopers)
constexpr uint64_t kTailTracks = 16384;
constexpr uint32_t kTailStepsPerLaunch = 32;
constexpr uint32_t kDonePrefetch = 4096;  // finished-event entries read with the counters

ems_status run_interval(ems_ctx* x, hipStream_t s, ems_step_record* rec, int iters,
                        bool admit_first, bool full_room, IntervalOut* io) {
  HIP_OK(launch_iter_begin(x->ctr, true, x->nG, x->nC, s));
  if (admit_first) {
    uint32_t m = 0;
    const ems_status st = admit(x, s, &m);
    if (st != EMS_OK) return st;
  }
  if (x->nG + x->nC == 0) {
    if (admit_first && !x->pending.empty())
      return fail(EMS_E_INTERNAL, "transport_events: queued events could not be admitted");
    return EMS_OK;
  }
  const uint32_t cap = x->cfg.pool_capacity;
  const bool mixed = x->cfg.precision == EMS_MIXED;
  const uint64_t n0 = (uint64_t)x->nG + x->nC;
  const uint32_t bound =
      full_room ? cap : (uint32_t)std::min<uint64_t>(cap, std::max<uint64_t>(n0, 2 * n0 + kBoundMargin));
  const uint32_t msteps = full_room ? 1u : (n0 < kTailTracks ? kTailStepsPerLaunch : kStepsPerLaunch);
  for (int j = 0; j < iters; ++j) {
    if (j > 0) HIP_OK(launch_iter_begin(x->ctr, false, 0, 0, s));
    if (x->ev[2 * j]) HIP_OK(hipEventRecord(x->ev[2 * j], s));
    HIP_OK(launch_iteration(x->P, x->set, cap, x->cur, x->iq, bound, msteps, mixed, rec, s));
    if (x->ev[2 * j + 1]) HIP_OK(hipEventRecord(x->ev[2 * j + 1], s));
    x->cur = 1 - x->cur;
  }
  const uint32_t pre = std::min<uint32_t>(x->cfg.max_events, kDonePrefetch);
  HIP_OK(hipMemcpyAsync(x->h_ctr, x->ctr, kNumLines * kLineWords * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(x->h_done, x->P.done, pre * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const unsigned long long* L = x->h_ctr;
  unsigned long long S[kLineWords] = {};
  for (int c = 0; c < kStatCopies; ++c)
    for (int w = 0; w < kLineWords; ++w) S[w] += L[(kLStats + c) * kLineWords + w];
  S[kSPeak] = L[kLStats * kLineWords + kSPeak];
  const unsigned long long out = L[kLOut * kLineWords] + L[kLOutI * kLineWords];
  const uint32_t outG = (uint32_t)(out & 0xFFFFFFFFull), outC = (uint32_t)(out >> 32);
  const uint32_t n_done = std::min((uint32_t)L[kLDone * kLineWords], x->cfg.max_events);
  uint64_t queued_last = 0;
  for (int l = 0; l < 4; ++l) {
    const unsigned long long v = L[(kLQueue + l) * kLineWords];
    queued_last += (v & 0xFFFFFFFFull) + (v >> 32);
  }
  x->run_steps[EMS_GAMMA] += S[kSStepG];
  x->run_steps[EMS_POSITRON] += S[kSStepPos];
  x->run_steps[EMS_ELECTRON] += S[kSStepC] - S[kSStepPos];
  x->stats.launches += S[kSBusy];
  x->stats.tracks_in += S[kSIn];
  x->stats.tracks_out += S[kSOut] + outG + outC;
  x->stats.queued += S[kSQueued] + queued_last;
  if (x->ev[0]) {
    for (int j = 0; j < iters; ++j) {
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, x->ev[2 * j], x->ev[2 * j + 1]));
      x->stats.kernel_ms += ms;
    }
  }
  if (n_done) {
    if (n_done > pre) {
      HIP_OK(hipMemcpyAsync(x->h_done, x->P.done, n_done * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
    }
    for (uint32_t j = 0; j < n_done; ++j) {
      const uint32_t sl = x->h_done[j];
      if (sl < x->slot_state.size() && x->slot_state[sl] == 1) {
        x->slot_state[sl] = 2;
        x->e_flight -= x->slot_e[sl];
      }
    }
    if (x->e_flight < 0.0) x->e_flight = 0.0;
  }
  x->nG = outG;
  x->nC = outC;
  io->stepped += S[kSStepG] + S[kSStepC];
  io->deferred += S[kSDeferred];
  io->busy += S[kSBusy];
  io->peak = std::max<uint64_t>(io->peak, S[kSPeak]);
  if (S[kSStall]) return fail(EMS_E_CAPACITY, "transport_events: pool full, no track can step");
  return EMS_OK;
}

}  // namespace

extern "C" {

ems_status transport_events(ems_ctx* x, const ems_event_batch* b, int32_t max_iterations,
                            void* stream, ems_progress* progress) {
  if (!x) return fail(EMS_E_ARG, "transport_events: null context");
  if (!x->tables || !x->geometry) return fail(EMS_E_STATE, "transport_events: initialise tables and geometry first");
  hipStream_t s = (hipStream_t)stream;
  if (b) {
    const ems_status st = submit(x, b, s);
    if (st != EMS_OK) return st;
  }
  uint64_t it = 0;
  IntervalOut io;
  io.peak = (uint64_t)x->nG + x->nC;
  const int per_sync = x->per_sync;
  while (max_iterations < 0 || it < (uint64_t)max_iterations) {
    if (x->nG + x->nC == 0 && x->pending.empty()) break;
    int k = per_sync;
    if (max_iterations >= 0) k = (int)std::min<uint64_t>((uint64_t)k, (uint64_t)max_iterations - it);
    const ems_status st = run_interval(x, s, nullptr, k, true, false, &io);
    if (st != EMS_OK) return st;
    it += k;
  }
  const uint64_t stepped = io.stepped, deferred = io.deferred, peak = io.peak;
  if (progress) {
    progress->alive = (uint64_t)x->nG + x->nC;
    progress->queued_primaries = x->pending_prims;
    progress->queued_events = x->pending.size();
    progress->iterations = io.busy;
    progress->track_steps = stepped;
    progress->deferred = deferred;
    progress->peak_alive = peak;
  }
  return EMS_OK;
}

ems_status tally_read(ems_ctx* x, uint32_t n, const uint32_t* ids, double* dep, double* ledger,
                      int32_t* status, void* stream) {
  if (!x || (n && (!ids || !dep || !ledger || !status))) return fail(EMS_E_ARG, "tally_read: null argument");
  if (!x->geometry) return fail(EMS_E_STATE, "tally_read: no geometry");
  hipStream_t s = (hipStream_t)stream;
  std::vector<uint32_t> slots;
  std::vector<uint32_t> rows;
  bool all = true;
  for (uint32_t j = 0; j < n; ++j) {
    auto it = x->id_to_slot.find(ids[j]);
    if (it == x->id_to_slot.end()) {
      status[j] = EMS_E_ARG;
      all = false;
    } else if (x->slot_state[it->second] != 2) {
      status[j] = EMS_NOT_READY;
      all = false;
    } else {
      status[j] = EMS_OK;
      slots.push_back(it->second);
      rows.push_back(j);
    }
  }
  const uint32_t nb = (uint32_t)x->P.nbins;
  const uint32_t w = nb + 5;
  const uint32_t chunk = x->cfg.max_events;
  std::vector<double> buf;
  for (size_t a = 0; a < slots.size(); a += chunk) {
    const uint32_t m = (uint32_t)std::min<size_t>(chunk, slots.size() - a);
    HIP_OK(hipMemcpyAsync(x->stage_slot, slots.data() + a, m * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    HIP_OK(launch_gather_tallies(x->P, x->stage_slot, m, x->e_in, x->stage_out, s));
    buf.resize((size_t)m * w);
    HIP_OK(hipMemcpyAsync(buf.data(), x->stage_out, buf.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (uint32_t r = 0; r < m; ++r) {
      const uint32_t j = rows[a + r];
      std::memcpy(dep + (size_t)j * nb, buf.data() + (size_t)r * w, nb * sizeof(double));
      std::memcpy(ledger + (size_t)j * 5, buf.data() + (size_t)r * w + nb, 5 * sizeof(double));
    }
  }
  for (uint32_t sl : slots) {  // release
    x->id_to_slot.erase(x->slot_id[sl]);
    x->slot_state[sl] = 0;
    x->free_slots.push_back(sl);
  }
  return all ? EMS_OK : EMS_NOT_READY;
}

ems_status ems_run_counters(ems_ctx* x, uint64_t* steps, uint64_t* esc_hist, void* stream) {
  if (!x || !steps) return fail(EMS_E_ARG, "ems_run_counters: null argument");
  if (!x->geometry) return fail(EMS_E_STATE, "ems_run_counters: no geometry");
  hipStream_t s = (hipStream_t)stream;
  if (esc_hist) {
    HIP_OK(hipMemcpyAsync(esc_hist, x->P.esc_hist, 3 * kGrid * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
  }
  for (int i = 0; i < 3; ++i) steps[i] = x->run_steps[i];
  return EMS_OK;
}

ems_status ems_step_stats(ems_ctx* x, ems_kernel_stats* out, int32_t reset) {
  if (!x || !out) return fail(EMS_E_ARG, "ems_step_stats: null argument");
  *out = x->stats;
  if (reset) x->stats = ems_kernel_stats{};
  return EMS_OK;
}

ems_status ems_step_once(ems_ctx* x, const ems_track_soa* in, uint32_t n, ems_step_record* rec,
                         ems_track_soa* out, uint32_t* n_out, void* stream) {
  if (!x || !in || !rec || !out || !n_out) return fail(EMS_E_ARG, "ems_step_once: null argument");
  if (!x->tables || !x->geometry) return fail(EMS_E_STATE, "ems_step_once: initialise tables and geometry first");
  if (n == 0 || (uint64_t)3 * n > x->cfg.pool_capacity)
    return fail(EMS_E_CAPACITY, "ems_step_once: 3 n must fit the pool");
  hipStream_t s = (hipStream_t)stream;
  // every slot of this context is reset: step_once discards any events in flight
  reset_events(x);
  HIP_OK(launch_slots_reset(x->P, s));
  HIP_OK(launch_iter_begin(x->ctr, true, 0, 0, s));
  HIP_OK(launch_pool_load(x->P, x->set, x->cfg.pool_capacity, *in, n, s));
  HIP_OK(hipMemcpyAsync(x->h_ctr, x->ctr, kNumLines * kLineWords * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  x->nG = (uint32_t)x->h_ctr[kLAdmit * kLineWords];
  x->nC = (uint32_t)(x->h_ctr[kLAdmit * kLineWords] >> 32);
  IntervalOut io;
  ems_status st = run_interval(x, s, rec, 1, false, true, &io);
  if (st != EMS_OK) return st;
  HIP_OK(launch_pool_dump(x->pool[0][x->cur], *out, x->nG, 0, s));
  HIP_OK(launch_pool_dump(x->pool[1][x->cur], *out, x->nC, x->nG, s));
  HIP_OK(hipStreamSynchronize(s));
  *n_out = x->nG + x->nC;
  x->nG = x->nC = 0;
  return EMS_OK;
}

}  // extern "C"
