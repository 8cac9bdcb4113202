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
//   3. one readback of the counters (pool sizes, statistics, the number of events
//      that finished: the kernels mark their slots on the device).
// The step count of a track, not the iteration, keys its random numbers, so
// admission order, put-off interactions and pool size change no result.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <string>
#include <vector>

#include "emshower.h"
#include "ems_device.h"
#include "ems_batches.h"
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
// curved-move substeps per track-step of a launch (field_substeps = 0)
constexpr uint32_t kSubPerStep = 2;
constexpr uint32_t kMaxVol = 4096;
constexpr uint32_t kMaxSurf = 4096;
constexpr uint32_t kMaxFaces = 32768;

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
  // staging of one batch (submission) or one chunk of a read, max_events rows
  int64_t* stage_off = nullptr;
  uint32_t* stage_flag = nullptr;  // per event of a batch: its id was entered
  uint32_t* stage_slot = nullptr;
  uint32_t* stage_id = nullptr;
  double* stage_e = nullptr;       // per event of a batch: kinetic energy
  int32_t* stage_status = nullptr;
  double* stage_dep = nullptr;
  double* stage_led = nullptr;
  unsigned long long* stage_steps = nullptr;
  unsigned long long* stage_esc = nullptr;  // per-event escape spectra read back, or null
  unsigned long long* ctr = nullptr;
  // host mirror of the counters: pinned, or in the vector below
  bool pinned = true;
  std::vector<unsigned long long> h_ctr_buf;
  unsigned long long* h_ctr = nullptr;
  uint64_t run_steps[3] = {0, 0, 0};  // track-steps by species since init_geometry
  // event slots and ids live on the device (EvSlots); the host mirrors the number of
  // free slots and counts erased id entries (the table is rebuilt past a quarter)
  EvSlots slots{};
  uint32_t n_free = 0;
  uint64_t tombs = 0;
  bool ev_reset = true;  // the device slot state must be (re)initialised
  ems::PendingEvents pending;
  uint32_t q_head = 0, q_count = 0;
  uint64_t done_unread = 0;  // finished events not yet read
  // kinetic energy of the pool after the last sync interval (measured on the device)
  // and of the primaries admitted since
  double e_pool = 0.0, e_adm = 0.0;
  // tracks waiting in pinned host memory: a stack of SoA rows [0, spill_top)
  Pool hs{};
  void* hs_block = nullptr;
  uint64_t spill_top = 0;
  unsigned long long* spill_hist = nullptr;  // device, kGrid
  uint32_t* spill_cnt = nullptr;             // device, 4
  // per-iteration records: device staging of one interval, host log
  uint32_t* iter_log = nullptr;
  std::vector<ems_iteration_record> log;
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
  set.fsub = c.take<uint32_t>(4 * N);
  set.fh = c.take<double>(4 * N);
  set.ftrav = c.take<double>(4 * N);
  IQueue iq;
  const size_t NQ = (size_t)kNumQueues * N;
  iq.rec = c.take<uint4>(NQ * 5);
  iq.src = c.take<uint32_t>(NQ);
  iq.capacity = (uint32_t)N;
  double* tab_d = c.take<double>((size_t)kMaxMat * 3 * kGrid * kQ);
  float* tab_f = c.take<float>((size_t)kMaxMat * 3 * kGrid * kQ);
  double* gb = c.take<double>(kMaxVol + 1);
  int* gm = c.take<int>(kMaxVol);
  int* gbin = c.take<int>(kMaxVol);
  double* gsurf = c.take<double>((size_t)kMaxSurf * 10);
  unsigned char* gplane = c.take<unsigned char>(kMaxSurf);
  int* gfoff = c.take<int>(kMaxVol + 1);
  int* gfaces = c.take<int>(kMaxFaces);
  int* gcoff = c.take<int>(2 * kMaxSurf + 1);
  int* gcand = c.take<int>(kMaxFaces);
  unsigned long long* tally = c.take<unsigned long long>(E * kEvCopies * B);
  unsigned long long* ledger = c.take<unsigned long long>(E * kEvCopies * kLedger);
  int* alive = c.take<int>(E * kEvCopies);
  double* scale = c.take<double>(E);
  double* e_in = c.take<double>(E);
  unsigned long long* ctr = c.take<unsigned long long>(kNumLines * kLineWords);
  unsigned long long* esc = c.take<unsigned long long>(3 * kGrid);
  unsigned long long* life = c.take<unsigned long long>(kStatCopies * kLifeStride);
  const bool ev_esc_on = (cfg.flags & EMS_FLAG_EVENT_ESCAPE) != 0;
  unsigned long long* ev_esc = ev_esc_on ? c.take<unsigned long long>(E * 3 * kGrid) : nullptr;
  unsigned long long* stage_esc = ev_esc_on ? c.take<unsigned long long>(E * 3 * kGrid) : nullptr;
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
  uint32_t* ilog = c.take<uint32_t>(4 * kMaxPerSync);
  unsigned long long* sh = c.take<unsigned long long>(kGrid);
  uint32_t* sc = c.take<uint32_t>(4);
  uint32_t* sg = c.take<uint32_t>(E);
  uint32_t* ss = c.take<uint32_t>(E);
  uint32_t* si = c.take<uint32_t>(E);
  double* se = c.take<double>(E);
  int32_t* sst = c.take<int32_t>(E);
  double* sdep = c.take<double>(E * B);
  double* sled = c.take<double>(E * 5);
  unsigned long long* sstep = c.take<unsigned long long>(E * 3);
  size_t mcap = 16;
  while (mcap < 2 * E) mcap <<= 1;
  EvSlots ev;
  ev.words = (uint32_t)((E + 31) / 32);
  ev.bits = c.take<uint32_t>(ev.words);
  ev.pre = c.take<uint32_t>((size_t)ev.words + 1);
  ev.tile = c.take<uint32_t>((size_t)(ev.words + kFreeTile - 1) / kFreeTile + 1);
  ev.map = c.take<unsigned long long>(mcap);
  ev.mask = (uint32_t)(mcap - 1);
  ev.state = c.take<uint32_t>(E);
  ev.id = c.take<uint32_t>(E);
  ev.claim = c.take<uint32_t>(E);
  ev.n = (uint32_t)E;
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
      p.fsub = set.fsub + o;
      p.fh = set.fh + o;
      p.ftrav = set.ftrav + o;
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
  x->P.surf = gsurf;
  x->P.plane = gplane;
  x->P.face_off = gfoff;
  x->P.faces = gfaces;
  x->P.cand_off = gcoff;
  x->P.cand = gcand;
  x->P.tally = tally;
  x->P.ledger = ledger;
  x->P.alive = alive;
  x->P.scale = scale;
  x->P.slot_state = ev.state;
  x->slots = ev;
  x->P.ctr = ctr;
  x->P.esc_hist = esc;
  x->P.ev_esc = ev_esc;
  x->P.life_hist = life;
  x->stage_esc = stage_esc;
  x->scale = scale;
  x->e_in = e_in;
  x->ctr = ctr;
  x->q = q;
  x->iter_log = ilog;
  x->spill_hist = sh;
  x->spill_cnt = sc;
  x->stage_off = so;
  x->stage_flag = sg;
  x->stage_slot = ss;
  x->stage_id = si;
  x->stage_e = se;
  x->stage_status = sst;
  x->stage_dep = sdep;
  x->stage_led = sled;
  x->stage_steps = sstep;
}

// Per-event score indices must fit the 28 index bits of the kernels' score keys.
bool config_ok(const ems_config* c) {
  if (!c) return false;
  const uint64_t E = c->max_events;
  const bool ev_esc = (c->flags & EMS_FLAG_EVENT_ESCAPE) != 0;
  return c->pool_capacity >= 64 && c->pool_capacity <= (1u << 30) && E >= 1 && E < (1u << 26) &&
         c->max_bins >= 1 && E * c->max_bins < (1ull << 28) &&
         (!ev_esc || E * 3 * kGrid < (1ull << 28)) && c->queue_capacity >= 1 &&
         c->iterations_per_sync <= kMaxPerSync && c->field_substeps <= 1024 &&
         (c->flags & ~(EMS_FLAG_TIME_STEPS | EMS_FLAG_EVENT_ESCAPE)) == 0 &&
         (c->precision == EMS_FP64 || c->precision == EMS_MIXED);
}

// Forget every event: all slots free (the device side is reset by the next call that
// has a stream, see ensure_events), nothing queued, nothing in flight.
void reset_events(ems_ctx* x) {
  x->n_free = x->cfg.max_events;
  x->tombs = 0;
  x->ev_reset = true;
  x->pending.clear();
  x->q_head = 0;
  x->q_count = 0;
  x->done_unread = 0;
  x->e_pool = x->e_adm = 0.0;
  x->nG = x->nC = 0;
  x->cur = 0;
  x->spill_top = 0;
}

// Bytes of pinned host memory per spilled track (the SoA state of Pool without src,
// with the state of a suspended curved move).
constexpr size_t kHostTrackBytes = 10 * sizeof(double) + 7 * sizeof(uint32_t);

void carve_host(ems_ctx* x, uint64_t cap) {
  char* b = static_cast<char*>(x->hs_block);
  auto take = [&](size_t elem) {
    char* p = b;
    b += cap * elem;
    return p;
  };
  Pool& h = x->hs;
  h.x = reinterpret_cast<double*>(take(8));
  h.y = reinterpret_cast<double*>(take(8));
  h.z = reinterpret_cast<double*>(take(8));
  h.u = reinterpret_cast<double*>(take(8));
  h.v = reinterpret_cast<double*>(take(8));
  h.w = reinterpret_cast<double*>(take(8));
  h.T = reinterpret_cast<double*>(take(8));
  h.nlam = reinterpret_cast<double*>(take(8));
  h.k0 = reinterpret_cast<uint32_t*>(take(4));
  h.k1 = reinterpret_cast<uint32_t*>(take(4));
  h.k2 = reinterpret_cast<uint32_t*>(take(4));
  h.evt = reinterpret_cast<uint32_t*>(take(4));
  h.nstep = reinterpret_cast<uint32_t*>(take(4));
  h.meta = reinterpret_cast<uint32_t*>(take(4));
  h.src = nullptr;
  h.fsub = reinterpret_cast<uint32_t*>(take(4));
  h.fh = reinterpret_cast<double*>(take(8));
  h.ftrav = reinterpret_cast<double*>(take(8));
}

// Copy n track rows between a device pool view (from row d) and the host stack
// (from row h), in the direction `kind`.
hipError_t copy_rows(const Pool& dev, size_t d, const Pool& host, size_t h, size_t n,
                     hipMemcpyKind kind, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const bool up = kind == hipMemcpyHostToDevice;
#define EMS_COPY_FIELD(f)                                                                     \
  do {                                                                                       \
    hipError_t e_ = up ? hipMemcpyAsync(dev.f + d, host.f + h, n * sizeof(*dev.f), kind, s)  \
                       : hipMemcpyAsync(host.f + h, dev.f + d, n * sizeof(*dev.f), kind, s); \
    if (e_ != hipSuccess) return e_;                                                         \
  } while (0)
  EMS_COPY_FIELD(x);
  EMS_COPY_FIELD(y);
  EMS_COPY_FIELD(z);
  EMS_COPY_FIELD(u);
  EMS_COPY_FIELD(v);
  EMS_COPY_FIELD(w);
  EMS_COPY_FIELD(T);
  EMS_COPY_FIELD(nlam);
  EMS_COPY_FIELD(k0);
  EMS_COPY_FIELD(k1);
  EMS_COPY_FIELD(k2);
  EMS_COPY_FIELD(evt);
  EMS_COPY_FIELD(nstep);
  EMS_COPY_FIELD(meta);
  EMS_COPY_FIELD(fsub);
  EMS_COPY_FIELD(fh);
  EMS_COPY_FIELD(ftrav);
#undef EMS_COPY_FIELD
  return hipSuccess;
}

}  // namespace

namespace ems {

ems_status fail_status(ems_status s, const std::string& msg) { return fail(s, msg); }

// Context over a device workspace.  pinned: counter readbacks go to pinned host
// memory and the optional spill buffer and step timers are allowed; otherwise the
// context uses plain host memory for readbacks and refuses both, so that creating
// it calls no allocating HIP routine.
ems_status create_context(const ems_config* cfg, void* d_workspace, size_t bytes, bool pinned,
                          const char* who, ems_ctx** out) {
  const std::string w = who;
  if (!out) return fail(EMS_E_ARG, w + ": out is null");
  *out = nullptr;
  if (!config_ok(cfg)) return fail(EMS_E_ARG, w + ": invalid configuration");
  if (!pinned && (cfg->spill_capacity > 0 || (cfg->flags & EMS_FLAG_TIME_STEPS)))
    return fail(EMS_E_ARG, w + ": spill_capacity and EMS_FLAG_TIME_STEPS need ems_create");
  if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0)
    return fail(EMS_E_ARG, w + ": workspace must be non-null and 256-byte aligned");
  const size_t need = ems_workspace_bytes(cfg);
  if (bytes < need)
    return fail(EMS_E_CAPACITY, w + ": workspace of " + std::to_string(bytes) + " bytes, need " +
                                    std::to_string(need));
  ems_ctx* x = new (std::nothrow) ems_ctx();
  if (!x) return fail(EMS_E_INTERNAL, w + ": out of host memory");
  x->cfg = *cfg;
  x->pinned = pinned;
  Carver c{static_cast<char*>(d_workspace)};
  carve(c, *cfg, x);
  x->P.seed = cfg->seed;
  x->P.max_events = cfg->max_events;
  if (pinned) {
    hipError_t e = hipHostMalloc((void**)&x->h_ctr, kNumLines * kLineWords * sizeof(unsigned long long),
                                 hipHostMallocDefault);
    if (e == hipSuccess && cfg->spill_capacity > 0) {
      e = hipHostMalloc(&x->hs_block, (size_t)cfg->spill_capacity * kHostTrackBytes, hipHostMallocDefault);
      if (e == hipSuccess) carve_host(x, cfg->spill_capacity);
    }
    if (e != hipSuccess) {
      ems_destroy(x);
      return fail(EMS_E_HIP, w + ": pinned host buffer: " + hipGetErrorString(e));
    }
  } else {
    x->h_ctr_buf.assign((size_t)kNumLines * kLineWords, 0ull);
    x->h_ctr = x->h_ctr_buf.data();
  }
  x->per_sync = cfg->iterations_per_sync == 0 ? 8 : (int)cfg->iterations_per_sync;
  if (cfg->flags & EMS_FLAG_TIME_STEPS) {
    for (int j = 0; j < 2 * x->per_sync; ++j)
      if (hipEventCreate(&x->ev[j]) != hipSuccess) {
        ems_destroy(x);
        return fail(EMS_E_HIP, w + ": hipEventCreate failed");
      }
  }
  reset_events(x);
  *out = x;
  return EMS_OK;
}

}  // namespace ems

extern "C" {

const char* ems_last_error(void) { return g_err.c_str(); }

size_t ems_workspace_bytes(const ems_config* cfg) {
  if (!config_ok(cfg)) return 0;
  Carver c{nullptr};
  carve(c, *cfg, nullptr);
  return c.off;
}

ems_status ems_create(const ems_config* cfg, void* d_workspace, size_t bytes, ems_ctx** out) {
  return ems::create_context(cfg, d_workspace, bytes, true, "ems_create", out);
}

void ems_destroy(ems_ctx* x) {
  if (!x) return;
  if (x->pinned) {
    if (x->h_ctr) (void)hipHostFree(x->h_ctr);
    if (x->hs_block) (void)hipHostFree(x->hs_block);
  }
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
  P.sub_per_step = x->cfg.field_substeps == 0 ? kSubPerStep : x->cfg.field_substeps;
  P.charged_local = o->charged_local != 0;
  P.cont_loss = o->continuous_loss != 0;
  P.msc = o->msc != 0;
  x->opts = *o;
  x->tables = true;
  x->geometry = false;
  return EMS_OK;
}

ems_status init_geometry(ems_ctx* x, const ems_geometry* g, void* stream) {
  if (!x || !g || (!g->bounds && g->kind != EMS_GEOM_CSG) || !g->material || !g->tally_bin)
    return fail(EMS_E_ARG, "init_geometry: null argument");
  if (!x->tables) return fail(EMS_E_STATE, "init_geometry: call init_physics_tables first");
  if (g->kind != EMS_GEOM_SLABS && g->kind != EMS_GEOM_CYLINDERS && g->kind != EMS_GEOM_CSG)
    return fail(EMS_E_ARG, "init_geometry: unknown kind");
  const bool csg = g->kind == EMS_GEOM_CSG;
  std::vector<int> cand_off, cand;
  if (csg) {
    if (g->n_surf < 1 || (uint32_t)g->n_surf > kMaxSurf || !g->surfaces || !g->face_off || !g->faces)
      return fail(EMS_E_ARG, "init_geometry: quadric cells need 1..4096 surfaces, face offsets and faces");
    if (g->n_vol < 1 || (uint32_t)g->n_vol > kMaxVol) return fail(EMS_E_ARG, "init_geometry: 1..4096 volumes");
    if (g->face_off[0] != 0) return fail(EMS_E_ARG, "init_geometry: face_off[0] must be 0");
    for (int k = 0; k < g->n_vol; ++k)
      if (g->face_off[k + 1] < g->face_off[k])
        return fail(EMS_E_ARG, "init_geometry: face offsets must not decrease");
    const int nf = g->face_off[g->n_vol];
    if ((uint32_t)nf > kMaxFaces) return fail(EMS_E_ARG, "init_geometry: more than 32768 faces");
    for (int j = 0; j < nf; ++j)
      if (g->faces[j] < 0 || (g->faces[j] >> 1) >= g->n_surf)
        return fail(EMS_E_ARG, "init_geometry: face names an unknown surface");
    for (int j = 0; j < 10 * g->n_surf; ++j)
      if (!std::isfinite(g->surfaces[j])) return fail(EMS_E_ARG, "init_geometry: surface coefficient not finite");
    // cells entered through each face code, in increasing cell order
    cand_off.assign(2 * (size_t)g->n_surf + 1, 0);
    for (int j = 0; j < nf; ++j) cand_off[g->faces[j] + 1] += 1;
    for (size_t c = 1; c < cand_off.size(); ++c) cand_off[c] += cand_off[c - 1];
    cand.assign(nf, 0);
    std::vector<int> fill(cand_off.begin(), cand_off.end() - 1);
    for (int k = 0; k < g->n_vol; ++k)
      for (int j = g->face_off[k]; j < g->face_off[k + 1]; ++j) cand[fill[g->faces[j]]++] = k;
  }
  if (g->n_vol < 1 || (uint32_t)g->n_vol > kMaxVol) return fail(EMS_E_ARG, "init_geometry: 1..4096 volumes");
  if (g->n_bins < 1 || (uint32_t)g->n_bins > x->cfg.max_bins)
    return fail(EMS_E_ARG, "init_geometry: n_bins exceeds the configured max_bins");
  for (int i = 0; i < g->n_vol; ++i) {
    if (!csg && !(g->bounds[i + 1] > g->bounds[i])) return fail(EMS_E_ARG, "init_geometry: bounds must increase");
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
  if (csg) {
    const int nf = g->face_off[g->n_vol];
    std::vector<double> zeros(g->n_vol + 1, 0.0);
    HIP_OK(hipMemcpyAsync(x->geo_bounds, zeros.data(), sizeof(double) * (g->n_vol + 1), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync((void*)x->P.surf, g->surfaces, sizeof(double) * 10 * g->n_surf, hipMemcpyHostToDevice, s));
    std::vector<unsigned char> plane(g->n_surf);
    for (int k = 0; k < g->n_surf; ++k) {
      const double* q = g->surfaces + 10 * k;
      plane[k] = q[0] == 0.0 && q[1] == 0.0 && q[2] == 0.0 && q[3] == 0.0 && q[4] == 0.0 && q[5] == 0.0;
    }
    HIP_OK(hipMemcpyAsync((void*)x->P.plane, plane.data(), g->n_surf, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync((void*)x->P.face_off, g->face_off, sizeof(int) * (g->n_vol + 1), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync((void*)x->P.faces, g->faces, sizeof(int) * (nf > 0 ? nf : 0), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync((void*)x->P.cand_off, cand_off.data(), sizeof(int) * cand_off.size(), hipMemcpyHostToDevice, s));
    if (nf > 0) HIP_OK(hipMemcpyAsync((void*)x->P.cand, cand.data(), sizeof(int) * nf, hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));  // the host vectors go out of scope
  } else {
    HIP_OK(hipMemcpyAsync(x->geo_bounds, g->bounds, sizeof(double) * (g->n_vol + 1), hipMemcpyHostToDevice, s));
  }
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
  P.n_surf = csg ? g->n_surf : 0;
  P.n_faces = csg ? g->face_off[g->n_vol] : 0;
  HIP_OK(launch_zero_u64(x->ctr, kNumLines * kLineWords, s));
  x->run_steps[0] = x->run_steps[1] = x->run_steps[2] = 0;
  HIP_OK(launch_zero_u64(P.esc_hist, 3 * kGrid, s));
  HIP_OK(launch_zero_u64(P.life_hist, kStatCopies * kLifeStride, s));
  HIP_OK(hipStreamSynchronize(s));
  reset_events(x);
  x->geometry = true;
  return EMS_OK;
}

}  // extern "C"

namespace {

// The device slot state after creation or a reset.
ems_status ensure_events(ems_ctx* x, hipStream_t s) {
  if (!x->ev_reset) return EMS_OK;
  HIP_OK(launch_events_reset(x->slots, s));
  x->ev_reset = false;
  return EMS_OK;
}

// Erased id entries slow every probe: past a quarter of the table it is rebuilt.
ems_status maybe_rebuild(ems_ctx* x, hipStream_t s) {
  if (x->tombs * 4 <= (uint64_t)x->slots.mask + 1u) return EMS_OK;
  HIP_OK(launch_map_rebuild(x->slots, s));
  x->tombs = 0;
  return EMS_OK;
}

// Submit a batch: slots, ids and checks on the device (kernels over the batch's
// events and primaries), one synchronisation; the host keeps the batch's offsets
// (and, with an energy budget, its events' energies) for admission.
ems_status submit(ems_ctx* x, const ems_event_batch* b, hipStream_t s) {
  const uint32_t ne = b->n_events;
  if (ne == 0) return EMS_OK;
  if (!b->event_ids || !b->offsets) return fail(EMS_E_ARG, "transport_events: null ids/offsets");
  if (b->offsets[0] != 0) return fail(EMS_E_ARG, "transport_events: offsets[0] must be 0");
  if (b->offsets[ne] < (int64_t)ne)
    return fail(EMS_E_ARG, "transport_events: every event needs at least one primary");
  const uint64_t n = (uint64_t)b->offsets[ne];
  if (!b->species || !b->energy || !b->pos || !b->dir)
    return fail(EMS_E_ARG, "transport_events: null primary arrays");
  if (ne > x->n_free) return fail(EMS_E_CAPACITY, "transport_events: not enough free event slots");
  if (n + x->q_count > x->cfg.queue_capacity)
    return fail(EMS_E_CAPACITY, "transport_events: primaries exceed the queue capacity");
  {
    const ems_status st = ensure_events(x, s);
    if (st != EMS_OK) return st;
  }
  const uint32_t tail = (x->q_head + x->q_count) % x->q.capacity;
  const bool by_energy = x->cfg.energy_budget > 0.0;
  // check word of the batch: a word of the done line, unused otherwise
  unsigned long long* bad = x->ctr + kLDone * kLineWords + 1;
  std::vector<double> ev_e(by_energy ? ne : 0);
  unsigned long long badw = 0;
  hipError_t e = hipMemcpyAsync(x->stage_off, b->offsets, sizeof(int64_t) * (ne + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(x->stage_id, b->event_ids, sizeof(uint32_t) * ne, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_zero_u64(bad, 1, s);
  if (e == hipSuccess)
    e = launch_slots_take(x->slots, x->stage_id, ne, x->stage_slot, x->stage_flag, bad, s);
  if (e == hipSuccess)
    e = launch_enqueue(x->q, tail, x->stage_off, x->stage_slot, x->stage_id, ne, b->species, b->energy,
                       b->pos, b->dir, (uint32_t)n, bad, s);
  if (e == hipSuccess)
    e = launch_event_init(x->P, x->stage_off, x->stage_slot, b->energy, b->species, ne, (int64_t)n,
                          x->e_in, x->scale, x->stage_e, (int64_t)(x->cfg.pool_capacity / 4), bad, s);
  if (e == hipSuccess && by_energy)
    e = hipMemcpyAsync(ev_e.data(), x->stage_e, ne * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&badw, bad, sizeof(badw), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {  // the device state of the batch is unknown: start over
    reset_events(x);
    return fail(EMS_E_HIP, std::string("transport_events: ") + hipGetErrorString(e));
  }
  if (badw) {  // nothing is submitted: the entries made are erased, the slots stay free
    e = launch_slots_undo(x->slots, x->stage_id, x->stage_slot, x->stage_flag, ne, s);
    x->tombs += ne;
    if (e == hipSuccess && maybe_rebuild(x, s) != EMS_OK) e = hipErrorUnknown;
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      reset_events(x);
      return fail(EMS_E_HIP, std::string("transport_events: ") + hipGetErrorString(e));
    }
    if (badw & kBadEmpty)
      return fail(EMS_E_ARG, "transport_events: offsets must increase (every event needs a primary)");
    if (badw & kBadLarge)
      return fail(EMS_E_CAPACITY, "transport_events: event larger than a quarter of the pool");
    if (badw & kBadDup) return fail(EMS_E_ARG, "transport_events: duplicate event id");
    if (badw & kBadMap) return fail(EMS_E_INTERNAL, "transport_events: event id table full");
    std::string m = "transport_events: invalid primaries:";
    if (badw & kBadSpecies) m += " species not 0, 1 or 2;";
    if (badw & kBadEnergy) m += " kinetic energy not in (0, 1e5] MeV;";
    if (badw & kBadPos) m += " position not finite;";
    if (badw & kBadDir) m += " direction not a unit vector;";
    return fail(EMS_E_ARG, m);
  }
  // the caller's offsets are used in place until transport_events returns
  x->pending.push(b->offsets, ne, by_energy ? ev_e.data() : nullptr, true);
  x->n_free -= ne;
  x->q_count += (uint32_t)n;
  return EMS_OK;
}

// Admit queued events while the pool has room for their primaries (a quarter of
// its capacity, for the showers to grow) and the energy budget allows; returns the
// number of primaries appended to the pools.
ems_status admit(ems_ctx* x, hipStream_t s, uint32_t* m_out) {
  const uint64_t room = x->cfg.pool_capacity / 4;
  const Admitted a = x->pending.admit((uint64_t)x->nG + x->nC, room, x->e_pool + x->e_adm,
                                      x->cfg.energy_budget);
  const uint32_t m = (uint32_t)a.prims;
  *m_out = m;
  if (m == 0) return EMS_OK;
  x->e_adm += a.energy;
  HIP_OK(launch_admit(x->P, x->q, x->set, x->cfg.pool_capacity, x->cur, x->q_head, m, s));
  x->q_head = (x->q_head + m) % x->q.capacity;
  x->q_count -= m;
  return EMS_OK;
}

// One sync interval: up to `iters` iterations enqueued back to back (admission
// only at its start), then one readback of the counters.  Pool sizes and queue
// sizes stay on the device between iterations.  The pool is kept within `bound`
// tracks by the interaction kernel (interactions that would not fit are put off),
// so every launch covers at most `bound` tracks: twice the pool at the start of
// the interval plus a margin, or the whole capacity when full_room is set.
struct IntervalOut {
  uint64_t stepped = 0, deferred = 0, busy = 0, peak = 0, spilled = 0;
  bool stalled = false;
};

constexpr uint32_t kBoundMargin = 65536;
// steps a track may take in one transport launch while it neither interacts nor
// dies (single-step diagnostics take one); measured on the 10 GeV calorimeter,
// FP64: 3 / 4 / 5 / 6 / 7 / 8 steps 1.29 / 1.38 / 1.43 / 1.42 / 1.39 / 1.35e10
// track-steps/s; mixed: 4 / 6 steps 1.47 / 1.54e10; with a field (curved moves,
// whose substep budget scales with the steps) 4 steps beat 6 by 8 %
constexpr uint32_t kStepsPerLaunch = 5;
constexpr uint32_t kStepsPerLaunchMixed = 6;
constexpr uint32_t kStepsPerLaunchField = 4;
// a pool this small cannot fill the GPU: its launches are latency bound, so each
// takes more steps per track (the tail of a run, long-lived loopers)
constexpr uint64_t kTailTracks = 16384;
constexpr uint32_t kTailStepsPerLaunch = 32;
constexpr size_t kLogCap = size_t(1) << 20;  // iteration records kept

// Bring back tracks waiting in host memory once the pool has drained below a quarter
// of its capacity, up to half of it, last spilled first.  Runs where admission
// would: no new event is admitted while tracks wait (older work first).
ems_status unspill(ems_ctx* x, hipStream_t s) {
  const uint64_t cap = x->cfg.pool_capacity, n = (uint64_t)x->nG + x->nC;
  if (x->spill_top == 0 || n >= cap / 4) return EMS_OK;
  const uint64_t m = std::min<uint64_t>(x->spill_top, cap / 2 - n);
  const uint64_t a = x->spill_top - m;
  uint32_t mg = 0;
  for (uint64_t r = a; r < x->spill_top; ++r) mg += (x->hs.meta[r] & 3u) == EMS_GAMMA;
  // staging: the bottom of the free photon buffer
  HIP_OK(copy_rows(x->pool[0][1 - x->cur], 0, x->hs, a, m, hipMemcpyHostToDevice, s));
  HIP_OK(launch_unspill(x->P, x->set, x->cfg.pool_capacity, x->cur, (uint32_t)m, s));
  x->spill_top = a;
  x->nG += mg;
  x->nC += (uint32_t)m - mg;
  return EMS_OK;
}

// Move the tracks of the highest energies to host memory: the fewest top bins of the
// energy grid that hold at least `want` tracks, fewer if the host room is smaller.
ems_status spill(ems_ctx* x, hipStream_t s, uint64_t want, uint64_t* moved) {
  *moved = 0;
  const uint64_t room = x->cfg.spill_capacity - x->spill_top;
  const uint32_t N = x->cfg.pool_capacity;
  if (want == 0 || room == 0 || x->nG + x->nC == 0) return EMS_OK;
  std::vector<uint64_t> h(kGrid);
  HIP_OK(launch_zero_u64(x->spill_hist, kGrid, s));
  HIP_OK(launch_spill_hist(x->P, x->set, N, x->cur, x->nG, x->nC, x->spill_hist, s));
  HIP_OK(hipMemcpyAsync(h.data(), x->spill_hist, kGrid * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  int b = kGrid;
  uint64_t c = 0;
  while (b > 0 && c < want) c += h[--b];
  while (b < kGrid && c > room) c -= h[b++];
  if (c == 0) return EMS_OK;
  uint32_t cnt[4] = {0, 0, 0, 0};
  HIP_OK(launch_zero_u32(x->spill_cnt, 4, s));
  HIP_OK(launch_spill_split(x->P, x->set, N, x->cur, x->nG, x->nC, b, x->spill_cnt, s));
  HIP_OK(hipMemcpyAsync(cnt, x->spill_cnt, sizeof(cnt), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if ((uint64_t)cnt[2] + cnt[3] != c || (uint64_t)cnt[0] + cnt[1] + c != (uint64_t)x->nG + x->nC)
    return fail(EMS_E_INTERNAL, "transport_events: spill counts disagree");
  const int o = 1 - x->cur;
  HIP_OK(copy_rows(x->pool[0][o], N - cnt[2], x->hs, x->spill_top, cnt[2], hipMemcpyDeviceToHost, s));
  HIP_OK(copy_rows(x->pool[1][o], N - cnt[3], x->hs, x->spill_top + cnt[2], cnt[3],
                   hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  x->spill_top += c;
  x->cur = o;
  x->nG = cnt[0];
  x->nC = cnt[1];
  *moved = c;
  return EMS_OK;
}

ems_status run_interval(ems_ctx* x, hipStream_t s, ems_step_record* rec, int iters,
                        bool admit_first, bool full_room, IntervalOut* io) {
  HIP_OK(launch_iter_begin(x->ctr, true, x->nG, x->nC, 0, nullptr, s));
  // primaries admitted now join the pools at the device's admission cursors (the
  // split into photons and charged tracks is read back after the interval)
  uint32_t m = 0;
  if (admit_first && x->spill_top > 0) {
    const ems_status st = unspill(x, s);
    if (st != EMS_OK) return st;
  } else if (admit_first) {
    const ems_status st = admit(x, s, &m);
    if (st != EMS_OK) return st;
  }
  const uint64_t n0 = (uint64_t)x->nG + x->nC + m;
  if (n0 == 0) {
    if (admit_first && !x->pending.empty())
      return fail(EMS_E_INTERNAL, "transport_events: queued events could not be admitted");
    return EMS_OK;
  }
  const uint32_t cap = x->cfg.pool_capacity;
  const bool mixed = x->cfg.precision == EMS_MIXED;
  const uint32_t bound =
      full_room ? cap : (uint32_t)std::min<uint64_t>(cap, std::max<uint64_t>(n0, 2 * n0 + kBoundMargin));
  const uint32_t big = x->P.bz != 0.0 ? kStepsPerLaunchField : (mixed ? kStepsPerLaunchMixed : kStepsPerLaunch);
  const uint32_t msteps = full_room ? 1u : (n0 < kTailTracks ? kTailStepsPerLaunch : big);
  for (int j = 0; j < iters; ++j) {
    if (j > 0) HIP_OK(launch_iter_begin(x->ctr, false, 0, 0, (uint32_t)j, x->iter_log, s));
    if (x->ev[2 * j]) HIP_OK(hipEventRecord(x->ev[2 * j], s));
    HIP_OK(launch_iteration(x->P, x->set, cap, x->cur, x->iq, bound, msteps, mixed, rec, s));
    if (x->ev[2 * j + 1]) HIP_OK(hipEventRecord(x->ev[2 * j + 1], s));
    x->cur = 1 - x->cur;
  }
  HIP_OK(launch_done_scan(x->P, s));  // events finished during the interval
  HIP_OK(hipMemcpyAsync(x->h_ctr, x->ctr, kNumLines * kLineWords * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, s));
  uint32_t ilog[4 * kMaxPerSync];
  if (iters > 1)
    HIP_OK(hipMemcpyAsync(ilog, x->iter_log, 4 * (iters - 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const unsigned long long* L = x->h_ctr;
  unsigned long long S[kLineWords] = {};
  for (int c = 0; c < kStatCopies; ++c)
    for (int w = 0; w < kLineWords; ++w) S[w] += L[(kLStats + c) * kLineWords + w];
  S[kSPeak] = L[kLStats * kLineWords + kSPeak];
  const unsigned long long out = L[kLOut * kLineWords] + L[kLOutI * kLineWords];
  const uint32_t outG = (uint32_t)(out & 0xFFFFFFFFull), outC = (uint32_t)(out >> 32);
  const uint32_t n_done = (uint32_t)(L[kLDone * kLineWords] & 0xFFFFFFFFull);  // events finished
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
  float it_ms[kMaxPerSync] = {};
  if (x->ev[0]) {
    for (int j = 0; j < iters; ++j) {
      HIP_OK(hipEventElapsedTime(&it_ms[j], x->ev[2 * j], x->ev[2 * j + 1]));
      x->stats.kernel_ms += it_ms[j];
    }
  }
  {  // per-iteration records: the device logged all but the last, read from the counters
    const unsigned long long in_last = L[kLAdmit * kLineWords];
    for (int j = 0; j < iters && x->log.size() < kLogCap; ++j) {
      ems_iteration_record r{};
      if (j + 1 < iters) {
        r.photons = ilog[4 * j];
        r.charged = ilog[4 * j + 1];
        r.interactions = ilog[4 * j + 2];
        r.tracks_out = ilog[4 * j + 3];
      } else {
        r.photons = (uint32_t)(in_last & 0xFFFFFFFFull);
        r.charged = (uint32_t)(in_last >> 32);
        r.interactions = (uint32_t)queued_last;
        r.tracks_out = outG + outC;
      }
      if (r.photons + r.charged == 0) continue;
      r.waiting_primaries = x->pending.prims();
      r.spilled = x->spill_top;
      r.ms = it_ms[j];
      x->log.push_back(r);
    }
  }
  x->done_unread += n_done;
  x->nG = outG;
  x->nC = outC;
  unsigned long long e_kev = 0;
  for (int c = 0; c < kStatCopies; ++c) e_kev += L[(kLStats + c) * kLineWords + kSEnergy];
  x->e_pool = 1e-3 * (double)e_kev;
  x->e_adm = 0.0;
  io->stepped += S[kSStepG] + S[kSStepC];
  io->deferred += S[kSDeferred];
  io->busy += S[kSBusy];
  io->peak = std::max<uint64_t>(io->peak, S[kSPeak]);
  io->stalled = io->stalled || S[kSStall] != 0;
  return EMS_OK;
}

}  // namespace

extern "C" {

static ems_status transport_events_impl(ems_ctx* x, const ems_event_batch* b, int32_t max_iterations,
                                        void* stream, ems_progress* progress);

ems_status transport_events(ems_ctx* x, const ems_event_batch* b, int32_t max_iterations,
                            void* stream, ems_progress* progress) {
  const ems_status st = transport_events_impl(x, b, max_iterations, stream, progress);
  if (x) x->pending.keep();  // events still queued keep a copy of the batch's offsets
  return st;
}

static ems_status transport_events_impl(ems_ctx* x, const ems_event_batch* b, int32_t max_iterations,
                                        void* stream, ems_progress* progress) {
  if (!x) return fail(EMS_E_ARG, "transport_events: null context");
  if (!x->tables || !x->geometry) return fail(EMS_E_STATE, "transport_events: initialise tables and geometry first");
  hipStream_t s = (hipStream_t)stream;
  {
    const ems_status st = ensure_events(x, s);
    if (st != EMS_OK) return st;
  }
  if (b) {
    const ems_status st = submit(x, b, s);
    if (st != EMS_OK) return st;
  }
  uint64_t it = 0;
  IntervalOut io;
  io.peak = (uint64_t)x->nG + x->nC;
  const int per_sync = x->per_sync;
  const uint64_t cap = x->cfg.pool_capacity;
  while (max_iterations < 0 || it < (uint64_t)max_iterations) {
    if (x->nG + x->nC == 0 && x->pending.empty() && x->spill_top == 0) break;
    int k = per_sync;
    if (max_iterations >= 0) k = (int)std::min<uint64_t>((uint64_t)k, (uint64_t)max_iterations - it);
    ems_status st = run_interval(x, s, nullptr, k, true, false, &io);
    if (st != EMS_OK) return st;
    it += k;
    // a pool above three quarters of its capacity, or one that cannot progress,
    // sends its highest-energy tracks to host memory down to half its capacity
    const uint64_t n = (uint64_t)x->nG + x->nC;
    if (x->cfg.spill_capacity > 0 && (io.stalled || n > cap - cap / 4)) {
      uint64_t moved = 0;
      st = spill(x, s, std::max<uint64_t>(n > cap / 2 ? n - cap / 2 : 0, io.stalled ? n / 2 : 0), &moved);
      if (st != EMS_OK) return st;
      io.spilled += moved;
      if (moved) io.stalled = false;
    }
    if (io.stalled)
      return fail(EMS_E_STALLED, "transport_events: pool full of put-off interactions, no track can step");
  }
  const uint64_t stepped = io.stepped, deferred = io.deferred, peak = io.peak;
  if (progress) {
    progress->alive = (uint64_t)x->nG + x->nC;
    progress->queued_primaries = x->pending.prims();
    progress->queued_events = x->pending.events();
    progress->iterations = io.busy;
    progress->track_steps = stepped;
    progress->deferred = deferred;
    progress->peak_alive = peak;
    progress->spilled = x->spill_top;
    progress->spilled_total = io.spilled;
    progress->events_done = x->done_unread;
  }
  return EMS_OK;
}

ems_status tally_read(ems_ctx* x, uint32_t n, const uint32_t* ids, double* dep, double* ledger,
                      uint64_t* steps, uint64_t* esc_hist, int32_t* status, void* stream) {
  if (!x || (n && (!ids || !dep || !ledger || !status))) return fail(EMS_E_ARG, "tally_read: null argument");
  if (!x->geometry) return fail(EMS_E_STATE, "tally_read: no geometry");
  if (esc_hist && !x->P.ev_esc)
    return fail(EMS_E_STATE, "tally_read: per-event escape spectra need EMS_FLAG_EVENT_ESCAPE");
  hipStream_t s = (hipStream_t)stream;
  {
    const ems_status st = ensure_events(x, s);
    if (st != EMS_OK) return st;
  }
  // per chunk of at most max_events ids, on the device: the slot of each id and its
  // status, the rows of the finished events (zero for the others) copied straight
  // into the caller's arrays, then the slots released
  const uint32_t nb = (uint32_t)x->P.nbins;
  const uint32_t chunk = x->cfg.max_events;
  const uint32_t ne = 3 * kGrid;
  std::vector<unsigned long long> st3(steps ? 0 : (size_t)std::min(n, chunk) * 3);
  bool all = true;
  for (uint32_t a = 0; a < n; a += chunk) {
    const uint32_t m = std::min(chunk, n - a);
    hipError_t e = hipMemcpyAsync(x->stage_id, ids + a, m * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_read_find(x->slots, x->stage_id, m, x->stage_slot, x->stage_status, s);
    if (e == hipSuccess)
      e = launch_gather_tallies(x->P, x->stage_slot, m, x->e_in, x->stage_dep, x->stage_led,
                                x->stage_steps, esc_hist ? x->stage_esc : nullptr, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(status + a, x->stage_status, m * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dep + (size_t)a * nb, x->stage_dep, (size_t)m * nb * sizeof(double),
                         hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ledger + (size_t)a * 5, x->stage_led, (size_t)m * 5 * sizeof(double),
                         hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(steps ? steps + (size_t)a * 3 : (uint64_t*)st3.data(), x->stage_steps,
                         (size_t)m * 3 * sizeof(uint64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && esc_hist)
      e = hipMemcpyAsync(esc_hist + (size_t)a * ne, x->stage_esc, (size_t)m * ne * sizeof(uint64_t),
                         hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {  // nothing of this chunk is released: every event stays readable
      (void)launch_read_unclaim(x->slots, x->stage_slot, m, s);
      (void)hipStreamSynchronize(s);
      return fail(EMS_E_HIP, std::string("tally_read: ") + hipGetErrorString(e));
    }
    uint32_t k = 0;
    for (uint32_t j = 0; j < m; ++j) {
      k += status[a + j] == EMS_OK;
      all = all && status[a + j] == EMS_OK;
    }
    if (k) {
      HIP_OK(launch_read_release(x->slots, x->stage_id, x->stage_slot, m, s));
      x->n_free += k;
      x->done_unread -= k;
      x->tombs += k;
      const ems_status st = maybe_rebuild(x, s);
      if (st != EMS_OK) return st;
    }
  }
  HIP_OK(hipStreamSynchronize(s));
  return all ? EMS_OK : EMS_NOT_READY;
}

ems_status ems_run_counters(ems_ctx* x, uint64_t* steps, uint64_t* esc_hist, uint64_t* life_hist,
                            void* stream) {
  if (!x || !steps) return fail(EMS_E_ARG, "ems_run_counters: null argument");
  if (!x->geometry) return fail(EMS_E_STATE, "ems_run_counters: no geometry");
  hipStream_t s = (hipStream_t)stream;
  if (esc_hist)
    HIP_OK(hipMemcpyAsync(esc_hist, x->P.esc_hist, 3 * kGrid * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  std::vector<uint64_t> lh;
  if (life_hist) {
    lh.resize(kStatCopies * kLifeStride);
    HIP_OK(hipMemcpyAsync(lh.data(), x->P.life_hist, lh.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  }
  if (esc_hist || life_hist) HIP_OK(hipStreamSynchronize(s));
  if (life_hist)
    for (int b = 0; b < 3 * kLifeBins; ++b) {
      uint64_t t = 0;
      for (int c = 0; c < kStatCopies; ++c) t += lh[(size_t)c * kLifeStride + b];
      life_hist[b] = t;
    }
  for (int i = 0; i < 3; ++i) steps[i] = x->run_steps[i];
  return EMS_OK;
}

ems_status ems_iteration_log(ems_ctx* x, ems_iteration_record* out, uint64_t max, uint64_t* n,
                             int32_t reset) {
  if (!x || !n || (max > 0 && !out)) return fail(EMS_E_ARG, "ems_iteration_log: null argument");
  *n = x->log.size();
  const uint64_t m = std::min<uint64_t>(max, x->log.size());
  if (m) std::memcpy(out, x->log.data(), m * sizeof(ems_iteration_record));
  if (reset) x->log.clear();
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
  {
    const ems_status st = ensure_events(x, s);
    if (st != EMS_OK) return st;
  }
  HIP_OK(launch_slots_reset(x->P, s));
  HIP_OK(launch_iter_begin(x->ctr, true, 0, 0, 0, nullptr, s));
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
