/*
 * emshower.h -- C ABI of the MI355X electromagnetic-shower step loop.
 *
 * The library transports photons, electrons and positrons through a simple
 * volume geometry, one track per GPU lane, stepping every track in flight
 * once per iteration over a device-resident track pool (paper Sec. 2.1
 * "Code Architecture": one thread per track, immutable shared parameter data
 * separated from per-track state, a fixed-capacity secondary allocator
 * reserved by atomic add; Sec. 3.2: many tracks in flight, events batched to
 * fill the device).  Physics per step follows Sec. 2.2 ("Physics"): tabulated
 * macroscopic cross sections of all processes, continuous slowing down,
 * selection among competing discrete processes, interaction sampling with
 * secondary emission, and energy cutoffs.
 *
 * Conventions for every call:
 *  - Units: MeV, cm, g/cm^3, tesla.  Values cross the ABI in double precision
 *    whatever the arithmetic precision of the run.
 *  - Ownership: the caller owns all device memory.  One workspace, sized by
 *    ems_workspace_bytes(), is handed to ems_create(); the library never
 *    allocates device memory and never frees the workspace.  Pointers marked
 *    "device" must point into device memory (e.g. a torch tensor on the GPU);
 *    pointers marked "host" into host memory.  Inputs are consumed (copied or
 *    read by kernels enqueued on `stream`) before the call returns on that
 *    stream; outputs marked "host" are complete when the call returns.
 *  - Streams: `stream` is a hipStream_t (NULL = default stream); all device
 *    work of a call is enqueued on it.  Calls on one context must not overlap.
 *  - Errors: no exception crosses the ABI.  A negative status means the call
 *    changed no state -- except EMS_E_STALLED, see transport_events --;
 *    ems_last_error() gives a message (thread-local).  EMS_NOT_READY (1) means
 *    "try later", not an error.
 */
#ifndef EMSHOWER_H
#define EMSHOWER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ems_ctx ems_ctx;

typedef enum {
  EMS_OK = 0,
  EMS_NOT_READY = 1,
  EMS_E_ARG = -1,      /* invalid argument (null, out of range, inconsistent sizes) */
  EMS_E_STATE = -2,    /* call out of order (tables before geometry before transport) */
  EMS_E_CAPACITY = -3, /* workspace, event slots, pending queue or pool exhausted */
  EMS_E_HIP = -4,      /* HIP runtime error */
  EMS_E_INTERNAL = -5,
  EMS_E_STALLED = -6   /* the track pool cannot progress (see transport_events); the
                          batch of the call was accepted and stays submitted */
} ems_status;

typedef enum { EMS_FP64 = 0, EMS_MIXED = 1 } ems_precision;
typedef enum { EMS_GAMMA = 0, EMS_ELECTRON = 1, EMS_POSITRON = 2 } ems_species;
typedef enum { EMS_GEOM_SLABS = 0, EMS_GEOM_CYLINDERS = 1, EMS_GEOM_CSG = 2 } ems_geometry_kind;

/* Sizes fixed at creation. */
typedef struct {
  uint32_t pool_capacity;   /* track slots (tracks in flight), >= 64 */
  uint32_t max_events;      /* event slots: events submitted and not yet read */
  uint32_t max_bins;        /* tally bins per event (>= the geometry's n_bins) */
  uint32_t queue_capacity;  /* primaries waiting for admission */
  uint32_t seed;            /* random stream seed of the run */
  ems_precision precision;  /* arithmetic of cross sections, interpolation and sampling */
  double energy_budget;     /* MeV: whole events are admitted while the kinetic energy of
                               the tracks in the pool (measured on the device at each
                               host synchronisation) plus that of the primaries admitted
                               since stays within it; <= 0: unlimited */
  uint32_t flags;           /* EMS_FLAG_* */
  uint32_t iterations_per_sync; /* step iterations enqueued per host synchronisation
                                   (admission and completion bookkeeping happen at
                                   synchronisations); 0 = 8, at most 32 */
  uint32_t spill_capacity;  /* tracks that may wait in pinned host memory when the pool
                               runs full (108 B each, allocated by ems_create); 0 = none */
  uint32_t field_substeps;  /* with a field: curved-move substeps a charged track may take
                               per step of one launch (a launch takes up to 4 steps, 32 for
                               a small pool); a move that needs more is suspended and
                               continued by the next launch exactly where it stood, so
                               results do not depend on it.  0 = 2, at most 1024 */
} ems_config;

/* flags: time every step-kernel launch with HIP events on the launch stream */
#define EMS_FLAG_TIME_STEPS 1u
/* flags: keep an escape spectrum per event (3 species x 200 log-energy bins of the
 * table grid, 4.8 KB of workspace per event slot, twice), read by tally_read */
#define EMS_FLAG_EVENT_ESCAPE 2u

/* Step-kernel statistics accumulated since creation or the last reset. */
typedef struct {
  uint64_t launches;
  uint64_t tracks_in;   /* tracks read by the transport kernel per launch, summed */
  uint64_t tracks_out;  /* tracks written (survivors + secondaries) */
  uint64_t queued;      /* tracks passed from transport to the interaction kernel */
  double kernel_ms;     /* summed durations (EMS_FLAG_TIME_STEPS), else 0 */
} ems_kernel_stats;

/* One material: element Z, atomic weight A (g/mol), density (g/cm^3; 0 = vacuum),
 * mean excitation energy I (MeV). */
typedef struct {
  double Z, A, density, mean_excitation;
} ems_material;

typedef struct {
  double tracking_cut;    /* MeV: tracks below it deposit their energy and stop */
  double production_cut;  /* cm: range cut converted per material into the delta-ray
                             and brems-photon thresholds; <= 0: both = tracking cut */
  int32_t compton, photoelectric, pair, ionisation, brems, annihilation; /* 0/1 */
  int32_t charged_local;  /* 1: e-/e+ secondaries deposit at birth (photon-only run) */
  int32_t continuous_loss;/* 1: along-step energy loss of e-/e+ */
  double step_alpha;      /* continuous step limit: fraction of residual range */
  double step_rfinal;     /* cm: residual range below which a track ranges out */
  uint32_t max_steps;     /* per-track step cap (loopers); energy goes to "killed" */
  int32_t msc;            /* 1: multiple-scattering deflection of e-/e+ steps in matter
                             (Gaussian, Highland width; paper Table "Current status of
                             Celeritas EM physics" lists multiple scattering in progress) */
} ems_physics_options;

/* Volumes are slabs between z-planes (lateral walls |x| <= half_x, |y| <= half_y),
 * shells between radii (|z| <= half_z), listed inside-out / front-to-back, or
 * quadric-surface cells (paper Sec. 2.3 "Geometry and EM fields": the ORANGE
 * model of cells bounded by quadric surfaces, one level): each cell is the
 * intersection of half-spaces f_s < 0 or f_s > 0 of surfaces
 *   f(x) = qxx x^2 + qyy y^2 + qzz z^2 + qxy xy + qyz yz + qzx zx + px x + py y + pz z + k,
 * and a point outside every cell is outside the world.  A track leaves its cell
 * at the nearest root, over the cell's faces, where f turns to the other side
 * (the first face listed wins ties); it enters the first cell (in index order)
 * that has the crossed surface on the other side and whose remaining faces hold
 * at the crossing point, else the first other cell without the crossed surface
 * on the side left that holds it, else it escapes.  On a surface, the direction
 * of motion decides the side.  Cells must not overlap. */
typedef struct {
  int32_t kind;              /* ems_geometry_kind */
  int32_t n_vol;             /* volumes (cells) */
  const double* bounds;      /* host, n_vol + 1 increasing planes or radii (ignored for
                                EMS_GEOM_CSG) */
  const int32_t* material;   /* host, n_vol material indices (-1 = vacuum) */
  const int32_t* tally_bin;  /* host, n_vol bins in [0, n_bins) */
  int32_t n_bins;
  double half_x, half_y, half_z;
  double bz;                 /* uniform field along z, tesla (charged tracks follow RK4
                                substeps; 0 = straight lines) */
  double field_tol;          /* cm: RK4 position error and boundary sagitta tolerance */
  /* EMS_GEOM_CSG only (else ignored): */
  int32_t n_surf;            /* surfaces, 1 .. 4096 */
  const double* surfaces;    /* host, n_surf x 10: qxx qyy qzz qxy qyz qzx px py pz k */
  const int32_t* face_off;   /* host, n_vol + 1: cell k has faces face_off[k] .. face_off[k+1]-1
                                (at most 32768 faces in all) */
  const int32_t* faces;      /* host: surface * 2 + (1 if the cell lies where f > 0) */
} ems_geometry;

/* Primaries of a batch of events; rows of event e are offsets[e] .. offsets[e+1]-1. */
typedef struct {
  uint32_t n_events;
  const uint32_t* event_ids; /* host, caller-chosen ids, unique among unread events */
  const int64_t* offsets;    /* host, n_events + 1 */
  const int32_t* species;    /* device, n_primaries */
  const double* energy;      /* device, kinetic energies, MeV, in (0, 1e5] (the tables' range) */
  const double* pos;         /* device, n_primaries x 3 (row-major) */
  const double* dir;         /* device, n_primaries x 3, unit vectors (|d|^2 within 1e-6 of 1) */
} ems_event_batch;

typedef struct {
  uint64_t alive;            /* tracks in flight after the call */
  uint64_t queued_primaries; /* primaries waiting for admission */
  uint64_t queued_events;
  uint64_t iterations;       /* step iterations run by this call */
  uint64_t track_steps;      /* track-steps taken by this call */
  uint64_t deferred;         /* interactions put off for lack of pool room (the track
                                returns to the pool and does it in a later iteration) */
  uint64_t peak_alive;       /* largest pool occupancy seen by this call */
  uint64_t spilled;          /* tracks waiting in host memory after the call */
  uint64_t spilled_total;    /* tracks moved to host memory by this call */
  uint64_t events_done;      /* finished events not yet read (tally_read) */
} ems_progress;

/* One step iteration of a transport_events call (paper Sec. 3.2, "Preliminary
 * results": tracks in flight and queued per step iteration, and the time each
 * iteration takes). */
typedef struct {
  uint32_t photons, charged; /* tracks in the pool when the iteration starts */
  uint32_t interactions;     /* tracks queued for an interaction, put-off ones included */
  uint32_t tracks_out;       /* tracks in the pool after the iteration */
  uint64_t waiting_primaries;/* primaries queued for admission (at the sync interval start) */
  uint64_t spilled;          /* tracks waiting in host memory (at the sync interval start) */
  double ms;                 /* step-kernel time of the iteration (EMS_FLAG_TIME_STEPS), else 0 */
} ems_iteration_record;

/* Per-track single-step record (diagnostics and parity tests). */
typedef struct {
  double dep, esc, killed, step_len;
  int32_t limiter;  /* 0 boundary, 1 discrete interaction, 2 continuous-loss limit,
                       3 looper in the field (killed), 4 a field step in vacuum that
                       ended on its substep cap (the track goes on) */
  int32_t process;  /* selected process, -1 none */
  int32_t n_pair, n_annih;
  int32_t n_out;    /* outputs: surviving parent + secondaries */
  int32_t escaped;
} ems_step_record;

/* Track states in structure-of-arrays form (device pointers, n entries each). */
typedef struct {
  double *x, *y, *z, *u, *v, *w, *T, *nlam;
  uint32_t *k0, *k1, *k2, *event, *nstep;
  int32_t *species, *vol;
  uint32_t* vcap;   /* field steps in vacuum that ended on their substep cap, in a row
                       (0 .. 39); may be NULL (all 0 / not written) */
} ems_track_soa;

/* Bytes of workspace ems_create() needs for `cfg` (0 if cfg is invalid). */
size_t ems_workspace_bytes(const ems_config* cfg);

/* Carve the caller's device workspace (>= ems_workspace_bytes(cfg) bytes, 256-byte
 * aligned) into the pool, tables, tallies and queues.  *out owns no device memory.
 * Paper Sec. 2.1 ("Code Architecture"): immutable parameter data (tables, geometry)
 * kept apart from per-track state, and secondaries reserved in a large device array
 * of fixed capacity; here every such array is sized once, from cfg, and lives in
 * the one workspace.  EMS_E_ARG for an invalid cfg or a misaligned workspace,
 * EMS_E_CAPACITY for a workspace smaller than needed. */
ems_status ems_create(const ems_config* cfg, void* d_workspace, size_t bytes, ems_ctx** out);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): as ems_create, but the
 * workspace is the library's static device scratch of 256 MiB, which every GPU the
 * library runs on holds until the process ends; the context uses the device that
 * is current at this call.  Allocates no device or pinned host memory and creates
 * no HIP object (host bookkeeping uses the C++ heap).  EMS_E_CAPACITY if
 * ems_workspace_bytes(cfg) exceeds 256 MiB; EMS_E_ARG for an invalid cfg, a
 * spill_capacity > 0 or EMS_FLAG_TIME_STEPS (both need allocations).  Every
 * static context on one GPU shares the one scratch: creating a second one, or
 * using two at once, races -- use one at a time per device (destroy, then create
 * again).  The scratch keeps what the last context left; init_physics_tables,
 * init_geometry and submission clear what must start at zero. */
ems_status ems_create_static(const ems_config* cfg, ems_ctx** out);
void ems_destroy(ems_ctx* ctx);
const char* ems_last_error(void);

/* Build the physics tables (paper Sec. 2.2: cross sections are pre-tabulated and
 * loaded to the device at initialisation): per material, the macroscopic cross
 * section of every process and the e-/e+ range on a 200-point log grid from 1 keV
 * to 100 GeV, the production thresholds from the range cut, in FP64 and FP32.
 * mats: host, n_mats <= 8.  Must precede init_geometry. */
ems_status init_physics_tables(ems_ctx* ctx, const ems_material* mats, int32_t n_mats,
                               const ems_physics_options* opts, void* stream);

/* Load the volume geometry and its scoring map (paper Sec. 2.4: the client
 * declares scoring regions, configured into kernel tally fields).  Material
 * indices must exist.  Resets the pool and all event slots. */
ems_status init_geometry(ems_ctx* ctx, const ems_geometry* geom, void* stream);

/* Submit a batch (may be NULL or empty) to the pending queue, then run up to
 * max_iterations step iterations (< 0: until every submitted event is done).
 * Paper Sec. 2.4 ("User-interface and I/O"): the device is used best with many
 * events in flight at once; Sec. 3.2 ("Preliminary results"): a step iteration is
 * several kernels with synchronisation points, run until the tracks of the
 * events drain.  Events are admitted whole, in submission order, while pool slots
 * and the energy budget allow; tracks of all admitted events share the pool and
 * are stepped together (an iteration = one transport launch, in which a track
 * takes up to four steps while it neither interacts nor dies, then one
 * interaction launch; interactions that would overflow the pool are put off to a
 * later iteration, which changes no result).  Calls may be bounded and repeated
 * (serving): the state of events in flight stays on the device between calls.
 * Errors: EMS_E_ARG (nothing submitted) for an invalid primary: species, energy,
 * position or direction, or a duplicate event id.  EMS_E_CAPACITY (nothing
 * submitted) if the batch does not fit the free event slots or the queue.
 * EMS_E_STALLED if the pool is full of interactions put off for lack of room, so
 * that no track can step: the batch stays submitted and every event stays in
 * flight; the context can still be read and destroyed.  progress (host) may be
 * NULL. */
ems_status transport_events(ems_ctx* ctx, const ems_event_batch* batch, int32_t max_iterations,
                            void* stream, ems_progress* progress);

/* Read finished events (paper Sec. 2.4: scoring regions declared by the client,
 * tallied in kernel code on the device and processed on the host):
 *   dep (host, n x n_bins): energy deposited per tally bin;
 *   ledger (host, n x 5): primary kinetic energy, escaped kinetic energy, killed
 *     energy, pair conversions, annihilations;
 *   steps (host, n x 3, or NULL): track-steps of photons, electrons, positrons;
 *   esc_hist (host, n x 3 x 200, or NULL; needs EMS_FLAG_EVENT_ESCAPE, else
 *     EMS_E_STATE): escaping tracks by species and log-energy bin of the grid;
 *   status (host, n): EMS_OK, EMS_NOT_READY (still in flight) or EMS_E_ARG
 *     (unknown id, or an id repeated in this call: only its first entry is read).
 * Rows whose status is not EMS_OK are zero.  A read event's slot is released.
 * The ids are looked up on the device, in chunks of max_events.  Returns EMS_OK if
 * every id was read, EMS_NOT_READY otherwise; EMS_E_HIP releases nothing of the
 * chunk it happened in. */
ems_status tally_read(ems_ctx* ctx, uint32_t n, const uint32_t* event_ids, double* dep,
                      double* ledger, uint64_t* steps, uint64_t* esc_hist, int32_t* status,
                      void* stream);

/* Run-level counters since init_geometry: steps (host, 3) track-steps by species,
 * esc_hist (host, 3 x 200 or NULL) escaping tracks by species and log-energy bin of
 * the grid, life_hist (host, 3 x 17 or NULL) tracks ended by species and steps taken
 * (bin 0: none, bin b: 2^(b-1) .. 2^b - 1 steps, bin 16: 32768 or more) -- the
 * steps-per-track distribution the paper compares between codes (Sec. 3.2,
 * "Preliminary results"). */
ems_status ems_run_counters(ems_ctx* ctx, uint64_t* steps, uint64_t* esc_hist, uint64_t* life_hist,
                            void* stream);

/* The iterations recorded since creation or the last reset (the first 2^20 of them;
 * iterations with an empty pool are not recorded): *n = how many; the first
 * min(*n, max) are copied to out (host, may be NULL when max = 0).  reset != 0
 * clears the record after reading. */
ems_status ems_iteration_log(ems_ctx* ctx, ems_iteration_record* out, uint64_t max, uint64_t* n,
                             int32_t reset);

/* Step-kernel statistics of the context (host *out); reset != 0 zeroes them after
 * reading. */
ems_status ems_step_stats(ems_ctx* ctx, ems_kernel_stats* out, int32_t reset);

/* Diagnostics: discard every event of the context, replace the pool by n states
 * (device SoA; 3n <= pool_capacity; event < max_events) and step every track once
 * with the production step kernel, writing records[i] (device, n) for input i;
 * copy the pool (surviving parents and secondaries, in no particular order) to
 * out (device SoA with room for 3n), *n_out (host).  States naming no valid
 * species, volume or event slot are dropped.  No admission runs. */
ems_status ems_step_once(ems_ctx* ctx, const ems_track_soa* in, uint32_t n,
                         ems_step_record* records, ems_track_soa* out, uint32_t* n_out,
                         void* stream);

#ifdef __cplusplus
}
#endif
#endif
