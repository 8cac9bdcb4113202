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
 *    changed no state; ems_last_error() gives a message (thread-local).
 *    EMS_NOT_READY (1) means "try later", not an error.
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
  EMS_E_INTERNAL = -5
} ems_status;

typedef enum { EMS_FP64 = 0, EMS_MIXED = 1 } ems_precision;
typedef enum { EMS_GAMMA = 0, EMS_ELECTRON = 1, EMS_POSITRON = 2 } ems_species;
typedef enum { EMS_GEOM_SLABS = 0, EMS_GEOM_CYLINDERS = 1 } ems_geometry_kind;

/* Sizes fixed at creation. */
typedef struct {
  uint32_t pool_capacity;   /* track slots (tracks in flight), >= 64 */
  uint32_t max_events;      /* event slots: events submitted and not yet read */
  uint32_t max_bins;        /* tally bins per event (>= the geometry's n_bins) */
  uint32_t queue_capacity;  /* primaries waiting for admission */
  uint32_t seed;            /* random stream seed of the run */
  ems_precision precision;  /* arithmetic of cross sections, interpolation and sampling */
  double energy_budget;     /* MeV of primary energy admitted at once; <= 0: unlimited */
  uint32_t flags;           /* EMS_FLAG_* */
  uint32_t iterations_per_sync; /* step iterations enqueued per host synchronisation
                                   (admission and completion bookkeeping happen at
                                   synchronisations); 0 = 8, at most 32 */
} ems_config;

/* flags: time every step-kernel launch with HIP events on the launch stream */
#define EMS_FLAG_TIME_STEPS 1u

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
} ems_physics_options;

/* Volumes are slabs between z-planes (lateral walls |x| <= half_x, |y| <= half_y)
 * or shells between radii (|z| <= half_z), listed inside-out / front-to-back. */
typedef struct {
  int32_t kind;              /* ems_geometry_kind */
  int32_t n_vol;
  const double* bounds;      /* host, n_vol + 1 increasing planes or radii */
  const int32_t* material;   /* host, n_vol material indices (-1 = vacuum) */
  const int32_t* tally_bin;  /* host, n_vol bins in [0, n_bins) */
  int32_t n_bins;
  double half_x, half_y, half_z;
  double bz;                 /* uniform field along z, tesla (charged tracks follow RK4
                                substeps; 0 = straight lines) */
  double field_tol;          /* cm: RK4 position error and boundary sagitta tolerance */
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
} ems_progress;

/* Per-track single-step record (diagnostics and parity tests). */
typedef struct {
  double dep, esc, killed, step_len;
  int32_t limiter;  /* 0 boundary, 1 discrete interaction, 2 continuous-loss limit,
                       3 looper in the field (killed) */
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
} ems_track_soa;

/* Bytes of workspace ems_create() needs for `cfg` (0 if cfg is invalid). */
size_t ems_workspace_bytes(const ems_config* cfg);

/* Carve the caller's device workspace (>= ems_workspace_bytes(cfg) bytes, 256-byte
 * aligned) into the pool, tables, tallies and queues.  *out owns no device memory. */
ems_status ems_create(const ems_config* cfg, void* d_workspace, size_t bytes, ems_ctx** out);
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
 * Events are admitted whole, in submission order, while pool slots and the
 * energy budget allow; tracks of all admitted events share the pool and are
 * stepped together (an iteration = one transport launch, in which a track takes
 * up to four steps while it neither interacts nor dies, then one interaction
 * launch; interactions that would overflow the pool are put off to a later
 * iteration, which changes no result).  EMS_E_ARG (nothing submitted) for an
 * invalid primary: species, energy, position or direction.  EMS_E_CAPACITY if the batch does not fit
 * the free event slots or the queue (nothing submitted), or if the pool can no
 * longer make progress.  progress (host) may be NULL. */
ems_status transport_events(ems_ctx* ctx, const ems_event_batch* batch, int32_t max_iterations,
                            void* stream, ems_progress* progress);

/* Read finished events: dep (host, n x n_bins) energy per tally bin, ledger
 * (host, n x 5: primary energy, escaped kinetic energy, killed energy, pair
 * conversions, annihilations), status (host, n): EMS_OK, EMS_NOT_READY (still in
 * flight) or EMS_E_ARG (unknown id).  A read event's slot is released.
 * Returns EMS_OK if every id was read. */
ems_status tally_read(ems_ctx* ctx, uint32_t n, const uint32_t* event_ids, double* dep,
                      double* ledger, int32_t* status, void* stream);

/* Run-level counters: steps (host, 3) track-steps by species, esc_hist (host,
 * 3 x 200 or NULL) escaping tracks by species and log-energy bin of the grid. */
ems_status ems_run_counters(ems_ctx* ctx, uint64_t* steps, uint64_t* esc_hist, void* stream);

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
