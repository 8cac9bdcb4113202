/*
 * oracle.h -- independent CPU oracle for the electromagnetic-shower step loop.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  The product path
 * (paper_2203_09467_amd/) never links, imports or calls it, and this code
 * shares nothing with the HIP path: its own constants, closed forms, tables,
 * samplers, geometry and random-number generator, written from the physics
 * they compute.
 *
 * What it computes: plain, single-threaded, history-based FP64 Monte Carlo
 * transport of photons, electrons and positrons (paper Sec. 2.2 "Physics":
 * continuous slowing down, selection among competing discrete processes,
 * scattering/absorption, secondary emission and energy cutoffs; Table
 * "Current status of Celeritas EM physics").  Each event is a stack of
 * tracks; a track is stepped until it dies and its secondaries are pushed.
 * The GPU method is a reordering of exactly these independent histories
 * (one track per thread, paper Sec. 2.1 "Code Architecture"), so with random
 * numbers keyed by (track key, step) the two agree up to rounding.
 *
 * Units: MeV, cm, g/cm^3, tesla.  All arithmetic is double precision.
 *
 * The paper gives no formulas; every physics definition here is a textbook
 * form chosen as a reading of the paper's model list, collected in the
 * design notes together with the pins that check it.  Functions whose
 * result no pin fixes are marked "parity unpinned" at their definition.
 */
#ifndef EMS_ORACLE_H
#define EMS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_GAMMA = 0, OR_ELECTRON = 1, OR_POSITRON = 2 };
enum { OR_NGRID = 200, OR_NQ = 4, OR_MAXMAT = 8 };
enum { OR_GEOM_SLABS = 0, OR_GEOM_CYLINDERS = 1, OR_GEOM_CSG = 2 };
enum { OR_OUTSIDE = -1 };
enum { OR_LIM_GEO = 0, OR_LIM_PHYS = 1, OR_LIM_CONT = 2, OR_LIM_LOOPER = 3, OR_LIM_VACCAP = 4 };
enum { OR_VAC_CAPS = 40 }; /* consecutive substep-capped vacuum steps that make a looper */

typedef struct {
  double Z, A, density, mean_excitation; /* mean_excitation in MeV; density 0 = vacuum */
} or_material;

typedef struct {
  double tracking_cut;       /* MeV: tracks below it deposit and stop */
  double production_cut;     /* cm: range cut for delta rays / brems photons; <= 0: none */
  int compton, photoelectric, pair, ionisation, brems, annihilation; /* 0/1 enables */
  int charged_local;         /* 1: e-/e+ secondaries deposit at birth (photon-only run) */
  int continuous_loss;       /* 0 disables along-step loss (for pins only) */
  double step_alpha;         /* continuous step limit: fraction of residual range */
  double step_rfinal;        /* cm: residual range below which a track ranges out */
  uint32_t max_steps;        /* looper cap per track */
  int msc;                   /* 1: Gaussian multiple-scattering deflection of e-/e+ steps */
} or_options;

typedef struct {
  int kind;          /* OR_GEOM_SLABS: z-planes; OR_GEOM_CYLINDERS: radii */
  int n_vol;
  const double* bounds;  /* n_vol + 1 increasing values (z planes or radii) */
  const int* material;   /* per volume: material index, or -1 for vacuum */
  const int* tally_bin;  /* per volume */
  int n_bins;
  double half_x, half_y; /* slabs: lateral half widths */
  double half_z;         /* cylinders: half length */
  double bz;             /* uniform field along z, tesla (cylinders only) */
  double field_tol;      /* cm: RK4 local error tolerance */
  /* OR_GEOM_CSG: cells (the volumes) as intersections of quadric half-spaces */
  int n_surf;
  const double* surf;    /* n_surf x 10: qxx qyy qzz qxy qyz qzx px py pz k */
  const int* face_off;   /* n_vol + 1: faces of cell k are face_off[k] .. face_off[k+1]-1 */
  const int* faces;      /* surface index * 2 + (1 if the cell is on the side f > 0) */
} or_geometry;

typedef struct {
  int species;
  double x, y, z, u, v, w;
  double T;          /* kinetic energy, MeV */
  double nlam;       /* interaction lengths left; < 0 means "sample on next step" */
  uint32_t key[3];   /* 96-bit lineage key */
  uint32_t event;    /* event slot */
  uint32_t nstep;    /* steps taken so far */
  int vol;           /* current volume */
  uint32_t vac_caps; /* field: vacuum steps in a row that ended on the substep cap */
} or_track;

typedef struct {
  or_track out[3];   /* surviving parent (if any) first, then secondaries */
  int n_out;
  int parent_alive;
  double dep;        /* energy deposited in the pre-step volume */
  int dep_bin;
  double esc;        /* kinetic energy carried out of the world */
  int esc_species;   /* species of the escaping track (if esc > 0 or escaped) */
  int escaped;
  double killed;     /* energy removed by the looper cap */
  int n_pair, n_annih;
  int limiter;       /* OR_LIM_* */
  int process;       /* selected discrete process, -1 if none */
  double step_len;
} or_step_result;

typedef struct or_world or_world;

/* ---- random numbers (Salmon et al., SC'11 "Parallel random numbers: as easy as 1, 2, 3") */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_uniform(uint32_t seed, const uint32_t key[3], uint32_t step, uint32_t draw);
void or_primary_key(uint32_t seed, uint32_t event_id, uint32_t index, uint32_t out[3]);
void or_child_key(uint32_t seed, const uint32_t parent[3], uint32_t step, uint32_t ordinal,
                  uint32_t out[3]);

/* ---- closed forms (per electron or per atom, cm^2; macroscopic 1/cm) */
double or_kn_sigma(double E);                         /* Klein-Nishina, per electron */
double or_kn_dsigma(double E, double eps);            /* d sigma / d eps, eps = E'/E */
double or_pe_sigma(double Z, double E);               /* synthetic photoelectric, per atom */
double or_pair_Sigma(double X0, double E);            /* complete-screening pair, 1/cm */
double or_pair_dSigma(double X0, double E, double x); /* d Sigma / d x, x = E-/E */
double or_brems_Sigma(double X0, double T, double kc);
double or_brems_dSigma(double X0, double T, double k);
double or_brems_Srad(double X0, double T, double kc); /* soft radiative loss, MeV/cm */
double or_moller_sigma(double T, double Tc);          /* per electron */
double or_moller_dsigma(double T, double eps);        /* d sigma / d eps, eps = Tdelta/T */
double or_bhabha_sigma(double T, double Tc);
double or_bhabha_dsigma(double T, double eps);
double or_heitler_sigma(double Z, double T);          /* e+ annihilation in flight, per atom */
double or_heitler_dsigma(double Z, double T, double eps);
double or_scol(int positron, double n_el, double I, double T, double cut); /* restricted, MeV/cm */
double or_radiation_length(double Z, double A, double density);           /* cm */
double or_msc_theta0(double T, double x, double X0); /* Highland width, rad */

/* ---- samplers: draws are u[0], u[1], ... ; returns number of draws consumed */
int or_sample_kn(double E, const double* u, int nu, double* eps, double* cost);
int or_sample_pair(double E, const double* u, int nu, double* x);
int or_sample_brems(double T, double kc, const double* u, int nu, double* k);
int or_sample_moller(double T, double Tc, const double* u, int nu, double* eps);
int or_sample_bhabha(double T, double Tc, const double* u, int nu, double* eps);
int or_sample_heitler(double T, const double* u, int nu, double* eps);
double or_accept_moller(double T, double eps);  /* acceptance ratios (must lie in [0,1]) */
double or_accept_bhabha(double T, double eps);
double or_accept_heitler(double T, double eps);
double or_accept_kn(double E, double eps);

/* ---- world: materials + tables + geometry + options */
or_world* or_create(const or_material* mats, int n_mats, const or_options* opt,
                    const or_geometry* geom);
void or_destroy(or_world* w);
double or_grid_energy(const or_world* w, int i);
double or_table_node(const or_world* w, int mat, int species, int q, int i);
double or_table_interp(const or_world* w, int mat, int species, int q, double T);
double or_range_inverse(const or_world* w, int mat, int species, double r);
double or_cut_electron(const or_world* w, int mat);
double or_cut_gamma(const or_world* w, int mat);
double or_range_at_cut(const or_world* w, int mat, int species); /* R at tracking cut */
double or_material_X0(const or_world* w, int mat);
int or_locate(const or_world* w, double x, double y, double z, double u, double v, double wz);
double or_distance(const or_world* w, int vol, const double pos[3], const double dir[3],
                   int* next);

/* Quadric-surface cells (csg.c): side of a surface (+1 / -1) at p moving along d,
 * and the distance along d to where f leaves side sigma (HUGE_VAL: never). */
int or_csg_side(const double* q, const double p[3], const double d[3]);
double or_csg_exit(const double* q, const double p[3], const double d[3], int sigma);

/* Charged tracks in the uniform field B_z: curvature, one RK4 step, and the curved
 * move of a step (returns 0 at s_max, 1 at a boundary, 2 for a looper in matter,
 * 3 at the substep cap of a vacuum step). */
double or_field_kappa(double q, double bz, double p);
void or_rk4(double kappa, double h, const double r[3], const double d[3], double ro[3],
            double dout[3]);
int or_field_move(const or_world* w, int vol, double kappa, double s_max, int vacuum, double r[3],
                  double d[3], double* s_out, int* next);

/* Turn unit direction d by polar cosine c and azimuth phi about itself (the rotation
 * every interaction uses for its products); o is a unit vector. */
void or_rotate(const double d[3], double c, double phi, double o[3]);

int or_step(const or_world* w, uint32_t seed, const or_track* in, or_step_result* res);

typedef struct {
  double* dep_bins;      /* n_bins, caller-owned, accumulated */
  double esc, killed;
  long n_pair, n_annih;
  long steps[3];         /* track-steps by species */
  long tracks[3];        /* tracks created (primaries included) by species */
  double* esc_hist;      /* 3 * OR_NGRID counts of escaping energy bins, or NULL */
  double* life_hist;     /* 3 * OR_LIFE_BINS tracks ended, by species and steps taken, or NULL */
  double e_in;
} or_event_tally;

/* Transport one event (all primaries) to completion; returns 0, or -1 on error. */
int or_run_event(const or_world* w, uint32_t seed, uint32_t event_id, int n_prim,
                 const int* species, const double* T, const double* pos, const double* dir,
                 or_event_tally* tally);

/* Steps-per-track distribution (Sec. 3.2, the steps each track takes, compared between
 * codes): bin 0 holds tracks that took no step, bin b >= 1 tracks whose step count n has
 * 2^(b-1) <= n < 2^b, the last bin everything from 2^(OR_LIFE_BINS-2) up. */
#define OR_LIFE_BINS 17
int or_life_bin(long n);

int or_run_batch(const or_world* w, uint32_t seed, int n_events, const uint32_t* event_ids,
                 const int64_t* offsets, const int* species, const double* T, const double* pos,
                 const double* dir, double* dep, double* ledger, int64_t* steps, int64_t* tracks,
                 double* esc_hist, double* life_hist);

#ifdef __cplusplus
}
#endif
#endif
