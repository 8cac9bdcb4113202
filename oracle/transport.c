/*
 * transport.c -- geometry, samplers, the single step and the history loop of
 * the CPU oracle (test infrastructure only; see oracle.h).
 *
 * One step of an alive track, in the order the paper lists the physics
 * (Sec. 2.2: continuous slowing down, selection among competing discrete
 * processes, scattering/absorption, secondary emission, energy cutoffs):
 *   1. interaction lengths left: if unset, nlam = -ln u_0;
 *   2. macroscopic cross sections Sigma_i(T) of the species' processes in the
 *      current material (tables, linear in ln T), Sigma = sum; s_phys = nlam/Sigma;
 *   3. e-/e+: residual range d = R(T) - R(T_cut); s_cont = d if d <= r_f,
 *      else max(alpha d, r_f);
 *   4. straight-line distance to the volume boundary s_geo (field: RK4);
 *   5. s = min, ties resolved geometry > discrete > continuous; move;
 *   6. e-/e+: T' = R^-1(R(T) - s) (never above T); range-out deposits all of T;
 *      nlam -= s Sigma unless the step ends in an interaction;
 *   7. boundary: enter the next volume or escape; interaction: choose process i
 *      with u_1 Sigma(T') < sum_{j<=i} Sigma_j(T'), sample it from u_2, u_3, ...;
 *   8. cutoffs: tracks below the tracking cut deposit their kinetic energy; a
 *      stopped positron annihilates at rest into two 511 keV photons.
 * All of a step's deposits are scored in the pre-step volume.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

#define OR_MAXTRIAL 1000
#define OR_REST_STEP 0xFFFFFFFFu
#define OR_MSC_DRAW 0x40000000 /* first of the two draws of a step's scattering angle */

/* ------------------------------------------------------------ geometry */

int or_geometry_init(or_world* w, const or_geometry* g) {
  or_geom_data* d = &w->geo;
  memset(d, 0, sizeof(*d));
  if (g->n_vol < 1) return -1;
  d->kind = g->kind;
  d->n_vol = g->n_vol;
  d->n_bins = g->n_bins;
  if (g->kind == OR_GEOM_CSG) {
    if (g->n_surf < 1 || !g->surf || !g->face_off || !g->faces || g->face_off[0] != 0) return -1;
    const int nf = g->face_off[g->n_vol];
    d->n_surf = g->n_surf;
    d->surf = (double*)malloc(sizeof(double) * 10 * (size_t)g->n_surf);
    d->face_off = (int*)malloc(sizeof(int) * (size_t)(g->n_vol + 1));
    d->faces = (int*)malloc(sizeof(int) * (size_t)(nf > 0 ? nf : 1));
    if (!d->surf || !d->face_off || !d->faces) return -1;
    memcpy(d->surf, g->surf, sizeof(double) * 10 * (size_t)g->n_surf);
    memcpy(d->face_off, g->face_off, sizeof(int) * (size_t)(g->n_vol + 1));
    memcpy(d->faces, g->faces, sizeof(int) * (size_t)nf);
    for (int k = 0; k < g->n_vol; ++k)
      if (g->face_off[k + 1] < g->face_off[k]) return -1;
    for (int j = 0; j < nf; ++j)
      if (g->faces[j] < 0 || (g->faces[j] >> 1) >= g->n_surf) return -1;
  }
  d->bounds = (double*)malloc(sizeof(double) * (size_t)(g->n_vol + 1));
  d->material = (int*)malloc(sizeof(int) * (size_t)g->n_vol);
  d->bin = (int*)malloc(sizeof(int) * (size_t)g->n_vol);
  if (!d->bounds || !d->material || !d->bin) return -1;
  if (g->bounds) memcpy(d->bounds, g->bounds, sizeof(double) * (size_t)(g->n_vol + 1));
  else memset(d->bounds, 0, sizeof(double) * (size_t)(g->n_vol + 1));
  memcpy(d->material, g->material, sizeof(int) * (size_t)g->n_vol);
  memcpy(d->bin, g->tally_bin, sizeof(int) * (size_t)g->n_vol);
  for (int i = 0; i < g->n_vol; ++i)
    if (d->material[i] >= w->n_mats || d->bin[i] < 0 || d->bin[i] >= g->n_bins) return -1;
  d->hx = g->half_x;
  d->hy = g->half_y;
  d->hz = g->half_z;
  d->bz = g->bz;
  d->tol = g->field_tol;
  return 0;
}

void or_geometry_free(or_world* w) {
  free(w->geo.bounds);
  free(w->geo.material);
  free(w->geo.bin);
  free(w->geo.surf);
  free(w->geo.face_off);
  free(w->geo.faces);
}

/* Volume containing the point; on a surface the direction decides. */
int or_locate(const or_world* w, double x, double y, double z, double u, double v, double wz) {
  const or_geom_data* g = &w->geo;
  if (g->kind == OR_GEOM_CSG) {
    const double p[3] = {x, y, z}, d[3] = {u, v, wz};
    return or_csg_locate(g, p, d);
  }
  if (g->kind == OR_GEOM_SLABS) {
    if (fabs(x) > g->hx || fabs(y) > g->hy) return OR_OUTSIDE;
    for (int j = 0; j < g->n_vol; ++j) {
      const double lo = g->bounds[j], hi = g->bounds[j + 1];
      if ((z > lo && z < hi) || (z == lo && wz >= 0.0) || (z == hi && wz < 0.0)) return j;
    }
    return OR_OUTSIDE;
  }
  if (fabs(z) > g->hz) return OR_OUTSIDE;
  const double r = sqrt(x * x + y * y);
  const double rd = x * u + y * v; /* sign of dr/ds */
  for (int j = 0; j < g->n_vol; ++j) {
    const double lo = g->bounds[j], hi = g->bounds[j + 1];
    if ((r > lo && r < hi) || (r == lo && rd >= 0.0) || (r == hi && rd < 0.0)) return j;
  }
  return OR_OUTSIDE;
}

/* Straight-line distance from pos along dir to the boundary of volume vol and the
 * volume entered there.  Slabs: planes z = bounds[vol], bounds[vol+1] lead to the
 * neighbours, lateral walls |x| = hx, |y| = hy to the outside; ties go to the walls.
 * Cylinders: the outer radius leads outward, the inner radius inward, the end caps
 * |z| = hz outside; ties go inner, then caps. */
double or_distance(const or_world* w, int vol, const double p[3], const double d[3], int* next) {
  const or_geom_data* g = &w->geo;
  const double INF = HUGE_VAL;
  double s = INF;
  int nx = OR_OUTSIDE;
  if (g->kind == OR_GEOM_CSG) return or_csg_distance(g, vol, p, d, next);
  if (g->kind == OR_GEOM_SLABS) {
    if (d[2] > 0.0) {
      s = (g->bounds[vol + 1] - p[2]) / d[2];
      nx = vol + 1 < g->n_vol ? vol + 1 : OR_OUTSIDE;
    } else if (d[2] < 0.0) {
      s = (g->bounds[vol] - p[2]) / d[2];
      nx = vol - 1 >= 0 ? vol - 1 : OR_OUTSIDE;
    }
    double sx = INF, sy = INF;
    if (d[0] > 0.0) sx = (g->hx - p[0]) / d[0];
    else if (d[0] < 0.0) sx = (-g->hx - p[0]) / d[0];
    if (d[1] > 0.0) sy = (g->hy - p[1]) / d[1];
    else if (d[1] < 0.0) sy = (-g->hy - p[1]) / d[1];
    if (sx <= s) {
      s = sx;
      nx = OR_OUTSIDE;
    }
    if (sy <= s) {
      s = sy;
      nx = OR_OUTSIDE;
    }
  } else {
    const double a = d[0] * d[0] + d[1] * d[1];
    const double b = p[0] * d[0] + p[1] * d[1];
    const double r2 = p[0] * p[0] + p[1] * p[1];
    if (a > 0.0) {
      /* outer surface: the root where the ray leaves the disc of radius R */
      const double R = g->bounds[vol + 1];
      const double c = r2 - R * R;
      double D = b * b - a * c;
      if (D < 0.0) D = 0.0;
      const double sq = sqrt(D);
      s = (b <= 0.0) ? (-b + sq) / a : -c / (b + sq);
      nx = vol + 1 < g->n_vol ? vol + 1 : OR_OUTSIDE;
      if (vol > 0 && b < 0.0) {
        const double Ri = g->bounds[vol];
        const double ci = r2 - Ri * Ri;
        const double Di = b * b - a * ci;
        if (Di >= 0.0) {
          const double si = ci / (-b + sqrt(Di));
          if (si <= s) {
            s = si;
            nx = vol - 1;
          }
        }
      }
    }
    double sz = INF;
    if (d[2] > 0.0) sz = (g->hz - p[2]) / d[2];
    else if (d[2] < 0.0) sz = (-g->hz - p[2]) / d[2];
    if (sz <= s) {
      s = sz;
      nx = OR_OUTSIDE;
    }
  }
  if (s < 0.0) s = 0.0;
  *next = nx;
  return s;
}

/* ------------------------------------------------------------ draws */

typedef struct {
  const double* arr; /* explicit draws, or NULL for the track's Philox stream */
  int n;
  uint32_t seed;
  const uint32_t* key;
  uint32_t step;
  int pos;
  int err;
} drawsrc;

static double next_u(drawsrc* s) {
  if (s->arr) {
    if (s->pos >= s->n) {
      s->err = 1;
      ++s->pos;
      return 0.5;
    }
    return s->arr[s->pos++];
  }
  return or_uniform(s->seed, s->key, s->step, (uint32_t)(s->pos++));
}

/* ------------------------------------------------------------ samplers */
/* Each rejection sampler draws (candidate, test) pairs until the test passes,
 * at most OR_MAXTRIAL times (the last candidate is then taken). */

double or_accept_kn(double E, double eps) {
  const double k = E / OR_ME;
  const double c = 1.0 - (1.0 - eps) / (k * eps);
  const double s2 = (1.0 - c) * (1.0 + c);
  return (1.0 + eps * eps - eps * s2) / 2.0;
}

/* Compton: eps = eps0^u on [eps0, 1] (a 1/eps envelope), accept with
 * (1 + eps^2 - eps sin^2 theta)/2. */
static void kn_sample(double E, drawsrc* s, double* eps, double* cost) {
  const double k = E / OR_ME;
  const double leps0 = -log(1.0 + 2.0 * k);
  double e = 1.0;
  for (int t = 0; t < OR_MAXTRIAL; ++t) {
    const double ua = next_u(s), ub = next_u(s);
    e = exp(ua * leps0);
    if (ub < or_accept_kn(E, e)) break;
  }
  *eps = e;
  *cost = 1.0 - (1.0 - e) / (k * e);
}

/* Pair: x uniform on [a, 1-a], accept with 1 - 4/3 x (1-x). */
static double pair_sample(double E, drawsrc* s) {
  const double a = OR_ME / E;
  double x = 0.5;
  for (int t = 0; t < OR_MAXTRIAL; ++t) {
    const double ua = next_u(s), ub = next_u(s);
    x = a + (1.0 - 2.0 * a) * ua;
    if (ub < 1.0 - 4.0 / 3.0 * x * (1.0 - x)) break;
  }
  return x;
}

/* Brems: k = kc (T/kc)^u (a 1/k envelope), accept with 1 - y + 3/4 y^2, y = k/T. */
static double brems_sample(double T, double kc, drawsrc* s) {
  const double L = log(T / kc);
  double k = kc;
  for (int t = 0; t < OR_MAXTRIAL; ++t) {
    const double ua = next_u(s), ub = next_u(s);
    k = kc * exp(ua * L);
    const double y = k / T;
    if (ub < 1.0 - y + 0.75 * y * y) break;
  }
  return k;
}

/* Moller: 1/eps^2 envelope on [x, 1/2], accept with eps^2 f(eps) / max, where the
 * maximum of eps^2 f over (0, 1/2] is (9g^2 - 10g + 5)/(4 g^2), reached at 1/2. */
double or_accept_moller(double T, double eps) {
  const double g = T / OR_ME + 1.0;
  const double c = (2.0 * g - 1.0) / (g * g);
  const double r = (g - 1.0) / g;
  const double f = r * r + 1.0 / (eps * eps) - c / eps + 1.0 / ((1.0 - eps) * (1.0 - eps)) -
                   c / (1.0 - eps);
  return eps * eps * f * 4.0 * g * g / (9.0 * g * g - 10.0 * g + 5.0);
}

static double moller_sample(double T, double Tc, drawsrc* s) {
  const double xi = T / Tc; /* 1/x */
  double e = 0.5;
  for (int t = 0; t < OR_MAXTRIAL; ++t) {
    const double ua = next_u(s), ub = next_u(s);
    e = 1.0 / (xi - ua * (xi - 2.0));
    if (ub < or_accept_moller(T, e)) break;
  }
  return e;
}

/* Bhabha: 1/eps^2 envelope on [x, 1], accept with beta^2 eps^2 f(eps) (<= 1). */
double or_accept_bhabha(double T, double eps) {
  const double g = T / OR_ME + 1.0;
  const double b2 = 1.0 - 1.0 / (g * g);
  const double y = 1.0 / (g + 1.0);
  const double h = 1.0 - 2.0 * y;
  const double B1 = 2.0 - y * y, B2 = h * (3.0 + y * y), B4 = h * h * h, B3 = B4 + h * h;
  const double f = 1.0 / (b2 * eps * eps) - B1 / eps + B2 - B3 * eps + B4 * eps * eps;
  return b2 * eps * eps * f;
}

static double bhabha_sample(double T, double Tc, drawsrc* s) {
  const double xi = T / Tc;
  double e = 1.0;
  for (int t = 0; t < OR_MAXTRIAL; ++t) {
    const double ua = next_u(s), ub = next_u(s);
    e = 1.0 / (xi - ua * (xi - 1.0));
    if (ub < or_accept_bhabha(T, e)) break;
  }
  return e;
}

/* Annihilation in flight: 1/eps envelope on [eps_min, 1-eps_min], accept with
 * eps S(eps) / (g^2 + 2g - 1), the maximum of eps S at eps = 1/(g+1). */
double or_accept_heitler(double T, double eps) {
  const double g = T / OR_ME + 1.0;
  const double S = -(g + 1.0) * (g + 1.0) + (g * g + 4.0 * g + 1.0) / eps - 1.0 / (eps * eps);
  return eps * S / (g * g + 2.0 * g - 1.0);
}

static double heitler_emin(double T) {
  const double g = T / OR_ME + 1.0;
  return 0.5 * (1.0 - sqrt((g - 1.0) / (g + 1.0)));
}

static double heitler_sample(double T, drawsrc* s) {
  const double emin = heitler_emin(T);
  const double L = log((1.0 - emin) / emin);
  double e = 0.5;
  for (int t = 0; t < OR_MAXTRIAL; ++t) {
    const double ua = next_u(s), ub = next_u(s);
    e = emin * exp(ua * L);
    if (ub < or_accept_heitler(T, e)) break;
  }
  return e;
}

/* Array-fed wrappers for sampling tests: return draws consumed, -1 if too few. */
int or_sample_kn(double E, const double* u, int nu, double* eps, double* cost) {
  drawsrc s = {u, nu, 0, NULL, 0, 0, 0};
  kn_sample(E, &s, eps, cost);
  return s.err ? -1 : s.pos;
}
int or_sample_pair(double E, const double* u, int nu, double* x) {
  drawsrc s = {u, nu, 0, NULL, 0, 0, 0};
  *x = pair_sample(E, &s);
  return s.err ? -1 : s.pos;
}
int or_sample_brems(double T, double kc, const double* u, int nu, double* k) {
  drawsrc s = {u, nu, 0, NULL, 0, 0, 0};
  *k = brems_sample(T, kc, &s);
  return s.err ? -1 : s.pos;
}
int or_sample_moller(double T, double Tc, const double* u, int nu, double* eps) {
  drawsrc s = {u, nu, 0, NULL, 0, 0, 0};
  *eps = moller_sample(T, Tc, &s);
  return s.err ? -1 : s.pos;
}
int or_sample_bhabha(double T, double Tc, const double* u, int nu, double* eps) {
  drawsrc s = {u, nu, 0, NULL, 0, 0, 0};
  *eps = bhabha_sample(T, Tc, &s);
  return s.err ? -1 : s.pos;
}
int or_sample_heitler(double T, const double* u, int nu, double* eps) {
  drawsrc s = {u, nu, 0, NULL, 0, 0, 0};
  *eps = heitler_sample(T, &s);
  return s.err ? -1 : s.pos;
}

/* ------------------------------------------------------------ kinematics */

/* Turn direction d by polar cosine c and azimuth phi about d itself:
 * new = c d + s cos(phi) e1 + s sin(phi) e2 with e1 = (u w, v w, -p)/p,
 * e2 = (-v, u, 0)/p, p = sqrt(u^2+v^2); along the z axis (p^2 <= 1e-20) the
 * frame is the lab frame.  The result is renormalised. */
static void rotate(const double d[3], double c, double phi, double o[3]) {
  double s = 1.0 - c * c;
  s = s > 0.0 ? sqrt(s) : 0.0;
  const double cp = cos(phi), sp = sin(phi);
  const double p2 = d[0] * d[0] + d[1] * d[1];
  if (p2 > 1e-20) {
    const double p = sqrt(p2);
    o[0] = c * d[0] + s * (d[0] * d[2] * cp - d[1] * sp) / p;
    o[1] = c * d[1] + s * (d[1] * d[2] * cp + d[0] * sp) / p;
    o[2] = c * d[2] - s * p * cp;
  } else {
    o[0] = s * cp;
    o[1] = s * sp;
    o[2] = d[2] >= 0.0 ? c : -c;
  }
  const double n = sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
  o[0] /= n;
  o[1] /= n;
  o[2] /= n;
}

/* Exported for the pins of the rotation (test infrastructure). */
void or_rotate(const double d[3], double c, double phi, double o[3]) { rotate(d, c, phi, o); }

/* direction of a p_a - b p_b */
static void momentum_diff(double a, const double da[3], double b, const double db[3], double o[3]) {
  o[0] = a * da[0] - b * db[0];
  o[1] = a * da[1] - b * db[1];
  o[2] = a * da[2] - b * db[2];
  const double n = sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
  if (n > 0.0) {
    o[0] /= n;
    o[1] /= n;
    o[2] /= n;
  } else {
    o[0] = da[0];
    o[1] = da[1];
    o[2] = da[2];
  }
}

/* ------------------------------------------------------------ the step */

typedef struct {
  or_step_result* r;
  const or_world* w;
  uint32_t seed;
  const or_track* parent; /* post-step parent (position, volume, event) */
} emitter;

static void add_track(emitter* e, int species, double T, const double dir[3], const uint32_t key[3]) {
  or_step_result* r = e->r;
  or_track* t = &r->out[r->n_out++];
  *t = *e->parent;
  t->species = species;
  t->T = T;
  t->u = dir[0];
  t->v = dir[1];
  t->w = dir[2];
  t->nlam = -1.0;
  t->nstep = 0;
  t->vac_caps = 0;
  t->key[0] = key[0];
  t->key[1] = key[1];
  t->key[2] = key[2];
}

/* Positron annihilating at rest at the parent's position: two photons of m c^2,
 * back to back, isotropic, drawn from the positron's own stream at step
 * 0xFFFFFFFF (u_0 -> cos theta = 2u-1, u_1 -> phi = 2 pi u). */
static void annihilate_at_rest(emitter* e, const uint32_t pkey[3]) {
  drawsrc s = {NULL, 0, e->seed, pkey, OR_REST_STEP, 0, 0};
  const double c = 2.0 * next_u(&s) - 1.0;
  const double phi = 2.0 * OR_PI * next_u(&s);
  double st = 1.0 - c * c;
  st = st > 0.0 ? sqrt(st) : 0.0;
  const double d1[3] = {st * cos(phi), st * sin(phi), c};
  const double d2[3] = {-d1[0], -d1[1], -d1[2]};
  uint32_t k[3];
  e->r->n_annih += 1;
  or_child_key(e->seed, pkey, OR_REST_STEP, 0, k);
  add_track(e, OR_GAMMA, OR_ME, d1, k);
  or_child_key(e->seed, pkey, OR_REST_STEP, 1, k);
  add_track(e, OR_GAMMA, OR_ME, d2, k);
}

/* A secondary born in an interaction: tracked if at or above the tracking cut
 * (and charged particles are tracked), otherwise its kinetic energy is deposited;
 * a positron that is not tracked annihilates at rest. */
static void emit(emitter* e, int species, double T, const double dir[3], uint32_t ordinal) {
  const or_world* w = e->w;
  uint32_t k[3];
  or_child_key(e->seed, e->parent->key, e->parent->nstep, ordinal, k);
  const int charged = species != OR_GAMMA;
  if (T >= w->opt.tracking_cut && !(charged && w->opt.charged_local)) {
    add_track(e, species, T, dir, k);
    return;
  }
  e->r->dep += T;
  if (species == OR_POSITRON) annihilate_at_rest(e, k);
}

static void cross_sections(const or_world* w, const or_mat_data* m, int sp, double T, double lnT,
                           double sig[3]) {
  for (int q = 0; q < 3; ++q) sig[q] = or_interp_ln(w, m->tab[sp][q], lnT);
  /* thresholds: no interpolated cross section below a process's kinematic limit */
  if (sp == OR_GAMMA) {
    if (T <= 2.0 * OR_ME) sig[2] = 0.0;
  } else {
    if (sp == OR_ELECTRON ? (T <= 2.0 * m->Tc) : (T <= m->Tc)) sig[0] = 0.0;
    if (T <= m->kc) sig[1] = 0.0;
    if (sp == OR_ELECTRON) sig[2] = 0.0;
  }
}

int or_step(const or_world* w, uint32_t seed, const or_track* in, or_step_result* r) {
  memset(r, 0, sizeof(*r));
  r->process = -1;
  or_track t = *in;
  const or_geom_data* g = &w->geo;
  if (t.vol < 0 || t.vol >= g->n_vol) return -1;
  const int mi = g->material[t.vol];
  const or_mat_data* m = mi >= 0 ? &w->mat[mi] : NULL;
  const int in_matter = m && !m->vacuum;
  const int sp = t.species;
  const int charged = sp != OR_GAMMA;
  r->dep_bin = g->bin[t.vol];

  drawsrc st = {NULL, 0, seed, t.key, t.nstep, 0, 0};
  const double INF = HUGE_VAL;
  const double lnT = log(t.T);

  if (t.nlam < 0.0) {
    st.pos = 0;
    t.nlam = -log(next_u(&st));
  }
  double sig[3] = {0, 0, 0}, sigtot = 0.0;
  if (in_matter) {
    cross_sections(w, m, sp, t.T, lnT, sig);
    sigtot = sig[0] + sig[1] + sig[2];
  }
  const double s_phys = sigtot > 0.0 ? t.nlam / sigtot : INF;

  double s_cont = INF, R0 = 0.0, dres = 0.0;
  const int lossy = charged && in_matter && w->opt.continuous_loss;
  if (lossy) {
    R0 = or_interp_ln(w, m->tab[sp][3], lnT);
    dres = R0 - m->Rtrk[sp];
    s_cont = dres <= w->opt.step_rfinal ? dres : fmax(w->opt.step_alpha * dres, w->opt.step_rfinal);
    if (s_cont < 0.0) s_cont = 0.0;
  }

  double pos[3] = {t.x, t.y, t.z}, dir[3] = {t.u, t.v, t.w};
  int next = OR_OUTSIDE;
  int lim;
  double s;
  if (charged && g->bz != 0.0) {
    /* curved path up to the physics limit; the boundary, if met first, wins */
    const double p = sqrt(t.T * (t.T + 2.0 * OR_ME));
    const double kappa = or_field_kappa(sp == OR_ELECTRON ? -1.0 : 1.0, g->bz, p);
    const int res = or_field_move(w, t.vol, kappa, fmin(s_phys, s_cont), !in_matter, pos, dir, &s,
                                  &next);
    if (res == 1) lim = OR_LIM_GEO;
    else if (res == 2) lim = OR_LIM_LOOPER;
    else if (res == 3) lim = t.vac_caps + 1 >= OR_VAC_CAPS ? OR_LIM_LOOPER : OR_LIM_VACCAP;
    else lim = s_phys <= s_cont ? OR_LIM_PHYS : OR_LIM_CONT;
    t.vac_caps = res == 3 ? t.vac_caps + 1 : 0;
  } else {
    const double s_geo = or_distance(w, t.vol, pos, dir, &next);
    if (s_geo <= s_phys && s_geo <= s_cont) {
      lim = OR_LIM_GEO;
      s = s_geo;
    } else if (s_phys <= s_cont) {
      lim = OR_LIM_PHYS;
      s = s_phys;
    } else {
      lim = OR_LIM_CONT;
      s = s_cont;
    }
    pos[0] += s * dir[0];
    pos[1] += s * dir[1];
    pos[2] += s * dir[2];
  }
  r->limiter = lim;
  r->step_len = s;

  double T1 = t.T, lnT1 = lnT;
  int stopped = 0;
  if (lossy) {
    if (lim == OR_LIM_CONT && dres <= w->opt.step_rfinal) {
      r->dep += t.T;
      T1 = 0.0;
      stopped = 1;
    } else {
      lnT1 = or_inverse_ln(w, m->tab[sp][3], R0 - s);
      T1 = exp(lnT1);
      if (T1 > t.T) {
        T1 = t.T;
        lnT1 = lnT;
      }
      r->dep += t.T - T1;
    }
  }
  if (lim != OR_LIM_PHYS && sigtot > 0.0) t.nlam -= s * sigtot;

  /* multiple scattering of an e-/e+ still moving in matter at the end of the step */
  if (w->opt.msc && charged && in_matter && s > 0.0 && !stopped && T1 >= w->opt.tracking_cut &&
      lim != OR_LIM_LOOPER && !(lim == OR_LIM_GEO && next == OR_OUTSIDE)) {
    const double th0 = or_msc_theta0(t.T, s, m->X0);
    st.pos = OR_MSC_DRAW;
    const double ua = next_u(&st), ub = next_u(&st);
    double th = th0 * sqrt(-2.0 * log(ua));
    if (th > OR_PI) th = OR_PI;
    double nd[3];
    rotate(dir, cos(th), 2.0 * OR_PI * ub, nd);
    dir[0] = nd[0];
    dir[1] = nd[1];
    dir[2] = nd[2];
  }

  /* post-step state of the parent */
  or_track post = t;
  post.x = pos[0];
  post.y = pos[1];
  post.z = pos[2];
  post.T = T1;
  post.u = dir[0];
  post.v = dir[1];
  post.w = dir[2];
  emitter em = {r, w, seed, &post};
  /* emit() keys children by the parent's pre-increment step */
  post.nstep = t.nstep;

  int alive = 1;
  if (stopped) {
    alive = 0;
    if (sp == OR_POSITRON) annihilate_at_rest(&em, t.key);
  } else if (charged && T1 < w->opt.tracking_cut) {
    r->dep += T1;
    alive = 0;
    if (sp == OR_POSITRON) annihilate_at_rest(&em, t.key);
  } else if (lim == OR_LIM_LOOPER) {
    r->killed += T1;
    alive = 0;
  } else if (lim == OR_LIM_GEO) {
    if (next == OR_OUTSIDE) {
      r->esc += T1;
      r->escaped = 1;
      r->esc_species = sp;
      alive = 0;
    } else {
      post.vol = next;
    }
  } else if (lim == OR_LIM_PHYS) {
    post.nlam = -1.0;
    double s2[3] = {0, 0, 0}, tot2 = 0.0;
    cross_sections(w, m, sp, T1, lnT1, s2);
    tot2 = s2[0] + s2[1] + s2[2];
    if (tot2 > 0.0) {
      st.pos = 1;
      const double target = next_u(&st) * tot2;
      int p = -1;
      double cum = 0.0;
      for (int q = 0; q < 3; ++q) {
        cum += s2[q];
        if (target < cum) {
          p = q;
          break;
        }
      }
      if (p < 0)
        for (int q = 2; q >= 0; --q)
          if (s2[q] > 0.0) {
            p = q;
            break;
          }
      r->process = p;
      st.pos = 2;
      if (sp == OR_GAMMA) {
        const double E = T1;
        if (p == 0) { /* Compton */
          double eps, cost;
          kn_sample(E, &st, &eps, &cost);
          const double phi = 2.0 * OR_PI * next_u(&st);
          const double E1 = eps * E;
          const double Te = E - E1;
          double d1[3], de[3];
          rotate(dir, cost, phi, d1);
          momentum_diff(E, dir, E1, d1, de);
          if (E1 >= w->opt.tracking_cut) {
            post.T = E1;
            post.u = d1[0];
            post.v = d1[1];
            post.w = d1[2];
          } else {
            r->dep += E1;
            alive = 0;
          }
          emit(&em, OR_ELECTRON, Te, de, 0);
        } else if (p == 1) { /* photoelectric: full absorption, electron along the photon */
          alive = 0;
          emit(&em, OR_ELECTRON, E, dir, 0);
        } else { /* pair */
          const double x = pair_sample(E, &st);
          const double Tm = x * E - OR_ME;
          const double Tp = (E - 2.0 * OR_ME) - Tm;
          alive = 0;
          r->n_pair += 1;
          emit(&em, OR_ELECTRON, Tm, dir, 0);
          emit(&em, OR_POSITRON, Tp, dir, 1);
        }
      } else {
        if (p == 0) { /* Moller / Bhabha delta ray */
          const double eps = sp == OR_ELECTRON ? moller_sample(T1, m->Tc, &st)
                                                : bhabha_sample(T1, m->Tc, &st);
          const double phi = 2.0 * OR_PI * next_u(&st);
          const double Td = eps * T1;
          const double Tp = T1 - Td;
          double cd = sqrt(Td * (T1 + 2.0 * OR_ME) / (T1 * (Td + 2.0 * OR_ME)));
          if (cd > 1.0) cd = 1.0;
          double dd[3], dp[3];
          rotate(dir, cd, phi, dd);
          const double P1 = sqrt(T1 * (T1 + 2.0 * OR_ME));
          const double Pd = sqrt(Td * (Td + 2.0 * OR_ME));
          momentum_diff(P1, dir, Pd, dd, dp);
          post.T = Tp;
          post.u = dp[0];
          post.v = dp[1];
          post.w = dp[2];
          if (Tp < w->opt.tracking_cut) {
            r->dep += Tp;
            alive = 0;
            if (sp == OR_POSITRON) annihilate_at_rest(&em, t.key);
          }
          emit(&em, OR_ELECTRON, Td, dd, 0);
        } else if (p == 1) { /* bremsstrahlung: photon along the parent direction */
          const double k = brems_sample(T1, m->kc, &st);
          const double Tp = T1 - k;
          post.T = Tp;
          if (Tp < w->opt.tracking_cut) {
            r->dep += Tp;
            alive = 0;
            if (sp == OR_POSITRON) annihilate_at_rest(&em, t.key);
          }
          emit(&em, OR_GAMMA, k, dir, 0);
        } else { /* annihilation in flight into two photons */
          const double eps = heitler_sample(T1, &st);
          const double phi = 2.0 * OR_PI * next_u(&st);
          const double gm = T1 / OR_ME + 1.0;
          const double Etot = T1 + 2.0 * OR_ME;
          const double E1 = eps * Etot;
          const double E2 = Etot - E1;
          double c1 = (eps * (gm + 1.0) - 1.0) / (eps * sqrt(gm * gm - 1.0));
          if (c1 > 1.0) c1 = 1.0;
          if (c1 < -1.0) c1 = -1.0;
          double d1[3], d2[3];
          rotate(dir, c1, phi, d1);
          const double P = sqrt(T1 * (T1 + 2.0 * OR_ME));
          momentum_diff(P, dir, E1, d1, d2);
          alive = 0;
          r->n_annih += 1;
          emit(&em, OR_GAMMA, E1, d1, 0);
          emit(&em, OR_GAMMA, E2, d2, 1);
        }
      }
    }
  }

  post.nstep = t.nstep + 1;
  if (alive && post.nstep >= w->opt.max_steps) {
    r->killed += post.T;
    alive = 0;
  }
  r->parent_alive = alive;
  if (alive) {
    /* the surviving parent goes first */
    for (int i = r->n_out; i > 0; --i) r->out[i] = r->out[i - 1];
    r->out[0] = post;
    r->n_out += 1;
  }
  return 0;
}

/* ------------------------------------------------------------ histories */

static int esc_bin(const or_world* w, double E) {
  const double t = (log(E) - w->lnE0) / w->dlnE;
  if (!(t > 0.0)) return 0;
  if (t >= (double)(OR_NGRID - 1)) return OR_NGRID - 1;
  return (int)floor(t);
}

int or_life_bin(long n) {
  int b = 0;
  while (n > 0 && b < OR_LIFE_BINS - 1) {  /* b = number of binary digits of n */
    n >>= 1;
    b += 1;
  }
  return b;
}

int or_run_event(const or_world* w, uint32_t seed, uint32_t event_id, int n_prim,
                 const int* species, const double* T, const double* pos, const double* dir,
                 or_event_tally* tl) {
  size_t cap = 1024, n = 0;
  or_track* stack = (or_track*)malloc(cap * sizeof(or_track));
  if (!stack) return -1;
  for (int i = 0; i < n_prim; ++i) {
    tl->e_in += T[i];
    tl->tracks[species[i]] += 1;
    const int vol = or_locate(w, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], dir[3 * i],
                              dir[3 * i + 1], dir[3 * i + 2]);
    if (vol == OR_OUTSIDE) {
      tl->esc += T[i];
      if (tl->esc_hist) tl->esc_hist[species[i] * OR_NGRID + esc_bin(w, T[i])] += 1.0;
      if (tl->life_hist) tl->life_hist[species[i] * OR_LIFE_BINS + 0] += 1.0;
      continue;
    }
    if (n == cap) {
      cap *= 2;
      or_track* ns = (or_track*)realloc(stack, cap * sizeof(or_track));
      if (!ns) {
        free(stack);
        return -1;
      }
      stack = ns;
    }
    or_track* t = &stack[n++];
    memset(t, 0, sizeof(*t));
    t->species = species[i];
    t->x = pos[3 * i];
    t->y = pos[3 * i + 1];
    t->z = pos[3 * i + 2];
    t->u = dir[3 * i];
    t->v = dir[3 * i + 1];
    t->w = dir[3 * i + 2];
    t->T = T[i];
    t->nlam = -1.0;
    t->event = event_id;
    t->nstep = 0;
    t->vol = vol;
    or_primary_key(seed, event_id, (uint32_t)i, t->key);
  }
  or_step_result r;
  while (n > 0) {
    or_track t = stack[--n];
    for (;;) {
      if (or_step(w, seed, &t, &r) != 0) {
        free(stack);
        return -1;
      }
      tl->steps[t.species] += 1;
      tl->dep_bins[r.dep_bin] += r.dep;
      tl->esc += r.esc;
      tl->killed += r.killed;
      tl->n_pair += r.n_pair;
      tl->n_annih += r.n_annih;
      if (r.escaped && tl->esc_hist) {
        const double Eesc = r.esc;
        tl->esc_hist[r.esc_species * OR_NGRID + esc_bin(w, Eesc)] += 1.0;
      }
      const int first_sec = r.parent_alive ? 1 : 0;
      for (int i = first_sec; i < r.n_out; ++i) {
        if (n == cap) {
          cap *= 2;
          or_track* ns = (or_track*)realloc(stack, cap * sizeof(or_track));
          if (!ns) {
            free(stack);
            return -1;
          }
          stack = ns;
        }
        stack[n++] = r.out[i];
        tl->tracks[r.out[i].species] += 1;
      }
      if (!r.parent_alive) {
        if (tl->life_hist) tl->life_hist[t.species * OR_LIFE_BINS + or_life_bin((long)t.nstep + 1)] += 1.0;
        break;
      }
      t = r.out[0];
    }
  }
  free(stack);
  return 0;
}

/* Run events [0, n_events) of a batch; primaries of event e are rows
 * offsets[e] .. offsets[e+1]-1.  dep is n_events x n_bins (accumulated),
 * ledger is n_events x 5 (e_in, escaped, killed, n_pair, n_annih),
 * steps/tracks are per species (accumulated), esc_hist is 3 x OR_NGRID or NULL,
 * life_hist is 3 x OR_LIFE_BINS or NULL (both accumulated). */
int or_run_batch(const or_world* w, uint32_t seed, int n_events, const uint32_t* event_ids,
                 const int64_t* offsets, const int* species, const double* T, const double* pos,
                 const double* dir, double* dep, double* ledger, int64_t* steps, int64_t* tracks,
                 double* esc_hist, double* life_hist) {
  const int nb = w->geo.n_bins;
  for (int e = 0; e < n_events; ++e) {
    const int64_t a = offsets[e], b = offsets[e + 1];
    or_event_tally tl;
    memset(&tl, 0, sizeof(tl));
    tl.dep_bins = dep + (size_t)e * (size_t)nb;
    tl.esc_hist = esc_hist;
    tl.life_hist = life_hist;
    if (or_run_event(w, seed, event_ids[e], (int)(b - a), species + a, T + a, pos + 3 * a,
                     dir + 3 * a, &tl) != 0)
      return -1;
    double* L = ledger + (size_t)e * 5;
    L[0] = tl.e_in;
    L[1] = tl.esc;
    L[2] = tl.killed;
    L[3] = (double)tl.n_pair;
    L[4] = (double)tl.n_annih;
    for (int s = 0; s < 3; ++s) {
      steps[s] += tl.steps[s];
      tracks[s] += tl.tracks[s];
    }
  }
  return 0;
}
