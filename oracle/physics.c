/*
 * physics.c -- closed-form cross sections, stopping powers and the tabulated
 * physics of the oracle (test infrastructure only; see oracle.h).
 *
 * The paper names the processes and models (Sec. 2.2, Table "Current status
 * of Celeritas EM physics": Bethe-Heitler conversion, Klein-Nishina Compton,
 * photoelectric effect, Moller-Bhabha ionisation, bremsstrahlung, EPlusGG
 * annihilation) and says cross sections are pre-tabulated at initialisation
 * (Sec. 2.2, last paragraph).  It prints no formulas, so each one below is
 * the textbook form named in its comment; the photoelectric law and the
 * 1 keV - 100 GeV, 200-point log grid are the ones the benchmark
 * configuration states.
 *
 * Tabulation (a reading): values at the grid nodes are the closed forms;
 * between nodes a quantity is linear in ln E.  The e-/e+ range R(T) is the
 * integral of dT/S(T) from the first grid node, accumulated node to node by
 * 8-point Gauss-Legendre quadrature in ln T of T/S(T); its inverse is the
 * exact inverse of the same piecewise-linear form.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

/* CODATA 2018 */
const double OR_ME = 0.51099895000;        /* electron mass, MeV */
const double OR_RE = 2.8179403262e-13;     /* classical electron radius, cm */
const double OR_NA = 6.02214076e23;        /* Avogadro, 1/mol */
const double OR_PI = 3.14159265358979323846;

/* ------------------------------------------------------------------ photons */

/* Klein-Nishina total cross section per electron (Klein & Nishina 1929),
 * k = E / (m c^2). */
double or_kn_sigma(double E) {
  const double k = E / OR_ME;
  const double a = 1.0 + 2.0 * k;
  const double L = log(a);
  const double t1 = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / a - L / k);
  const double t2 = L / (2.0 * k);
  const double t3 = (1.0 + 3.0 * k) / (a * a);
  return 2.0 * OR_PI * OR_RE * OR_RE * (t1 + t2 - t3);
}

/* d sigma / d eps per electron, eps = E'/E in [1/(1+2k), 1]:
 * (pi r_e^2 / k) (eps + 1/eps - sin^2 theta), cos theta = 1 - (1-eps)/(k eps). */
double or_kn_dsigma(double E, double eps) {
  const double k = E / OR_ME;
  const double c = 1.0 - (1.0 - eps) / (k * eps);
  const double s2 = (1.0 - c) * (1.0 + c);
  return OR_PI * OR_RE * OR_RE / k * (eps + 1.0 / eps - s2);
}

/* Synthetic photoelectric law of the benchmark: 1 barn * Z^5 * (100 keV/E)^3.5 * 1e-6
 * per atom.  parity unpinned beyond its own definition (no Livermore data). */
double or_pe_sigma(double Z, double E) {
  return 1.0e-30 * pow(Z, 5.0) * pow(0.1 / E, 3.5);
}

/* Complete-screening pair production (Tsai / PDG "passage of particles through
 * matter", high-energy form) with kinematic limits x in [a, 1-a], a = m/E:
 * d Sigma / dx = (1/X0) (1 - 4/3 x (1-x)). */
double or_pair_dSigma(double X0, double E, double x) {
  (void)E;
  return (1.0 - 4.0 / 3.0 * x * (1.0 - x)) / X0;
}

static double pair_g(double x) { return x * x / 2.0 - x * x * x / 3.0; }

double or_pair_Sigma(double X0, double E) {
  if (E <= 2.0 * OR_ME) return 0.0;
  const double a = OR_ME / E;
  return ((1.0 - 2.0 * a) - 4.0 / 3.0 * (pair_g(1.0 - a) - pair_g(a))) / X0;
}

/* --------------------------------------------------------- bremsstrahlung */

/* PDG complete-screening spectrum with y = k/T (T kinetic):
 * d Sigma / dk = (1/(X0 k)) (4/3 - 4/3 y + y^2), 0 < k <= T. */
double or_brems_dSigma(double X0, double T, double k) {
  const double y = k / T;
  return (4.0 / 3.0 - 4.0 / 3.0 * y + y * y) / (X0 * k);
}

/* Integral of d Sigma/dk over (kc, T]. */
double or_brems_Sigma(double X0, double T, double kc) {
  if (T <= kc) return 0.0;
  return (4.0 / 3.0 * log(T / kc) - 4.0 / 3.0 * (T - kc) / T + (T * T - kc * kc) / (2.0 * T * T)) / X0;
}

/* Integral of k d Sigma/dk over (0, min(kc,T)]: energy radiated below the cut. */
double or_brems_Srad(double X0, double T, double kc) {
  const double k = kc < T ? kc : T;
  return (4.0 / 3.0 * k - 2.0 / 3.0 * k * k / T + k * k * k / (3.0 * T * T)) / X0;
}

/* ----------------------------------------------------- Moller / Bhabha */

/* Moller cross section (Moller 1932) per target electron, differential in
 * eps = T_delta / T:  (2 pi r_e^2 m / (beta^2 T)) [ ((g-1)/g)^2 + 1/eps^2
 *   - (2g-1)/(g^2 eps) + 1/(1-eps)^2 - (2g-1)/(g^2 (1-eps)) ]. */
double or_moller_dsigma(double T, double eps) {
  const double g = T / OR_ME + 1.0;
  const double b2 = 1.0 - 1.0 / (g * g);
  const double c = (2.0 * g - 1.0) / (g * g);
  const double r = (g - 1.0) / g;
  const double f = r * r + 1.0 / (eps * eps) - c / eps + 1.0 / ((1.0 - eps) * (1.0 - eps)) -
                   c / (1.0 - eps);
  return 2.0 * OR_PI * OR_RE * OR_RE * OR_ME / (b2 * T) * f;
}

/* Integral over eps in [x, 1/2], x = Tc/T (delta rays above the cut). */
double or_moller_sigma(double T, double Tc) {
  if (T <= 2.0 * Tc) return 0.0;
  const double x = Tc / T;
  const double g = T / OR_ME + 1.0;
  const double b2 = 1.0 - 1.0 / (g * g);
  const double c = (2.0 * g - 1.0) / (g * g);
  const double r = (g - 1.0) / g;
  const double br = r * r * (0.5 - x) + 1.0 / x - 1.0 / (1.0 - x) - c * log((1.0 - x) / x);
  return 2.0 * OR_PI * OR_RE * OR_RE * OR_ME / (b2 * T) * br;
}

/* Bhabha cross section (Bhabha 1936) per target electron, eps in [x, 1]:
 * (2 pi r_e^2 m / T) [ 1/(beta^2 eps^2) - B1/eps + B2 - B3 eps + B4 eps^2 ],
 * y = 1/(g+1), B1 = 2 - y^2, B2 = (1-2y)(3+y^2), B4 = (1-2y)^3, B3 = B4 + (1-2y)^2. */
static void bhabha_coef(double g, double B[4]) {
  const double y = 1.0 / (g + 1.0);
  const double h = 1.0 - 2.0 * y;
  B[0] = 2.0 - y * y;
  B[1] = h * (3.0 + y * y);
  B[3] = h * h * h;
  B[2] = B[3] + h * h;
}

double or_bhabha_dsigma(double T, double eps) {
  const double g = T / OR_ME + 1.0;
  const double b2 = 1.0 - 1.0 / (g * g);
  double B[4];
  bhabha_coef(g, B);
  const double f = 1.0 / (b2 * eps * eps) - B[0] / eps + B[1] - B[2] * eps + B[3] * eps * eps;
  return 2.0 * OR_PI * OR_RE * OR_RE * OR_ME / T * f;
}

double or_bhabha_sigma(double T, double Tc) {
  if (T <= Tc) return 0.0;
  const double x = Tc / T;
  const double g = T / OR_ME + 1.0;
  const double b2 = 1.0 - 1.0 / (g * g);
  double B[4];
  bhabha_coef(g, B);
  const double br = (1.0 / x - 1.0) / b2 + B[0] * log(x) + B[1] * (1.0 - x) -
                    B[2] / 2.0 * (1.0 - x * x) + B[3] / 3.0 * (1.0 - x * x * x);
  return 2.0 * OR_PI * OR_RE * OR_RE * OR_ME / T * br;
}

/* ------------------------------------------------- annihilation (Heitler) */

/* Two-photon annihilation in flight on a free electron (Heitler 1954), per atom
 * (Z electrons), differential in eps = E_photon1 / (T + 2m):
 * (Z pi r_e^2 / ((g+1)(g^2-1))) S(eps), S(e) = -(g+1)^2 + (g^2+4g+1)/e - 1/e^2,
 * over eps in [eps_min, 1 - eps_min], eps_min = (1 - sqrt((g-1)/(g+1)))/2. */
double or_heitler_dsigma(double Z, double T, double eps) {
  const double g = T / OR_ME + 1.0;
  const double S = -(g + 1.0) * (g + 1.0) + (g * g + 4.0 * g + 1.0) / eps - 1.0 / (eps * eps);
  return Z * OR_PI * OR_RE * OR_RE / ((g + 1.0) * (g * g - 1.0)) * S;
}

double or_heitler_sigma(double Z, double T) {
  const double g = T / OR_ME + 1.0;
  const double s = sqrt(g * g - 1.0);
  return Z * OR_PI * OR_RE * OR_RE / (g + 1.0) *
         ((g * g + 4.0 * g + 1.0) / (g * g - 1.0) * log(g + s) - (g + 3.0) / s);
}

/* ------------------------------------------------------ stopping powers */

/* Restricted collision stopping power (Berger-Seltzer form, ICRU Report 37)
 * without density effect, delta-ray energies up to `cut`:
 * S = 2 pi r_e^2 m n_el / beta^2 [ ln(2(tau+2)/I^2) + F(tau, Delta) ], energies in
 * units of m.  Electron: Delta <= tau/2,
 *   F- = -1 - beta^2 + ln((tau-Delta) Delta) + tau/(tau-Delta)
 *        + (Delta^2/2 + (2 tau + 1) ln(1 - Delta/tau)) / g^2.
 * Positron: Delta <= tau, y = 1/(g+1),
 *   F+ = ln(tau Delta) - (beta^2/tau) [ tau + 2 Delta - 3/2 Delta^2 y - (Delta - Delta^3/3) y^2
 *        - (Delta^2/2 - tau Delta^3/3 + Delta^4/4) y^3 ]. */
double or_scol(int positron, double n_el, double I, double T, double cut) {
  const double tau = T / OR_ME;
  const double g = tau + 1.0;
  const double b2 = tau * (tau + 2.0) / (g * g);
  const double Im = I / OR_ME;
  double F;
  if (!positron) {
    const double dmax = 0.5 * T;
    const double D = (cut < dmax ? cut : dmax) / OR_ME;
    F = -1.0 - b2 + log((tau - D) * D) + tau / (tau - D) +
        (D * D / 2.0 + (2.0 * tau + 1.0) * log(1.0 - D / tau)) / (g * g);
  } else {
    const double D = (cut < T ? cut : T) / OR_ME;
    const double y = 1.0 / (g + 1.0);
    const double br = tau + 2.0 * D - 1.5 * D * D * y - (D - D * D * D / 3.0) * y * y -
                      (D * D / 2.0 - tau * D * D * D / 3.0 + D * D * D * D / 4.0) * y * y * y;
    F = log(tau * D) - b2 / tau * br;
  }
  return 2.0 * OR_PI * OR_RE * OR_RE * OR_ME * n_el / b2 * (log(2.0 * (tau + 2.0) / (Im * Im)) + F);
}

/* Radiation length, PDG approximate fit: X0 = 716.4 A / (Z (Z+1) ln(287/sqrt Z)) g/cm^2. */
double or_radiation_length(double Z, double A, double density) {
  return 716.4 * A / (Z * (Z + 1.0) * log(287.0 / sqrt(Z))) / density;
}

/* ------------------------------------------------------------- tables */

/* 8-point Gauss-Legendre nodes/weights on [-1, 1] (Abramowitz & Stegun, Table 25.4). */
static const double GL_X[4] = {0.1834346424956498049, 0.5255324099163289858,
                               0.7966664774136267396, 0.9602898564975362317};
static const double GL_W[4] = {0.3626837833783619830, 0.3137066458778872873,
                               0.2223810344533744706, 0.1012285362903762592};

double or_gl8(double (*f)(const void*, double), const void* ctx, double a, double b) {
  const double h = 0.5 * (b - a), c = 0.5 * (b + a);
  double s = 0.0;
  for (int j = 0; j < 4; ++j) s += GL_W[j] * (f(ctx, c - h * GL_X[j]) + f(ctx, c + h * GL_X[j]));
  return s * h;
}

typedef struct {
  const or_mat_data* m;
  int positron;
  double Tc, kc; /* cuts; <0 means unrestricted */
} sloss_ctx;

static double total_sloss(const sloss_ctx* c, double T) {
  const double scut = c->Tc < 0 ? T : c->Tc;
  const double kcut = c->kc < 0 ? T : c->kc;
  return or_scol(c->positron, c->m->n_el, c->m->I, T, scut) + or_brems_Srad(c->m->X0, T, kcut);
}

/* integrand of the range in ln T: dR/dlnT = T / S(T) */
static double range_integrand(const void* ctx, double lnT) {
  const double T = exp(lnT);
  return T / total_sloss((const sloss_ctx*)ctx, T);
}

/* Node-to-node range accumulation.  The restricted loss has a kink where a cut
 * stops limiting it (T = 2 Tc for electrons, T = Tc for positrons, T = kc for
 * brems); an interval containing a kink is integrated in two pieces split there. */
static void build_range(const or_world* w, const sloss_ctx* c, double* R) {
  double kinks[2];
  int nk = 0;
  if (c->Tc > 0) kinks[nk++] = log(c->positron ? c->Tc : 2.0 * c->Tc);
  if (c->kc > 0) kinks[nk++] = log(c->kc);
  R[0] = 0.0;
  for (int i = 1; i < OR_NGRID; ++i) {
    double a = w->lnE[i - 1], b = w->lnE[i];
    double cuts[2];
    int nc = 0;
    for (int k = 0; k < nk; ++k)
      if (kinks[k] > a && kinks[k] < b) cuts[nc++] = kinks[k];
    if (nc == 2 && cuts[1] < cuts[0]) {
      const double t = cuts[0];
      cuts[0] = cuts[1];
      cuts[1] = t;
    }
    double acc = 0.0;
    for (int k = 0; k < nc; ++k) {
      acc += or_gl8(range_integrand, c, a, cuts[k]);
      a = cuts[k];
    }
    acc += or_gl8(range_integrand, c, a, b);
    R[i] = R[i - 1] + acc;
  }
}

static void grid_locate(const or_world* w, double lnT, int* i, double* f) {
  const double t = (lnT - w->lnE0) / w->dlnE;
  if (!(t > 0.0)) {
    *i = 0;
    *f = 0.0;
    return;
  }
  if (t >= (double)(OR_NGRID - 1)) {
    *i = OR_NGRID - 2;
    *f = 1.0;
    return;
  }
  int k = (int)floor(t);
  if (k > OR_NGRID - 2) k = OR_NGRID - 2;
  *i = k;
  *f = t - (double)k;
}

double or_interp_ln(const or_world* w, const double* v, double lnT) {
  int i;
  double f;
  grid_locate(w, lnT, &i, &f);
  return v[i] + f * (v[i + 1] - v[i]);
}

/* Exact inverse of the piecewise-linear-in-ln-T table v (increasing): returns ln T. */
double or_inverse_ln(const or_world* w, const double* v, double r) {
  if (r <= v[0]) return w->lnE0;
  if (r >= v[OR_NGRID - 1]) return w->lnE0 + (double)(OR_NGRID - 1) * w->dlnE;
  int lo = 0, hi = OR_NGRID - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (v[mid] <= r)
      lo = mid;
    else
      hi = mid;
  }
  const double f = (r - v[lo]) / (v[lo + 1] - v[lo]);
  return w->lnE0 + ((double)lo + f) * w->dlnE;
}

/* Production thresholds from the range cut L (a reading; the paper names none):
 *  e-/e+: the energy whose unrestricted CSDA range (collision loss with all delta
 *         rays + all radiated energy) equals L, using the same node-to-node
 *         Gauss-Legendre range and its piecewise-linear inverse;
 *  photon: the energy at which 5 total mean free paths equal L, linear in ln E
 *         between the nodes that bracket it (first crossing from below);
 *  both at least the tracking cut. */
static void build_cuts(or_world* w, or_mat_data* m) {
  const double tcut = w->opt.tracking_cut;
  if (!(w->opt.production_cut > 0.0) || m->vacuum) {
    m->Tc = tcut;
    m->kc = tcut;
    return;
  }
  const double L = w->opt.production_cut;
  double Ru[OR_NGRID];
  sloss_ctx c = {m, 0, -1.0, -1.0};
  build_range(w, &c, Ru);
  double Tc = exp(or_inverse_ln(w, Ru, L));
  m->Tc = Tc > tcut ? Tc : tcut;

  const double target = 5.0 / L;
  double sig[OR_NGRID];
  for (int i = 0; i < OR_NGRID; ++i) {
    const double E = w->E[i];
    sig[i] = m->n_el * or_kn_sigma(E) + m->n_at * or_pe_sigma(m->Z, E) + or_pair_Sigma(m->X0, E);
  }
  double kc;
  if (sig[0] <= target) {
    kc = w->E[0];
  } else {
    int i = 0;
    while (i < OR_NGRID - 2 && sig[i + 1] > target) ++i;
    const double f = (sig[i] - target) / (sig[i] - sig[i + 1]);
    kc = exp(w->lnE[i] + f * w->dlnE);
  }
  m->kc = kc > tcut ? kc : tcut;
}

static void build_tables(or_world* w, or_mat_data* m) {
  memset(m->tab, 0, sizeof(m->tab));
  if (m->vacuum) return;
  const or_options* o = &w->opt;
  for (int i = 0; i < OR_NGRID; ++i) {
    const double E = w->E[i];
    /* photon: Compton, photoelectric, pair */
    m->tab[OR_GAMMA][0][i] = o->compton ? m->n_el * or_kn_sigma(E) : 0.0;
    m->tab[OR_GAMMA][1][i] = o->photoelectric ? m->n_at * or_pe_sigma(m->Z, E) : 0.0;
    m->tab[OR_GAMMA][2][i] = o->pair ? or_pair_Sigma(m->X0, E) : 0.0;
    /* electron: Moller, brems */
    m->tab[OR_ELECTRON][0][i] = o->ionisation ? m->n_el * or_moller_sigma(E, m->Tc) : 0.0;
    m->tab[OR_ELECTRON][1][i] = o->brems ? or_brems_Sigma(m->X0, E, m->kc) : 0.0;
    /* positron: Bhabha, brems, annihilation in flight */
    m->tab[OR_POSITRON][0][i] = o->ionisation ? m->n_el * or_bhabha_sigma(E, m->Tc) : 0.0;
    m->tab[OR_POSITRON][1][i] = m->tab[OR_ELECTRON][1][i];
    m->tab[OR_POSITRON][2][i] = o->annihilation ? m->n_at * or_heitler_sigma(m->Z, E) : 0.0;
  }
  for (int s = OR_ELECTRON; s <= OR_POSITRON; ++s) {
    /* Restricted loss: delta rays below Tc (if Moller/Bhabha are discrete) and
     * photons below kc (if brems is discrete); otherwise the full loss. */
    sloss_ctx c = {m, s == OR_POSITRON, o->ionisation ? m->Tc : -1.0, o->brems ? m->kc : -1.0};
    build_range(w, &c, m->tab[s][3]);
    m->Rtrk[s] = or_interp_ln(w, m->tab[s][3], log(o->tracking_cut));
  }
}

or_world* or_create(const or_material* mats, int n_mats, const or_options* opt,
                    const or_geometry* geom) {
  if (n_mats < 0 || n_mats > OR_MAXMAT || !opt || !geom) return NULL;
  or_world* w = (or_world*)calloc(1, sizeof(or_world));
  if (!w) return NULL;
  w->opt = *opt;
  w->lnE0 = log(1.0e-3);
  w->dlnE = log(1.0e5 / 1.0e-3) / (double)(OR_NGRID - 1);
  for (int i = 0; i < OR_NGRID; ++i) {
    w->lnE[i] = w->lnE0 + (double)i * w->dlnE;
    w->E[i] = exp(w->lnE[i]);
  }
  w->n_mats = n_mats;
  for (int k = 0; k < n_mats; ++k) {
    or_mat_data* m = &w->mat[k];
    m->Z = mats[k].Z;
    m->A = mats[k].A;
    m->rho = mats[k].density;
    m->I = mats[k].mean_excitation;
    m->vacuum = !(m->rho > 0.0);
    if (!m->vacuum) {
      m->n_at = m->rho * OR_NA / m->A;
      m->n_el = m->Z * m->n_at;
      m->X0 = or_radiation_length(m->Z, m->A, m->rho);
    }
    build_cuts(w, m);
    build_tables(w, m);
  }
  if (or_geometry_init(w, geom) != 0) {
    free(w);
    return NULL;
  }
  return w;
}

void or_destroy(or_world* w) {
  if (!w) return;
  or_geometry_free(w);
  free(w);
}

double or_grid_energy(const or_world* w, int i) { return w->E[i]; }
double or_table_node(const or_world* w, int mat, int species, int q, int i) {
  return w->mat[mat].tab[species][q][i];
}
double or_table_interp(const or_world* w, int mat, int species, int q, double T) {
  return or_interp_ln(w, w->mat[mat].tab[species][q], log(T));
}
double or_range_inverse(const or_world* w, int mat, int species, double r) {
  return exp(or_inverse_ln(w, w->mat[mat].tab[species][3], r));
}
double or_cut_electron(const or_world* w, int mat) { return w->mat[mat].Tc; }
double or_cut_gamma(const or_world* w, int mat) { return w->mat[mat].kc; }
double or_range_at_cut(const or_world* w, int mat, int species) { return w->mat[mat].Rtrk[species]; }
double or_material_X0(const or_world* w, int mat) { return w->mat[mat].X0; }

/* Highland's fit to the width of the projected angular distribution of multiple
 * Coulomb scattering (V. L. Highland, NIM 129 (1975) 497; G. R. Lynch and O. I. Dahl,
 * NIM B58 (1991) 6): theta0 = 13.6 MeV / (beta c p) sqrt(x/X0) [1 + 0.038 ln(x / (X0 beta^2))]
 * for a singly charged particle of kinetic energy T over a path x; 0 where the
 * bracket is not positive (paths far below the fit's range). */
double or_msc_theta0(double T, double x, double X0) {
  const double p = sqrt(T * (T + 2.0 * OR_ME));
  const double beta = p / (T + OR_ME);
  const double r = x / X0;
  const double bracket = 1.0 + 0.038 * log(r / (beta * beta));
  if (!(r > 0.0) || !(bracket > 0.0)) return 0.0;
  return 13.6 / (beta * p) * sqrt(r) * bracket;
}
