// ems_tables.cpp -- host-side physics table builder behind init_physics_tables().
//
// Paper Sec. 2.2: cross sections are pre-tabulated and loaded to host and device
// at initialisation.  The paper does not print its models; the forms below are the
// textbook ones its model table names (Klein-Nishina Compton, Bethe-Heitler pair
// production in the complete-screening limit, Moller-Bhabha ionisation with the
// Berger-Seltzer restricted stopping power, a complete-screening bremsstrahlung
// spectrum, Heitler two-photon annihilation) plus the synthetic photoelectric law
// of the benchmark workload.  Layout for the device: for material m, species s and
// node i, four consecutive values (three cross sections and, for e-/e+, the range),
// so the two nodes bracketing an energy are one 64-byte (FP64) or 32-byte (FP32)
// contiguous read.
#include <cmath>
#include <cstring>
#include <vector>

#include "ems_host.h"

namespace ems {
namespace {

constexpr double kMeH = 0.51099895000;   // MeV
constexpr double kReH = 2.8179403262e-13;  // cm
constexpr double kAvogadro = 6.02214076e23;
constexpr double kPiH = 3.14159265358979323846;
constexpr double kTwoPiRe2 = 2.0 * kPiH * kReH * kReH;  // cm^2

// 8-point Gauss-Legendre rule on [-1, 1] (Abramowitz & Stegun 25.4.30).
constexpr double kGLx[4] = {0.1834346424956498049, 0.5255324099163289858, 0.7966664774136267396,
                            0.9602898564975362317};
constexpr double kGLw[4] = {0.3626837833783619830, 0.3137066458778872873, 0.2223810344533744706,
                            0.1012285362903762592};

template <class F>
double gauss8(F&& f, double a, double b) {
  const double half = 0.5 * (b - a), mid = 0.5 * (a + b);
  double acc = 0.0;
  for (int j = 0; j < 4; ++j) acc += kGLw[j] * (f(mid - half * kGLx[j]) + f(mid + half * kGLx[j]));
  return acc * half;
}

struct Element {
  double Z, A, rho, I;
  double atoms, electrons, X0;  // per cm^3, per cm^3, cm
};

// --- photons
double klein_nishina(double E) {  // per electron
  const double k = E / kMeH, q = 1.0 + 2.0 * k, lq = std::log(q);
  return kTwoPiRe2 * ((1.0 + k) / (k * k) * (2.0 * (1.0 + k) / q - lq / k) + lq / (2.0 * k) -
                      (1.0 + 3.0 * k) / (q * q));
}
double photoelectric(double Z, double E) {  // per atom
  return 1.0e-30 * std::pow(Z, 5.0) * std::pow(0.1 / E, 3.5);
}
double pair_macro(const Element& el, double E) {
  if (E <= 2.0 * kMeH) return 0.0;
  const double a = kMeH / E, b = 1.0 - a;
  auto G = [](double x) { return x * x * (0.5 - x / 3.0); };
  return (b - a - (4.0 / 3.0) * (G(b) - G(a))) / el.X0;
}

// --- charged
double brems_macro(const Element& el, double T, double kc) {  // photons above kc
  if (T <= kc) return 0.0;
  const double r = kc / T;
  return ((4.0 / 3.0) * std::log(1.0 / r) - (4.0 / 3.0) * (1.0 - r) + 0.5 * (1.0 - r * r)) / el.X0;
}
double brems_soft_loss(const Element& el, double T, double kc) {  // energy radiated below kc
  const double k = kc < T ? kc : T, y = k / T;
  return k * ((4.0 / 3.0) - (2.0 / 3.0) * y + y * y / 3.0) / el.X0;
}
double moller(double T, double Tc) {  // per electron, delta rays above Tc
  if (T <= 2.0 * Tc) return 0.0;
  const double x = Tc / T, gam = T / kMeH + 1.0, g2 = gam * gam, beta2 = 1.0 - 1.0 / g2;
  const double cg = (2.0 * gam - 1.0) / g2, t = (gam - 1.0) / gam;
  const double bracket = t * t * (0.5 - x) + 1.0 / x - 1.0 / (1.0 - x) - cg * std::log((1.0 - x) / x);
  return kTwoPiRe2 * kMeH / (beta2 * T) * bracket;
}
double bhabha(double T, double Tc) {  // per electron, delta rays above Tc
  if (T <= Tc) return 0.0;
  const double x = Tc / T, gam = T / kMeH + 1.0, beta2 = 1.0 - 1.0 / (gam * gam);
  const double y = 1.0 / (gam + 1.0), h = 1.0 - 2.0 * y;
  const double b1 = 2.0 - y * y, b2 = h * (3.0 + y * y), b4 = h * h * h, b3 = b4 + h * h;
  const double bracket = (1.0 / x - 1.0) / beta2 + b1 * std::log(x) + b2 * (1.0 - x) -
                         0.5 * b3 * (1.0 - x * x) + b4 * (1.0 - x * x * x) / 3.0;
  return kTwoPiRe2 * kMeH / T * bracket;
}
double heitler(double Z, double T) {  // per atom
  const double gam = T / kMeH + 1.0, root = std::sqrt(gam * gam - 1.0);
  return Z * kPiH * kReH * kReH / (gam + 1.0) *
         ((gam * gam + 4.0 * gam + 1.0) / (gam * gam - 1.0) * std::log(gam + root) -
          (gam + 3.0) / root);
}
// Berger-Seltzer restricted collision stopping power, no density effect.
double collision_loss(const Element& el, bool positron, double T, double cut) {
  const double tau = T / kMeH, gam = tau + 1.0, g2 = gam * gam, beta2 = tau * (tau + 2.0) / g2;
  const double im = el.I / kMeH;
  const double head = std::log(2.0 * (tau + 2.0) / (im * im));
  double F;
  if (!positron) {
    const double d = std::fmin(cut, 0.5 * T) / kMeH;
    F = -1.0 - beta2 + std::log((tau - d) * d) + tau / (tau - d) +
        (0.5 * d * d + (2.0 * tau + 1.0) * std::log(1.0 - d / tau)) / g2;
  } else {
    const double d = std::fmin(cut, T) / kMeH, y = 1.0 / (gam + 1.0);
    const double d2 = d * d, d3 = d2 * d, d4 = d3 * d;
    const double poly = tau + 2.0 * d - 1.5 * d2 * y - (d - d3 / 3.0) * y * y -
                        (0.5 * d2 - tau * d3 / 3.0 + 0.25 * d4) * y * y * y;
    F = std::log(tau * d) - beta2 / tau * poly;
  }
  return kTwoPiRe2 * kMeH * el.electrons / beta2 * (head + F);
}

struct Grid {
  double ln0, dln;
  double lnE[kGrid], E[kGrid];
  Grid() {
    ln0 = std::log(1.0e-3);
    dln = std::log(1.0e8) / (kGrid - 1);
    for (int i = 0; i < kGrid; ++i) {
      lnE[i] = ln0 + i * dln;
      E[i] = std::exp(lnE[i]);
    }
  }
  double interp(const double* v, double lnT) const {
    const double t = (lnT - ln0) / dln;
    int i;
    double f;
    if (!(t > 0.0)) {
      i = 0;
      f = 0.0;
    } else if (t >= kGrid - 1) {
      i = kGrid - 2;
      f = 1.0;
    } else {
      i = (int)std::floor(t);
      if (i > kGrid - 2) i = kGrid - 2;
      f = t - i;
    }
    return v[i] + f * (v[i + 1] - v[i]);
  }
  double inverse(const double* v, double r) const {  // ln T of the piecewise-linear inverse
    if (r <= v[0]) return ln0;
    if (r >= v[kGrid - 1]) return ln0 + (kGrid - 1) * dln;
    int lo = 0, hi = kGrid - 1;
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      (v[mid] <= r ? lo : hi) = mid;
    }
    return ln0 + (lo + (r - v[lo]) / (v[lo + 1] - v[lo])) * dln;
  }
};

// Range from the first node: node-to-node Gauss-Legendre of T/S(T) in ln T, each
// interval split where the restricted loss has a kink (cuts stop binding).
template <class LossFn>
void range_table(const Grid& g, LossFn&& loss, const std::vector<double>& kinks, double* R) {
  auto integrand = [&](double l) {
    const double T = std::exp(l);
    return T / loss(T);
  };
  R[0] = 0.0;
  for (int i = 1; i < kGrid; ++i) {
    double lo = g.lnE[i - 1];
    const double hi = g.lnE[i];
    std::vector<double> inside;
    for (double k : kinks)
      if (k > lo && k < hi) inside.push_back(k);
    if (inside.size() == 2 && inside[1] < inside[0]) std::swap(inside[0], inside[1]);
    double sum = 0.0;
    for (double k : inside) {
      sum += gauss8(integrand, lo, k);
      lo = k;
    }
    sum += gauss8(integrand, lo, hi);
    R[i] = R[i - 1] + sum;
  }
}

}  // namespace

// Fill tab (kMaxMat x 3 x kGrid x kQ doubles) and the per-material parameters.
int build_physics_tables(const ems_material* mats, int n_mats, const ems_physics_options& o,
                         std::vector<double>& tab, MatParams* mp) {
  const Grid g;
  tab.assign((size_t)kMaxMat * 3 * kGrid * kQ, 0.0);
  for (int m = 0; m < n_mats; ++m) {
    Element el{mats[m].Z, mats[m].A, mats[m].density, mats[m].mean_excitation, 0, 0, 0};
    MatParams& P = mp[m];
    std::memset(&P, 0, sizeof(P));
    P.vacuum = !(el.rho > 0.0);
    if (P.vacuum) {
      P.Tc = P.kc = o.tracking_cut;
      continue;
    }
    if (!(el.Z > 0 && el.A > 0 && el.I > 0)) return -1;
    el.atoms = el.rho * kAvogadro / el.A;
    el.electrons = el.Z * el.atoms;
    el.X0 = 716.4 * el.A / (el.Z * (el.Z + 1.0) * std::log(287.0 / std::sqrt(el.Z))) / el.rho;
    P.X0 = el.X0;

    // production thresholds from the range cut
    double Tc = o.tracking_cut, kc = o.tracking_cut;
    if (o.production_cut > 0.0) {
      const double L = o.production_cut;
      std::vector<double> Ru(kGrid);
      range_table(g, [&](double T) { return collision_loss(el, false, T, T) + T / el.X0; }, {},
                  Ru.data());
      Tc = std::exp(g.inverse(Ru.data(), L));
      const double want = 5.0 / L;
      std::vector<double> mu(kGrid);
      for (int i = 0; i < kGrid; ++i)
        mu[i] = el.electrons * klein_nishina(g.E[i]) + el.atoms * photoelectric(el.Z, g.E[i]) +
                pair_macro(el, g.E[i]);
      if (mu[0] <= want) {
        kc = g.E[0];
      } else {
        int i = 0;
        while (i < kGrid - 2 && mu[i + 1] > want) ++i;
        kc = std::exp(g.lnE[i] + (mu[i] - want) / (mu[i] - mu[i + 1]) * g.dln);
      }
      Tc = std::fmax(Tc, o.tracking_cut);
      kc = std::fmax(kc, o.tracking_cut);
    }
    P.Tc = Tc;
    P.kc = kc;

    auto at = [&](int s, int i, int q) -> double& {
      return tab[(((size_t)m * 3 + s) * kGrid + i) * kQ + q];
    };
    for (int i = 0; i < kGrid; ++i) {
      const double E = g.E[i];
      at(EMS_GAMMA, i, 0) = o.compton ? el.electrons * klein_nishina(E) : 0.0;
      at(EMS_GAMMA, i, 1) = o.photoelectric ? el.atoms * photoelectric(el.Z, E) : 0.0;
      at(EMS_GAMMA, i, 2) = o.pair ? pair_macro(el, E) : 0.0;
      const double br = o.brems ? brems_macro(el, E, kc) : 0.0;
      at(EMS_ELECTRON, i, 0) = o.ionisation ? el.electrons * moller(E, Tc) : 0.0;
      at(EMS_ELECTRON, i, 1) = br;
      at(EMS_POSITRON, i, 0) = o.ionisation ? el.electrons * bhabha(E, Tc) : 0.0;
      at(EMS_POSITRON, i, 1) = br;
      at(EMS_POSITRON, i, 2) = o.annihilation ? el.atoms * heitler(el.Z, E) : 0.0;
    }
    for (int s = EMS_ELECTRON; s <= EMS_POSITRON; ++s) {
      const bool pos = s == EMS_POSITRON;
      // delta rays below Tc and photons below kc are continuous when those processes
      // are discrete; otherwise the whole loss is continuous
      const double ccut = o.ionisation ? Tc : -1.0, rcut = o.brems ? kc : -1.0;
      std::vector<double> kinks;
      if (ccut > 0) kinks.push_back(std::log(pos ? ccut : 2.0 * ccut));
      if (rcut > 0) kinks.push_back(std::log(rcut));
      std::vector<double> R(kGrid);
      range_table(
          g,
          [&](double T) {
            return collision_loss(el, pos, T, ccut > 0 ? ccut : T) +
                   brems_soft_loss(el, T, rcut > 0 ? rcut : T);
          },
          kinks, R.data());
      for (int i = 0; i < kGrid; ++i) at(s, i, 3) = R[i];
      P.Rtrk[s] = g.interp(R.data(), std::log(o.tracking_cut));
      P.Rtrk_f[s] = (float)P.Rtrk[s];
    }
  }
  for (int m = 0; m < n_mats; ++m) {
    mp[m].Tc_f = (float)mp[m].Tc;
    mp[m].kc_f = (float)mp[m].kc;
    mp[m].X0_f = (float)mp[m].X0;
  }
  return 0;
}

}  // namespace ems
