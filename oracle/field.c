/*
 * field.c -- charged-track propagation in a uniform magnetic field along z for
 * the CPU oracle (test infrastructure only; see oracle.h).
 *
 * The paper propagates charged particles through fields on the device with
 * templated integrators (Sec. 2.3 "Geometry and EM fields") but gives no
 * algorithm; the reading taken here:
 *   - equation of motion per unit path length s: dr/ds = d,
 *     dd/ds = kappa (d_y, -d_x, 0), kappa = 2.99792458 q B_z / p  (1/cm, p in MeV/c,
 *     B in tesla, q = -1 for e-, +1 for e+);
 *   - classical fourth-order Runge-Kutta substeps; the error of a substep h is the
 *     distance between one step of h and two steps of h/2, which must not exceed
 *     the tolerance (else h is halved); the two-half-step result is kept and the
 *     direction renormalised; h doubles after a substep with error < tol/32;
 *   - the boundary is sought on each substep's chord: if the straight-line
 *     distance from the substep's start along the chord is shorter than the chord,
 *     the crossing is accepted once the sagitta (distance of the half-step point
 *     from the chord) is within the tolerance -- position on the chord at the
 *     boundary, path length the same fraction of h, direction from one RK4 step of
 *     that length -- otherwise h shrinks by that fraction and the substep is redone;
 *   - a step in matter ends at the physics limit (discrete or continuous) or the
 *     boundary; one needing more than 10^4 substeps is a looper and is killed;
 *   - a step in vacuum (no physics limit) ends at the boundary or after 256
 *     substeps; the step that ends the 40th such capped step in a row is a
 *     looper (or_step keeps the count).
 */
#include <math.h>

#include "oracle_internal.h"

#define OR_FIELD_MAXSUB 10000
#define OR_FIELD_VACSUB 256
#define OR_FIELD_HMIN 1.0e-9

double or_field_kappa(double q, double bz, double p) { return 2.99792458 * q * bz / p; }

/* one classical RK4 step of length h */
void or_rk4(double kappa, double h, const double r[3], const double d[3], double ro[3],
            double dout[3]) {
  double k1r[3], k1d[3], k2r[3], k2d[3], k3r[3], k3d[3], k4r[3], k4d[3], t[3];
  /* f(r, d) = (d, kappa (d_y, -d_x, 0)) */
  k1r[0] = d[0];
  k1r[1] = d[1];
  k1r[2] = d[2];
  k1d[0] = kappa * d[1];
  k1d[1] = -kappa * d[0];
  k1d[2] = 0.0;
  for (int i = 0; i < 3; ++i) t[i] = d[i] + 0.5 * h * k1d[i];
  k2r[0] = t[0];
  k2r[1] = t[1];
  k2r[2] = t[2];
  k2d[0] = kappa * t[1];
  k2d[1] = -kappa * t[0];
  k2d[2] = 0.0;
  for (int i = 0; i < 3; ++i) t[i] = d[i] + 0.5 * h * k2d[i];
  k3r[0] = t[0];
  k3r[1] = t[1];
  k3r[2] = t[2];
  k3d[0] = kappa * t[1];
  k3d[1] = -kappa * t[0];
  k3d[2] = 0.0;
  for (int i = 0; i < 3; ++i) t[i] = d[i] + h * k3d[i];
  k4r[0] = t[0];
  k4r[1] = t[1];
  k4r[2] = t[2];
  k4d[0] = kappa * t[1];
  k4d[1] = -kappa * t[0];
  k4d[2] = 0.0;
  for (int i = 0; i < 3; ++i) {
    ro[i] = r[i] + h / 6.0 * (k1r[i] + 2.0 * k2r[i] + 2.0 * k3r[i] + k4r[i]);
    dout[i] = d[i] + h / 6.0 * (k1d[i] + 2.0 * k2d[i] + 2.0 * k3d[i] + k4d[i]);
  }
}

static void normalise(double v[3]) {
  const double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  v[0] /= n;
  v[1] /= n;
  v[2] /= n;
}

/* Move (r, d) in volume vol along the curved path for at most s_max (may be
 * infinite).  Returns 0 when s_max was reached, 1 at a boundary (*next set), 2 for
 * a looper in matter, 3 when a vacuum step used its 256 substeps; *s_out = path
 * length travelled. */
int or_field_move(const or_world* w, int vol, double kappa, double s_max, int vacuum, double r[3],
                  double d[3], double* s_out, int* next) {
  const double tol = w->geo.tol;
  const double limit = s_max;
  double travelled = 0.0;
  double h = fabs(kappa) > 0.0 ? fmin(limit, 1.0 / fabs(kappa)) : limit;
  *next = OR_OUTSIDE;
  const int max_sub = vacuum ? OR_FIELD_VACSUB : OR_FIELD_MAXSUB;
  for (int nsub = 0; nsub < max_sub; ++nsub) {
    double hh = fmin(h, limit - travelled);
    double rf[3], df[3], rm[3], dm[3], r2[3], d2[3];
    or_rk4(kappa, hh, r, d, rf, df);
    or_rk4(kappa, 0.5 * hh, r, d, rm, dm);
    or_rk4(kappa, 0.5 * hh, rm, dm, r2, d2);
    const double ex = r2[0] - rf[0], ey = r2[1] - rf[1], ez = r2[2] - rf[2];
    const double err = sqrt(ex * ex + ey * ey + ez * ez);
    if (err > tol && hh > OR_FIELD_HMIN) {
      h = 0.5 * hh;
      continue;
    }
    double c[3] = {r2[0] - r[0], r2[1] - r[1], r2[2] - r[2]};
    const double L = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    int nx = OR_OUTSIDE;
    double sb = HUGE_VAL;
    if (L > 0.0) {
      c[0] /= L;
      c[1] /= L;
      c[2] /= L;
      sb = or_distance(w, vol, r, c, &nx);
    }
    if (sb < L) {
      const double mx = rm[0] - r[0], my = rm[1] - r[1], mz = rm[2] - r[2];
      const double along = mx * c[0] + my * c[1] + mz * c[2];
      const double px = mx - along * c[0], py = my - along * c[1], pz = mz - along * c[2];
      const double sag = sqrt(px * px + py * py + pz * pz);
      if (sag <= tol || hh <= OR_FIELD_HMIN) {
        const double part = hh * (sb / L);
        double rc[3], dc[3];
        or_rk4(kappa, part, r, d, rc, dc);
        r[0] += sb * c[0];
        r[1] += sb * c[1];
        r[2] += sb * c[2];
        normalise(dc);
        d[0] = dc[0];
        d[1] = dc[1];
        d[2] = dc[2];
        *s_out = travelled + part;
        *next = nx;
        return 1;
      }
      h = fmax(hh * (sb / L), OR_FIELD_HMIN);
      continue;
    }
    r[0] = r2[0];
    r[1] = r2[1];
    r[2] = r2[2];
    normalise(d2);
    d[0] = d2[0];
    d[1] = d2[1];
    d[2] = d2[2];
    travelled += hh;
    if (travelled >= limit) {
      *s_out = travelled;
      return 0;
    }
    h = err < tol / 32.0 ? 2.0 * hh : hh;
  }
  *s_out = travelled;
  return vacuum ? 3 : 2;
}
