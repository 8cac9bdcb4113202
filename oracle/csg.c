/*
 * csg.c -- single-level quadric-surface geometry of the CPU oracle (test
 * infrastructure only; see oracle.h).
 *
 * Paper Sec. 2.3 ("Geometry and EM fields"): the ORANGE navigation model --
 * cells bounded by quadric surfaces, found by their sense with respect to each
 * surface, in a single level (no nested universes).  Here every surface is a
 * general quadric
 *   f(x) = qxx x^2 + qyy y^2 + qzz z^2 + qxy x y + qyz y z + qzx z x
 *          + px x + py y + pz z + k,
 * and every cell is the intersection of half-spaces "f < 0" (sense -1) or
 * "f > 0" (sense +1).  On a ray x = p + t d, f = a t^2 + B t + c with
 *   a = the quadratic part evaluated at d,
 *   B = the gradient of f at p dotted with d,
 *   c = f(p).
 * A track in cell K leaves through face (s, sigma) where f_s turns from the
 * sigma side to the other, i.e. at the root where df/dt has the sign -sigma;
 * the boundary distance is the smallest such root over the faces of K (the
 * first face in the cell's list wins ties).  The cell entered is the first cell,
 * in index order, that has the crossed surface with the opposite sense and whose
 * other faces all hold at the crossing point; if none does (the crossing point
 * also lies on another surface), the first other cell without the crossed
 * surface on the side just left that holds the crossing point moving along d; if
 * none, the track leaves the world.  In both searches the crossed surface counts
 * as satisfied.  A point on a surface takes the side its direction moves to.
 *
 * Everything is evaluated in IEEE double precision in the order written
 * (-ffp-contract=off): the sense decisions at a crossing point compare values
 * that are exactly zero on the surface.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

/* f(p) and its derivative along d at p, and the quadratic coefficient a. */
static void ray_coeffs(const double* q, const double p[3], const double d[3], double* a, double* B,
                       double* c) {
  const double x = p[0], y = p[1], z = p[2], u = d[0], v = d[1], w = d[2];
  *a = q[0] * u * u + q[1] * v * v + q[2] * w * w + q[3] * u * v + q[4] * v * w + q[5] * w * u;
  *B = 2.0 * (q[0] * x * u + q[1] * y * v + q[2] * z * w) + q[3] * (x * v + y * u) +
       q[4] * (y * w + z * v) + q[5] * (z * u + x * w) + q[6] * u + q[7] * v + q[8] * w;
  *c = q[0] * x * x + q[1] * y * y + q[2] * z * z + q[3] * x * y + q[4] * y * z + q[5] * z * x +
       q[6] * x + q[7] * y + q[8] * z + q[9];
}

/* Side (+1 / -1) of surface q at point p moving along d: the sign of f, or on the
 * surface the sign of its derivative along d (tangent: the sign of a, zero -> +1). */
int or_csg_side(const double* q, const double p[3], const double d[3]) {
  double a, B, c;
  ray_coeffs(q, p, d, &a, &B, &c);
  if (c > 0.0) return 1;
  if (c < 0.0) return -1;
  if (B > 0.0) return 1;
  if (B < 0.0) return -1;
  return a >= 0.0 ? 1 : -1;
}

/* Distance along d from p to where f leaves the side sigma, HUGE_VAL if never.
 * Roots of a t^2 + B t + c = 0 with b = B/2: the exit root is the one where
 * 2 (a t + b) has the sign -sigma, t = (-b - sigma sqrt(b^2 - a c)) / a, evaluated
 * as c / (-b + sigma sqrt(...)) when that denominator involves no cancellation
 * (sigma b <= 0), which also covers a = 0 (a plane: t = -c / B).  A root behind the
 * point counts as 0 if the track is moving off the sigma side right now (df/dt at
 * the point has the sign -sigma: a point rounded just past the surface it leaves),
 * else as no crossing (the surface was crossed the other way, behind). */
double or_csg_exit(const double* q, const double p[3], const double d[3], int sigma) {
  double a, B, c;
  ray_coeffs(q, p, d, &a, &B, &c);
  const double b = 0.5 * B;
  const double sg = (double)sigma;
  double t;
  if (a == 0.0) {
    if (!(sg * b < 0.0)) return HUGE_VAL;
    t = c / (-2.0 * b);
  } else {
    const double D = b * b - a * c;
    if (!(D > 0.0)) return HUGE_VAL;
    const double r = sqrt(D);
    if (sg * b <= 0.0) t = c / (-b + sg * r);
    else t = (-b - sg * r) / a;
  }
  if (!(t >= 0.0)) return sg * b < 0.0 ? 0.0 : HUGE_VAL;
  return t;
}

static const double* surf(const or_geom_data* g, int s) { return g->surf + 10 * (size_t)s; }

/* Does cell k hold point p moving along d?  A face on surface `forced` (or -1) is
 * taken as satisfied. */
static int cell_holds(const or_geom_data* g, int k, const double p[3], const double d[3],
                      int forced) {
  for (int j = g->face_off[k]; j < g->face_off[k + 1]; ++j) {
    const int s = g->faces[j] >> 1;
    const int sense = (g->faces[j] & 1) ? 1 : -1;
    if (s == forced) continue;
    if (or_csg_side(surf(g, s), p, d) != sense) return 0;
  }
  return 1;
}

int or_csg_locate(const or_geom_data* g, const double p[3], const double d[3]) {
  for (int k = 0; k < g->n_vol; ++k)
    if (cell_holds(g, k, p, d, -1)) return k;
  return OR_OUTSIDE;
}

/* Boundary distance from p along d inside cell k and the cell entered there. */
double or_csg_distance(const or_geom_data* g, int k, const double p[3], const double d[3],
                       int* next) {
  double s_min = HUGE_VAL;
  int face = -1;
  for (int j = g->face_off[k]; j < g->face_off[k + 1]; ++j) {
    const int s = g->faces[j] >> 1;
    const int sense = (g->faces[j] & 1) ? 1 : -1;
    const double t = or_csg_exit(surf(g, s), p, d, sense);
    if (t < s_min) {
      s_min = t;
      face = j;
    }
  }
  *next = OR_OUTSIDE;
  if (face < 0) return HUGE_VAL;
  const int left = g->faces[face];       /* crossed surface with the side left */
  const int s = left >> 1;
  const int entered = 2 * s + (1 - (left & 1)); /* the same surface, other side */
  const double x[3] = {p[0] + s_min * d[0], p[1] + s_min * d[1], p[2] + s_min * d[2]};
  for (int pass = 0; pass < 2; ++pass) {
    for (int m = 0; m < g->n_vol; ++m) {
      if (m == k) continue;
      int has_entered = 0, has_left = 0;
      for (int j = g->face_off[m]; j < g->face_off[m + 1]; ++j) {
        if (g->faces[j] == entered) has_entered = 1;
        if (g->faces[j] == left) has_left = 1;
      }
      const int candidate = pass == 0 ? has_entered : !has_left;
      if (candidate && cell_holds(g, m, x, d, s)) {
        *next = m;
        return s_min;
      }
    }
  }
  return s_min;
}
