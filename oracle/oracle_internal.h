/* oracle_internal.h -- private state of the CPU oracle (test infrastructure only). */
#ifndef EMS_ORACLE_INTERNAL_H
#define EMS_ORACLE_INTERNAL_H

#include "oracle.h"

extern const double OR_ME, OR_RE, OR_NA, OR_PI;

typedef struct {
  double Z, A, rho, I;
  int vacuum;
  double n_at, n_el, X0;
  double Tc, kc;                          /* production thresholds */
  double tab[3][OR_NQ][OR_NGRID];         /* [species][quantity][node] */
  double Rtrk[3];                         /* range table at the tracking cut */
} or_mat_data;

typedef struct {
  int kind, n_vol, n_bins;
  double* bounds;
  int* material;
  int* bin;
  double hx, hy, hz, bz, tol;
  int n_surf;
  double* surf;   /* CSG: n_surf x 10 quadric coefficients */
  int* face_off;  /* CSG: n_vol + 1 */
  int* faces;     /* CSG: surface * 2 + (cell on the f > 0 side) */
} or_geom_data;

struct or_world {
  or_options opt;
  double lnE0, dlnE;
  double lnE[OR_NGRID], E[OR_NGRID];
  int n_mats;
  or_mat_data mat[OR_MAXMAT];
  or_geom_data geo;
};

double or_gl8(double (*f)(const void*, double), const void* ctx, double a, double b);
double or_interp_ln(const or_world* w, const double* v, double lnT);
double or_inverse_ln(const or_world* w, const double* v, double r);
int or_geometry_init(or_world* w, const or_geometry* g);
void or_geometry_free(or_world* w);
int or_csg_locate(const or_geom_data* g, const double p[3], const double d[3]);
double or_csg_distance(const or_geom_data* g, int k, const double p[3], const double d[3], int* next);

#endif
