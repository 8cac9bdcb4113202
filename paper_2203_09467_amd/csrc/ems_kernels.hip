// ems_kernels.hip -- gfx950 kernels of the electromagnetic-shower step loop.
//
// One lane per track (paper Sec. 2.1 "Code Architecture").  A step iteration is
// two kernels over the compacted pools (paper Sec. 3.2: a step is several
// kernels with synchronisation points).  k_transport: cross-section lookup,
// interaction-length sampling, continuous step limit, distance to boundary (or a
// curved move in a field), move and continuous loss, cutoffs, process selection
// (paper Sec. 2.2 items (i)-(vi)); survivors go to the other pool buffer, tracks
// that interact to one queue per process.  k_interact: the interaction of one
// process per block, secondary emission, and the room check that puts off
// interactions which would not fit.  Outputs are reserved with one atomic per
// block and stream (ballot + popcount prefix in LDS), the block-aggregated form
// of the paper's atomic stack allocator (Sec. 2.1); per-event scores are summed
// per block in LDS before one global atomic per key.  Nothing here is a dense
// contraction, so there is no MFMA: the kernels stream SoA state (coalesced
// 64-lane accesses) and read tables and geometry from a per-block LDS copy.
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the track's
// 96-bit lineage key and its own step count, so a track's history does not
// depend on which lane, slot or iteration runs it.
//
// Precision: Real = double (FP64 run) or float (mixed run).  In a mixed run the
// tables, interpolation, interaction lengths and sampling are FP32 while
// positions, directions, kinetic energies and tallies stay FP64.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "emshower.h"
#include "ems_device.h"

namespace ems {

__constant__ double kMe = 0.51099895000;  // electron mass, MeV (CODATA 2018)
constexpr double kTwoPi = 6.283185307179586476925;

// ------------------------------------------------------------------ random numbers

__device__ __forceinline__ void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1, uint32_t& o0, uint32_t& o1,
                                         uint32_t& o2, uint32_t& o3) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  o0 = c0;
  o1 = c1;
  o2 = c2;
  o3 = c3;
}

// Draw d of (key, step): block d>>1 of Philox(ctr = (k0, k1, step, d>>1), key = (seed, k2)).
struct Stream {
  uint32_t k0, k1, k2, step, seed;
  uint32_t blk, o0, o1, o2, o3;
  __device__ __forceinline__ void init(uint32_t a, uint32_t b, uint32_t c, uint32_t s,
                                       uint32_t sd) {
    k0 = a;
    k1 = b;
    k2 = c;
    step = s;
    seed = sd;
    blk = 0xFFFFFFFFu;
  }
  __device__ __forceinline__ uint64_t word(uint32_t d) {
    const uint32_t b = d >> 1;
    if (b != blk) {
      philox10(k0, k1, step, b, seed, k2, o0, o1, o2, o3);
      blk = b;
    }
    return (d & 1u) ? (((uint64_t)o2 << 32) | o3) : (((uint64_t)o0 << 32) | o1);
  }
};

__device__ __forceinline__ void child_key(uint32_t seed, uint32_t p0, uint32_t p1, uint32_t p2,
                                          uint32_t step, uint32_t ordinal, uint32_t& c0,
                                          uint32_t& c1, uint32_t& c2) {
  uint32_t o3;
  philox10(p0, p1, p2, step, seed, 0xB7E15162u ^ ordinal, c0, c1, c2, o3);
}

// ------------------------------------------------------------------ precision traits

template <class R>
struct Px;

// Multiple-scattering draws of a step: two words far above the interaction draws.
constexpr uint32_t kMscDraw = 0x40000000u;

template <>
struct Px<double> {
  static __device__ __forceinline__ double uni(uint64_t w) {
    return ((double)(w >> 12) + 0.5) * 0x1p-52;
  }
  static __device__ __forceinline__ double lg(double x) { return log(x); }
  static __device__ __forceinline__ double ex(double x) { return exp(x); }
  static __device__ __forceinline__ double sq(double x) { return sqrt(x); }
  static __device__ __forceinline__ double dv(double a, double b) { return a / b; }
  static __device__ __forceinline__ void sc(double a, double* s, double* c) { sincos(a, s, c); }
  static __device__ __forceinline__ const double* tab(const Params& P) { return P.tab_d; }
  static __device__ __forceinline__ double lnE0(const Params& P) { return P.lnE0; }
  static __device__ __forceinline__ double inv(const Params& P) { return P.inv_dlnE; }
  static __device__ __forceinline__ double dln(const Params& P) { return P.dlnE; }
  static __device__ __forceinline__ double rtrk(const MatParams& m, int s) { return m.Rtrk[s]; }
  static __device__ __forceinline__ double alpha(const Params& P) { return P.alpha; }
  static __device__ __forceinline__ double rfin(const Params& P) { return P.rfinal; }
  static __device__ __forceinline__ double x0(const MatParams& m) { return m.X0; }
};

template <>
struct Px<float> {
  static __device__ __forceinline__ float uni(uint64_t w) {
    return ((float)(uint32_t)(w >> 41) + 0.5f) * 0x1p-23f;
  }
  static __device__ __forceinline__ float lg(float x) { return __logf(x); }
  static __device__ __forceinline__ float ex(float x) { return __expf(x); }
  static __device__ __forceinline__ float sq(float x) { return __fsqrt_rn(x); }
  static __device__ __forceinline__ float dv(float a, float b) { return __fdividef(a, b); }
  static __device__ __forceinline__ void sc(float a, float* s, float* c) { __sincosf(a, s, c); }
  static __device__ __forceinline__ const float* tab(const Params& P) { return P.tab_f; }
  static __device__ __forceinline__ float lnE0(const Params& P) { return P.lnE0_f; }
  static __device__ __forceinline__ float inv(const Params& P) { return P.inv_dlnE_f; }
  static __device__ __forceinline__ float dln(const Params& P) { return P.dlnE_f; }
  static __device__ __forceinline__ float rtrk(const MatParams& m, int s) { return m.Rtrk_f[s]; }
  static __device__ __forceinline__ float alpha(const Params& P) { return P.alpha_f; }
  static __device__ __forceinline__ float rfin(const Params& P) { return P.rfinal_f; }
  static __device__ __forceinline__ float x0(const MatParams& m) { return m.X0_f; }
};

// ------------------------------------------------------------------ tables

// Run data read during a step: the cross-section/range table of (material m,
// species sp), volume bounds, volume -> material and volume -> tally-bin maps and
// the material parameters.  The step kernels address them either in global memory
// or in a copy staged in LDS by each block (the tables of the block's species
// class only, so a staged table starts at species sp0).
// Geometry read by the navigation: slab planes or shell radii, or the quadric cells'
// surfaces (with a per-surface plane flag), faces and entry candidates.
struct Geo {
  const double* bounds;
  const double* surf;
  const unsigned char* plane;
  const int* face_off;
  const int* faces;
  const int* cand_off;
  const int* cand;
};

__device__ __forceinline__ Geo global_geo(const Params& P) {
  return Geo{P.bounds, P.surf, P.plane, P.face_off, P.faces, P.cand_off, P.cand};
}

template <class R>
struct View {
  const R* tab;
  int mstride, sp0;  // elements per material, first species held
  Geo g;
  const int* vmat;
  const int* vbin;
  const MatParams* mat;
  __device__ __forceinline__ const R* of(int m, int sp) const {
    return tab + m * mstride + (sp - sp0) * (kGrid * kQ);
  }
};

// Grid interval and fraction of ln T (linear interpolation in ln E between nodes).
template <class R>
__device__ __forceinline__ void grid_pos(const Params& P, R lnT, int& i, R& f) {
  const R t = (lnT - Px<R>::lnE0(P)) * Px<R>::inv(P);
  if (!(t > R(0))) {
    i = 0;
    f = R(0);
  } else if (t >= R(kGrid - 1)) {
    i = kGrid - 2;
    f = R(1);
  } else {
    int k = (int)t;
    if (k > kGrid - 2) k = kGrid - 2;
    i = k;
    f = t - (R)k;
  }
}

// All kQ interpolated quantities of (material, species) at ln T.
template <class R>
__device__ __forceinline__ void lookup(const Params& P, const R* tb, R lnT, R q[kQ], int& i) {
  R f;
  grid_pos<R>(P, lnT, i, f);
  const R* t = tb + i * kQ;
#pragma unroll
  for (int j = 0; j < kQ; ++j) {
    const R a = t[j], b = t[kQ + j];
    q[j] = a + f * (b - a);
  }
}

// Zero the interpolated cross sections below each process's threshold.
__device__ __forceinline__ void thresholds(const MatParams& M, int sp, double T, bool& on0,
                                           bool& on1, bool& on2) {
  if (sp == EMS_GAMMA) {
    on0 = true;
    on1 = true;
    on2 = T > 2.0 * kMe;
  } else {
    on0 = sp == EMS_ELECTRON ? (T > 2.0 * M.Tc) : (T > M.Tc);
    on1 = T > M.kc;
    on2 = sp == EMS_POSITRON;
  }
}

// ln T' of the exact inverse of the piecewise-linear range table, starting the
// search at interval i0 (T' <= T, so the answer is at or below it).
template <class R>
__device__ __forceinline__ R range_inverse(const Params& P, const R* tb, R r, int i0) {
  const R* t = tb + 3;
  if (r <= t[0]) return Px<R>::lnE0(P);
  if (r >= t[(kGrid - 1) * kQ]) return Px<R>::lnE0(P) + R(kGrid - 1) * Px<R>::dln(P);
  int i = i0 > kGrid - 2 ? kGrid - 2 : i0;
  for (int k = 0; k < 4 && i > 0 && t[i * kQ] > r; ++k) --i;
  if (t[i * kQ] > r) {  // binary search in [0, i]
    int lo = 0, hi = i;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (t[mid * kQ] <= r) lo = mid;
      else hi = mid;
    }
    i = lo;
  }
  while (i < kGrid - 2 && t[(i + 1) * kQ] <= r) ++i;
  const R a = t[i * kQ], b = t[(i + 1) * kQ];
  const R f = Px<R>::dv(r - a, b - a);
  return Px<R>::lnE0(P) + ((R)i + f) * Px<R>::dln(P);
}

// ------------------------------------------------------------------ geometry


// Quadric-surface cells (paper Sec. 2.3 "Geometry and EM fields": the ORANGE model,
// cells bounded by quadric surfaces and told apart by their sense to each surface,
// one level).  Surface f(x) = qxx x^2 + qyy y^2 + qzz z^2 + qxy xy + qyz yz + qzx zx
// + px x + py y + pz z + k; a cell is the intersection of half-spaces f < 0 (side -1)
// or f > 0 (side +1).  Along a ray, f = a t^2 + B t + c.  Every expression is
// evaluated unfused in the order written: sides are decided by the sign of values
// that vanish on the surfaces.
__device__ __forceinline__ double csg_c(const double* q, double x, double y, double z) {
#pragma clang fp contract(off)
  return q[0] * x * x + q[1] * y * y + q[2] * z * z + q[3] * x * y + q[4] * y * z + q[5] * z * x +
         q[6] * x + q[7] * y + q[8] * z + q[9];
}
__device__ __forceinline__ double csg_B(const double* q, double x, double y, double z, double u,
                                        double v, double w) {
#pragma clang fp contract(off)
  return 2.0 * (q[0] * x * u + q[1] * y * v + q[2] * z * w) + q[3] * (x * v + y * u) +
         q[4] * (y * w + z * v) + q[5] * (z * u + x * w) + q[6] * u + q[7] * v + q[8] * w;
}
__device__ __forceinline__ double csg_a(const double* q, double u, double v, double w) {
#pragma clang fp contract(off)
  return q[0] * u * u + q[1] * v * v + q[2] * w * w + q[3] * u * v + q[4] * v * w + q[5] * w * u;
}

// A plane (every quadratic coefficient zero) is evaluated from its linear terms
// alone: the zero terms add nothing but the sign of a zero, which no decision reads.
__device__ __forceinline__ double plane_c(const double* q, double x, double y, double z) {
#pragma clang fp contract(off)
  return q[6] * x + q[7] * y + q[8] * z + q[9];
}
__device__ __forceinline__ double plane_B(const double* q, double u, double v, double w) {
#pragma clang fp contract(off)
  return q[6] * u + q[7] * v + q[8] * w;
}

// Side of surface q at (x,y,z) moving along (u,v,w): sign of f, on the surface the
// sign of df/dt, on a tangent the sign of a (zero counts as +1).
__device__ __forceinline__ int csg_side(const double* q, bool pl, double x, double y, double z,
                                        double u, double v, double w) {
  const double c = pl ? plane_c(q, x, y, z) : csg_c(q, x, y, z);
  if (c > 0.0) return 1;
  if (c < 0.0) return -1;
  const double B = pl ? plane_B(q, u, v, w) : csg_B(q, x, y, z, u, v, w);
  if (B > 0.0) return 1;
  if (B < 0.0) return -1;
  return (pl ? 0.0 : csg_a(q, u, v, w)) >= 0.0 ? 1 : -1;
}

// Distance to where f leaves side sg: the root at which df/dt has the sign -sg,
// written without cancellation; a root behind counts as 0 if the track is moving
// off side sg right now, else as no crossing.
__device__ __forceinline__ double csg_exit(const double* q, bool pl, double x, double y, double z,
                                           double u, double v, double w, double sg) {
#pragma clang fp contract(off)
  const double a = pl ? 0.0 : csg_a(q, u, v, w);
  const double B = pl ? plane_B(q, u, v, w) : csg_B(q, x, y, z, u, v, w);
  const double b = 0.5 * B;
  if (a == 0.0 && !(sg * b < 0.0)) return HUGE_VAL;  // a plane never left this way
  const double c = pl ? plane_c(q, x, y, z) : csg_c(q, x, y, z);
  double t;
  if (a == 0.0) {
    t = c / (-2.0 * b);
  } else {
    const double D = b * b - a * c;
    if (!(D > 0.0)) return HUGE_VAL;
    const double r = sqrt(D);
    t = sg * b <= 0.0 ? c / (-b + sg * r) : (-b - sg * r) / a;
  }
  if (!(t >= 0.0)) return sg * b < 0.0 ? 0.0 : HUGE_VAL;
  return t;
}

// Does cell m hold the point moving along (u,v,w)?  Faces on surface `forced` count
// as satisfied.
__device__ __forceinline__ bool csg_holds(const Geo& G, int m, double x, double y, double z,
                                          double u, double v, double w, int forced) {
  for (int j = G.face_off[m]; j < G.face_off[m + 1]; ++j) {
    const int f = G.faces[j];
    const int sf = f >> 1;
    if (sf == forced) continue;
    if (csg_side(G.surf + 10 * sf, G.plane[sf] != 0, x, y, z, u, v, w) != ((f & 1) ? 1 : -1))
      return false;
  }
  return true;
}

__device__ __forceinline__ int csg_locate(const Geo& G, int nvol, double x, double y, double z,
                                          double u, double v, double w) {
  for (int m = 0; m < nvol; ++m)
    if (csg_holds(G, m, x, y, z, u, v, w, -1)) return m;
  return -1;
}

// Boundary distance in cell k: the nearest exit over the cell's faces (first face
// wins ties); *left = the face crossed (surface * 2 + side), -1 if none.
__device__ __forceinline__ double csg_distance(const Geo& G, int k, double px, double py,
                                               double pz, double dx, double dy, double dz,
                                               int& left) {
  double s_min = HUGE_VAL;
  left = -1;
  for (int j = G.face_off[k]; j < G.face_off[k + 1]; ++j) {
    const int f = G.faces[j];
    const int sf = f >> 1;
    const double t =
        csg_exit(G.surf + 10 * sf, G.plane[sf] != 0, px, py, pz, dx, dy, dz, (f & 1) ? 1.0 : -1.0);
    if (t < s_min) {
      s_min = t;
      left = f;
    }
  }
  return s_min;
}

// The cell entered through face `left` of cell k at p + s d: the first cell with the
// crossed surface on the other side whose remaining faces hold at that point, else
// the first other cell without the crossed surface on the side left that holds it,
// else none (-1).  Resolved only for steps that end on the boundary.
__device__ __forceinline__ int csg_next(const Geo& G, int nvol, int k, int left, double px, double py,
                                        double pz, double dx, double dy, double dz, double s_min) {
#pragma clang fp contract(off)
  if (left < 0) return -1;
  const int sf = left >> 1, entered = left ^ 1;
  const double x = px + s_min * dx, y = py + s_min * dy, z = pz + s_min * dz;
  for (int j = G.cand_off[entered]; j < G.cand_off[entered + 1]; ++j) {
    const int m = G.cand[j];
    if (m != k && csg_holds(G, m, x, y, z, dx, dy, dz, sf)) return m;
  }
  for (int m = 0; m < nvol; ++m) {
    if (m == k) continue;
    bool has_left = false;
    for (int j = G.face_off[m]; j < G.face_off[m + 1]; ++j) has_left |= G.faces[j] == left;
    if (!has_left && csg_holds(G, m, x, y, z, dx, dy, dz, sf)) return m;
  }
  return -1;
}

__device__ __forceinline__ int locate(const Params& P, double x, double y, double z, double u,
                                      double v, double w) {
  if (P.gkind == EMS_GEOM_CSG) return csg_locate(global_geo(P), P.nvol, x, y, z, u, v, w);
  if (P.gkind == EMS_GEOM_SLABS) {
    if (fabs(x) > P.hx || fabs(y) > P.hy) return -1;
    for (int j = 0; j < P.nvol; ++j) {
      const double lo = P.bounds[j], hi = P.bounds[j + 1];
      if ((z > lo && z < hi) || (z == lo && w >= 0.0) || (z == hi && w < 0.0)) return j;
    }
    return -1;
  }
  if (fabs(z) > P.hz) return -1;
  const double r = sqrt(x * x + y * y), rd = x * u + y * v;
  for (int j = 0; j < P.nvol; ++j) {
    const double lo = P.bounds[j], hi = P.bounds[j + 1];
    if ((r > lo && r < hi) || (r == lo && rd >= 0.0) || (r == hi && rd < 0.0)) return j;
  }
  return -1;
}

// Straight-line distance to the boundary of volume `vol` and the volume beyond
// (-1 = outside the world).  Slabs: z-planes to neighbours, walls |x|,|y| to the
// outside (ties to the walls).  Shells: outer radius outward, inner radius inward,
// end caps outside (ties inner, then caps).
// With quadric cells, `next` holds -2 - (face crossed) until csg_next resolves it.
template <bool CSG>
__device__ __forceinline__ double distance(const Params& P, const Geo& G, int vol,
                                           double px, double py, double pz, double dx, double dy,
                                           double dz, int& next) {
#pragma clang fp contract(off)
  if (CSG) {
    int left;
    const double sd = csg_distance(G, vol, px, py, pz, dx, dy, dz, left);
    next = -2 - left;
    return sd;
  }
  const double* bounds = G.bounds;
  double s = HUGE_VAL;
  int nx = -1;
  if (P.gkind == EMS_GEOM_SLABS) {
    if (dz > 0.0) {
      s = (bounds[vol + 1] - pz) / dz;
      nx = vol + 1 < P.nvol ? vol + 1 : -1;
    } else if (dz < 0.0) {
      s = (bounds[vol] - pz) / dz;
      nx = vol > 0 ? vol - 1 : -1;
    }
    if (dx != 0.0) {
      const double sx = ((dx > 0.0 ? P.hx : -P.hx) - px) / dx;
      if (sx <= s) {
        s = sx;
        nx = -1;
      }
    }
    if (dy != 0.0) {
      const double sy = ((dy > 0.0 ? P.hy : -P.hy) - py) / dy;
      if (sy <= s) {
        s = sy;
        nx = -1;
      }
    }
  } else {
    const double a = dx * dx + dy * dy;
    const double b = px * dx + py * dy;
    const double r2 = px * px + py * py;
    if (a > 0.0) {
      const double Ro = bounds[vol + 1];
      const double c = r2 - Ro * Ro;
      const double D = fmax(b * b - a * c, 0.0);
      const double sq = sqrt(D);
      s = (b <= 0.0) ? (sq - b) / a : -c / (b + sq);
      nx = vol + 1 < P.nvol ? vol + 1 : -1;
      if (vol > 0 && b < 0.0) {
        const double Ri = bounds[vol];
        const double ci = r2 - Ri * Ri;
        const double Di = b * b - a * ci;
        if (Di >= 0.0) {
          const double si = ci / (sqrt(Di) - b);
          if (si <= s) {
            s = si;
            nx = vol - 1;
          }
        }
      }
    }
    if (dz != 0.0) {
      const double sz = ((dz > 0.0 ? P.hz : -P.hz) - pz) / dz;
      if (sz <= s) {
        s = sz;
        nx = -1;
      }
    }
  }
  next = nx;
  return s < 0.0 ? 0.0 : s;
}

// ------------------------------------------------------------------ kinematics

// Turn (u,v,w) by polar cosine c and azimuth (cp = cos phi, sp = sin phi) about itself,
// frame e1 = (u w, v w, -p)/p, e2 = (-v, u, 0)/p; lab frame when p^2 <= 1e-20.
__device__ __forceinline__ void rotate(double u, double v, double w, double c, double cp,
                                       double sp, double& ou, double& ov, double& ow) {
  const double s = sqrt(fmax(1.0 - c * c, 0.0));
  const double p2 = u * u + v * v;
  if (p2 > 1e-20) {
    const double p = sqrt(p2);
    const double a = s / p;
    ou = c * u + a * (u * w * cp - v * sp);
    ov = c * v + a * (v * w * cp + u * sp);
    ow = c * w - s * p * cp;
  } else {
    ou = s * cp;
    ov = s * sp;
    ow = w >= 0.0 ? c : -c;
  }
  const double n = 1.0 / sqrt(ou * ou + ov * ov + ow * ow);
  ou *= n;
  ov *= n;
  ow *= n;
}

// Direction of a*da - b*db.
__device__ __forceinline__ void mom_diff(double a, double ax, double ay, double az, double b,
                                         double bx, double by, double bz, double& ox, double& oy,
                                         double& oz) {
  ox = a * ax - b * bx;
  oy = a * ay - b * by;
  oz = a * az - b * bz;
  const double n2 = ox * ox + oy * oy + oz * oz;
  if (n2 > 0.0) {
    const double n = 1.0 / sqrt(n2);
    ox *= n;
    oy *= n;
    oz *= n;
  } else {
    ox = ax;
    oy = ay;
    oz = az;
  }
}

// ------------------------------------------------------------------ magnetic field

// Charged tracks in a uniform field B_z, always in FP64: dr/ds = d,
// dd/ds = kappa (d_y, -d_x, 0), kappa = 2.99792458 q B_z / p (1/cm, MeV/c, tesla).
constexpr int kFieldMaxSub = 10000;
constexpr double kFieldHmin = 1.0e-9;
constexpr int kFieldVacSub = 256;  // substeps of one step in vacuum
constexpr uint32_t kVacCaps = 40;  // vacuum steps in a row ending on that cap: a looper

// One classical fourth-order Runge-Kutta step of length h.  The field-step
// decisions (error against tolerance, chord against boundary) compare differences
// of nearly equal positions, so every operation here and in field_move() and
// distance() is evaluated unfused, in the order the equations are written:
// then both decisions and results are those of IEEE FP64 arithmetic, independent
// of how the compiler schedules the code.
__device__ __forceinline__ void rk4(double kappa, double h, double rx, double ry, double rz,
                                    double dx, double dy, double dz, double& ox, double& oy,
                                    double& oz, double& ex, double& ey, double& ez) {
#pragma clang fp contract(off)
  const double hh = 0.5 * h;
  // stage k: position derivative t_k, direction derivative kappa (t_k,y, -t_k,x, 0)
  const double g1x = kappa * dy, g1y = -kappa * dx;
  const double t2x = dx + hh * g1x, t2y = dy + hh * g1y;
  const double g2x = kappa * t2y, g2y = -kappa * t2x;
  const double t3x = dx + hh * g2x, t3y = dy + hh * g2y;
  const double g3x = kappa * t3y, g3y = -kappa * t3x;
  const double t4x = dx + h * g3x, t4y = dy + h * g3y;
  const double g4x = kappa * t4y, g4y = -kappa * t4x;
  const double h6 = h / 6.0;
  ox = rx + h6 * (dx + 2.0 * t2x + 2.0 * t3x + t4x);
  oy = ry + h6 * (dy + 2.0 * t2y + 2.0 * t3y + t4y);
  oz = rz + h6 * (dz + 2.0 * dz + 2.0 * dz + dz);
  ex = dx + h6 * (g1x + 2.0 * g2x + 2.0 * g3x + g4x);
  ey = dy + h6 * (g1y + 2.0 * g2y + 2.0 * g3y + g4y);
  ez = dz + h6 * 0.0;
}

// Where a curved move stands between substeps: substeps done, trial length of the
// next substep, path travelled.  nsub = 0 is a move not yet begun.
struct MoveState {
  uint32_t nsub;
  double h, travelled;
};

// Curved move within volume `vol` for at most s_max (maybe infinite): substeps
// with step-doubling error control, the boundary searched on each substep's chord
// and accepted once the chord's sagitta is within tolerance.  Returns 0 at s_max,
// 1 at a boundary (next set), 2 for a looper in matter (10^4 substeps), 3 when a
// step in vacuum used its 256 substeps (the step ends there).  The move starts from
// ms (a move begun earlier continues where it stood) and takes at most `budget`
// substeps now: when they are used up it returns 4 with ms, the position and the
// direction holding exactly the loop's state, so that continuing later takes the
// same substeps, in the same arithmetic, as one uninterrupted move.
template <bool CSG>
__device__ __forceinline__ int field_move(const Params& P, const Geo& G, int vol,
                                          double kappa, double s_max,
                                          bool vacuum, double& x, double& y, double& z,
                                          double& u, double& v, double& w, double& s_out,
                                          int& next, MoveState& ms, uint32_t& budget) {
#pragma clang fp contract(off)
  const double tol = P.ftol;
  const double limit = s_max;
  double travelled = ms.nsub ? ms.travelled : 0.0;
  double h = ms.nsub ? ms.h : (fabs(kappa) > 0.0 ? fmin(limit, 1.0 / fabs(kappa)) : limit);
  next = -1;
  const uint32_t max_sub = vacuum ? kFieldVacSub : kFieldMaxSub;
  for (uint32_t nsub = ms.nsub; nsub < max_sub; ++nsub) {
    if (budget == 0u) {  // suspended between substeps
      ms.nsub = nsub;
      ms.h = h;
      ms.travelled = travelled;
      return 4;
    }
    --budget;
    const double hh = fmin(h, limit - travelled);
    double fx, fy, fz, fu, fv, fw, mx, my, mz, mu, mv, mw, px, py, pz, pu, pv, pw;
    rk4(kappa, hh, x, y, z, u, v, w, fx, fy, fz, fu, fv, fw);
    rk4(kappa, 0.5 * hh, x, y, z, u, v, w, mx, my, mz, mu, mv, mw);
    rk4(kappa, 0.5 * hh, mx, my, mz, mu, mv, mw, px, py, pz, pu, pv, pw);
    const double err = sqrt((px - fx) * (px - fx) + (py - fy) * (py - fy) + (pz - fz) * (pz - fz));
    if (err > tol && hh > kFieldHmin) {
      h = 0.5 * hh;
      continue;
    }
    double cx = px - x, cy = py - y, cz = pz - z;
    const double L = sqrt(cx * cx + cy * cy + cz * cz);
    int nx = -1;
    double sb = HUGE_VAL;
    if (L > 0.0) {
      cx /= L;
      cy /= L;
      cz /= L;
      sb = distance<CSG>(P, G, vol, x, y, z, cx, cy, cz, nx);
    }
    if (sb < L) {
      const double qx = mx - x, qy = my - y, qz = mz - z;
      const double along = qx * cx + qy * cy + qz * cz;
      const double sx = qx - along * cx, sy = qy - along * cy, sz = qz - along * cz;
      const double sag = sqrt(sx * sx + sy * sy + sz * sz);
      if (sag <= tol || hh <= kFieldHmin) {
        if (CSG) nx = csg_next(G, P.nvol, vol, -2 - nx, x, y, z, cx, cy, cz, sb);
        const double part = hh * (sb / L);
        double ox, oy, oz, du, dv, dw;
        rk4(kappa, part, x, y, z, u, v, w, ox, oy, oz, du, dv, dw);
        x += sb * cx;
        y += sb * cy;
        z += sb * cz;
        const double n = sqrt(du * du + dv * dv + dw * dw);
        u = du / n;
        v = dv / n;
        w = dw / n;
        s_out = travelled + part;
        next = nx;
        ms.nsub = 0;
        return 1;
      }
      h = fmax(hh * (sb / L), kFieldHmin);
      continue;
    }
    x = px;
    y = py;
    z = pz;
    const double n = sqrt(pu * pu + pv * pv + pw * pw);
    u = pu / n;
    v = pv / n;
    w = pw / n;
    travelled += hh;
    if (travelled >= limit) {
      s_out = travelled;
      ms.nsub = 0;
      return 0;
    }
    h = err < tol / 32.0 ? 2.0 * hh : hh;
  }
  s_out = travelled;
  ms.nsub = 0;
  return vacuum ? 3 : 2;
}

// ------------------------------------------------------------------ track records

struct Track {
  int sp, vol;
  double x, y, z, u, v, w, T, nlam;
  uint32_t k0, k1, k2, evt, nstep, src;
  uint32_t vcap;  // field steps in vacuum that ended on their substep cap, in a row
  MoveState mv;   // a curved move suspended at the end of the last launch (mv.nsub > 0)
};

struct Sec {
  int sp;
  double T, u, v, w;
  uint32_t k0, k1, k2;
};

// Products of an interaction: up to three secondaries and the local deposit.
struct Emit {
  int nsec;
  Sec s0, s1, s2;
  double dep;
  int n_pair, n_annih;
};

// Append a secondary.  Written as per-field value selects (not a branch on which
// record to fill) so the three records stay in registers.
__device__ __forceinline__ void put(Sec& r, bool on, int sp, double T, double u, double v,
                                    double w, uint32_t k0, uint32_t k1, uint32_t k2) {
  r.sp = on ? sp : r.sp;
  r.T = on ? T : r.T;
  r.u = on ? u : r.u;
  r.v = on ? v : r.v;
  r.w = on ? w : r.w;
  r.k0 = on ? k0 : r.k0;
  r.k1 = on ? k1 : r.k1;
  r.k2 = on ? k2 : r.k2;
}

__device__ __forceinline__ void push(Emit& o, int sp, double T, double u, double v, double w,
                                     uint32_t k0, uint32_t k1, uint32_t k2) {
  const int n = o.nsec;
  put(o.s0, n == 0, sp, T, u, v, w, k0, k1, k2);
  put(o.s1, n == 1, sp, T, u, v, w, k0, k1, k2);
  put(o.s2, n == 2, sp, T, u, v, w, k0, k1, k2);
  o.nsec = n + 1;
}

// Two back-to-back photons of m c^2, isotropic, from the positron's stream at
// step 0xFFFFFFFF (draw 0 -> cos theta = 2u-1, draw 1 -> phi = 2 pi u).
template <class R>
__device__ __forceinline__ void annihilate_at_rest(const Params& P, Emit& o, uint32_t p0,
                                                   uint32_t p1, uint32_t p2) {
  Stream st;
  st.init(p0, p1, p2, kRestStep, P.seed);
  const R c = R(2) * Px<R>::uni(st.word(0)) - R(1);
  const R phi = R(kTwoPi) * Px<R>::uni(st.word(1));
  R sphi, cphi;
  Px<R>::sc(phi, &sphi, &cphi);
  const double cd = (double)c;
  const double s = sqrt(fmax(1.0 - cd * cd, 0.0));
  const double du = s * (double)cphi, dv = s * (double)sphi;
  uint32_t a, b, d;
  o.n_annih += 1;
  child_key(P.seed, p0, p1, p2, kRestStep, 0, a, b, d);
  push(o, EMS_GAMMA, kMe, du, dv, cd, a, b, d);
  child_key(P.seed, p0, p1, p2, kRestStep, 1, a, b, d);
  push(o, EMS_GAMMA, kMe, -du, -dv, -cd, a, b, d);
}

// A secondary from an interaction of the parent at its (pre-increment) step:
// tracked at or above the tracking cut, else deposited (a positron then
// annihilates at rest).
template <class R>
__device__ __forceinline__ void emit(const Params& P, Emit& o, const Track& t, int sp, double T,
                                     double u, double v, double w, uint32_t ordinal) {
  uint32_t a, b, d;
  child_key(P.seed, t.k0, t.k1, t.k2, t.nstep, ordinal, a, b, d);
  const bool charged = sp != EMS_GAMMA;
  if (T >= P.tcut && !(charged && P.charged_local)) {
    push(o, sp, T, u, v, w, a, b, d);
    return;
  }
  o.dep += T;
  if (sp == EMS_POSITRON) annihilate_at_rest<R>(P, o, a, b, d);
}

// ------------------------------------------------------------------ transport part

struct Moved {
  double dep, esc, killed, step_len;
  int limiter, process, escaped;
  int dest;        // -1 survives, -2 dead, >= 0 queue of its interaction
  bool suspended;  // the step's curved move ran out of substeps: nothing else happened
};

// The part of a step before the interaction: interaction length, cross sections,
// step limits, distance to boundary, move, continuous loss, boundary crossing or
// escape, process selection (u_1 against Sigma_i(T')), cutoffs.  A track whose
// step ends in an interaction (or a positron that stops) is sent to a queue with
// its step count not yet incremented; every other survivor's count is incremented.
template <class R, bool FIELD, bool CSG, bool MSC>
__device__ __forceinline__ void transport(const Params& P, const View<R>& V, Track& t, Moved& o,
                                          uint32_t& budget) {
  const double INF = HUGE_VAL;
  const int sp = t.sp;
  const int m = V.vmat[t.vol];
  const int mm = m < 0 ? 0 : m;
  const bool matter = m >= 0 && !V.mat[mm].vacuum;
  const R* tb = V.of(mm, sp);
  const bool charged = sp != EMS_GAMMA;
  Stream st;
  st.init(t.k0, t.k1, t.k2, t.nstep, P.seed);

  const R lnT = Px<R>::lg((R)t.T);
  if (t.nlam < 0.0) t.nlam = (double)(-Px<R>::lg(Px<R>::uni(st.word(0))));

  R q[kQ] = {R(0), R(0), R(0), R(0)};
  int i0 = 0;
  R sigtot = R(0);
  if (matter) {
    lookup<R>(P, tb, lnT, q, i0);
    bool on0, on1, on2;
    thresholds(V.mat[mm], sp, t.T, on0, on1, on2);
    sigtot = (on0 ? q[0] : R(0)) + (on1 ? q[1] : R(0)) + (on2 ? q[2] : R(0));
  }
  const double s_phys = sigtot > R(0) ? (double)Px<R>::dv((R)t.nlam, sigtot) : INF;

  const bool lossy = charged && matter && P.cont_loss;
  double s_cont = INF;
  R R0 = R(0), dres = R(0);
  if (lossy) {
    R0 = q[3];
    dres = R0 - Px<R>::rtrk(V.mat[mm], sp);
    const R rf = Px<R>::rfin(P);
    R sc = dres <= rf ? dres : fmax(Px<R>::alpha(P) * dres, rf);
    s_cont = sc < R(0) ? 0.0 : (double)sc;
  }

  int next;
  int lim;
  double s;
  if (FIELD && charged) {  // curved path up to the physics limit; a boundary met first wins
    const double p = sqrt(t.T * (t.T + 2.0 * kMe));
    const double kappa = 2.99792458 * (sp == EMS_ELECTRON ? -1.0 : 1.0) * P.bz / p;
    const int res = field_move<CSG>(P, V.g, t.vol, kappa, fmin(s_phys, s_cont), !matter, t.x, t.y, t.z,
                                    t.u, t.v, t.w, s, next, t.mv, budget);
    if (res == 4) {  // continued next launch: nλ, T, volume and step count untouched
      o.suspended = true;
      o.dest = -1;
      return;
    }
    lim = res == 1 ? 0 : (res == 2 ? 3 : (s_phys <= s_cont ? 1 : 2));
    if (res == 3) lim = t.vcap + 1 >= kVacCaps ? 3 : 4;  // 4: vacuum step on its substep cap
    t.vcap = res == 3 ? t.vcap + 1 : 0;
  } else {
    const double s_geo = distance<CSG>(P, V.g, t.vol, t.x, t.y, t.z, t.u, t.v, t.w, next);
    if (s_geo <= s_phys && s_geo <= s_cont) {
      lim = 0;
      s = s_geo;
      if (CSG) next = csg_next(V.g, P.nvol, t.vol, -2 - next, t.x, t.y, t.z, t.u, t.v, t.w, s_geo);
    } else if (s_phys <= s_cont) {
      lim = 1;
      s = s_phys;
    } else {
      lim = 2;
      s = s_cont;
    }
    t.x += s * t.u;
    t.y += s * t.v;
    t.z += s * t.w;
  }
  o.limiter = lim;
  o.step_len = s;

  const double T0 = t.T;
  double T1 = T0;
  R lnT1 = lnT;
  bool stopped = false;
  if (lossy) {
    if (lim == 2 && dres <= Px<R>::rfin(P)) {
      o.dep += T0;
      T1 = 0.0;
      stopped = true;
    } else {
      lnT1 = range_inverse<R>(P, tb, R0 - (R)s, i0);
      T1 = (double)Px<R>::ex(lnT1);
      if (T1 > T0) {
        T1 = T0;
        lnT1 = lnT;
      }
      o.dep += T0 - T1;
    }
  }
  if (lim != 1 && sigtot > R(0)) t.nlam -= s * (double)sigtot;
  // multiple scattering of an e-/e+ still moving in matter at the end of the step:
  // Highland's width theta0 = 13.6 MeV/(beta p) sqrt(s/X0) (1 + 0.038 ln(s/(X0 beta^2)))
  // at the pre-step energy (0 where the bracket is not positive), space angle
  // theta0 sqrt(-2 ln u) (at most pi), uniform azimuth
  if (MSC && charged && matter && s > 0.0 && !stopped && T1 >= P.tcut && lim != 3 &&
      !(lim == 0 && next < 0)) {
    const R Tr = (R)T0;
    const R pm = Px<R>::sq(Tr * (Tr + R(2.0 * 0.51099895)));
    const R beta = Px<R>::dv(pm, Tr + R(0.51099895));
    const R r = Px<R>::dv((R)s, Px<R>::x0(V.mat[mm]));
    const R bracket = R(1) + R(0.038) * Px<R>::lg(Px<R>::dv(r, beta * beta));
    const R th0 = (r > R(0) && bracket > R(0)) ? Px<R>::dv(R(13.6), beta * pm) * Px<R>::sq(r) * bracket
                                               : R(0);
    const R ua = Px<R>::uni(st.word(kMscDraw)), ub = Px<R>::uni(st.word(kMscDraw + 1));
    R th = th0 * Px<R>::sq(R(-2) * Px<R>::lg(ua));
    if (th > R(3.14159265358979323846)) th = R(3.14159265358979323846);
    R sth, cth, sphi, cphi;
    Px<R>::sc(th, &sth, &cth);
    Px<R>::sc(R(kTwoPi) * ub, &sphi, &cphi);
    double nu, nv, nw;
    rotate(t.u, t.v, t.w, (double)cth, (double)cphi, (double)sphi, nu, nv, nw);
    t.u = nu;
    t.v = nv;
    t.w = nw;
  }
  t.T = T1;

  o.dest = -1;
  if (stopped) {
    o.dest = sp == EMS_POSITRON ? kQRest : -2;
  } else if (charged && T1 < P.tcut) {
    o.dep += T1;
    o.dest = sp == EMS_POSITRON ? kQRest : -2;
  } else if (lim == 3) {  // looper
    o.killed += T1;
    o.dest = -2;
  } else if (lim == 0) {
    if (next < 0) {
      o.esc += T1;
      o.escaped = 1;
      o.dest = -2;
    } else {
      t.vol = next;
    }
  } else if (lim == 1) {
    t.nlam = -1.0;
    R q2[kQ];
    int i1;
    lookup<R>(P, tb, lnT1, q2, i1);
    bool on0, on1, on2;
    thresholds(V.mat[mm], sp, T1, on0, on1, on2);
    const R x0 = on0 ? q2[0] : R(0), x1 = on1 ? q2[1] : R(0), x2 = on2 ? q2[2] : R(0);
    const R tot = x0 + x1 + x2;
    if (tot > R(0)) {
      const R target = Px<R>::uni(st.word(1)) * tot;
      int p;
      if (target < x0) p = 0;
      else if (target < x0 + x1) p = 1;
      else if (target < x0 + x1 + x2) p = 2;
      else p = x2 > R(0) ? 2 : (x1 > R(0) ? 1 : 0);
      o.process = p;
      if (sp == EMS_GAMMA) o.dest = p;  // Compton, photoelectric, pair
      else if (p == 0) o.dest = sp == EMS_ELECTRON ? kQMoller : kQBhabha;
      else if (p == 1) o.dest = kQBrems;
      else o.dest = kQAnnihilation;
    }
  }
  if (o.dest == -1) {
    t.nstep += 1;
    if (t.nstep >= P.max_steps) {
      o.killed += t.T;
      o.dest = -2;
    }
  } else if (o.dest == -2) {
    t.nstep += 1;  // a track that ends here: its count now includes this step
  }
}

// ------------------------------------------------------------------ interactions

// The interaction of queue q (uniform over a block) for a track at its post-step
// state; draws from u_2 on.  On return the parent's step count is incremented and
// `alive` says whether it survives.
template <class R>
__device__ __forceinline__ void interact(const Params& P, int q, Track& t, Emit& o, bool& alive) {
  alive = true;
  if (q == kQRest) {
    alive = false;
    annihilate_at_rest<R>(P, o, t.k0, t.k1, t.k2);
    t.nstep += 1;
    return;
  }
  const int mm = P.vmat[t.vol] < 0 ? 0 : P.vmat[t.vol];
  const MatParams& M = P.mat[mm];
  Stream st;
  st.init(t.k0, t.k1, t.k2, t.nstep, P.seed);
  uint32_t d = 2;  // draw cursor of the interaction
  const double T1 = t.T;
  if (q == kQCompton) {  // 1/eps envelope
    const double E = T1;
    const R k = (R)(E / kMe);
    const R leps0 = -Px<R>::lg(R(1) + R(2) * k);
    R e = R(1), c = R(1);
    for (int tr = 0; tr < kMaxTrial; ++tr) {
      const R ua = Px<R>::uni(st.word(d)), ub = Px<R>::uni(st.word(d + 1));
      d += 2;
      e = Px<R>::ex(ua * leps0);
      c = R(1) - Px<R>::dv(R(1) - e, k * e);
      const R s2 = (R(1) - c) * (R(1) + c);
      if (ub < (R(1) + e * e - e * s2) * R(0.5)) break;
    }
    R sphi, cphi;
    Px<R>::sc(R(kTwoPi) * Px<R>::uni(st.word(d)), &sphi, &cphi);
    const double E1 = (double)e * E;
    const double Te = E - E1;
    double du, dv, dw, eu, ev, ew;
    rotate(t.u, t.v, t.w, (double)c, (double)cphi, (double)sphi, du, dv, dw);
    mom_diff(E, t.u, t.v, t.w, E1, du, dv, dw, eu, ev, ew);
    if (E1 >= P.tcut) {
      t.T = E1;
      t.u = du;
      t.v = dv;
      t.w = dw;
    } else {
      o.dep += E1;
      alive = false;
    }
    emit<R>(P, o, t, EMS_ELECTRON, Te, eu, ev, ew, 0);
  } else if (q == kQPhoto) {  // electron along the photon
    alive = false;
    emit<R>(P, o, t, EMS_ELECTRON, T1, t.u, t.v, t.w, 0);
  } else if (q == kQPair) {
    const double E = T1;
    const R a = (R)(kMe / E);
    R x = R(0.5);
    for (int tr = 0; tr < kMaxTrial; ++tr) {
      const R ua = Px<R>::uni(st.word(d)), ub = Px<R>::uni(st.word(d + 1));
      d += 2;
      x = a + (R(1) - R(2) * a) * ua;
      if (ub < R(1) - R(4.0 / 3.0) * x * (R(1) - x)) break;
    }
    const double Tm = (double)x * E - kMe;
    const double Tp = (E - 2.0 * kMe) - Tm;
    alive = false;
    o.n_pair += 1;
    emit<R>(P, o, t, EMS_ELECTRON, Tm, t.u, t.v, t.w, 0);
    emit<R>(P, o, t, EMS_POSITRON, Tp, t.u, t.v, t.w, 1);
  } else if (q == kQMoller || q == kQBhabha) {  // 1/eps^2 envelope
    const R g = (R)(T1 / kMe + 1.0);
    const R xi = (R)(T1 / M.Tc);
    R e = R(0.5);
    if (q == kQMoller) {
      const R cc = Px<R>::dv(R(2) * g - R(1), g * g);
      const R rr = Px<R>::dv(g - R(1), g);
      const R norm = Px<R>::dv(R(4) * g * g, R(9) * g * g - R(10) * g + R(5));
      for (int tr = 0; tr < kMaxTrial; ++tr) {
        const R ua = Px<R>::uni(st.word(d)), ub = Px<R>::uni(st.word(d + 1));
        d += 2;
        e = Px<R>::dv(R(1), xi - ua * (xi - R(2)));
        const R om = R(1) - e;
        const R f = rr * rr + Px<R>::dv(R(1), e * e) - Px<R>::dv(cc, e) +
                    Px<R>::dv(R(1), om * om) - Px<R>::dv(cc, om);
        if (ub < e * e * f * norm) break;
      }
    } else {
      const R b2 = R(1) - Px<R>::dv(R(1), g * g);
      const R y = Px<R>::dv(R(1), g + R(1));
      const R h = R(1) - R(2) * y;
      const R B1 = R(2) - y * y, B2 = h * (R(3) + y * y), B4 = h * h * h, B3 = B4 + h * h;
      for (int tr = 0; tr < kMaxTrial; ++tr) {
        const R ua = Px<R>::uni(st.word(d)), ub = Px<R>::uni(st.word(d + 1));
        d += 2;
        e = Px<R>::dv(R(1), xi - ua * (xi - R(1)));
        const R f = Px<R>::dv(R(1), b2 * e * e) - Px<R>::dv(B1, e) + B2 - B3 * e + B4 * e * e;
        if (ub < b2 * e * e * f) break;
      }
    }
    R sphi, cphi;
    Px<R>::sc(R(kTwoPi) * Px<R>::uni(st.word(d)), &sphi, &cphi);
    const double Td = (double)e * T1;
    const double Tp = T1 - Td;
    const double cd = fmin(sqrt(Td * (T1 + 2.0 * kMe) / (T1 * (Td + 2.0 * kMe))), 1.0);
    double du, dv, dw, pu, pv, pw;
    rotate(t.u, t.v, t.w, cd, (double)cphi, (double)sphi, du, dv, dw);
    const double P1 = sqrt(T1 * (T1 + 2.0 * kMe)), Pd = sqrt(Td * (Td + 2.0 * kMe));
    mom_diff(P1, t.u, t.v, t.w, Pd, du, dv, dw, pu, pv, pw);
    t.T = Tp;
    t.u = pu;
    t.v = pv;
    t.w = pw;
    if (Tp < P.tcut) {
      o.dep += Tp;
      alive = false;
      if (t.sp == EMS_POSITRON) annihilate_at_rest<R>(P, o, t.k0, t.k1, t.k2);
    }
    emit<R>(P, o, t, EMS_ELECTRON, Td, du, dv, dw, 0);
  } else if (q == kQBrems) {  // 1/k envelope; photon along the parent
    const double kc = M.kc;
    const R TR = (R)T1;
    const R L = Px<R>::lg((R)(T1 / kc));
    R k = (R)kc;
    for (int tr = 0; tr < kMaxTrial; ++tr) {
      const R ua = Px<R>::uni(st.word(d)), ub = Px<R>::uni(st.word(d + 1));
      d += 2;
      k = (R)kc * Px<R>::ex(ua * L);
      const R y = Px<R>::dv(k, TR);
      if (ub < R(1) - y + R(0.75) * y * y) break;
    }
    const double kd = (double)k;
    const double Tp = T1 - kd;
    t.T = Tp;
    if (Tp < P.tcut) {
      o.dep += Tp;
      alive = false;
      if (t.sp == EMS_POSITRON) annihilate_at_rest<R>(P, o, t.k0, t.k1, t.k2);
    }
    emit<R>(P, o, t, EMS_GAMMA, kd, t.u, t.v, t.w, 0);
  } else {  // annihilation in flight, 1/eps envelope
    const R g = (R)(T1 / kMe + 1.0);
    const R emin = R(0.5) * (R(1) - Px<R>::sq(Px<R>::dv(g - R(1), g + R(1))));
    const R L = Px<R>::lg(Px<R>::dv(R(1) - emin, emin));
    const R A = g * g + R(4) * g + R(1), norm = g * g + R(2) * g - R(1);
    R e = R(0.5);
    for (int tr = 0; tr < kMaxTrial; ++tr) {
      const R ua = Px<R>::uni(st.word(d)), ub = Px<R>::uni(st.word(d + 1));
      d += 2;
      e = emin * Px<R>::ex(ua * L);
      const R S = -(g + R(1)) * (g + R(1)) + Px<R>::dv(A, e) - Px<R>::dv(R(1), e * e);
      if (ub < Px<R>::dv(e * S, norm)) break;
    }
    R sphi, cphi;
    Px<R>::sc(R(kTwoPi) * Px<R>::uni(st.word(d)), &sphi, &cphi);
    const double gd = T1 / kMe + 1.0;
    const double Etot = T1 + 2.0 * kMe;
    const double E1 = (double)e * Etot;
    const double E2 = Etot - E1;
    const double ed = (double)e;
    const double c1 = fmin(fmax((ed * (gd + 1.0) - 1.0) / (ed * sqrt(gd * gd - 1.0)), -1.0), 1.0);
    double au, av, aw, bu, bv, bw;
    rotate(t.u, t.v, t.w, c1, (double)cphi, (double)sphi, au, av, aw);
    const double Pp = sqrt(T1 * (T1 + 2.0 * kMe));
    mom_diff(Pp, t.u, t.v, t.w, E1, au, av, aw, bu, bv, bw);
    alive = false;
    o.n_annih += 1;
    emit<R>(P, o, t, EMS_GAMMA, E1, au, av, aw, 0);
    emit<R>(P, o, t, EMS_GAMMA, E2, bu, bv, bw, 1);
  }
  t.nstep += 1;
}

// ------------------------------------------------------------------ kernels

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask, int lane) {
  return (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
}

__device__ __forceinline__ unsigned long long* ctr_line(const Params& P, int l) {
  return P.ctr + (size_t)l * kLineWords;
}

__device__ __forceinline__ uint32_t lo32(unsigned long long v) { return (uint32_t)(v & 0xFFFFFFFFull); }
__device__ __forceinline__ uint32_t hi32(unsigned long long v) { return (uint32_t)(v >> 32); }

// Kinetic energy of the pool after an iteration, in keV (fixed point): the
// transport survivors and the interaction outputs add to word kSEnergy of the
// block's statistics line; the host sums the copies at a synchronisation and
// admits events against it.
__device__ __forceinline__ unsigned long long kev(double T) {
  return (unsigned long long)llrint(T * 1000.0);
}
__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// statistics line of this block
__device__ __forceinline__ unsigned long long* stat_line(const Params& P) {
  return ctr_line(P, kLStats + (int)(blockIdx.x % kStatCopies));
}

// size of interaction queue q this iteration
__device__ __forceinline__ uint32_t queue_size(const Params& P, int q) {
  const unsigned long long v = *ctr_line(P, kLQueue + (q >> 1));
  return (q & 1) ? hi32(v) : lo32(v);
}

__device__ __forceinline__ uint32_t make_meta(int sp, uint32_t vol, uint32_t vcap = 0u) {
  return (uint32_t)sp | (vol << 6) | (vcap << kVcapShift);
}
// a track whose curved move was suspended: its move state is in fsub, fh, ftrav
__device__ __forceinline__ bool meta_mid_move(uint32_t meta) { return (meta & (4u | kMidMove)) == kMidMove; }
__device__ __forceinline__ uint32_t make_pending_meta(int sp, int q, uint32_t vol) {
  return (uint32_t)sp | 4u | ((uint32_t)q << 3) | (vol << 6);
}

__device__ __forceinline__ void write_track(const Pool& p, size_t j, int sp, int vol, double x,
                                            double y, double z, double u, double v, double w,
                                            double T, double nlam, uint32_t k0, uint32_t k1,
                                            uint32_t k2, uint32_t evt, uint32_t nstep,
                                            uint32_t vcap = 0u) {
  p.x[j] = x;
  p.y[j] = y;
  p.z[j] = z;
  p.u[j] = u;
  p.v[j] = v;
  p.w[j] = w;
  p.T[j] = T;
  p.nlam[j] = nlam;
  p.k0[j] = k0;
  p.k1[j] = k1;
  p.k2[j] = k2;
  p.evt[j] = evt;
  p.nstep[j] = nstep;
  p.meta[j] = make_meta(sp, (uint32_t)vol, vcap);
}

// Element offset of pool buffer (class, parity) in the pool set: for every field
// the four buffers are consecutive, photon buffers first.
__device__ __forceinline__ size_t buf_off(bool charged, int parity, uint32_t N) {
  return (size_t)((charged ? 2 : 0) + parity) * N;
}

__device__ __forceinline__ unsigned long long fixed_point(double e, double scale) {
  return (unsigned long long)llrint(e * scale);
}

// Per-event scores of one block -- tally bins, ledger words, escape-spectrum bins,
// track-steps by species and changes of the events' alive counts -- are summed in
// an LDS hash table and added to global memory once per distinct key.  The sums are
// integers (fixed-point energies, counts), so grouping them changes no result.
// Key = tag << 28 | index.
constexpr int kAggSlots = 512;
constexpr int kAggProbes = 32;
constexpr uint32_t kAggEmpty = 0xFFFFFFFFu;
constexpr uint32_t kAggIndexBits = 28;
enum AggTag : uint32_t {
  kTagTally = 0,   // index = slot * nbins + bin
  kTagLedger = 1,  // tags 1..4: ledger word tag - 1, index = slot
  kTagAlive = 5,   // index = slot, value = change of the alive count (two's complement)
  kTagEsc = 6,     // index = species * kGrid + bin of the run's escape spectrum
  kTagSteps = 7,   // index = slot * 3 + species: track-steps of the event
  kTagEvEsc = 8    // index = (slot * 3 + species) * kGrid + bin: the event's escape spectrum
};

// Bin of the number of steps n a track took: 0 for none, else 1 + floor(log2 n),
// at most kLifeBins - 1.
__device__ __forceinline__ uint32_t life_bin(uint32_t n) {
  if (n == 0u) return 0u;
  const uint32_t b = 32u - (uint32_t)__clz(n);
  return b < (uint32_t)kLifeBins ? b : (uint32_t)kLifeBins - 1u;
}

// The steps-per-track histogram of one block: a few bins take an update from nearly
// every ending track, so lanes of a wavefront that end in the same bin are counted
// together (one LDS add per distinct bin and wavefront), and the block adds its
// non-zero bins to copy blockIdx % kStatCopies once, after its last barrier.
struct LifeHist {
  uint32_t n[3 * kLifeBins];
};
__device__ __forceinline__ void life_init(LifeHist& L) {
  for (int j = threadIdx.x; j < 3 * kLifeBins; j += kBlock) L.n[j] = 0u;
}
// called by exactly the lanes whose track ends, with bin = species * kLifeBins + life_bin
__device__ __forceinline__ void life_add(LifeHist& L, uint32_t bin) {
  uint64_t pend = __ballot(1);
  while (pend) {
    const int leader = __builtin_ctzll(pend);
    const uint32_t k = (uint32_t)__shfl((int)bin, leader);
    const uint64_t same = __ballot(bin == k);
    if ((int)(threadIdx.x & 63) == leader) atomicAdd(&L.n[k], (uint32_t)__popcll(same));
    pend &= ~same;
  }
}
__device__ __forceinline__ void life_flush(const Params& P, const LifeHist& L) {
  for (int j = threadIdx.x; j < 3 * kLifeBins; j += kBlock)
    if (L.n[j]) atomicAdd(&P.life_hist[(blockIdx.x % kStatCopies) * kLifeStride + j], (unsigned long long)L.n[j]);
}
struct Agg {
  uint32_t key[kAggSlots];
  unsigned long long val[kAggSlots];
};

__device__ __forceinline__ uint32_t agg_key(uint32_t tag, uint32_t index) {
  return (tag << kAggIndexBits) | index;
}

// Add one aggregated score to global memory.  An alive count that reaches zero
// puts its event slot on the finished list.
__device__ __forceinline__ void agg_global(const Params& P, uint32_t key, unsigned long long v) {
  const uint32_t tag = key >> kAggIndexBits, idx = key & ((1u << kAggIndexBits) - 1u);
  const uint32_t copy = blockIdx.x % kEvCopies;
  if (tag == kTagTally) {
    const uint32_t e = idx / (uint32_t)P.nbins, b = idx % (uint32_t)P.nbins;
    atomicAdd(&P.tally[((size_t)e * kEvCopies + copy) * P.nbins + b], v);
  } else if (tag < kTagAlive) {
    atomicAdd(&P.ledger[((size_t)idx * kEvCopies + copy) * kLedger + (tag - kTagLedger)], v);
  } else if (tag == kTagAlive) {
    atomicAdd(&P.alive[(size_t)idx * kEvCopies + copy], (int)(long long)v);
  } else if (tag == kTagEsc) {
    atomicAdd(&P.esc_hist[idx], v);
  } else if (tag == kTagSteps) {
    atomicAdd(&P.ledger[((size_t)(idx / 3u) * kEvCopies + copy) * kLedger + kLedgerSteps + idx % 3u], v);
  } else {
    atomicAdd(&P.ev_esc[idx], v);
  }
}

__device__ __forceinline__ void agg_init(Agg& A) {
  for (int j = threadIdx.x; j < kAggSlots; j += kBlock) {
    A.key[j] = kAggEmpty;
    A.val[j] = 0ull;
  }
}

// Insert with linear probing (bounded: a crowded table falls back to a global add).
__device__ __forceinline__ void agg_add(const Params& P, Agg& A, uint32_t key,
                                        unsigned long long v) {
  uint32_t h = (key * 0x9E3779B1u) >> 23;  // top log2(kAggSlots) bits
#pragma nounroll
  for (int p = 0; p < kAggProbes; ++p) {
    const uint32_t prev = atomicCAS(&A.key[h], kAggEmpty, key);
    if (prev == kAggEmpty || prev == key) {
      atomicAdd(&A.val[h], v);
      return;
    }
    h = (h + 1u) & (kAggSlots - 1);
  }
  agg_global(P, key, v);
}

// One global add per distinct key; called after a block barrier that follows every
// lane's inserts.
__device__ __forceinline__ void agg_flush(const Params& P, Agg& A) {
  for (int j = threadIdx.x; j < kAggSlots; j += kBlock) {
    const uint32_t key = A.key[j];
    const unsigned long long v = A.val[j];
    if (key != kAggEmpty && v != 0ull) agg_global(P, key, v);
  }
}

// Bytes of the per-block LDS copy of the run data: the tables of the larger
// species class (electron and positron) of every material, then the volume
// bounds, the volume -> material map and the volume -> tally-bin map.
__host__ __device__ __forceinline__ uint32_t stage_tab_bytes(int n_mats, uint32_t rsize) {
  return (uint32_t)n_mats * 2u * kGrid * kQ * rsize;
}
__host__ __device__ __forceinline__ uint32_t align16(uint32_t b) { return (b + 15u) & ~15u; }
__host__ __device__ __forceinline__ uint32_t stage_bytes(int n_mats, int nvol, uint32_t rsize,
                                                         int n_surf = 0, int n_faces = 0) {
  uint32_t b = stage_tab_bytes(n_mats, rsize) + align16(8u * (uint32_t)(nvol + 1)) +
               2u * align16(4u * (uint32_t)nvol);
  if (n_surf > 0)  // quadric cells: surfaces, plane flags, face offsets, faces, candidates
    b += align16(80u * (uint32_t)n_surf) + align16((uint32_t)n_surf) +
         align16(4u * (uint32_t)(nvol + 1)) + align16(4u * (uint32_t)n_faces) +
         align16(4u * (uint32_t)(2 * n_surf + 1)) + align16(4u * (uint32_t)n_faces);
  return b;
}

extern __shared__ uint4 ems_stage[];  // dynamic LDS of the step kernels

// Build the block's view of the run data.  Material parameters are always copied
// to LDS; with STAGED the tables of the block's species class (charged: electron
// and positron) and the geometry maps are too.  Ends with a block barrier.
template <class R, bool STAGED>
__device__ __forceinline__ View<R> stage_view(const Params& P, bool charged_class,
                                              MatParams* sh_mat) {
  View<R> V;
  if (threadIdx.x < (unsigned)P.n_mats) sh_mat[threadIdx.x] = P.mat[threadIdx.x];
  V.mat = sh_mat;
  if (STAGED) {
    unsigned char* base = reinterpret_cast<unsigned char*>(ems_stage);
    const int sp0 = charged_class ? 1 : 0;
    const uint32_t per = (charged_class ? 2u : 1u) * kGrid * kQ;  // elements per material
    const uint32_t per16 = per * (uint32_t)sizeof(R) / 16u;
    const uint4* g = reinterpret_cast<const uint4*>(Px<R>::tab(P));
    uint4* l = ems_stage;
    for (int m = 0; m < P.n_mats; ++m) {
      const uint4* src = g + (size_t)(m * 3 + sp0) * (kGrid * kQ * sizeof(R) / 16u);
      for (uint32_t j = threadIdx.x; j < per16; j += kBlock) l[m * per16 + j] = src[j];
    }
    const uint32_t ob = stage_tab_bytes(P.n_mats, sizeof(R));
    const uint32_t om = ob + align16(8u * (uint32_t)(P.nvol + 1));
    const uint32_t oi = om + align16(4u * (uint32_t)P.nvol);
    double* bnd = reinterpret_cast<double*>(base + ob);
    int* vm = reinterpret_cast<int*>(base + om);
    int* vb = reinterpret_cast<int*>(base + oi);
    for (int j = threadIdx.x; j <= P.nvol; j += kBlock) bnd[j] = P.bounds[j];
    for (int j = threadIdx.x; j < P.nvol; j += kBlock) {
      vm[j] = P.vmat[j];
      vb[j] = P.vbin[j];
    }
    V.tab = reinterpret_cast<const R*>(base);
    V.mstride = (int)per;
    V.sp0 = sp0;
    V.g = global_geo(P);
    V.g.bounds = bnd;
    V.vmat = vm;
    V.vbin = vb;
    if (P.gkind == EMS_GEOM_CSG) {  // the cells' surfaces, faces and candidates too
      const uint32_t os = oi + align16(4u * (uint32_t)P.nvol);
      double* sf = reinterpret_cast<double*>(base + os);
      const uint32_t op = os + align16(80u * (uint32_t)P.n_surf);
      unsigned char* pl = base + op;
      const uint32_t ofo = op + align16((uint32_t)P.n_surf);
      int* fo = reinterpret_cast<int*>(base + ofo);
      const uint32_t ofa = ofo + align16(4u * (uint32_t)(P.nvol + 1));
      int* fa = reinterpret_cast<int*>(base + ofa);
      const uint32_t oco = ofa + align16(4u * (uint32_t)P.n_faces);
      int* co = reinterpret_cast<int*>(base + oco);
      const uint32_t oca = oco + align16(4u * (uint32_t)(2 * P.n_surf + 1));
      int* ca = reinterpret_cast<int*>(base + oca);
      for (int j = threadIdx.x; j < 10 * P.n_surf; j += kBlock) sf[j] = P.surf[j];
      for (int j = threadIdx.x; j < P.n_surf; j += kBlock) pl[j] = P.plane[j];
      for (int j = threadIdx.x; j <= P.nvol; j += kBlock) fo[j] = P.face_off[j];
      for (int j = threadIdx.x; j < P.n_faces; j += kBlock) {
        fa[j] = P.faces[j];
        ca[j] = P.cand[j];
      }
      for (int j = threadIdx.x; j <= 2 * P.n_surf; j += kBlock) co[j] = P.cand_off[j];
      V.g = Geo{bnd, sf, pl, fo, fa, co, ca};
    }
  } else {
    V.tab = Px<R>::tab(P);
    V.mstride = 3 * kGrid * kQ;
    V.sp0 = 0;
    V.g = global_geo(P);
    V.vmat = P.vmat;
    V.vbin = P.vbin;
  }
  __syncthreads();
  return V;
}

// One iteration, part 1, for chunk c of kBlock tracks: chunks [0, nbG) of the
// photon pool, then the charged pool (so every wavefront holds one species class).
// Every track takes up to msteps steps (a track whose interaction was put off
// goes straight to its queue); survivors go to the output pool of their class,
// tracks that interact to their process queue; both are reserved once per block.
template <class R, bool FIELD, bool STAGED, bool CSG, bool MSC>
__device__ __forceinline__ void transport_chunk(const Params& P, const Pool& S, uint32_t N, int cur,
                                                const IQueue& Q, ems_step_record* rec,
                                                uint32_t c, uint32_t nG, uint32_t nC,
                                                uint32_t nbG, uint32_t msteps) {
  const bool cblk = c >= nbG;
  const size_t io = buf_off(cblk, cur, N), oo = buf_off(cblk, 1 - cur, N);
  const uint32_t n = cblk ? nC : nG;
  const uint32_t i = (c - (cblk ? nbG : 0u)) * kBlock + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = i < n;
  Track t{};
  Moved o{};
  o.process = -1;
  o.dest = -2;
  bool stepped = false, vol_out = false, pending = false;
  uint32_t vol = 0, nsteps = 0;
  int pq = 0;
  // every field of the state is loaded at once (one round trip), checked after
  if (valid) {
    const uint32_t meta = S.meta[io + i];
    t.sp = (int)(meta & 3u);
    pending = (meta & 4u) != 0u;
    pq = (int)((meta >> 3) & 7u);
    vol = (meta >> 6) & kVolMask;
    t.vcap = meta >> kVcapShift;
    t.evt = S.evt[io + i];
    t.x = S.x[io + i];
    t.y = S.y[io + i];
    t.z = S.z[io + i];
    t.u = S.u[io + i];
    t.v = S.v[io + i];
    t.w = S.w[io + i];
    t.T = S.T[io + i];
    t.nlam = S.nlam[io + i];
    t.k0 = S.k0[io + i];
    t.k1 = S.k1[io + i];
    t.k2 = S.k2[io + i];
    t.nstep = S.nstep[io + i];
    t.src = rec ? S.src[io + i] : 0u;
    if (FIELD && meta_mid_move(meta)) {
      t.mv.nsub = S.fsub[io + i];
      t.mv.h = S.fh[io + i];
      t.mv.travelled = S.ftrav[io + i];
    }
  }
  __shared__ MatParams sh_mat[kMaxMat];
  __shared__ Agg sh_agg;
  __shared__ LifeHist sh_life;
  agg_init(sh_agg);
  life_init(sh_life);
  const View<R> V = stage_view<R, STAGED>(P, cblk, sh_mat);
  // a state that names no species, volume or event slot of this run is dropped
  const bool usable =
      valid && t.sp <= 2 && (vol == kVolOut || vol < (uint32_t)P.nvol) && t.evt < P.max_events;
  if (usable) {
    if (vol == kVolOut) {  // primary born outside the world: escapes with no step
      vol_out = true;
      t.vol = 0;
      o.esc = t.T;
      o.escaped = 1;
    } else {
      t.vol = (int)vol;
      if (pending) {
        o.dest = pq;  // its interaction, put off last iteration, is done now
      } else {
        // up to msteps steps while the track survives without interacting; each
        // step's deposit is scored in its pre-step volume
        const uint32_t e = t.evt;
        const double sc = P.scale[e];
        // substeps of curved moves this lane may take in this launch: a move that
        // needs more is suspended and continued next launch, so that a wavefront's
        // time is not set by its one lane with the longest move
        uint32_t budget = (!FIELD || rec) ? 0xFFFFFFFFu : P.sub_per_step * msteps;
        for (uint32_t m = 0; m < msteps; ++m) {
          const int v0 = t.vol;
          o = Moved{};
          o.process = -1;
          o.dest = -2;
          transport<R, FIELD, CSG, MSC>(P, V, t, o, budget);
          if (FIELD && o.suspended) break;
          ++nsteps;
          if (o.limiter == 4) break;  // a capped vacuum step: one per launch
          if (o.dep > 0.0)
            agg_add(P, sh_agg, agg_key(kTagTally, e * (uint32_t)P.nbins + (uint32_t)V.vbin[v0]),
                    fixed_point(o.dep, sc));
          if (o.dest != -1) break;
          if (FIELD && budget == 0u) break;
        }
        stepped = true;
      }
    }
  }

  // ---- scores of the event slot
  if (usable && (stepped || vol_out)) {
    const uint32_t e = t.evt;
    const double sc = P.scale[e];
    if (o.esc > 0.0) agg_add(P, sh_agg, agg_key(kTagLedger + 0, e), fixed_point(o.esc, sc));
    if (o.killed > 0.0) agg_add(P, sh_agg, agg_key(kTagLedger + 1, e), fixed_point(o.killed, sc));
    if (o.escaped) {
      const double tt = (log(o.esc) - P.lnE0) * P.inv_dlnE;
      const int b = !(tt > 0.0) ? 0 : (tt >= (double)(kGrid - 1) ? kGrid - 1 : (int)tt);
      agg_add(P, sh_agg, agg_key(kTagEsc, (uint32_t)(t.sp * kGrid + b)), 1ull);
      if (P.ev_esc)
        agg_add(P, sh_agg, agg_key(kTagEvEsc, (e * 3u + (uint32_t)t.sp) * kGrid + (uint32_t)b), 1ull);
    }
    if (o.dest == -2) {
      // the track ends: its step count (one per step, including steps that ended in
      // an interaction) goes to the event's track-steps of its species once
      const uint32_t n = vol_out ? 0u : t.nstep;
      agg_add(P, sh_agg, agg_key(kTagAlive, e), (unsigned long long)(long long)-1);
      if (n) agg_add(P, sh_agg, agg_key(kTagSteps, e * 3u + (uint32_t)t.sp), n);
      life_add(sh_life, (uint32_t)t.sp * kLifeBins + life_bin(n));
    }
    if (rec && stepped) {
      ems_step_record& r = rec[t.src];
      r.dep = o.dep;
      r.esc = o.esc;
      r.killed = o.killed;
      r.step_len = o.step_len;
      r.limiter = o.limiter;
      r.process = o.process;
      r.n_pair = 0;
      r.n_annih = 0;
      r.n_out = o.dest == -1 ? 1 : 0;
      r.escaped = o.escaped;
    }
  }
  // ---- block-level reservation: stream 0 survivors (output pool of this class),
  // 1..8 process queues, 9 positron track-steps; one 64-bit atomic per counter line
  constexpr int kW = kBlock / 64, kS = 12;
  __shared__ uint32_t sh_cnt[kW][kS];
  __shared__ uint32_t sh_base[kS];
  const int wave = threadIdx.x >> 6;
  const uint64_t mS = __ballot(o.dest == -1);
  uint64_t mq[kNumQueues];
#pragma unroll
  for (int q = 0; q < kNumQueues; ++q) mq[q] = __ballot(o.dest == q);
  const uint64_t mpend = __ballot(pending && usable);
  uint32_t wsteps = nsteps, wpos = t.sp == EMS_POSITRON ? nsteps : 0u;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    wsteps += __shfl_xor(wsteps, off);
    wpos += __shfl_xor(wpos, off);
  }
  const unsigned long long we = wave_sum64(o.dest == -1 ? kev(t.T) : 0ull);
  __shared__ unsigned long long sh_e[kW];
  __syncthreads();  // the previous chunk's readers are done with sh_cnt / sh_base
  if (lane == 0) {
    sh_e[wave] = we;
    sh_cnt[wave][0] = (uint32_t)__popcll(mS);
#pragma unroll
    for (int q = 0; q < kNumQueues; ++q) sh_cnt[wave][1 + q] = (uint32_t)__popcll(mq[q]);
    sh_cnt[wave][9] = wsteps;
    sh_cnt[wave][10] = wpos;
    sh_cnt[wave][11] = (uint32_t)__popcll(mpend);
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int l = threadIdx.x;  // counter line handled by this thread
    auto tot = [&](int st) {
      uint32_t t2 = 0;
#pragma unroll
      for (int w2 = 0; w2 < kW; ++w2) t2 += sh_cnt[w2][st];
      return t2;
    };
    if (l == 0) {
      const uint32_t a = tot(0);
      unsigned long long old = 0;
      if (a) old = atomicAdd(ctr_line(P, kLOut), cblk ? ((unsigned long long)a << 32) : a);
      sh_base[0] = cblk ? hi32(old) : lo32(old);
    } else if (l <= 4) {
      const int s0 = 1 + 2 * (l - 1);
      const uint32_t a = tot(s0), b = tot(s0 + 1);
      unsigned long long old = 0;
      if (a | b) old = atomicAdd(ctr_line(P, kLQueue + l - 1), ((unsigned long long)b << 32) | a);
      sh_base[s0] = lo32(old);
      sh_base[s0 + 1] = hi32(old);
    } else {
      // block statistics: photon or charged track-steps, positron track-steps, pending tracks
      const uint32_t st = tot(9), pos = tot(10), pend = tot(11);
      unsigned long long* L = stat_line(P);
      if (st) atomicAdd(&L[cblk ? kSStepC : kSStepG], (unsigned long long)st);
      if (pos) atomicAdd(&L[kSStepPos], (unsigned long long)pos);
      if (pend) atomicAdd(&L[kSPending], (unsigned long long)pend);
      unsigned long long e = 0;
#pragma unroll
      for (int w2 = 0; w2 < kW; ++w2) e += sh_e[w2];
      if (e) atomicAdd(&L[kSEnergy], e);
    }
  }
  __syncthreads();  // also completes every lane's score inserts
  agg_flush(P, sh_agg);
  life_flush(P, sh_life);
  if (o.dest == -1) {
    uint32_t j = sh_base[0] + lanes_below(mS, lane);
    for (int w2 = 0; w2 < wave; ++w2) j += sh_cnt[w2][0];
    write_track(S, oo + j, t.sp, t.vol, t.x, t.y, t.z, t.u, t.v, t.w, t.T, t.nlam, t.k0, t.k1,
                t.k2, t.evt, t.nstep, t.vcap);
    if (rec) S.src[oo + j] = t.src;
    if (FIELD && o.suspended) {
      S.meta[oo + j] |= kMidMove;
      S.fsub[oo + j] = t.mv.nsub;
      S.fh[oo + j] = t.mv.h;
      S.ftrav[oo + j] = t.mv.travelled;
    }
  } else if (o.dest >= 0) {  // interacting track -> its process queue
    const int q = o.dest;
    uint64_t own = mq[0];
#pragma unroll
    for (int q2 = 1; q2 < kNumQueues; ++q2) own = q == q2 ? mq[q2] : own;
    uint32_t j = sh_base[1 + q] + lanes_below(own, lane);
    for (int w2 = 0; w2 < wave; ++w2) j += sh_cnt[w2][1 + q];
    j += (uint32_t)q * Q.capacity;
    uint4* qe = Q.rec + (size_t)j * 5;
    const unsigned long long Tb = (unsigned long long)__double_as_longlong(t.T);
    reinterpret_cast<double2*>(qe)[0] = make_double2(t.x, t.y);
    reinterpret_cast<double2*>(qe)[1] = make_double2(t.z, t.u);
    reinterpret_cast<double2*>(qe)[2] = make_double2(t.v, t.w);
    qe[3] = make_uint4((uint32_t)Tb, (uint32_t)(Tb >> 32), t.k0, t.k1);
    qe[4] = make_uint4(t.k2, t.evt, t.nstep, make_meta(t.sp, (uint32_t)t.vol));
    if (rec) Q.src[j] = t.src;  // the step record of its state (diagnostics only)
  }
}

// Part 1 as a kernel, one chunk per block: pool sizes come from the admission
// cursors, so the host launches an upper bound of blocks and the surplus exits at
// once.  Every track of the pool is stepped (output room is kept by the
// interaction kernel, which puts off interactions that would not fit).
// At least four waves per SIMD without a field (four blocks of 256 per CU): the
// loop of steps would otherwise take twice the registers of one step; the curved
// move needs the registers (three waves in mixed precision: +5 % on the barrel;
// in FP64 the third wave's spills cost more than it gains).
// part: 0 every chunk, 1 the photon chunks only, 2 the charged chunks only (with a
// field, photons run in a launch of the straight-line variant: the curved-move
// variant's registers would halve their occupancy).
template <class R, bool FIELD, bool STAGED, bool CSG, bool MSC>
__global__ __launch_bounds__(kBlock, FIELD ? (sizeof(R) == 4 ? 3 : 2) : 4) void k_transport(Params P, Pool S, uint32_t N, int cur,
                                                      IQueue Q, ems_step_record* rec,
                                                      uint32_t msteps, int part) {
  const unsigned long long a = *ctr_line(P, kLAdmit);
  const uint32_t nG = lo32(a), nC = hi32(a), n = nG + nC;
  const uint32_t nbG = (nG + kBlock - 1) / kBlock, nbC = (nC + kBlock - 1) / kBlock;
  if (part != 2 && blockIdx.x == 0 && threadIdx.x == 0 && n) {
    unsigned long long* st = ctr_line(P, kLStats);
    atomicAdd(&st[kSIn], (unsigned long long)n);
    atomicAdd(&st[kSBusy], 1ull);
    atomicMax(&st[kSPeak], (unsigned long long)n);
  }
  const uint32_t first = part == 2 ? nbG : 0u, count = part == 0 ? nbG + nbC : (part == 1 ? nbG : nbC);
  if (blockIdx.x >= count) return;  // (uniform) beyond the work
  transport_chunk<R, FIELD, STAGED, CSG, MSC>(P, S, N, cur, Q, rec, first + blockIdx.x, nG, nC, nbG,
                                              msteps);
}

// Wave-aggregated append of one output stream (parent or secondary j) into the
// two class pools: per class a ballot, a rank and one atomic per wavefront.
struct OutBase {
  uint32_t g, c;
};

// One iteration, part 2: the interactions, for virtual block v.  Virtual blocks
// are partitioned among the queues (block-uniform process, so a wavefront runs
// one sampler); survivors and secondaries go to the output pool of their class.
//
// Output room: after the iteration the pool holds the transport survivors s, one
// track per put-off interaction and at most three per interaction done, so with
// the queues' entries ranked in queue order, entry r is done iff
// r < L = (bound - s - sum of queue sizes) / 2 and the pool stays within `bound`.
template <class R>
__device__ __forceinline__ void interact_chunk(const Params& P, const IQueue& Q, const Pool& S,
                                               uint32_t N, int cur, ems_step_record* rec,
                                               uint32_t v, uint32_t bound) {
  uint32_t start = 0, qsel = kNumQueues, cnt = 0, before = 0, total = 0;
#pragma unroll
  for (int q = 0; q < kNumQueues; ++q) {
    const uint32_t c = queue_size(P, q);
    const uint32_t nb = (c + kBlock - 1) / kBlock;
    if (qsel == kNumQueues && v < start + nb) {
      qsel = q;
      cnt = c;
      before = total;
    } else if (qsel == kNumQueues) {
      start += nb;
    }
    total += c;
  }
  if (qsel == kNumQueues) return;  // (uniform) beyond the work
  const unsigned long long so = *ctr_line(P, kLOut);
  const uint64_t used = (uint64_t)lo32(so) + hi32(so) + total;
  const uint32_t limit = used < bound ? (uint32_t)((bound - used) / 2) : 0u;
  __shared__ Agg sh_agg;
  __shared__ LifeHist sh_life;
  agg_init(sh_agg);
  life_init(sh_life);
  __syncthreads();  // the table is empty before any lane inserts
  const int q = (int)qsel;
  const uint32_t i = (v - start) * kBlock + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = i < cnt;
  const bool put_off = valid && before + i >= limit;
  Track t{};
  Emit o{};
  bool alive = false, looped = false;
  if (valid) {
    const uint32_t j = q * Q.capacity + i;
    const uint4* qe = Q.rec + (size_t)j * 5;
    const double2 a0 = reinterpret_cast<const double2*>(qe)[0];
    const double2 a1 = reinterpret_cast<const double2*>(qe)[1];
    const double2 a2 = reinterpret_cast<const double2*>(qe)[2];
    const uint4 a3 = qe[3], a4 = qe[4];
    t.x = a0.x;
    t.y = a0.y;
    t.z = a1.x;
    t.u = a1.y;
    t.v = a2.x;
    t.w = a2.y;
    t.T = __longlong_as_double((long long)(((unsigned long long)a3.y << 32) | a3.x));
    t.k0 = a3.z;
    t.k1 = a3.w;
    t.k2 = a4.x;
    t.evt = a4.y;
    t.nstep = a4.z;
    const uint32_t meta = a4.w;
    t.sp = (int)(meta & 3u);
    t.vol = (int)((meta >> 6) & kVolMask);
    t.src = rec ? Q.src[j] : 0u;
    t.nlam = -1.0;
    if (put_off) {
      alive = true;  // back to the pool unchanged, flagged with its queue
    } else {
      interact<R>(P, q, t, o, alive);
      if (alive && t.nstep >= P.max_steps) {  // looper cap after the interaction
        alive = false;
        looped = true;
      }
    }
  }
  // ---- scores of the event slot
  if (valid) {
    const uint32_t e = t.evt;
    const double sc = P.scale[e];
    // every local deposit is scored, a negative one too: a product sampled in FP32 a
    // hair below its kinematic limit (pair production just above threshold) gets a
    // kinetic energy of about -1e-7 of its rest energy, balanced exactly by its
    // partner's; dropping it would create that energy
    if (o.dep != 0.0)
      agg_add(P, sh_agg, agg_key(kTagTally, e * (uint32_t)P.nbins + (uint32_t)P.vbin[t.vol]),
              fixed_point(o.dep, sc));
    if (o.n_pair) agg_add(P, sh_agg, agg_key(kTagLedger + 2, e), (unsigned long long)o.n_pair);
    if (o.n_annih) agg_add(P, sh_agg, agg_key(kTagLedger + 3, e), (unsigned long long)o.n_annih);
    if (looped) agg_add(P, sh_agg, agg_key(kTagLedger + 1, e), fixed_point(t.T, sc));
    const int delta = (alive ? 1 : 0) + o.nsec - 1;
    if (delta) agg_add(P, sh_agg, agg_key(kTagAlive, e), (unsigned long long)(long long)delta);
    if (!alive) {  // the track ends: its steps go to the event's track-steps once
      if (t.nstep) agg_add(P, sh_agg, agg_key(kTagSteps, e * 3u + (uint32_t)t.sp), t.nstep);
      life_add(sh_life, (uint32_t)t.sp * kLifeBins + life_bin(t.nstep));
    }
    if (rec) {
      ems_step_record& r = rec[t.src];
      r.dep += o.dep;
      r.n_pair = o.n_pair;
      r.n_annih = o.n_annih;
      r.n_out = (alive ? 1 : 0) + o.nsec;
      if (looped) r.killed += t.T;
    }
  }
  // ---- outputs: stream 0 = parent, 1..3 = secondaries, each to its class pool
  const bool h0 = alive, h1 = o.nsec > 0, h2 = o.nsec > 1, h3 = o.nsec > 2;
  const bool g0 = t.sp == EMS_GAMMA, g1 = o.s0.sp == EMS_GAMMA, g2 = o.s1.sp == EMS_GAMMA,
             g3 = o.s2.sp == EMS_GAMMA;
  const uint64_t mg0 = __ballot(h0 && g0), mc0 = __ballot(h0 && !g0);
  const uint64_t mg1 = __ballot(h1 && g1), mc1 = __ballot(h1 && !g1);
  const uint64_t mg2 = __ballot(h2 && g2), mc2 = __ballot(h2 && !g2);
  const uint64_t mg3 = __ballot(h3 && g3), mc3 = __ballot(h3 && !g3);
  const uint32_t ng0 = __popcll(mg0), ng1 = __popcll(mg1), ng2 = __popcll(mg2), ng3 = __popcll(mg3);
  const uint32_t nc0 = __popcll(mc0), nc1 = __popcll(mc1), nc2 = __popcll(mc2), nc3 = __popcll(mc3);
  // block-level reservation of the two output pools, one atomic per block and pool
  constexpr int kW = kBlock / 64;
  __shared__ uint32_t sh_cnt[kW][3];
  __shared__ uint32_t sh_base[2];
  const int wave = threadIdx.x >> 6;
  const uint64_t moff = __ballot(put_off);
  const unsigned long long we =
      wave_sum64((h0 ? kev(t.T) : 0ull) + (h1 ? kev(o.s0.T) : 0ull) + (h2 ? kev(o.s1.T) : 0ull) +
                 (h3 ? kev(o.s2.T) : 0ull));
  __shared__ unsigned long long sh_e[kW];
  __syncthreads();  // the previous chunk's readers are done with sh_cnt / sh_base
  if (lane == 0) {
    sh_e[wave] = we;
    sh_cnt[wave][0] = ng0 + ng1 + ng2 + ng3;
    sh_cnt[wave][1] = nc0 + nc1 + nc2 + nc3;
    sh_cnt[wave][2] = (uint32_t)__popcll(moff);
  }
  __syncthreads();
  if (threadIdx.x == 0) {  // after the transport survivors: this kernel's own counter
    uint32_t a = 0, b = 0;
#pragma unroll
    for (int w2 = 0; w2 < kW; ++w2) {
      a += sh_cnt[w2][0];
      b += sh_cnt[w2][1];
    }
    unsigned long long old = 0;
    if (a | b) old = atomicAdd(ctr_line(P, kLOutI), ((unsigned long long)b << 32) | a);
    sh_base[0] = lo32(so) + lo32(old);
    sh_base[1] = hi32(so) + hi32(old);
  } else if (threadIdx.x == 64) {
    uint32_t d = 0;
#pragma unroll
    for (int w2 = 0; w2 < kW; ++w2) d += sh_cnt[w2][2];
    if (d) atomicAdd(&stat_line(P)[kSDeferred], (unsigned long long)d);
    unsigned long long e = 0;
#pragma unroll
    for (int w2 = 0; w2 < kW; ++w2) e += sh_e[w2];
    if (e) atomicAdd(&stat_line(P)[kSEnergy], e);
    // the whole capacity in use, no room for any interaction and nothing else in
    // flight: the pool cannot progress
    if (v == 0 && limit == 0 && total > 0 && lo32(so) + hi32(so) == 0 && bound >= N)
      atomicAdd(&ctr_line(P, kLStats)[kSStall], 1ull);
  }
  __syncthreads();  // also completes every lane's score inserts
  agg_flush(P, sh_agg);
  life_flush(P, sh_life);
  uint32_t bg = sh_base[0], bc = sh_base[1];
  for (int w2 = 0; w2 < wave; ++w2) {
    bg += sh_cnt[w2][0];
    bc += sh_cnt[w2][1];
  }
  const size_t offG = buf_off(false, 1 - cur, N), offC = buf_off(true, 1 - cur, N);
  if (h0) {
    const size_t j = g0 ? offG + bg + lanes_below(mg0, lane) : offC + bc + lanes_below(mc0, lane);
    write_track(S, j, t.sp, t.vol, t.x, t.y, t.z, t.u, t.v, t.w, t.T, -1.0, t.k0, t.k1, t.k2,
                t.evt, t.nstep);
    if (put_off) S.meta[j] = make_pending_meta(t.sp, q, (uint32_t)t.vol);
    if (rec) S.src[j] = t.src;
  }
  if (h1) {
    const size_t j = g1 ? offG + bg + ng0 + lanes_below(mg1, lane)
                        : offC + bc + nc0 + lanes_below(mc1, lane);
    write_track(S, j, o.s0.sp, t.vol, t.x, t.y, t.z, o.s0.u, o.s0.v, o.s0.w, o.s0.T, -1.0,
                o.s0.k0, o.s0.k1, o.s0.k2, t.evt, 0u);
  }
  if (h2) {
    const size_t j = g2 ? offG + bg + ng0 + ng1 + lanes_below(mg2, lane)
                        : offC + bc + nc0 + nc1 + lanes_below(mc2, lane);
    write_track(S, j, o.s1.sp, t.vol, t.x, t.y, t.z, o.s1.u, o.s1.v, o.s1.w, o.s1.T, -1.0,
                o.s1.k0, o.s1.k1, o.s1.k2, t.evt, 0u);
  }
  if (h3) {
    const size_t j = g3 ? offG + bg + ng0 + ng1 + ng2 + lanes_below(mg3, lane)
                        : offC + bc + nc0 + nc1 + nc2 + lanes_below(mc3, lane);
    write_track(S, j, o.s2.sp, t.vol, t.x, t.y, t.z, o.s2.u, o.s2.v, o.s2.w, o.s2.T, -1.0,
                o.s2.k0, o.s2.k1, o.s2.k2, t.evt, 0u);
  }
}

// Part 2 as a kernel, one virtual block of the queues per block.
template <class R>
__global__ __launch_bounds__(kBlock) void k_interact(Params P, IQueue Q, Pool S, uint32_t N,
                                                     int cur, ems_step_record* rec, uint32_t bound) {
  interact_chunk<R>(P, Q, S, N, cur, rec, blockIdx.x, bound);
}

// Start of an iteration.  explicit_counts: begin a sync interval -- clear every
// counter line and set the admission cursors to (nG, nC).  Otherwise continue from
// the previous iteration: its output counts (transport survivors plus tracks
// written by the interaction kernel) become this iteration's pool sizes, its output
// and queue sizes are added to the interval statistics and cleared, and its record
// -- pool sizes in, interactions queued, pool size out -- goes to log[j - 1] for
// iteration j of the interval.
__global__ void k_iter_begin(unsigned long long* ctr, int explicit_counts, uint32_t nG,
                             uint32_t nC, uint32_t j_iter, uint32_t* log) {
  const int j = threadIdx.x;
  if (explicit_counts) {
    if (j < kNumLines * kLineWords)
      ctr[j] = j == kLAdmit * kLineWords ? (((unsigned long long)nC << 32) | nG) : 0ull;
    return;
  }
  if (j != 0) return;
  const unsigned long long out = ctr[kLOut * kLineWords] + ctr[kLOutI * kLineWords];
  unsigned long long queued = 0;
  for (int l = 0; l < 4; ++l) {
    const unsigned long long v = ctr[(kLQueue + l) * kLineWords];
    queued += (v & 0xFFFFFFFFull) + (v >> 32);
    ctr[(kLQueue + l) * kLineWords] = 0ull;
  }
  if (log && j_iter > 0) {
    const unsigned long long in = ctr[kLAdmit * kLineWords];
    uint32_t* r = log + (size_t)(j_iter - 1) * 4;
    r[0] = (uint32_t)(in & 0xFFFFFFFFull);
    r[1] = (uint32_t)(in >> 32);
    r[2] = (uint32_t)queued;
    r[3] = (uint32_t)((out & 0xFFFFFFFFull) + (out >> 32));
  }
  ctr[kLStats * kLineWords + kSOut] += (out & 0xFFFFFFFFull) + (out >> 32);
  ctr[kLStats * kLineWords + kSQueued] += queued;
  ctr[kLAdmit * kLineWords] = out;
  ctr[kLOut * kLineWords] = 0ull;
  ctr[kLOutI * kLineWords] = 0ull;
  for (int c = 0; c < kStatCopies; ++c) ctr[(kLStats + c) * kLineWords + kSEnergy] = 0ull;
}

// Before the host reads the counters of a sync interval: an event in flight whose
// alive copies sum to zero has no track left anywhere (pool, queues, host spill):
// it is finished and can be read.
// Grid-stride over the slots, one count per block: one atomic per finished event
// (one per wavefront, once merged) would queue on the counter's one address.
__global__ __launch_bounds__(256) void k_done_scan(Params P) {
  __shared__ uint32_t sh_n[256 / 64];
  uint32_t done = 0;
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < P.max_events;
       e += gridDim.x * blockDim.x) {
    if (P.slot_state[e] != 1u) continue;
    int a = 0;
#pragma unroll
    for (int c = 0; c < kEvCopies; ++c) a += P.alive[(size_t)e * kEvCopies + c];
    if (a == 0) {
      P.slot_state[e] = 2u;
      ++done;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) done += __shfl_xor(done, off);
  if ((threadIdx.x & 63) == 0) sh_n[threadIdx.x >> 6] = done;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t t = sh_n[0] + sh_n[1] + sh_n[2] + sh_n[3];
    if (t) atomicAdd(reinterpret_cast<uint32_t*>(ctr_line(P, kLDone)), t);
  }
}

// Admit queued primaries: ring entries [head, head + m) appended to the photon or
// charged pool at the admission cursors (one atomic per wavefront and class).
// Blocks of kAdmitBlock threads reserve their photon and charged rows with one
// atomic on the admission cursors (a batch of 1e7 one-photon events would otherwise
// queue 1.6e5 wavefront atomics on that one address).
constexpr int kAdmitBlock = 1024;
__global__ __launch_bounds__(kAdmitBlock) void k_admit(Params P, Queue q, Pool S, uint32_t N, int cur,
                                                       uint32_t head, uint32_t m) {
  constexpr int kW = kAdmitBlock / 64;
  __shared__ uint32_t sh_g[kW], sh_c[kW];
  __shared__ unsigned long long sh_old;
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool valid = j < m;
  const uint32_t r = valid ? (head + j) % q.capacity : 0u;
  const int sp = valid ? q.species[r] : 0;
  const bool g = valid && sp == EMS_GAMMA, c = valid && sp != EMS_GAMMA;
  const uint64_t mg = __ballot(g), mc = __ballot(c);
  if (lane == 0) {
    sh_g[wave] = (uint32_t)__popcll(mg);
    sh_c[wave] = (uint32_t)__popcll(mc);
  }
  __syncthreads();
  uint32_t bg = 0, bc = 0, tg = 0, tc = 0;
#pragma unroll
  for (int w2 = 0; w2 < kW; ++w2) {
    if (w2 < wave) {
      bg += sh_g[w2];
      bc += sh_c[w2];
    }
    tg += sh_g[w2];
    tc += sh_c[w2];
  }
  if (threadIdx.x == 0)
    sh_old = (tg | tc) ? atomicAdd(ctr_line(P, kLAdmit), ((unsigned long long)tc << 32) | tg) : 0ull;
  __syncthreads();
  bg += lo32(sh_old);
  bc += hi32(sh_old);
  if (!valid) return;
  const double x = q.x[r], y = q.y[r], z = q.z[r], u = q.u[r], v = q.v[r], w = q.w[r];
  uint32_t a, b, cc, d;
  philox10(q.event_id[r], q.index[r], 0u, 0u, P.seed, 0x243F6A88u, a, b, cc, d);
  const int vol = locate(P, x, y, z, u, v, w);
  const size_t k = buf_off(!g, cur, N) + (g ? bg + lanes_below(mg, lane) : bc + lanes_below(mc, lane));
  write_track(S, k, sp, 0, x, y, z, u, v, w, q.T[r], -1.0, a, b, cc, q.slot[r], 0u);
  S.meta[k] = make_meta(sp, vol < 0 ? kVolOut : (uint32_t)vol);
}

// Copy a batch's primaries into the ring at tail; row r belongs to the event e with
// off[e] <= r < off[e+1] (binary search over the staged offsets).
// Rows that are not a valid primary set bits of *bad: 1 species, 2 kinetic energy
// not in (0, 100 GeV], 4 position not finite, 8 direction not a finite unit vector.
__global__ void k_enqueue(Queue q, uint32_t tail, const int64_t* off, const uint32_t* slots,
                          const uint32_t* ids, uint32_t n_events, const int32_t* sp,
                          const double* T, const double* pos, const double* dir, uint32_t n,
                          unsigned long long* bad) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  {
    const double t = T[r], x = pos[3 * (size_t)r], y = pos[3 * (size_t)r + 1],
                 z = pos[3 * (size_t)r + 2], u = dir[3 * (size_t)r], v = dir[3 * (size_t)r + 1],
                 w = dir[3 * (size_t)r + 2];
    const double d2 = u * u + v * v + w * w;
    unsigned long long f = 0;
    if (sp[r] < 0 || sp[r] > 2) f |= 1ull;
    if (!(t > 0.0 && t <= 1.0e5)) f |= 2ull;
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) f |= 4ull;
    if (!(fabs(d2 - 1.0) <= 1e-6)) f |= 8ull;
    if (f) atomicOr(bad, f);
  }
  uint32_t lo = 0, hi = n_events;  // find e: off[e] <= r < off[e+1]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if ((int64_t)r >= off[mid]) lo = mid;
    else hi = mid;
  }
  const uint32_t k = (tail + r) % q.capacity;
  q.species[k] = sp[r];
  q.T[k] = T[r];
  q.x[k] = pos[3 * (size_t)r];
  q.y[k] = pos[3 * (size_t)r + 1];
  q.z[k] = pos[3 * (size_t)r + 2];
  q.u[k] = dir[3 * (size_t)r];
  q.v[k] = dir[3 * (size_t)r + 1];
  q.w[k] = dir[3 * (size_t)r + 2];
  q.slot[k] = slots[lo];
  q.index[k] = (uint32_t)(r - (uint32_t)off[lo]);
  q.event_id[k] = ids[lo];
}

// Initialise the event slots of a batch: one thread per event, summing its primaries
// in their order (the same order for an event in any batch, and the oracle's).
// E_in = sum of its primaries' kinetic energies.  No tally or ledger sum of the event
// can exceed E_max = E_in + 2 m per primary positron (its annihilation releases the
// rest energy; pairs produced later consume what their positrons release), so the
// fixed-point scale 2^(61 - ceil(log2 E_max)) keeps every sum below 2^61 quanta.
// Tallies, ledger and escape spectrum zeroed; photons per event counted for the host.
// One thread per event of a submitted batch: checks its offsets (they must increase
// within [0, n]; the loop below never leaves that range), zeroes its slot's scores,
// sets its alive count and fixed-point scale.
__global__ void k_event_init(Params P, const int64_t* off, const uint32_t* slots, uint32_t n_events,
                             int64_t n, const double* T, const int32_t* sp, double* e_in,
                             double* scale, double* e_row, int64_t quarter, unsigned long long* bad) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_events) return;
  const int64_t a = off[e], b = off[e + 1];
  if (b - a < 1 || a < 0 || b > n) atomicOr(bad, (unsigned long long)kBadEmpty);
  if (b - a > quarter) atomicOr(bad, (unsigned long long)kBadLarge);
  double s = 0.0, sm = 0.0;
  const int64_t r0 = a < 0 ? 0 : a, r1 = b > n ? n : b;
  for (int64_t r = r0; r < r1; ++r) {
    const double t = T[r];
    const int k = sp[r];
    s += t;
    sm += t + (k == EMS_POSITRON ? 2.0 * kMe : 0.0);
  }
  const uint32_t slot = slots[e];
  if (slot >= P.max_events) return;  // a refused batch (no slot)
  P.slot_state[slot] = 1u;
  int ex = 0;
  if (sm > 0.0) frexp(sm, &ex);  // E_max < 2^ex
  e_in[slot] = s;
  e_row[e] = s;  // per batch row, read back by the host when it admits by energy
  scale[slot] = ldexp(1.0, 61 - ex);
  P.alive[(size_t)slot * kEvCopies] = (int)(b - a);
  for (int c = 1; c < kEvCopies; ++c) P.alive[(size_t)slot * kEvCopies + c] = 0;
}

// Zero the score rows (tally bins, ledger words and the optional escape spectrum, in
// every copy) of a batch's event slots, 16 bytes per store: consecutive threads
// write consecutive parts of a row, so the stores of slots that follow one another
// are coalesced.  A row is a multiple of 16 bytes (kEvCopies or 3 * kGrid words),
// and a batch's 16-byte parts number below 2^31 (the score indices of the event
// slots fit 28 bits; the ledger has 32 parts per slot and at most 2^26 slots).
static_assert(kEvCopies % 2 == 0 && (3 * kGrid) % 2 == 0, "score rows are whole 16-byte parts");
__device__ __forceinline__ void zero_rows(unsigned long long* base, const uint32_t* slots,
                                          uint32_t n_events, uint32_t words, uint32_t max_events) {
  uint4* const b16 = reinterpret_cast<uint4*>(base);
  const uint32_t row = words / 2u, total = n_events * row;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
    const uint32_t e = t / row, w = t - e * row;
    const uint32_t slot = slots[e];
    if (slot < max_events) b16[(size_t)slot * row + w] = make_uint4(0u, 0u, 0u, 0u);
  }
}
__global__ void k_event_zero(Params P, const uint32_t* slots, uint32_t n_events) {
  zero_rows(P.tally, slots, n_events, (uint32_t)(kEvCopies * P.nbins), P.max_events);
  zero_rows(P.ledger, slots, n_events, (uint32_t)(kEvCopies * kLedger), P.max_events);
  if (P.ev_esc) zero_rows(P.ev_esc, slots, n_events, (uint32_t)(3 * kGrid), P.max_events);
}

// ------------------------------------------------------------------ spilling to host memory
//
// When the pool runs full, the tracks of highest kinetic energy -- those that would
// still multiply -- are moved out to host memory and brought back once the pool has
// drained (paper Sec. 3.2: preferring lower-energy particles lowers the capacity a
// shower needs; secondaries may wait in CPU memory).  A track's random numbers are
// keyed by its lineage and step count, so where and when it waits changes no result.

__device__ __forceinline__ int energy_bin(const Params& P, double T) {
  const double t = (log(T) - P.lnE0) * P.inv_dlnE;
  return !(t > 0.0) ? 0 : (t >= (double)(kGrid - 1) ? kGrid - 1 : (int)t);
}

__device__ __forceinline__ void copy_track(const Pool& p, size_t from, size_t to) {
  p.x[to] = p.x[from];
  p.y[to] = p.y[from];
  p.z[to] = p.z[from];
  p.u[to] = p.u[from];
  p.v[to] = p.v[from];
  p.w[to] = p.w[from];
  p.T[to] = p.T[from];
  p.nlam[to] = p.nlam[from];
  p.k0[to] = p.k0[from];
  p.k1[to] = p.k1[from];
  p.k2[to] = p.k2[from];
  p.evt[to] = p.evt[from];
  p.nstep[to] = p.nstep[from];
  const uint32_t meta = p.meta[from];
  p.meta[to] = meta;
  if (meta_mid_move(meta)) {
    p.fsub[to] = p.fsub[from];
    p.fh[to] = p.fh[from];
    p.ftrav[to] = p.ftrav[from];
  }
}

// Histogram of the tracks of both class pools (buffer cur) over the energy grid.
__global__ void k_spill_hist(Params P, Pool S, uint32_t N, int cur, uint32_t nG, uint32_t nC,
                             unsigned long long* hist) {
  __shared__ uint32_t h[kGrid];
  for (int j = threadIdx.x; j < kGrid; j += blockDim.x) h[j] = 0u;
  __syncthreads();
  const uint32_t n = nG + nC;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const bool c = i >= nG;
    const double T = S.T[buf_off(c, cur, N) + (c ? i - nG : i)];
    atomicAdd(&h[energy_bin(P, T)], 1u);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < kGrid; j += blockDim.x)
    if (h[j]) atomicAdd(&hist[j], (unsigned long long)h[j]);
}

// Split each class pool of buffer cur into buffer 1 - cur: tracks in energy bins >=
// bmin to its top (index N-1 downward), the others compacted at its bottom.
// cnt = kept photons, kept charged, spilled photons, spilled charged.  Blocks
// [0, nbG) take photons, the rest charged tracks, so a wavefront holds one class.
__global__ void k_spill_split(Params P, Pool S, uint32_t N, int cur, uint32_t nG, uint32_t nC,
                              int bmin, uint32_t* cnt) {
  const uint32_t nbG = (nG + blockDim.x - 1) / blockDim.x;
  const bool c = blockIdx.x >= nbG;
  const uint32_t n = c ? nC : nG;
  const uint32_t i = (blockIdx.x - (c ? nbG : 0u)) * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = i < n;
  const size_t from = buf_off(c, cur, N) + i;
  bool out = false;
  if (valid) out = energy_bin(P, S.T[from]) >= bmin;
  const uint64_t mk = __ballot(valid && !out), ms = __ballot(out);
  uint32_t bk = 0, bs = 0;
  if (lane == 0) {
    if (mk) bk = atomicAdd(&cnt[c ? 1 : 0], (uint32_t)__popcll(mk));
    if (ms) bs = atomicAdd(&cnt[c ? 3 : 2], (uint32_t)__popcll(ms));
  }
  bk = __shfl(bk, 0);
  bs = __shfl(bs, 0);
  if (!valid) return;
  const size_t o = buf_off(c, 1 - cur, N);
  const size_t to = out ? o + (N - 1u - (bs + lanes_below(ms, lane))) : o + bk + lanes_below(mk, lane);
  copy_track(S, from, to);
}

// Bring m tracks back from host memory: they were copied to the bottom of the photon
// buffer 1 - cur and are appended here to the pool of their class (buffer cur) at
// the admission cursors, one atomic per wavefront and class.
__global__ void k_unspill(Params P, Pool S, uint32_t N, int cur, uint32_t m) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = j < m;
  const size_t from = buf_off(false, 1 - cur, N) + j;
  const int sp = valid ? (int)(S.meta[from] & 3u) : 0;
  const bool g = valid && sp == EMS_GAMMA, ch = valid && sp != EMS_GAMMA;
  const uint64_t mg = __ballot(g), mc = __ballot(ch);
  unsigned long long old = 0;
  if (lane == 0 && (mg | mc))
    old = atomicAdd(ctr_line(P, kLAdmit),
                    ((unsigned long long)__popcll(mc) << 32) | (unsigned long long)__popcll(mg));
  old = __shfl(old, 0);
  if (!valid) return;
  const size_t to = buf_off(!g, cur, N) + (g ? lo32(old) + lanes_below(mg, lane)
                                             : hi32(old) + lanes_below(mc, lane));
  copy_track(S, from, to);
}

// Diagnostics: event slots that never finish (alive count far from zero) with a fixed
// 2^40 fixed-point scale and zeroed tallies.
__global__ void k_slots_reset(Params P) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P.max_events) return;
  P.alive[(size_t)e * kEvCopies] = 1 << 30;
  for (int c = 1; c < kEvCopies; ++c) P.alive[(size_t)e * kEvCopies + c] = 0;
  const_cast<double*>(P.scale)[e] = 0x1p40;
  for (int b = 0; b < kEvCopies * P.nbins; ++b) P.tally[(size_t)e * kEvCopies * P.nbins + b] = 0ull;
  for (int b = 0; b < kEvCopies * kLedger; ++b) P.ledger[(size_t)e * kEvCopies * kLedger + b] = 0ull;
  if (P.ev_esc)
    for (int b = 0; b < 3 * kGrid; ++b) P.ev_esc[(size_t)e * 3 * kGrid + b] = 0ull;
}

__global__ void k_zero_u32(uint32_t* p, uint32_t n) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) p[j] = 0u;
}

__global__ void k_zero_u64(unsigned long long* p, uint32_t n) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) p[j] = 0ull;
}

// Diagnostics: external SoA <-> pool layout (states sorted into the two class
// pools at the admission cursors; src remembers the input index).
__global__ void k_pool_load(Params P, Pool S, uint32_t N, ems_track_soa s, uint32_t n) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = j < n;
  const int sp = valid ? s.species[j] : 0;
  const bool g = valid && sp == EMS_GAMMA, c = valid && sp != EMS_GAMMA;
  const uint64_t mg = __ballot(g), mc = __ballot(c);
  unsigned long long old = 0;
  if (lane == 0 && (mg | mc))
    old = atomicAdd(ctr_line(P, kLAdmit),
                    ((unsigned long long)__popcll(mc) << 32) | (unsigned long long)__popcll(mg));
  old = __shfl(old, 0);
  const uint32_t bg = lo32(old), bc = hi32(old);
  if (!valid) return;
  const size_t k = buf_off(!g, 0, N) + (g ? bg + lanes_below(mg, lane) : bc + lanes_below(mc, lane));
  write_track(S, k, sp, s.vol[j], s.x[j], s.y[j], s.z[j], s.u[j], s.v[j], s.w[j], s.T[j],
              s.nlam[j], s.k0[j], s.k1[j], s.k2[j], s.event[j], s.nstep[j],
              s.vcap ? s.vcap[j] : 0u);
  S.src[k] = j;
}

__global__ void k_pool_dump(Pool p, ems_track_soa s, uint32_t n, uint32_t off) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t j = off + i;
  s.x[j] = p.x[i];
  s.y[j] = p.y[i];
  s.z[j] = p.z[i];
  s.u[j] = p.u[i];
  s.v[j] = p.v[i];
  s.w[j] = p.w[i];
  s.T[j] = p.T[i];
  s.nlam[j] = p.nlam[i];
  s.k0[j] = p.k0[i];
  s.k1[j] = p.k1[i];
  s.k2[j] = p.k2[i];
  s.event[j] = p.evt[i];
  s.nstep[j] = p.nstep[i];
  s.species[j] = (int32_t)(p.meta[i] & 3u);
  s.vol[j] = (int32_t)((p.meta[i] >> 6) & kVolMask);
  if (s.vcap) s.vcap[j] = p.meta[i] >> kVcapShift;
}

}  // namespace ems

// ------------------------------------------------------------------ launchers (internal)

namespace ems {

static inline uint32_t blocks_for(uint64_t n, uint32_t b) { return (uint32_t)((n + b - 1) / b); }

// One iteration: transport then interactions; `bound` is an upper bound of the pool
// size (the sizes themselves stay on the device).
hipError_t launch_iteration(const Params& P, const Pool& S, uint32_t N, int cur, const IQueue& Q,
                            uint32_t bound, uint32_t msteps, bool mixed, ems_step_record* rec,
                            hipStream_t s) {
  const dim3 b(kBlock);
  const dim3 gT(blocks_for(bound, kBlock) + 1), gI(blocks_for(bound, kBlock) + kNumQueues);
  const bool field = P.bz != 0.0;
  const bool csg = P.gkind == EMS_GEOM_CSG;
  const bool msc = P.msc != 0;
  // the run data is staged in LDS when it fits the per-block budget
  const uint32_t lds = stage_bytes(P.n_mats, P.nvol, mixed ? sizeof(float) : sizeof(double),
                                  csg ? P.n_surf : 0, csg ? P.n_faces : 0);
  const bool staged = lds <= kStageMaxBytes;
  const uint32_t sh = staged ? lds : 0u;
#define EMS_LAUNCH_T(R, F, ST, G, M)                                                       \
  do {                                                                                     \
    if (F) {                                                                               \
      hipLaunchKernelGGL((k_transport<R, false, ST, G, M>), gT, b, sh, s, P, S, N, cur, Q, rec, \
                         msteps, 1);                                                       \
      hipLaunchKernelGGL((k_transport<R, F, ST, G, M>), gT, b, sh, s, P, S, N, cur, Q, rec,     \
                         msteps, 2);                                                       \
    } else {                                                                               \
      hipLaunchKernelGGL((k_transport<R, F, ST, G, M>), gT, b, sh, s, P, S, N, cur, Q, rec,     \
                         msteps, 0);                                                       \
    }                                                                                      \
  } while (0)
#define EMS_LAUNCH_TG(R, F, ST)                    \
  do {                                             \
    if (csg && msc) EMS_LAUNCH_T(R, F, ST, true, true);   \
    else if (csg) EMS_LAUNCH_T(R, F, ST, true, false);    \
    else if (msc) EMS_LAUNCH_T(R, F, ST, false, true);    \
    else EMS_LAUNCH_T(R, F, ST, false, false);            \
  } while (0)
  if (mixed) {
    if (field) {
      if (staged) EMS_LAUNCH_TG(float, true, true);
      else EMS_LAUNCH_TG(float, true, false);
    } else {
      if (staged) EMS_LAUNCH_TG(float, false, true);
      else EMS_LAUNCH_TG(float, false, false);
    }
  } else {
    if (field) {
      if (staged) EMS_LAUNCH_TG(double, true, true);
      else EMS_LAUNCH_TG(double, true, false);
    } else {
      if (staged) EMS_LAUNCH_TG(double, false, true);
      else EMS_LAUNCH_TG(double, false, false);
    }
  }
#undef EMS_LAUNCH_TG
#undef EMS_LAUNCH_T
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (mixed) hipLaunchKernelGGL(k_interact<float>, gI, b, 0, s, P, Q, S, N, cur, rec, bound);
  else hipLaunchKernelGGL(k_interact<double>, gI, b, 0, s, P, Q, S, N, cur, rec, bound);
  return hipGetLastError();
}

hipError_t launch_done_scan(const Params& P, hipStream_t s) {
  hipLaunchKernelGGL(k_done_scan, dim3(std::min<uint32_t>(blocks_for(P.max_events, 256), 2048)), dim3(256),
                     0, s, P);
  return hipGetLastError();
}

hipError_t launch_iter_begin(unsigned long long* ctr, bool explicit_counts, uint32_t nG,
                             uint32_t nC, uint32_t j_iter, uint32_t* log, hipStream_t s) {
  hipLaunchKernelGGL(k_iter_begin, dim3(1), dim3(kNumLines * kLineWords), 0, s, ctr,
                     explicit_counts ? 1 : 0, nG, nC, j_iter, log);
  return hipGetLastError();
}

hipError_t launch_admit(const Params& P, const Queue& q, const Pool& S, uint32_t N, int cur,
                        uint32_t head, uint32_t m, hipStream_t s) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_admit, dim3(blocks_for(m, kAdmitBlock)), dim3(kAdmitBlock), 0, s, P, q, S, N, cur,
                     head, m);
  return hipGetLastError();
}

hipError_t launch_enqueue(const Queue& q, uint32_t tail, const int64_t* off, const uint32_t* slots,
                          const uint32_t* ids, uint32_t n_events, const int32_t* sp,
                          const double* T, const double* pos, const double* dir, uint32_t n,
                          unsigned long long* bad, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_enqueue, dim3(blocks_for(n, 256)), dim3(256), 0, s, q, tail, off, slots, ids,
                     n_events, sp, T, pos, dir, n, bad);
  return hipGetLastError();
}

hipError_t launch_event_init(const Params& P, const int64_t* off, const uint32_t* slots,
                             const double* T, const int32_t* sp, uint32_t n_events, int64_t n,
                             double* e_in, double* scale, double* e_row, int64_t quarter,
                             unsigned long long* bad, hipStream_t s) {
  if (n_events == 0) return hipSuccess;
  hipLaunchKernelGGL(k_event_init, dim3(blocks_for(n_events, 256)), dim3(256), 0, s, P, off, slots,
                     n_events, n, T, sp, e_in, scale, e_row, quarter, bad);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint64_t words = (uint64_t)n_events * (kEvCopies / 2) * (uint64_t)(P.nbins > kLedger ? P.nbins : kLedger);
  const uint32_t blocks = (uint32_t)std::min<uint64_t>(blocks_for(words, 256), 8192);
  hipLaunchKernelGGL(k_event_zero, dim3(blocks), dim3(256), 0, s, P, slots, n_events);
  return hipGetLastError();
}


hipError_t launch_spill_hist(const Params& P, const Pool& S, uint32_t N, int cur, uint32_t nG,
                             uint32_t nC, unsigned long long* hist, hipStream_t s) {
  const uint32_t n = nG + nC;
  if (n == 0) return hipSuccess;
  const uint32_t blocks = std::min<uint32_t>(blocks_for(n, 256), 2048);
  hipLaunchKernelGGL(k_spill_hist, dim3(blocks), dim3(256), 0, s, P, S, N, cur, nG, nC, hist);
  return hipGetLastError();
}

hipError_t launch_spill_split(const Params& P, const Pool& S, uint32_t N, int cur, uint32_t nG,
                              uint32_t nC, int bmin, uint32_t* cnt, hipStream_t s) {
  const uint32_t blocks = blocks_for(nG, 256) + blocks_for(nC, 256);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_spill_split, dim3(blocks), dim3(256), 0, s, P, S, N, cur, nG, nC, bmin, cnt);
  return hipGetLastError();
}

hipError_t launch_unspill(const Params& P, const Pool& S, uint32_t N, int cur, uint32_t m,
                          hipStream_t s) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unspill, dim3(blocks_for(m, 256)), dim3(256), 0, s, P, S, N, cur, m);
  return hipGetLastError();
}

hipError_t launch_slots_reset(const Params& P, hipStream_t s) {
  hipLaunchKernelGGL(k_slots_reset, dim3(blocks_for(P.max_events, 256)), dim3(256), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u64, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_pool_load(const Params& P, const Pool& S, uint32_t N, const ems_track_soa& src,
                            uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pool_load, dim3(blocks_for(n, 256)), dim3(256), 0, s, P, S, N, src, n);
  return hipGetLastError();
}

hipError_t launch_pool_dump(const Pool& p, const ems_track_soa& dst, uint32_t n, uint32_t off,
                            hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pool_dump, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, dst, n, off);
  return hipGetLastError();
}

}  // namespace ems

namespace ems {

// Gather the tallies of n event slots into rows of (nbins + kRowLedger) doubles:
// deposits per bin, then primary energy, escaped, killed, pair conversions,
// annihilations, track-steps of photons, electrons and positrons; with esc non-null
// also the events' escape spectra (3 x kGrid counts per row).
// Rows of a read in the caller's layouts: dep (n x nbins), ledger (n x 5), steps
// (n x 3), esc (n x 3 x kGrid); a row whose slot is kNoSlot (an id not read) is zero.
__global__ void k_gather_tallies(Params P, const uint32_t* slots, uint32_t n, const double* e_in,
                                 double* dep, double* ledger, unsigned long long* steps,
                                 unsigned long long* esc) {
  const uint32_t row = blockIdx.x;
  if (row >= n) return;
  const uint32_t s = slots[row];
  const bool ok = s != kNoSlot;
  const double inv = ok ? 1.0 / P.scale[s] : 0.0;
  for (int b = threadIdx.x; b < P.nbins; b += blockDim.x) {
    unsigned long long t = 0;
    if (ok)
      for (int c = 0; c < kEvCopies; ++c) t += P.tally[((size_t)s * kEvCopies + c) * P.nbins + b];
    dep[(size_t)row * P.nbins + b] = ok ? (double)(long long)t * inv : 0.0;
  }
  if (esc && P.ev_esc)
    for (int b = threadIdx.x; b < 3 * kGrid; b += blockDim.x)
      esc[(size_t)row * 3 * kGrid + b] = ok ? P.ev_esc[(size_t)s * 3 * kGrid + b] : 0ull;
  if (threadIdx.x == 0) {
    double* L = ledger + (size_t)row * 5;
    unsigned long long* St = steps + (size_t)row * 3;
    if (!ok) {
      for (int k = 0; k < 5; ++k) L[k] = 0.0;
      for (int k = 0; k < 3; ++k) St[k] = 0ull;
      return;
    }
    unsigned long long G[kLedger];
    for (int k = 0; k < kLedger; ++k) {
      G[k] = 0ull;
      for (int c = 0; c < kEvCopies; ++c) G[k] += P.ledger[((size_t)s * kEvCopies + c) * kLedger + k];
    }
    L[0] = e_in[s];
    L[1] = (double)(long long)G[0] * inv;
    L[2] = (double)(long long)G[1] * inv;
    L[3] = (double)G[2];
    L[4] = (double)G[3];
    for (int k = 0; k < 3; ++k) St[k] = G[kLedgerSteps + k];
  }
}

// ------------------------------------------------------------------ event slots and ids

struct DeviceCas {
  __device__ static unsigned long long cas(unsigned long long* p, unsigned long long cmp,
                                           unsigned long long val) {
    return atomicCAS(p, cmp, val);
  }
};

// Submission, part 1 (one block): pre[w] = free slots in the bitmap words [0, w).
// Submission, part 1: pre[w], the free slots in words [0, w), in three passes --
// each tile of kFreeTile words (one block, 16 words per thread) counts within
// itself and keeps its total, one block turns the totals into offsets, and every
// word adds its tile's offset.
__global__ __launch_bounds__(256) void k_free_tile(EvSlots M) {
  constexpr uint32_t kPer = kFreeTile / 256u;
  __shared__ uint32_t sh_w[4];
  const uint32_t base = blockIdx.x * kFreeTile + threadIdx.x * kPer;
  uint32_t c[kPer], sum = 0;
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    c[k] = base + k < M.words ? (uint32_t)__popc(M.bits[base + k]) : 0u;
    sum += c[k];
  }
  // exclusive scan of the threads' sums: within the wavefront, then over wavefronts
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = sum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t v = __shfl_up(incl, off);
    if (lane >= off) incl += v;
  }
  if (lane == 63) sh_w[wave] = incl;
  __syncthreads();
  uint32_t run = incl - sum;
  for (int w2 = 0; w2 < wave; ++w2) run += sh_w[w2];
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    if (base + k < M.words) M.pre[base + k] = run;
    run += c[k];
  }
  if (threadIdx.x == 255) M.tile[blockIdx.x] = run;
}
__global__ __launch_bounds__(1024) void k_free_tiles(EvSlots M, uint32_t tiles) {
  __shared__ uint32_t part[1024];
  const uint32_t t = threadIdx.x, per = (tiles + 1023u) / 1024u;
  const uint32_t a = min(tiles, t * per), b = min(tiles, a + per);
  uint32_t c = 0;
  for (uint32_t j = a; j < b; ++j) c += M.tile[j];
  part[t] = c;
  __syncthreads();
  for (uint32_t off = 1; off < 1024u; off <<= 1) {  // inclusive scan of the parts
    const uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = part[t] - c;
  for (uint32_t j = a; j < b; ++j) {
    const uint32_t v = M.tile[j];
    M.tile[j] = run;
    run += v;
  }
  if (t == 1023u) M.pre[M.words] = part[t];
}
__global__ void k_free_add(EvSlots M) {
  const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < M.words && w >= kFreeTile) M.pre[w] += M.tile[w / kFreeTile];
}

// Submission, part 2: event e of the batch takes the free slot of rank e -- a batch
// gets the lowest free slots, in submission order -- and enters its id into the
// table; flag[e] = 1 if it did (a rejected batch removes exactly those entries).
__global__ void k_slots_take(EvSlots M, const uint32_t* ids, uint32_t n, uint32_t* slots,
                             uint32_t* flag, unsigned long long* bad) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  // (the host checked that the batch fits the free slots; a rank beyond them would
  // mean a lost count: the batch is then refused and no kernel touches a slot)
  const uint32_t slot = e < M.pre[M.words] ? free_slot_of_rank(M.bits, M.pre, M.words, e) : kNoSlot;
  slots[e] = slot < M.n ? slot : kNoSlot;
  if (slot >= M.n) {
    flag[e] = 0u;
    atomicOr(bad, (unsigned long long)kBadMap);
    return;
  }
  M.id[slot] = ids[e];
  const int r = map_insert<DeviceCas>(M.map, M.mask, ids[e], slot);
  flag[e] = r > 0 ? 1u : 0u;
  if (r == 0) atomicOr(bad, (unsigned long long)kBadDup);
  if (r < 0) atomicOr(bad, (unsigned long long)kBadMap);
}

// Submission, part 3 (after part 2 has read the bitmap): the taken slots leave it.
// A batch's slots rise with its event index (kNoSlot, if any, last), so lanes whose
// slots share a bitmap word are adjacent: each lane gathers the bits of the lanes
// after it in its run, and the run's first lane clears them with one atomic.
__global__ void k_slots_mark(EvSlots M, const uint32_t* slots, uint32_t n) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t sl = e < n ? slots[e] : kNoSlot;
  const bool ok = sl != kNoSlot;
  const uint32_t w = ok ? sl >> 5 : 0xFFFFFFFFu;
  uint32_t m = ok ? 1u << (sl & 31u) : 0u;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t w2 = __shfl_down(w, off), m2 = __shfl_down(m, off);
    if (lane + off < 64 && w2 == w) m |= m2;
  }
  const uint32_t wp = __shfl_up(w, 1);
  if (ok && (lane == 0 || wp != w)) atomicAnd(&M.bits[w], ~m);
}

// A rejected batch: its entries are erased and its slots are free again.
__global__ void k_slots_undo(EvSlots M, const uint32_t* ids, const uint32_t* slots,
                             const uint32_t* flag, uint32_t n) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n || slots[e] == kNoSlot) return;
  M.state[slots[e]] = 0u;
  atomicOr(&M.bits[slots[e] >> 5], 1u << (slots[e] & 31u));
  if (flag[e]) map_erase(M.map, M.mask, ids[e], slots[e]);
}

// Reset: every slot free, table empty.
__global__ void k_events_reset(EvSlots M) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j <= M.mask) M.map[j] = 0ull;
  if (j < M.words) {
    const uint32_t left = M.n - 32u * j;  // slots in this word
    M.bits[j] = left >= 32u ? 0xFFFFFFFFu : ((1u << left) - 1u);
  }
  if (j < M.n) {
    M.state[j] = 0u;
    M.claim[j] = kNoSlot;
  }
}

// Rebuild the table without its erased entries: clear, then re-enter the id of every
// slot in use.
__global__ void k_map_clear(EvSlots M) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j <= M.mask) M.map[j] = 0ull;
}
__global__ void k_map_refill(EvSlots M) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < M.n && M.state[j] != 0u) (void)map_insert<DeviceCas>(M.map, M.mask, M.id[j], j);
}

// Read, part 1: the slot of each id; a finished slot is claimed by the first
// position naming it (claim = least position).
__global__ void k_read_find(EvSlots M, const uint32_t* ids, uint32_t n, uint32_t* slots) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t h = map_find(M.map, M.mask, ids[i]);
  const uint32_t slot = h == kNoSlot ? kNoSlot : map_slot(M.map, h);
  slots[i] = slot;
  if (slot != kNoSlot && M.state[slot] == 2u) atomicMin(&M.claim[slot], i);
}

// Read, part 2: status of each position (EMS_OK for the claiming position of a
// finished slot, EMS_NOT_READY for an event in flight, EMS_E_ARG for an unknown id
// or a repeat); slots[i] = kNoSlot unless read here.
__global__ void k_read_status(EvSlots M, uint32_t n, uint32_t* slots, int32_t* status) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t slot = slots[i];
  int32_t st = EMS_E_ARG;
  if (slot != kNoSlot) {
    const uint32_t s = M.state[slot];
    if (s == 2u) st = M.claim[slot] == i ? EMS_OK : EMS_E_ARG;
    else if (s == 1u) st = EMS_NOT_READY;
  }
  status[i] = st;
  if (st != EMS_OK) slots[i] = kNoSlot;
}

// A read that failed after part 2: its claims are withdrawn, nothing is released.
__global__ void k_read_unclaim(EvSlots M, const uint32_t* slots, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && slots[i] != kNoSlot) M.claim[slots[i]] = kNoSlot;
}

// Read, part 3: release every slot read -- erase its id, free it.
__global__ void k_read_release(EvSlots M, const uint32_t* ids, const uint32_t* slots, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t slot = slots[i];
  if (slot == kNoSlot) return;
  map_erase(M.map, M.mask, ids[i], slot);
  M.state[slot] = 0u;
  M.claim[slot] = kNoSlot;
  atomicOr(&M.bits[slot >> 5], 1u << (slot & 31u));
}

hipError_t launch_gather_tallies(const Params& P, const uint32_t* slots, uint32_t n,
                                 const double* e_in, double* dep, double* ledger,
                                 unsigned long long* steps, unsigned long long* esc, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_tallies, dim3(n), dim3(128), 0, s, P, slots, n, e_in, dep, ledger, steps,
                     esc);
  return hipGetLastError();
}

hipError_t launch_slots_take(const EvSlots& M, const uint32_t* ids, uint32_t n, uint32_t* slots,
                             uint32_t* flag, unsigned long long* bad, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t tiles = (M.words + kFreeTile - 1) / kFreeTile;
  hipLaunchKernelGGL(k_free_tile, dim3(tiles), dim3(256), 0, s, M);
  hipLaunchKernelGGL(k_free_tiles, dim3(1), dim3(1024), 0, s, M, tiles);
  if (tiles > 1) hipLaunchKernelGGL(k_free_add, dim3(blocks_for(M.words, 256)), dim3(256), 0, s, M);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_slots_take, dim3(blocks_for(n, 256)), dim3(256), 0, s, M, ids, n, slots, flag,
                     bad);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_slots_mark, dim3(blocks_for(n, 256)), dim3(256), 0, s, M, slots, n);
  return hipGetLastError();
}

hipError_t launch_slots_undo(const EvSlots& M, const uint32_t* ids, const uint32_t* slots,
                             const uint32_t* flag, uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_slots_undo, dim3(blocks_for(n, 256)), dim3(256), 0, s, M, ids, slots, flag, n);
  return hipGetLastError();
}

hipError_t launch_events_reset(const EvSlots& M, hipStream_t s) {
  const uint64_t n = std::max<uint64_t>((uint64_t)M.mask + 1u, M.n);  // >= words
  hipLaunchKernelGGL(k_events_reset, dim3(blocks_for(n, 256)), dim3(256), 0, s, M);
  return hipGetLastError();
}

hipError_t launch_map_rebuild(const EvSlots& M, hipStream_t s) {
  hipLaunchKernelGGL(k_map_clear, dim3(blocks_for((uint64_t)M.mask + 1u, 256)), dim3(256), 0, s, M);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_map_refill, dim3(blocks_for(M.n, 256)), dim3(256), 0, s, M);
  return hipGetLastError();
}

hipError_t launch_read_find(const EvSlots& M, const uint32_t* ids, uint32_t n, uint32_t* slots,
                            int32_t* status, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_read_find, dim3(blocks_for(n, 256)), dim3(256), 0, s, M, ids, n, slots);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_read_status, dim3(blocks_for(n, 256)), dim3(256), 0, s, M, n, slots, status);
  return hipGetLastError();
}

hipError_t launch_read_unclaim(const EvSlots& M, const uint32_t* slots, uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_read_unclaim, dim3(blocks_for(n, 256)), dim3(256), 0, s, M, slots, n);
  return hipGetLastError();
}

hipError_t launch_read_release(const EvSlots& M, const uint32_t* ids, const uint32_t* slots,
                               uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_read_release, dim3(blocks_for(n, 256)), dim3(256), 0, s, M, ids, slots, n);
  return hipGetLastError();
}

}  // namespace ems
