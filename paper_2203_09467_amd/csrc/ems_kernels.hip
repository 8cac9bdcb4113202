// ems_kernels.hip -- gfx950 kernels of the electromagnetic-shower step loop.
//
// One lane per track (paper Sec. 2.1 "Code Architecture").  A step iteration is
// one fused kernel over the compacted pool: cross-section lookup, interaction
// length sampling, continuous step limit, distance to boundary, move and
// continuous loss, discrete interaction with secondary emission, cutoffs, and
// tallies (paper Sec. 2.2 items (i)-(vi)); survivors and secondaries are then
// written, compacted, into the other pool buffer with one atomic per wavefront
// (ballot + popcount prefix), the wave-aggregated form of the paper's atomic
// stack allocator (Sec. 2.1).  Nothing here is a dense contraction, so there is
// no MFMA: the kernel streams SoA state (coalesced 64-lane accesses) and reads
// the small cross-section tables through the L1/L2 caches.
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
};

// ------------------------------------------------------------------ tables

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
__device__ __forceinline__ void lookup(const Params& P, int m, int sp, R lnT, R q[kQ], int& i) {
  R f;
  grid_pos<R>(P, lnT, i, f);
  const R* t = Px<R>::tab(P) + ((size_t)(m * 3 + sp) * kGrid + i) * kQ;
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
__device__ __forceinline__ R range_inverse(const Params& P, int m, int sp, R r, int i0) {
  const R* t = Px<R>::tab(P) + (size_t)(m * 3 + sp) * kGrid * kQ + 3;
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

__device__ __forceinline__ int locate(const Params& P, double x, double y, double z, double u,
                                      double v, double w) {
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
__device__ __forceinline__ double distance(const Params& P, int vol, double px, double py,
                                           double pz, double dx, double dy, double dz,
                                           int& next) {
  double s = HUGE_VAL;
  int nx = -1;
  if (P.gkind == EMS_GEOM_SLABS) {
    if (dz > 0.0) {
      s = (P.bounds[vol + 1] - pz) / dz;
      nx = vol + 1 < P.nvol ? vol + 1 : -1;
    } else if (dz < 0.0) {
      s = (P.bounds[vol] - pz) / dz;
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
      const double Ro = P.bounds[vol + 1];
      const double c = r2 - Ro * Ro;
      const double D = fmax(b * b - a * c, 0.0);
      const double sq = sqrt(D);
      s = (b <= 0.0) ? (sq - b) / a : -c / (b + sq);
      nx = vol + 1 < P.nvol ? vol + 1 : -1;
      if (vol > 0 && b < 0.0) {
        const double Ri = P.bounds[vol];
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

// ------------------------------------------------------------------ one step

struct Sec {
  int sp;
  double T, u, v, w;
  uint32_t k0, k1, k2;
};

struct StepOut {
  int nsec;
  Sec s0, s1, s2;
  bool alive;
  double dep, esc, killed, step_len;
  int n_pair, n_annih, limiter, process, escaped;
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

__device__ __forceinline__ void push(StepOut& o, int sp, double T, double u, double v, double w,
                                     uint32_t k0, uint32_t k1, uint32_t k2) {
  const int n = o.nsec;
  put(o.s0, n == 0, sp, T, u, v, w, k0, k1, k2);
  put(o.s1, n == 1, sp, T, u, v, w, k0, k1, k2);
  put(o.s2, n == 2, sp, T, u, v, w, k0, k1, k2);
  o.nsec = n + 1;
}

struct Track {
  int sp, vol;
  double x, y, z, u, v, w, T, nlam;
  uint32_t k0, k1, k2, evt, nstep;
};

// Two back-to-back photons of m c^2, isotropic, from the positron's stream at
// step 0xFFFFFFFF (draw 0 -> cos theta = 2u-1, draw 1 -> phi = 2 pi u).
template <class R>
__device__ __forceinline__ void annihilate_at_rest(const Params& P, StepOut& o, uint32_t p0, uint32_t p1,
                                   uint32_t p2) {
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

// A secondary from an interaction of the parent at (its pre-increment) step.
template <class R>
__device__ __forceinline__ void emit(const Params& P, StepOut& o, const Track& t, int sp,
                                     double T, double u, double v, double w, uint32_t ordinal) {
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

// One step of an alive track (see the file header for the order of operations).
template <class R>
__device__ __forceinline__ void step_track(const Params& P, Track& t, StepOut& o) {
  const double INF = HUGE_VAL;
  const int sp = t.sp;
  const int m = P.vmat[t.vol];
  const bool matter = m >= 0 && !P.mat[m < 0 ? 0 : m].vacuum;
  const bool charged = sp != EMS_GAMMA;
  const int mm = m < 0 ? 0 : m;
  Stream st;
  st.init(t.k0, t.k1, t.k2, t.nstep, P.seed);

  const R lnT = Px<R>::lg((R)t.T);
  if (t.nlam < 0.0) t.nlam = (double)(-Px<R>::lg(Px<R>::uni(st.word(0))));

  R q[kQ] = {R(0), R(0), R(0), R(0)};
  int i0 = 0;
  R sigtot = R(0);
  if (matter) {
    lookup<R>(P, mm, sp, lnT, q, i0);
    bool on0, on1, on2;
    thresholds(P.mat[mm], sp, t.T, on0, on1, on2);
    sigtot = (on0 ? q[0] : R(0)) + (on1 ? q[1] : R(0)) + (on2 ? q[2] : R(0));
  }
  const double s_phys = sigtot > R(0) ? (double)Px<R>::dv((R)t.nlam, sigtot) : INF;

  const bool lossy = charged && matter && P.cont_loss;
  double s_cont = INF;
  R R0 = R(0), dres = R(0);
  if (lossy) {
    R0 = q[3];
    dres = R0 - Px<R>::rtrk(P.mat[mm], sp);
    const R rf = Px<R>::rfin(P);
    R sc = dres <= rf ? dres : fmax(Px<R>::alpha(P) * dres, rf);
    s_cont = sc < R(0) ? 0.0 : (double)sc;
  }

  int next;
  const double s_geo = distance(P, t.vol, t.x, t.y, t.z, t.u, t.v, t.w, next);
  int lim;
  double s;
  if (s_geo <= s_phys && s_geo <= s_cont) {
    lim = 0;
    s = s_geo;
  } else if (s_phys <= s_cont) {
    lim = 1;
    s = s_phys;
  } else {
    lim = 2;
    s = s_cont;
  }
  o.limiter = lim;
  o.step_len = s;
  t.x += s * t.u;
  t.y += s * t.v;
  t.z += s * t.w;

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
      lnT1 = range_inverse<R>(P, mm, sp, R0 - (R)s, i0);
      T1 = (double)Px<R>::ex(lnT1);
      if (T1 > T0) {
        T1 = T0;
        lnT1 = lnT;
      }
      o.dep += T0 - T1;
    }
  }
  if (lim != 1 && sigtot > R(0)) t.nlam -= s * (double)sigtot;
  t.T = T1;

  bool alive = true;
  if (stopped) {
    alive = false;
    if (sp == EMS_POSITRON) annihilate_at_rest<R>(P, o, t.k0, t.k1, t.k2);
  } else if (charged && T1 < P.tcut) {
    o.dep += T1;
    alive = false;
    if (sp == EMS_POSITRON) annihilate_at_rest<R>(P, o, t.k0, t.k1, t.k2);
  } else if (lim == 0) {
    if (next < 0) {
      o.esc += T1;
      o.escaped = 1;
      alive = false;
    } else {
      t.vol = next;
    }
  } else if (lim == 1) {
    t.nlam = -1.0;
    R q2[kQ];
    int i1;
    lookup<R>(P, mm, sp, lnT1, q2, i1);
    bool on0, on1, on2;
    thresholds(P.mat[mm], sp, T1, on0, on1, on2);
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
      uint32_t d = 2;  // draw cursor of the interaction
      const MatParams& M = P.mat[mm];
      if (sp == EMS_GAMMA) {
        const double E = T1;
        if (p == 0) {  // Compton, 1/eps envelope
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
        } else if (p == 1) {  // photoelectric: electron along the photon
          alive = false;
          emit<R>(P, o, t, EMS_ELECTRON, E, t.u, t.v, t.w, 0);
        } else {  // pair
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
        }
      } else {
        const R TR = (R)T1;
        if (p == 0) {  // Moller / Bhabha, 1/eps^2 envelope
          const R g = (R)(T1 / kMe + 1.0);
          const R xi = (R)(T1 / M.Tc);
          R e = R(0.5);
          if (sp == EMS_ELECTRON) {
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
            if (sp == EMS_POSITRON) annihilate_at_rest<R>(P, o, t.k0, t.k1, t.k2);
          }
          emit<R>(P, o, t, EMS_ELECTRON, Td, du, dv, dw, 0);
        } else if (p == 1) {  // bremsstrahlung, 1/k envelope; photon along the parent
          const double kc = M.kc;
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
            if (sp == EMS_POSITRON) annihilate_at_rest<R>(P, o, t.k0, t.k1, t.k2);
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
      }
    }
  }
  t.nstep += 1;
  if (alive && t.nstep >= P.max_steps) {
    o.killed += t.T;
    alive = false;
  }
  o.alive = alive;
}

// ------------------------------------------------------------------ kernels

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask, int lane) {
  return (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
}

__device__ __forceinline__ void write_track(const Pool& p, uint32_t j, int sp, int vol, double x,
                                            double y, double z, double u, double v, double w,
                                            double T, double nlam, uint32_t k0, uint32_t k1,
                                            uint32_t k2, uint32_t evt, uint32_t nstep) {
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
  p.meta[j] = (uint32_t)sp | ((uint32_t)vol << 2);
}

__device__ __forceinline__ unsigned long long fixed_point(double e, double scale) {
  return (unsigned long long)llrint(e * scale);
}

// One step iteration: tracks [0, n_in) of `in`; the first n_step are stepped,
// the rest are copied unchanged (deferred for lack of output room).  Outputs are
// appended to `out` at counters[0].
template <class R>
__global__ __launch_bounds__(kBlock) void k_step(Params P, Pool in, Pool out, uint32_t n_in,
                                                 uint32_t n_step, ems_step_record* rec) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = i < n_in;
  Track t{};
  StepOut o{};
  o.process = -1;
  bool stepped = false, keep = false;
  int vol_out = 0;
  bool usable = valid;
  uint32_t vol = 0;
  if (valid) {
    const uint32_t meta = in.meta[i];
    t.sp = (int)(meta & 3u);
    vol = meta >> 2;
    t.evt = in.evt[i];
    // a state that names no species, volume or event slot of this run is dropped
    usable = t.sp <= 2 && (vol == kVolOut || vol < (uint32_t)P.nvol) && t.evt < P.max_events;
  }
  if (usable) {
    t.x = in.x[i];
    t.y = in.y[i];
    t.z = in.z[i];
    t.u = in.u[i];
    t.v = in.v[i];
    t.w = in.w[i];
    t.T = in.T[i];
    t.nlam = in.nlam[i];
    t.k0 = in.k0[i];
    t.k1 = in.k1[i];
    t.k2 = in.k2[i];
    t.nstep = in.nstep[i];
    if (vol == kVolOut) {  // primary born outside the world: escapes with no step
      t.vol = 0;
      o.esc = t.T;
      o.escaped = 1;
      o.alive = false;
      stepped = false;
      keep = false;
      vol_out = 1;
    } else if (i < n_step) {
      t.vol = (int)vol;
      step_track<R>(P, t, o);
      stepped = true;
      keep = o.alive;
    } else {
      t.vol = (int)vol;
      keep = true;
    }
  }
  const int dep_vol_bin = (usable && !vol_out) ? P.vbin[(int)vol] : 0;

  // ---- wave-aggregated allocation of output slots
  const uint64_t mP = __ballot(keep);
  const uint64_t m0 = __ballot(o.nsec > 0);
  const uint64_t m1 = __ballot(o.nsec > 1);
  const uint64_t m2 = __ballot(o.nsec > 2);
  const uint32_t cP = (uint32_t)__popcll(mP), c0 = (uint32_t)__popcll(m0),
                 c1 = (uint32_t)__popcll(m1), c2 = (uint32_t)__popcll(m2);
  const uint32_t total = cP + c0 + c1 + c2;
  uint32_t base = 0;
  if (lane == 0 && total) base = atomicAdd(&P.counters[0], total);
  base = __shfl(base, 0);
  if (keep)
    write_track(out, base + lanes_below(mP, lane), t.sp, t.vol, t.x, t.y, t.z, t.u, t.v, t.w, t.T,
                t.nlam, t.k0, t.k1, t.k2, t.evt, t.nstep);
  if (o.nsec > 0)
    write_track(out, base + cP + lanes_below(m0, lane), o.s0.sp, t.vol, t.x, t.y, t.z, o.s0.u,
                o.s0.v, o.s0.w, o.s0.T, -1.0, o.s0.k0, o.s0.k1, o.s0.k2, t.evt, 0);
  if (o.nsec > 1)
    write_track(out, base + cP + c0 + lanes_below(m1, lane), o.s1.sp, t.vol, t.x, t.y, t.z,
                o.s1.u, o.s1.v, o.s1.w, o.s1.T, -1.0, o.s1.k0, o.s1.k1, o.s1.k2, t.evt, 0);
  if (o.nsec > 2)
    write_track(out, base + cP + c0 + c1 + lanes_below(m2, lane), o.s2.sp, t.vol, t.x, t.y, t.z,
                o.s2.u, o.s2.v, o.s2.w, o.s2.T, -1.0, o.s2.k0, o.s2.k1, o.s2.k2, t.evt, 0);

  // ---- run counters: track-steps by species, one atomic per wave
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const uint64_t ms = __ballot(stepped && t.sp == s);
    if (lane == 0 && ms) atomicAdd(&P.steps[s], (unsigned long long)__popcll(ms));
  }

  if (!usable) return;
  // ---- tallies of the event slot
  const uint32_t e = t.evt;
  if (stepped || vol_out) {
    const double sc = P.scale[e];
    if (o.dep > 0.0) atomicAdd(&P.tally[(size_t)e * P.nbins + dep_vol_bin], fixed_point(o.dep, sc));
    if (o.esc > 0.0) atomicAdd(&P.ledger[(size_t)e * kLedger + 0], fixed_point(o.esc, sc));
    if (o.killed > 0.0) atomicAdd(&P.ledger[(size_t)e * kLedger + 1], fixed_point(o.killed, sc));
    if (o.n_pair) atomicAdd(&P.ledger[(size_t)e * kLedger + 2], (unsigned long long)o.n_pair);
    if (o.n_annih) atomicAdd(&P.ledger[(size_t)e * kLedger + 3], (unsigned long long)o.n_annih);
    if (o.escaped) {
      const double tt = (log(o.esc) - P.lnE0) * P.inv_dlnE;
      int b = !(tt > 0.0) ? 0 : (tt >= (double)(kGrid - 1) ? kGrid - 1 : (int)tt);
      atomicAdd(&P.esc_hist[t.sp * kGrid + b], 1ull);
    }
    const int delta = (keep ? 1 : 0) + o.nsec - 1;
    if (delta != 0) {
      const int old = atomicAdd(&P.alive[e], delta);
      if (old + delta == 0) {
        const uint32_t k = atomicAdd(&P.counters[1], 1u);
        if (k < P.max_events) P.done[k] = e;
      }
    }
  }
  if (rec && i < n_step) {
    ems_step_record r;
    r.dep = o.dep;
    r.esc = o.esc;
    r.killed = o.killed;
    r.step_len = o.step_len;
    r.limiter = o.limiter;
    r.process = o.process;
    r.n_pair = o.n_pair;
    r.n_annih = o.n_annih;
    r.n_out = (keep ? 1 : 0) + o.nsec;
    r.escaped = o.escaped;
    rec[i] = r;
  }
}

// Admit queued primaries: ring entries [head, head + m) -> pool slots [n0, n0 + m).
__global__ void k_admit(Params P, Queue q, Pool pool, uint32_t head, uint32_t m, uint32_t n0) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const uint32_t r = (head + j) % q.capacity;
  const double x = q.x[r], y = q.y[r], z = q.z[r], u = q.u[r], v = q.v[r], w = q.w[r];
  uint32_t a, b, c, d;
  philox10(q.event_id[r], q.index[r], 0u, 0u, P.seed, 0x243F6A88u, a, b, c, d);
  const int vol = locate(P, x, y, z, u, v, w);
  const uint32_t k = n0 + j;
  write_track(pool, k, q.species[r], 0, x, y, z, u, v, w, q.T[r], -1.0, a, b, c, q.slot[r], 0u);
  pool.meta[k] = (uint32_t)q.species[r] | ((vol < 0 ? kVolOut : (uint32_t)vol) << 2);
}

// Copy a batch's primaries into the ring at tail; row r belongs to the event e with
// off[e] <= r < off[e+1] (binary search over the staged offsets).
__global__ void k_enqueue(Queue q, uint32_t tail, const int64_t* off, const uint32_t* slots,
                          const uint32_t* ids, uint32_t n_events, const int32_t* sp,
                          const double* T, const double* pos, const double* dir, uint32_t n) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
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

// Initialise the event slots of a batch: one block per event.  E_in = sum of its
// primaries' kinetic energies; fixed-point scale 2^(61 - ceil(log2 E_in)) keeps the
// sum of its deposits below 2^61 quanta; tallies and ledger zeroed.
__global__ void k_event_init(Params P, const int64_t* off, const uint32_t* slots,
                             const double* T, double* e_in, double* scale) {
  const uint32_t e = blockIdx.x;
  const int64_t a = off[e], b = off[e + 1];
  __shared__ double part[kBlock];
  double s = 0.0;
  for (int64_t r = a + threadIdx.x; r < b; r += blockDim.x) s += T[r];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  const uint32_t slot = slots[e];
  for (int j = threadIdx.x; j < P.nbins; j += blockDim.x) P.tally[(size_t)slot * P.nbins + j] = 0ull;
  if (threadIdx.x < kLedger) P.ledger[(size_t)slot * kLedger + threadIdx.x] = 0ull;
  if (threadIdx.x == 0) {
    const double E = part[0];
    int ex = 0;
    if (E > 0.0) {
      frexp(E, &ex);  // E < 2^ex
    }
    e_in[slot] = E;
    scale[slot] = ldexp(1.0, 61 - ex);
    P.alive[slot] = (int)(b - a);
  }
}

// Diagnostics: event slots that never finish (alive count far from zero) with a fixed
// 2^40 fixed-point scale and zeroed tallies.
__global__ void k_slots_reset(Params P) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P.max_events) return;
  P.alive[e] = 1 << 30;
  const_cast<double*>(P.scale)[e] = 0x1p40;
  for (int b = 0; b < P.nbins; ++b) P.tally[(size_t)e * P.nbins + b] = 0ull;
  for (int b = 0; b < kLedger; ++b) P.ledger[(size_t)e * kLedger + b] = 0ull;
}

__global__ void k_zero_u32(uint32_t* p, uint32_t n) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) p[j] = 0u;
}

__global__ void k_zero_u64(unsigned long long* p, uint32_t n) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) p[j] = 0ull;
}

// Diagnostics: external SoA <-> pool layout.
__global__ void k_pool_load(Pool p, ems_track_soa s, uint32_t n) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  write_track(p, j, s.species[j], s.vol[j], s.x[j], s.y[j], s.z[j], s.u[j], s.v[j], s.w[j],
              s.T[j], s.nlam[j], s.k0[j], s.k1[j], s.k2[j], s.event[j], s.nstep[j]);
}

__global__ void k_pool_dump(Pool p, ems_track_soa s, uint32_t n) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  s.x[j] = p.x[j];
  s.y[j] = p.y[j];
  s.z[j] = p.z[j];
  s.u[j] = p.u[j];
  s.v[j] = p.v[j];
  s.w[j] = p.w[j];
  s.T[j] = p.T[j];
  s.nlam[j] = p.nlam[j];
  s.k0[j] = p.k0[j];
  s.k1[j] = p.k1[j];
  s.k2[j] = p.k2[j];
  s.event[j] = p.evt[j];
  s.nstep[j] = p.nstep[j];
  s.species[j] = (int32_t)(p.meta[j] & 3u);
  s.vol[j] = (int32_t)(p.meta[j] >> 2);
}

}  // namespace ems

// ------------------------------------------------------------------ launchers (internal)

namespace ems {

static inline uint32_t blocks_for(uint64_t n, uint32_t b) { return (uint32_t)((n + b - 1) / b); }

hipError_t launch_step(const Params& P, const Pool& in, const Pool& out, uint32_t n_in,
                       uint32_t n_step, bool mixed, ems_step_record* rec, hipStream_t s) {
  if (n_in == 0) return hipSuccess;
  const dim3 g(blocks_for(n_in, kBlock)), b(kBlock);
  if (mixed) hipLaunchKernelGGL(k_step<float>, g, b, 0, s, P, in, out, n_in, n_step, rec);
  else hipLaunchKernelGGL(k_step<double>, g, b, 0, s, P, in, out, n_in, n_step, rec);
  return hipGetLastError();
}

hipError_t launch_admit(const Params& P, const Queue& q, const Pool& pool, uint32_t head,
                        uint32_t m, uint32_t n0, hipStream_t s) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_admit, dim3(blocks_for(m, 256)), dim3(256), 0, s, P, q, pool, head, m, n0);
  return hipGetLastError();
}

hipError_t launch_enqueue(const Queue& q, uint32_t tail, const int64_t* off, const uint32_t* slots,
                          const uint32_t* ids, uint32_t n_events, const int32_t* sp,
                          const double* T, const double* pos, const double* dir, uint32_t n,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_enqueue, dim3(blocks_for(n, 256)), dim3(256), 0, s, q, tail, off, slots, ids,
                     n_events, sp, T, pos, dir, n);
  return hipGetLastError();
}

hipError_t launch_event_init(const Params& P, const int64_t* off, const uint32_t* slots,
                             const double* T, uint32_t n_events, double* e_in, double* scale,
                             hipStream_t s) {
  if (n_events == 0) return hipSuccess;
  hipLaunchKernelGGL(k_event_init, dim3(n_events), dim3(kBlock), 0, s, P, off, slots, T, e_in,
                     scale);
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

hipError_t launch_pool_load(const Pool& p, const ems_track_soa& src, uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pool_load, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, src, n);
  return hipGetLastError();
}

hipError_t launch_pool_dump(const Pool& p, const ems_track_soa& dst, uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pool_dump, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, dst, n);
  return hipGetLastError();
}

}  // namespace ems

namespace ems {

// Gather the tallies of n event slots into rows of (nbins + 5) doubles: deposits per
// bin, then primary energy, escaped, killed, pair conversions, annihilations.
__global__ void k_gather_tallies(Params P, const uint32_t* slots, uint32_t n, const double* e_in,
                                 double* out) {
  const uint32_t row = blockIdx.x;
  if (row >= n) return;
  const uint32_t s = slots[row];
  const double inv = 1.0 / P.scale[s];
  const uint32_t w = (uint32_t)P.nbins + 5u;
  for (int b = threadIdx.x; b < P.nbins; b += blockDim.x)
    out[(size_t)row * w + b] = (double)(long long)P.tally[(size_t)s * P.nbins + b] * inv;
  if (threadIdx.x == 0) {
    double* L = out + (size_t)row * w + P.nbins;
    L[0] = e_in[s];
    L[1] = (double)(long long)P.ledger[(size_t)s * kLedger + 0] * inv;
    L[2] = (double)(long long)P.ledger[(size_t)s * kLedger + 1] * inv;
    L[3] = (double)P.ledger[(size_t)s * kLedger + 2];
    L[4] = (double)P.ledger[(size_t)s * kLedger + 3];
  }
}

hipError_t launch_gather_tallies(const Params& P, const uint32_t* slots, uint32_t n,
                                 const double* e_in, double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_tallies, dim3(n), dim3(128), 0, s, P, slots, n, e_in, out);
  return hipGetLastError();
}

}  // namespace ems
