// ecpic_push.hip -- implicit mid-point particle push split at cell-face
// crossings (Eq. (4) of Sec. 2.1 with mid-point centring), the
// charge-conserving current deposit (Eq. (3) with spline order 1,
// orbit-averaged per sub-step), wall absorption, and the null-collision
// Monte Carlo step (Sec. 2.1), for gfx950.
//
// One thread per particle.  Particles are kept sorted by cell, so the four
// field values a thread gathers are shared by its neighbours (L1/L2 hits) and
// the four face currents of a sub-step are mostly the same faces for a whole
// wavefront: the first sub-step's currents are combined by a segmented
// wavefront reduction keyed by cell before one lane per run issues the
// global FP64 atomics; later sub-steps (cell crossers) use direct atomics.
//
// The same template serves the FP64 path (T = double, positions stored as
// global xi, eta) and the mixed path (T = float, positions stored as int32
// cell + FP32 offsets); current increments are always formed and
// accumulated in FP64.
#include <climits>

#include "ecpic_internal.h"

namespace ecpic {

namespace {

constexpr double kQE = 1.602176634e-19;  // elementary charge [C]

template <typename T>
struct Tol;
template <>
struct Tol<double> {
  static __device__ __forceinline__ double v() { return 1e-14; }
};
template <>
struct Tol<float> {
  static __device__ __forceinline__ float v() { return 4e-7f; }
};

// particle state relative to its cell: offsets a = xi - i, b = eta - j in [0,1]
template <typename T>
struct PState {
  int i, j;
  T a, b, vr, vt, vz;
};

template <typename T>
struct Mid {
  T a, b, vr, vt, vz;  // mid-point offsets (cell-local) and mid velocities
  T kr, kz;            // solve_fast only: vr - v_r, vz - v_z (the kicks)
};

// 1/x from the hardware reciprocal estimate refined by Newton steps
// (y <- y + y (1 - x y)): two in FP64, one in FP32, which leaves the result
// within an ulp or two of the rounded quotient for the finite, normal,
// non-zero x the sub-step solves pass (a fraction of the cost of an IEEE
// division); 0 gives NaN, which the callers' admissibility checks reject or
// never select.
__device__ __forceinline__ double rcp_refined(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}
__device__ __forceinline__ float rcp_refined(float x) {
  const float y = __builtin_amdgcn_rcpf(x);
  return fmaf(y, fmaf(-x, y, 1.0f), y);
}

// sqrt(x) from the hardware reciprocal-square-root estimate: two Newton
// steps on 1/sqrt(x), then one on the root, which leaves it within an ulp or
// two of the rounded root for the positive, normal x the sub-step solves
// pass (0 gives 0, a negative x NaN); a fraction of the cost of the
// correctly rounded sequence.
__device__ __forceinline__ double sqrt_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  double r = x * y;
  r = fma(0.5 * y, fma(-r, r, x), r);
  return x > 0.0 ? r : (x == 0.0 ? 0.0 : __builtin_nan(""));
}
__device__ __forceinline__ float sqrt_refined(float x) { return sqrtf(x); }

// Element access by a 32-bit byte offset from a uniform base, which the
// loads and stores take as a scalar base plus one vector offset (no 64-bit
// address arithmetic per array); species capacities keep every offset
// below 4 GiB.
template <typename V>
__device__ __forceinline__ V& at32(V* base, uint32_t byte_off) {
  return *reinterpret_cast<V*>(reinterpret_cast<char*>(base) + byte_off);
}
template <typename V>
__device__ __forceinline__ const V& at32(const V* base, uint32_t byte_off) {
  return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + byte_off);
}

template <typename T>
__device__ __forceinline__ T clamp01(T x) {
  return x < T(0) ? T(0) : (x > T(1) ? T(1) : x);
}

// r and 1/J_r at cell-local offset a of radial cell i.
template <typename T>
__device__ __forceinline__ void map_r(const MapP& m, int i, T a, T& r, T& ijr) {
  if (double(i) + double(a) < m.xi_a) {
    const T xi = T(i) + a;
    const T sx = sqrt_refined(xi);
    r = T(2.0 * m.s * sqrt(m.xi_a)) * sx;
    ijr = sx * T(m.rsqrt_xa * m.inv_s);
  } else {
    r = T(m.s * (double(i) + m.xi_a)) + T(m.s) * a;
    ijr = T(m.inv_s);
  }
}

// Position equation of the mid-point rule in xi, solved exactly for the
// mid offset: linear part of the map, or the square-root part as a quadratic
// in sqrt(xi_bar) (positive root), whichever is consistent.
//
// Written as a value-returning function with one exit: an earlier form that
// wrote the result through a reference from several early-return branches was
// compiled (hipcc, gfx950) so that, in wavefronts where some lanes took the
// linear branch and others the square-root branch, square-root lanes received
// the linear value.  The single-exit form is exact in that situation.
template <typename T>
__device__ __forceinline__ T mid_a_val(const MapP& m, int i, T a, T vbr, T dtau) {
  const T al = a + T(0.5) * dtau * vbr * T(m.inv_s);
  if (m.xi_a > 0.0 && T(i) + al < T(m.xi_a)) {
    const T xi = T(i) + a;
    const T beta = T(0.5) * dtau * vbr * T(m.inv_s * m.rsqrt_xa);
    const T y = T(0.5) * (beta + sqrt_refined(beta * beta + T(4) * xi));
    return y * y - T(i);
  }
  return al;
}

// the mid position is admissible unless the uniform map (xi_a = 0) puts it
// behind the axis
template <typename T>
__device__ __forceinline__ bool mid_a(const MapP& m, int i, T a, T vbr, T dtau, T& abar) {
  abar = mid_a_val(m, i, a, vbr, dtau);
  return m.xi_a > 0.0 || T(i) + abar >= T(0);
}

// Mid-point acceleration with the theta mid velocity from the angular
// equation vb_t (1 + dtau vb_r / (2 rb)) = v_t.  F = {ur[i][j], ur[i][j+1],
// uz[i][j], uz[i+1][j]} of the half-step field.
template <typename T>
__device__ __forceinline__ bool accel(const MapP& m, const T F[4], int i, T abar, T bbar, T vbr,
                                      T vt0, T dtau, T qm, T& ar, T& az, T& vtb) {
  T rb, ijr;
  map_r(m, i, abar, rb, ijr);
  const T ac = clamp01(abar), bc = clamp01(bbar);
  const T er = ((T(1) - bc) * F[0] + bc * F[1]) * ijr;
  const T ez = ((T(1) - ac) * F[2] + ac * F[3]) * T(m.inv_dz);
  // vtb = vt0 / (1 + dtau vbr / (2 rb)) = vt0 rb q and vtb^2 / rb = vt0^2 rb q^2
  // with q = 1 / (rb + dtau vbr / 2): one division; on the axis (rb = 0)
  // only a particle without v_theta is admissible.  Selects, no branches.
  const bool off_axis = rb > T(0);
  const T den = rb + T(0.5) * dtau * vbr;
  const T q = rcp_refined(den);
  vtb = off_axis ? vt0 * rb * q : T(0);
  ar = qm * er + (off_axis ? vtb * vt0 * q : T(0));
  az = qm * ez;
  const bool adm = off_axis ? (den > T(0)) : (vt0 == T(0));
  return adm & isfinite(ar) & isfinite(az) & isfinite(vtb);
}

// Unconstrained sub-step of length dtau in the particle's cell: fixed point
// on the mid velocities, mid positions solved exactly from them.
template <typename T>
__device__ bool solve_free(const MapP& m, const T F[4], const PState<T>& p, T dtau, T qm,
                           Mid<T>& M) {
  T vr = p.vr, vt = p.vt, vz = p.vz;
  const T hd = T(0.5) * dtau;
  const T idz = T(m.inv_dz);
  for (int it = 0; it < kMaxFixed; ++it) {
    T abar;
    const bool oka = mid_a(m, p.i, p.a, vr, dtau, abar);
    const T bbar = p.b + hd * vz * idz;
    T ar, az, vtb;
    // admissibility as flags, one exit per iteration
    if (!(oka & isfinite(bbar) & accel(m, F, p.i, abar, bbar, vr, p.vt, dtau, qm, ar, az, vtb)))
      return false;
    const T nvr = p.vr + hd * ar, nvz = p.vz + hd * az, nvt = vtb;
    const T scale = fabs(nvr) + fabs(nvt) + fabs(nvz);
    const T d = fmax(fabs(nvr - vr), fmax(fabs(nvt - vt), fabs(nvz - vz)));
    vr = nvr;
    vt = nvt;
    vz = nvz;
    if (d <= Tol<T>::v() * scale) {
      if (!mid_a(m, p.i, p.a, vr, dtau, M.a)) return false;
      M.b = p.b + hd * vz * idz;
      M.vr = vr;
      M.vt = vt;
      M.vz = vz;
      return true;
    }
  }
  return false;
}

// The same mid-point system for a particle of a linear-map cell (i >= i_lin)
// whose sub-step stays in its cell, solved without the general fixed point.
// There E_r = ((1-b)F0 + b F1)/s depends on the mid offset b only, E_z on
// the mid offset a only, and a = a0 + (dt/2s) vb_r, b = b0 + (dt/2dz) vb_z,
// so (vb_r, vb_z) obey a 2x2 linear system:
//   vb_z = Cz + Kz vb_r,   vb_r (1 - Kr Kz) = Cr + Kr Cz + (dt/2) cf,
// with the centrifugal term cf = vb_t^2 / r_bar = v_t^2 r_bar / r_end^2
// (vb_t = v_t r_bar / r_end from the angular equation, r_bar = r0 + dt vb_r / 2,
// r_end = r0 + dt vb_r): a scalar fixed point in vb_r that converges in a few
// steps.  Returns false when the case does not apply (the caller then runs
// the general solve).
template <typename T>
__device__ __forceinline__ bool solve_fast(const MapP& m, const T F[4], const PState<T>& p, T dtau,
                                           T qm, Mid<T>& M) {
  // Written for the kicks kr = vb_r - v_r, kz = vb_z - v_z, so that in FP32
  // the rounding acts on the small field-driven part only:
  //   kz = beta Ez + Kz (v_r + kr),
  //   kr (1 - Kr Kz) = alpha Er + Kr (v_z + beta Ez + Kz v_r) + (dt/2) cf,
  // with Er, Ez the weighted fields at the start offsets.
  const T hd = T(0.5) * dtau;
  const T delta = hd * T(m.inv_s);  // d a_bar / d vb_r
  const T gamma = hd * T(m.inv_dz); // d b_bar / d vb_z
  const T alpha = qm * delta;       // d vb_r / d (weighted ur)
  const T beta = qm * gamma;        // d vb_z / d (weighted uz)
  const T dFr = F[1] - F[0], dFz = F[3] - F[2];
  const T Ez = F[2] + p.a * dFz;
  const T Er = F[0] + p.b * dFr;
  const T Kz = beta * delta * dFz;
  const T Kr = alpha * gamma * dFr;
  const T den = T(1) - Kr * Kz;
  const T r0 = T(m.s * (double(p.i) + m.xi_a)) + T(m.s) * p.a;
  // admissibility as flags (no early exits): a failed lane computes on and
  // is rejected at the end
  bool ok = (den > T(0)) & (r0 > T(0));
  const T inv_den = rcp_refined(den);
  const T bz = beta * Ez;
  const T k0 = (alpha * Er + Kr * (p.vz + bz + Kz * p.vr)) * inv_den;
  const T cc = hd * inv_den;
  const T vt2 = p.vt * p.vt;
  const T c2 = cc * vt2;
  T kr = k0 + c2 * rcp_refined(r0);  // centrifugal term at the start position
  // g(kr) = k0 + c2 rb / re^2 is a contraction (slope about (dt v_t / r)^2,
  // tiny in a linear cell): iterate until the step |g(kr) - kr| is below the
  // tolerance of the velocity scale, which bounds the distance to the fixed
  // point by the step itself.  The scale is taken once, from the first
  // estimate of the mid velocity (a fixed threshold keeps the loop to the
  // update and one compare); admissibility is checked once, on the result.
  const T thr = Tol<T>::v() * (fabs(p.vr + kr) + fabs(p.vt) + fabs(p.vz + bz + Kz * (p.vr + kr)));
  bool conv = false;
  for (int it = 0; it < 12; ++it) {
    const T vr = p.vr + kr;
    const T rb = r0 + hd * vr;
    const T ire = rcp_refined(r0 + dtau * vr);
    const T nkr = k0 + c2 * ire * ire * rb;
    const T d = fabs(nkr - kr);
    kr = nkr;
    if (d <= thr) {
      conv = true;
      break;
    }
  }
  const T vrb = p.vr + kr;
  const T rb1 = r0 + hd * vrb;
  const T re1 = r0 + dtau * vrb;
  ok = ok & (rb1 > T(0)) & (re1 > T(0));
  conv = conv & ok;
  const T kz = bz + Kz * vrb;
  M.kr = kr;
  M.kz = kz;
  M.vr = vrb;
  M.vz = p.vz + kz;
  M.vt = p.vt * rb1 * rcp_refined(re1);
  M.a = p.a + delta * vrb;
  M.b = p.b + gamma * M.vz;
  return conv & (re1 > T(0));
}

// Smallest positive root of (a/2) t^2 + v t - D = 0 in cancellation-free
// form, or +inf.
template <typename T>
__device__ __forceinline__ T smallest_pos_root(T a, T v, T D) {
  const T A = T(0.5) * a, B = v, C = -D;
  T best = T(INFINITY);
  if (A == T(0)) {
    if (B != T(0)) {
      const T t = -C * rcp_refined(B);
      if (t > T(0)) best = t;
    }
    return best;
  }
  const T disc = B * B - T(4) * A * C;
  if (disc < T(0)) return best;
  const T sq = sqrt_refined(disc);
  const T q = T(-0.5) * (B + (B >= T(0) ? sq : -sq));
  if (q != T(0)) {
    const T t1 = q * rcp_refined(A), t2 = C * rcp_refined(q);
    if (t1 > T(0) && t1 < best) best = t1;
    if (t2 > T(0) && t2 < best) best = t2;
  }
  return best;
}

// Sub-step that ends exactly on the local face f (0 or 1) of axis d (0: xi,
// 1: eta): the crossed coordinate's mid value is (x + f)/2 and the length
// solves the position equation as a quadratic given the mid acceleration.
template <typename T>
__device__ bool solve_cross(const MapP& m, const T F[4], const PState<T>& p, int d, T f, T dmax,
                            T dt0, const Mid<T>& M0, T qm, T& dtau_out, Mid<T>& M, bool& capped) {
  const T xd = d == 0 ? p.a : p.b;
  const T xbar = T(0.5) * (xd + f);
  T Jd;
  if (d == 0) {
    T rb, ijr;
    map_r(m, p.i, xbar, rb, ijr);
    Jd = rcp_refined(ijr);
  } else {
    Jd = T(m.dz);
  }
  const T D = (f == xd) ? T(0) : (f - xd) * Jd;
  const T v0d = d == 0 ? p.vr : p.vz;
  capped = false;
  if (D == T(0)) {
    if (f == T(0) ? (v0d < T(0)) : (v0d > T(0))) {
      dtau_out = T(0);
      M.a = p.a;
      M.b = p.b;
      M.vr = p.vr;
      M.vt = p.vt;
      M.vz = p.vz;
      return true;
    }
  }
  T vr = M0.vr, vt = M0.vt, vz = M0.vz;
  T dtau = dt0;
  const T idz = T(m.inv_dz);
  for (int it = 0; it < kMaxFixed; ++it) {
    // admissibility as flags, one exit per iteration
    T abar, bbar;
    bool ok = true;
    if (d == 0) {
      abar = xbar;
      bbar = p.b + T(0.5) * dtau * vz * idz;
    } else {
      bbar = xbar;
      ok = mid_a(m, p.i, p.a, vr, dtau, abar);
    }
    T ar, az, vtb;
    ok = ok & isfinite(bbar) & accel(m, F, p.i, abar, bbar, vr, p.vt, dtau, qm, ar, az, vtb);
    if (!ok) return false;
    T nd = smallest_pos_root(d == 0 ? ar : az, v0d, D);
    bool cap = false;
    if (!(nd <= dmax)) {
      nd = dmax;
      cap = true;
    }
    const T nvr = p.vr + T(0.5) * nd * ar, nvz = p.vz + T(0.5) * nd * az, nvt = vtb;
    const T scale = fabs(nvr) + fabs(nvt) + fabs(nvz);
    const T dv = fmax(fabs(nvr - vr), fmax(fabs(nvt - vt), fabs(nvz - vz)));
    const T ddt = fabs(nd - dtau);
    vr = nvr;
    vt = nvt;
    vz = nvz;
    dtau = nd;
    if (dv <= Tol<T>::v() * scale && ddt <= Tol<T>::v() * dmax) {
      capped = cap;
      dtau_out = dtau;
      if (d == 0) {
        M.a = xbar;
        M.b = p.b + T(0.5) * dtau * vz * idz;
      } else {
        M.b = xbar;
        if (!mid_a(m, p.i, p.a, vr, dtau, M.a)) return false;
      }
      M.vr = vr;
      M.vt = vt;
      M.vz = vz;
      return true;
    }
  }
  return false;
}

// Face currents of one straight logical sub-step inside cell (i, j):
// Eq. (3) with m = 1 integrated along the sub-step.
struct Dep {
  double r0, r1, z0, z1;  // ur[i][j], ur[i][j+1], uz[i][j], uz[i+1][j] increments
};

__device__ __forceinline__ Dep make_dep(double a0, double b0, double a1, double b1, double c) {
  const double dx = a1 - a0, de = b1 - b0;
  const double xm = 0.5 * (a0 + a1), em = 0.5 * (b0 + b1);
  Dep d;
  d.r0 = c * dx * (1.0 - em);
  d.r1 = c * dx * em;
  d.z0 = c * de * (1.0 - xm);
  d.z1 = c * de * xm;
  return d;
}

__device__ __forceinline__ void atomic_dep(double* Ir, double* Iz, int nz, int i, int j,
                                           const Dep& d) {
  if (!Ir) return;  // a pass that deposits nothing
  double* pr = Ir + (size_t)i * (nz + 1) + j;
  unsafeAtomicAdd(pr, d.r0);
  unsafeAtomicAdd(pr + 1, d.r1);
  unsafeAtomicAdd(Iz + (size_t)i * nz + j, d.z0);
  unsafeAtomicAdd(Iz + (size_t)(i + 1) * nz + j, d.z1);
}

// A block's currents are gathered in LDS over the cells [c_lo, c_lo + W):
// r-edges i*(nz+1)+j of those cells and their j+1 neighbours at TR[e - er0]
// (er0 = c_lo + c_lo / nz), z-edges i*nz+j and the (i+1) neighbours at
// TZ[e - c_lo].  Deposits of cells outside the window go to global atomics.
struct Tile {
  double* TR;
  double* TZ;
  int c_lo, W, er0;
};

// the window: one radial row below the block's first cell and one above its
// last (a block's 1024 particles span a few dozen cells at most in sorted
// order), cells that particles drift to between sorts
__host__ __device__ inline int tile_cells(int nz) { return 2 * nz + 64; }
__host__ __device__ inline int tile_r_len(int nz) {
  const int W = tile_cells(nz);
  return W + W / nz + 2;
}
__host__ __device__ inline int tile_z_len(int nz) { return tile_cells(nz) + nz; }

// The slow pass's window (per wavefront): the fast pass's where that is at
// most kSlowW cells (one radial row either side of the unit's lowest cell);
// for longer rows kSlowW cells from 32 below that cell, so that crossings of
// z-faces stay in it and those of r-faces (to cells nz away) go to global
// atomics, and the tile does not limit how many wavefronts a CU holds.
constexpr int kSlowW = 576;
__host__ __device__ inline int slow_cells(int nz) {
  return tile_cells(nz) < kSlowW ? tile_cells(nz) : kSlowW;
}
__host__ __device__ inline int slow_r_len(int nz) {
  const int W = slow_cells(nz);
  return W + W / nz + 2;
}
__host__ __device__ inline int slow_z_len(int nz) { return slow_cells(nz) + nz; }
__host__ __device__ inline int slow_below(int nz) {
  return tile_cells(nz) <= kSlowW ? nz + 2 : 32;
}


// Deposit of one sub-step: into the tile when its cell is in the window (LDS
// atomics), else by global atomics.
__device__ __forceinline__ void tile_or_global(const Tile& t, double* Ir, double* Iz, int nz,
                                               int i, int j, const Dep& d) {
  if (!Ir) return;  // a pass that deposits nothing
  const int key = i * nz + j;
  if (key >= t.c_lo && key < t.c_lo + t.W) {
    const int er = key + i - t.er0, ez = key - t.c_lo;
    atomicAdd(&t.TR[er], d.r0);
    atomicAdd(&t.TR[er + 1], d.r1);
    atomicAdd(&t.TZ[ez], d.z0);
    atomicAdd(&t.TZ[ez + nz], d.z1);
  } else {
    atomic_dep(Ir, Iz, nz, i, j, d);
  }
}

enum { kAlive = 0, kAbsorbed = 1, kError = 2 };

struct PushOut {
  int status;
  int wall;           // 1 bottom, 2 top, 3 side
  int nsub, ncross;
  double work;        // sum of q w E.dx over sub-steps (in units of J)
};

template <typename T>
__device__ __forceinline__ void load_field(const MapP& m, const T* __restrict__ ur,
                                           const T* __restrict__ uz, int i, int j, T F[4]) {
  const uint32_t orr = (uint32_t)(i * (m.nz + 1) + j) * (uint32_t)sizeof(T);
  const uint32_t oz = (uint32_t)(i * m.nz + j) * (uint32_t)sizeof(T);
  F[0] = at32(ur, orr);
  F[1] = at32(ur, orr + (uint32_t)sizeof(T));
  F[2] = at32(uz, oz);
  F[3] = at32(uz, oz + (uint32_t)(m.nz * (int)sizeof(T)));
}

// Push one particle over dt, depositing each sub-step into the caller's
// tile (cells outside its window by global atomics).  LDS atomics keep the
// sub-step loop free of global ones: vector loads and stores (atomics
// included) retire in issue order on one counter, so a field load issued
// after a global atomic still in flight waits for it (microseconds for
// device-wide FP64 atomics).
template <typename T>
__device__ void push_particle(const MapP& m, const T* __restrict__ ur, const T* __restrict__ uz,
                              double* Ir, double* Iz, const Tile& tl, PState<T>& p, T qm,
                              double qw_dt, bool want_work, PushOut& out) {
  out.status = kAlive;
  out.wall = 0;
  out.nsub = 0;
  out.ncross = 0;
  out.work = 0.0;
  const int nr = m.nr, nz = m.nz;
  T tau = T(m.dt);
  // the field of the cell the particle is expected to enter, loaded while
  // the crossing is solved (pf_i < 0: none)
  T Fn[4];
  int pf_i = -1, pf_j = -1;
  // halvings of the sub-step after crossing solves that found no face
  int cut = 0;
  while (tau > T(0)) {
    if (out.nsub >= kMaxSub) {
      out.status = kError;
      return;
    }
    out.nsub++;
    // on a face, the cell the motion goes to
    if (p.a == T(1) && p.vr >= T(0) && p.i < nr - 1) {
      p.i += 1;
      p.a = T(0);
    } else if (p.a == T(0) && p.vr < T(0) && p.i > 0) {
      p.i -= 1;
      p.a = T(1);
    }
    if (p.b == T(1) && p.vz >= T(0) && p.j < nz - 1) {
      p.j += 1;
      p.b = T(0);
    } else if (p.b == T(0) && p.vz < T(0) && p.j > 0) {
      p.j -= 1;
      p.b = T(1);
    }
    T F[4];
    if (p.i == pf_i && p.j == pf_j) {
      F[0] = Fn[0];
      F[1] = Fn[1];
      F[2] = Fn[2];
      F[3] = Fn[3];
    } else {
      load_field(m, ur, uz, p.i, p.j, F);
    }
    // the field of the neighbour the particle is expected to enter next,
    // guessed from free flight over the rest of the step (the linear-map
    // scale in xi; the xi face first when both are left) and loaded now, so
    // that the load overlaps this sub-step's solves
    {
      const T ea0 = p.a + tau * p.vr * T(m.inv_s), eb0 = p.b + tau * p.vz * T(m.inv_dz);
      const bool ix0 = ea0 >= T(0) && ea0 <= T(1), ie0 = eb0 >= T(0) && eb0 <= T(1);
      pf_i = -1;
      if (!(ix0 && ie0)) {
        int ni = p.i, nj = p.j;
        if (!ix0)
          ni += ea0 < T(0) ? -1 : 1;
        else
          nj += eb0 < T(0) ? -1 : 1;
        if (ni >= 0 && ni < nr && nj >= 0 && nj < nz) {
          load_field(m, ur, uz, ni, nj, Fn);
          pf_i = ni;
          pf_j = nj;
        }
      }
    }
    T dtry = tau;
    for (int k = 0; k < cut; ++k) dtry *= T(0.5);
    Mid<T> M;
    // linear-map cells: the closed-form solve (the same mid point as the
    // fixed point, to its tolerance); otherwise the fixed point, halving
    // the sub-step while it fails
    bool ok = p.i >= m.i_lin && solve_fast(m, F, p, dtry, qm, M);
    for (int h = 0; !ok && h <= kMaxHalve; ++h) {
      ok = solve_free(m, F, p, dtry, qm, M);
      if (!ok) dtry *= T(0.5);
    }
    if (!ok) {
      out.status = kError;
      return;
    }
    const T ea = T(2) * M.a - p.a, eb = T(2) * M.b - p.b;
    const bool in_x = ea >= T(0) && ea <= T(1);
    const bool in_e = eb >= T(0) && eb <= T(1);
    // the neighbour across the face the solved free orbit leaves by (the xi
    // face when both are left): loaded here unless the guess above was it;
    // used only if the particle is in that cell at the next sub-step
    if (!(in_x && in_e)) {
      int ni = p.i, nj = p.j;
      if (!in_x)
        ni += ea < T(0) ? -1 : 1;
      else
        nj += eb < T(0) ? -1 : 1;
      if (ni >= 0 && ni < nr && nj >= 0 && nj < nz && !(ni == pf_i && nj == pf_j)) {
        load_field(m, ur, uz, ni, nj, Fn);
        pf_i = ni;
        pf_j = nj;
      }
    }
    PState<T> q;
    q.i = p.i;
    q.j = p.j;
    T used;
    int cd = -1;
    T cf = T(0);
    if (in_x && in_e) {
      q.a = ea;
      q.b = eb;
      q.vr = T(2) * M.vr - p.vr;
      q.vt = T(2) * M.vt - p.vt;
      q.vz = T(2) * M.vz - p.vz;
      used = dtry;
    } else {
      // one crossing solve per lane on its own axis (the xi face first when
      // both are left), so that lanes leaving by different axes share one
      // pass of the solve; lanes that leave by both solve the eta face in a
      // second pass and keep the earlier crossing (xi on a tie)
      T best_t = T(0);
      Mid<T> BM;
      const bool both = !in_x && !in_e;
      for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1 && !both) break;
        const int d = (pass == 0 && !in_x) ? 0 : 1;
        const T e_end = d == 0 ? ea : eb;
        const T f = e_end < T(0) ? T(0) : T(1);
        const T xd = d == 0 ? p.a : p.b;
        const T t0 = dtry * (f - xd) * rcp_refined(e_end - xd);
        T tt;
        Mid<T> CM;
        bool cap;
        if (!solve_cross(m, F, p, d, f, dtry, t0, M, qm, tt, CM, cap)) continue;
        if (cd < 0 || tt < best_t - T(1e-15 * m.dt)) {
          best_t = tt;
          cd = d;
          cf = f;
          BM = CM;
        }
      }
      if (cd < 0) {
        // the free orbit leaves the cell but no face can be reached
        // consistently (it turns at the face: the crossing solve jumps
        // between a root and none): the sub-step is taken again at half
        // the length
        if (cut >= kMaxHalve) {
          out.status = kError;
          return;
        }
        ++cut;
        continue;
      }
      out.ncross++;
      q.vr = T(2) * BM.vr - p.vr;
      q.vt = T(2) * BM.vt - p.vt;
      q.vz = T(2) * BM.vz - p.vz;
      if (cd == 0) {
        q.a = cf;
        q.b = clamp01(T(2) * BM.b - p.b);
      } else {
        q.b = cf;
        q.a = clamp01(T(2) * BM.a - p.a);
      }
      used = best_t;
    }
    const Dep dp = make_dep(double(p.a), double(p.b), double(q.a), double(q.b), qw_dt);
    if (want_work) {
      out.work += m.dt * (dp.r0 * double(F[0]) + dp.r1 * double(F[1]) + dp.z0 * double(F[2]) +
                          dp.z1 * double(F[3]));
    }
    tile_or_global(tl, Ir, Iz, nz, p.i, p.j, dp);
    p = q;
    tau -= used;
    cut = 0;
    if (cd == 0 && cf == T(1) && p.i == nr - 1) {
      out.status = kAbsorbed;
      out.wall = 3;
      return;
    }
    if (cd == 1 && cf == T(0) && p.j == 0) {
      out.status = kAbsorbed;
      out.wall = 1;
      return;
    }
    if (cd == 1 && cf == T(1) && p.j == nz - 1) {
      out.status = kAbsorbed;
      out.wall = 2;
      return;
    }
    if (cd == 0 && cf == T(0) && p.i == 0) p.vr = -p.vr;  // axis: mirror
  }
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11) and the null-collision step
// ---------------------------------------------------------------------------
// The full 128-bit product of a and the constant m from four 32 x 32 -> 64
// products, each with a 64-bit addend (one multiply-add instruction each),
// so that the low and high halves share their partial products.
__device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t m, uint64_t& hi, uint64_t& lo) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t m0 = (uint32_t)m, m1 = (uint32_t)(m >> 32);
  const uint64_t t = (uint64_t)a0 * m0;
  const uint64_t u = (uint64_t)a1 * m0 + (t >> 32);
  const uint64_t v = (uint64_t)a0 * m1 + (uint32_t)u;
  hi = (uint64_t)a1 * m1 + ((u >> 32) + (v >> 32));
  lo = (v << 32) | (uint32_t)t;
}

__device__ __forceinline__ void philox(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B97F4A7C15ull;
      k1 += 0xBB67AE8584CAA73Bull;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(c[0], M0, hi0, lo0);
    mulhilo64(c[2], M1, hi1, lo1);
    const uint64_t y0 = hi1 ^ c[1] ^ k0, y2 = hi0 ^ c[3] ^ k1;
    c[0] = y0;
    c[1] = lo1;
    c[2] = y2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ void draws(uint64_t seed, int sid, uint64_t uid, int64_t step, int blk,
                                      double u[4]) {
  uint64_t c[4] = {uid, (uint64_t)step, (uint64_t)blk, 0ull};
  philox(c, seed, (uint64_t)sid);
#pragma unroll
  for (int k = 0; k < 4; ++k) u[k] = double(c[k] >> 11) * 0x1.0p-53;
}

__device__ __forceinline__ uint64_t child_uid(uint64_t parent, int64_t step) {
  // SplitMix64 finaliser of a Weyl-shifted parent id, top bit set
  uint64_t z = parent + 0x9E3779B97F4A7C15ull * (uint64_t)(step + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return (z ^ (z >> 31)) | 0x8000000000000000ull;
}

// synthetic argon cross-sections [m^2]
__host__ __device__ __forceinline__ void xsec(double e, double& el, double& ex, double& iz) {
  el = 1.0e-19;
  ex = (e > 11.5) ? 1.0e-20 * (1.0 - 11.5 / e) : 0.0;
  if (e > 15.76) {
    const double x = e / 15.76;
    iz = 8.0e-20 * log(x) / x;
  } else {
    iz = 0.0;
  }
}

__device__ __forceinline__ void iso(double u1, double u2, double d[3]) {
  const double ct = 1.0 - 2.0 * u1;
  const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
  const double ph = 2.0 * M_PI * u2;
  d[0] = st * cos(ph);
  d[1] = st * sin(ph);
  d[2] = ct;
}

template <typename T>
__device__ __forceinline__ void store_slot(const SpecDev& s, const MapP& m, int64_t k, int i, int j,
                                           T a, T b, double vr, double vt, double vz,
                                           uint64_t uid);

template <>
__device__ __forceinline__ void store_slot<double>(const SpecDev& s, const MapP& m, int64_t k,
                                                   int i, int j, double a, double b, double vr,
                                                   double vt, double vz, uint64_t uid) {
  s.xi[k] = double(i) + a;
  s.eta[k] = double(j) + b;
  s.vr[k] = vr;
  s.vt[k] = vt;
  s.vz[k] = vz;
  s.uid[k] = uid;
}

template <>
__device__ __forceinline__ void store_slot<float>(const SpecDev& s, const MapP& m, int64_t k, int i,
                                                  int j, float a, float b, double vr, double vt,
                                                  double vz, uint64_t uid) {
  s.cell[k] = i * m.nz + j;
  s.fa[k] = a;
  s.fb[k] = b;
  s.fvr[k] = float(vr);
  s.fvt[k] = float(vt);
  s.fvz[k] = float(vz);
  s.uid[k] = uid;
}

template <typename T>
__device__ __forceinline__ void kill_slot(const SpecDev& s, int64_t k);
template <>
__device__ __forceinline__ void kill_slot<double>(const SpecDev& s, int64_t k) {
  s.xi[k] = -1.0;
}
template <>
__device__ __forceinline__ void kill_slot<float>(const SpecDev& s, int64_t k) {
  s.cell[k] = -1;
}

struct CollOut {
  double dke;    // kinetic energy lost (J)
  int coll;      // 1 if a real collision happened
  int ionized;
  int over;
  int overflow;
};

// Null-collision Monte Carlo for one particle with velocity (vr, vt, vz),
// updated in place.  Ionisation appends an electron to the own species and
// an ion to the partner species at the parent's position.
template <typename T>
__device__ CollOut collide_one(const MccDev& c, const SpecDev& s, const MapP& m, int sid,
                               uint64_t uid, int i, int j, T a, T b, double& vr, double& vt,
                               double& vz, Tally* tally) {
  CollOut o = {0.0, 0, 0, 0, 0};
  double u[4];
  draws(c.seed, sid, uid, c.step, 0, u);
  if (!(u[0] < c.pnull)) return o;
  const double v2 = vr * vr + vt * vt + vz * vz;
  const double v = sqrt(v2);
  const double ke0 = 0.5 * s.m * s.w * v2;
  if (c.role == 1) {
    const double e = 0.5 * s.m * v2 / kQE;
    if (e > c.eps_max_ev) o.over = 1;
    double sel, sex, siz;
    xsec(e, sel, sex, siz);
    const double nel = c.n_gas * sel * v, nex = c.n_gas * sex * v, niz = c.n_gas * siz * v;
    const double x = u[1] * c.numax;
    double d[3];
    iso(u[2], u[3], d);
    if (x < nel) {
      const double cosx = (v > 0.0) ? (d[0] * vr + d[1] * vt + d[2] * vz) / v : 1.0;
      const double e1 = e * (1.0 - 2.0 * s.m / c.m_gas * (1.0 - cosx));
      const double v1 = sqrt(2.0 * e1 * kQE / s.m);
      vr = v1 * d[0];
      vt = v1 * d[1];
      vz = v1 * d[2];
      o.dke = ke0 - 0.5 * s.m * s.w * v1 * v1;
      o.coll = 1;
    } else if (x < nel + nex) {
      const double e1 = e - 11.5;
      const double v1 = sqrt(2.0 * e1 * kQE / s.m);
      vr = v1 * d[0];
      vt = v1 * d[1];
      vz = v1 * d[2];
      o.dke = ke0 - 0.5 * s.m * s.w * v1 * v1;
      o.coll = 1;
    } else if (x < nel + nex + niz) {
      double w1[4], w2[4];
      draws(c.seed, sid, uid, c.step, 1, w1);
      draws(c.seed, sid, uid, c.step, 2, w2);
      const double er = e - 15.76;
      const double e1 = w1[0] * er, e2 = er - e1;
      const double v1 = sqrt(2.0 * e1 * kQE / s.m), v2n = sqrt(2.0 * e2 * kQE / s.m);
      double d2[3];
      iso(w1[1], w1[2], d2);
      const double sg = c.sig_ion;
      const double ra = sqrt(-2.0 * log(1.0 - w1[3])), rb = sqrt(-2.0 * log(1.0 - w2[1]));
      const double ivr = sg * ra * cos(2.0 * M_PI * w2[0]);
      const double ivt = sg * ra * sin(2.0 * M_PI * w2[0]);
      const double ivz = sg * rb * cos(2.0 * M_PI * w2[2]);
      const uint64_t nu = child_uid(uid, c.step);
      const unsigned long long ke = atomicAdd(&tally->append[sid], 1ull);
      const unsigned long long ki = atomicAdd(&tally->append[c.partner.sid], 1ull);
      const int64_t se = c.base_self + (int64_t)ke, si = c.base_partner + (int64_t)ki;
      if (se >= s.cap || si >= c.partner.cap) {
        // the pair does not fit: no ionisation at all (the primary keeps
        // its velocity), and a slot reserved within capacity is marked dead
        // so that no unwritten slot becomes a live particle
        o.overflow = 1;
        if (se < s.cap) kill_slot<T>(s, se);
        if (si < c.partner.cap) kill_slot<T>(c.partner, si);
      } else {
        vr = v1 * d[0];
        vt = v1 * d[1];
        vz = v1 * d[2];
        store_slot<T>(s, m, se, i, j, a, b, v2n * d2[0], v2n * d2[1], v2n * d2[2], nu);
        store_slot<T>(c.partner, m, si, i, j, a, b, ivr, ivt, ivz, nu);
        o.ionized = 1;
        o.coll = 1;
        o.dke = ke0 - 0.5 * s.m * s.w * (v1 * v1 + v2n * v2n) -
                0.5 * c.partner.m * c.partner.w * (ivr * ivr + ivt * ivt + ivz * ivz);
      }
    }
  } else if (c.role == 2) {
    double w1[4];
    draws(c.seed, sid, uid, c.step, 1, w1);
    const double sg = c.sig_gas;
    const double ra = sqrt(-2.0 * log(1.0 - u[1])), rb = sqrt(-2.0 * log(1.0 - u[3]));
    const double nvr = sg * ra * cos(2.0 * M_PI * u[2]);
    const double nvt = sg * ra * sin(2.0 * M_PI * u[2]);
    const double nvz = sg * rb * cos(2.0 * M_PI * w1[0]);
    const double gr = vr - nvr, gt = vt - nvt, gz = vz - nvz;
    const double g = sqrt(gr * gr + gt * gt + gz * gz);
    const double nu = c.n_gas * 5.0e-19 * g;
    if (nu > c.numax) o.over = 1;
    if (w1[1] * c.numax < nu) {
      vr = nvr;
      vt = nvt;
      vz = nvz;
      o.dke = ke0 - 0.5 * s.m * s.w * (nvr * nvr + nvt * nvt + nvz * nvz);
      o.coll = 1;
    }
  }
  return o;
}

// block-wide sum of a double into *dst (one atomic per block)
__device__ void block_sum_atomic(double v, double* dst) {
  __shared__ double red[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < kBlock / 64; ++k) s += red[k];
    if (s != 0.0) unsafeAtomicAdd(dst, s);
  }
  __syncthreads();
}

__device__ void block_count_atomic(unsigned v, unsigned long long* dst) {
  __shared__ unsigned redc[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) redc[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int k = 0; k < kBlock / 64; ++k) s += redc[k];
    if (s) atomicAdd(dst, s);
  }
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ bool load_particle(const SpecDev& s, const MapP& m, int64_t k,
                                              PState<T>& p);

template <>
__device__ __forceinline__ bool load_particle<double>(const SpecDev& s, const MapP& m, int64_t k,
                                                      PState<double>& p) {
  const double xi = s.xi[k], eta = s.eta[k];
  p.vr = s.vr[k];
  p.vt = s.vt[k];
  p.vz = s.vz[k];
  if (!(xi >= 0.0)) return false;
  int i = int(floor(xi)), j = int(floor(eta));
  i = i < 0 ? 0 : (i > m.nr - 1 ? m.nr - 1 : i);
  j = j < 0 ? 0 : (j > m.nz - 1 ? m.nz - 1 : j);
  p.i = i;
  p.j = j;
  p.a = xi - double(i);
  p.b = eta - double(j);
  return true;
}

template <>
__device__ __forceinline__ bool load_particle<float>(const SpecDev& s, const MapP& m, int64_t k,
                                                     PState<float>& p) {
  const int c = s.cell[k];
  p.a = s.fa[k];
  p.b = s.fb[k];
  p.vr = s.fvr[k];
  p.vt = s.fvt[k];
  p.vz = s.fvz[k];
  if (c < 0) return false;
  p.i = c / m.nz;
  p.j = c - p.i * m.nz;
  return true;
}

// The stored record of a particle, fetched ahead of its decoding so that a
// loop can have the next particle's loads in flight while it works on the
// current one.
template <typename T>
struct Raw;
template <>
struct Raw<double> {
  double xi, eta, vr, vt, vz;
};
template <>
struct Raw<float> {
  int32_t cell;
  float a, b, vr, vt, vz;
};
__device__ __forceinline__ void fetch_raw(const SpecDev& s, int64_t k, Raw<double>& q) {
  const uint32_t o = (uint32_t)k * 8u;
  q.xi = at32(s.xi, o);
  q.eta = at32(s.eta, o);
  q.vr = at32(s.vr, o);
  q.vt = at32(s.vt, o);
  q.vz = at32(s.vz, o);
}
__device__ __forceinline__ void fetch_raw(const SpecDev& s, int64_t k, Raw<float>& q) {
  const uint32_t o = (uint32_t)k * 4u;
  q.cell = at32(s.cell, o);
  q.a = at32(s.fa, o);
  q.b = at32(s.fb, o);
  q.vr = at32(s.fvr, o);
  q.vt = at32(s.fvt, o);
  q.vz = at32(s.fvz, o);
}
// same decoding as load_particle
__device__ __forceinline__ bool decode_raw(const MapP& m, const Raw<double>& q, PState<double>& p) {
  p.vr = q.vr;
  p.vt = q.vt;
  p.vz = q.vz;
  const bool alive = q.xi >= 0.0;
  int i = int(floor(alive ? q.xi : 0.0)), j = int(floor(alive ? q.eta : 0.0));
  i = i < 0 ? 0 : (i > m.nr - 1 ? m.nr - 1 : i);
  j = j < 0 ? 0 : (j > m.nz - 1 ? m.nz - 1 : j);
  p.i = i;
  p.j = j;
  p.a = q.xi - double(i);
  p.b = q.eta - double(j);
  return alive;
}
__device__ __forceinline__ bool decode_raw(const MapP& m, const Raw<float>& q, PState<float>& p) {
  p.a = q.a;
  p.b = q.b;
  p.vr = q.vr;
  p.vt = q.vt;
  p.vz = q.vz;
  if (q.cell < 0) return false;
  p.i = q.cell / m.nz;
  p.j = q.cell - p.i * m.nz;
  return true;
}

// The stored record of a decoded particle that has not moved: xi = i + a
// exactly (a = xi - i was exact), likewise eta, and the cell key.  The face
// step of a push start (a = 1 to the next cell's a = 0) keeps i + a.
__device__ __forceinline__ Raw<double> raw_of(const PState<double>& p, int nz) {
  Raw<double> r;
  r.xi = double(p.i) + p.a;
  r.eta = double(p.j) + p.b;
  r.vr = p.vr;
  r.vt = p.vt;
  r.vz = p.vz;
  return r;
}
__device__ __forceinline__ Raw<float> raw_of(const PState<float>& p, int nz) {
  Raw<float> r;
  r.cell = p.i * nz + p.j;
  r.a = p.a;
  r.b = p.b;
  r.vr = p.vr;
  r.vt = p.vt;
  r.vz = p.vz;
  return r;
}

// The record of a slow-queue entry (the particle's stored record when it was
// queued), field f at rec[f * cap + pos].
__device__ __forceinline__ void store_rec(double* rec, int64_t cap, int64_t pos,
                                          const Raw<double>& r) {
  rec[pos] = r.xi;
  rec[cap + pos] = r.eta;
  rec[2 * cap + pos] = r.vr;
  rec[3 * cap + pos] = r.vt;
  rec[4 * cap + pos] = r.vz;
}
__device__ __forceinline__ void load_rec(const double* rec, int64_t cap, int64_t pos,
                                         Raw<double>& r) {
  r.xi = rec[pos];
  r.eta = rec[cap + pos];
  r.vr = rec[2 * cap + pos];
  r.vt = rec[3 * cap + pos];
  r.vz = rec[4 * cap + pos];
}
__device__ __forceinline__ void store_rec(double* rec, int64_t cap, int64_t pos,
                                          const Raw<float>& r) {
  int32_t* ri = reinterpret_cast<int32_t*>(rec);
  float* rf = reinterpret_cast<float*>(rec);
  ri[pos] = r.cell;
  rf[cap + pos] = r.a;
  rf[2 * cap + pos] = r.b;
  rf[3 * cap + pos] = r.vr;
  rf[4 * cap + pos] = r.vt;
  rf[5 * cap + pos] = r.vz;
}
__device__ __forceinline__ void load_rec(const double* rec, int64_t cap, int64_t pos,
                                         Raw<float>& r) {
  const int32_t* ri = reinterpret_cast<const int32_t*>(rec);
  const float* rf = reinterpret_cast<const float*>(rec);
  r.cell = ri[pos];
  r.a = rf[cap + pos];
  r.b = rf[2 * cap + pos];
  r.vr = rf[3 * cap + pos];
  r.vt = rf[4 * cap + pos];
  r.vz = rf[5 * cap + pos];
}

// cell key i * nz + j of particle k, or -1 if it is dead
template <typename T>
__device__ __forceinline__ int particle_cell(const SpecDev& s, const MapP& m, int64_t k);
template <>
__device__ __forceinline__ int particle_cell<double>(const SpecDev& s, const MapP& m, int64_t k) {
  const double xi = s.xi[k], eta = s.eta[k];
  if (!(xi >= 0.0)) return -1;
  int i = int(floor(xi)), j = int(floor(eta));
  i = i < 0 ? 0 : (i > m.nr - 1 ? m.nr - 1 : i);
  j = j < 0 ? 0 : (j > m.nz - 1 ? m.nz - 1 : j);
  return i * m.nz + j;
}
template <>
__device__ __forceinline__ int particle_cell<float>(const SpecDev& s, const MapP& m, int64_t k) {
  const int c = s.cell[k];
  return c < 0 ? -1 : c;
}

template <typename T>
__device__ __forceinline__ void store_particle(const SpecDev& s, const MapP& m, int64_t k,
                                               const PState<T>& p);
template <>
__device__ __forceinline__ void store_particle<double>(const SpecDev& s, const MapP& m, int64_t k,
                                                       const PState<double>& p) {
  const uint32_t o = (uint32_t)k * 8u;
  at32(s.xi, o) = double(p.i) + p.a;
  at32(s.eta, o) = double(p.j) + p.b;
  at32(s.vr, o) = p.vr;
  at32(s.vt, o) = p.vt;
  at32(s.vz, o) = p.vz;
}
template <>
__device__ __forceinline__ void store_particle<float>(const SpecDev& s, const MapP& m, int64_t k,
                                                      const PState<float>& p) {
  const uint32_t o = (uint32_t)k * 4u;
  at32(s.cell, o) = p.i * m.nz + p.j;
  at32(s.fa, o) = p.a;
  at32(s.fb, o) = p.b;
  at32(s.fvr, o) = p.vr;
  at32(s.fvt, o) = p.vt;
  at32(s.fvz, o) = p.vz;
}

// whether two views of a species are the same particle buffer (the uid
// array is shared by both buffers, the state arrays are not)
__device__ __forceinline__ bool same_buffer(const SpecDev& a, const SpecDev& b) {
  return a.xi == b.xi && a.cell == b.cell;
}

template <typename T>
struct FieldPtr;
template <>
struct FieldPtr<double> {
  static __device__ __forceinline__ const double* r(const PushArgs& a) { return a.ur; }
  static __device__ __forceinline__ const double* z(const PushArgs& a) { return a.uz; }
};
template <>
struct FieldPtr<float> {
  static __device__ __forceinline__ const float* r(const PushArgs& a) { return a.urf; }
  static __device__ __forceinline__ const float* z(const PushArgs& a) { return a.uzf; }
};

// per-thread tallies of a commit pass, reduced once per block
struct Tl {
  double work, dke_abs, dke_coll;
  unsigned absorbed, coll, ion, err, over, ovf, nsub, ncross;
};

__device__ __forceinline__ void tl_zero(Tl& t) {
  t.work = t.dke_abs = t.dke_coll = 0.0;
  t.absorbed = t.coll = t.ion = t.err = t.over = t.ovf = t.nsub = t.ncross = 0;
}

template <int kThreads = kBlock>
__device__ void tl_flush(const Tl& t, Tally* tally, int sid) {
  // wavefront sums, one barrier, then one atomic per non-zero field
  constexpr int kW = kThreads / 64;
  __shared__ double red_d[kW][3];
  __shared__ unsigned red_u[kW][8];
  double d[3] = {t.work, t.dke_abs, t.dke_coll};
  unsigned u[8] = {t.absorbed, t.coll, t.ion, t.err, t.over, t.ovf, t.nsub, t.ncross};
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int q = 0; q < 3; ++q) d[q] += __shfl_down(d[q], off, 64);
#pragma unroll
    for (int q = 0; q < 8; ++q) u[q] += __shfl_down(u[q], off, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) red_d[w][q] = d[q];
#pragma unroll
    for (int q = 0; q < 8; ++q) red_u[w][q] = u[q];
  }
  __syncthreads();
  const int f = threadIdx.x;
  if (f < 3) {
    double sd = 0.0;
    for (int k = 0; k < kW; ++k) sd += red_d[k][f];
    double* dst = f == 0 ? &tally->w_particles : (f == 1 ? &tally->w_absorbed : &tally->w_coll);
    if (sd != 0.0) unsafeAtomicAdd(dst, sd);
  } else if (f < 11) {
    unsigned long long su = 0;
    for (int k = 0; k < kW; ++k) su += red_u[k][f - 3];
    unsigned long long* dst;
    switch (f - 3) {
      case 0: dst = &tally->n_absorbed[sid]; break;
      case 1: dst = &tally->n_coll[sid]; break;
      case 2: dst = &tally->n_ionized; break;
      case 3: dst = &tally->n_errors; break;
      case 4: dst = &tally->n_over_range; break;
      case 5: dst = &tally->n_overflow; break;
      case 6: dst = &tally->n_substeps; break;
      default: dst = &tally->n_crossings; break;
    }
    if (su) atomicAdd(dst, su);
  }
}

// commit of one pushed particle: absorption (wall charge, energy) or state
// write after the null-collision step
template <typename T>
__device__ void commit_one(const PushArgs& A, int64_t k, uint64_t uid, PState<T>& p, int status,
                           int wall, Tl& t) {
  const SpecDev& s = A.out;
  const MapP& m = A.m;
  const double qw = s.q * s.w;
  if (status == kError) t.err += 1;
  if (status == kAbsorbed) {
    kill_slot<T>(s, k);
    t.absorbed += 1;
    t.dke_abs += 0.5 * s.m * s.w * (double(p.vr) * p.vr + double(p.vt) * p.vt + double(p.vz) * p.vz);
    if (wall == 1 || wall == 2) {
      double* w = wall == 1 ? A.wall_bot : A.wall_top;
      unsafeAtomicAdd(&w[p.i], qw * (1.0 - double(p.a)));
      unsafeAtomicAdd(&w[p.i + 1], qw * double(p.a));
    } else {
      unsafeAtomicAdd(&A.wall_side[p.j], qw * (1.0 - double(p.b)));
      unsafeAtomicAdd(&A.wall_side[p.j + 1], qw * double(p.b));
    }
    return;
  }
  if (A.mcc.enabled) {
    double vr = p.vr, vt = p.vt, vz = p.vz;
    const CollOut co = collide_one<T>(A.mcc, s, m, s.sid, uid, p.i, p.j, p.a, p.b, vr, vt, vz,
                                      A.tally);
    t.dke_coll += co.dke;
    t.coll += co.coll;
    t.ion += co.ionized;
    t.over += co.over;
    t.ovf += co.overflow;
    p.vr = T(vr);
    p.vt = T(vt);
    p.vz = T(vz);
  }
  store_particle<T>(s, m, k, p);
}

// ---------------------------------------------------------------------------
// LDS-staged current tile of a fast-pass block
// ---------------------------------------------------------------------------
// One DPP step of a wavefront scan on a double: the value of the lane CTRL
// selects (row_shr:n or row_bcast:15/31) in the rows ROW_MASK enables, 0
// elsewhere.  Needs all 64 lanes active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_take(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xF, true);
  const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xF, true);
  return __hiloint2double(h2, l2);
}

// Sum over the lanes of `mem` of the four edge increments of cell k0 (row
// i0), added to the tile.  A transposing reduction: lane pairs swap halves of
// their values so that each step adds fewer of them; after the two quad
// steps lane l holds component l % 4 of its quad, and two row shifts leave
// the row totals in lanes 12..15 of each row of 16, which add them to the
// tile.  Called by all 64 lanes with uniform k0, i0.
__device__ __forceinline__ void tile_group_add(const Tile& t, int nz, int k0, int i0, bool mem,
                                               const Dep& d) {
  const double r0 = mem ? d.r0 : 0.0, r1 = mem ? d.r1 : 0.0;
  const double z0 = mem ? d.z0 : 0.0, z1 = mem ? d.z1 : 0.0;
  const int lane = threadIdx.x & 63;
  // lanes l, l^1 (quad_perm 1,0,3,2): even lanes keep the r pair, odd the z pair
  const bool odd = lane & 1;
  const double a0 = (odd ? z0 : r0) + dpp_take<0xB1, 0xF>(odd ? r0 : z0);
  const double a1 = (odd ? z1 : r1) + dpp_take<0xB1, 0xF>(odd ? r1 : z1);
  // lanes l, l^2 (quad_perm 2,3,0,1): lane l % 4 = 0, 1, 2, 3 keeps r0, z0, r1, z1
  const bool hi = lane & 2;
  double v = (hi ? a1 : a0) + dpp_take<0x4E, 0xF>(hi ? a0 : a1);
  v += dpp_take<0x114, 0xF>(v);  // row_shr:4
  v += dpp_take<0x118, 0xF>(v);  // row_shr:8
  if ((lane & 15) >= 12 && v != 0.0) {
    const int er = k0 + i0 - t.er0;  // i0 * (nz + 1) + j0
    const int ez = k0 - t.c_lo;
    const int c = lane & 3;
    double* dst = c == 0 ? &t.TR[er] : c == 1 ? &t.TZ[ez] : c == 2 ? &t.TR[er + 1] : &t.TZ[ez + nz];
    atomicAdd(dst, v);
  }
}

// Deposit of one particle per lane.  In cell-sorted order a wavefront's
// particles fall in few cells: the lanes of the first in-tile lane's cell
// are summed by tile_group_add, and so is the next cell's group while the
// groups are large (one LDS atomic per lane would serialise on the shared
// addresses); lanes left over add with LDS atomics, out-of-tile lanes with
// global atomics.  Called by all 64 lanes.
__device__ __forceinline__ void tile_deposit(const Tile& t, double* Ir, double* Iz, int nz, int key,
                                             int i, int j, const Dep& d) {
  constexpr int kGroups = 3;     // at most this many summed groups
  constexpr int kMinGroup = 8;   // smaller groups use LDS atomics
  const bool in = key >= t.c_lo && key < t.c_lo + t.W;
  if (key >= 0 && !in) atomic_dep(Ir, Iz, nz, i, j, d);
  uint64_t pending = __ballot(in);
  const uint64_t me = 1ull << (threadIdx.x & 63);
  for (int g = 0; g < kGroups && pending; ++g) {
    const int lead = __ffsll((unsigned long long)pending) - 1;
    const int k0 = __builtin_amdgcn_readlane(key, lead);
    const int i0 = __builtin_amdgcn_readlane(i, lead);
    const bool mem = (pending & me) && key == k0;
    const uint64_t mm = __ballot(mem);
    if (__popcll(mm) < kMinGroup) break;
    tile_group_add(t, nz, k0, i0, mem, d);
    pending &= ~mm;
  }
  if (pending & me) {
    const int er = key + i - t.er0;
    const int ez = key - t.c_lo;
    atomicAdd(&t.TR[er], d.r0);
    atomicAdd(&t.TR[er + 1], d.r1);
    atomicAdd(&t.TZ[ez], d.z0);
    atomicAdd(&t.TZ[ez + nz], d.z1);
  }
}

// Commit of an in-cell particle in the fast pass: the pushed state is
// stored; with MCC, true when the null-collision draw selects it (the same
// draw collide_one makes first).
template <typename T>
__device__ __forceinline__ bool commit_store(const PushArgs& A, int64_t k, const PState<T>& p) {
  store_particle<T>(A.out, A.m, k, p);
  if (!A.mcc.enabled) return false;
  const uint64_t uid = A.s.uid[k];  // both buffers share the uid array
  double u[4];
  draws(A.mcc.seed, A.s.sid, uid, A.mcc.step, 0, u);
  return u[0] < A.mcc.pnull;
}

// Set bits of a wavefront mask in the lanes below this one.
__device__ __forceinline__ int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Fast pass: every particle solves the mid-point system over the whole step
// in its cell.  Those that stay in the closed cell are done (this is exactly
// the first sub-step of the full algorithm); their currents are gathered in
// the block's LDS tile and flushed once per block.  The others are queued
// for the slow pass.  A block takes kPerThread particles per thread,
// consecutive in memory (sorted by cell after a sort), strided by kBlock.
// Grid (blocks of the larger slot, slots): blockIdx.y is the species slot.
// Dynamic LDS: tile_r_len(nz) + tile_z_len(nz) doubles.
template <typename T, bool COMMIT, bool DEPOSIT>
__global__ void __launch_bounds__(kBlock) k_push_fast(PassArgs P) {
  if (P.a[0].stop && *P.a[0].stop) return;
  extern __shared__ double tile_mem[];
  // the slow and collision lists, a region of kPerWave entries per
  // wavefront filled in order (no atomics), and the records of each
  // wavefront's first kStageW slow particles, kept when they are queued
  // (later ones are fetched again at the end)
  constexpr int kWaves = kBlock / 64, kPerWave = kPerBlock / kWaves, kStageW = 16;
  static_assert(kPerWave == kPerThread * 64, "a list place per particle of the wavefront");
  // entries are offsets in the block (k - k_first < kPerBlock), 16 bits; a
  // wavefront's region holds its slow entries from the front and its
  // collision entries from the back (a particle is at most one of the two,
  // and the region has a place per particle), which keeps the block's LDS
  // small enough for six blocks per CU at c5
  static_assert(kPerBlock <= 65536, "16-bit list offsets");
  __shared__ uint16_t plist[kPerBlock];
  __shared__ Raw<T> slow_rec[kWaves * kStageW];
  __shared__ int wslow[kWaves], wcoll[kWaves], gbase, cbase;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // the species slot indexes the arguments directly (a select between the
  // slots' fields would keep both sets in scalar registers)
  const int slot = blockIdx.y;
  const PushArgs& A = P.a[slot];
  const int64_t bx = blockIdx.x;
  const int64_t k_first = bx * kPerBlock;
  if (k_first >= A.s.n) return;  // the grid covers the larger slot
  int32_t* queue = P.queue[slot];
  int32_t* qcount = P.qcount[slot];
  int32_t* cqueue = P.cqueue[slot];
  int32_t* cqcount = P.cqcount[slot];
  const int64_t qseg = P.qseg[slot];
  const MapP& m = A.m;
  const SpecDev& s = A.s;
  const T qm = T(s.qm);
  const double qw_dt = s.qw_dt;
  const int nz = m.nz;
  // the tile window: one radial row of drift either side of the block's
  // first particle's cell
  Tile tl;
  tl.W = tile_cells(nz);
  tl.TR = tile_mem;
  tl.TZ = tile_mem + tile_r_len(nz);
  {
    int c_first = -1;
    if (k_first < s.n) c_first = particle_cell<T>(s, m, k_first);
    if (c_first < 0) c_first = 0;
    tl.c_lo = max(c_first - nz - 2, 0);
    tl.er0 = tl.c_lo + tl.c_lo / nz;
  }
  if (DEPOSIT) {
    const int ntile = tile_r_len(nz) + tile_z_len(nz);
    for (int e = threadIdx.x; e < ntile; e += kBlock) tile_mem[e] = 0.0;
  }
  __syncthreads();
  int wn_slow = 0, wn_coll = 0;  // this wavefront's list lengths (uniform)
  Tl t;
  tl_zero(t);
  const int lane = threadIdx.x & 63;
  Raw<T> cur, nxt;
  fetch_raw(s, min(k_first + (int64_t)threadIdx.x, s.n - 1), cur);
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t k = k_first + (int64_t)r * kBlock + threadIdx.x;
    PState<T> p;
    bool alive = false;
    if (k < s.n) alive = decode_raw(m, cur, p);
    bool slow = false;
    int key = -1;
    Dep dp{0.0, 0.0, 0.0, 0.0};
    T F[4];
    if (alive) {
      // on a face, the cell the motion goes to (selects, no branches)
      const bool ru = (p.a == T(1)) & (p.vr >= T(0)) & (p.i < m.nr - 1);
      const bool rd = (p.a == T(0)) & (p.vr < T(0)) & (p.i > 0);
      const bool zu = (p.b == T(1)) & (p.vz >= T(0)) & (p.j < m.nz - 1);
      const bool zd = (p.b == T(0)) & (p.vz < T(0)) & (p.j > 0);
      p.i += ru ? 1 : (rd ? -1 : 0);
      p.a = ru ? T(0) : (rd ? T(1) : p.a);
      p.j += zu ? 1 : (zd ? -1 : 0);
      p.b = zu ? T(0) : (zd ? T(1) : p.b);
      load_field(m, FieldPtr<T>::r(A), FieldPtr<T>::z(A), p.i, p.j, F);
    }
    // the next particle's record, issued after this one's field gather; the
    // index is selected (the same particle again in the last round, cached)
    // and clamped (k_first < n) rather than the load skipped, so that no
    // branch joins the loads' results and the gather's wait leaves them in
    // flight
    fetch_raw(s, min(r + 1 < kPerThread ? k + kBlock : k, s.n - 1), nxt);
    if (alive) {
      Mid<T> M;
      slow = true;
      if (p.i >= m.i_lin && solve_fast(m, F, p, T(m.dt), qm, M)) {
        const T ea = T(2) * M.a - p.a, eb = T(2) * M.b - p.b;
        if (ea >= T(0) && ea <= T(1) && eb >= T(0) && eb <= T(1)) {
          slow = false;
          if constexpr (sizeof(T) == 4) {
            // mixed path: the current of the FP32 displacement, taken as its
            // field-free part plus its kick part (summed in FP64) before the
            // new offset is rounded for storage; a current that moved in
            // steps of the stored offset's ulp, or of the mid velocity's,
            // would stall Picard above the tolerance
            const T delta = T(0.5) * T(m.dt) * T(m.inv_s);
            const T gamma = T(0.5) * T(m.dt) * T(m.inv_dz);
            const double da = double(delta * p.vr) + double(delta * M.kr);
            const double db = double(gamma * p.vz) + double(gamma * M.kz);
            dp = make_dep(double(p.a), double(p.b), double(p.a) + 2.0 * da,
                          double(p.b) + 2.0 * db, qw_dt);
          } else {
            dp = make_dep(double(p.a), double(p.b), double(ea), double(eb), qw_dt);
          }
          key = p.i * nz + p.j;
          if (COMMIT) {
            t.work += m.dt * (dp.r0 * double(F[0]) + dp.r1 * double(F[1]) +
                              dp.z0 * double(F[2]) + dp.z1 * double(F[3]));
            t.nsub += 1;
          }
          p.a = ea;
          p.b = eb;
          if constexpr (sizeof(T) == 4) {
            p.vr = p.vr + T(2) * M.kr;
            p.vz = p.vz + T(2) * M.kz;
          } else {
            p.vr = T(2) * M.vr - p.vr;
            p.vz = T(2) * M.vz - p.vz;
          }
          p.vt = T(2) * M.vt - p.vt;
        }
      }
    }
    if (DEPOSIT) tile_deposit(tl, A.Ir, A.Iz, nz, key, p.i, p.j, dp);
    // the wavefront's slow list
    const uint64_t mask = __ballot(slow);
    if (slow) {
      const int qi = wn_slow + lanes_below(mask);
      plist[wv * kPerWave + qi] = (uint16_t)(k - k_first);
      if (qi < kStageW) slow_rec[wv * kStageW + qi] = raw_of(p, nz);
    }
    wn_slow = __builtin_amdgcn_readfirstlane(wn_slow + (int)__popcll(mask));
    if (COMMIT) {
      // in-cell particles are stored as pushed; those the null-collision
      // draw selects go to the collision list
      bool coll = false;
      if (alive && !slow) coll = commit_store<T>(A, k, p);
      // into the other buffer: dead slots stay dead there
      if (k < s.n && !alive && !same_buffer(A.out, A.s)) kill_slot<T>(A.out, k);
      const uint64_t cm = __ballot(coll);
      if (coll)
        plist[wv * kPerWave + kPerWave - 1 - (wn_coll + lanes_below(cm))] = (uint16_t)(k - k_first);
      wn_coll = __builtin_amdgcn_readfirstlane(wn_coll + (int)__popcll(cm));
    }
    cur = nxt;
  }
  if (lane == 0) {
    wslow[wv] = wn_slow;
    wcoll[wv] = wn_coll;
  }
  __syncthreads();
  // flush the tile: one global atomic per touched edge
  if (DEPOSIT) {
    const int64_t ner = (int64_t)m.nr * (nz + 1), nez = (int64_t)(m.nr + 1) * nz;
    const int lr = tile_r_len(nz), lz = tile_z_len(nz);
    for (int e = threadIdx.x; e < lr; e += kBlock) {
      const double v = tl.TR[e];
      if (v != 0.0 && tl.er0 + e < ner) unsafeAtomicAdd(A.Ir + tl.er0 + e, v);
    }
    for (int e = threadIdx.x; e < lz; e += kBlock) {
      const double v = tl.TZ[e];
      if (v != 0.0 && tl.c_lo + e < nez) unsafeAtomicAdd(A.Iz + tl.c_lo + e, v);
    }
  }
  // queue the slow ones (and the colliding ones): one global atomic per block
  const int64_t seg = bx % kSpread;
  // list entry q of the block: wavefront w of the first whose lists end
  // beyond q, at offset q - (entries of the wavefronts before w)
  int spre[kWaves + 1], cpre[kWaves + 1];
  spre[0] = cpre[0] = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    spre[w + 1] = spre[w] + wslow[w];
    cpre[w + 1] = cpre[w] + wcoll[w];
  }
  const int ns = spre[kWaves];
  if (ns) {
    if (threadIdx.x == 0) gbase = atomicAdd(qcount + seg * kLineInts, ns);
    __syncthreads();
    // with each entry the particle's record, which the slow pass then reads
    // in order instead of gathering it
    double* rec = P.qrec[slot];
    for (int q = threadIdx.x; q < ns; q += kBlock) {
      int w = 0;
#pragma unroll
      for (int u = 1; u < kWaves; ++u) w += q >= spre[u] ? 1 : 0;
      const int o = q - spre[w];
      const int32_t kq = (int32_t)(k_first + plist[w * kPerWave + o]);
      const int64_t pos = seg * qseg + gbase + q;
      queue[pos] = kq;
      Raw<T> r;
      if (o < kStageW)
        r = slow_rec[w * kStageW + o];
      else
        fetch_raw(s, kq, r);
      store_rec(rec, P.qcap, pos, r);
    }
  }
  if (!COMMIT) return;
  const int nc = cpre[kWaves];
  if (nc) {
    if (threadIdx.x == 0) cbase = atomicAdd(cqcount + seg * kLineInts, nc);
    __syncthreads();
    for (int q = threadIdx.x; q < nc; q += kBlock) {
      int w = 0;
#pragma unroll
      for (int u = 1; u < kWaves; ++u) w += q >= cpre[u] ? 1 : 0;
      cqueue[seg * qseg + cbase + q] =
          (int32_t)(k_first + plist[w * kPerWave + kPerWave - 1 - (q - cpre[w])]);
    }
  }
  tl_flush(t, A.tally + (blockIdx.x % kSpread), s.sid);
}

// Queue passes: the slow pass over the particles the fast pass queued, the
// collisions of the particles a committing fast pass listed, or both in one
// launch.  A pass has roles (the slow queue or the collision list of a
// slot); the entries of each role's kSpread segments are read as one list
// in segment order, the lists of the roles follow each other, and
// wavefront w takes entries [64 u, 64 u + 64) of the whole for
// u = w, w + W, ... (W wavefronts).  Blocks are one wavefront, so the work
// lands on the first wavefronts of the grid, spread over every XCD and
// compute unit: the pass is latency-bound (one particle per lane, a chain of
// dependent FP64 steps per face crossing), and a SIMD that runs two such
// wavefronts runs each more slowly.
static_assert(kSpread == 64, "one queue segment per lane");
constexpr int kQThreads = 64;

struct QView {
  int excl;   // lane g: entries in segments before g
  int total;  // entries in all segments
};

__device__ __forceinline__ QView queue_view(const int32_t* qcount) {
  const int lane = threadIdx.x & 63;
  const int c = qcount[lane * kLineInts];
  int incl = c;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  QView q;
  q.excl = incl - c;
  q.total = __builtin_amdgcn_readlane(incl, 63);  // uniform: the role loop stays scalar
  return q;
}

// Position in the queue buffer of list entry e < total: the last segment
// whose exclusive prefix is <= e (empty segments before it share its
// prefix), at offset e - prefix.  All lanes must be active.
__device__ __forceinline__ int64_t queue_pos(const QView& q, int e, int64_t qseg) {
  int g = 0;
#pragma unroll
  for (int step = 32; step > 0; step >>= 1) {
    const int cand = g + step;
    const int v = __shfl(q.excl, cand & 63, 64);
    if (cand < 64 && v <= e) g = cand;
  }
  return (int64_t)g * qseg + (e - __shfl(q.excl, g, 64));
}

// Slow pass of one queued particle (loaded into p): the full push with
// splitting at every face crossing (restarted from the particle's state),
// currents into the wavefront's tile.
template <typename T, bool COMMIT>
__device__ __forceinline__ void slow_one(const PushArgs& A, int64_t k, uint64_t uid, PState<T>& p,
                                         const Tile& tl, Tl& t) {
  const MapP& m = A.m;
  const SpecDev& s = A.s;
  const double qw_dt = s.qw_dt;
  PushOut o;
  if constexpr (sizeof(T) == 4) {
    // mixed path: the few face crossers are pushed in FP64 arithmetic
    // (in the FP64 half-step field) from their FP32 state and stored back
    // rounded, so that their currents vary smoothly with the field
    PState<double> pd;
    pd.i = p.i;
    pd.j = p.j;
    pd.a = p.a;
    pd.b = p.b;
    pd.vr = p.vr;
    pd.vt = p.vt;
    pd.vz = p.vz;
    push_particle<double>(m, A.ur, A.uz, A.Ir, A.Iz, tl, pd, s.qm, qw_dt, COMMIT, o);
    p.i = pd.i;
    p.j = pd.j;
    p.a = T(pd.a);
    p.b = T(pd.b);
    p.vr = T(pd.vr);
    p.vt = T(pd.vt);
    p.vz = T(pd.vz);
  } else {
    push_particle<T>(m, FieldPtr<T>::r(A), FieldPtr<T>::z(A), A.Ir, A.Iz, tl, p, T(s.qm),
                     qw_dt, COMMIT, o);
  }
  if (COMMIT) {
    t.work += o.work;
    t.nsub += o.nsub;
    t.ncross += o.ncross;
    commit_one<T>(A, k, uid, p, o.status, o.wall, t);
  }
}

// Collision of one listed particle (its pushed state is already stored).
// Particles born here are appended beyond the pass's start counts.
template <typename T>
__device__ __forceinline__ void listed_one(const PushArgs& A, int64_t k, Tl& t) {
  const MapP& m = A.m;
  const SpecDev& s = A.out;  // the pushed state, where the commit stored it
  const uint64_t uid = s.uid[k];  // issued with the record's loads
  PState<T> p;
  if (!load_particle<T>(s, m, k, p)) return;
  double vr = p.vr, vt = p.vt, vz = p.vz;
  const CollOut co = collide_one<T>(A.mcc, s, m, s.sid, uid, p.i, p.j, p.a, p.b, vr, vt, vz,
                                    A.tally);
  t.dke_coll += co.dke;
  t.coll += co.coll;
  t.ion += co.ionized;
  t.over += co.over;
  t.ovf += co.overflow;
  p.vr = T(vr);
  p.vt = T(vt);
  p.vz = T(vz);
  store_particle<T>(s, m, k, p);
}

// MODE 0: slow pass (roles: the slots' queues); 1: committing slow pass;
// 2: collision lists; 3: committing slow pass then collision lists (2 slots
// roles).  The slow roles do nothing once the residual has stopped the
// iteration.  Grid: 1-D, one wavefront per block.
enum { kQSlow = 0, kQSlowCommit = 1, kQCollide = 2, kQSlowCollide = 3 };

// WAVES: the wavefronts per SIMD the register budget is cut for.  Two keep
// the push in registers; three (the plain slow pass on large workloads,
// where it is throughput-bound) spill a few and hold more wavefronts.
template <typename T, int MODE, int WAVES>
__global__ void __launch_bounds__(kQThreads, WAVES) k_queue(PassArgs P) {
  // dynamic LDS (slow roles): the tile, slow_r_len(nz) + slow_z_len(nz)
  // doubles
  extern __shared__ double qtile[];
  const bool stopped = P.a[0].stop && *P.a[0].stop;
  if (MODE == kQSlow && stopped) return;
  constexpr int kMaxRoles = MODE == kQSlowCollide ? 4 : 2;
  const int nroles = MODE == kQSlowCollide ? 2 * P.nsp : P.nsp;
  const int lane = threadIdx.x;
  constexpr bool kTally = MODE != kQSlow;
  // every role's view up front: its counter loads then precede the
  // particle work, whose deposit atomics a later load would wait for
  QView vw[kMaxRoles];
#pragma unroll
  for (int r = 0; r < kMaxRoles; ++r) {
    vw[r].excl = 0;
    vw[r].total = 0;
    if (r < nroles) {
      const int sl = r % P.nsp;
      const bool sw = MODE == kQCollide ? false : (MODE == kQSlowCollide ? r < P.nsp : true);
      if (!(sw && stopped)) vw[r] = queue_view(sw ? P.qcount[sl] : P.cqcount[sl]);
    }
  }
  int role = 0;
  int64_t base = 0;  // units of the roles before `role`
  bool worked = false;
  Tl t;
  tl_zero(t);
  for (int64_t u = blockIdx.x;; u += gridDim.x) {
    // wavefront-uniform: the role of unit u
    QView v = vw[0];
#pragma unroll
    for (int r = 1; r < kMaxRoles; ++r)
      if (role == r) v = vw[r];
    while (role < nroles && u >= base + (v.total + 63) / 64) {
      if (kTally && worked) {
        const PushArgs& A = P.a[role % P.nsp];
        tl_flush<kQThreads>(t, A.tally + (blockIdx.x % kSpread), A.s.sid);
        tl_zero(t);
        worked = false;
      }
      base += (v.total + 63) / 64;
      ++role;
#pragma unroll
      for (int r = 1; r < kMaxRoles; ++r)
        if (role == r) v = vw[r];
    }
    if (role >= nroles) break;
    // uniform by construction; said so, so that the slot's arguments are
    // read by scalar loads and kept in scalar registers
    role = __builtin_amdgcn_readfirstlane(role);
    const int slot = role % P.nsp;
    const bool slow = MODE == kQCollide ? false : (MODE == kQSlowCollide ? role < P.nsp : true);
    const int64_t e = (u - base) * 64 + lane;
    const int64_t pos = queue_pos(v, (int)(e < v.total ? e : v.total - 1), P.qseg[slot]);
    worked = true;
    const PushArgs& A = P.a[slot];
    if (MODE != kQCollide && slow) {
      // the unit's particles, then a tile over their cells from just below
      // the lowest (a unit holds consecutive queue entries, which come from
      // one or two fast-pass blocks of cell-sorted particles)
      int64_t k = 0;
      uint64_t uid = 0;
      PState<T> p;
      bool ok = false;
      if (e < v.total) {
        k = P.queue[slot][pos];
        // a commit's id load (both buffers share the id array), issued now
        // so that it is in flight during the push
        if (MODE != kQSlow) uid = A.s.uid[k];
        Raw<T> r;
        load_rec(P.qrec[slot], P.qcap, pos, r);
        ok = decode_raw(A.m, r, p);
      }
      const int nz = A.m.nz;
      int c = ok ? p.i * nz + p.j : INT_MAX;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) c = min(c, __shfl_xor(c, off, 64));
      Tile tl;
      tl.W = slow_cells(nz);
      tl.TR = qtile;
      tl.TZ = qtile + slow_r_len(nz);
      tl.c_lo = max((c == INT_MAX ? 0 : c) - slow_below(nz), 0);
      tl.er0 = tl.c_lo + tl.c_lo / nz;
      const int lr = slow_r_len(nz), lz = slow_z_len(nz);
      // a pass without deposit (null currents) leaves the tile untouched
      const bool dep = A.Ir != nullptr;
      if (dep)
        for (int q = lane; q < lr + lz; q += kQThreads) qtile[q] = 0.0;
      __syncthreads();
      if (ok) slow_one<T, MODE != kQSlow>(A, k, uid, p, tl, t);
      __syncthreads();
      if (dep) {
        // flush: one global atomic per touched edge
        const int64_t ner = (int64_t)A.m.nr * (nz + 1), nez = (int64_t)(A.m.nr + 1) * nz;
        for (int q = lane; q < lr; q += kQThreads) {
          const double x = tl.TR[q];
          if (x != 0.0 && tl.er0 + q < ner) unsafeAtomicAdd(A.Ir + tl.er0 + q, x);
        }
        for (int q = lane; q < lz; q += kQThreads) {
          const double x = tl.TZ[q];
          if (x != 0.0 && tl.c_lo + q < nez) unsafeAtomicAdd(A.Iz + tl.c_lo + q, x);
        }
      }
      __syncthreads();
    } else if (MODE != kQSlow) {
      if (e < v.total) listed_one<T>(A, P.cqueue[slot][pos], t);
    }
  }
}

// wavefronts (one-wavefront blocks) of a queue pass over slots of at most
// nmax particles: enough for 1/16 of them in one round (more loop); a
// multiple of 8 XCDs
inline unsigned queue_grid(int64_t nmax, int nsp) {
  int64_t w = (nmax * nsp) / 1024;
  w = w < 64 ? 64 : w;
  w = (w + 7) / 8 * 8;
  return (unsigned)(w > (1 << 30) ? (1 << 30) : w);
}

// standalone collision pass over the live particles
template <typename T>
__global__ void __launch_bounds__(kBlock) k_collide(MapP m, SpecDev s, MccDev c, Tally* tally) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  PState<T> p;
  bool alive = false;
  if (k < c.base_self) alive = load_particle<T>(s, m, k, p);
  double dke = 0.0;
  unsigned coll = 0, ion = 0, over = 0, ovf = 0;
  if (alive) {
    double vr = p.vr, vt = p.vt, vz = p.vz;
    const CollOut co = collide_one<T>(c, s, m, s.sid, s.uid[k], p.i, p.j, p.a, p.b, vr, vt, vz, tally);
    dke = co.dke;
    coll = co.coll;
    ion = co.ionized;
    over = co.over;
    ovf = co.overflow;
    if (co.coll) {
      p.vr = T(vr);
      p.vt = T(vt);
      p.vz = T(vz);
      store_particle<T>(s, m, k, p);
    }
  }
  Tally* tt = tally + (blockIdx.x % kSpread);
  block_sum_atomic(dke, &tt->w_coll);
  block_count_atomic(coll, &tt->n_coll[s.sid]);
  block_count_atomic(ion, &tt->n_ionized);
  block_count_atomic(over, &tt->n_over_range);
  block_count_atomic(ovf, &tt->n_overflow);
}

// physical (r, z) -> logical state
__device__ __forceinline__ double xi_of_r(const MapP& m, double r) {
  if (m.xi_a > 0.0 && r < 2.0 * m.s * m.xi_a) return r * r / (4.0 * m.s * m.s * m.xi_a);
  return r * m.inv_s - m.xi_a;
}

__global__ void k_load(MapP m, SpecDev s, const double* r, const double* z, const double* vr,
                       const double* vt, const double* vz, const uint64_t* uid, int64_t n,
                       int mixed) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  double xi = xi_of_r(m, r[k]);
  double eta = z[k] * m.inv_dz;
  xi = fmin(fmax(xi, 0.0), double(m.nr));
  eta = fmin(fmax(eta, 0.0), double(m.nz));
  if (!mixed) {
    s.xi[k] = xi;
    s.eta[k] = eta;
    s.vr[k] = vr[k];
    s.vt[k] = vt[k];
    s.vz[k] = vz[k];
  } else {
    int i = int(floor(xi)), j = int(floor(eta));
    i = i > m.nr - 1 ? m.nr - 1 : i;
    j = j > m.nz - 1 ? m.nz - 1 : j;
    s.cell[k] = i * m.nz + j;
    s.fa[k] = float(xi - i);
    s.fb[k] = float(eta - j);
    s.fvr[k] = float(vr[k]);
    s.fvt[k] = float(vt[k]);
    s.fvz[k] = float(vz[k]);
  }
  s.uid[k] = uid[k];
}

// stable compaction of live particles into FP64 outputs
__global__ void k_flag_count(MapP m, SpecDev s, int64_t n, int mixed, int32_t* blk) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool alive = false;
  if (k < n) alive = mixed ? (s.cell[k] >= 0) : (s.xi[k] >= 0.0);
  const int c = __syncthreads_count(alive);
  if (threadIdx.x == 0) blk[blockIdx.x] = c;
}

__global__ void k_compact_read(MapP m, SpecDev s, int64_t n, int mixed, const int32_t* blk_off,
                               double* xi, double* eta, double* vr, double* vt, double* vz,
                               uint64_t* uid) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool alive = false;
  if (k < n) alive = mixed ? (s.cell[k] >= 0) : (s.xi[k] >= 0.0);
  __shared__ int wsum[kBlock / 64];
  const uint64_t bal = __ballot(alive);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int before = __popcll(bal & ((1ull << lane) - 1ull));
  if (lane == 0) wsum[w] = __popcll(bal);
  __syncthreads();
  int off = blk_off[blockIdx.x];
  for (int q = 0; q < w; ++q) off += wsum[q];
  if (!alive) return;
  const int64_t d = off + before;
  if (!mixed) {
    xi[d] = s.xi[k];
    eta[d] = s.eta[k];
    vr[d] = s.vr[k];
    vt[d] = s.vt[k];
    vz[d] = s.vz[k];
  } else {
    const int c = s.cell[k];
    const int i = c / m.nz, j = c - (c / m.nz) * m.nz;
    xi[d] = double(i) + double(s.fa[k]);
    eta[d] = double(j) + double(s.fb[k]);
    vr[d] = s.fvr[k];
    vt[d] = s.fvt[k];
    vz[d] = s.fvz[k];
  }
  uid[d] = s.uid[k];
}

}  // namespace

// nu_max = 1.05 n_g max_{eps <= eps_max} sigma_tot(eps) v(eps) on a 2e5-point
// energy grid (electrons), or 1.05 n_g sigma_cx g(eps_max) (ions)
double nu_max_host(const ecpic_mcc_desc& c, int role, double mp) {
  if (role == 1) {
    double best = 0.0;
    const int K = 200000;
    for (int k = 1; k <= K; ++k) {
      const double e = c.eps_max_ev * (double)k / (double)K;
      double a, b, d;
      xsec(e, a, b, d);
      const double f = (a + b + d) * sqrt(2.0 * e * kQE / mp);
      if (f > best) best = f;
    }
    return 1.05 * c.n_gas * best;
  }
  if (role == 2) return 1.05 * c.n_gas * 5.0e-19 * sqrt(2.0 * c.eps_max_ev * kQE / mp);
  return 0.0;
}

int64_t fast_blocks(int64_t n) { return (n + kPerBlock - 1) / kPerBlock; }

size_t fast_lds_bytes(int nz) {
  return sizeof(double) * (size_t)(tile_r_len(nz) + tile_z_len(nz));
}

hipError_t launch_push_fast(const PassArgs& P, bool deposit, hipStream_t st) {
  int64_t nb = 0;
  for (int q = 0; q < P.nsp; ++q) nb = fast_blocks(P.a[q].s.n) > nb ? fast_blocks(P.a[q].s.n) : nb;
  if (nb <= 0) return hipSuccess;
  const size_t lds = deposit ? fast_lds_bytes(P.a[0].m.nz) : 0;
  if (lds > 56 * 1024) return hipErrorInvalidValue;
  const bool mixed = (P.a[0].s.cell != nullptr);
  const bool commit = P.a[0].commit != 0;
  if (!commit && !deposit) return hipErrorInvalidValue;
  const dim3 g((unsigned)nb, (unsigned)P.nsp), b(kBlock);
  if (!mixed) {
    if (!commit)
      hipLaunchKernelGGL((k_push_fast<double, false, true>), g, b, lds, st, P);
    else if (deposit)
      hipLaunchKernelGGL((k_push_fast<double, true, true>), g, b, lds, st, P);
    else
      hipLaunchKernelGGL((k_push_fast<double, true, false>), g, b, lds, st, P);
  } else {
    if (!commit)
      hipLaunchKernelGGL((k_push_fast<float, false, true>), g, b, lds, st, P);
    else if (deposit)
      hipLaunchKernelGGL((k_push_fast<float, true, true>), g, b, lds, st, P);
    else
      hipLaunchKernelGGL((k_push_fast<float, true, false>), g, b, lds, st, P);
  }
  return hipGetLastError();
}

namespace {
int64_t max_slot_n(const PassArgs& P) {
  int64_t nmax = 0;
  for (int q = 0; q < P.nsp; ++q) nmax = P.a[q].s.n > nmax ? P.a[q].s.n : nmax;
  return nmax;
}

template <int MODE, int WAVES>
void launch_queue_w(const PassArgs& P, int64_t nmax, hipStream_t st) {
  const dim3 gs(queue_grid(nmax, P.nsp), 1, 1);
  const int nz = P.a[0].m.nz;
  const size_t lds = MODE == kQCollide ? 0 : sizeof(double) * (size_t)(slow_r_len(nz) + slow_z_len(nz));
  if (P.a[0].s.cell != nullptr)
    hipLaunchKernelGGL((k_queue<float, MODE, WAVES>), gs, dim3(kQThreads), lds, st, P);
  else
    hipLaunchKernelGGL((k_queue<double, MODE, WAVES>), gs, dim3(kQThreads), lds, st, P);
}

// particles in a pass from which the plain slow pass takes the three-wavefront
// build (at 4.2M its queue fits the GPU in one round and latency decides; at
// 268M it is throughput-bound: 2.5 -> 2.2 ms per pass)
constexpr int64_t kWideQueue = (int64_t)16 << 20;

template <int MODE>
void launch_queue(const PassArgs& P, int64_t nmax, hipStream_t st) {
  if constexpr (MODE == kQSlow) {
    if (P.queue_waves == 3 || (P.queue_waves == 0 && nmax * P.nsp >= kWideQueue)) {
      launch_queue_w<MODE, 3>(P, nmax, st);
      return;
    }
  }
  launch_queue_w<MODE, 2>(P, nmax, st);
}
}  // namespace

hipError_t launch_collide_list(const PassArgs& P, hipStream_t st) {
  const int64_t nmax = max_slot_n(P);
  if (nmax <= 0) return hipSuccess;
  launch_queue<kQCollide>(P, nmax, st);
  return hipGetLastError();
}

hipError_t launch_slow_collide(const PassArgs& P, hipStream_t st) {
  const int64_t nmax = max_slot_n(P);
  if (nmax <= 0) return hipSuccess;
  if (P.a[0].commit == 0) return hipErrorInvalidValue;
  launch_queue<kQSlowCollide>(P, nmax, st);
  return hipGetLastError();
}

hipError_t launch_push_slow(const PassArgs& P, hipStream_t st) {
  const int64_t nmax = max_slot_n(P);
  if (nmax <= 0) return hipSuccess;
  if (P.a[0].commit != 0)
    launch_queue<kQSlowCommit>(P, nmax, st);
  else
    launch_queue<kQSlow>(P, nmax, st);
  return hipGetLastError();
}

hipError_t launch_collide(const MapP& m, const SpecDev& s, const MccDev& c, Tally* tally, int mixed,
                          hipStream_t st) {
  if (c.base_self <= 0) return hipSuccess;
  const int64_t nb = (c.base_self + kBlock - 1) / kBlock;
  if (mixed)
    hipLaunchKernelGGL((k_collide<float>), dim3(nb), dim3(kBlock), 0, st, m, s, c, tally);
  else
    hipLaunchKernelGGL((k_collide<double>), dim3(nb), dim3(kBlock), 0, st, m, s, c, tally);
  return hipGetLastError();
}

hipError_t launch_load(const MapP& m, const SpecDev& s, const double* r, const double* z,
                       const double* vr, const double* vt, const double* vz, const uint64_t* uid,
                       int64_t n, double R, int mixed, hipStream_t st) {
  (void)R;
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_load, dim3(nb), dim3(kBlock), 0, st, m, s, r, z, vr, vt, vz, uid, n, mixed);
  return hipGetLastError();
}

hipError_t launch_flag_count(const MapP& m, const SpecDev& s, int64_t n, int mixed, int32_t* blk,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_flag_count, dim3(nb), dim3(kBlock), 0, st, m, s, n, mixed, blk);
  return hipGetLastError();
}

hipError_t launch_compact_read(const MapP& m, const SpecDev& s, int64_t n, int mixed,
                               const int32_t* blk_off, double* xi, double* eta, double* vr,
                               double* vt, double* vz, uint64_t* uid, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_compact_read, dim3(nb), dim3(kBlock), 0, st, m, s, n, mixed, blk_off, xi,
                     eta, vr, vt, vz, uid);
  return hipGetLastError();
}

}  // namespace ecpic
