// ecpic_field.hip -- Crank-Nicolson update of the TM fields (Eq. (2) of
// Sec. 2.1 with mid-point centring) with H_theta as the unknown.
//
// Eliminating the interior edge voltages leaves an SPD system for
// h^{n+1/2} of the form T (x) I + G (x) N, where N is the Neumann second
// difference in z (the PEC r-edges of the z walls decouple the end cells).
// Three kernels solve it:
//   k_rhs_dct      one block per group of radial rows: the right-hand side of
//                  the rows into LDS, then their orthonormal DCT-II
//                  (precomputed FP64 matrix, L2-resident), written mode-major;
//   k_tri_scan     one block per z-mode: the tridiagonal system in r with
//                  precomputed LU factors, forward and backward substitution
//                  done as parallel scans of affine maps (the recurrences
//                  y_i = d_i - l_i y_{i-1}, x_i = (y_i - e_{i+1} x_{i+1}) / c_i
//                  compose associatively);
//   k_idct_recover one block per group of rows: inverse DCT of the rows and of
//                  the row below them, the edge voltages from Ampere's law,
//                  h^{n+1}, the next half-step field, per-block partial sums of
//                  the Picard residual, and the reset of the consumed currents.
// Grouping rows lets each load of the transform matrix feed several rows.
#include <cmath>
#include <cstring>
#include <mutex>

#include "ecpic_internal.h"

// The transform intermediate of ecpic_field_solve_noalloc: a static array of
// the library on every GPU it runs on (held until the process ends), used
// in place of the context's scratch by the entry point that may not
// allocate.  Host code reaches it only through the per-device address that
// hipGetSymbolAddress returns (static_scratch_setup); the name itself is a
// host-side stand-in and must not be passed to a kernel.
static __device__ __align__(256) double scratch[ecpic::kStaticScratchDoubles];

namespace ecpic {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  // with `device` current: its own copy of the array, at its own address
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[device] = static_cast<double*>(p);
  return hipSuccess;
}

double* static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch[device];
}

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kFB = 256;  // threads per block of the field kernels
constexpr int kRB = 4;    // radial rows per block of the transform kernels
constexpr int kCC = 32;   // output columns per block of the transform kernels

inline int64_t nblk(int64_t n) { return (n + kBlock - 1) / kBlock; }
inline int row_blocks(int nr) { return (nr + kRB - 1) / kRB; }
inline int col_blocks(int nz) { return (nz + kCC - 1) / kCC; }

// Blocked dense transform shared by both directions:
//   out[r][c] = sum_s M[s][c0 + c] in[r][s],  r < R, c < nc, s < ns,
// for R rows of `in` (LDS, stride ns) and a chunk of nc output columns, M
// row-major with row stride ldm.  With P = kFB / nc parts the thread (c, p)
// sums s over the p-th part; the parts land in psum[p][r][c] and are added
// in part order (deterministic).  A block covers kRB rows and kCC columns,
// so the grid has enough blocks to fill the chip and each thread a short
// chain.  Independent loads of M are issued ahead in groups of kUnroll.
constexpr int kUnroll = 8;
__host__ __device__ __forceinline__ int chunk_parts(int nc) { return nc >= kFB ? 1 : kFB / nc; }

// The thread's task of a chunk (at most one: nc * P <= kFB) with the first
// kUnroll entries of its column of M, loaded by dense_pre so that a kernel
// can issue them before it fills `in`.
struct DenseTask {
  bool on;
  int p, c, s0, s1;
  double q0[kUnroll];
};

__device__ __forceinline__ void dense_pre(const double* __restrict__ M, int ldm, int ns, int c0,
                                          int nc, DenseTask& d) {
  const int P = chunk_parts(nc);
  const int t = threadIdx.x;
  d.on = t < nc * P;
  d.p = d.on ? t / nc : 0;
  d.c = t - d.p * nc;
  d.s0 = d.p * ns / P;
  d.s1 = d.on ? (d.p + 1) * ns / P : d.s0;
  if (d.s0 + kUnroll <= d.s1) {
    const double* q = M + c0 + d.c;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) d.q0[u] = q[(int64_t)(d.s0 + u) * ldm];
  }
}

template <int R>
__device__ __forceinline__ void dense_run(const double* __restrict__ M, int ldm,
                                          const double* __restrict__ in, int ns, int c0, int nc,
                                          double* __restrict__ psum, const DenseTask& d) {
  if (d.on) {
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    const double* q = M + c0 + d.c;
    int j = d.s0;
    if (j + kUnroll <= d.s1) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = fma(in[r * ns + j + u], d.q0[u], acc[r]);
      j += kUnroll;
    }
    for (; j + kUnroll <= d.s1; j += kUnroll) {
      double qv[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) qv[u] = q[(int64_t)(j + u) * ldm];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = fma(in[r * ns + j + u], qv[u], acc[r]);
    }
    for (; j < d.s1; ++j) {
      const double qv = q[(int64_t)j * ldm];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = fma(in[r * ns + j], qv, acc[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) psum[(d.p * R + r) * nc + d.c] = acc[r];
  }
  __syncthreads();
}

template <int R>
__device__ __forceinline__ void dense_chunk(const double* __restrict__ M, int ldm,
                                            const double* __restrict__ in, int ns, int c0, int nc,
                                            double* __restrict__ psum) {
  DenseTask d;
  dense_pre(M, ldm, ns, c0, nc, d);
  dense_run<R>(M, ldm, in, ns, c0, nc, psum, d);
}

__device__ __forceinline__ double chunk_total(const double* __restrict__ psum, int nc, int r, int c,
                                              int R) {
  const int P = chunk_parts(nc);
  double v = psum[r * nc + c];
  for (int p = 1; p < P; ++p) v += psum[(p * R + r) * nc + c];
  return v;
}

// rhs[i][j] = 2 pi r_{i+1/2} (2 mu A_c / dt h0 + circulation of u0 - D^-1 I)
// with the half-step drive value on the gap edge and zero on other walls,
// then hat[k][i] = sum_j Q[k][j] rhs[i][j].
__global__ void __launch_bounds__(kFB) k_rhs_dct(MapP m, const double* __restrict__ rh,
                                                 const double* __restrict__ wr,
                                                 const double* __restrict__ wz,
                                                 const double* __restrict__ area, double mu,
                                                 const double* __restrict__ ur0,
                                                 const double* __restrict__ uz0,
                                                 const double* __restrict__ h0,
                                                 const double* __restrict__ Ir,
                                                 const double* __restrict__ Iz, double vhalf,
                                                 const double* __restrict__ gapv,
                                                 const double* __restrict__ Qt,
                                                 double* __restrict__ hat,
                                                 const int32_t* __restrict__ stop, PortDev P) {
  if (stop && *stop) return;
  extern __shared__ double sh[];  // kRB rows of the right-hand side, then the part sums
  const int nr = m.nr, nz = m.nz;
  // blocking capacitor: the gap's half-step voltage from the electrode's
  // potential at t^n (u0's gap edge) and the circuit's current iterate
  if (gapv && P.ip == 0) vhalf = 0.5 * (ur0[(int64_t)(nr - 1) * (nz + 1)] + gapv[0]);
  const double dphi = port_dphi(P);
  const int i0 = blockIdx.x * kRB;
  const int rows = min(kRB, nr - i0);
  const int k0 = blockIdx.y * kCC;
  const int nk = min(kCC, nz - k0);
  DenseTask dt;  // the transform's first loads, in flight while the rows are formed
  dense_pre(Qt, nz, nz, k0, nk, dt);
  const double hdt = 0.5 * m.dt;
  for (int e = threadIdx.x; e < rows * nz; e += blockDim.x) {
    const int r = e / nz, j = e - r * nz, i = i0 + r;
    const double mi = 2.0 * kPi * rh[i];
    const double mass = 2.0 * mu * area[i] / m.dt;
    const double iwr = hdt / wr[i], iwz = hdt / wz[i];
    const double iwz1 = (i + 1 < nr) ? hdt / wz[i + 1] : 0.0;
    const double* urr = ur0 + (int64_t)i * (nz + 1);
    const double* Irr = Ir + (int64_t)i * (nz + 1);
    // r-edges j (bottom) and j+1 (top) of cell (i, j)
    double rb, rt;
    if (j == 0) {
      if (P.ip == 0) {
        rb = (i == nr - 1) ? vhalf : 0.0;
      } else if (i >= P.ip) {
        // port edge: u^n plus the h-free part of its half-step change
        const double g = P.pc[kPortG * nr + i], pa = P.pc[kPortA * nr + i];
        rb = urr[0] + 0.5 * g * (mi * P.hb[i] + pa * dphi - Irr[0]);
      } else {
        rb = 0.0;
      }
    } else {
      rb = urr[j] - Irr[j] * iwr;
    }
    if (j + 1 == nz)
      rt = 0.0;
    else
      rt = urr[j + 1] - Irr[j + 1] * iwr;
    // z-edges i (left) and i+1 (right)
    const int64_t el = (int64_t)i * nz + j;
    const double zl = uz0[el] - Iz[el] * iwz;
    const double zr = (i + 1 < nr) ? uz0[el + nz] - Iz[el + nz] * iwz1 : 0.0;
    sh[r * nz + j] = mi * (mass * h0[el] + (zr - zl - rt + rb));
  }
  __syncthreads();
  // hat[k][i] = sum_j Qt[j][k] rhs[i][j] for the block's modes k0 .. k0+nk-1
  double* psum = sh + kRB * nz;
  dense_run<kRB>(Qt, nz, sh, nz, k0, nk, psum, dt);
  for (int e = threadIdx.x; e < nk * kRB; e += blockDim.x) {
    const int kl = e / kRB, r = e - kl * kRB;
    if (r < rows) hat[(int64_t)(k0 + kl) * nr + i0 + r] = chunk_total(psum, nk, r, kl, kRB);
  }
}

// (A, B) maps y -> A y + B; compose(later, earlier) = later o earlier
struct Aff {
  double A, B;
};
__device__ __forceinline__ Aff compose(Aff later, Aff earlier) {
  return Aff{later.A * earlier.A, fma(later.A, earlier.B, later.B)};
}

__device__ __forceinline__ Aff shfl_aff(Aff v, int src) {
  return Aff{__shfl(v.A, src, 64), __shfl(v.B, src, 64)};
}

// Exclusive scan of per-thread affine maps in thread order (reverse = false)
// or in reverse thread order; returns the composition of all maps before
// me.  Within a wavefront by shuffles, then across the block's wavefronts
// through LDS (one barrier); sW holds one map per wavefront.  The
// association differs from a sequential composition by rounding only.
__device__ Aff block_exscan(Aff v, bool reverse, Aff* sW) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const Aff id{1.0, 0.0};
  // inclusive scan in the wavefront: lanes below (forward) or above (reverse)
  // come first
  Aff inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int src = reverse ? lane + off : lane - off;
    const Aff o = shfl_aff(inc, src & 63);
    if (reverse ? (lane + off < 64) : (lane >= off)) inc = compose(inc, o);
  }
  const int prev = reverse ? lane + 1 : lane - 1;
  Aff ex = shfl_aff(inc, prev & 63);
  if (reverse ? lane == 63 : lane == 0) ex = id;
  if (lane == (reverse ? 0 : 63)) sW[w] = inc;
  __syncthreads();
  // the wavefronts before this one, the farthest first
  Aff acc = id;
  if (!reverse) {
    for (int u = 0; u < w; ++u) acc = compose(sW[u], acc);
  } else {
    for (int u = nw - 1; u > w; --u) acc = compose(sW[u], acc);
  }
  __syncthreads();  // sW is reused by the next scan
  return compose(ex, acc);
}

constexpr int kMaxE = 8;  // rows per thread: nr <= kFB * kMaxE
static_assert(kFB * kMaxE == kMaxNr && kRB == 4 && kCC == 32, "grid_fits() limits");

// kCorr: the port's correction pass.  The right-hand side of mode k is
// q0[k] z on the port rows (zero elsewhere) and the solution is subtracted
// from hat (x = y - A0^-1 U z).
template <bool kCorr>
__global__ void __launch_bounds__(kFB) k_tri_scan(int nr, const double* __restrict__ lo,
                                                  const double* __restrict__ inv,
                                                  const double* __restrict__ up,
                                                  double* __restrict__ hat,
                                                  const int32_t* __restrict__ stop, int ip,
                                                  const double* __restrict__ q0,
                                                  const double* __restrict__ zq) {
  if (stop && *stop) return;
  __shared__ Aff sA[kFB / 64];
  const int k = blockIdx.x;
  double* x = hat + (int64_t)k * nr;
  const double* L = lo + (int64_t)k * nr;
  const double* Iv = inv + (int64_t)k * nr;
  const int E = (nr + blockDim.x - 1) / blockDim.x;
  const int i0 = threadIdx.x * E;
  const int i1 = min(i0 + E, nr);
  double y[kMaxE];
  // forward: y_i = -l_i y_{i-1} + d_i (l_0 = 0)
  Aff f{1.0, 0.0};
  const double qk = kCorr ? q0[k] : 0.0;
  for (int q = 0; q < E; ++q) {
    const int i = i0 + q;
    if (i < i1) {
      y[q] = kCorr ? (i >= ip ? qk * zq[i - ip] : 0.0) : x[i];
      const Aff g{i == 0 ? 0.0 : -L[i], y[q]};
      f = compose(g, f);
    }
  }
  const Aff pf = block_exscan(f, false, sA);
  double yp = pf.B;
  for (int q = 0; q < E; ++q) {
    const int i = i0 + q;
    if (i < i1) {
      const double a = (i == 0) ? 0.0 : -L[i];
      yp = fma(a, yp, y[q]);
      y[q] = yp;
    }
  }
  // backward: x_i = (-inv_i e_{i+1}) x_{i+1} + inv_i y_i (e_nr = 0)
  Aff g{1.0, 0.0};
  for (int q = E - 1; q >= 0; --q) {
    const int i = i0 + q;
    if (i < i1) {
      const double c = (i + 1 < nr) ? -Iv[i] * up[i + 1] : 0.0;
      const Aff h{c, Iv[i] * y[q]};
      g = compose(h, g);
    }
  }
  const Aff pb = block_exscan(g, true, sA);
  double xn = pb.B;
  for (int q = E - 1; q >= 0; --q) {
    const int i = i0 + q;
    if (i < i1) {
      const double c = (i + 1 < nr) ? -Iv[i] * up[i + 1] : 0.0;
      xn = fma(c, xn, Iv[i] * y[q]);
      x[i] = kCorr ? x[i] - xn : xn;
    }
  }
}

// The port's coupling, in two launches with deterministic sums:
//   k_port_gather  p = U^T y, the wall cells (i, 0), i >= ip, of the first
//                  solve: y(i, 0) = sum_k q0[k] yhat[k][i].  Block (b, kp)
//                  sums its mode range kp for 256 port rows (loads coalesced
//                  over the rows), into part[kp][r];
//   k_port_solve   z = F p: every block adds the mode parts in order, then
//                  16 rows of z, each split over 16 column parts added in
//                  order (F symmetric: its columns read as rows, coalesced).
constexpr int kPortRows = 16;
constexpr int kPortKParts = 32;  // mode parts at most
inline int port_kparts(int nz) { return std::max(1, std::min(kPortKParts, nz / 16)); }

__global__ void __launch_bounds__(kFB) k_port_gather(int nr, int nz, int ip, int kparts,
                                                    const double* __restrict__ hat,
                                                    const double* __restrict__ q0,
                                                    double* __restrict__ part,
                                                    const int32_t* __restrict__ stop) {
  if (stop && *stop) return;
  const int m = nr - ip;
  const int r = blockIdx.x * kFB + threadIdx.x;
  if (r >= m) return;
  const int kp = blockIdx.y;
  const int k0 = kp * nz / kparts, k1 = (kp + 1) * nz / kparts;
  const double* col = hat + ip + r;
  double acc = 0.0;
  int k = k0;
  for (; k + kUnroll <= k1; k += kUnroll) {
    double v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) v[u] = col[(int64_t)(k + u) * nr];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc = fma(q0[k + u], v[u], acc);
  }
  for (; k < k1; ++k) acc = fma(q0[k], col[(int64_t)k * nr], acc);
  part[(int64_t)kp * m + r] = acc;
}

__global__ void __launch_bounds__(kFB) k_port_solve(int m, int kparts,
                                                   const double* __restrict__ part,
                                                   const double* __restrict__ F,
                                                   double* __restrict__ zq,
                                                   const int32_t* __restrict__ stop) {
  if (stop && *stop) return;
  __shared__ double pv[kFB * kMaxE];
  __shared__ double ps[kFB];
  for (int c = threadIdx.x; c < m; c += kFB) {
    // the parts' loads issued together, then added in order
    double t[kPortKParts];
#pragma unroll
    for (int kp = 0; kp < kPortKParts; ++kp) t[kp] = kp < kparts ? part[(int64_t)kp * m + c] : 0.0;
    double v = t[0];
#pragma unroll
    for (int kp = 1; kp < kPortKParts; ++kp)
      if (kp < kparts) v += t[kp];
    pv[c] = v;
  }
  __syncthreads();
  constexpr int kParts = kFB / kPortRows;
  const int lr = threadIdx.x % kPortRows, q = threadIdx.x / kPortRows;
  const int r = blockIdx.x * kPortRows + lr;
  double acc = 0.0;
  if (r < m) {
    const int c0 = q * m / kParts, c1 = (q + 1) * m / kParts;
    int c = c0;
    for (; c + kUnroll <= c1; c += kUnroll) {
      double f[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) f[u] = F[(int64_t)(c + u) * m + r];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) acc = fma(f[u], pv[c + u], acc);
    }
    for (; c < c1; ++c) acc = fma(F[(int64_t)c * m + r], pv[c], acc);
  }
  ps[threadIdx.x] = acc;
  __syncthreads();
  if (q == 0 && r < m) {
    double v = ps[lr];
    for (int u = 1; u < kParts; ++u) v += ps[u * kPortRows + lr];
    zq[r] = v;
  }
}

__device__ __forceinline__ void block_sum2(double& s0, double& s1, double* red) {
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_down(s0, off, 64);
    s1 += __shfl_down(s1, off, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[2 * w] = s0;
    red[2 * w + 1] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
      a += red[2 * q];
      b += red[2 * q + 1];
    }
    s0 = a;
    s1 = b;
  }
}

__global__ void __launch_bounds__(kFB) k_idct_recover(SolveArgs a, MapP m,
                                                      const double* __restrict__ rh,
                                                      const double* __restrict__ wr,
                                                      const double* __restrict__ wz,
                                                      const double* __restrict__ Q,
                                                      const double* __restrict__ hat,
                                                      PortDev P) {
  if (a.stop && *a.stop) return;
  constexpr int R1 = kRB + 1;  // rows i0 - 1 .. i0 + kRB - 1
  // one r-edge and one z-edge per thread at most
  static_assert(kRB * (kCC + 1) <= kFB, "edges per block");
  extern __shared__ double sh[];
  const int nr = m.nr, nz = m.nz;
  const int i0 = blockIdx.x * kRB;
  const int rows = min(kRB, nr - i0);
  // the block's cells j0 .. j0+nj-1 need x at jlo = j0 - 1 (the r-edge
  // below) .. j0+nj-1
  const int j0 = blockIdx.y * kCC;
  const int nj = min(kCC, nz - j0);
  const int jlo = j0 > 0 ? j0 - 1 : 0;
  const int nx = j0 + nj - jlo;
  // this thread's edges: r-edges j0 .. j0+nj-1 of the rows (and the
  // top-wall edge nz in the last chunk), z-edges j0 .. j0+nj-1 of the rows;
  // their inputs are loaded first, so that the loads are in flight during
  // the transform
  const int ne = nj + (j0 + nj == nz ? 1 : 0);
  const int t = threadIdx.x;
  const bool has_r = t < rows * ne, has_z = t < rows * nj;
  const int rr = has_r ? t / ne : 0, jr = j0 + (t - rr * ne), ir = i0 + rr;
  const int rz = has_z ? t / nj : 0, jz = j0 + (t - rz * nj), iz = i0 + rz;
  const int64_t gr = (int64_t)ir * (nz + 1) + jr, gz = (int64_t)iz * nz + jz;
  double r_u0 = 0.0, r_I = 0.0, r_old = 0.0, z_u0 = 0.0, z_I = 0.0, z_old = 0.0, z_h0 = 0.0;
  if (has_r) {
    r_u0 = a.ur0[gr];
    r_I = a.Ir[gr];
    if (a.part) r_old = a.ur_old[gr];
  }
  if (has_z) {
    z_u0 = a.uz0[gz];
    z_I = a.Iz[gz];
    z_h0 = a.h0[gz];
    if (a.part) z_old = a.uz_old[gz];
  }
  DenseTask dt;
  dense_pre(Q, nz, nz, jlo, nx, dt);
  double* hs = sh;                 // hat of the R1 rows, [r][k]
  double* xs = sh + R1 * nz;       // x of the R1 rows, [r][j - jlo]; row r is i0 - 1 + r
  double* psum = xs + R1 * (kCC + 1);
  __shared__ double red[2 * (kFB / 64)];
  for (int e = threadIdx.x; e < R1 * nz; e += blockDim.x) {
    const int k = e / R1, r = e - k * R1, i = i0 - 1 + r;
    hs[r * nz + k] = (i >= 0 && i < nr) ? hat[(int64_t)k * nr + i] : 0.0;
  }
  __syncthreads();
  dense_run<R1>(Q, nz, hs, nz, jlo, nx, psum, dt);
  for (int e = threadIdx.x; e < R1 * nx; e += blockDim.x) {
    const int r = e / nx, c = e - r * nx;
    xs[e] = chunk_total(psum, nx, r, c, R1);
  }
  __syncthreads();
  const double hdt = 0.5 * m.dt;
  const double two_pi = 2.0 * kPi;
  const double vnext = a.gapv ? a.gapv[0] : a.vnext;
  const double dphi = port_dphi(P);
  double s0 = 0.0, s1 = 0.0;
  if (has_r) {
    const int i = ir, j = jr;
    const int64_t g = gr;
    const double* xr = xs + (rr + 1) * nx - jlo;  // xr[j] = x[i][j]
    double v;
    if (j == 0 && P.ip > 0 && i >= P.ip) {
      // port edge: its change from h^{n+1/2} of the wall cell
      const double M = two_pi * rh[i];
      const double du = P.pc[kPortG * nr + i] *
                        (-M * xr[0] + M * P.hb[i] + P.pc[kPortA * nr + i] * dphi - r_I);
      v = r_u0 + du;
      if (a.part) {
        const double w = 0.5 * wr[i];
        const double d = v - r_old;
        s0 += w * d * d;
        s1 += w * v * v;
      }
    } else if (j == 0) {
      v = (P.ip == 0 && i == nr - 1) ? vnext : 0.0;
    } else if (j == nz) {
      v = 0.0;
    } else {
      const double w = wr[i];
      const double K = -two_pi * rh[i] * (xr[j] - xr[j - 1]);
      const double uh = r_u0 + (K - r_I) * (hdt / w);
      v = 2.0 * uh - r_u0;
      if (a.part) {
        const double d = v - r_old;
        s0 += w * d * d;
        s1 += w * v * v;
      }
    }
    a.ur1[g] = v;
    if (a.ur_h) {
      const double hv = 0.5 * (r_u0 + v);
      a.ur_h[g] = hv;
      if (a.ur_hf) a.ur_hf[g] = float(hv);
    }
    if (a.Ir_clr) a.Ir_clr[g] = 0.0;
  }
  // z-edges of the rows (and the PEC row nr, owned by the blocks of row nr - 1)
  if (has_z) {
    const int i = iz, j = jz;
    const int64_t g = gz;
    const double* xr = xs + (rz + 1) * nx - jlo;
    const double* xm = xs + rz * nx - jlo;
    const double w = wz[i];
    const double ri = two_pi * rh[i];
    const double rm = (i > 0) ? two_pi * rh[i - 1] : 0.0;
    const double K = ri * xr[j] - rm * xm[j];
    const double uh = z_u0 + (K - z_I) * (hdt / w);
    const double v = 2.0 * uh - z_u0;
    if (a.part) {
      const double d = v - z_old;
      s0 += w * d * d;
      s1 += w * v * v;
    }
    a.uz1[g] = v;
    if (a.uz_h) {
      const double hv = 0.5 * (z_u0 + v);
      a.uz_h[g] = hv;
      if (a.uz_hf) a.uz_hf[g] = float(hv);
    }
    if (a.Iz_clr) a.Iz_clr[g] = 0.0;
    a.h1[g] = 2.0 * xr[j] - z_h0;
    if (i == nr - 1) {
      const int64_t ew = (int64_t)nr * nz + j;
      a.uz1[ew] = 0.0;
      if (a.uz_h) {
        const double hv = 0.5 * a.uz0[ew];
        a.uz_h[ew] = hv;
        if (a.uz_hf) a.uz_hf[ew] = float(hv);
      }
      if (a.Iz_clr) a.Iz_clr[ew] = 0.0;
    }
  }
  if (a.part) {
    block_sum2(s0, s1, red);
    if (threadIdx.x == 0) {
      const int b = blockIdx.y * gridDim.x + blockIdx.x;
      a.part[2 * b] = s0;
      a.part[2 * b + 1] = s1;
    }
  }
}

// Electrostatic model (Sec. 2.2, Eq. (8)), charge-conserving update form:
// L dphi = -dt div I on the free nodes (i < nr, 0 < j < nz), with the
// plate potential's step dv on the powered plate below (bottom nodes
// i < nr) and zero on the grounded top, side wall and corner.  L is
// W_r (x) I + diag(wz) (x) T_z (finite integration, weights eps A*/l), so
// the same three-kernel scheme solves it with the DST-I over the nz - 1 free
// rows in place of the DCT.
//
// rhs[i][j-1] = -dt (div I)(i, j) (+ wz_i dv next to the plate), then
// hat[k][i] = sum_j S[j][k] rhs[i][j].
__global__ void __launch_bounds__(kFB) k_es_rhs_dst(MapP m, const double* __restrict__ wz,
                                                    const double* __restrict__ Ir,
                                                    const double* __restrict__ Iz, double dv,
                                                    const double* __restrict__ gapv,
                                                    const double* __restrict__ ur0,
                                                    const double* __restrict__ St,
                                                    double* __restrict__ hat,
                                                    const int32_t* __restrict__ stop,
                                                    const double* __restrict__ prof,
                                                    const double* __restrict__ phin) {
  if (stop && *stop) return;
  extern __shared__ double sh[];  // kRB rows of the right-hand side, then the part sums
  const int nr = m.nr, nz = m.nz, nf = nz - 1;
  if (gapv) dv = gapv[0] - (phin ? phin[0] : ur0[(int64_t)(nr - 1) * (nz + 1)]);
  const int i0 = blockIdx.x * kRB;
  const int rows = min(kRB, nr - i0);
  const int k0 = blockIdx.y * kCC;
  const int nk = min(kCC, nf - k0);
  for (int e = threadIdx.x; e < rows * nf; e += blockDim.x) {
    const int r = e / nf, jj = e - r * nf, i = i0 + r, j = jj + 1;
    const double* Irr = Ir + (int64_t)i * (nz + 1);
    const double* Izr = Iz + (int64_t)i * nz;
    double div = Irr[j] + Izr[j] - Izr[j - 1];
    if (i > 0) div -= Irr[j - (nz + 1)];
    double v = -m.dt * div;
    if (j == 1) v += wz[i] * dv * prof[i];  // the powered wall below
    sh[r * nf + jj] = v;
  }
  __syncthreads();
  double* psum = sh + kRB * nf;
  dense_chunk<kRB>(St, nf, sh, nf, k0, nk, psum);
  for (int e = threadIdx.x; e < nk * kRB; e += blockDim.x) {
    const int kl = e / kRB, r = e - kl * kRB;
    if (r < rows) hat[(int64_t)(k0 + kl) * nr + i0 + r] = chunk_total(psum, nk, r, kl, kRB);
  }
}

// The inverse DST of the rows i0 .. i0+kRB (the last may be the grounded
// wall row) over the block's nodes j0 .. j0+nj, then on the block's edges
// u^{n+1} = u^n + dphi(start) - dphi(end), the next half-step field, the
// residual partials, h^{n+1} = 0, and the reset of the consumed currents.
// Edge ownership and partial layout are those of k_idct_recover.
__global__ void __launch_bounds__(kFB) k_es_recover(SolveArgs a, MapP m,
                                                    const double* __restrict__ wr,
                                                    const double* __restrict__ wz,
                                                    const double* __restrict__ S,
                                                    const double* __restrict__ hat, double dv,
                                                    const double* __restrict__ prof) {
  if (a.stop && *a.stop) return;
  constexpr int R1 = kRB + 1;  // rows i0 .. i0 + kRB
  constexpr int XS = kCC + 1;  // node columns j0 .. j0 + nj
  extern __shared__ double sh[];
  const int nr = m.nr, nz = m.nz, nf = nz - 1;
  const double vnext = a.gapv ? a.gapv[0] : a.vnext;
  if (a.gapv) dv = a.gapv[0] - (a.phin ? a.phin[0] : a.ur0[(int64_t)(nr - 1) * (nz + 1)]);
  const int i0 = blockIdx.x * kRB;
  const int rows = min(kRB, nr - i0);
  const int j0 = blockIdx.y * kCC;
  const int nj = min(kCC, nz - j0);
  // free rows among the block's nodes: jf_lo .. jf_hi (never empty: nz >= 2)
  const int jf_lo = j0 > 1 ? j0 : 1;
  const int jf_hi = (j0 + nj < nf) ? j0 + nj : nf;
  const int nc = jf_hi - jf_lo + 1;
  double* hs = sh;            // hat of the R1 rows, [r][k]
  double* xs = sh + R1 * nf;  // dphi of the R1 rows, [r][j - j0]
  double* psum = xs + R1 * XS;
  __shared__ double red[2 * (kFB / 64)];
  for (int e = threadIdx.x; e < R1 * nf; e += blockDim.x) {
    const int k = e / R1, r = e - k * R1, i = i0 + r;
    hs[r * nf + k] = (i < nr) ? hat[(int64_t)k * nr + i] : 0.0;
  }
  __syncthreads();
  dense_chunk<R1>(S, nf, hs, nf, jf_lo - 1, nc, psum);
  for (int e = threadIdx.x; e < R1 * (nj + 1); e += blockDim.x) {
    const int r = e / (nj + 1), jn = e - r * (nj + 1), j = j0 + jn, i = i0 + r;
    double x;
    if (i >= nr || j == nz)
      x = 0.0;  // grounded wall row, top plate (and the corners)
    else if (j == 0)
      x = dv * prof[i];  // the powered wall (electrode and port mouth)
    else
      x = chunk_total(psum, nc, r, j - jf_lo, R1);
    xs[r * XS + jn] = x;
  }
  __syncthreads();
  double s0 = 0.0, s1 = 0.0;
  const int ne = nj + (j0 + nj == nz ? 1 : 0);
  for (int e = threadIdx.x; e < rows * ne; e += blockDim.x) {
    const int r = e / ne, jn = e - r * ne, j = j0 + jn, i = i0 + r;
    const int64_t g = (int64_t)i * (nz + 1) + j;
    double v;
    if (j == 0 && m.ip > 0 && i >= m.ip) {
      // port edge: the profile's drop, on the half cell above the wall
      v = a.ur0[g] + (xs[r * XS + jn] - xs[(r + 1) * XS + jn]);
      if (a.part) {
        const double w = 0.5 * wr[i];
        const double d = v - a.ur_old[g];
        s0 += w * d * d;
        s1 += w * v * v;
      }
    } else if (j == 0) {
      v = (m.ip == 0 && i == nr - 1) ? vnext : 0.0;
    } else if (j == nz) {
      v = 0.0;
    } else {
      v = a.ur0[g] + (xs[r * XS + jn] - xs[(r + 1) * XS + jn]);
      if (a.part) {
        const double w = wr[i];
        const double d = v - a.ur_old[g];
        s0 += w * d * d;
        s1 += w * v * v;
      }
    }
    a.ur1[g] = v;
    if (a.ur_h) {
      const double hv = 0.5 * (a.ur0[g] + v);
      a.ur_h[g] = hv;
      if (a.ur_hf) a.ur_hf[g] = float(hv);
    }
    if (a.Ir_clr) a.Ir_clr[g] = 0.0;
  }
  for (int e = threadIdx.x; e < rows * nj; e += blockDim.x) {
    const int r = e / nj, jn = e - r * nj, j = j0 + jn, i = i0 + r;
    const int64_t g = (int64_t)i * nz + j;
    const double v = a.uz0[g] + (xs[r * XS + jn] - xs[r * XS + jn + 1]);
    if (a.part) {
      const double w = wz[i];
      const double d = v - a.uz_old[g];
      s0 += w * d * d;
      s1 += w * v * v;
    }
    a.uz1[g] = v;
    if (a.uz_h) {
      const double hv = 0.5 * (a.uz0[g] + v);
      a.uz_h[g] = hv;
      if (a.uz_hf) a.uz_hf[g] = float(hv);
    }
    if (a.Iz_clr) a.Iz_clr[g] = 0.0;
    a.h1[g] = 0.0;
    if (i == nr - 1) {
      const int64_t ew = (int64_t)nr * nz + j;
      a.uz1[ew] = 0.0;
      if (a.uz_h) {
        const double hv = 0.5 * a.uz0[ew];
        a.uz_h[ew] = hv;
        if (a.uz_hf) a.uz_hf[ew] = float(hv);
      }
      if (a.Iz_clr) a.Iz_clr[ew] = 0.0;
    }
  }
  if (a.part) {
    block_sum2(s0, s1, red);
    if (threadIdx.x == 0) {
      const int b = blockIdx.y * gridDim.x + blockIdx.x;
      a.part[2 * b] = s0;
      a.part[2 * b + 1] = s1;
    }
  }
}

// Clear the per-pass queue counters, one tally set and one wall-charge
// scratch set (thread t of nthreads).
__device__ __forceinline__ void clear_pass_scratch(int64_t t, int64_t nthreads, int32_t* qcount,
                                                   Tally* tally, double* wscr, int64_t wlen) {
  for (int64_t q = t; q < 2 * (int64_t)kQCount; q += nthreads) qcount[q] = 0;
  uint64_t* tw = reinterpret_cast<uint64_t*>(tally);
  const int64_t nw = (int64_t)kSpread * (int64_t)(sizeof(Tally) / sizeof(uint64_t));
  for (int64_t q = t; q < nw; q += nthreads) tw[q] = 0;
  for (int64_t q = t; q < wlen; q += nthreads) wscr[q] = 0.0;
}

// guess u^{n+1,(0)} = 2 u^n - u^{n-1} (walls at t^{n+1}), the half-step field
// of the first push, the wall values of u^n at t^n, and zeroed currents.
__global__ void k_guess_half(MapP m, double* ur, double* uz, const double* ur_prev,
                             const double* uz_prev, double* ur_it, double* uz_it, double* ur_h,
                             double* uz_h, float* ur_hf, float* uz_hf, double* Ir, double* Iz,
                             double vnow, double vnext, int32_t* stop, int32_t* qcount,
                             Tally* tally, double* wscr, int64_t wlen, double* circ) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int nr = m.nr, nz = m.nz;
  const int64_t nur = (int64_t)nr * (nz + 1), nuz = (int64_t)(nr + 1) * nz;
  if (t == 0) {
    stop[0] = 0;
    stop[1] = -1;
    // blocking capacitor with a port: the first potential iterate is the
    // extrapolation 2 phi^n - phi^{n-1}
    if (circ && m.ip > 0) circ[3] = 2.0 * circ[0] - circ[1];
  }
  clear_pass_scratch(t, (int64_t)gridDim.x * blockDim.x, qcount, tally, wscr, wlen);
  if (t < nur) {
    const int i = int(t / (nz + 1)), j = int(t - (int64_t)i * (nz + 1));
    double u0 = ur[t], u1;
    if (j == 0 && m.ip > 0 && i >= m.ip) {
      // port edge: an unknown, extrapolated like the interior edges
      u1 = 2.0 * u0 - ur_prev[t];
    } else if (j == 0 && i == nr - 1 && circ && m.ip == 0) {
      // blocking capacitor: the gap carries the electrode potential; its
      // first iterate is extrapolated like the interior edges
      u1 = 2.0 * u0 - ur_prev[t];
      circ[3] = u1;
    } else if (j == 0 || j == nz) {
      const bool gap = (j == 0 && i == nr - 1 && m.ip == 0);
      u0 = gap ? vnow : 0.0;
      ur[t] = u0;
      u1 = gap ? vnext : 0.0;
    } else {
      u1 = 2.0 * u0 - ur_prev[t];
    }
    ur_it[t] = u1;
    const double h = 0.5 * (u0 + u1);
    ur_h[t] = h;
    if (ur_hf) ur_hf[t] = float(h);
    Ir[t] = 0.0;
  }
  if (t < nuz) {
    const int i = int(t / nz);
    double u0 = uz[t], u1;
    if (i == nr) {
      u0 = 0.0;
      uz[t] = 0.0;
      u1 = 0.0;
    } else {
      u1 = 2.0 * u0 - uz_prev[t];
    }
    uz_it[t] = u1;
    const double h = 0.5 * (u0 + u1);
    uz_h[t] = h;
    if (uz_hf) uz_hf[t] = float(h);
    Iz[t] = 0.0;
  }
}

__global__ void k_half(MapP m, const double* u0r, const double* u0z, const double* u1r,
                       const double* u1z, double* ur_h, double* uz_h, float* ur_hf,
                       float* uz_hf) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t nur = (int64_t)m.nr * (m.nz + 1), nuz = (int64_t)(m.nr + 1) * m.nz;
  if (t < nur) {
    const double h = 0.5 * (u0r[t] + u1r[t]);
    ur_h[t] = h;
    if (ur_hf) ur_hf[t] = float(h);
  }
  if (t < nuz) {
    const double h = 0.5 * (u0z[t] + u1z[t]);
    uz_h[t] = h;
    if (uz_hf) uz_hf[t] = float(h);
  }
}

// partial sums over interior edges of w a^2 (weights eps A*/l): one value per
// block, summed on the host in block order
__global__ void __launch_bounds__(kBlock) k_norm2(MapP m, const double* __restrict__ wr,
                                                  const double* __restrict__ wz,
                                                  const double* __restrict__ ar,
                                                  const double* __restrict__ az,
                                                  double* __restrict__ part) {
  const int nr = m.nr, nz = m.nz;
  const int64_t nur = (int64_t)nr * (nz + 1), nuz = (int64_t)nr * nz;
  double s = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < nur + nuz;
       t += (int64_t)gridDim.x * kBlock) {
    if (t < nur) {
      const int i = int(t / (nz + 1)), j = int(t - (int64_t)i * (nz + 1));
      const bool port = j == 0 && m.ip > 0 && i >= m.ip;  // the half cell above the wall
      if ((j == 0 && !port) || j == nz) continue;
      s += (port ? 0.5 * wr[i] : wr[i]) * ar[t] * ar[t];
    } else {
      const int64_t e = t - nur;
      s += wz[e / nz] * az[e] * az[e];
    }
  }
  __shared__ double r0[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) r0[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) v += r0[q];
    part[blockIdx.x] = v;
  }
}

// partial sums of 2 pi r A_c h^2 (magnetic energy weight)
__global__ void __launch_bounds__(kBlock) k_hsum(MapP m, const double* __restrict__ rh,
                                                 const double* __restrict__ area,
                                                 const double* __restrict__ h,
                                                 double* __restrict__ part) {
  const int nr = m.nr, nz = m.nz;
  double s = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < (int64_t)nr * nz;
       t += (int64_t)gridDim.x * kBlock) {
    const int i = int(t / nz);
    s += 2.0 * kPi * rh[i] * area[i] * h[t] * h[t];
  }
  __shared__ double r0[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) r0[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) v += r0[q];
    part[blockIdx.x] = v;
  }
}

// partial sums over interior edges of ((a + b)/2) I (field-side exchange)
__global__ void __launch_bounds__(kBlock) k_xsum(MapP m, const double* __restrict__ ar,
                                                 const double* __restrict__ az,
                                                 const double* __restrict__ br,
                                                 const double* __restrict__ bz,
                                                 const double* __restrict__ Ir,
                                                 const double* __restrict__ Iz,
                                                 double* __restrict__ part) {
  const int nr = m.nr, nz = m.nz;
  const int64_t nur = (int64_t)nr * (nz + 1), nuz = (int64_t)nr * nz;
  double s = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < nur + nuz;
       t += (int64_t)gridDim.x * kBlock) {
    if (t < nur) {
      const int i = int(t / (nz + 1)), j = int(t - (int64_t)i * (nz + 1));
      if ((j == 0 && !(m.ip > 0 && i >= m.ip)) || j == nz) continue;
      s += 0.5 * (ar[t] + br[t]) * Ir[t];
    } else {
      const int64_t e = t - nur;
      s += 0.5 * (az[e] + bz[e]) * Iz[e];
    }
  }
  __shared__ double r0[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) r0[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) v += r0[q];
    part[blockIdx.x] = v;
  }
}

// Residual of a Picard iterate: r = sqrt(sum w (u1 - u_old)^2 / sum w u1^2)
// over the interior edges, from the per-block partials of the solve: the first
// wavefront sums blocks l, l + 64, ... per lane and then combines the lanes in
// a fixed butterfly order (deterministic).  The other threads clear the pass
// scratch for the next push.
// The blocking capacitor's part of a Picard iteration: the current the
// electrode sent into the domain with this iterate, and the next electrode
// potential from the capacitor charge (Sec. 2.1, Eq. (6)).
struct CircArgs {
  double* circ;  // null: no circuit
  const double *h0, *h1, *Ir, *Iz, *uz0, *uz1, *wz, *rh;
  double dt, cap, vnext_gen, scale;
  int es, nr, nz;
  int ip;  // TEM port: first port edge, 0: the delta gap
};

__global__ void __launch_bounds__(256) k_converge(const double* __restrict__ part, int nparts, int k,
                                                  double tol, int32_t* stop, double* res,
                                                  int32_t* qcount, Tally* tally, double* wscr,
                                                  int64_t wlen, CircArgs ca) {
  if (*stop) return;
  const int t = threadIdx.x;
  if (t >= 64) {
    clear_pass_scratch(t - 64, blockDim.x - 64, qcount, tally, wscr, wlen);
    return;
  }
  double num = 0.0, den = 0.0;
  for (int i = t; i < nparts; i += 64) {
    num += part[2 * i];
    den += part[2 * i + 1];
  }
  for (int off = 32; off > 0; off >>= 1) {
    num += __shfl_xor(num, off, 64);
    den += __shfl_xor(den, off, 64);
  }
  double ie = 0.0;
  if (ca.circ && ca.ip > 0) {
    if (ca.es) {
      // Eq. (6) over the electrode's face r <= r_p: the z-edges of its nodes
      double dq = 0.0, ip = 0.0;
      for (int i = t; i <= ca.ip; i += 64) {
        const int64_t e = (int64_t)i * ca.nz;
        dq += ca.wz[i] * (ca.uz1[e] - ca.uz0[e]);
        ip += ca.Iz[e];
      }
      for (int off = 32; off > 0; off >>= 1) {
        dq += __shfl_xor(dq, off, 64);
        ip += __shfl_xor(ip, off, 64);
      }
      ie = dq / ca.dt + ip;
    } else {
      // the same current by Ampere's law: the loop through the first port cell
      const int64_t gc = (int64_t)ca.ip * ca.nz;
      ie = 2.0 * kPi * ca.rh[ca.ip] * (0.5 * (ca.h0[gc] + ca.h1[gc]));
    }
  } else if (ca.circ) {
    const double ir_gap = ca.Ir[(int64_t)(ca.nr - 1) * (ca.nz + 1)];
    if (ca.es) {
      double dq = 0.0, ip = 0.0;
      for (int i = t; i < ca.nr; i += 64) {
        const int64_t e = (int64_t)i * ca.nz;
        dq += ca.wz[i] * (ca.uz1[e] - ca.uz0[e]);
        ip += ca.Iz[e];
      }
      for (int off = 32; off > 0; off >>= 1) {
        dq += __shfl_xor(dq, off, 64);
        ip += __shfl_xor(ip, off, 64);
      }
      ie = dq / ca.dt + ip + ir_gap;
    } else {
      const int64_t gc = (int64_t)(ca.nr - 1) * ca.nz;
      ie = 2.0 * kPi * ca.rh[ca.nr - 1] * (0.5 * (ca.h0[gc] + ca.h1[gc])) + ir_gap;
    }
  }
  if (t != 0) return;
  double r = den > 0.0 ? sqrt(num / den) : (num > 0.0 ? INFINITY : 0.0);
  if (ca.circ) {
    // the potential this iterate used, the next one, and the circuit's share
    // of the residual (the change against the drive's amplitude)
    const double used = ca.circ[3];
    const double next = ca.vnext_gen - (ca.circ[2] + ca.dt * ie) / ca.cap;
    const double rc = fabs(next - used) / ca.scale;
    if (rc > r) r = rc;
    ca.circ[6 + 2 * (k & 1)] = used;
    ca.circ[7 + 2 * (k & 1)] = ie;
    ca.circ[3] = next;
  }
  if (r != r) r = __longlong_as_double(0x7ff8000000000000ll);  // one quiet NaN
  store_sys(res + k, r);
  if (r <= tol) {
    stop[0] = 1;
    stop[1] = k;  // the iteration that converged
  }
}

// Commit summary: the tally copies summed word by word (lane f adds word f of
// the 64 copies in copy order: independent loads, no cross-lane steps), the
// exchange partials reduced by one wavefront in a fixed butterfly order (both
// deterministic), the drive-gap values, and the sequence number stored last
// after a system-scope fence.
__device__ __forceinline__ double wsum_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int kTallyWords = (int)(sizeof(Tally) / sizeof(uint64_t));
constexpr int kTallyDoubles = 4;  // w_absorbed, w_coll, w_particles, pad lead the record
static_assert(sizeof(Tally) % sizeof(uint64_t) == 0 && kTallyWords <= 64, "one word per lane");
static_assert(offsetof(Tally, n_absorbed) == kTallyDoubles * sizeof(double), "doubles first");

// The TEM port's part of the commit summary: its tables, the line's wall
// field (moved to t^{n+1} when the step is accepted), the wall profile and
// the fields at t^n and of the accepted iterate.
struct PortFin {
  int ip;  // 0: no port
  const double* pc;
  double* hb;
  const double *prof, *ur0, *ur1, *rh, *wr;
  double vnow, vnext;  // the generator at t^n, t^{n+1} (no capacitor)
};

__global__ void __launch_bounds__(64) k_finalize(const Tally* __restrict__ tally,
                                                 const double* __restrict__ xpart,
                                                 const double* __restrict__ hn,
                                                 const double* __restrict__ h1,
                                                 const double* __restrict__ Ir, int nr, int nz,
                                                 const double* __restrict__ uzn,
                                                 const double* __restrict__ uz1,
                                                 const double* __restrict__ Iz,
                                                 const double* __restrict__ wz, int es,
                                                 const double* __restrict__ wall_add,
                                                 double* __restrict__ wall_tot, uint64_t seq,
                                                 StepFinal* out, const int32_t* __restrict__ conv,
                                                 int want_k, double* __restrict__ circ, int cpar,
                                                 double dt, PortFin pf) {
  static_assert(kSpread == 64, "64 tally copies");
  // enqueued ahead of the residual it depends on: only if iteration want_k
  // is the one that converged
  if (conv && conv[1] != want_k) return;
  const int l = threadIdx.x;
  uint64_t iacc = 0;  // this lane's integer tally word
  if (l < kTallyWords) {
    const uint64_t* w = reinterpret_cast<const uint64_t*>(tally) + l;
    uint64_t* dst = reinterpret_cast<uint64_t*>(&out->t) + l;
    if (l < kTallyDoubles) {
      double acc = 0.0;
      for (int c = 0; c < kSpread; ++c) acc += __longlong_as_double((long long)w[c * kTallyWords]);
      *dst = (uint64_t)__double_as_longlong(acc);
    } else {
      for (int c = 0; c < kSpread; ++c) iacc += w[c * kTallyWords];
      *dst = iacc;
    }
  }
  // a commit with an ionisation that did not fit, or a particle beyond the
  // null-collision bound, is not accepted: its wall charge stays out of the
  // totals
  constexpr int kOvf = (int)(offsetof(Tally, n_overflow) / sizeof(uint64_t));
  constexpr int kOver = (int)(offsetof(Tally, n_over_range) / sizeof(uint64_t));
  const uint64_t rejected = __shfl(iacc, kOvf, 64) | __shfl(iacc, kOver, 64);
  double xs = 0.0;
  for (int b = l; b < kRedBlocks; b += 64) xs += xpart[b];
  xs = wsum_d(xs);
  double qp = 0.0, izp = 0.0;
  if (es) {
    // the powered plate's nodes (i, 0), i < nr: their field flux change and
    // the current leaving them
    for (int i = l; i < nr; i += 64) {
      const int64_t e = (int64_t)i * nz;
      qp += wz[i] * (uz1[e] - uzn[e]);
      izp += Iz[e];
    }
    qp = wsum_d(qp);
    izp = wsum_d(izp);
  }
  double port_w = 0.0, port_v = 0.0;
  if (pf.ip > 0) {
    // the electrode potential's step of the accepted iterate (read before
    // the circuit state moves below)
    const double dphi = circ ? circ[6 + 2 * cpar] - circ[0] : pf.vnext - pf.vnow;
    for (int i = pf.ip + l; i < nr; i += 64) port_v += pf.ur1[(int64_t)i * (nz + 1)];
    port_v = wsum_d(port_v);
    if (!es) {
      // H_b^{n+1} from the Mur condition and the accepted edge voltages, and
      // the power through the mouth, M H_b^{n+1/2} u^{n+1/2} per edge; each
      // lane owns its edges' H_b
      for (int i = pf.ip + l; i < nr; i += 64) {
        const int64_t e = (int64_t)i * (nz + 1);
        const double u0 = pf.ur0[e], u1 = pf.ur1[e], h0 = pf.hb[i];
        const double h1 = h0 + (pf.pc[kPortK * nr + i] * dphi - (u1 - u0)) * pf.pc[kPortIEL * nr + i];
        port_w += 2.0 * kPi * pf.rh[i] * (0.5 * (h0 + h1)) * (0.5 * (u0 + u1));
        if (!rejected) pf.hb[i] = h1;
      }
      port_w = dt * wsum_d(port_w);
    } else {
      // the source's charge on the powered wall nodes, weighted by the wall
      // profile: the change of each node's Gauss charge (port edges on their
      // half cells) and the current leaving it
      qp = 0.0;
      izp = 0.0;
      for (int i = l; i <= nr; i += 64) {
        double dg = 0.0, dv = 0.0;
        if (i < nr) {
          const int64_t e = (int64_t)i * nz, f = (int64_t)i * (nz + 1);
          dg += wz[i] * (uz1[e] - uzn[e]);
          dv += Iz[e] + Ir[f];
          if (i >= pf.ip) dg += 0.5 * pf.wr[i] * (pf.ur1[f] - pf.ur0[f]);
        }
        if (i > 0) {
          const int64_t f = (int64_t)(i - 1) * (nz + 1);
          dv -= Ir[f];
          if (i - 1 >= pf.ip) dg -= 0.5 * pf.wr[i - 1] * (pf.ur1[f] - pf.ur0[f]);
        }
        qp += pf.prof[i] * dg;
        izp += pf.prof[i] * dv;
      }
      qp = wsum_d(qp);
      izp = wsum_d(izp);
    }
  }
  if (wall_add && !rejected) {
    // the wall charge of a committing iteration joins the totals (the three
    // wall arrays are contiguous in both)
    const int64_t wlen = 2 * (int64_t)(nr + 1) + nz + 1;
    for (int64_t e = l; e < wlen; e += 64) wall_tot[e] += wall_add[e];
  }
  if (l == 0) {
    out->xs = xs;
    out->h_gap_n = hn[(int64_t)(nr - 1) * nz];
    out->h_gap_1 = h1[(int64_t)(nr - 1) * nz];
    out->ir_gap = Ir[(int64_t)(nr - 1) * (nz + 1)];
    out->qp_delta = qp;
    out->iz_plate = izp;
    out->port_w = port_w;
    out->port_v = port_v;
    if (circ) {
      // the accepted iterate's electrode potential and current; the circuit
      // state moves to t^{n+1} only if the step is accepted
      const double phi = circ[6 + 2 * cpar], ie = circ[7 + 2 * cpar];
      const double q1 = circ[2] + dt * ie;
      out->phi_n = circ[0];
      out->phi_1 = phi;
      out->q_1 = q1;
      out->ie = ie;
      if (!rejected) {
        circ[1] = circ[0];
        circ[0] = phi;
        circ[2] = q1;
      }
    }
  }
  // every lane's stores are ordered before the sequence number
  __threadfence_system();
  __syncthreads();
  if (l == 0) store_sys(&out->seq, seq);
}

// -- JFNK vector kernels (the unknown is [ur | uz]) --------------------------
__device__ __forceinline__ double jf_weight(const MapP& m, const double* __restrict__ wr,
                                            const double* __restrict__ wz, int64_t e) {
  const int64_t nur = (int64_t)m.nr * (m.nz + 1);
  if (e < nur) {
    const int64_t i = e / (m.nz + 1);
    const int64_t j = e - i * (m.nz + 1);
    if (j == 0 && m.ip > 0 && i >= m.ip) return 0.5 * wr[i];  // port edge
    return (j >= 1 && j < m.nz) ? wr[i] : 0.0;
  }
  const int64_t i = (e - nur) / m.nz;
  return i < m.nr ? wz[i] : 0.0;
}

__global__ void k_jf_axpby(int64_t n, double a, const double* __restrict__ x, double b,
                           const double* __restrict__ y, double* __restrict__ z) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    z[e] = a * x[e] + b * y[e];
}

__global__ void k_jf_jv(int64_t nur, int64_t n, const double* __restrict__ v,
                        const double* __restrict__ gr, const double* __restrict__ gz,
                        const double* __restrict__ gx, double eps, double* __restrict__ w) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double g = e < nur ? gr[e] : gz[e - nur];
    w[e] = v[e] - (g - gx[e]) / eps;
  }
}

__global__ void k_jf_sub(int64_t nur, int64_t n, const double* __restrict__ y,
                         const double* __restrict__ gr, const double* __restrict__ gz,
                         double* __restrict__ f, double* __restrict__ gcopy) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double g = e < nur ? gr[e] : gz[e - nur];
    f[e] = y[e] - g;
    if (gcopy) gcopy[e] = g;
  }
}

// one block's share of <w, V_k> for k < K: a fixed grid-stride split and a
// fixed reduction order, so the sums do not depend on timing
template <int KB>
__global__ void __launch_bounds__(256) k_jf_dots(MapP m, const double* __restrict__ wr,
                                                 const double* __restrict__ wz, int64_t n,
                                                 const double* __restrict__ w,
                                                 const double* __restrict__ V, int64_t ldv, int K,
                                                 double* __restrict__ part) {
  __shared__ double red[KB][256 / 64];
  double acc[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) acc[k] = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double ww = jf_weight(m, wr, wz, e) * w[e];
#pragma unroll
    for (int k = 0; k < KB; ++k)
      if (k < K) acc[k] = fma(ww, V[k * ldv + e], acc[k]);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    double v = acc[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[k][wv] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    double v = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) v += red[k][q];
    part[(int64_t)k * gridDim.x + blockIdx.x] = v;
  }
}

__global__ void k_jf_gemv(int64_t n, int K, const double* __restrict__ V, int64_t ldv,
                          JfCoef coef, double alpha, double* __restrict__ y) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double acc = alpha == 0.0 ? 0.0 : alpha * y[e];
    for (int k = 0; k < K; ++k) acc = fma(coef.v[k], V[k * ldv + e], acc);
    y[e] = acc;
  }
}

// field shift of a committed step done by copies: prev <- cur <- next
__global__ void k_shift(int64_t nur, int64_t nuz, int64_t nh, double* ur, double* uz, double* h,
                        double* ur_prev, double* uz_prev, double* h_prev,
                        const double* __restrict__ ur_next, const double* __restrict__ uz_next,
                        const double* __restrict__ h_next) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < nur) {
    ur_prev[t] = ur[t];
    ur[t] = ur_next[t];
  }
  if (t < nuz) {
    uz_prev[t] = uz[t];
    uz[t] = uz_next[t];
  }
  if (t < nh) {
    h_prev[t] = h[t];
    h[t] = h_next[t];
  }
}

__global__ void k_zero_tally(Tally* tally) {
  uint64_t* tw = reinterpret_cast<uint64_t*>(tally);
  const int64_t nw = (int64_t)kSpread * (int64_t)(sizeof(Tally) / sizeof(uint64_t));
  for (int64_t q = threadIdx.x; q < nw; q += blockDim.x) tw[q] = 0;
}

}  // namespace

hipError_t launch_converge(const Ctx& c, int k, double tol, hipStream_t s, const SolveArgs* a) {
  // the solve writes the residual row partials at the start of sol.partial
  if (k < 0 || k >= kMaxIter) return hipErrorInvalidValue;
  // the next iteration (parity k+1) gets a cleared tally set and wall scratch
  const int np = (k + 1) & 1;
  CircArgs ca;
  std::memset(&ca, 0, sizeof(ca));
  if (a && a->gapv) {
    double scale = 0.0;
    for (int q = 0; q < c.g.n_drive && q < 32; ++q) scale += std::fabs(c.g.drive_amp[q]);
    ca.circ = c.circ;
    ca.h0 = a->h0;
    ca.h1 = a->h1;
    ca.Ir = a->Ir;
    ca.Iz = a->Iz;
    ca.uz0 = a->uz0;
    ca.uz1 = a->uz1;
    ca.wz = c.sol.wz;
    ca.dt = c.g.dt;
    ca.cap = c.g.blocking_cap;
    ca.vnext_gen = a->vnext;
    ca.scale = scale > 0.0 ? scale : 1.0;
    ca.rh = c.sol.rh;
    ca.es = c.g.model == ECPIC_MODEL_ES ? 1 : 0;
    ca.nr = c.g.nr;
    ca.nz = c.g.nz;
    ca.ip = c.g.port_i;
  }
  hipLaunchKernelGGL(k_converge, dim3(1), dim3(256), 0, s, c.sol.partial,
                     row_blocks(c.g.nr) * col_blocks(c.g.nz),
                     k, tol, c.stop, c.res_dev, c.qcount, tally_set(c, np),
                     wall_scratch(c, np), wall_len(c), ca);
  return hipGetLastError();
}

hipError_t launch_finalize(const Ctx& c, const Tally* tally, const double* xpart, const double* Ir,
                           const double* Iz, const double* wall_add, uint64_t seq, int guard_k,
                           hipStream_t s, int iter) {
  PortFin pf;
  std::memset(&pf, 0, sizeof(pf));
  if (c.g.port_i > 0) {
    pf.ip = c.g.port_i;
    pf.pc = c.sol.port_pc;
    pf.hb = c.port_hb;
    pf.prof = c.sol.prof;
    pf.ur0 = c.ur;
    pf.ur1 = c.ur_it;
    pf.rh = c.sol.rh;
    pf.wr = c.sol.wr;
    pf.vnow = drive_voltage(c.g, c.t);
    pf.vnext = drive_voltage(c.g, c.t + c.g.dt);
  }
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, tally, xpart, c.h, c.h_it, Ir,
                     c.g.nr, c.g.nz, c.uz, c.uz_it, Iz, c.sol.wz,
                     c.g.model == ECPIC_MODEL_ES ? 1 : 0, wall_add, c.wall_bot, seq, c.fin_dev,
                     guard_k >= 0 ? (const int32_t*)c.stop : nullptr, guard_k,
                     c.g.blocking_cap > 0.0 ? c.circ : nullptr, iter & 1, c.g.dt, pf);
  return hipGetLastError();
}

hipError_t launch_shift(const Ctx& c, hipStream_t s) {
  const int64_t nur = (int64_t)c.g.nr * (c.g.nz + 1), nuz = (int64_t)(c.g.nr + 1) * c.g.nz;
  const int64_t nh = (int64_t)c.g.nr * c.g.nz;
  hipLaunchKernelGGL(k_shift, dim3(nblk(nuz > nur ? nuz : nur)), dim3(kBlock), 0, s, nur, nuz, nh,
                     c.ur, c.uz, c.h, c.ur_prev, c.uz_prev, c.h_prev, c.ur_it, c.uz_it, c.h_it);
  return hipGetLastError();
}

namespace {
int64_t jf_len(const Ctx& c) {
  return (int64_t)c.g.nr * (c.g.nz + 1) + (int64_t)(c.g.nr + 1) * c.g.nz;
}
int jf_grid(int64_t n) { return (int)std::min<int64_t>(nblk(n), 4096); }
}  // namespace

hipError_t launch_jf_axpby(const Ctx& c, double a, const double* x, double b, const double* y,
                           double* z, hipStream_t s) {
  const int64_t n = jf_len(c);
  hipLaunchKernelGGL(k_jf_axpby, dim3(jf_grid(n)), dim3(kBlock), 0, s, n, a, x, b, y, z);
  return hipGetLastError();
}

hipError_t launch_jf_jv(const Ctx& c, const double* v, const double* gr, const double* gz,
                        const double* gx, double e, double* w, hipStream_t s) {
  const int64_t n = jf_len(c), nur = (int64_t)c.g.nr * (c.g.nz + 1);
  hipLaunchKernelGGL(k_jf_jv, dim3(jf_grid(n)), dim3(kBlock), 0, s, nur, n, v, gr, gz, gx, e, w);
  return hipGetLastError();
}

hipError_t launch_jf_sub(const Ctx& c, const double* y, const double* gr, const double* gz,
                         double* f, double* gcopy, hipStream_t s) {
  const int64_t n = jf_len(c), nur = (int64_t)c.g.nr * (c.g.nz + 1);
  hipLaunchKernelGGL(k_jf_sub, dim3(jf_grid(n)), dim3(kBlock), 0, s, nur, n, y, gr, gz, f, gcopy);
  return hipGetLastError();
}

hipError_t launch_jf_dots(const Ctx& c, const double* w, const double* V, int64_t ldv, int K,
                          hipStream_t s) {
  if (K < 1 || K > kMaxKrylov + 1) return hipErrorInvalidValue;
  const int64_t n = jf_len(c);
  if (K <= 4)
    hipLaunchKernelGGL(k_jf_dots<4>, dim3(kJfBlocks), dim3(256), 0, s, c.m, c.sol.wr, c.sol.wz, n,
                       w, V, ldv, K, c.jf_part);
  else if (K <= 16)
    hipLaunchKernelGGL(k_jf_dots<16>, dim3(kJfBlocks), dim3(256), 0, s, c.m, c.sol.wr, c.sol.wz,
                       n, w, V, ldv, K, c.jf_part);
  else
    hipLaunchKernelGGL(k_jf_dots<kMaxKrylov + 1>, dim3(kJfBlocks), dim3(256), 0, s, c.m,
                       c.sol.wr, c.sol.wz, n, w, V, ldv, K, c.jf_part);
  return hipGetLastError();
}

hipError_t launch_jf_gemv(const Ctx& c, int K, const double* V, int64_t ldv, const JfCoef& coef,
                          double alpha, double* y, hipStream_t s) {
  if (K < 0 || K > kMaxKrylov + 1) return hipErrorInvalidValue;
  const int64_t n = jf_len(c);
  hipLaunchKernelGGL(k_jf_gemv, dim3(jf_grid(n)), dim3(kBlock), 0, s, n, K, V, ldv, coef, alpha,
                     y);
  return hipGetLastError();
}

hipError_t launch_zero_tally(const Ctx& c, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_tally, dim3(1), dim3(256), 0, s, c.tally);
  return hipGetLastError();
}

hipError_t launch_guess_half(const Ctx& c, double vnow, double vnext, hipStream_t s) {
  const int64_t n = (int64_t)(c.g.nr + 1) * (c.g.nz + 1);
  hipLaunchKernelGGL(k_guess_half, dim3(nblk(n)), dim3(kBlock), 0, s, c.m, c.ur, c.uz, c.ur_prev,
                     c.uz_prev, c.ur_it, c.uz_it, c.ur_half, c.uz_half, c.ur_half_f, c.uz_half_f,
                     c.Ir, c.Iz, vnow, vnext, c.stop, c.qcount, tally_set(c, 0),
                     wall_scratch(c, 0), wall_len(c), c.g.blocking_cap > 0.0 ? c.circ : nullptr);
  return hipGetLastError();
}

hipError_t launch_half(const Ctx& c, const double* u0r, const double* u0z, const double* u1r,
                       const double* u1z, hipStream_t s) {
  const int64_t n = (int64_t)(c.g.nr + 1) * (c.g.nz + 1);
  hipLaunchKernelGGL(k_half, dim3(nblk(n)), dim3(kBlock), 0, s, c.m, u0r, u0z, u1r, u1z,
                     c.ur_half, c.uz_half, c.ur_half_f, c.uz_half_f);
  return hipGetLastError();
}

hipError_t field_solve(const Ctx& c, const SolveArgs& a, hipStream_t s, double* hat) {
  const int nr = c.g.nr, nz = c.g.nz;
  const SolverDev& S = c.sol;
  if (!hat) hat = S.work1;  // the mode-major transform of the right-hand side
  if (nr > kFB * kMaxE) return hipErrorInvalidValue;
  const int cb = col_blocks(nz);
  // residual partials: two per block of k_idct_recover
  if ((int64_t)row_blocks(nr) * cb > kResParts) return hipErrorInvalidValue;
  if (c.g.model == ECPIC_MODEL_ES) {
    const int nf = nz - 1;
    if (nf < 1) return hipErrorInvalidValue;
    const size_t lds_es_rhs = sizeof(double) * ((size_t)kRB * nf + (size_t)kFB * kRB);
    const size_t lds_es_rec = sizeof(double) * ((size_t)(kRB + 1) * nf + (kRB + 1) * (kCC + 1) +
                                                (size_t)kFB * (kRB + 1));
    if (lds_es_rhs > 65536 || lds_es_rec > 65536) return hipErrorInvalidValue;
    const double dv = a.vnext - a.vnow;
    hipLaunchKernelGGL(k_es_rhs_dst, dim3(row_blocks(nr), col_blocks(nf)), dim3(kFB),
                       lds_es_rhs, s, c.m, S.wz, a.Ir, a.Iz, dv, a.gapv, a.ur0, S.Qt, hat,
                       a.stop, S.prof, a.phin);
    hipLaunchKernelGGL(k_tri_scan<false>, dim3(nf), dim3(kFB), 0, s, nr, S.tri_lo, S.tri_inv,
                       S.tri_up, hat, a.stop, 0, nullptr, nullptr);
    hipLaunchKernelGGL(k_es_recover, dim3(row_blocks(nr), cb), dim3(kFB), lds_es_rec, s, a, c.m,
                       S.wr, S.wz, S.Q, hat, dv, S.prof);
    return hipGetLastError();
  }
  PortDev P;
  std::memset(&P, 0, sizeof(P));
  if (c.g.port_i > 0) {
    P.ip = c.g.port_i;
    P.pc = S.port_pc;
    P.hb = c.port_hb;
    P.vnow = a.vnow;
    P.vnext = a.vnext;
    P.phin = a.phin;
    P.phi1 = a.gapv;
  }
  // part sums: P * R * nc <= kFB * R for nc < kFB (chunks have at most kCC + 1 columns)
  const size_t lds_rhs = sizeof(double) * ((size_t)kRB * nz + (size_t)kFB * kRB);
  const size_t lds_rec = sizeof(double) * ((size_t)(kRB + 1) * nz + (kRB + 1) * (kCC + 1) +
                                           (size_t)kFB * (kRB + 1));
  if (lds_rhs > 65536 || lds_rec > 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rhs_dct, dim3(row_blocks(nr), cb), dim3(kFB), lds_rhs, s, c.m, S.rh, S.wr,
                     S.wz, S.area, c.g.mu, a.ur0, a.uz0, a.h0, a.Ir, a.Iz, a.vhalf, a.gapv, S.Qt,
                     hat, a.stop, P);
  hipLaunchKernelGGL(k_tri_scan<false>, dim3(nz), dim3(kFB), 0, s, nr, S.tri_lo, S.tri_inv,
                     S.tri_up, hat, a.stop, 0, nullptr, nullptr);
  if (P.ip > 0) {
    // the port's diagonal on the wall cells, by the Woodbury identity:
    // z = F U^T y, then hat -= A0^-1 U z (a second scan on q0[k] z)
    const int mp = nr - P.ip, kparts = port_kparts(nz);
    double* part = S.port_z + mp;  // [kparts][m] after z
    hipLaunchKernelGGL(k_port_gather, dim3((mp + kFB - 1) / kFB, kparts), dim3(kFB), 0, s, nr,
                       nz, P.ip, kparts, hat, S.port_q0, part, a.stop);
    hipLaunchKernelGGL(k_port_solve, dim3((mp + kPortRows - 1) / kPortRows), dim3(kFB), 0, s, mp,
                       kparts, part, S.port_F, S.port_z, a.stop);
    hipLaunchKernelGGL(k_tri_scan<true>, dim3(nz), dim3(kFB), 0, s, nr, S.tri_lo, S.tri_inv,
                       S.tri_up, hat, a.stop, P.ip, S.port_q0, S.port_z);
  }
  hipLaunchKernelGGL(k_idct_recover, dim3(row_blocks(nr), cb), dim3(kFB), lds_rec, s, a, c.m,
                     S.rh, S.wr, S.wz, S.Q, hat, P);
  return hipGetLastError();
}

hipError_t launch_field_energy(const Ctx& c, const double* ur, const double* uz, const double* h,
                               double* part, hipStream_t s) {
  // part[0..kRed) = sum w u^2 partials, part[kRed..2 kRed) = sum 2 pi r A_c h^2
  hipLaunchKernelGGL(k_norm2, dim3(kRedBlocks), dim3(kBlock), 0, s, c.m, c.sol.wr, c.sol.wz, ur,
                     uz, part);
  hipLaunchKernelGGL(k_hsum, dim3(kRedBlocks), dim3(kBlock), 0, s, c.m, c.sol.rh, c.sol.area, h,
                     part + kRedBlocks);
  return hipGetLastError();
}

hipError_t launch_exchange(const Ctx& c, const double* ar, const double* az, const double* br,
                           const double* bz, const double* Ir, const double* Iz, double* part,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_xsum, dim3(kRedBlocks), dim3(kBlock), 0, s, c.m, ar, az, br, bz, Ir, Iz,
                     part);
  return hipGetLastError();
}

}  // namespace ecpic
