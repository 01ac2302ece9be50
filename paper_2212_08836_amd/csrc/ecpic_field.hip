// ecpic_field.hip -- Crank-Nicolson update of the TM fields (Eq. (2) of
// Sec. 2.1 with mid-point centring) with H_theta as the unknown.
//
// Eliminating the interior edge voltages leaves an SPD system for
// h^{n+1/2} that is T (x) I + G (x) N, where N is the Neumann second
// difference in z (the PEC r-edges of the z walls decouple the end cells).
// It is solved by an orthonormal DCT-II in z (dense FP64 product with a
// precomputed matrix), one tridiagonal (Thomas) solve in r per z-mode, and the
// inverse DCT; then the edge voltages are recovered from Ampere's law.
#include "ecpic_internal.h"

namespace ecpic {

namespace {

constexpr double kPi = 3.14159265358979323846;

inline int64_t nblk(int64_t n) { return (n + kBlock - 1) / kBlock; }

// rhs[i][j] = 2 pi r_{i+1/2} (2 mu A_c / dt h0 + circulation of u0 - D^-1 I)
// with the half-step drive value on the gap edge and zero on other walls.
__global__ void k_rhs(MapP m, const double* __restrict__ rh, const double* __restrict__ wr,
                      const double* __restrict__ wz, const double* __restrict__ area, double mu,
                      const double* __restrict__ ur0, const double* __restrict__ uz0,
                      const double* __restrict__ h0, const double* __restrict__ Ir,
                      const double* __restrict__ Iz, double vhalf, double* __restrict__ rhs) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int nr = m.nr, nz = m.nz;
  if (c >= (int64_t)nr * nz) return;
  const int i = int(c / nz), j = int(c - (int64_t)i * nz);
  const double hdt = 0.5 * m.dt;
  auto tr = [&](int jj) -> double {
    if (jj == 0) return (i == nr - 1) ? vhalf : 0.0;
    if (jj == nz) return 0.0;
    const int64_t e = (int64_t)i * (nz + 1) + jj;
    return ur0[e] - hdt * Ir[e] / wr[i];
  };
  auto tz = [&](int ii) -> double {
    if (ii == nr) return 0.0;
    const int64_t e = (int64_t)ii * nz + j;
    return uz0[e] - hdt * Iz[e] / wz[ii];
  };
  const double circ = tz(i + 1) - tz(i) - tr(j + 1) + tr(j);
  const double mi = 2.0 * kPi * rh[i];
  rhs[c] = mi * (2.0 * mu * area[i] / m.dt * h0[c] + circ);
}

// C[M][N] = A[M][K] B[K][N], FP64, 64x64 tiles, 16 x 16 threads x (4 x 4)
constexpr int GT = 64, GK = 16;
__global__ void __launch_bounds__(256) k_gemm(const double* __restrict__ A,
                                              const double* __restrict__ B, double* __restrict__ C,
                                              int M, int N, int K) {
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int row0 = blockIdx.y * GT, col0 = blockIdx.x * GT;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = threadIdx.x + q * 256;
      const int r = idx / GK, cc = idx % GK;
      As[cc][r] = (row0 + r < M && k0 + cc < K) ? A[(int64_t)(row0 + r) * K + k0 + cc] : 0.0;
      const int rb = idx / GT, cb = idx % GT;
      Bs[rb][cb] = (k0 + rb < K && col0 + cb < N) ? B[(int64_t)(k0 + rb) * N + col0 + cb] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][ty + 16 * q];
        b[q] = Bs[kk][tx + 16 * q];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = fma(a[p], b[q], acc[p][q]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = row0 + ty + 16 * p, cc = col0 + tx + 16 * q;
      if (r < M && cc < N) C[(int64_t)r * N + cc] = acc[p][q];
    }
}

// per z-mode k: (T + lambda_k G) x = d over i, factors precomputed
__global__ void k_thomas(int nr, int nz, const double* __restrict__ lo,
                         const double* __restrict__ inv, const double* __restrict__ up,
                         double* __restrict__ x) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nz) return;
  const double* L = lo + (int64_t)k * nr;
  const double* Iv = inv + (int64_t)k * nr;
  double y = x[k];
  for (int i = 1; i < nr; ++i) {
    const double d = x[(int64_t)i * nz + k] - L[i] * y;
    x[(int64_t)i * nz + k] = d;
    y = d;
  }
  double xn = x[(int64_t)(nr - 1) * nz + k] * Iv[nr - 1];
  x[(int64_t)(nr - 1) * nz + k] = xn;
  for (int i = nr - 2; i >= 0; --i) {
    const double v = (x[(int64_t)i * nz + k] - up[i + 1] * xn) * Iv[i];
    x[(int64_t)i * nz + k] = v;
    xn = v;
  }
}

// u^{1/2} = u0 + D^-1 (K h^{1/2} - I) on interior edges; n+1 values; walls.
__global__ void k_recover(MapP m, const double* __restrict__ rh, const double* __restrict__ wr,
                          const double* __restrict__ wz, const double* __restrict__ ur0,
                          const double* __restrict__ uz0, const double* __restrict__ h0,
                          const double* __restrict__ Ir, const double* __restrict__ Iz,
                          const double* __restrict__ x, double vnext, double* __restrict__ ur1,
                          double* __restrict__ uz1, double* __restrict__ h1) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int nr = m.nr, nz = m.nz;
  const double hdt = 0.5 * m.dt;
  const int64_t nur = (int64_t)nr * (nz + 1), nuz = (int64_t)(nr + 1) * nz, nh = (int64_t)nr * nz;
  if (t < nur) {
    const int i = int(t / (nz + 1)), j = int(t - (int64_t)i * (nz + 1));
    double v;
    if (j == 0) {
      v = (i == nr - 1) ? vnext : 0.0;
    } else if (j == nz) {
      v = 0.0;
    } else {
      const double K = -2.0 * kPi * rh[i] * (x[(int64_t)i * nz + j] - x[(int64_t)i * nz + j - 1]);
      const double uh = ur0[t] + hdt * (K - Ir[t]) / wr[i];
      v = 2.0 * uh - ur0[t];
    }
    ur1[t] = v;
  }
  if (t < nuz) {
    const int i = int(t / nz), j = int(t - (int64_t)i * nz);
    double v = 0.0;
    if (i < nr) {
      double K = 2.0 * kPi * rh[i] * x[(int64_t)i * nz + j];
      if (i > 0) K -= 2.0 * kPi * rh[i - 1] * x[(int64_t)(i - 1) * nz + j];
      const double uh = uz0[t] + hdt * (K - Iz[t]) / wz[i];
      v = 2.0 * uh - uz0[t];
    }
    uz1[t] = v;
  }
  if (t < nh) h1[t] = 2.0 * x[t] - h0[t];
}

// guess u^{n+1,(0)} = 2 u^n - u^{n-1} (walls at t^{n+1}), the half-step field
// of the first push, and the wall values of u^n at t^n.
__global__ void k_guess_half(MapP m, double* ur, double* uz, const double* ur_prev,
                             const double* uz_prev, double* ur_it, double* uz_it, double* ur_h,
                             double* uz_h, float* ur_hf, float* uz_hf, double vnow, double vnext) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int nr = m.nr, nz = m.nz;
  const int64_t nur = (int64_t)nr * (nz + 1), nuz = (int64_t)(nr + 1) * nz;
  if (t < nur) {
    const int i = int(t / (nz + 1)), j = int(t - (int64_t)i * (nz + 1));
    double u0 = ur[t], u1;
    if (j == 0 || j == nz) {
      const bool gap = (j == 0 && i == nr - 1);
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

constexpr int kRedBlocks = 256;

// partial sums over interior edges: [0] sum w (a-b)^2, [1] sum w a^2
// (b may be null: then [0] = sum w a^2 too)
__global__ void __launch_bounds__(kBlock) k_norm2(MapP m, const double* __restrict__ wr,
                                                  const double* __restrict__ wz,
                                                  const double* __restrict__ ar,
                                                  const double* __restrict__ az,
                                                  const double* __restrict__ br,
                                                  const double* __restrict__ bz,
                                                  double* __restrict__ part) {
  const int nr = m.nr, nz = m.nz;
  const int64_t nur = (int64_t)nr * (nz + 1), nuz = (int64_t)nr * nz;  // interior z-edges i<nr
  double s0 = 0.0, s1 = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < nur + nuz;
       t += (int64_t)gridDim.x * kBlock) {
    double w, a, b;
    if (t < nur) {
      const int i = int(t / (nz + 1)), j = int(t - (int64_t)i * (nz + 1));
      if (j == 0 || j == nz) continue;
      w = wr[i];
      a = ar[t];
      b = br ? br[t] : 0.0;
    } else {
      const int64_t e = t - nur;
      const int i = int(e / nz);
      w = wz[i];
      a = az[e];
      b = bz ? bz[e] : 0.0;
    }
    s0 += w * (a - b) * (a - b);
    s1 += w * a * a;
  }
  __shared__ double r0[kBlock / 64], r1[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_down(s0, off, 64);
    s1 += __shfl_down(s1, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    r0[threadIdx.x >> 6] = s0;
    r1[threadIdx.x >> 6] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) {
      a += r0[q];
      b += r1[q];
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

// sum w_c h^2 with w_c = 2 pi r A_c (magnetic energy weight), and
// sum over interior edges of ((a+b)/2) I (field-side exchange)
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
    double a = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) a += r0[q];
    part[blockIdx.x] = a;
  }
}

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
      (void)i;
      if (j == 0 || j == nz) continue;
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
    double a = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) a += r0[q];
    part[blockIdx.x] = a;
  }
}

// fixed-order final sum of `cnt` interleaved partial vectors of width w
__global__ void k_final(const double* part, int nb, int w, double* out) {
  if (threadIdx.x >= w) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(int64_t)b * w + threadIdx.x];
  out[threadIdx.x] = s;
}

}  // namespace

hipError_t launch_guess_half(const Ctx& c, double vnow, double vnext, hipStream_t s) {
  const int64_t n = (int64_t)(c.g.nr + 1) * (c.g.nz + 1);
  hipLaunchKernelGGL(k_guess_half, dim3(nblk(n)), dim3(kBlock), 0, s, c.m, c.ur, c.uz, c.ur_prev,
                     c.uz_prev, c.ur_it, c.uz_it, c.ur_half, c.uz_half, c.ur_half_f, c.uz_half_f,
                     vnow, vnext);
  return hipGetLastError();
}

hipError_t launch_half(const Ctx& c, const double* u0r, const double* u0z, const double* u1r,
                       const double* u1z, hipStream_t s) {
  const int64_t n = (int64_t)(c.g.nr + 1) * (c.g.nz + 1);
  hipLaunchKernelGGL(k_half, dim3(nblk(n)), dim3(kBlock), 0, s, c.m, u0r, u0z, u1r, u1z,
                     c.ur_half, c.uz_half, c.ur_half_f, c.uz_half_f);
  return hipGetLastError();
}

hipError_t field_solve(const Ctx& c, const double* ur0, const double* uz0, const double* h0,
                       const double* Ir, const double* Iz, double vhalf, double vnext,
                       double* ur1, double* uz1, double* h1, hipStream_t s) {
  const int nr = c.g.nr, nz = c.g.nz;
  const SolverDev& S = c.sol;
  const int64_t nh = (int64_t)nr * nz;
  hipLaunchKernelGGL(k_rhs, dim3(nblk(nh)), dim3(kBlock), 0, s, c.m, S.rh, S.wr, S.wz, S.area,
                     c.g.mu, ur0, uz0, h0, Ir, Iz, vhalf, S.work0);
  const dim3 gg((nz + GT - 1) / GT, (nr + GT - 1) / GT);
  hipLaunchKernelGGL(k_gemm, gg, dim3(256), 0, s, S.work0, S.Qt, S.work1, nr, nz, nz);
  hipLaunchKernelGGL(k_thomas, dim3((nz + 63) / 64), dim3(64), 0, s, nr, nz, S.tri_lo, S.tri_inv,
                     S.tri_up, S.work1);
  hipLaunchKernelGGL(k_gemm, gg, dim3(256), 0, s, S.work1, S.Q, S.work0, nr, nz, nz);
  const int64_t n = (int64_t)(nr + 1) * (nz + 1);
  hipLaunchKernelGGL(k_recover, dim3(nblk(n)), dim3(kBlock), 0, s, c.m, S.rh, S.wr, S.wz, ur0, uz0,
                     h0, Ir, Iz, S.work0, vnext, ur1, uz1, h1);
  return hipGetLastError();
}

hipError_t launch_resid(const Ctx& c, const double* anr, const double* anz, const double* bor,
                        const double* boz, double* out2, hipStream_t s) {
  hipLaunchKernelGGL(k_norm2, dim3(kRedBlocks), dim3(kBlock), 0, s, c.m, c.sol.wr, c.sol.wz, anr,
                     anz, bor, boz, c.sol.partial);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(64), 0, s, c.sol.partial, kRedBlocks, 2, out2);
  return hipGetLastError();
}

hipError_t launch_field_energy(const Ctx& c, const double* ur, const double* uz, const double* h,
                               double* out2, hipStream_t s) {
  // out2[0] = sum w u^2 (2 W_E / 1), out2[1] = sum 2 pi r A_c h^2 (2 W_B / mu)
  hipLaunchKernelGGL(k_norm2, dim3(kRedBlocks), dim3(kBlock), 0, s, c.m, c.sol.wr, c.sol.wz, ur,
                     uz, nullptr, nullptr, c.sol.partial);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(64), 0, s, c.sol.partial, kRedBlocks, 2, out2);
  hipLaunchKernelGGL(k_hsum, dim3(kRedBlocks), dim3(kBlock), 0, s, c.m, c.sol.rh, c.sol.area, h,
                     c.sol.partial + 2 * kRedBlocks);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(64), 0, s, c.sol.partial + 2 * kRedBlocks, kRedBlocks,
                     1, out2 + 1);
  return hipGetLastError();
}

hipError_t launch_exchange(const Ctx& c, const double* ar, const double* az, const double* br,
                           const double* bz, const double* Ir, const double* Iz, double* out1,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_xsum, dim3(kRedBlocks), dim3(kBlock), 0, s, c.m, ar, az, br, bz, Ir, Iz,
                     c.sol.partial + 3 * kRedBlocks);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(64), 0, s, c.sol.partial + 3 * kRedBlocks, kRedBlocks,
                     1, out1);
  return hipGetLastError();
}

}  // namespace ecpic
