// ecpic_nn.hip -- learned initial guess of the Picard iteration (the
// iteration of Sec. 2.1 that solves the coupled field/orbit system): a
// four-layer 3x3 convolutional network, 6 -> 32 -> 32 -> 32 -> 2 channels,
// ReLU between layers, on the (nr+1) x (nz+1) canvas of the staggered field
// arrays, predicting the correction of the extrapolated guess 2u^n - u^{n-1}
// of u^{n+1}.  BF16 weights and activations on the matrix cores
// (v_mfma_f32_32x32x16_bf16), FP32 accumulation.
//
// Layout: activations channels-last, [image][i][j][channel], 32 channels
// (8 for the 6-channel input).  Each wavefront computes a 32 (output
// channels) x 32 (positions along j of one row) tile: the A operand is the
// weight slice [tap][cout][cin], the B operand the input channels of 32
// neighbouring positions, K = 9 taps x cin.  The input gradient is the same
// product with the taps flipped and the channel roles swapped; the weight
// gradient is a product over positions, reduced per wavefront and then over
// wavefronts in a fixed order.
//
// The products use gfx950's double-K BF16 instruction
// (v_mfma_f32_32x32x16_bf16): lane l holds A[l % 32][8 (l / 32) + 0..7] and
// B[8 (l / 32) + 0..7][l % 32], and D in the layout of the 32x32x8 form.  A
// 32-channel tap takes two of them; the 8-channel input layer puts two taps
// in one (each half of the wavefront takes one tap's 8 channels).
#include <cmath>
#include <cstring>
#include <vector>

#include "ecpic_internal.h"

namespace ecpic {
namespace {

constexpr int kNL = 4;
constexpr int kCin[kNL] = {6, 32, 32, 32};
constexpr int kCout[kNL] = {32, 32, 32, 2};
constexpr int kCinP[kNL] = {8, 32, 32, 32};
constexpr int kCH = 32;          // channels of a hidden activation / MFMA M
constexpr int kWaves = 4;        // wavefronts per block
constexpr int kGradWaves = 256;  // wavefronts of the weight-gradient pass

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// 8 BF16 values (16 bytes, 16-byte aligned) as an MFMA operand
__device__ __forceinline__ v8bf ld8(const uint16_t* p) {
  return __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(p));
}
__device__ __forceinline__ v8bf zero8() { return __builtin_bit_cast(v8bf, make_uint4(0u, 0u, 0u, 0u)); }
__device__ __forceinline__ v8bf pack8(const uint16_t (&v)[8]) {
  uint4 u;
  u.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
  u.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
  u.z = (uint32_t)v[4] | ((uint32_t)v[5] << 16);
  u.w = (uint32_t)v[6] | ((uint32_t)v[7] << 16);
  return __builtin_bit_cast(v8bf, u);
}

__host__ __device__ inline int64_t layer_w_off(int l) {
  int64_t o = 0;
  for (int k = 0; k < l; ++k) o += (int64_t)kCout[k] * kCin[k] * 9 + kCout[k];
  return o;
}

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// MODE 0: hidden layer, bias + ReLU, BF16 out [pos][32]
// MODE 1: last layer, bias, FP32 out [image][2][H][W]
// MODE 2: input gradient, times the ReLU mask of `gate` ([pos][32] > 0),
//         BF16 out [pos][32]
template <int CINP, int MODE>
__global__ void __launch_bounds__(64 * kWaves)
    k_conv(const uint16_t* __restrict__ in, const uint16_t* __restrict__ A,
           const float* __restrict__ bias, int nimg, int H, int W, void* out,
           const uint16_t* __restrict__ gate) {
  const int lane = threadIdx.x & 63;
  const int64_t tw = (W + 31) / 32;
  const int64_t tile = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (tile >= (int64_t)nimg * H * tw) return;
  const int jt = (int)(tile % tw);
  const int64_t ni = tile / tw;
  const int i = (int)(ni % H);
  const int n = (int)(ni / H);
  const int col = lane & 31, kh = lane >> 5, kq = kh * 4;
  const int j = jt * 32 + col;
  v16f acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  if (CINP == 32) {
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int ii = i + tap / 3 - 1, jj = j + tap % 3 - 1;
      const bool ok = j < W && ii >= 0 && ii < H && jj >= 0 && jj < W;
      const uint16_t* src = in + (((int64_t)n * H + ii) * W + jj) * CINP + 8 * kh;
      const uint16_t* wa = A + ((int64_t)tap * kCH + col) * CINP + 8 * kh;
#pragma unroll
      for (int c16 = 0; c16 < 2; ++c16) {
        const v8bf a = ld8(wa + 16 * c16);
        const v8bf b = ok ? ld8(src + 16 * c16) : zero8();
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    }
  } else {
    // 8 channels: taps 2p (lanes 0-31) and 2p + 1 (lanes 32-63) per product
#pragma unroll
    for (int p = 0; p < 5; ++p) {
      const int tap = 2 * p + kh;
      const int ii = i + tap / 3 - 1, jj = j + tap % 3 - 1;
      const bool ok = tap < 9 && j < W && ii >= 0 && ii < H && jj >= 0 && jj < W;
      const v8bf a = tap < 9 ? ld8(A + ((int64_t)tap * kCH + col) * CINP) : zero8();
      const v8bf b = ok ? ld8(in + (((int64_t)n * H + ii) * W + jj) * CINP) : zero8();
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
  }
  if (j >= W) return;
  const int64_t pos = ((int64_t)n * H + i) * W + j;
  if (MODE == 1) {
    if (lane < 32) {
      float* y = static_cast<float*>(out);
      for (int v = 0; v < 2; ++v)
        y[(((int64_t)n * 2 + v) * H + i) * W + j] = acc[v] + bias[v];
    }
    return;
  }
  uint16_t* o = static_cast<uint16_t*>(out) + pos * kCH;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int ch = 8 * g + kq;
    uint16_t r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float x = acc[4 * g + q];
      if (MODE == 0) {
        x += bias[ch + q];
        x = x > 0.f ? x : 0.f;
      } else {
        x = bf2f(gate[pos * kCH + ch + q]) > 0.f ? x : 0.f;
      }
      r[q] = f2bf(x);
    }
    uint2 pk;
    pk.x = (uint32_t)r[0] | ((uint32_t)r[1] << 16);
    pk.y = (uint32_t)r[2] | ((uint32_t)r[3] << 16);
    *reinterpret_cast<uint2*>(o + ch) = pk;
  }
}

// Weight gradient partials: wavefront w accumulates, over its tiles of 32
// positions, dW[tap][cout][cin] = sum_pos g[pos][cout] x[pos + off(tap)][cin]
// (A = g^T, B = x) and db[cout] = sum_pos g[pos][cout].
template <int CINP>
__global__ void __launch_bounds__(64 * kWaves)
    k_wgrad(const uint16_t* __restrict__ x, const uint16_t* __restrict__ g, int nimg, int H,
            int W, float* __restrict__ part, float* __restrict__ part_db) {
  const int lane = threadIdx.x & 63;
  const int wv = blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int64_t tw = (W + 31) / 32;
  const int64_t ntile = (int64_t)nimg * H * tw;
  const int row = lane & 31, kh = lane >> 5, kq = kh * 4;
  v16f acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[t][v] = 0.f;
  float db = 0.f;
  for (int64_t tile = wv; tile < ntile; tile += kGradWaves) {
    const int jt = (int)(tile % tw);
    const int64_t ni = tile / tw;
    const int i = (int)(ni % H);
    const int n = (int)(ni / H);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      // the 8 positions of this lane's K slice: j = jt*32 + ks*16 + 8*kh + 0..7
      uint16_t av[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int j = jt * 32 + ks * 16 + 8 * kh + q;
        uint16_t gv = 0;
        if (j < W) gv = g[(((int64_t)n * H + i) * W + j) * kCH + row];
        av[q] = gv;
        db += bf2f(gv);
      }
      const v8bf a = pack8(av);
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int ii = i + tap / 3 - 1;
        uint16_t bv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int j = jt * 32 + ks * 16 + 8 * kh + q;
          const int jj = j + tap % 3 - 1;
          uint16_t xv = 0;
          if (row < CINP && j < W && ii >= 0 && ii < H && jj >= 0 && jj < W)
            xv = x[(((int64_t)n * H + ii) * W + jj) * CINP + row];
          bv[q] = xv;
        }
        acc[tap] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, pack8(bv), acc[tap], 0, 0, 0);
      }
    }
  }
  // D[row = cout][col = cin]: lane holds column lane%32, rows 8(v/4)+4(lane/32)+v%4
  float* p = part + (int64_t)wv * 9 * kCH * kCH;
#pragma unroll
  for (int tap = 0; tap < 9; ++tap)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int co = 8 * (v / 4) + kq + (v % 4);
      p[((int64_t)tap * kCH + co) * kCH + row] = acc[tap][v];
    }
  db += __shfl_xor(db, 32, 64);
  if (lane < 32) part_db[(int64_t)wv * kCH + row] = db;
}

// dw (canonical [cout][cin][3][3] then b[cout]) = sum of the partials in
// wavefront order
__global__ void k_wgrad_reduce(const float* __restrict__ part, const float* __restrict__ part_db,
                               int cin, int cout, float* __restrict__ dw) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int nw = cout * cin * 9;
  if (e < nw) {
    const int co = e / (cin * 9), ci = (e / 9) % cin, tap = e % 9;
    float s = 0.f;
    for (int w = 0; w < kGradWaves; ++w) s += part[(((int64_t)w * 9 + tap) * kCH + co) * kCH + ci];
    dw[e] = s;
  } else if (e < nw + cout) {
    const int co = e - nw;
    float s = 0.f;
    for (int w = 0; w < kGradWaves; ++w) s += part_db[(int64_t)w * kCH + co];
    dw[e] = s;
  }
}

// BF16 operand layouts of layer l from the FP32 canonical weights:
// fwd[tap][cout(32)][cinp] and, for the input gradient, bwd[tap'][cin(32)][cout(32)]
// with tap' the flipped tap; bias padded to 32 (FP32).
__global__ void k_prep_layer(const float* __restrict__ w, int cin, int cout, int cinp,
                             uint16_t* __restrict__ fwd, uint16_t* __restrict__ bwd,
                             float* __restrict__ bias) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int nf = 9 * kCH * cinp;
  if (e < nf) {
    const int tap = e / (kCH * cinp), co = (e / cinp) % kCH, ci = e % cinp;
    const float v = (co < cout && ci < cin) ? w[((int64_t)co * cin + ci) * 9 + tap] : 0.f;
    fwd[e] = f2bf(v);
  }
  if (bwd && e < 9 * kCH * kCH) {
    const int tp = e / (kCH * kCH), ci = (e / kCH) % kCH, co = e % kCH;
    const int tap = 8 - tp;  // (2 - p, 2 - q)
    const float v = (co < cout && ci < cin) ? w[((int64_t)co * cin + ci) * 9 + tap] : 0.f;
    bwd[e] = f2bf(v);
  }
  if (e < kCH) bias[e] = e < cout ? w[(int64_t)cout * cin * 9 + e] : 0.f;
}

// [image][6][H][W] BF16 -> [image][i][j][8] BF16 (channels 6, 7 zero)
__global__ void k_pack_input(const uint16_t* __restrict__ x, int nimg, int H, int W,
                             uint16_t* __restrict__ act0) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t hw = (int64_t)H * W;
  if (pos >= nimg * hw) return;
  const int64_t n = pos / hw, r = pos % hw;
  uint16_t v[8];
  for (int c = 0; c < 6; ++c) v[c] = x[(n * 6 + c) * hw + r];
  v[6] = v[7] = 0;
  uint4 pk;
  pk.x = v[0] | ((uint32_t)v[1] << 16);
  pk.y = v[2] | ((uint32_t)v[3] << 16);
  pk.z = v[4] | ((uint32_t)v[5] << 16);
  pk.w = 0;
  *reinterpret_cast<uint4*>(act0 + pos * 8) = pk;
}

// output positions that are unknowns of the guess: interior r-edges
// (i < nr, 0 < j < nz) and z-edges off the PEC wall (i < nr, j < nz)
__device__ __forceinline__ bool out_valid(int c, int i, int j, int nr, int nz) {
  return c == 0 ? (i < nr && j > 0 && j < nz) : (i < nr && j < nz);
}

// mean squared error over the valid outputs; gradient [pos][32] BF16
__global__ void __launch_bounds__(256)
    k_mse(const float* __restrict__ y, const float* __restrict__ t, int nimg, int nr, int nz,
          double inv_count, uint16_t* __restrict__ gout, double* __restrict__ part) {
  const int H = nr + 1, W = nz + 1;
  const int64_t hw = (int64_t)H * W;
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (pos < nimg * hw) {
    const int64_t n = pos / hw, r = pos % hw;
    const int i = (int)(r / W), j = (int)(r % W);
    uint16_t gv[2];
    for (int c = 0; c < 2; ++c) {
      const int64_t e = (n * 2 + c) * hw + r;
      const double d = out_valid(c, i, j, nr, nz) ? double(y[e]) - double(t[e]) : 0.0;
      l += d * d;
      gv[c] = f2bf(float(2.0 * d * inv_count));
    }
    uint4* o = reinterpret_cast<uint4*>(gout + pos * kCH);
    o[0] = make_uint4(gv[0] | ((uint32_t)gv[1] << 16), 0u, 0u, 0u);
    o[1] = make_uint4(0u, 0u, 0u, 0u);
    o[2] = make_uint4(0u, 0u, 0u, 0u);
    o[3] = make_uint4(0u, 0u, 0u, 0u);
  }
  __shared__ double red[4];
  for (int off = 32; off > 0; off >>= 1) l += __shfl_down(l, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t n, float lr, float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = 0.9f * m[e] + 0.1f * gi;
  const float vi = 0.999f * v[e] + 0.001f * gi * gi;
  m[e] = mi;
  v[e] = vi;
  w[e] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
}

// The network's input for the current step, normalised, from the FP64
// fields: channels u_r, u_z, h at t^n and their change since t^{n-1}.
__global__ void k_canvas(MapP m, const double* __restrict__ ur, const double* __restrict__ uz,
                         const double* __restrict__ h, const double* __restrict__ urp,
                         const double* __restrict__ uzp, const double* __restrict__ hp,
                         float s0, float s1, float s2, float s3, float s4, float s5,
                         uint16_t* __restrict__ act0) {
  const int nr = m.nr, nz = m.nz, W = nz + 1;
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= (int64_t)(nr + 1) * W) return;
  const int i = (int)(pos / W), j = (int)(pos % W);
  float v[6] = {0, 0, 0, 0, 0, 0};
  if (i < nr) {
    const int64_t e = (int64_t)i * (nz + 1) + j;
    v[0] = float(ur[e]) / s0;
    v[3] = float(ur[e] - urp[e]) / s3;
  }
  if (j < nz) {
    const int64_t e = (int64_t)i * nz + j;
    v[1] = float(uz[e]) / s1;
    v[4] = float(uz[e] - uzp[e]) / s4;
  }
  if (i < nr && j < nz) {
    const int64_t e = (int64_t)i * nz + j;
    v[2] = float(h[e]) / s2;
    v[5] = float(h[e] - hp[e]) / s5;
  }
  uint4 pk;
  pk.x = f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
  pk.y = f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
  pk.z = f2bf(v[4]) | ((uint32_t)f2bf(v[5]) << 16);
  pk.w = 0;
  *reinterpret_cast<uint4*>(act0 + pos * 8) = pk;
}

// guess += scaled network output on the unknown edges; half-step field
__global__ void k_apply_guess(MapP m, const float* __restrict__ y, float o0, float o1,
                              const double* __restrict__ ur, const double* __restrict__ uz,
                              double* __restrict__ ur_it, double* __restrict__ uz_it,
                              double* __restrict__ ur_h, double* __restrict__ uz_h,
                              float* __restrict__ ur_hf, float* __restrict__ uz_hf) {
  const int nr = m.nr, nz = m.nz, W = nz + 1;
  const int64_t hw = (int64_t)(nr + 1) * W;
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= hw) return;
  const int i = (int)(pos / W), j = (int)(pos % W);
  if (out_valid(0, i, j, nr, nz)) {
    const int64_t e = (int64_t)i * (nz + 1) + j;
    const double g = ur_it[e] + double(o0) * double(y[pos]);
    ur_it[e] = g;
    const double hv = 0.5 * (ur[e] + g);
    ur_h[e] = hv;
    if (ur_hf) ur_hf[e] = float(hv);
  }
  if (out_valid(1, i, j, nr, nz)) {
    const int64_t e = (int64_t)i * nz + j;
    const double g = uz_it[e] + double(o1) * double(y[hw + pos]);
    uz_it[e] = g;
    const double hv = 0.5 * (uz[e] + g);
    uz_h[e] = hv;
    if (uz_hf) uz_hf[e] = float(hv);
  }
}

inline int64_t nblk256(int64_t n) { return (n + 255) / 256; }

struct Ws {
  uint16_t* act[kNL];   // layer inputs
  float* y;             // output [img][2][H][W]
  uint16_t *ga, *gb;    // gradient ping-pong [pos][32]
  uint16_t* fwd[kNL];
  uint16_t* bwd[kNL];
  float* bias[kNL];
  float* part;          // kGradWaves * 9 * 32 * 32
  float* part_db;       // kGradWaves * 32
  double* loss_part;
};

// carve a workspace for nimg images out of the buffer (buf, bytes), growing
// the allocation when needed (grow = false: a buffer carved from the
// context's device region, which must already be large enough); with
// need_only, only the size is computed (into *need_only)
ecpic_status workspace(const Ctx& c, int nimg, Ws& w, void*& buf, size_t& bytes,
                       bool grow = true, size_t* need_only = nullptr) {
  const int64_t P = (int64_t)nimg * (c.g.nr + 1) * (c.g.nz + 1);
  size_t need = 0;
  auto take = [&](size_t bytes) {
    const size_t o = need;
    need += (bytes + 255) & ~(size_t)255;
    return o;
  };
  size_t o_act[kNL], o_fwd[kNL], o_bwd[kNL], o_bias[kNL];
  for (int l = 0; l < kNL; ++l) o_act[l] = take(sizeof(uint16_t) * P * kCinP[l]);
  const size_t o_y = take(sizeof(float) * P * 2);
  const size_t o_ga = take(sizeof(uint16_t) * P * kCH);
  const size_t o_gb = take(sizeof(uint16_t) * P * kCH);
  for (int l = 0; l < kNL; ++l) {
    o_fwd[l] = take(sizeof(uint16_t) * 9 * kCH * kCinP[l]);
    o_bwd[l] = take(sizeof(uint16_t) * 9 * kCH * kCH);
    o_bias[l] = take(sizeof(float) * kCH);
  }
  const size_t o_part = take(sizeof(float) * (size_t)kGradWaves * 9 * kCH * kCH);
  const size_t o_pdb = take(sizeof(float) * (size_t)kGradWaves * kCH);
  const size_t o_loss = take(sizeof(double) * (size_t)nblk256(P));
  if (need_only) {
    *need_only = need;
    return ECPIC_OK;
  }
  if (need > bytes) {
    if (!grow) return ECPIC_ENOMEM;
    if (buf) {
      if (hipStreamSynchronize(c.stream) != hipSuccess) return ECPIC_EHIP;
      (void)hipFree(buf);
      buf = nullptr;
      bytes = 0;
    }
    if (hipMalloc(&buf, need) != hipSuccess) return ECPIC_ENOMEM;
    bytes = need;
  }
  char* b = static_cast<char*>(buf);
  for (int l = 0; l < kNL; ++l) {
    w.act[l] = reinterpret_cast<uint16_t*>(b + o_act[l]);
    w.fwd[l] = reinterpret_cast<uint16_t*>(b + o_fwd[l]);
    w.bwd[l] = reinterpret_cast<uint16_t*>(b + o_bwd[l]);
    w.bias[l] = reinterpret_cast<float*>(b + o_bias[l]);
  }
  w.y = reinterpret_cast<float*>(b + o_y);
  w.ga = reinterpret_cast<uint16_t*>(b + o_ga);
  w.gb = reinterpret_cast<uint16_t*>(b + o_gb);
  w.part = reinterpret_cast<float*>(b + o_part);
  w.part_db = reinterpret_cast<float*>(b + o_pdb);
  w.loss_part = reinterpret_cast<double*>(b + o_loss);
  return ECPIC_OK;
}

hipError_t prep_weights(const float* wts, const Ws& w, hipStream_t s) {
  for (int l = 0; l < kNL; ++l) {
    const int n = 9 * kCH * (kCinP[l] > kCH ? kCinP[l] : kCH);
    hipLaunchKernelGGL(k_prep_layer, dim3(nblk256(n)), dim3(256), 0, s, wts + layer_w_off(l),
                       kCin[l], kCout[l], kCinP[l], w.fwd[l], l > 0 ? w.bwd[l] : nullptr,
                       w.bias[l]);
  }
  return hipGetLastError();
}

// forward through all layers from w.act[0]; output in w.y (FP32)
hipError_t forward(const Ws& w, int nimg, int H, int W, hipStream_t s) {
  const int64_t tiles = (int64_t)nimg * H * ((W + 31) / 32);
  const dim3 grid((unsigned)((tiles + kWaves - 1) / kWaves)), blk(64 * kWaves);
  hipLaunchKernelGGL((k_conv<8, 0>), grid, blk, 0, s, w.act[0], w.fwd[0], w.bias[0], nimg, H, W,
                     (void*)w.act[1], nullptr);
  hipLaunchKernelGGL((k_conv<32, 0>), grid, blk, 0, s, w.act[1], w.fwd[1], w.bias[1], nimg, H, W,
                     (void*)w.act[2], nullptr);
  hipLaunchKernelGGL((k_conv<32, 0>), grid, blk, 0, s, w.act[2], w.fwd[2], w.bias[2], nimg, H, W,
                     (void*)w.act[3], nullptr);
  hipLaunchKernelGGL((k_conv<32, 1>), grid, blk, 0, s, w.act[3], w.fwd[3], w.bias[3], nimg, H, W,
                     (void*)w.y, nullptr);
  return hipGetLastError();
}

ecpic_status check_ctx(ecpic_ctx* x) { return x ? ECPIC_OK : ECPIC_EINVAL; }

}  // namespace

size_t nn_guess_ws_bytes(const Ctx& c) {
  Ws w;
  void* buf = nullptr;
  size_t bytes = 0, need = 0;
  (void)workspace(c, 1, w, buf, bytes, false, &need);
  return need;
}

// Learned guess inside ecpic_step: called after the extrapolated guess.
ecpic_status nn_guess(Ctx& c, bool* used) {
  *used = false;
  if (!c.nn_ready) return ECPIC_OK;
  // the guess buffer: its BF16 weights were prepared by ecpic_nn_set_weights
  Ws w;
  ecpic_status rc = workspace(c, 1, w, c.nn_gws, c.nn_gws_bytes, false);
  if (rc != ECPIC_OK) return rc;
  const int H = c.g.nr + 1, W = c.g.nz + 1;
  const int64_t hw = (int64_t)H * W;
  const float* s = c.nn_norm;
  hipLaunchKernelGGL(k_canvas, dim3(nblk256(hw)), dim3(256), 0, c.stream, c.m, c.ur, c.uz, c.h,
                     c.ur_prev, c.uz_prev, c.h_prev, s[0], s[1], s[2], s[3], s[4], s[5],
                     w.act[0]);
  HIPCHK(hipGetLastError());
  HIPCHK(forward(w, 1, H, W, c.stream));
  hipLaunchKernelGGL(k_apply_guess, dim3(nblk256(hw)), dim3(256), 0, c.stream, c.m, w.y, s[6],
                     s[7], c.ur, c.uz, c.ur_it, c.uz_it, c.ur_half, c.uz_half, c.ur_half_f,
                     c.uz_half_f);
  HIPCHK(hipGetLastError());
  *used = true;
  return ECPIC_OK;
}

}  // namespace ecpic

using namespace ecpic;

extern "C" {

int64_t ecpic_nn_param_count(void) { return layer_w_off(kNL); }

ecpic_status ecpic_nn_set_weights(ecpic_ctx* x, const float* w, const float* norm) {
  if (check_ctx(x) != ECPIC_OK) return ECPIC_EINVAL;
  Ctx& c = x->c;
  if (!w) {
    c.nn_ready = false;
    return ECPIC_OK;
  }
  if (!norm) return ECPIC_EINVAL;
  for (int k = 0; k < 8; ++k)
    if (!(norm[k] > 0.f) || !std::isfinite(norm[k])) return ECPIC_EINVAL;
  {
    const ecpic_status r0 = materialise(c);
    if (r0 != ECPIC_OK) return r0;
  }
  const int64_t n = layer_w_off(kNL);
  HIPCHK(hipMemcpyAsync(c.nn_w, w, sizeof(float) * n, hipMemcpyDeviceToDevice, c.stream));
  Ws g;
  ecpic_status rc = workspace(c, 1, g, c.nn_gws, c.nn_gws_bytes, false);
  if (rc != ECPIC_OK) return rc;
  HIPCHK(prep_weights(c.nn_w, g, c.stream));
  std::memcpy(c.nn_norm, norm, 8 * sizeof(float));
  c.nn_ready = true;
  return ECPIC_OK;
}

ecpic_status ecpic_nn_forward(ecpic_ctx* x, const float* wts, const uint16_t* in, float* y,
                              int32_t batch) {
  if (check_ctx(x) != ECPIC_OK || !wts || !in || !y || batch < 1) return ECPIC_EINVAL;
  Ctx& c = x->c;
  {
    const ecpic_status r0 = materialise(c);
    if (r0 != ECPIC_OK) return r0;
  }
  Ws w;
  ecpic_status rc = workspace(c, batch, w, c.nn_ws, c.nn_ws_bytes);
  if (rc != ECPIC_OK) return rc;
  const int H = c.g.nr + 1, W = c.g.nz + 1;
  const int64_t P = (int64_t)batch * H * W;
  HIPCHK(prep_weights(wts, w, c.stream));
  hipLaunchKernelGGL(k_pack_input, dim3(nblk256(P)), dim3(256), 0, c.stream, in, batch, H, W,
                     w.act[0]);
  HIPCHK(forward(w, batch, H, W, c.stream));
  HIPCHK(hipMemcpyAsync(y, w.y, sizeof(float) * P * 2, hipMemcpyDeviceToDevice, c.stream));
  return ECPIC_OK;
}

ecpic_status ecpic_nn_grad(ecpic_ctx* x, const float* wts, const uint16_t* in, const float* t,
                           int32_t batch, float* dw, float* loss) {
  if (check_ctx(x) != ECPIC_OK || !wts || !in || !t || !dw || batch < 1) return ECPIC_EINVAL;
  Ctx& c = x->c;
  {
    const ecpic_status r0 = materialise(c);
    if (r0 != ECPIC_OK) return r0;
  }
  Ws w;
  ecpic_status rc = workspace(c, batch, w, c.nn_ws, c.nn_ws_bytes);
  if (rc != ECPIC_OK) return rc;
  const int nr = c.g.nr, nz = c.g.nz, H = nr + 1, W = nz + 1;
  const int64_t P = (int64_t)batch * H * W;
  HIPCHK(prep_weights(wts, w, c.stream));
  hipLaunchKernelGGL(k_pack_input, dim3(nblk256(P)), dim3(256), 0, c.stream, in, batch, H, W,
                     w.act[0]);
  HIPCHK(forward(w, batch, H, W, c.stream));
  const double count = (double)batch * ((double)nr * (nz - 1) + (double)nr * nz);
  const int64_t nb = nblk256(P);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, c.stream, w.y, t, batch, nr, nz,
                     1.0 / count, w.ga, w.loss_part);
  HIPCHK(hipGetLastError());
  const int64_t tiles = (int64_t)batch * H * ((W + 31) / 32);
  const dim3 grid((unsigned)((tiles + kWaves - 1) / kWaves)), blk(64 * kWaves);
  const dim3 ggrid(kGradWaves / kWaves);
  uint16_t* g = w.ga;
  uint16_t* gn = w.gb;
  for (int l = kNL - 1; l >= 0; --l) {
    if (kCinP[l] == 8)
      hipLaunchKernelGGL((k_wgrad<8>), ggrid, blk, 0, c.stream, w.act[l], g, batch, H, W, w.part,
                         w.part_db);
    else
      hipLaunchKernelGGL((k_wgrad<32>), ggrid, blk, 0, c.stream, w.act[l], g, batch, H, W,
                         w.part, w.part_db);
    const int nw = kCout[l] * kCin[l] * 9 + kCout[l];
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nblk256(nw)), dim3(256), 0, c.stream, w.part,
                       w.part_db, kCin[l], kCout[l], dw + layer_w_off(l));
    if (l > 0) {
      hipLaunchKernelGGL((k_conv<32, 2>), grid, blk, 0, c.stream, g, w.bwd[l], w.bias[l], batch,
                         H, W, (void*)gn, w.act[l]);
      std::swap(g, gn);
    }
  }
  HIPCHK(hipGetLastError());
  std::vector<double> lp((size_t)nb);
  HIPCHK(hipMemcpyAsync(lp.data(), w.loss_part, sizeof(double) * nb, hipMemcpyDeviceToHost,
                        c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  double s = 0.0;
  for (double v : lp) s += v;
  if (loss) *loss = float(s / count);
  return ECPIC_OK;
}

ecpic_status ecpic_nn_adam(ecpic_ctx* x, float* w, float* m, float* v, const float* dw, float lr,
                           int32_t t) {
  if (check_ctx(x) != ECPIC_OK || !w || !m || !v || !dw || t < 1 || !(lr > 0.f))
    return ECPIC_EINVAL;
  Ctx& c = x->c;
  const int64_t n = layer_w_off(kNL);
  const float c1 = float(1.0 / (1.0 - std::pow(0.9, t)));
  const float c2 = float(1.0 / (1.0 - std::pow(0.999, t)));
  hipLaunchKernelGGL(k_adam, dim3(nblk256(n)), dim3(256), 0, c.stream, w, m, v, dw, n, lr, c1, c2);
  HIPCHK(hipGetLastError());
  return ECPIC_OK;
}

}  // extern "C"
