// ecpic_sort.hip -- counting sort of particles by cell (the fine sorting the
// paper's GPU parallelisation builds on, Sec. 2.1) with compaction of
// absorbed particles, an exclusive scan, and particle-side reductions.
#include <climits>

#include "ecpic_internal.h"

namespace ecpic {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanChunk = kScanThreads * kScanPer;  // 1024 elements per block

// block-local exclusive scan; block totals to part[blockIdx.x]
__global__ void __launch_bounds__(kScanThreads) k_scan_local(int32_t* data, int64_t n,
                                                             int32_t* part) {
  __shared__ int32_t wsum[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
  int32_t v[kScanPer];
  int32_t s = 0;
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    v[q] = (base + q < n) ? data[base + q] : 0;
    s += v[q];
  }
  // inclusive scan of the per-thread sums across the wavefront
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t inc = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t o = __shfl_up(inc, off, 64);
    if (lane >= off) inc += o;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int32_t wbase = 0;
  for (int q = 0; q < w; ++q) wbase += wsum[q];
  int32_t run = wbase + inc - s;
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    if (base + q < n) data[base + q] = run;
    run += v[q];
  }
  if (threadIdx.x == kScanThreads - 1) part[blockIdx.x] = run;
}

// single block: exclusive scan of the block totals; grand total to data[n]
__global__ void __launch_bounds__(1024) k_scan_part(int32_t* part, int64_t nb, int32_t* data,
                                                    int64_t n) {
  __shared__ int32_t wsum[16];
  __shared__ int32_t carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
    const int64_t k = b0 + threadIdx.x;
    const int32_t x = (k < nb) ? part[k] : 0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t inc = x;
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t o = __shfl_up(inc, off, 64);
      if (lane >= off) inc += o;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int32_t wbase = 0;
    for (int q = 0; q < w; ++q) wbase += wsum[q];
    const int32_t carry = carry_s;
    if (k < nb) part[k] = carry + wbase + inc - x;
    __syncthreads();
    if (threadIdx.x == 1023) carry_s = carry + wbase + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) data[n] = carry_s;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_add(int32_t* data, int64_t n,
                                                           const int32_t* part) {
  const int32_t add = part[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  for (int q = threadIdx.x; q < kScanChunk; q += kScanThreads) {
    if (base + q < n) data[base + q] += add;
  }
}

__device__ __forceinline__ int cell_key(const MapP& m, const SpecDev& s, int64_t k, bool mixed) {
  if (mixed) return s.cell[k];
  const double xi = s.xi[k];
  if (!(xi >= 0.0)) return -1;
  int i = int(floor(xi)), j = int(floor(s.eta[k]));
  i = i < 0 ? 0 : (i > m.nr - 1 ? m.nr - 1 : i);
  j = j < 0 ? 0 : (j > m.nz - 1 ? m.nz - 1 : j);
  return i * m.nz + j;
}

// Block-local counting (histogram and scatter).  A block takes kSortChunk
// consecutive slots; between sorts they hold the particles of a few
// neighbouring cells that have drifted a few cells in z or a row in r, so
// their cells fall in a window of sort_window(nz) = 2 nz + 256 cells from
// lo = max(lowest cell, first slot's cell - nz - 32): counts and ranks are
// taken with LDS atomics there and the global counters see one atomic per
// occupied window cell and block.  Slots of cells outside the window (born
// elsewhere and appended, or before the first sort) use global atomics of
// their own.  Dead slots (cell < 0) are dropped.
constexpr int kSortThreads = 256;
constexpr int kSortPer = 8;
constexpr int kSortChunk = kSortThreads * kSortPer;  // 2048 slots per block
__host__ __device__ inline int sort_window(int nz) { return 2 * nz + 256; }
static_assert(2 * kMaxNz + 256 <= 4096, "window counters within 16 KB of LDS");

// the cells of a thread's slots (k = block start + q * kSortThreads + tid)
// and the window's first cell; every thread of the block calls it
__device__ __forceinline__ int sort_keys(const MapP& m, const SpecDev& s, int64_t n, bool mixed,
                                         int64_t k0, int key[kSortPer]) {
  __shared__ int wmin[kSortThreads / 64];
  __shared__ int cref;
  int mn = INT_MAX;
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const int64_t k = k0 + (int64_t)q * kSortThreads + threadIdx.x;
    key[q] = (k < n) ? cell_key(m, s, k, mixed) : -1;
    if (key[q] >= 0) mn = min(mn, key[q]);
  }
  if (threadIdx.x == 0) cref = key[0];
  for (int off = 32; off > 0; off >>= 1) mn = min(mn, __shfl_xor(mn, off, 64));
  if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = mn;
  __syncthreads();
#pragma unroll
  for (int w = 0; w < kSortThreads / 64; ++w) mn = min(mn, wmin[w]);
  int lo = mn == INT_MAX ? 0 : mn;
  if (cref >= 0) lo = max(lo, cref - m.nz - 32);
  return lo;
}

// per-cell counts of one species (hist zeroed beforehand)
__global__ void __launch_bounds__(kSortThreads)
    k_hist(MapP m, SpecDev s, int64_t n, int mixed, int32_t* hist) {
  extern __shared__ int32_t cnt[];
  const int W = sort_window(m.nz);
  for (int e = threadIdx.x; e < W; e += kSortThreads) cnt[e] = 0;
  int key[kSortPer];
  const int lo = sort_keys(m, s, n, mixed != 0, (int64_t)blockIdx.x * kSortChunk, key);
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const int c = key[q], e = c - lo;
    if (c < 0) continue;
    if (e >= 0 && e < W)
      atomicAdd(&cnt[e], 1);
    else
      atomicAdd(&hist[c], 1);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < W; e += kSortThreads) {
    const int v = cnt[e];
    if (v) atomicAdd(&hist[lo + e], v);
  }
}

// Where a block's slots go: for a window slot, its place lp in the block's
// cell-ordered stage (its cell's offset in the block + its rank) and, for
// the writer of stage place t, the destination dest[t]; for the others the
// global slot claimed on their own.
struct SortPlan {
  int key[kSortPer];   // cell, -1 for a dead slot
  int pos[kSortPer];   // lp (>= 0), or -(global slot) - 1
  int dest[kSortPer];  // destination of stage place q * kSortThreads + tid
  int lo, W, ns;       // window and number of staged slots
};

// One column moved through the stage: loads of the block's slots (one per
// thread and round, coalesced), staged in cell order, then stored by the
// writers to consecutive destinations of each cell.  CELL: the mixed
// layout's cell column, whose values are the keys themselves.
template <typename E, bool CELL = false>
__device__ __forceinline__ void scatter_col(const SortPlan& P, int64_t k0, const E* __restrict__ src,
                                            E* __restrict__ dst, E* stage) {
  E v[kSortPer];
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const int64_t k = k0 + (int64_t)q * kSortThreads + threadIdx.x;
    if constexpr (CELL)
      v[q] = (E)P.key[q];
    else
      v[q] = P.key[q] >= 0 ? src[k] : E(0);
  }
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    if (P.key[q] < 0) continue;
    if (P.pos[q] >= 0)
      stage[P.pos[q]] = v[q];
    else
      dst[-(int64_t)P.pos[q] - 1] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const int t = q * kSortThreads + threadIdx.x;
    if (t < P.ns) dst[P.dest[q]] = stage[t];
  }
  __syncthreads();
}

// Scatter to the cells' slots (offs: the exclusive scan of the counts, each
// entry advanced by what is claimed from it).  The block's window slots are
// ranked per cell by LDS atomics and laid out in cell order in LDS; one
// global atomic per occupied cell claims the cell's range, and the columns
// go out one at a time through the LDS stage, consecutive threads writing
// consecutive slots of a cell.  Order within a cell is not kept.
template <bool MIXED>
__global__ void __launch_bounds__(kSortThreads)
    k_scatter(MapP m, SpecDev src, SpecDev dst, int64_t n, int32_t* offs) {
  extern __shared__ int32_t cnt[];                      // [W], then offset << 16 | list index
  __shared__ uint64_t stage[kSortChunk];                // lists, then slot lists, then columns
  __shared__ int nocc, nstaged;
  int32_t* occ_e = reinterpret_cast<int32_t*>(stage);   // occupied cells [nocc]
  int32_t* occ_v = occ_e + kSortChunk;                  // their counts, then dest - lp
  SortPlan P;
  P.W = sort_window(m.nz);
  const int W = P.W;
  for (int e = threadIdx.x; e < W; e += kSortThreads) cnt[e] = 0;
  const int64_t k0 = (int64_t)blockIdx.x * kSortChunk;
  P.lo = sort_keys(m, src, n, MIXED, k0, P.key);
  const int lo = P.lo;
  // ranks within the block's cells, or global slots for the others
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const int c = P.key[q], e = c - lo;
    P.pos[q] = 0;
    if (c < 0) continue;
    if (e >= 0 && e < W)
      P.pos[q] = atomicAdd(&cnt[e], 1);
    else
      P.pos[q] = -atomicAdd(&offs[c], 1) - 1;
  }
  __syncthreads();
  // exclusive scan of the counts over the window (consecutive entries per
  // thread) with the occupied cells listed in order
  {
    const int per = (W + kSortThreads - 1) / kSortThreads;
    const int e0 = threadIdx.x * per, e1 = min(e0 + per, W);
    int tot = 0, nnz = 0;
    for (int e = e0; e < e1; ++e) {
      const int v = cnt[e];
      tot += v;
      nnz += v ? 1 : 0;
    }
    // counts and occupied cells packed (each at most kSortChunk) and scanned together
    const int x = (tot << 16) | nnz;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int o = __shfl_up(inc, off, 64);
      if (lane >= off) inc += o;
    }
    __shared__ int wsum[kSortThreads / 64];
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int base = 0, all = 0;
#pragma unroll
    for (int u = 0; u < kSortThreads / 64; ++u) {
      base += u < w ? wsum[u] : 0;
      all += wsum[u];
    }
    const int run = base + inc - x;
    int off = run >> 16, li = run & 0xffff;
    for (int e = e0; e < e1; ++e) {
      const int v = cnt[e];
      if (v) {
        occ_e[li] = e;
        occ_v[li] = v;
        cnt[e] = (off << 16) | li;
        off += v;
        ++li;
      }
    }
    if (threadIdx.x == 0) {
      nocc = all & 0xffff;
      nstaged = all >> 16;
    }
  }
  __syncthreads();
  // one global atomic per occupied cell: dest = lp + (claimed slot - offset)
  for (int li = threadIdx.x; li < nocc; li += kSortThreads) {
    const int e = occ_e[li];
    const int g = atomicAdd(&offs[lo + e], occ_v[li]);
    occ_v[li] = g - (cnt[e] >> 16);
  }
  // places in the stage
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const int c = P.key[q], e = c - lo;
    if (c >= 0 && e >= 0 && e < W) P.pos[q] += cnt[e] >> 16;
  }
  __syncthreads();
  // the list index of each staged slot, then each writer's destinations
  int32_t* slot_li = occ_e;  // occ_e is no longer read
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const int c = P.key[q], e = c - lo;
    if (c >= 0 && e >= 0 && e < W) slot_li[P.pos[q]] = cnt[e] & 0xffff;
  }
  __syncthreads();
  P.ns = nstaged;
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const int t = q * kSortThreads + threadIdx.x;
    P.dest[q] = t < P.ns ? t + occ_v[slot_li[t]] : 0;
  }
  __syncthreads();
  if constexpr (!MIXED) {
    double* sd = reinterpret_cast<double*>(stage);
    scatter_col<double>(P, k0, src.xi, dst.xi, sd);
    scatter_col<double>(P, k0, src.eta, dst.eta, sd);
    scatter_col<double>(P, k0, src.vr, dst.vr, sd);
    scatter_col<double>(P, k0, src.vt, dst.vt, sd);
    scatter_col<double>(P, k0, src.vz, dst.vz, sd);
  } else {
    float* sf = reinterpret_cast<float*>(stage);
    scatter_col<int32_t, true>(P, k0, src.cell, dst.cell, reinterpret_cast<int32_t*>(stage));
    scatter_col<float>(P, k0, src.fa, dst.fa, sf);
    scatter_col<float>(P, k0, src.fb, dst.fb, sf);
    scatter_col<float>(P, k0, src.fvr, dst.fvr, sf);
    scatter_col<float>(P, k0, src.fvt, dst.fvt, sf);
    scatter_col<float>(P, k0, src.fvz, dst.fvz, sf);
  }
  scatter_col<uint64_t>(P, k0, src.uid, dst.uid, stage);
}

// Kinetic energy of a species: a fixed grid (kKineticBlocks) strides over
// the particles, so that only that many blocks add their sums into one word
// (one block per 256 particles serialised 0.5M atomic adds on it at 134M
// particles).
constexpr int kKineticBlocks = 2048;

__global__ void k_kinetic(SpecDev s, int64_t n, int mixed, double* out) {
  double e = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kBlock) {
    if (!mixed) {
      if (s.xi[k] >= 0.0) e += s.vr[k] * s.vr[k] + s.vt[k] * s.vt[k] + s.vz[k] * s.vz[k];
    } else if (s.cell[k] >= 0) {
      const double a = s.fvr[k], b = s.fvt[k], c = s.fvz[k];
      e += a * a + b * b + c * c;
    }
  }
  __shared__ double red[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) e += __shfl_down(e, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) t += red[q];
    if (t != 0.0) unsafeAtomicAdd(out, 0.5 * s.m * s.w * t);
  }
}

// Bilinear node charge, block-local as the sort: a block's slots add their
// four corner charges in LDS over the nodes of its cell window (node
// i (nz + 1) + j of cell i nz + j, and the corners +1, +nz+1, +nz+2), then
// one global atomic per touched node; slots outside the window add theirs
// globally.  In a wavefront the lanes of the most common cells (up to
// kNodeGroups cells of at least kNodeMinGroup lanes: between sorts a
// wavefront holds a few cells) are summed by a butterfly first, so that
// one lane adds their charge; LDS atomics from many lanes on one address
// would serialise.
__host__ __device__ inline int node_window(int nz) {
  const int W = sort_window(nz);
  return W + W / nz + nz + 4;
}

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int kNodeGroups = 2, kNodeMinGroup = 16;

__global__ void __launch_bounds__(kSortThreads)
    k_node_charge(MapP m, SpecDev s, int64_t n, int mixed, double* q) {
  extern __shared__ double qn[];
  const int nz = m.nz, nz1 = nz + 1;
  const int W = sort_window(nz), NW = node_window(nz);
  for (int e = threadIdx.x; e < NW; e += kSortThreads) qn[e] = 0.0;
  const int64_t k0 = (int64_t)blockIdx.x * kSortChunk;
  int key[kSortPer];
  const int lo = sort_keys(m, s, n, mixed != 0, k0, key);
  const int n0 = lo + lo / nz;  // node of cell lo's lower corner
  const double qw = s.q * s.w;
  const uint64_t me = 1ull << (threadIdx.x & 63);
#pragma unroll 1
  for (int r = 0; r < kSortPer; ++r) {
    const int c = key[r];
    const int64_t k = k0 + (int64_t)r * kSortThreads + threadIdx.x;
    double w00 = 0.0, w10 = 0.0, w01 = 0.0, w11 = 0.0;
    int nd = 0;
    if (c >= 0) {
      const int i = c / nz, j = c - i * nz;
      double a, b;
      if (!mixed) {
        a = s.xi[k] - i;
        b = s.eta[k] - j;
      } else {
        a = s.fa[k];
        b = s.fb[k];
      }
      w00 = qw * (1 - a) * (1 - b);
      w10 = qw * a * (1 - b);
      w01 = qw * (1 - a) * b;
      w11 = qw * a * b;
      nd = c + i;  // i (nz + 1) + j
    }
    const bool in = c >= lo && c < lo + W;
    if (c >= 0 && !in) {
      unsafeAtomicAdd(&q[nd], w00);
      unsafeAtomicAdd(&q[nd + nz1], w10);
      unsafeAtomicAdd(&q[nd + 1], w01);
      unsafeAtomicAdd(&q[nd + nz1 + 1], w11);
    }
    uint64_t pending = __ballot(in);
    for (int g = 0; g < kNodeGroups && pending; ++g) {
      const int lead = __ffsll((unsigned long long)pending) - 1;
      const int lk = __shfl(c, lead, 64);
      const bool mem = (pending & me) && c == lk;
      const uint64_t mm = __ballot(mem);
      if (__popcll(mm) < kNodeMinGroup) break;
      const double s00 = wave_sum_d(mem ? w00 : 0.0), s10 = wave_sum_d(mem ? w10 : 0.0);
      const double s01 = wave_sum_d(mem ? w01 : 0.0), s11 = wave_sum_d(mem ? w11 : 0.0);
      if ((int)(threadIdx.x & 63) == lead) {
        const int e = nd - n0;
        atomicAdd(&qn[e], s00);
        atomicAdd(&qn[e + nz1], s10);
        atomicAdd(&qn[e + 1], s01);
        atomicAdd(&qn[e + nz1 + 1], s11);
      }
      pending &= ~mm;
    }
    if (pending & me) {
      const int e = nd - n0;
      atomicAdd(&qn[e], w00);
      atomicAdd(&qn[e + nz1], w10);
      atomicAdd(&qn[e + 1], w01);
      atomicAdd(&qn[e + nz1 + 1], w11);
    }
  }
  __syncthreads();
  const int64_t nn = (int64_t)(m.nr + 1) * nz1;
  for (int e = threadIdx.x; e < NW; e += kSortThreads) {
    const double v = qn[e];
    if (v != 0.0 && n0 + e < nn) unsafeAtomicAdd(&q[n0 + e], v);
  }
}

__global__ void k_zero(double* p, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) p[k] = 0.0;
}

__global__ void k_zero_i(int32_t* p, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) p[k] = 0;
}

__global__ void k_copy(double* d, const double* s, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) d[k] = s[k];
}

inline int64_t nblk(int64_t n) { return (n + kBlock - 1) / kBlock; }

}  // namespace

hipError_t scan_exclusive(int32_t* data, int64_t n, int32_t* part, hipStream_t st) {
  const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
  if (nb > 0) {
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(kScanThreads), 0, st, data, n, part);
  }
  hipLaunchKernelGGL(k_scan_part, dim3(1), dim3(1024), 0, st, part, nb, data, n);
  if (nb > 0) {
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kScanThreads), 0, st, data, n, part);
  }
  return hipGetLastError();
}

hipError_t launch_sort_async(Ctx& c, Species& sp, int32_t* total_pinned, hipStream_t st) {
  const int64_t ncell = (int64_t)c.g.nr * c.g.nz;
  const int mixed = c.prec == ECPIC_MIXED;
  SpecDev& src = sp.d[sp.cur];
  SpecDev& dst = sp.d[1 - sp.cur];
  hipLaunchKernelGGL(k_zero_i, dim3(nblk(ncell + 1)), dim3(kBlock), 0, st, c.hist, ncell + 1);
  const int64_t nsb = (sp.n + kSortChunk - 1) / kSortChunk;
  const size_t win = (size_t)sort_window(c.g.nz) * sizeof(int32_t);
  if (sp.n > 0)
    hipLaunchKernelGGL(k_hist, dim3(nsb), dim3(kSortThreads), win, st, c.m, src, sp.n, mixed,
                       c.hist);
  hipError_t e = scan_exclusive(c.hist, ncell, c.scan_part, st);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(total_pinned, c.hist + ncell, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  if (sp.n > 0)
    hipLaunchKernelGGL(mixed ? k_scatter<true> : k_scatter<false>, dim3(nsb), dim3(kSortThreads),
                       win, st, c.m, src, dst, sp.n, c.hist);
  return hipGetLastError();
}

void finish_sort(Species& sp, int32_t total) {
  sp.cur = 1 - sp.cur;
  sp.n = total;
  sp.d[sp.cur].n = total;
}

hipError_t launch_sort(Ctx& c, Species& sp, hipStream_t st, int64_t* n_alive_host) {
  hipError_t e = launch_sort_async(c, sp, c.sort_total_host, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  finish_sort(sp, c.sort_total_host[0]);
  if (n_alive_host) *n_alive_host = sp.n;
  return hipSuccess;
}

hipError_t launch_kinetic(const Species& sp, int mixed, double* out, hipStream_t st) {
  if (sp.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kinetic, dim3((unsigned)std::min<int64_t>(nblk(sp.n), kKineticBlocks)),
                     dim3(kBlock), 0, st, sp.d[sp.cur], sp.n, mixed,
                     out);
  return hipGetLastError();
}

hipError_t launch_node_charge(const Ctx& c, double* q, hipStream_t st) {
  const int64_t nn = (int64_t)(c.g.nr + 1) * (c.g.nz + 1);
  hipLaunchKernelGGL(k_zero, dim3(nblk(nn)), dim3(kBlock), 0, st, q, nn);
  const int mixed = c.prec == ECPIC_MIXED;
  for (const Species& sp : c.sp) {
    if (sp.n <= 0) continue;
    const int64_t nsb = (sp.n + kSortChunk - 1) / kSortChunk;
    hipLaunchKernelGGL(k_node_charge, dim3(nsb), dim3(kSortThreads),
                       (size_t)node_window(c.g.nz) * sizeof(double), st, c.m, sp.d[sp.cur], sp.n,
                       mixed, q);
  }
  return hipGetLastError();
}

namespace {

// Charge-conservation check of a committed step (Sec. 2.1: the deposit is
// charge-conserving, so continuity holds at every node and Gauss's law,
// once it holds, keeps holding).  Per node (i, j) of [nr+1][nz+1]:
//   Q   = particle charge (bilinear weights) + wall charge on wall nodes
//   div = net flux out of the node's dual cell of a face quantity on the
//         r-edges (f_r) and z-edges (f_z):
//         f_r[i][j] - f_r[i-1][j] + f_z[i][j] - f_z[i][j-1] (missing terms 0)
//   continuity  = Q^{n+1} - Q^n + dt div(I)
//   Gauss       = div(D) - Q_particles with D the displacement flux
//                 eps A*/l u (halved dual faces of r-edges on the z walls),
//                 compared with its value at t^n on the nodes off the
//                 conducting walls (0 <= i < nr, 0 < j < nz)
// The state of t^{n+1} replaces that of t^n in q0 / gq0.  Maxima of
// |continuity|, |Gauss change| and |Q| go to out[0..2] as the bit patterns of
// non-negative doubles, whose integer order is their numeric order.
__global__ void __launch_bounds__(kBlock)
    k_conservation(MapP m, const double* __restrict__ wr, const double* __restrict__ wz,
                   const double* __restrict__ ur, const double* __restrict__ uz,
                   const double* __restrict__ Ir, const double* __restrict__ Iz,
                   const double* __restrict__ qp, const double* __restrict__ wbot,
                   const double* __restrict__ wtop, const double* __restrict__ wside,
                   double* __restrict__ q0, double* __restrict__ gq0, int first, double dt,
                   unsigned long long* out) {
  const int nr = m.nr, nz = m.nz;
  const int64_t nn = (int64_t)(nr + 1) * (nz + 1);
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double c_cont = 0.0, c_gauss = 0.0, c_q = 0.0;
  if (t < nn) {
    const int i = int(t / (nz + 1)), j = int(t - (int64_t)i * (nz + 1));
    double q = qp[t];
    const double qpart = q;
    if (j == 0) q += wbot[i];
    if (j == nz) q += wtop[i];
    if (i == nr) q += wside[j];
    // r-edges (i, j) and (i-1, j); z-edges (i, j) and (i, j-1)
    const int64_t er = (int64_t)i * (nz + 1) + j, erm = er - (nz + 1);
    const int64_t ez = (int64_t)i * nz + j, ezm = ez - 1;
    double dI = 0.0, dD = 0.0;
    const double half = (j == 0 || j == nz) ? 0.5 : 1.0;
    if (i < nr) {
      dI += Ir[er];
      dD += half * wr[i] * ur[er];
    }
    if (i > 0) {
      dI -= Ir[erm];
      dD -= half * wr[i - 1] * ur[erm];
    }
    if (j < nz) {
      dI += Iz[ez];
      if (i < nr) dD += wz[i] * uz[ez];
    }
    if (j > 0) {
      dI -= Iz[ezm];
      if (i < nr) dD -= wz[i] * uz[ezm];
    }
    const double gq = dD - qpart;
    if (!first) {
      c_cont = fabs(q - q0[t] + dt * dI);
      if (i < nr && j > 0 && j < nz) c_gauss = fabs(gq - gq0[t]);
    }
    c_q = fabs(qpart);
    q0[t] = q;
    gq0[t] = gq;
  }
  double v[3] = {c_cont, c_gauss, c_q};
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = fmax(v[k], __shfl_xor(v[k], off, 64));
  __shared__ double red[kBlock / 64][3];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 3; ++k) red[w][k] = v[k];
  __syncthreads();
  if (threadIdx.x < 3) {
    double x = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) x = fmax(x, red[q][threadIdx.x]);
    if (x > 0.0) atomicMax(out + threadIdx.x, (unsigned long long)__double_as_longlong(x));
  }
}

}  // namespace

hipError_t launch_conservation(const Ctx& c, const double* ur, const double* uz, const double* Ir,
                               const double* Iz, bool first, hipStream_t st) {
  const int64_t nn = (int64_t)(c.g.nr + 1) * (c.g.nz + 1);
  hipLaunchKernelGGL(k_conservation, dim3(nblk(nn)), dim3(kBlock), 0, st, c.m, c.sol.wr,
                     c.sol.wz, ur, uz, Ir, Iz, c.q_node, c.wall_bot, c.wall_top, c.wall_side,
                     c.q0, c.gq0, first ? 1 : 0, c.g.dt, c.cons_dev);
  return hipGetLastError();
}

hipError_t launch_zero(double* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3(nblk(n)), dim3(kBlock), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_zero_i(int32_t* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_i, dim3(nblk(n)), dim3(kBlock), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_copy(double* d, const double* s, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(nblk(n)), dim3(kBlock), 0, st, d, s, n);
  return hipGetLastError();
}

}  // namespace ecpic
