// ecpic_internal.h -- kernel argument structures, the context, and the
// launchers each translation unit exports to the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ecpic.h"

namespace ecpic {

constexpr int kMaxSpecies = 4;
constexpr int kMaxSub = 64;     // sub-steps per particle per step
constexpr int kMaxHalve = 20;   // halvings of a sub-step whose solve fails
constexpr int kMaxFixed = 50;   // fixed-point iterations per sub-step solve
constexpr int kMaxIter = 64;    // Picard iterations per step
constexpr int kMaxKrylov = 32;  // JFNK: GMRES iterations per Newton step
constexpr int kJfBlocks = 256;  // JFNK: blocks of the dot-product kernel
constexpr int kBlock = 256;     // threads per block for particle kernels
constexpr int kPerThread = 4;   // particles per thread of the fast push
constexpr int kPerBlock = kBlock * kPerThread;
// Contended counters are spread over copies on separate cache lines: block b
// uses copy b % kSpread (queue segments, commit tallies).
constexpr int kSpread = 64;
constexpr int kLineInts = 32;   // 128-byte stride between queue counters
// queue counters of one kind: [kMaxSpecies][kSpread][kLineInts]; two kinds
// (the slow-pass queue, then the collision list) in one allocation
constexpr int kQCount = kMaxSpecies * kSpread * kLineInts;

// Mesh map r(xi) (C^1 two-piece: r = 2 s sqrt(xi xi_a) below xi_a, s (xi+xi_a)
// above) and the uniform axial map z = eta dz.
struct MapP {
  int nr, nz;
  double xi_a, s, inv_s, rsqrt_xa, dz, inv_dz, dt;
  int i_lin;  // first radial cell entirely in the linear part of the map
  int ip;     // TEM port: first port edge (i, 0) of the bottom wall, 0: none
};

// The TEM port's tables and state as the field kernels see them (Sec. 2.1,
// Eqs. (5), (7)).  pc holds four rows of nr values, entries i >= ip used:
// g_i = 1 / (w_b/dt + M/(2 eta l)), a_i = M kappa_i / (2 eta l), kappa_i, and
// 1 / (eta l), with M = 2 pi r_{i+1/2}, w_b = wr/2, l the edge length.
struct PortDev {
  int ip;               // 0: no port
  const double* pc;
  const double* hb;     // H_b^n, [nr]
  double vnow, vnext;   // the electrode potential at t^n, t^{n+1} (no capacitor)
  const double* phin;   // with the capacitor: phi^n on the device, else null
  const double* phi1;   // with the capacitor: the iterate's phi^{n+1}, else null
};
constexpr int kPortG = 0, kPortA = 1, kPortK = 2, kPortIEL = 3;
__host__ __device__ inline double port_dphi(const PortDev& P) {
  return (P.phi1 ? P.phi1[0] : P.vnext) - (P.phin ? P.phin[0] : P.vnow);
}

// One species as the kernels see it.  FP64 path: xi, eta, v*; mixed path:
// cell (= i*nz + j), fa, fb (offsets in [0,1]) and fv*.  Dead particles have
// xi < 0 (FP64) or cell < 0 (mixed).
struct SpecDev {
  double *xi, *eta, *vr, *vt, *vz;
  int32_t* cell;
  float *fa, *fb, *fvr, *fvt, *fvz;
  uint64_t* uid;
  int64_t n, cap;
  double q, m, w;
  double qm, qw_dt;   // q/m and q w/dt, formed on the host
  int32_t mobile, sid;
};

// Sentinel-free results the device leaves in host memory use 8-byte
// system-scope stores (one access each, visible to a polling host).
__device__ __forceinline__ void store_sys(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void store_sys(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Device-side tallies of a commit / collision pass.
struct Tally {
  double w_absorbed, w_coll, w_particles;
  double pad;
  unsigned long long n_absorbed[kMaxSpecies];
  unsigned long long n_coll[kMaxSpecies];
  unsigned long long n_ionized, n_errors, n_crossings, n_substeps, n_over_range, n_overflow;
  unsigned long long append[kMaxSpecies];
};

// What the host needs after a commit: the tallies summed over their copies,
// the field-particle exchange, and the drive-gap values of the energy balance.
struct StepFinal {
  Tally t;
  double xs;        // sum over interior edges of u^{1/2} . I
  double h_gap_n;   // h^n at the drive-gap cell
  double h_gap_1;   // h^{n+1} at the drive-gap cell
  double ir_gap;    // I_r on the drive-gap edge
  // electrostatic model: the change of the field flux leaving the powered
  // plate's nodes, sum_i wz_i (uz^{n+1} - uz^n)[i][0], and the current
  // leaving them, sum_i Iz[i][0] (the source's work)
  double qp_delta;
  double iz_plate;
  // blocking capacitor: electrode potential at t^n and t^{n+1}, capacitor
  // charge at t^{n+1}, and the electrode current of the accepted iterate
  double phi_n, phi_1, q_1, ie;
  // TEM port: EM, the power through the mouth times dt,
  // dt sum M H_b^{n+1/2} u^{n+1/2}; either model, the mouth voltage at t^{n+1}
  double port_w, port_v;
  uint64_t seq;     // written last: the host polls it
};

// Null-collision parameters of one pass, prepared on the host.
struct MccDev {
  int32_t enabled, role;        // role 1: electron-Ar, 2: Ar+-Ar
  double pnull, numax, n_gas, m_gas, sig_gas;  // sig_gas = sqrt(kT/m_gas)
  double sig_ion;               // sqrt(kT/m_ion) for ions born in ionisation
  double eps_max_ev;
  uint64_t seed;
  int64_t step;
  SpecDev partner;              // ion species receiving ionisation products
  int64_t base_self, base_partner;  // append offsets (counts before the pass)
};

struct PushArgs {
  MapP m;
  const double* ur;  // half-step field, FP64
  const double* uz;
  const float* urf;  // half-step field, FP32 copy (mixed path)
  const float* uzf;
  double* Ir;
  double* Iz;
  SpecDev s;
  SpecDev out;       // where a commit writes the new state (s itself, or the
                     // species' other buffer); ids are copied when it differs
  int32_t commit;
  double* wall_bot;
  double* wall_top;
  double* wall_side;
  Tally* tally;
  MccDev mcc;
  const int32_t* stop;  // when set and nonzero the pass does nothing (or null)
};

// One push pass over up to two species in one launch (slot 0 and slot 1):
// the fast kernel takes the slot from blockIdx.y, the slow and collision
// kernels from blockIdx.z.  Both slots share the pass-wide members of a[0]
// (fields, currents, walls, tallies, stop, commit).
struct PassArgs {
  PushArgs a[2];
  int32_t* queue[2];   // kSpread segments of qseg entries per slot
  int32_t* qcount[2];  // kSpread counters, kLineInts apart, zero on entry
  int32_t* cqueue[2];  // the same for the collision list of a commit pass
  int32_t* cqcount[2];
  int64_t qseg[2];
  // per slot, the particle record of every slow-queue entry at the entry's
  // position: field f at qrec[f * qcap + position] (FP64: xi, eta, vr, vt,
  // vz; FP32: cell, a, b, vr, vt, vz as 4-byte words)
  double* qrec[2];
  int64_t qcap;
  int32_t nsp;         // slots in use (1 or 2)
  int32_t queue_waves; // build of the plain slow pass: 0 by size, else 2 or 3
};

// One Crank-Nicolson field solve.  Optional outputs (null = skipped): the
// residual partials against the previous iterate, the next half-step field,
// and the reset of the consumed currents.
struct SolveArgs {
  const double *ur0, *uz0, *h0;
  double *Ir, *Iz;
  double vhalf, vnext;
  double vnow;          // drive at t^n (the electrostatic model's plate step)
  // blocking capacitor: the gap voltage at t^{n+1} is read from here (the
  // circuit's current iterate) and at t^n from ur0's gap edge; null: vnow,
  // vnext
  const double* gapv;
  // blocking capacitor with a port: the electrode potential at t^n (the
  // circuit state), else null
  const double* phin;
  double *ur1, *uz1, *h1;
  const double *ur_old, *uz_old;
  double* part;         // [2 * nr]: per row sum w (u1 - u_old)^2, sum w u1^2
  double *ur_h, *uz_h;  // (u0 + u1) / 2
  float *ur_hf, *uz_hf;
  double *Ir_clr, *Iz_clr;  // set to zero once read (may alias Ir, Iz), or null
  const int32_t* stop;  // when set and nonzero the solve does nothing (or null)
};

constexpr int kRedBlocks = 256;  // partial-sum blocks of the field reductions
constexpr int kResParts = 8192;  // blocks of the field solve that write residual partials
// Grid limits checked at creation: the field solve's per-mode scan holds at
// most 2048 rows (256 threads x 8), its transform blocks (4 rows x 32
// columns) write at most kResParts residual partials, and the row-sized
// LDS arrays of the transform and push kernels fit 64 KB with nz <= 1024.
constexpr int kMaxNr = 2048;
constexpr int kMaxNz = 1024;
inline bool grid_fits(int nr, int nz) {
  return nr <= kMaxNr && nz <= kMaxNz &&
         (int64_t)((nr + 3) / 4) * ((nz + 31) / 32) <= kResParts;
}

struct Species {
  ecpic_species_desc desc;
  SpecDev d[2];  // ping-pong buffers for the sort
  int cur = 0;
  int64_t n = 0;  // slots in use (live + dead until the next sort)
};

struct SolverDev {
  // geometry per radial index
  double* rh;    // r_{i+1/2}, nr
  double* wr;    // eps A*_r / l, nr
  double* wz;    // eps A*_z / dz, nr
  double* area;  // meridional cell area, nr
  // separable solve
  double* Q;     // orthonormal DCT-II, [nz][nz], Q[k][j]
  double* Qt;    // transpose
  double* tri_lo;   // Thomas: sub-diagonal multipliers, [nz][nr]
  double* tri_inv;  // Thomas: inverse pivots, [nz][nr]
  double* tri_up;   // super-diagonal of the system, [nr]
  // TEM port (Woodbury form of the port's diagonal on the separable solve):
  // pc [4][nr] (PortDev), F = (D^-1 + U^T A0^-1 U)^-1 over the m port cells
  // [m][m] (symmetric), q0[k] = Q[k][0] [nz], z = F U^T y [m] followed by
  // the coupling's partial sums [32][m]; the
  // electrostatic wall profile [nr+1] (always present)
  double* port_pc;
  double* port_F;
  double* port_q0;
  double* port_z;
  double* prof;
  double* work0;    // [nr][nz]
  double* work1;    // [nr][nz]
  double* partial;  // reduction partials
};

struct Ctx {
  ecpic_grid_desc g;
  ecpic_precision prec;
  hipStream_t stream;
  int device = 0;                  // the device current at ecpic_create
  MapP m;
  std::string err;
  std::vector<Species> sp;
  // fields (FP64) at t^n, t^{n-1}, the current iterate, the previous iterate
  double *ur, *uz, *h, *ur_prev, *uz_prev, *h_prev;
  double *ur_it, *uz_it, *h_it;    // u^{n+1,(k)}, h^{n+1,(k)}
  double *ur_nx, *uz_nx, *h_nx;    // u^{n+1,(k+1)} being produced
  double *ur_half, *uz_half;       // half-step field of the current push
  float *ur_half_f, *uz_half_f;    // FP32 copy (mixed path)
  double *ur_half2, *uz_half2;     // half-step field of the next push
  float *ur_half_f2, *uz_half_f2;
  double* part_host;               // pinned host copy of reduction partials
  // speculative Picard iterations: a device flag set once an iterate meets
  // the tolerance (every kernel of a later iteration then returns at once),
  // and the residuals written by the device into pinned host memory
  int32_t* stop = nullptr;  // [0]: stop flag, [1]: the iteration that converged
  double* res_host = nullptr;      // [kMaxIter], coherent pinned, device-written
  double* res_dev = nullptr;       // device alias of res_host
  struct StepFinal* fin_host = nullptr;  // commit summary, coherent pinned
  struct StepFinal* fin_dev = nullptr;   // device alias
  uint64_t fin_seq = 0;            // sequence number of the last summary asked for
  int32_t* sort_total_host = nullptr;    // [kMaxSpecies], pinned
  double *Ir, *Iz;                 // currents deposited by the current pass
  double *Ir_alt, *Iz_alt;         // the other pair: inside a step the Picard
                                   // iterations alternate, so that the currents
                                   // of the accepted iterate outlive its solve
  double *wall_bot, *wall_top, *wall_side;
  int32_t* hist;                   // per-cell counts [nr*nz + 1]
  int32_t* offs;                   // per-cell offsets [nr*nz + 1]
  int32_t* scan_part;              // scan block sums
  Tally* tally;                    // device tallies: two sets of kSpread copies,
                                   // used by Picard iterations of either parity
  double* wall_scr = nullptr;      // wall charge of a committing iteration, by
                                   // parity: 2 x [bot nr+1, top nr+1, side nz+1]
  int32_t* queue = nullptr;        // slow-pass particle queues, one per species,
                                   // then as many collision lists
  int64_t queue_cap = 0;           // entries per species and kind
  double* qrec = nullptr;          // slow-queue entry records, 5 x queue_cap
                                   // words of 8 bytes per species
  int32_t* qcount = nullptr;       // queue lengths: 2 kQCount (slow queues, then
                                   // collision lists)
  Tally* tally_host;               // pinned host mirror of the copies
  double* red_host;                // pinned host reduction results
  SolverDev sol;
  double t = 0.0;
  int64_t step = 0;
  ecpic_mcc_desc mcc{};
  double numax[kMaxSpecies] = {0, 0, 0, 0};  // null-collision rate per species
  // learned guess
  float* nn_w = nullptr;           // FP32 weights, canonical layout
  float nn_norm[8] = {1, 1, 1, 1, 1, 1, 1, 1};  // input (6) and output (2) scales
  bool nn_ready = false;
  void* nn_ws = nullptr;           // training/batch workspace
  size_t nn_ws_bytes = 0;
  void* nn_gws = nullptr;          // workspace of the in-step guess (one image)
  size_t nn_gws_bytes = 0;
  // Device memory.  Nothing is allocated at create: at first use (or when
  // the caller binds a workspace) every device array of the context and of
  // the species added so far is carved from one region, the caller's bound
  // workspace or one block the library allocates.  Species added after that
  // (library-owned memory only) get allocations of their own.
  bool materialised = false;
  void* ws = nullptr;              // the caller's workspace, or null
  size_t ws_bytes = 0;
  void* own_block = nullptr;       // the library's block when none is bound
  std::vector<void*> owned;        // allocations made after the first use
  int32_t queue_species = 0;       // species slots the queues are sized for
  int32_t queue_waves = 0;         // ECPIC_OPT_QUEUE_WAVES
  int32_t nn_force_fallback = 0;   // ECPIC_OPT_NN_FORCE_FALLBACK
  // Jacobian-free Newton-Krylov: ECPIC_OPT_JFNK_KRYLOV reserves jfnk_m + 1
  // Krylov vectors and six work vectors ([ur | uz] each) in the layout
  // blocking capacitor (g.blocking_cap > 0), device state: [0] phi^n,
  // [1] phi^{n-1}, [2] q^n, [3] the electrode potential the next solve uses,
  // [6 + 2p], [7 + 2p] the potential and electrode current of the last
  // Picard iteration of parity p
  double* circ = nullptr;
  // TEM port: the line's wall field H_b at t^n under every port edge [nr]
  double* port_hb = nullptr;
  int32_t jfnk_m = 0;
  double* jf_vec = nullptr;
  double* jf_part = nullptr;       // dot partials [kMaxKrylov + 1][kJfBlocks]
  double* jf_host = nullptr;       // pinned copy of the partials
  // the rotation of u^{n-1}, u^n, u^{n+1} takes a fourth buffer, so that a
  // step that is not committed still has u^{n-1} after the next step's guess
  // has been enqueued
  double *ur_spare = nullptr, *uz_spare = nullptr;
  // fields bound by the caller (ecpic_bind_fields): u^n and u^{n-1} live in
  // the caller's arrays, shifted by copies at each commit
  bool fields_bound = false;
  double* lib_fields[6] = {};      // the library's own ur, uz, h, ur_prev, uz_prev, h_prev
  // charge-conservation diagnostics of a committed step
  double* q_node = nullptr;        // particle node charge [nr+1][nz+1]
  double* q0 = nullptr;            // total node charge (with walls) at t^n
  double* gq0 = nullptr;           // Gauss residual G - Q at t^n
  unsigned long long* cons_dev = nullptr;   // maxima as double bit patterns
  unsigned long long* cons_host = nullptr;  // pinned copy
  bool cons_valid = false;         // q0, gq0 describe the current state
  int32_t* rd_scratch = nullptr;   // block counts of ecpic_read_particles
  int64_t rd_scratch_len = 0;
  // event timing of the hot kernels
  uint32_t prof_mask = 0;          // bit k: time launches of kind k
  int32_t prof_every = 1;          // time every prof_every-th launch of a kind
  uint64_t prof_seq[ECPIC_K_COUNT] = {};
  struct Count {
    int kind;
    int64_t particles;
    int tag;
  };
  std::vector<Count> count_pending;  // launches not yet folded into the totals
  int cur_tag = 0;                 // iteration whose launches are being enqueued
  ecpic_profile prof{};
  struct Pending {
    hipEvent_t a, b;
    int kind;
    double bytes;
    int64_t particles;
    int tag;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> ev_pool;
  std::vector<hipEvent_t> ev_dropped;  // back to the pool at the next collect
};

// The generator voltage V(t): a sum of up to 32 harmonics, zero from
// drive_t_end on when that is set (host).
double drive_voltage(const ecpic_grid_desc& g, double t);

// ---- launchers (stream-ordered, no synchronisation) ----
// push
// fast pass over all particles of a species, then the slow pass over the
// ones it queued (cell crossers, failed solves).  queue holds kSpread
// segments of queue_seg entries; qcount (kSpread counters, kLineInts apart)
// must be zero on entry.  tally points at kSpread copies.
hipError_t launch_push_fast(const PassArgs& p, bool deposit, hipStream_t s);
hipError_t launch_push_slow(const PassArgs& p, hipStream_t s);
// the committing slow pass and the collisions of the listed particles, in
// one launch
hipError_t launch_slow_collide(const PassArgs& P, hipStream_t st);
// commit pass with MCC: the collisions of the particles the fast pass listed
hipError_t launch_collide_list(const PassArgs& p, hipStream_t s);
// entries per queue segment for n particles: fast-pass block b queues into
// segment b % kSpread
inline int64_t queue_segment(int64_t n) {
  const int64_t nb = (n + kPerBlock - 1) / kPerBlock;
  return ((nb + kSpread - 1) / kSpread) * kPerBlock;
}
// fast-pass blocks for n particles; fast-pass dynamic LDS for nz cells in z
int64_t fast_blocks(int64_t n);
size_t fast_lds_bytes(int nz);
hipError_t launch_load(const MapP& m, const SpecDev& s, const double* r, const double* z,
                       const double* vr, const double* vt, const double* vz, const uint64_t* uid,
                       int64_t n, double R, int mixed, hipStream_t st);
hipError_t launch_flag_count(const MapP& m, const SpecDev& s, int64_t n, int mixed, int32_t* blk,
                             hipStream_t st);
hipError_t launch_compact_read(const MapP& m, const SpecDev& s, int64_t n, int mixed,
                               const int32_t* blk_off, double* xi, double* eta, double* vr,
                               double* vt, double* vz, uint64_t* uid, hipStream_t st);
// exclusive scan of data[0..n) in place; the total goes to data[n]; part
// needs (n + 1023) / 1024 + 1 entries
hipError_t scan_exclusive(int32_t* data, int64_t n, int32_t* part, hipStream_t st);
hipError_t launch_collide(const MapP& m, const SpecDev& s, const MccDev& c, Tally* tally,
                          int mixed, hipStream_t st);
// fields
hipError_t launch_guess_half(const Ctx& c, double vnow, double vnext, hipStream_t s);
hipError_t launch_half(const Ctx& c, const double* u0r, const double* u0z, const double* u1r,
                       const double* u1z, hipStream_t s);
// hat: the [nz][nr] transform intermediate (null: the context's scratch)
hipError_t field_solve(const Ctx& c, const SolveArgs& a, hipStream_t s, double* hat = nullptr);
// the static scratch of the allocation-free solve: its address on `device`
// (taken once, with that device current, by static_scratch_setup), or null
constexpr int64_t kStaticScratchDoubles = (int64_t)1 << 20;
hipError_t static_scratch_setup(int device);
double* static_scratch(int device);
// residual of iterate k from the solve's row partials, stored to res_dev[k]
// (host memory, polled); sets *stop when it is <= tol (tol < 0: never) and
// clears the queue counters and tallies for the next pass.  Does nothing
// when *stop is already set.
hipError_t launch_converge(const Ctx& c, int k, double tol, hipStream_t s,
                           const SolveArgs* a = nullptr);
constexpr int kCircLen = 16;
// commit summary into fin_dev (host memory), seq written last
// tally set (kSpread copies) and wall scratch of iterations of parity p
inline Tally* tally_set(const Ctx& c, int p) { return c.tally + (int64_t)p * kSpread; }
inline int64_t wall_len(const Ctx& c) { return 2 * (int64_t)(c.g.nr + 1) + c.g.nz + 1; }
inline double* wall_scratch(const Ctx& c, int p) { return c.wall_scr + p * wall_len(c); }
// commit summary from the tally set `tally`; when wall_add is set, that
// wall-charge scratch is also added into the wall totals.  guard_k >= 0: the
// kernel does nothing unless Picard iteration guard_k is the one the residual
// kernel found converged (stop[1]), so it can be enqueued before that is known.
hipError_t launch_finalize(const Ctx& c, const Tally* tally, const double* xpart, const double* Ir,
                           const double* Iz, const double* wall_add, uint64_t seq, int guard_k,
                           hipStream_t s, int iter = 0);
hipError_t launch_zero_tally(const Ctx& c, hipStream_t s);
// JFNK vector kernels.  A vector is [ur (nr (nz+1)) | uz ((nr+1) nz)]; the
// inner product weights interior edges by eps A*/l (the residual's norm).
struct JfCoef {
  double v[kMaxKrylov + 1];
};
// z = a x + b y
hipError_t launch_jf_axpby(const Ctx& c, double a, const double* x, double b, const double* y,
                           double* z, hipStream_t s);
// w = v - (g - gx) / e, with g given as its two parts (library field buffers)
hipError_t launch_jf_jv(const Ctx& c, const double* v, const double* gr, const double* gz,
                        const double* gx, double e, double* w, hipStream_t s);
// f = y - g and, if gcopy, gcopy = g (g as two parts)
hipError_t launch_jf_sub(const Ctx& c, const double* y, const double* gr, const double* gz,
                         double* f, double* gcopy, hipStream_t s);
// partials of <w, V_k>, k < K (V_k = V + k ldv), into c.jf_part[k][block]
hipError_t launch_jf_dots(const Ctx& c, const double* w, const double* V, int64_t ldv, int K,
                          hipStream_t s);
// y = alpha y + sum_k coef_k V_k, k < K
hipError_t launch_jf_gemv(const Ctx& c, int K, const double* V, int64_t ldv, const JfCoef& coef,
                          double alpha, double* y, hipStream_t s);
// the value a residual slot holds until the device has written it
constexpr uint64_t kResPending = 0x7ff4dead0badf00dull;
// partials: [0, kRedBlocks) sum w u^2, [kRedBlocks, 2 kRedBlocks) sum 2 pi r A h^2
hipError_t launch_field_energy(const Ctx& c, const double* ur, const double* uz, const double* h,
                               double* part, hipStream_t s);
// partials [0, kRedBlocks): sum over interior edges of ((a + b)/2) I
hipError_t launch_exchange(const Ctx& c, const double* ur_a, const double* uz_a,
                           const double* ur_b, const double* uz_b, const double* Ir,
                           const double* Iz, double* part, hipStream_t s);
// null-collision bound (host): electrons (role 1) or ions (role 2)
double nu_max_host(const ecpic_mcc_desc& mcc, int role, double m_particle);
// learned initial guess: overwrites the guess of the iterate when a network
// is installed; *used tells whether it did
ecpic_status nn_guess(Ctx& c, bool* used);
// sort and diagnostics
hipError_t launch_sort(Ctx& c, Species& sp, hipStream_t s, int64_t* n_alive_host);
// the same without synchronising: the survivor count goes to *total_pinned
// (pinned host memory); once the stream is synchronised, finish_sort makes
// the sorted buffer current.  Species sorted back to back share the
// histogram buffers and must be enqueued on one stream.
hipError_t launch_sort_async(Ctx& c, Species& sp, int32_t* total_pinned, hipStream_t s);
void finish_sort(Species& sp, int32_t total);
hipError_t launch_kinetic(const Species& sp, int mixed, double* out, hipStream_t s);
hipError_t launch_node_charge(const Ctx& c, double* q, hipStream_t s);
// charge-conservation maxima of a committed step (first: only record the
// state at t^n); needs the particle node charge in c.q_node
hipError_t launch_conservation(const Ctx& c, const double* ur, const double* uz, const double* Ir,
                               const double* Iz, bool first, hipStream_t s);
// bytes of the learned guess's one-image workspace (weights prepared in it)
size_t nn_guess_ws_bytes(const Ctx& c);
// assign the context's device arrays at first use (from the bound workspace
// or one block of the library's own); ECPIC_OK when already done
ecpic_status materialise(Ctx& c);
// u^{n-1} <- u^n, u^n <- u^{n+1} by copies (fields bound by the caller)
hipError_t launch_shift(const Ctx& c, hipStream_t s);
hipError_t launch_zero(double* p, int64_t n, hipStream_t s);
hipError_t launch_zero_i(int32_t* p, int64_t n, hipStream_t s);
hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);

// Record a failed HIP call in the context `c` in scope and return EHIP.
#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      c.err = std::string(#expr) + ": " + hipGetErrorString(e_);                  \
      return ECPIC_EHIP;                                                          \
    }                                                                             \
  } while (0)

}  // namespace ecpic

// the opaque handle of the C ABI
struct ecpic_ctx {
  ecpic::Ctx c;
};
