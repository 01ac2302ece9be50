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
constexpr int kBlock = 256;     // threads per block for particle kernels
// Contended counters are spread over copies on separate cache lines: block b
// uses copy b % kSpread (queue segments, commit tallies).
constexpr int kSpread = 64;
constexpr int kLineInts = 32;   // 128-byte stride between queue counters

// Mesh map r(xi) (C^1 two-piece: r = 2 s sqrt(xi xi_a) below xi_a, s (xi+xi_a)
// above) and the uniform axial map z = eta dz.
struct MapP {
  int nr, nz;
  double xi_a, s, inv_s, rsqrt_xa, dz, inv_dz, dt;
  int i_lin;  // first radial cell entirely in the linear part of the map
};

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
  int32_t mobile, sid;
};

// Device-side tallies of a commit / collision pass.
struct Tally {
  double w_absorbed, w_coll, w_particles;
  double pad;
  unsigned long long n_absorbed[kMaxSpecies];
  unsigned long long n_coll[kMaxSpecies];
  unsigned long long n_ionized, n_errors, n_crossings, n_substeps, n_over_range, n_overflow;
  unsigned long long append[kMaxSpecies];
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
  int32_t commit;
  double* wall_bot;
  double* wall_top;
  double* wall_side;
  Tally* tally;
  MccDev mcc;
  int32_t* hist;     // per-cell counts of the survivors (commit), or null
};

// One Crank-Nicolson field solve.  Optional outputs (null = skipped): the
// residual partials against the previous iterate, the next half-step field,
// and the reset of the consumed currents.
struct SolveArgs {
  const double *ur0, *uz0, *h0;
  double *Ir, *Iz;
  double vhalf, vnext;
  double *ur1, *uz1, *h1;
  const double *ur_old, *uz_old;
  double* part;         // [2 * nr]: per row sum w (u1 - u_old)^2, sum w u1^2
  double *ur_h, *uz_h;  // (u0 + u1) / 2
  float *ur_hf, *uz_hf;
  int32_t zero_I;
};

constexpr int kRedBlocks = 256;  // partial-sum blocks of the field reductions

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
  double* work0;    // [nr][nz]
  double* work1;    // [nr][nz]
  double* partial;  // reduction partials
};

struct Ctx {
  ecpic_grid_desc g;
  ecpic_precision prec;
  hipStream_t stream;
  MapP m;
  std::string err;
  std::vector<Species> sp;
  // fields (FP64) at t^n, t^{n-1}, the current iterate, the previous iterate
  double *ur, *uz, *h, *ur_prev, *uz_prev;
  double *ur_it, *uz_it, *h_it;    // u^{n+1,(k)}, h^{n+1,(k)}
  double *ur_nx, *uz_nx, *h_nx;    // u^{n+1,(k+1)} being produced
  double *ur_half, *uz_half;       // half-step field of the current push
  float *ur_half_f, *uz_half_f;    // FP32 copy (mixed path)
  double *ur_half2, *uz_half2;     // half-step field of the next push
  float *ur_half_f2, *uz_half_f2;
  double* part_host;               // pinned host copy of reduction partials
  double *Ir, *Iz;                 // currents
  double *wall_bot, *wall_top, *wall_side;
  int32_t* hist;                   // per-cell counts [nr*nz + 1]
  int32_t* offs;                   // per-cell offsets [nr*nz + 1]
  int32_t* scan_part;              // scan block sums
  Tally* tally;                    // device tallies, kSpread copies
  int32_t* queue = nullptr;        // slow-pass particle queues, one per species
  int64_t queue_cap = 0;           // entries per species
  hipStream_t aux[kMaxSpecies] = {};  // slow passes overlap the next fast pass
  hipEvent_t ev_fast[kMaxSpecies] = {}, ev_slow[kMaxSpecies] = {};
  int32_t* qcount = nullptr;       // queue lengths [kMaxSpecies][kSpread][kLineInts]
  Tally* tally_host;               // pinned host mirror of the copies
  double* red_host;                // pinned host reduction results
  SolverDev sol;
  double t = 0.0;
  int64_t step = 0;
  ecpic_mcc_desc mcc{};
  double numax[kMaxSpecies] = {0, 0, 0, 0};  // null-collision rate per species
  // learned guess
  uint16_t* nn_w = nullptr;
  float nn_norm[9] = {1, 1, 1, 1, 1, 1, 1, 1, 1};
  bool nn_ready = false;
  void* nn_ws = nullptr;           // activation workspace
  size_t nn_ws_bytes = 0;
  // event timing of the hot kernels
  bool prof_on = false;
  ecpic_profile prof{};
  struct Pending {
    hipEvent_t a, b;
    int kind;
    double bytes;
    int64_t particles;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> ev_pool;
};

// ---- launchers (stream-ordered, no synchronisation) ----
// push
// fast pass over all particles of a species, then the slow pass over the
// ones it queued (cell crossers, failed solves).  queue holds kSpread
// segments of queue_seg entries; qcount (kSpread counters, kLineInts apart)
// must be zero on entry.  tally points at kSpread copies.
hipError_t launch_push_fast(const PushArgs& a, int32_t* queue, int64_t queue_seg,
                            int32_t* qcount, hipStream_t s);
hipError_t launch_push_slow(const PushArgs& a, int32_t* queue, int64_t queue_seg,
                            int32_t* qcount, hipStream_t s);
// entries per queue segment for n particles
inline int64_t queue_segment(int64_t n) {
  const int64_t nb = (n + kBlock - 1) / kBlock;
  return ((nb + kSpread - 1) / kSpread) * kBlock;
}
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
hipError_t field_solve(const Ctx& c, const SolveArgs& a, hipStream_t s);
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
hipError_t launch_kinetic(const Species& sp, int mixed, double* out, hipStream_t s);
hipError_t launch_node_charge(const Ctx& c, double* q, hipStream_t s);
hipError_t launch_zero(double* p, int64_t n, hipStream_t s);
hipError_t launch_zero_i(int32_t* p, int64_t n, hipStream_t s);
hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);

}  // namespace ecpic
