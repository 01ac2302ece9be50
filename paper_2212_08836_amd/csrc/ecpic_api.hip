// ecpic_api.hip -- host runtime behind the C ABI of include/ecpic.h: context
// and species management, the Picard driver of the implicit step (Sec. 2.1:
// the coupled field/orbit system is solved by Picard iteration), and the
// setup of the separable H_theta solver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ecpic_internal.h"

using namespace ecpic;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kKB = 1.380649e-23;  // Boltzmann constant [J/K]
// layout of the device / pinned-host reduction buffer (doubles)
constexpr int kOffRes = 0;                        // 2 per solve block, residual partials
constexpr int kOffFE = 2 * kResParts;             // 2 kRedBlocks field energy
constexpr int kOffEx = kOffFE + 2 * kRedBlocks;   // kRedBlocks exchange
constexpr int kOffKE = kOffEx + kRedBlocks;       // kMaxSpecies kinetic energies
constexpr int kOffSc = kOffKE + 8;                // a few scalars
constexpr int kPartLen = kOffSc + 16;

ecpic_status fail(Ctx& c, ecpic_status s, const std::string& msg) {
  c.err = msg;
  return s;
}

double drive(const ecpic_grid_desc& g, double t) { return drive_voltage(g, t); }

double r_of_xi(const MapP& m, double xi) {
  if (xi < m.xi_a) return 2.0 * m.s * std::sqrt(xi * m.xi_a);
  return m.s * (xi + m.xi_a);
}

// Device memory layout.  One walk over every device array computes the
// size of the region (base null); a second assigns the arrays from a region
// of that size.  Arrays start on 256-byte boundaries.
struct Carver {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  void take(T** p, size_t n) {
    off = (off + 255) & ~(size_t)255;
    if (base) *p = reinterpret_cast<T*>(base + off);
    off += std::max<size_t>(n, 1) * sizeof(T);
  }
};

void carve_species_buf(const Ctx& c, Carver& k, SpecDev& d, int64_t cap) {
  const size_t n = (size_t)std::max<int64_t>(cap, 1);
  if (c.prec == ECPIC_FP64) {
    k.take(&d.xi, n);
    k.take(&d.eta, n);
    k.take(&d.vr, n);
    k.take(&d.vt, n);
    k.take(&d.vz, n);
  } else {
    k.take(&d.cell, n);
    k.take(&d.fa, n);
    k.take(&d.fb, n);
    k.take(&d.fvr, n);
    k.take(&d.fvt, n);
    k.take(&d.fvz, n);
  }
  k.take(&d.uid, n);
}

// queue entries per species and kind for a species of capacity cap
int64_t queue_len(int64_t cap) { return kSpread * queue_segment(cap); }

// int32 words of the block counts ecpic_read_particles needs at capacity cap
int64_t read_scratch_len(int64_t cap) {
  const int64_t nb = (cap + kBlock - 1) / kBlock;
  return nb + 1 + (nb + 1023) / 1024 + 2;
}

void carve_queues(Ctx& c, Carver& k, int64_t max_cap, int32_t nsp) {
  const int64_t ql = queue_len(max_cap);
  k.take(&c.queue, (size_t)ql * nsp * 2);   // slow queues, then collision lists
  k.take(&c.qrec, (size_t)ql * nsp * 5);    // records of slow-queue entries
  k.take(&c.rd_scratch, (size_t)read_scratch_len(max_cap));
  if (k.base) {
    c.queue_cap = ql;
    c.queue_species = nsp;
    c.rd_scratch_len = read_scratch_len(max_cap);
  }
}

int64_t n_edges_r(const Ctx& c) { return (int64_t)c.g.nr * (c.g.nz + 1); }
int64_t n_edges_z(const Ctx& c) { return (int64_t)(c.g.nr + 1) * c.g.nz; }
int64_t n_cells(const Ctx& c) { return (int64_t)c.g.nr * c.g.nz; }
int64_t n_nodes(const Ctx& c) { return (int64_t)(c.g.nr + 1) * (c.g.nz + 1); }

// Every device array of the context and of its species so far.
void carve_all(Ctx& c, Carver& k) {
  const int nr = c.g.nr, nz = c.g.nz;
  const size_t nur = (size_t)n_edges_r(c), nuz = (size_t)n_edges_z(c), nh = (size_t)n_cells(c);
  double** er[] = {&c.ur, &c.ur_prev, &c.ur_it, &c.ur_nx, &c.ur_half, &c.Ir, &c.Ir_alt,
                   &c.ur_half2, &c.ur_spare};
  double** ez[] = {&c.uz, &c.uz_prev, &c.uz_it, &c.uz_nx, &c.uz_half, &c.Iz, &c.Iz_alt,
                   &c.uz_half2, &c.uz_spare};
  for (double** p : er) k.take(p, nur);
  for (double** p : ez) k.take(p, nuz);
  double** eh[] = {&c.h, &c.h_prev, &c.h_it, &c.h_nx};
  for (double** p : eh) k.take(p, nh);
  // wall charge: bottom, top and side in one array (the layout of the
  // committing iterations' scratch, which is added into it)
  k.take(&c.wall_bot, (size_t)wall_len(c));
  k.take(&c.wall_scr, 2 * (size_t)wall_len(c));
  if (c.prec == ECPIC_MIXED) {
    k.take(&c.ur_half_f, nur);
    k.take(&c.uz_half_f, nuz);
    k.take(&c.ur_half_f2, nur);
    k.take(&c.uz_half_f2, nuz);
  }
  k.take(&c.hist, nh + 1);
  k.take(&c.offs, nh + 1);
  k.take(&c.scan_part, (nh + 1023) / 1024 + 2);
  k.take(&c.tally, 2 * kSpread);
  k.take(&c.qcount, 2 * kQCount);
  k.take(&c.stop, 2);
  SolverDev& S = c.sol;
  k.take(&S.rh, nr);
  k.take(&S.wr, nr);
  k.take(&S.wz, nr);
  k.take(&S.area, nr);
  k.take(&S.Q, (size_t)nz * nz);
  k.take(&S.Qt, (size_t)nz * nz);
  k.take(&S.tri_lo, (size_t)nz * nr);
  k.take(&S.tri_inv, (size_t)nz * nr);
  k.take(&S.tri_up, nr);
  k.take(&S.prof, nr + 1);
  if (c.g.port_i > 0) {
    const size_t mp = (size_t)(nr - c.g.port_i);
    k.take(&S.port_pc, 4 * (size_t)nr);
    k.take(&c.port_hb, nr);
    if (c.g.model == ECPIC_MODEL_EM) {
      k.take(&S.port_F, mp * mp);
      k.take(&S.port_q0, nz);
      // z, then the coupling's mode parts ([32][m] at most)
      k.take(&S.port_z, mp * 33);
    }
  }
  k.take(&S.work0, nh);
  k.take(&S.work1, nh);
  k.take(&S.partial, kPartLen);
  const size_t nn = (size_t)n_nodes(c);
  k.take(&c.q_node, nn);
  k.take(&c.q0, nn);
  k.take(&c.gq0, nn);
  k.take(&c.cons_dev, 4);
  k.take(&c.circ, kCircLen);
  k.take(&c.nn_w, (size_t)ecpic_nn_param_count());
  char* gws = nullptr;
  k.take(&gws, nn_guess_ws_bytes(c));
  if (k.base) {
    c.nn_gws = gws;
    c.nn_gws_bytes = nn_guess_ws_bytes(c);
  }
  int64_t max_cap = 0;
  for (Species& s : c.sp) {
    carve_species_buf(c, k, s.d[0], s.desc.capacity);
    carve_species_buf(c, k, s.d[1], s.desc.capacity);
    max_cap = std::max<int64_t>(max_cap, s.desc.capacity);
  }
  carve_queues(c, k, max_cap, std::max<int32_t>((int32_t)c.sp.size(), 1));
  if (c.jfnk_m > 0) {
    k.take(&c.jf_vec, (size_t)(c.jfnk_m + 7) * (nur + nuz));
    k.take(&c.jf_part, (size_t)(kMaxKrylov + 1) * kJfBlocks);
  }
}

// a device allocation of the library's own, freed at destroy
template <typename T>
hipError_t owned_alloc(Ctx& c, T** p, size_t n) {
  const hipError_t e = hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T));
  if (e == hipSuccess) c.owned.push_back((void*)*p);
  return e;
}

SpecDev view(Species& s) {
  SpecDev d = s.d[s.cur];
  d.n = s.n;
  d.cap = s.desc.capacity;
  d.q = s.desc.q;
  d.m = s.desc.m;
  d.w = s.desc.weight;
  d.mobile = s.desc.mobile;
  return d;
}

// the species' other buffer, sized like the current one (a committing Picard
// iteration writes the new state there); the uid array stays the current
// one: a commit keeps every particle in its slot, so both buffers share it
// (a flip swaps the uid arrays along with the buffers)
SpecDev other_view(Species& s) {
  SpecDev d = view(s);
  const SpecDev& o = s.d[1 - s.cur];
  d.xi = o.xi;
  d.eta = o.eta;
  d.vr = o.vr;
  d.vt = o.vt;
  d.vz = o.vz;
  d.cell = o.cell;
  d.fa = o.fa;
  d.fb = o.fb;
  d.fvr = o.fvr;
  d.fvt = o.fvt;
  d.fvz = o.fvz;
  return d;
}

// Geometry and separable-solver tables (host FP64), uploaded once.
hipError_t setup_solver(Ctx& c) {
  const int nr = c.g.nr, nz = c.g.nz;
  const MapP& m = c.m;
  const double dt = c.g.dt, eps = c.g.eps, mu = c.g.mu;
  std::vector<double> rn(nr + 1), rh(nr), ell(nr), area(nr), azs(nr), wr(nr), wz(nr);
  for (int i = 0; i <= nr; ++i) rn[i] = r_of_xi(m, i);
  rn[nr] = c.g.R;
  for (int i = 0; i < nr; ++i) {
    rh[i] = r_of_xi(m, i + 0.5);
    ell[i] = rn[i + 1] - rn[i];
    area[i] = ell[i] * m.dz;
    const double rm = i > 0 ? rh[i - 1] : 0.0;
    azs[i] = kPi * (rh[i] * rh[i] - rm * rm);
    wr[i] = eps * 2.0 * kPi * rh[i] * m.dz / ell[i];
    wz[i] = eps * azs[i] / m.dz;
  }
  // tridiagonal radial part T and the z-coupling weights G
  std::vector<double> Td(nr), To(nr, 0.0), G(nr);
  for (int i = 0; i < nr; ++i) {
    const double mi = 2.0 * kPi * rh[i];
    const double Dz = 2.0 * wz[i] / dt;
    Td[i] = mi * 2.0 * mu * area[i] / dt + mi * mi / Dz;
    if (i + 1 < nr) {
      const double Dz1 = 2.0 * wz[i + 1] / dt;
      Td[i] += mi * mi / Dz1;
    }
    if (i > 0) To[i] = -(2.0 * kPi * rh[i - 1]) * mi / Dz;
    const double Dr = 2.0 * wr[i] / dt;
    G[i] = mi * mi / Dr;
  }
  std::vector<double> Q((size_t)nz * nz), Qt((size_t)nz * nz);
  std::vector<double> lo((size_t)nz * nr, 0.0), inv((size_t)nz * nr);
  if (c.g.model == ECPIC_MODEL_ES) {
    // Electrostatic model: the Poisson operator on the free nodes is
    // W_r (x) I + diag(wz) (x) T_z with T_z the Dirichlet second difference
    // over the nz - 1 free rows, diagonalised by the orthonormal DST-I
    // S[j][k] = sqrt(2/nz) sin(pi (j+1)(k+1) / nz) (symmetric, its own
    // inverse); per mode a tridiagonal system in r with the grounded side
    // wall as the Dirichlet end.
    const int nf = nz - 1;
    for (int k = 0; k < nf; ++k)
      for (int j = 0; j < nf; ++j) {
        const double v = std::sqrt(2.0 / nz) * std::sin(kPi * (j + 1.0) * (k + 1.0) / nz);
        Q[(size_t)k * nf + j] = v;
        Qt[(size_t)j * nf + k] = v;
      }
    for (int i = 0; i < nr; ++i) To[i] = (i > 0) ? -wr[i - 1] : 0.0;
    for (int k = 0; k < nf; ++k) {
      const double lam = 2.0 - 2.0 * std::cos(kPi * (k + 1.0) / nz);
      auto diag = [&](int i) { return wr[i] + (i > 0 ? wr[i - 1] : 0.0) + lam * wz[i]; };
      double cp = diag(0);
      inv[(size_t)k * nr] = 1.0 / cp;
      for (int i = 1; i < nr; ++i) {
        const double l = To[i] / cp;
        cp = diag(i) - l * To[i];
        lo[(size_t)k * nr + i] = l;
        inv[(size_t)k * nr + i] = 1.0 / cp;
      }
    }
  } else {
    // orthonormal DCT-II diagonalising the Neumann second difference
    for (int k = 0; k < nz; ++k) {
      const double a = (k == 0) ? std::sqrt(1.0 / nz) : std::sqrt(2.0 / nz);
      for (int j = 0; j < nz; ++j) {
        const double v = a * std::cos(kPi * k * (2.0 * j + 1.0) / (2.0 * nz));
        Q[(size_t)k * nz + j] = v;
        Qt[(size_t)j * nz + k] = v;
      }
    }
    for (int k = 0; k < nz; ++k) {
      const double lam = 2.0 - 2.0 * std::cos(kPi * k / nz);
      double cp = Td[0] + lam * G[0];
      inv[(size_t)k * nr] = 1.0 / cp;
      for (int i = 1; i < nr; ++i) {
        const double l = To[i] / cp;
        cp = Td[i] + lam * G[i] - l * To[i];
        lo[(size_t)k * nr + i] = l;
        inv[(size_t)k * nr + i] = 1.0 / cp;
      }
    }
  }
  // TEM port (Sec. 2.1, Eqs. (5), (7)): the electrostatic wall profile, the
  // per-edge tables, and for EM the Woodbury coupling of the port's diagonal
  // d_i = M_i^2 g_i / 2 on the wall cells (i, 0), i >= ip:
  // F = (D^-1 + U^T A0^-1 U)^-1, where the port block of A0^-1 is
  // sum_k Q[k][0]^2 T_k^-1 restricted to the port rows.
  const int ip = c.g.port_i;
  std::vector<double> prof(nr + 1), pc, Fm, q0;
  for (int i = 0; i <= nr; ++i) prof[i] = (i < nr) ? 1.0 : 0.0;
  if (ip > 0) {
    const int mp = nr - ip;
    const double lnr = std::log(c.g.R / rn[ip]);
    for (int i = 0; i <= nr; ++i) prof[i] = (i <= ip) ? 1.0 : std::log(c.g.R / rn[i]) / lnr;
    prof[nr] = 0.0;
    const double eta = std::sqrt(mu / (eps * c.g.port_eps));
    pc.assign(4 * (size_t)nr, 0.0);
    std::vector<double> dg(mp);
    for (int i = ip; i < nr; ++i) {
      const double M = 2.0 * kPi * rh[i];
      const double kap = std::log(rn[i + 1] / rn[i]) / lnr;
      const double g = 1.0 / (0.5 * wr[i] / dt + M / (2.0 * eta * ell[i]));
      pc[kPortG * (size_t)nr + i] = g;
      pc[kPortA * (size_t)nr + i] = M * kap / (2.0 * eta * ell[i]);
      pc[kPortK * (size_t)nr + i] = kap;
      pc[kPortIEL * (size_t)nr + i] = 1.0 / (eta * ell[i]);
      dg[i - ip] = 0.5 * M * M * g;
    }
    if (c.g.model == ECPIC_MODEL_EM) {
      std::vector<double> C((size_t)mp * mp, 0.0), y(nr), x(nr + 1);
      q0.resize(nz);
      for (int k = 0; k < nz; ++k) {
        q0[k] = Q[(size_t)k * nz];
        const double w = q0[k] * q0[k];
        const double* L = lo.data() + (size_t)k * nr;
        const double* Iv = inv.data() + (size_t)k * nr;
        for (int p = 0; p < mp; ++p) {
          // T_k x = e_{ip+p}: forward from row ip+p, backward down to row ip
          for (int i = ip; i < ip + p; ++i) y[i] = 0.0;
          y[ip + p] = 1.0;
          for (int i = ip + p + 1; i < nr; ++i) y[i] = -L[i] * y[i - 1];
          x[nr] = 0.0;
          for (int i = nr - 1; i >= ip; --i)
            x[i] = Iv[i] * (y[i] - (i + 1 < nr ? To[i + 1] : 0.0) * x[i + 1]);
          for (int q = 0; q < mp; ++q) C[(size_t)q * mp + p] += w * x[ip + q];
        }
      }
      for (int q = 0; q < mp; ++q) C[(size_t)q * mp + q] += 1.0 / dg[q];
      // F = C^-1 by Cholesky (C is SPD), column by column
      for (int j = 0; j < mp; ++j) {
        for (int q = 0; q < j; ++q) {
          double v = C[(size_t)j * mp + q];
          for (int t = 0; t < q; ++t) v -= C[(size_t)j * mp + t] * C[(size_t)q * mp + t];
          C[(size_t)j * mp + q] = v / C[(size_t)q * mp + q];
        }
        double d = C[(size_t)j * mp + j];
        for (int t = 0; t < j; ++t) d -= C[(size_t)j * mp + t] * C[(size_t)j * mp + t];
        if (!(d > 0.0)) return hipErrorInvalidValue;
        C[(size_t)j * mp + j] = std::sqrt(d);
      }
      Fm.assign((size_t)mp * mp, 0.0);
      std::vector<double> b(mp);
      for (int col = 0; col < mp; ++col) {
        for (int q = 0; q < mp; ++q) b[q] = (q == col) ? 1.0 : 0.0;
        for (int q = 0; q < mp; ++q) {
          double v = b[q];
          for (int t = 0; t < q; ++t) v -= C[(size_t)q * mp + t] * b[t];
          b[q] = v / C[(size_t)q * mp + q];
        }
        for (int q = mp - 1; q >= 0; --q) {
          double v = b[q];
          for (int t = q + 1; t < mp; ++t) v -= C[(size_t)t * mp + q] * b[t];
          b[q] = v / C[(size_t)q * mp + q];
        }
        for (int q = 0; q < mp; ++q) Fm[(size_t)q * mp + col] = b[q];
      }
    }
  }
  SolverDev& S = c.sol;
  hipError_t e;
  auto up = [&](double* d, const std::vector<double>& h) -> hipError_t {
    return hipMemcpyAsync(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice,
                          c.stream);
  };
  if ((e = up(S.prof, prof)) != hipSuccess) return e;
  if (ip > 0 && (e = up(S.port_pc, pc)) != hipSuccess) return e;
  if (!Fm.empty() && (e = up(S.port_F, Fm)) != hipSuccess) return e;
  if (!q0.empty() && (e = up(S.port_q0, q0)) != hipSuccess) return e;
  if ((e = up(S.rh, rh)) != hipSuccess) return e;
  if ((e = up(S.wr, wr)) != hipSuccess) return e;
  if ((e = up(S.wz, wz)) != hipSuccess) return e;
  if ((e = up(S.area, area)) != hipSuccess) return e;
  if ((e = up(S.Q, Q)) != hipSuccess) return e;
  if ((e = up(S.Qt, Qt)) != hipSuccess) return e;
  if ((e = up(S.tri_lo, lo)) != hipSuccess) return e;
  if ((e = up(S.tri_inv, inv)) != hipSuccess) return e;
  if ((e = up(S.tri_up, To)) != hipSuccess) return e;
  // the host vectors die here: wait for the copies
  return hipStreamSynchronize(c.stream);
}

hipError_t zero(double* p, int64_t n, hipStream_t s) { return launch_zero(p, n, s); }

// -- event timing: a start/stop pair around a launch, resolved after a sync --
hipEvent_t get_event(Ctx& c) {
  if (c.ev_pool.empty()) {
    // timing only: no system-scope cache writeback at each record
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = c.ev_pool.back();
  c.ev_pool.pop_back();
  return e;
}

struct Timed {
  Ctx& c;
  hipStream_t st;
  hipEvent_t a = nullptr;
  int kind;
  double bytes;
  int64_t particles;
  Timed(Ctx& cc, int k, double b, int64_t n, hipStream_t s = nullptr)
      : c(cc), st(s ? s : cc.stream), kind(k), bytes(b), particles(n) {
    if (c.prof_mask & (1u << k)) {
      c.count_pending.push_back({k, n, c.cur_tag});
      if (c.prof_seq[k]++ % (uint64_t)c.prof_every == 0) {
        a = get_event(c);
        if (a) (void)hipEventRecord(a, st);
      }
    }
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = get_event(c);
    if (!b) return;
    (void)hipEventRecord(b, st);
    c.pending.push_back({a, b, kind, bytes, particles, c.cur_tag});
  }
};

// fold finished pairs into the totals; unfinished ones stay pending (all
// are finished once the stream has been synchronised)
void collect(Ctx& c) {
  // launch counts: those of an iteration enqueued ahead are dropped by
  // drop_tag before this runs if the iteration turns out not to be needed
  for (const auto& q : c.count_pending) {
    c.prof.calls[q.kind] += 1;
    c.prof.call_particles[q.kind] += q.particles;
  }
  c.count_pending.clear();
  std::vector<Ctx::Pending> keep;
  for (auto& p : c.pending) {
    if (hipEventQuery(p.b) == hipErrorNotReady) {
      keep.push_back(p);
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c.prof.launches[p.kind] += 1;
      c.prof.ms[p.kind] += ms;
      c.prof.bytes[p.kind] += p.bytes;
      c.prof.particles[p.kind] += p.particles;
    }
    c.ev_pool.push_back(p.a);
    c.ev_pool.push_back(p.b);
  }
  c.pending.swap(keep);
  std::vector<hipEvent_t> still;
  for (hipEvent_t e : c.ev_dropped) {
    if (hipEventQuery(e) == hipErrorNotReady)
      still.push_back(e);
    else
      c.ev_pool.push_back(e);
  }
  c.ev_dropped.swap(still);
}

// forget the timings of launches enqueued under `tag` (a speculative
// iteration that was not needed); their events still complete normally
void drop_tag(Ctx& c, int tag) {
  std::vector<Ctx::Count> kc;
  for (const auto& q : c.count_pending)
    if (q.tag != tag) kc.push_back(q);
  c.count_pending.swap(kc);
  std::vector<Ctx::Pending> keep;
  for (auto& p : c.pending) {
    if (p.tag == tag) {
      c.ev_dropped.push_back(p.a);
      c.ev_dropped.push_back(p.b);
    } else {
      keep.push_back(p);
    }
  }
  c.pending.swap(keep);
}

// algorithmic bytes per particle of a push pass: the state read once
double state_bytes(const Ctx& c) { return c.prec == ECPIC_FP64 ? 40.0 : 24.0; }

MccDev make_mcc(Ctx& c, int sid, int64_t step, bool to_other = false) {
  MccDev d;
  std::memset(&d, 0, sizeof(d));
  const ecpic_mcc_desc& M = c.mcc;
  if (!M.enabled) return d;
  const int role = (sid == M.electron_sid) ? 1 : (sid == M.ion_sid ? 2 : 0);
  if (!role) return d;
  Species& s = c.sp[sid];
  if (!s.desc.mobile) return d;
  d.enabled = 1;
  d.role = role;
  d.numax = c.numax[sid];
  d.pnull = 1.0 - std::exp(-d.numax * c.g.dt);
  d.n_gas = M.n_gas;
  d.m_gas = M.m_gas;
  d.sig_gas = std::sqrt(kKB * M.t_gas / M.m_gas);
  d.eps_max_ev = M.eps_max_ev;
  d.seed = M.seed;
  d.step = step;
  d.base_self = s.n;
  if (role == 1 && M.ion_sid >= 0 && M.ion_sid < (int)c.sp.size()) {
    Species& ion = c.sp[M.ion_sid];
    // a committing pass into the other buffers appends ions there too,
    // unless the ion species is immobile (its buffers never flip)
    d.partner = (to_other && ion.desc.mobile) ? other_view(ion) : view(ion);
    d.partner.sid = M.ion_sid;
    d.base_partner = ion.n;
    d.sig_ion = std::sqrt(kKB * M.t_gas / ion.desc.m);
  }
  return d;
}

PushArgs push_args(Ctx& c, int sid, int commit) {
  PushArgs a;
  std::memset(&a, 0, sizeof(a));
  a.m = c.m;
  a.ur = c.ur_half;
  a.uz = c.uz_half;
  a.urf = c.ur_half_f;
  a.uzf = c.uz_half_f;
  a.Ir = c.Ir;
  a.Iz = c.Iz;
  a.s = view(c.sp[sid]);
  a.s.sid = sid;
  a.out = a.s;
  a.commit = commit;
  a.wall_bot = c.wall_bot;
  a.wall_top = c.wall_top;
  a.wall_side = c.wall_side;
  a.tally = c.tally;
  return a;
}

// One pass over all species, two species per launch, all on the context
// stream.  Inside a step the currents, queue counters and tallies were
// already reset (by the guess kernel, the last field solve and the residual
// kernel); a standalone pass (prezeroed false) resets them itself.
// A committing pass with to_other writes the new states into the species'
// other buffers (the current ones stay as they are until the host accepts
// it) and its wall charge into the scratch of parity `set`; its tallies go
// to tally set `set` in any case.
ecpic_status pass(Ctx& c, int commit, bool with_mcc, int64_t step, bool prezeroed,
                  bool guarded = false, bool deposit = true, bool to_other = false,
                  int set = 0) {
  if (!prezeroed) {
    HIPCHK(zero(c.Ir, n_edges_r(c), c.stream));
    HIPCHK(zero(c.Iz, n_edges_z(c), c.stream));
    if (commit) HIPCHK(launch_zero_tally(c, c.stream));
    HIPCHK(launch_zero_i(c.qcount, 2 * kQCount, c.stream));
  }
  // append offsets of every species are taken before any pass appends
  std::vector<MccDev> mcc(c.sp.size());
  for (size_t s = 0; s < c.sp.size(); ++s) {
    std::memset(&mcc[s], 0, sizeof(MccDev));
    if (commit && with_mcc) mcc[s] = make_mcc(c, (int)s, step, to_other);
  }
  std::vector<int> act;
  for (size_t s = 0; s < c.sp.size(); ++s)
    if (c.sp[s].desc.mobile && c.sp[s].n > 0) act.push_back((int)s);
  for (size_t b = 0; b < act.size(); b += 2) {
    PassArgs P;
    std::memset(&P, 0, sizeof(P));
    P.nsp = (b + 1 < act.size()) ? 2 : 1;
    P.qcap = c.queue_cap;
    P.queue_waves = c.queue_waves;
    double bytes = 0.0;
    int64_t parts = 0;
    for (int q = 0; q < P.nsp; ++q) {
      const int s = act[b + q];
      PushArgs& a = P.a[q];
      a = push_args(c, s, commit);
      a.mcc = mcc[s];
      a.stop = guarded ? c.stop : nullptr;
      a.tally = tally_set(c, set);
      if (to_other) {
        a.out = other_view(c.sp[s]);
        a.out.sid = s;
        double* w = wall_scratch(c, set);
        a.wall_bot = w;
        a.wall_top = w + (c.g.nr + 1);
        a.wall_side = w + 2 * (c.g.nr + 1);
      }
      if (!deposit) {
        a.Ir = nullptr;
        a.Iz = nullptr;
      }
      P.queue[q] = c.queue + (int64_t)s * c.queue_cap;
      P.qrec[q] = c.qrec + (int64_t)s * 5 * c.queue_cap;
      P.cqueue[q] = c.queue + (int64_t)(c.queue_species + s) * c.queue_cap;
      P.cqcount[q] = c.qcount + kQCount + s * kSpread * kLineInts;
      P.qcount[q] = c.qcount + s * kSpread * kLineInts;
      P.qseg[q] = queue_segment(c.sp[s].n);
      // iteration: state read; commit: state read and written, and the id
      // read for the collision draw (both buffers share the ids)
      bytes += (commit ? 2.0 * state_bytes(c) + 8.0 : state_bytes(c)) * (double)c.sp[s].n;
      parts += c.sp[s].n;
    }
    {
      // a committing Picard iteration deposits; a separate commit does not
      const int kind = !commit ? ECPIC_K_PUSH
                               : ((to_other && deposit) ? ECPIC_K_PUSH_COMMIT : ECPIC_K_COMMIT);
      Timed tm(c, kind, bytes, parts);
      HIPCHK(launch_push_fast(P, deposit, c.stream));
    }
    {
      Timed tm(c, commit ? ECPIC_K_COMMIT_SLOW : ECPIC_K_PUSH_SLOW, 0.0, 0);
      if (commit && with_mcc)
        HIPCHK(launch_slow_collide(P, c.stream));
      else
        HIPCHK(launch_push_slow(P, c.stream));
    }
  }
  return ECPIC_OK;
}

// After a commit/collision pass: fetch the tally and grow species counts.
ecpic_status finish_tally(Ctx& c, Tally& t) {
  HIPCHK(hipMemcpyAsync(c.tally_host, c.tally, kSpread * sizeof(Tally), hipMemcpyDeviceToHost,
                        c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  t = c.tally_host[0];
  for (int q = 1; q < kSpread; ++q) {
    const Tally& u = c.tally_host[q];
    t.w_absorbed += u.w_absorbed;
    t.w_coll += u.w_coll;
    t.w_particles += u.w_particles;
    for (int s = 0; s < kMaxSpecies; ++s) {
      t.n_absorbed[s] += u.n_absorbed[s];
      t.n_coll[s] += u.n_coll[s];
      t.append[s] += u.append[s];
    }
    t.n_ionized += u.n_ionized;
    t.n_errors += u.n_errors;
    t.n_crossings += u.n_crossings;
    t.n_substeps += u.n_substeps;
    t.n_over_range += u.n_over_range;
    t.n_overflow += u.n_overflow;
  }
  collect(c);
  ecpic_status rc = ECPIC_OK;
  for (size_t s = 0; s < c.sp.size(); ++s) {
    const int64_t add = (int64_t)t.append[s];
    int64_t n = c.sp[s].n + add;
    if (n > c.sp[s].desc.capacity) n = c.sp[s].desc.capacity;
    c.sp[s].n = n;
  }
  if (t.n_overflow) rc = fail(c, ECPIC_ECAPACITY, "species capacity exceeded by ionisation");
  return rc;
}

}  // namespace

namespace ecpic {

double drive_voltage(const ecpic_grid_desc& g, double t) {
  double v = 0.0;
  if (g.drive_t_end > 0.0 && t >= g.drive_t_end) return 0.0;
  for (int k = 0; k < g.n_drive && k < 32; ++k)
    v += g.drive_amp[k] * std::sin(2.0 * kPi * g.drive_freq[k] * t + g.drive_phase[k]);
  return v;
}

// Assign every device array (from the bound workspace, or from one block of
// the library's own), upload the solver tables and clear the state.  Done
// once, at the first call that needs the device.
ecpic_status materialise(Ctx& c) {
  if (c.materialised) return ECPIC_OK;
  Carver dry;
  carve_all(c, dry);
  char* base = nullptr;
  if (c.ws) {
    if (c.ws_bytes < dry.off)
      return fail(c, ECPIC_ENOMEM, "workspace smaller than ecpic_workspace_size reports");
    base = static_cast<char*>(c.ws);
  } else {
    if (hipMalloc(&c.own_block, dry.off) != hipSuccess) {
      c.own_block = nullptr;
      return fail(c, ECPIC_ENOMEM, "device allocation failed");
    }
    base = static_cast<char*>(c.own_block);
  }
  Carver k{base};
  carve_all(c, k);
  c.wall_top = c.wall_bot + (c.g.nr + 1);
  c.wall_side = c.wall_top + (c.g.nr + 1);
  HIPCHK(setup_solver(c));
  const int64_t nur = n_edges_r(c), nuz = n_edges_z(c), nh = n_cells(c);
  double* zs[] = {c.ur, c.uz, c.h, c.ur_prev, c.uz_prev, c.ur_it, c.uz_it, c.h_it,
                  c.ur_half, c.uz_half, c.Ir, c.Iz, c.ur_half2, c.uz_half2, c.h_prev,
                  c.Ir_alt, c.Iz_alt};
  int64_t zn[] = {nur, nuz, nh, nur, nuz, nur, nuz, nh, nur, nuz, nur, nuz, nur, nuz, nh, nur, nuz};
  for (int q = 0; q < 17; ++q) HIPCHK(launch_zero(zs[q], zn[q], c.stream));
  HIPCHK(launch_zero_i(c.stop, 2, c.stream));
  HIPCHK(launch_zero(c.circ, kCircLen, c.stream));
  if (c.port_hb) HIPCHK(launch_zero(c.port_hb, c.g.nr, c.stream));
  HIPCHK(launch_zero_i(c.qcount, 2 * kQCount, c.stream));
  HIPCHK(launch_zero(c.wall_bot, wall_len(c), c.stream));
  HIPCHK(launch_zero(c.wall_scr, 2 * wall_len(c), c.stream));
  HIPCHK(launch_zero_tally(c, c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  c.materialised = true;
  return ECPIC_OK;
}

}  // namespace ecpic

namespace {

#define ENSURE_DEVICE(c)                          \
  do {                                            \
    const ecpic_status r_ = materialise(c);       \
    if (r_ != ECPIC_OK) return r_;                \
  } while (0)

}  // namespace

extern "C" {

const char* ecpic_status_string(ecpic_status s) {
  switch (s) {
    case ECPIC_OK: return "ok";
    case ECPIC_EINVAL: return "invalid argument";
    case ECPIC_ENOMEM: return "out of device memory";
    case ECPIC_EHIP: return "HIP runtime error";
    case ECPIC_ENOTCONV: return "Picard iteration did not converge";
    case ECPIC_EPUSH: return "particle push failed";
    case ECPIC_ECAPACITY: return "species capacity exceeded";
    case ECPIC_ERANGE: return "particle beyond the null-collision bound";
    case ECPIC_ENOTIMPL: return "not implemented";
  }
  return "unknown status";
}

const char* ecpic_last_error(const ecpic_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->c.err.c_str();
}

ecpic_status ecpic_create(const ecpic_grid_desc* g, ecpic_precision prec, void* stream,
                          ecpic_ctx** out) {
  if (!g || !out) return ECPIC_EINVAL;
  *out = nullptr;
  if (g->nr < 1 || g->nz < 1 || !(g->R > 0) || !(g->L > 0) || !(g->dt > 0) || !(g->eps > 0) ||
      !(g->mu > 0) || !(g->xi_axis >= 0) || g->xi_axis > g->nr || g->n_drive < 0 ||
      g->n_drive > 32 || !(g->drive_t_end >= 0) || (prec != ECPIC_FP64 && prec != ECPIC_MIXED) ||
      (g->model != ECPIC_MODEL_EM && g->model != ECPIC_MODEL_ES) ||
      !(g->blocking_cap >= 0.0) || !std::isfinite(g->blocking_cap) ||
      (g->model == ECPIC_MODEL_ES && g->nz < 2) ||
      !grid_fits(g->nr, g->nz) || g->port_i < 0 ||
      (g->port_i > 0 && (g->port_i >= g->nr || !(g->port_eps > 0.0) ||
                         !std::isfinite(g->port_eps))))
    return ECPIC_EINVAL;
  ecpic_ctx* x = new (std::nothrow) ecpic_ctx();
  if (!x) return ECPIC_ENOMEM;
  Ctx& c = x->c;
  c.g = *g;
  c.prec = prec;
  c.stream = (hipStream_t)stream;
  c.m.nr = g->nr;
  c.m.nz = g->nz;
  c.m.xi_a = g->xi_axis;
  c.m.s = g->R / (g->nr + g->xi_axis);
  c.m.inv_s = 1.0 / c.m.s;
  c.m.rsqrt_xa = g->xi_axis > 0 ? 1.0 / std::sqrt(g->xi_axis) : 0.0;
  c.m.dz = g->L / g->nz;
  c.m.inv_dz = 1.0 / c.m.dz;
  c.m.dt = g->dt;
  c.m.i_lin = (int)std::ceil(g->xi_axis);
  c.m.ip = g->port_i;
  // host memory the device writes or the host reads back (pinned); device
  // memory waits for the first use or a bound workspace
  bool ok = true;
  ok = ok && hipHostMalloc((void**)&c.tally_host, kSpread * sizeof(Tally)) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&c.red_host, 64 * sizeof(double)) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&c.part_host, kPartLen * sizeof(double)) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&c.cons_host, 4 * sizeof(unsigned long long)) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&c.jf_host, (kMaxKrylov + 1) * kJfBlocks * sizeof(double)) ==
                 hipSuccess;
  // written by kernels with system-scope stores and polled by the host
  ok = ok && hipHostMalloc((void**)&c.res_host, kMaxIter * sizeof(double),
                           hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&c.fin_host, sizeof(StepFinal),
                           hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&c.sort_total_host, kMaxSpecies * sizeof(int32_t)) == hipSuccess;
  ok = ok && hipHostGetDevicePointer((void**)&c.res_dev, c.res_host, 0) == hipSuccess;
  ok = ok && hipHostGetDevicePointer((void**)&c.fin_dev, c.fin_host, 0) == hipSuccess;
  if (!ok) {
    ecpic_destroy(x);
    return ECPIC_ENOMEM;
  }
  std::memset((void*)c.fin_host, 0, sizeof(StepFinal));
  for (int k = 0; k < kMaxIter; ++k) std::memcpy(&c.res_host[k], &kResPending, sizeof(double));
  // this device's address of the static scratch of ecpic_field_solve_noalloc
  if (hipGetDevice(&c.device) != hipSuccess || static_scratch_setup(c.device) != hipSuccess) {
    ecpic_destroy(x);
    return ECPIC_EHIP;
  }
  *out = x;
  return ECPIC_OK;
}

ecpic_status ecpic_destroy(ecpic_ctx* x) {
  if (!x) return ECPIC_EINVAL;
  Ctx& c = x->c;
  (void)hipStreamSynchronize(c.stream);
  // device arrays live in the bound workspace (the caller's) or in the
  // library's block, plus the allocations made after the first use
  if (c.own_block) (void)hipFree(c.own_block);
  for (void* p : c.owned) (void)hipFree(p);
  (void)hipFree(c.nn_ws);  // training workspace (grown on demand)
  collect(c);
  for (auto& p : c.pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : c.ev_dropped) (void)hipEventDestroy(e);
  for (hipEvent_t e : c.ev_pool) (void)hipEventDestroy(e);
  if (c.tally_host) (void)hipHostFree(c.tally_host);
  if (c.red_host) (void)hipHostFree(c.red_host);
  if (c.part_host) (void)hipHostFree(c.part_host);
  if (c.cons_host) (void)hipHostFree(c.cons_host);
  if (c.jf_host) (void)hipHostFree(c.jf_host);
  if (c.res_host) (void)hipHostFree(c.res_host);
  if (c.fin_host) (void)hipHostFree(c.fin_host);
  if (c.sort_total_host) (void)hipHostFree(c.sort_total_host);
  delete x;
  return ECPIC_OK;
}

ecpic_status ecpic_workspace_size(const ecpic_ctx* x, size_t* bytes) {
  if (!x || !bytes) return ECPIC_EINVAL;
  Carver dry;
  carve_all(const_cast<Ctx&>(x->c), dry);
  *bytes = dry.off;
  return ECPIC_OK;
}

ecpic_status ecpic_bind_workspace(ecpic_ctx* x, void* ws, size_t bytes) {
  if (!x || !ws) return ECPIC_EINVAL;
  Ctx& c = x->c;
  if (c.materialised)
    return fail(c, ECPIC_EINVAL, "device memory is in use: bind the workspace before any call "
                                 "that touches the device");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(c, ECPIC_EINVAL, "workspace must be 256-byte aligned");
  c.ws = ws;
  c.ws_bytes = bytes;
  const ecpic_status rc = materialise(c);
  if (rc != ECPIC_OK) {
    c.ws = nullptr;
    c.ws_bytes = 0;
  }
  return rc;
}

ecpic_status ecpic_bind_fields(ecpic_ctx* x, const ecpic_field_view* v) {
  if (!x) return ECPIC_EINVAL;
  Ctx& c = x->c;
  ENSURE_DEVICE(c);
  const int64_t nur = n_edges_r(c), nuz = n_edges_z(c), nh = n_cells(c);
  double** roles[6] = {&c.ur, &c.uz, &c.h, &c.ur_prev, &c.uz_prev, &c.h_prev};
  const int64_t len[6] = {nur, nuz, nh, nur, nuz, nh};
  if (v) {
    double* p[6] = {v->ur, v->uz, v->h, v->ur_prev, v->uz_prev, v->h_prev};
    for (int q = 0; q < 6; ++q) {
      if (!p[q]) return fail(c, ECPIC_EINVAL, "null field array");
      for (int r = 0; r < q; ++r)
        if (p[r] == p[q]) return fail(c, ECPIC_EINVAL, "field arrays must be distinct");
    }
    if (!c.fields_bound)
      for (int q = 0; q < 6; ++q) c.lib_fields[q] = *roles[q];
    for (int q = 0; q < 6; ++q) *roles[q] = p[q];
    c.fields_bound = true;
  } else if (c.fields_bound) {
    // the state goes back into the library's own arrays
    for (int q = 0; q < 6; ++q) {
      HIPCHK(launch_copy(c.lib_fields[q], *roles[q], len[q], c.stream));
      *roles[q] = c.lib_fields[q];
    }
    c.fields_bound = false;
    HIPCHK(hipStreamSynchronize(c.stream));
  }
  c.cons_valid = false;
  return ECPIC_OK;
}

ecpic_status ecpic_add_species(ecpic_ctx* x, const ecpic_species_desc* d, int32_t* sid) {
  if (!x || !d || !sid) return ECPIC_EINVAL;
  Ctx& c = x->c;
  if ((int)c.sp.size() >= kMaxSpecies) return fail(c, ECPIC_EINVAL, "at most 4 species");
  // the kernels address particle arrays by 32-bit byte offsets: at most
  // 2^29 slots of 8 bytes
  if (d->capacity < 0 || d->capacity > ((int64_t)1 << 29) || !(d->m > 0) || !(d->weight > 0) ||
      d->sort_stride < 0)
    return fail(c, ECPIC_EINVAL, "bad species descriptor");
  if (c.materialised && c.ws)
    return fail(c, ECPIC_EINVAL, "add every species before binding the workspace");
  Species s;
  std::memset(&s.d, 0, sizeof(s.d));
  s.desc = *d;
  if (c.materialised) {
    // library-owned memory: the species' buffers, and larger queues when
    // they no longer cover it
    Carver dry;
    carve_species_buf(c, dry, s.d[0], d->capacity);
    char* b0 = nullptr;
    char* b1 = nullptr;
    if (owned_alloc(c, &b0, dry.off) != hipSuccess || owned_alloc(c, &b1, dry.off) != hipSuccess)
      return fail(c, ECPIC_ENOMEM, "species allocation failed");
    Carver k0{b0}, k1{b1};
    carve_species_buf(c, k0, s.d[0], d->capacity);
    carve_species_buf(c, k1, s.d[1], d->capacity);
    const int32_t nsp = (int32_t)c.sp.size() + 1;
    int64_t max_cap = d->capacity;
    for (const Species& o : c.sp) max_cap = std::max<int64_t>(max_cap, o.desc.capacity);
    if (queue_len(max_cap) > c.queue_cap || nsp > c.queue_species ||
        read_scratch_len(max_cap) > c.rd_scratch_len) {
      Carver qd;
      carve_queues(c, qd, max_cap, kMaxSpecies);
      char* qb = nullptr;
      if (owned_alloc(c, &qb, qd.off) != hipSuccess)
        return fail(c, ECPIC_ENOMEM, "queue allocation failed");
      Carver qk{qb};
      carve_queues(c, qk, max_cap, kMaxSpecies);
    }
  }
  s.n = 0;
  // both sort buffers carry the species constants, so every kernel that is
  // handed a buffer descriptor sees the charge, mass and weight
  for (SpecDev& b : s.d) {
    b.cap = d->capacity;
    b.q = d->q;
    b.m = d->m;
    b.w = d->weight;
    b.qm = d->q / d->m;
    b.qw_dt = d->q * d->weight / c.g.dt;
    b.mobile = d->mobile;
    b.sid = (int32_t)c.sp.size();
  }
  c.sp.push_back(s);
  *sid = (int32_t)c.sp.size() - 1;
  return ECPIC_OK;
}

ecpic_status ecpic_load_particles(ecpic_ctx* x, int32_t sid, const double* r, const double* z,
                                  const double* vr, const double* vt, const double* vz,
                                  const uint64_t* uid, int64_t n) {
  if (!x) return ECPIC_EINVAL;
  Ctx& c = x->c;
  ENSURE_DEVICE(c);
  if (sid < 0 || sid >= (int)c.sp.size()) return fail(c, ECPIC_EINVAL, "bad species id");
  Species& s = c.sp[sid];
  if (n < 0 || n > s.desc.capacity) return fail(c, ECPIC_EINVAL, "n exceeds capacity");
  if (n > 0 && (!r || !z || !vr || !vt || !vz || !uid))
    return fail(c, ECPIC_EINVAL, "null particle array");
  HIPCHK(launch_load(c.m, view(s), r, z, vr, vt, vz, uid, n, c.g.R, c.prec == ECPIC_MIXED,
                     c.stream));
  c.cons_valid = false;
  s.n = n;
  return ECPIC_OK;
}

ecpic_status ecpic_read_particles(ecpic_ctx* x, int32_t sid, double* xi, double* eta, double* vr,
                                  double* vt, double* vz, uint64_t* uid, int64_t cap,
                                  int64_t* n_out) {
  if (!x || !n_out) return ECPIC_EINVAL;
  Ctx& c = x->c;
  ENSURE_DEVICE(c);
  if (sid < 0 || sid >= (int)c.sp.size()) return fail(c, ECPIC_EINVAL, "bad species id");
  Species& s = c.sp[sid];
  *n_out = 0;
  if (s.n == 0) return ECPIC_OK;
  const int64_t nb = (s.n + kBlock - 1) / kBlock;
  // block counts and their scan partials in the context's scratch
  if (read_scratch_len(s.n) > c.rd_scratch_len) return fail(c, ECPIC_EINVAL, "read scratch");
  int32_t* blk = c.rd_scratch;
  int32_t* part = c.rd_scratch + nb + 1;
  const int mixed = c.prec == ECPIC_MIXED;
  ecpic_status rc = ECPIC_OK;
  hipError_t e = launch_flag_count(c.m, view(s), s.n, mixed, blk, c.stream);
  if (e == hipSuccess) e = scan_exclusive(blk, nb, part, c.stream);
  int32_t total = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(&total, blk + nb, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  if (e == hipSuccess) {
    if (total > cap || !xi || !eta || !vr || !vt || !vz || !uid) {
      rc = fail(c, ECPIC_EINVAL, "output capacity too small or null output");
    } else {
      e = launch_compact_read(c.m, view(s), s.n, mixed, blk, xi, eta, vr, vt, vz, uid, c.stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    }
  }
  if (e != hipSuccess) return fail(c, ECPIC_EHIP, hipGetErrorString(e));
  *n_out = total;
  return rc;
}

ecpic_status ecpic_set_fields(ecpic_ctx* x, const double* ur, const double* uz, const double* h,
                              const double* ur_prev, const double* uz_prev, double t,
                              int64_t step) {
  if (!x || !ur || !uz || !h) return ECPIC_EINVAL;
  Ctx& c = x->c;
  ENSURE_DEVICE(c);
  const int64_t nur = n_edges_r(c), nuz = n_edges_z(c), nh = n_cells(c);
  HIPCHK(launch_copy(c.ur, ur, nur, c.stream));
  HIPCHK(launch_copy(c.uz, uz, nuz, c.stream));
  HIPCHK(launch_copy(c.h, h, nh, c.stream));
  HIPCHK(launch_copy(c.ur_prev, ur_prev ? ur_prev : ur, nur, c.stream));
  HIPCHK(launch_copy(c.uz_prev, uz_prev ? uz_prev : uz, nuz, c.stream));
  HIPCHK(launch_copy(c.h_prev, h, nh, c.stream));
  c.cons_valid = false;
  c.t = t;
  c.step = step;
  return ECPIC_OK;
}

ecpic_status ecpic_get_fields(ecpic_ctx* x, double* ur, double* uz, double* h) {
  if (!x) return ECPIC_EINVAL;
  Ctx& c = x->c;
  ENSURE_DEVICE(c);
  if (ur) HIPCHK(launch_copy(ur, c.ur, n_edges_r(c), c.stream));
  if (uz) HIPCHK(launch_copy(uz, c.uz, n_edges_z(c), c.stream));
  if (h) HIPCHK(launch_copy(h, c.h, n_cells(c), c.stream));
  return ECPIC_OK;
}

ecpic_status ecpic_set_port_field(ecpic_ctx* x, const double* hb) {
  if (!x || !hb) return ECPIC_EINVAL;
  Ctx& c = x->c;
  if (c.g.port_i <= 0) return fail(c, ECPIC_EINVAL, "no port");
  ENSURE_DEVICE(c);
  std::vector<double> h(hb, hb + c.g.nr);
  for (int i = 0; i < c.g.port_i; ++i) h[i] = 0.0;
  HIPCHK(hipMemcpyAsync(c.port_hb, h.data(), sizeof(double) * c.g.nr, hipMemcpyHostToDevice,
                        c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  return ECPIC_OK;
}

ecpic_status ecpic_get_port_field(ecpic_ctx* x, double* hb) {
  if (!x || !hb) return ECPIC_EINVAL;
  Ctx& c = x->c;
  if (c.g.port_i <= 0) return fail(c, ECPIC_EINVAL, "no port");
  ENSURE_DEVICE(c);
  HIPCHK(hipMemcpyAsync(hb, c.port_hb, sizeof(double) * c.g.nr, hipMemcpyDeviceToHost,
                        c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  return ECPIC_OK;
}

ecpic_status ecpic_set_half_field(ecpic_ctx* x, const double* urh, const double* uzh) {
  if (!x || !urh || !uzh) return ECPIC_EINVAL;
  Ctx& c = x->c;
  ENSURE_DEVICE(c);
  // half = (u0 + u1)/2 with u0 = u1 = the given field reproduces it exactly
  HIPCHK(launch_half(c, urh, uzh, urh, uzh, c.stream));
  return ECPIC_OK;
}

ecpic_status ecpic_push_deposit(ecpic_ctx* x, int32_t commit, double* Ir, double* Iz) {
  if (!x) return ECPIC_EINVAL;
  Ctx& c = x->c;
  ENSURE_DEVICE(c);
  ecpic_status rc = pass(c, commit ? 1 : 0, false, c.step, false);
  if (rc != ECPIC_OK) return rc;
  if (commit) c.cons_valid = false;
  if (Ir) HIPCHK(launch_copy(Ir, c.Ir, n_edges_r(c), c.stream));
  if (Iz) HIPCHK(launch_copy(Iz, c.Iz, n_edges_z(c), c.stream));
  if (commit) {
    Tally t;
    rc = finish_tally(c, t);
    if (rc == ECPIC_OK && t.n_errors) rc = fail(c, ECPIC_EPUSH, "particle push failed");
  }
  return rc;
}

ecpic_status ecpic_field_solve(ecpic_ctx* x, const double* ur0, const double* uz0, const double* h0,
                               const double* Ir, const double* Iz, double t, double* ur1,
                               double* uz1, double* h1) {
  if (!x || !ur0 || !uz0 || !h0 || !Ir || !Iz || !ur1 || !uz1 || !h1) return ECPIC_EINVAL;
  Ctx& c = x->c;
  ENSURE_DEVICE(c);
  SolveArgs a;
  std::memset(&a, 0, sizeof(a));
  a.ur0 = ur0;
  a.uz0 = uz0;
  a.h0 = h0;
  a.Ir = const_cast<double*>(Ir);  // read only (no clear target)
  a.Iz = const_cast<double*>(Iz);
  a.vnext = drive(c.g, t + c.g.dt);
  a.vnow = drive(c.g, t);
  a.vhalf = 0.5 * (a.vnow + a.vnext);
  a.ur1 = ur1;
  a.uz1 = uz1;
  a.h1 = h1;
  HIPCHK(field_solve(c, a, c.stream));
  return ECPIC_OK;
}

ecpic_status ecpic_field_solve_noalloc(ecpic_ctx* x, const double* ur0, const double* uz0,
                                       const double* h0, const double* Ir, const double* Iz,
                                       double t, double* ur1, double* uz1, double* h1) {
  if (!x || !ur0 || !uz0 || !h0 || !Ir || !Iz || !ur1 || !uz1 || !h1) return ECPIC_EINVAL;
  Ctx& c = x->c;
  // setting the context's device memory up would allocate: it must be in
  // place already
  if (!c.materialised)
    return fail(c, ECPIC_EINVAL, "context device memory not set up (bind a workspace or make "
                                 "any device call first)");
  if (n_cells(c) > kStaticScratchDoubles)
    return fail(c, ECPIC_EINVAL, "grid larger than the static scratch (2^20 cells)");
  double* hat = static_scratch(c.device);
  if (!hat) return fail(c, ECPIC_EHIP, "static scratch address not set up on this device");
  SolveArgs a;
  std::memset(&a, 0, sizeof(a));
  a.ur0 = ur0;
  a.uz0 = uz0;
  a.h0 = h0;
  a.Ir = const_cast<double*>(Ir);  // read only (no clear target)
  a.Iz = const_cast<double*>(Iz);
  a.vnext = drive(c.g, t + c.g.dt);
  a.vnow = drive(c.g, t);
  a.vhalf = 0.5 * (a.vnow + a.vnext);
  a.ur1 = ur1;
  a.uz1 = uz1;
  a.h1 = h1;
  HIPCHK(field_solve(c, a, c.stream, hat));
  return ECPIC_OK;
}

// Enqueue the field part of Picard iteration k: solve with the current I into
// the *_nx buffers, write the next half-step field into *_half2, zero I, and
// the residual against the previous iterate into res_host[k] (polled with
// wait_residual); the new iterate becomes *_it.  Guarded: every kernel returns at
// once when the stop flag is set (a speculative iteration after convergence);
// the flag is set when the residual is <= tol.
static ecpic_status enqueue_solve(Ctx& c, int k, double tol, bool guarded, bool alternate) {
  SolveArgs a;
  std::memset(&a, 0, sizeof(a));
  a.ur0 = c.ur;
  a.uz0 = c.uz;
  a.h0 = c.h;
  a.Ir = c.Ir;
  a.Iz = c.Iz;
  a.vnext = drive(c.g, c.t + c.g.dt);
  a.vnow = drive(c.g, c.t);
  a.vhalf = 0.5 * (a.vnow + a.vnext);
  a.ur1 = c.ur_nx;
  a.uz1 = c.uz_nx;
  a.h1 = c.h_nx;
  a.gapv = c.g.blocking_cap > 0.0 ? c.circ + 3 : nullptr;
  a.phin = (c.g.blocking_cap > 0.0 && c.g.port_i > 0) ? c.circ : nullptr;
  a.ur_old = c.ur_it;
  a.uz_old = c.uz_it;
  a.part = c.sol.partial + kOffRes;
  a.ur_h = c.ur_half2;
  a.uz_h = c.uz_half2;
  a.ur_hf = c.ur_half_f2;
  a.uz_hf = c.uz_half_f2;
  // alternate: clear the other current pair, which the next pass deposits
  // into, and keep these currents; otherwise clear them once read
  a.Ir_clr = alternate ? c.Ir_alt : c.Ir;
  a.Iz_clr = alternate ? c.Iz_alt : c.Iz;
  a.stop = guarded ? c.stop : nullptr;
  {
    // field arrays: u0, I, u_old read, u1 and the half field written, h0 read,
    // h1 written (FP64)
    const double fb = 8.0 * (6.0 * (n_edges_r(c) + n_edges_z(c)) + 2.0 * n_cells(c));
    Timed tm(c, ECPIC_K_FIELD, fb, 0);
    HIPCHK(field_solve(c, a, c.stream));
  }
  static_assert(kOffRes == 0, "the residual kernel reads the partials at offset 0");
  std::memcpy(&c.res_host[k], &kResPending, sizeof(double));
  HIPCHK(launch_converge(c, k, tol, c.stream, &a));
  std::swap(c.ur_it, c.ur_nx);
  std::swap(c.uz_it, c.uz_nx);
  std::swap(c.h_it, c.h_nx);
  if (alternate) {
    std::swap(c.Ir, c.Ir_alt);
    std::swap(c.Iz, c.Iz_alt);
  }
  return ECPIC_OK;
}

// Spin until the device has stored the 8-byte word at p (a value other
// than `pending`), checking the stream now and then so that a failed or
// drained stream cannot leave the host waiting for ever.
static ecpic_status wait_word(Ctx& c, const volatile uint64_t* p, uint64_t pending,
                              uint64_t* out) {
  for (uint64_t spin = 0;; ++spin) {
    const uint64_t v = *p;
    if (v != pending) {
      *out = v;
      std::atomic_thread_fence(std::memory_order_acquire);
      return ECPIC_OK;
    }
    if ((spin & 1023) == 1023) {
      const hipError_t e = hipStreamQuery(c.stream);
      if (e != hipSuccess && e != hipErrorNotReady) return fail(c, ECPIC_EHIP, hipGetErrorString(e));
      if (e == hipSuccess && *p == pending)
        return fail(c, ECPIC_EHIP, "stream drained without the expected device result");
    }
  }
}

// Spin until the device has stored the sequence number `want` at p.
static ecpic_status wait_seq(Ctx& c, const volatile uint64_t* p, uint64_t want) {
  for (uint64_t spin = 0;; ++spin) {
    if (*p == want) {
      std::atomic_thread_fence(std::memory_order_acquire);
      return ECPIC_OK;
    }
    if ((spin & 1023) == 1023) {
      const hipError_t e = hipStreamQuery(c.stream);
      if (e != hipSuccess && e != hipErrorNotReady) return fail(c, ECPIC_EHIP, hipGetErrorString(e));
      if (e == hipSuccess && *p != want)
        return fail(c, ECPIC_EHIP, "stream drained without the expected device result");
    }
  }
}

static ecpic_status wait_residual(Ctx& c, int k, double* r) {
  uint64_t bits = 0;
  ecpic_status rc = wait_word(c, reinterpret_cast<volatile uint64_t*>(c.res_host + k),
                              kResPending, &bits);
  if (rc != ECPIC_OK) return rc;
  std::memcpy(r, &bits, sizeof(double));
  return ECPIC_OK;
}

// One unguarded field iterate with the current I; returns the residual.
static ecpic_status iterate(Ctx& c, double* r_out) {
  HIPCHK(launch_zero_i(c.stop, 1, c.stream));
  ecpic_status rc = enqueue_solve(c, 0, -1.0, false, false);
  if (rc != ECPIC_OK) return rc;
  rc = wait_residual(c, 0, r_out);
  if (rc != ECPIC_OK) return rc;
  HIPCHK(hipStreamSynchronize(c.stream));
  collect(c);
  return ECPIC_OK;
}

static void swap_half(Ctx& c) {
  std::swap(c.ur_half, c.ur_half2);
  std::swap(c.uz_half, c.uz_half2);
  std::swap(c.ur_half_f, c.ur_half_f2);
  std::swap(c.uz_half_f, c.uz_half_f2);
}

ecpic_status ecpic_field_iterate(ecpic_ctx* x, double* rel) {
  if (!x || !rel) return ECPIC_EINVAL;
  Ctx& c = x->c;
  ENSURE_DEVICE(c);
  ecpic_status rc = iterate(c, rel);
  if (rc != ECPIC_OK) return rc;
  swap_half(c);
  return ECPIC_OK;
}

ecpic_status ecpic_set_mcc(ecpic_ctx* x, const ecpic_mcc_desc* m) {
  if (!x) return ECPIC_EINVAL;
  Ctx& c = x->c;
  if (!m || !m->enabled) {
    std::memset(&c.mcc, 0, sizeof(c.mcc));
    return ECPIC_OK;
  }
  if (m->electron_sid < 0 || m->electron_sid >= (int)c.sp.size() || m->ion_sid < 0 ||
      m->ion_sid >= (int)c.sp.size() || !(m->n_gas >= 0) || !(m->t_gas > 0) ||
      !(m->m_gas > 0) || !(m->eps_max_ev > 0))
    return fail(c, ECPIC_EINVAL, "bad collision descriptor");
  c.mcc = *m;
  for (size_t s = 0; s < c.sp.size() && s < (size_t)kMaxSpecies; ++s) {
    const int role = ((int)s == m->electron_sid) ? 1 : ((int)s == m->ion_sid ? 2 : 0);
    c.numax[s] = nu_max_host(*m, role, c.sp[s].desc.m);
  }
  return ECPIC_OK;
}

ecpic_status ecpic_collide(ecpic_ctx* x, const ecpic_mcc_desc* m, int64_t step) {
  if (!x || !m) return ECPIC_EINVAL;
  Ctx& c = x->c;
  ENSURE_DEVICE(c);
  ecpic_mcc_desc saved = c.mcc;
  ecpic_status rc = ecpic_set_mcc(x, m);
  if (rc != ECPIC_OK) return rc;
  HIPCHK(launch_zero_tally(c, c.stream));
  std::vector<MccDev> d(c.sp.size());
  for (size_t s = 0; s < c.sp.size(); ++s) d[s] = make_mcc(c, (int)s, step);
  for (size_t s = 0; s < c.sp.size(); ++s) {
    if (!d[s].enabled) continue;
    SpecDev v = view(c.sp[s]);
    v.sid = (int)s;
    HIPCHK(launch_collide(c.m, v, d[s], c.tally, c.prec == ECPIC_MIXED, c.stream));
  }
  c.mcc = saved;
  c.cons_valid = false;
  Tally t;
  rc = finish_tally(c, t);
  if (rc == ECPIC_OK && t.n_over_range)
    rc = fail(c, ECPIC_ERANGE, "particles beyond the null-collision bound (collisions applied)");
  return rc;
}

ecpic_status ecpic_sort(ecpic_ctx* x) {
  if (!x) return ECPIC_EINVAL;
  Ctx& c = x->c;
  ENSURE_DEVICE(c);
  for (Species& s : c.sp) HIPCHK(launch_sort(c, s, c.stream, nullptr));
  return ECPIC_OK;
}

ecpic_status ecpic_node_charge(ecpic_ctx* x, double* q, double* bot, double* top, double* side) {
  if (!x) return ECPIC_EINVAL;
  Ctx& c = x->c;
  ENSURE_DEVICE(c);
  if (q) HIPCHK(launch_node_charge(c, q, c.stream));
  if (bot) HIPCHK(launch_copy(bot, c.wall_bot, c.g.nr + 1, c.stream));
  if (top) HIPCHK(launch_copy(top, c.wall_top, c.g.nr + 1, c.stream));
  if (side) HIPCHK(launch_copy(side, c.wall_side, c.g.nz + 1, c.stream));
  return ECPIC_OK;
}

static ecpic_status diag_into(Ctx& c, ecpic_step_stats* st) {
  double* d = c.sol.partial;
  HIPCHK(launch_zero(d + kOffKE, 8, c.stream));
  for (size_t s = 0; s < c.sp.size() && s < 4; ++s)
    HIPCHK(launch_kinetic(c.sp[s], c.prec == ECPIC_MIXED, d + kOffKE + s, c.stream));
  HIPCHK(launch_field_energy(c, c.ur, c.uz, c.h, d + kOffFE, c.stream));
  HIPCHK(hipMemcpyAsync(c.part_host + kOffFE, d + kOffFE, (kOffSc - kOffFE) * sizeof(double),
                        hipMemcpyDeviceToHost, c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  double se = 0.0, sb = 0.0;
  for (int b = 0; b < kRedBlocks; ++b) {
    se += c.part_host[kOffFE + b];
    sb += c.part_host[kOffFE + kRedBlocks + b];
  }
  st->we = 0.5 * se;
  st->wb = 0.5 * c.g.mu * sb;
  for (size_t s = 0; s < 4; ++s) st->ke[s] = (s < c.sp.size()) ? c.part_host[kOffKE + s] : 0.0;
  for (size_t s = 0; s < c.sp.size() && s < 4; ++s) st->n_alive[s] = c.sp[s].n;
  st->t = c.t;
  st->step = c.step;
  return ECPIC_OK;
}

ecpic_status ecpic_set_option(ecpic_ctx* x, int32_t option, int64_t value) {
  if (!x) return ECPIC_EINVAL;
  Ctx& c = x->c;
  switch (option) {
    case ECPIC_OPT_QUEUE_WAVES:
      if (value != 0 && value != 2 && value != 3)
        return fail(c, ECPIC_EINVAL, "queue waves: 0, 2 or 3");
      c.queue_waves = (int32_t)value;
      return ECPIC_OK;
    case ECPIC_OPT_NN_FORCE_FALLBACK:
      if (value < 0 || value >= kMaxIter) return fail(c, ECPIC_EINVAL, "fallback iteration");
      c.nn_force_fallback = (int32_t)value;
      return ECPIC_OK;
    case ECPIC_OPT_JFNK_KRYLOV:
      if (value < 0 || value > kMaxKrylov) return fail(c, ECPIC_EINVAL, "Krylov space: 0..32");
      if (c.materialised)
        return fail(c, ECPIC_EINVAL, "reserve the Krylov space before the device memory is set up");
      c.jfnk_m = (int32_t)value;
      return ECPIC_OK;
  }
  return fail(c, ECPIC_EINVAL, "unknown option");
}

ecpic_status ecpic_set_profiling(ecpic_ctx* x, int32_t kind_mask) {
  if (!x) return ECPIC_EINVAL;
  Ctx& c = x->c;
  HIPCHK(hipStreamSynchronize(c.stream));
  collect(c);
  c.prof_mask = (uint32_t)kind_mask & ((1u << ECPIC_K_COUNT) - 1u);
  std::memset(&c.prof, 0, sizeof(c.prof));
  std::memset(c.prof_seq, 0, sizeof(c.prof_seq));
  return ECPIC_OK;
}

ecpic_status ecpic_set_profiling_every(ecpic_ctx* x, int32_t every) {
  if (!x || every < 1) return ECPIC_EINVAL;
  Ctx& c = x->c;
  HIPCHK(hipStreamSynchronize(c.stream));
  collect(c);
  c.prof_every = every;
  std::memset(&c.prof, 0, sizeof(c.prof));
  std::memset(c.prof_seq, 0, sizeof(c.prof_seq));
  return ECPIC_OK;
}

ecpic_status ecpic_get_profile(ecpic_ctx* x, ecpic_profile* out) {
  if (!x || !out) return ECPIC_EINVAL;
  Ctx& c = x->c;
  HIPCHK(hipStreamSynchronize(c.stream));
  collect(c);
  *out = c.prof;
  return ECPIC_OK;
}

ecpic_status ecpic_diagnostics(ecpic_ctx* x, ecpic_step_stats* st) {
  if (!x || !st) return ECPIC_EINVAL;
  ENSURE_DEVICE(x->c);
  std::memset(st, 0, sizeof(*st));
  return diag_into(x->c, st);
}

}  // extern "C"

// One implicit step.  guess_ready: the previous step of a run already
// enqueued this step's extrapolated guess.  prepare_next: a next step follows
// at once, so its guess (fields only) is enqueued as soon as this step's
// fields are final, before the host waits for the commit summary.
// Jacobian-free Newton-Krylov iterations of one step (ECPIC_SOLVER_JFNK;
// the algorithm is stated with the solver enum in ecpic.h).  Starts from
// the guess in c.ur_it / c.uz_it.  Ends with the state the Picard loop
// leaves for a separate commit: the accepted iterate's fields in c.*_it,
// its half-step field in c.*_half, its push's currents in c.Ir_alt /
// c.Iz_alt, and the pass scratch of parity slot + 1 cleared by the residual
// kernel of `slot`, the residual slot of the last evaluation (*last_slot).
// Every evaluation is waited for: the Krylov loop needs its inner products
// on the host.
// relative forward-difference step of the JFNK Jacobian (see ecpic.h)
constexpr double kJfDiff = 1e-6;

static ecpic_status jfnk_iterate(Ctx& c, const ecpic_step_opts* o, ecpic_step_stats* S,
                                 int* last_slot, int* evals_out, bool* conv) {
  const int64_t nur = n_edges_r(c), n = nur + n_edges_z(c);
  const int m = o->krylov;
  const bool fixed = o->fixed_iter > 0;
  const int nmax = fixed ? o->fixed_iter : o->max_iter;
  double* V = c.jf_vec;  // m + 1 Krylov vectors, then six work vectors
  double* X = V + (int64_t)(c.jfnk_m + 1) * n;
  double* GX = X + n;
  double* F = GX + n;
  double* Y = F + n;
  double* W = Y + n;
  double* D = W + n;
  int slot = 0, evals = 0;
  *conv = false;
  auto dots = [&](const double* w, const double* Vb, int K, double* out) -> ecpic_status {
    HIPCHK(launch_jf_dots(c, w, Vb, n, K, c.stream));
    HIPCHK(hipMemcpyAsync(c.jf_host, c.jf_part, sizeof(double) * K * kJfBlocks,
                          hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    for (int k = 0; k < K; ++k) {
      double acc = 0.0;
      for (int b = 0; b < kJfBlocks; ++b) acc += c.jf_host[(size_t)k * kJfBlocks + b];
      out[k] = acc;
    }
    return ECPIC_OK;
  };
  auto norm = [&](const double* a, double* out) -> ecpic_status {
    double d = 0.0;
    const ecpic_status rc = dots(a, a, 1, &d);
    *out = std::sqrt(std::max(d, 0.0));
    return rc;
  };
  // G at Yv: the push in (u^n + Yv) / 2, the field solve from u^n; the
  // result is left in c.ur_it / c.uz_it / c.h_it and the push's currents in
  // c.Ir_alt / c.Iz_alt
  auto eval = [&](double* Yv) -> ecpic_status {
    slot = evals % kMaxIter;
    ++evals;
    HIPCHK(launch_half(c, c.ur, c.uz, Yv, Yv + nur, c.stream));
    double* keep_r = c.ur_it;
    double* keep_z = c.uz_it;
    // the residual kernel measures the solve against the previous iterate
    c.ur_it = Yv;
    c.uz_it = Yv + nur;
    ecpic_status rc = pass(c, 0, false, c.step, true, false);
    if (rc != ECPIC_OK) {
      c.ur_it = keep_r;
      c.uz_it = keep_z;
      return rc;
    }
    rc = enqueue_solve(c, slot, -1.0, false, true);
    // the solve wrote a library buffer, now the iterate, and left Yv as the
    // next target: the target role goes back to the library buffer
    c.ur_nx = keep_r;
    c.uz_nx = keep_z;
    if (rc != ECPIC_OK) return rc;
    double r = 0.0;
    return wait_residual(c, slot, &r);
  };
#define JF(call)                          \
  do {                                    \
    const ecpic_status rc_ = (call);      \
    if (rc_ != ECPIC_OK) return rc_;      \
  } while (0)
  HIPCHK(hipMemcpyAsync(X, c.ur_it, sizeof(double) * nur, hipMemcpyDeviceToDevice, c.stream));
  HIPCHK(hipMemcpyAsync(X + nur, c.uz_it, sizeof(double) * (n - nur), hipMemcpyDeviceToDevice,
                        c.stream));
  JF(eval(X));
  HIPCHK(launch_jf_sub(c, X, c.ur_it, c.uz_it, F, GX, c.stream));
  double fn = 0.0, gn = 0.0;
  JF(norm(F, &fn));
  JF(norm(GX, &gn));
  double H[kMaxKrylov + 1][kMaxKrylov];
  double cs[kMaxKrylov], sn[kMaxKrylov], g[kMaxKrylov + 1], yv[kMaxKrylov];
  double h1[kMaxKrylov + 1], h2[kMaxKrylov + 1];
  for (int k = 0; k < nmax; ++k) {
    const double r = gn > 0.0 ? fn / gn : (fn > 0.0 ? INFINITY : 0.0);
    S->residual[k] = r;
    S->newton_iters = k + 1;
    if (fixed ? (k == nmax - 1) : (r <= o->tol)) {
      *conv = true;
      break;
    }
    if (!(fn > 0.0)) {
      *conv = true;
      break;
    }
    // GMRES on J d = -F from d = 0
    double xn = 0.0;
    JF(norm(X, &xn));
    const double eps = kJfDiff * std::max(xn, fn);
    HIPCHK(launch_jf_axpby(c, -1.0 / fn, F, 0.0, F, V, c.stream));
    g[0] = fn;
    int used = 0;
    for (int j = 0; j < m; ++j) {
      double* vj = V + (int64_t)j * n;
      HIPCHK(launch_jf_axpby(c, 1.0, X, eps, vj, Y, c.stream));
      JF(eval(Y));
      HIPCHK(launch_jf_jv(c, vj, c.ur_it, c.uz_it, GX, eps, W, c.stream));
      // classical Gram-Schmidt, applied twice, in the energy inner product
      JfCoef cf;
      JF(dots(W, V, j + 1, h1));
      for (int i = 0; i <= j; ++i) cf.v[i] = -h1[i];
      HIPCHK(launch_jf_gemv(c, j + 1, V, n, cf, 1.0, W, c.stream));
      JF(dots(W, V, j + 1, h2));
      for (int i = 0; i <= j; ++i) cf.v[i] = -h2[i];
      HIPCHK(launch_jf_gemv(c, j + 1, V, n, cf, 1.0, W, c.stream));
      for (int i = 0; i <= j; ++i) H[i][j] = h1[i] + h2[i];
      double hn = 0.0;
      JF(norm(W, &hn));
      H[j + 1][j] = hn;
      HIPCHK(launch_jf_axpby(c, hn > 0.0 ? 1.0 / hn : 0.0, W, 0.0, W, V + (int64_t)(j + 1) * n,
                             c.stream));
      // the earlier rotations on the new column, then its own
      for (int i = 0; i < j; ++i) {
        const double a = H[i][j], b = H[i + 1][j];
        H[i][j] = cs[i] * a + sn[i] * b;
        H[i + 1][j] = -sn[i] * a + cs[i] * b;
      }
      const double a = H[j][j], b = H[j + 1][j];
      const double d = std::sqrt(a * a + b * b);
      cs[j] = d > 0.0 ? a / d : 1.0;
      sn[j] = d > 0.0 ? b / d : 0.0;
      H[j][j] = d;
      H[j + 1][j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      used = j + 1;
      S->krylov_iters++;
      if (!fixed && std::fabs(g[j + 1]) <= o->eta * fn) break;
    }
    for (int i = used - 1; i >= 0; --i) {
      double acc = g[i];
      for (int q = i + 1; q < used; ++q) acc -= H[i][q] * yv[q];
      yv[i] = acc / H[i][i];
    }
    JfCoef cd;
    for (int i = 0; i < used; ++i) cd.v[i] = yv[i];
    HIPCHK(launch_jf_gemv(c, used, V, n, cd, 0.0, D, c.stream));
    // the step, backtracking in tolerance mode; the accepted trial's map is
    // the next residual evaluation
    double lam = 1.0;
    for (int ls = 0;; ++ls) {
      HIPCHK(launch_jf_axpby(c, 1.0, X, lam, D, Y, c.stream));
      JF(eval(Y));
      HIPCHK(launch_jf_sub(c, Y, c.ur_it, c.uz_it, W, nullptr, c.stream));
      double fy = 0.0;
      JF(norm(W, &fy));
      if (fixed || ls == 8 || fy <= (1.0 - 1e-4 * lam) * fn) {
        std::swap(X, Y);
        std::swap(F, W);
        HIPCHK(launch_jf_sub(c, X, c.ur_it, c.uz_it, F, GX, c.stream));
        fn = fy;
        JF(norm(GX, &gn));
        break;
      }
      lam *= 0.5;
    }
  }
#undef JF
  *last_slot = slot;
  *evals_out = evals;
  return ECPIC_OK;
}

static ecpic_status step_impl(Ctx& c, const ecpic_step_opts* o, ecpic_step_stats* st,
                              bool guess_ready, bool prepare_next) {
  ecpic_step_stats local;
  ecpic_step_stats* S = st ? st : &local;
  std::memset(S, 0, sizeof(*S));
  int kmax = o->fixed_iter > 0 ? o->fixed_iter : o->max_iter;
  if (kmax < 1 || kmax > 64) return fail(c, ECPIC_EINVAL, "iterations must be in 1..64");
  const bool jfnk = o->solver == ECPIC_SOLVER_JFNK;
  if (o->solver != ECPIC_SOLVER_PICARD && !jfnk) return fail(c, ECPIC_EINVAL, "unknown solver");
  if (jfnk && c.g.blocking_cap > 0.0)
    return fail(c, ECPIC_EINVAL, "JFNK with a blocking capacitor is not supported");
  if (jfnk && (c.jfnk_m < 1 || o->krylov < 1 || o->krylov > c.jfnk_m || !(o->eta >= 0.0)))
    return fail(c, ECPIC_EINVAL,
                "JFNK: krylov must be in 1..the space reserved with ECPIC_OPT_JFNK_KRYLOV, "
                "eta >= 0");
  const double vnow = drive(c.g, c.t), vnext = drive(c.g, c.t + c.g.dt);
  const bool check = o->check_conservation != 0 && st != nullptr;
  if (check && !c.cons_valid) {
    // the charge and Gauss residual of t^n, which the commit compares with
    HIPCHK(launch_node_charge(c, c.q_node, c.stream));
    HIPCHK(launch_conservation(c, c.ur, c.uz, c.Ir, c.Iz, true, c.stream));
    c.cons_valid = true;
  }
  if (!guess_ready) HIPCHK(launch_guess_half(c, vnow, vnext, c.stream));
  if (o->use_nn) {
    bool used = false;
    ecpic_status rc = nn_guess(c, &used);
    if (rc != ECPIC_OK) return rc;
    S->used_nn = used ? 1 : 0;
  }
  // Picard iterations, one enqueued ahead of the one being waited for: the
  // next push starts while the host reads the residual.  If the residual
  // meets the tolerance, the iteration enqueued ahead finds the stop flag set
  // and does nothing, and the buffer roles are put back as they were.
  const bool tol_mode = o->fixed_iter <= 0;
  const double dtol = tol_mode ? o->tol : -1.0;
  struct Roles {
    double *ur_it, *uz_it, *h_it, *ur_nx, *uz_nx, *h_nx, *ur_half, *uz_half, *ur_half2,
        *uz_half2;
    float *ur_half_f, *uz_half_f, *ur_half_f2, *uz_half_f2;
    double *Ir, *Iz, *Ir_alt, *Iz_alt;
  };
  auto save = [&](Roles& r) {
    r = Roles{c.ur_it, c.uz_it, c.h_it, c.ur_nx, c.uz_nx, c.h_nx, c.ur_half, c.uz_half,
              c.ur_half2, c.uz_half2, c.ur_half_f, c.uz_half_f, c.ur_half_f2, c.uz_half_f2,
              c.Ir, c.Iz, c.Ir_alt, c.Iz_alt};
  };
  auto restore = [&](const Roles& r) {
    c.Ir = r.Ir; c.Iz = r.Iz; c.Ir_alt = r.Ir_alt; c.Iz_alt = r.Iz_alt;
    c.ur_it = r.ur_it; c.uz_it = r.uz_it; c.h_it = r.h_it;
    c.ur_nx = r.ur_nx; c.uz_nx = r.uz_nx; c.h_nx = r.h_nx;
    c.ur_half = r.ur_half; c.uz_half = r.uz_half;
    c.ur_half2 = r.ur_half2; c.uz_half2 = r.uz_half2;
    c.ur_half_f = r.ur_half_f; c.uz_half_f = r.uz_half_f;
    c.ur_half_f2 = r.ur_half_f2; c.uz_half_f2 = r.uz_half_f2;
  };
  // A Picard iteration that is expected to be the last one also commits:
  // its push writes the new particle states into the other buffers (and
  // collides the particles its null-collision draws select), its tallies
  // and wall charge go to the scratch of its parity.  If its residual meets
  // the tolerance the host accepts it (flips the buffers); otherwise nothing
  // of it is kept.  Expected: in fixed-iteration mode the last iteration; in
  // tolerance mode iteration j >= 2 when r_{j-2} (r_{j-2} / r_{j-3})^2, the
  // residual extrapolated at the observed contraction, is below tol / 10.
  // every commit writes the mobile species' new states into their other
  // buffers (an immobile species is not written; ions born into it are
  // appended to its current buffer beyond its count), so any iteration may
  // commit
  const bool fuse_ok = true;
  bool committed[kMaxIter] = {};
  auto expect_last = [&](int j) -> bool {
    if (!fuse_ok) return false;
    if (!tol_mode) return j == kmax - 1;
    if (j < 3) return false;
    const double a = S->residual[j - 2], b = S->residual[j - 3];
    if (!(a > 0.0) || !(b > 0.0)) return false;
    const double rho = a / b;
    return rho < 1.0 && a * rho * rho <= 0.1 * o->tol;
  };
  // sequence number of the commit summary enqueued behind a committing
  // iteration (0: none)
  uint64_t spec_seq[kMaxIter] = {};
  auto enqueue_iteration = [&](int k) -> ecpic_status {
    c.cur_tag = k;
    const bool fuse = expect_last(k);
    committed[k] = fuse;
    spec_seq[k] = 0;
    ecpic_status rc = fuse ? pass(c, 1, c.mcc.enabled != 0, c.step, true, true, true, true, k & 1)
                           : pass(c, 0, false, c.step, true, true);
    if (rc != ECPIC_OK) return rc;
    rc = enqueue_solve(c, k, dtol, true, true);
    if (rc != ECPIC_OK) return rc;
    if (fuse) {
      // the commit summary goes in right behind the iteration expected to
      // be the last, so the stream does not wait for the host to read the
      // residual; on the device it runs only if this iteration converged
      // (in fixed-count mode it is the last one)
      HIPCHK(launch_exchange(c, c.ur, c.uz, c.ur_it, c.uz_it, c.Ir_alt, c.Iz_alt,
                             c.sol.partial + kOffEx, c.stream));
      spec_seq[k] = ++c.fin_seq;
      HIPCHK(launch_finalize(c, tally_set(c, k & 1), c.sol.partial + kOffEx, c.Ir_alt,
                             c.Iz_alt, wall_scratch(c, k & 1), spec_seq[k], tol_mode ? k : -1,
                             c.stream, k));
    }
    return ECPIC_OK;
  };
  // With the learned guess, a residual that does not fall from one iterate
  // to the next sends the step back to the extrapolated guess (the
  // iteration is restarted; nn_fallback reports it).
  bool nn_active = S->used_nn != 0;
  int k = 0;
  bool conv = false;
  int iters_done = 0;
  if (jfnk) {
    int last = 0;
    ecpic_status rc = jfnk_iterate(c, o, S, &last, &iters_done, &conv);
    if (rc != ECPIC_OK) return rc;
    // the common commit below takes iterate k - 1, with committed[] unset
    k = last + 1;
  }
  for (int attempt = 0; attempt < 2 && !jfnk; ++attempt) {
    bool restart = false;
    {
      ecpic_status rc = enqueue_iteration(0);
      if (rc != ECPIC_OK) return rc;
    }
    double prev_r = INFINITY;
    for (k = 0; k < kmax; ++k) {
      Roles after_k;
      save(after_k);
      // the next iteration goes in ahead, unless this one is expected to be
      // the last (then it is enqueued only if the residual says otherwise)
      const bool ahead = k + 1 < kmax && !committed[k];
      if (ahead) {
        // the next push uses (u^n + u^{n+1,(k+1)}) / 2
        swap_half(c);
        ecpic_status rc = enqueue_iteration(k + 1);
        if (rc != ECPIC_OK) return rc;
      }
      double r = 0.0;
      {
        ecpic_status rc = wait_residual(c, k, &r);
        if (rc != ECPIC_OK) return rc;
      }
      S->residual[k] = r;
      if (tol_mode && r <= o->tol) {
        conv = true;
        if (ahead) {
          // the commit keeps the half-step field of push k and iterate k
          restore(after_k);
          drop_tag(c, k + 1);
        }
        ++k;
        break;
      }
      // timings of iterations that are known to be needed
      collect(c);
      if (tol_mode && nn_active && k >= 1 && (!(r < prev_r) || k == c.nn_force_fallback)) {
        if (ahead) {
          // iteration k+1 is already on the stream and commits (fused)
          // if it converges: then it is accepted rather than restarted
          double r1 = 0.0;
          ecpic_status rc = wait_residual(c, k + 1, &r1);
          if (rc != ECPIC_OK) return rc;
          S->residual[k + 1] = r1;
          if (r1 <= o->tol) {
            conv = true;
            k += 2;
            break;
          }
        }
        restart = true;
        break;
      }
      prev_r = r;
      if (!ahead && k + 1 < kmax) {
        swap_half(c);
        ecpic_status rc = enqueue_iteration(k + 1);
        if (rc != ECPIC_OK) return rc;
      }
    }
    if (!restart) break;
    // back to the extrapolated guess: drain the iteration enqueued ahead,
    // then start again (the guess kernel clears the stop flag, currents and
    // pass scratch, and sets every iterate and half-step buffer it uses)
    HIPCHK(hipStreamSynchronize(c.stream));
    collect(c);
    S->nn_fallback = 1;
    nn_active = false;
    HIPCHK(launch_guess_half(c, vnow, vnext, c.stream));
  }
  c.cur_tag = -1;
  S->iters = jfnk ? iters_done : k;
  if (!tol_mode) conv = true;
  S->converged = conv ? 1 : 0;
  if (!conv) {
    HIPCHK(hipStreamSynchronize(c.stream));
    collect(c);
    return fail(c, ECPIC_ENOTCONV, "Picard iteration did not converge");
  }
  // The accepted iteration k* = k - 1 either committed already (into the
  // other buffers, tallies in its parity's set) or the particles pushed in
  // its half-step field are committed now, with MCC, in place (tallies in
  // the set of parity k, cleared by its residual kernel).  Either way the
  // commit's currents are, bitwise, those of the accepted push, kept in the
  // alternate pair, so the commit deposits nothing.
  const int ks = k - 1;
  const bool fused = committed[ks];
  // a separate commit (the prediction missed) also writes into the other
  // buffers, with its wall charge in the scratch of parity ks + 1, which
  // the residual kernel of iteration ks cleared
  const int cset = fused ? (ks & 1) : ((ks + 1) & 1);
  const Tally* tset = tally_set(c, cset);
  ecpic_status rc = ECPIC_OK;
  if (!fused) {
    rc = pass(c, 1, c.mcc.enabled != 0, c.step, true, false, false, true, cset);
    if (rc != ECPIC_OK) return rc;
  }
  uint64_t seq = fused ? spec_seq[ks] : 0;
  if (seq == 0) {
    double* d = c.sol.partial;
    HIPCHK(launch_exchange(c, c.ur, c.uz, c.ur_it, c.uz_it, c.Ir_alt, c.Iz_alt, d + kOffEx,
                           c.stream));
    seq = ++c.fin_seq;
    HIPCHK(launch_finalize(c, tset, d + kOffEx, c.Ir_alt, c.Iz_alt, wall_scratch(c, cset), seq,
                           -1, c.stream, ks));
  }
  // field shift u^{n-1} <- u^n <- u^{n+1}.  Library buffers: by pointer
  // roles, at once (the summary kernels above hold the pointers they read),
  // so that the next step's guess can go in before the host reads the
  // summary; u^{n-1} moves to the spare buffer, which the guess does not
  // write, so that a step that is not committed can be put back.  Fields
  // bound by the caller: by copies once the commit is known to stand.
  struct FieldRoles {
    double *ur, *uz, *h, *ur_prev, *uz_prev, *h_prev, *ur_it, *uz_it, *h_it, *ur_spare,
        *uz_spare;
  };
  const FieldRoles before{c.ur, c.uz, c.h, c.ur_prev, c.uz_prev, c.h_prev,
                          c.ur_it, c.uz_it, c.h_it, c.ur_spare, c.uz_spare};
  const bool early_shift = !c.fields_bound;
  if (early_shift) {
    c.ur_prev = before.ur;
    c.uz_prev = before.uz;
    c.ur = before.ur_it;
    c.uz = before.uz_it;
    c.ur_it = before.ur_spare;
    c.uz_it = before.uz_spare;
    c.ur_spare = before.ur_prev;
    c.uz_spare = before.uz_prev;
    // h^{n-1} <- h^n, h^n <- h^{n+1}; the old h^{n-1} buffer becomes scratch
    c.h_prev = before.h;
    c.h = before.h_it;
    c.h_it = before.h_prev;
    if (prepare_next) {
      const double t1 = c.t + c.g.dt;
      HIPCHK(launch_guess_half(c, drive(c.g, t1), drive(c.g, t1 + c.g.dt), c.stream));
    }
  }
  rc = wait_seq(c, reinterpret_cast<volatile uint64_t*>(&c.fin_host->seq), seq);
  if (rc != ECPIC_OK) return rc;
  StepFinal fin;
  std::memcpy(&fin, (const void*)c.fin_host, sizeof(fin));
  collect(c);
  const Tally& t = fin.t;
  const bool circ = c.g.blocking_cap > 0.0;
  const double vgen = 0.5 * (vnow + vnext);
  // the gap's half-step voltage: the electrode potential with a capacitor
  const double vh = circ ? 0.5 * (fin.phi_n + fin.phi_1) : vgen;
  const double rgap = r_of_xi(c.m, c.g.nr - 0.5);
  S->electrode_v = circ ? fin.phi_1 : vnext;
  S->cap_charge = circ ? fin.q_1 : 0.0;
  S->w_gen = circ ? c.g.dt * vgen * fin.ie : 0.0;
  S->w_field_io = c.g.dt * fin.xs;
  S->port_v = fin.port_v;
  if (c.g.port_i > 0 && c.g.model == ECPIC_MODEL_ES)
    // the source's work on the powered wall nodes, weighted by the wall profile
    S->w_drive = vh * (fin.qp_delta + c.g.dt * fin.iz_plate);
  else if (c.g.port_i > 0)
    // the power the line delivered through the mouth
    S->w_drive = fin.port_w;
  else if (c.g.model == ECPIC_MODEL_ES)
    // the source's work: V^{1/2} times the charge it moves onto the powered
    // plate (the change of the plate nodes' field flux and the current
    // leaving them), plus the gap edge's share
    S->w_drive = vh * (fin.qp_delta + c.g.dt * fin.iz_plate) + c.g.dt * vh * fin.ir_gap;
  else
    S->w_drive = c.g.dt * (2.0 * kPi * rgap * 0.5 * (fin.h_gap_n + fin.h_gap_1) * vh +
                           vh * fin.ir_gap);
  S->w_particles = t.w_particles;
  S->w_absorbed = t.w_absorbed;
  S->w_coll = t.w_coll;
  for (size_t s = 0; s < c.sp.size() && s < 4; ++s) {
    S->n_absorbed[s] = (int64_t)t.n_absorbed[s];
    S->n_coll[s] = (int64_t)t.n_coll[s];
  }
  S->n_ionized = (int64_t)t.n_ionized;
  S->n_substeps = (int64_t)t.n_substeps;
  S->n_crossings = (int64_t)t.n_crossings;
  S->n_errors = (int64_t)t.n_errors;
  S->n_over_range = (int64_t)t.n_over_range;
  if (t.n_overflow || t.n_over_range) {
    // not committed: the particle buffers are not flipped (the new states,
    // and any pair that was appended, stay in the other buffers or beyond
    // the counts), the counts, clock and fields stay as they were, and the
    // finalize kernel left the wall charge out
    if (early_shift) {
      c.ur = before.ur;
      c.uz = before.uz;
      c.h = before.h;
      c.ur_prev = before.ur_prev;
      c.uz_prev = before.uz_prev;
      c.h_prev = before.h_prev;
      c.ur_it = before.ur_it;
      c.uz_it = before.uz_it;
      c.h_it = before.h_it;
      c.ur_spare = before.ur_spare;
      c.uz_spare = before.uz_spare;
    }
    HIPCHK(hipStreamSynchronize(c.stream));
    collect(c);
    S->t = c.t;
    S->step = c.step;
    for (size_t s = 0; s < c.sp.size() && s < 4; ++s) S->n_alive[s] = c.sp[s].n;
    if (t.n_overflow)
      return fail(c, ECPIC_ECAPACITY,
                  "species capacity exceeded by ionisation (step not committed)");
    return fail(c, ECPIC_ERANGE,
                "a particle exceeded the null-collision bound eps_max (step not committed)");
  }
  if (!early_shift) {
    HIPCHK(launch_shift(c, c.stream));
    if (prepare_next) {
      const double t1 = c.t + c.g.dt;
      HIPCHK(launch_guess_half(c, drive(c.g, t1), drive(c.g, t1 + c.g.dt), c.stream));
    }
  }
  // the new states are in the mobile species' other buffers
  for (size_t s = 0; s < c.sp.size(); ++s) {
    Species& sp = c.sp[s];
    if (!sp.desc.mobile) continue;
    if (sp.n <= 0 && t.append[s] == 0) continue;
    sp.cur = 1 - sp.cur;
    std::swap(sp.d[0].uid, sp.d[1].uid);  // the uids stay with the state
  }
  for (size_t s = 0; s < c.sp.size(); ++s) {
    int64_t n = c.sp[s].n + (int64_t)t.append[s];
    if (n > c.sp[s].desc.capacity) n = c.sp[s].desc.capacity;
    c.sp[s].n = n;
  }
  c.t += c.g.dt;
  c.step += 1;
  if (check) {
    // continuity and Gauss against t^n with the accepted currents
    HIPCHK(launch_zero(reinterpret_cast<double*>(c.cons_dev), 4, c.stream));
    HIPCHK(launch_node_charge(c, c.q_node, c.stream));
    HIPCHK(launch_conservation(c, c.ur, c.uz, c.Ir_alt, c.Iz_alt, false, c.stream));
    HIPCHK(hipMemcpyAsync(c.cons_host, c.cons_dev, 3 * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, c.stream));
  } else {
    c.cons_valid = false;
  }
  if (o->sort_every > 0 && c.step % o->sort_every == 0) {
    // the species whose stride this sort reaches
    const int64_t nth = c.step / o->sort_every;
    bool due[kMaxSpecies] = {false, false, false, false};
    for (size_t s = 0; s < c.sp.size(); ++s) {
      const int32_t k = c.sp[s].desc.sort_stride;
      due[s] = k <= 1 || nth % k == 0;
      if (!due[s]) continue;
      const int64_t n0 = c.sp[s].n;
      Timed tm(c, ECPIC_K_SORT, (2.0 * (state_bytes(c) + 8.0) + 16.0) * (double)n0, n0);
      HIPCHK(launch_sort_async(c, c.sp[s], c.sort_total_host + s, c.stream));
    }
    HIPCHK(hipStreamSynchronize(c.stream));
    collect(c);
    for (size_t s = 0; s < c.sp.size(); ++s)
      if (due[s]) finish_sort(c.sp[s], c.sort_total_host[s]);
  }
  if (st) {
    ecpic_status r2 = diag_into(c, S);
    if (r2 != ECPIC_OK) return r2;
    if (check) {
      double v[3];
      std::memcpy(v, c.cons_host, sizeof(v));
      S->continuity_max = v[0];
      S->gauss_max = v[1];
      S->q_max = v[2];
    }
  }
  if (t.n_errors) rc = fail(c, ECPIC_EPUSH, "particle push failed");
  return rc;
}

extern "C" {

ecpic_status ecpic_step(ecpic_ctx* x, const ecpic_step_opts* o, ecpic_step_stats* st) {
  if (!x || !o) return ECPIC_EINVAL;
  ENSURE_DEVICE(x->c);
  return step_impl(x->c, o, st, false, false);
}

ecpic_status ecpic_run(ecpic_ctx* x, const ecpic_step_opts* o, int32_t n_steps, int32_t* done,
                       ecpic_step_stats* last) {
  if (done) *done = 0;
  if (!x || !o || n_steps < 0) return ECPIC_EINVAL;
  Ctx& c = x->c;
  ENSURE_DEVICE(c);
  bool ready = false;
  for (int32_t k = 0; k < n_steps; ++k) {
    const bool more = k + 1 < n_steps;
    const ecpic_status rc = step_impl(c, o, more ? nullptr : last, ready, more);
    if (rc != ECPIC_OK) {
      if (ready || more) {
        // a guess enqueued for a step that will not run is harmless (it
        // writes only the iterate and half-step buffers), but let the
        // stream settle before returning an error
        (void)hipStreamSynchronize(c.stream);
      }
      return rc;
    }
    ready = more;
    if (done) *done = k + 1;
  }
  return ECPIC_OK;
}

}  // extern "C"
