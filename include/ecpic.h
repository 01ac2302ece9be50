/*
 * ecpic.h -- C ABI of the MI355X (gfx950) hot path of the implicit,
 * energy- and charge-conserving electromagnetic PIC/MCC method on an
 * axisymmetric r-z grid (Eremin et al., "Modeling of very high frequency
 * large-electrode capacitively coupled plasmas with a fully electromagnetic
 * particle-in-cell code", Sec. 2.1).
 *
 * Conventions
 *  - Every call returns ecpic_status (0 = ECPIC_OK, negative = error).  No
 *    exception or abort crosses the ABI; ecpic_last_error(ctx) gives a
 *    NUL-terminated message owned by the context, valid until the next call.
 *  - All work is enqueued on the HIP stream given to ecpic_create.  Calls that
 *    return host scalars (field_iterate, step, diagnostics, read_particles'
 *    count) synchronise that stream; the others are asynchronous.
 *  - Array pointers marked (device) are device memory owned by the caller;
 *    the library reads or writes them during the call (stream-ordered) and
 *    keeps no reference (ecpic_bind_fields excepted).
 *  - Device memory of the context.  ecpic_create allocates none.  All of the
 *    context's device arrays (particle SoA of every species, fields, solver
 *    tables, queues, scratch) live in one region: either a workspace the
 *    caller allocates and binds (ecpic_workspace_size, then
 *    ecpic_bind_workspace, after every ecpic_add_species; the library then
 *    never allocates device memory for them), or, if none is bound, one
 *    block the library allocates at the first call that needs the device
 *    and frees in ecpic_destroy.  Species added after that first call get
 *    allocations of their own (library-owned region only).  The training
 *    calls ecpic_nn_forward / ecpic_nn_grad grow a batch workspace of their
 *    own.  Pinned host words (residuals, summaries) are the library's.
 *  - A context is not thread-safe; calls on one context must be serialised.
 *  - Layouts (row-major, FP64):
 *      ur[i][j], 0<=i<nr, 0<=j<=nz : voltage of r-edge (i+1/2, j)      [V]
 *      uz[i][j], 0<=i<=nr, 0<=j<nz : voltage of z-edge (i, j+1/2)      [V]
 *      h [i][j], 0<=i<nr, 0<=j<nz  : H_theta at the cell centre        [A/m]
 *      Ir, Iz as ur, uz            : current through the dual faces    [A]
 *      node arrays [nr+1][nz+1]    : charge per node                   [C]
 *    Logical positions xi in [0,nr], eta in [0,nz] are in cell units.
 */
#ifndef ECPIC_H
#define ECPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ECPIC_OK = 0,
  ECPIC_EINVAL = -1,    /* invalid argument, shape or descriptor            */
  ECPIC_ENOMEM = -2,    /* device allocation failed                         */
  ECPIC_EHIP = -3,      /* HIP runtime error (message in ecpic_last_error)  */
  ECPIC_ENOTCONV = -4,  /* Picard iteration did not reach the tolerance     */
  ECPIC_EPUSH = -5,     /* a particle push failed (sub-step cap / no solve) */
  ECPIC_ECAPACITY = -6, /* species capacity exceeded by ionisation          */
  ECPIC_ERANGE = -7,    /* a particle exceeded the null-collision bound     */
  ECPIC_ENOTIMPL = -8   /* not available in this build                      */
} ecpic_status;

typedef enum {
  ECPIC_FP64 = 0,  /* FP64 particle state and push                          */
  ECPIC_MIXED = 1  /* int32 cell + FP32 offsets/velocities, FP32 push; FP64
                      current accumulation, field solve, residual, energies */
} ecpic_precision;

/* Field model.  ECPIC_MODEL_EM: the TM Maxwell system (Sec. 2.1, Eq. (2)).
 * ECPIC_MODEL_ES: the electrostatic version (Sec. 2.2, Eq. (8)): the field
 * is the gradient of a potential that solves the mapped Poisson equation,
 * here in its charge-conserving update form L (phi^{n+1} - phi^n) =
 * -dt div I over the free nodes (0 <= i < nr, 0 < j < nz), with the drive
 * voltage's change on the powered plate's nodes (the bottom nodes i < nr)
 * and zero on the grounded top, side and corner; h stays zero.  Needs
 * nz >= 2. */
typedef enum { ECPIC_MODEL_EM = 0, ECPIC_MODEL_ES = 1 } ecpic_model;

/* Grid, field constants and drive (Sec. 2.1: separable map r(xi), z(eta);
 * TM fields E_r, E_z, H_theta; PEC walls).  SI units. */
typedef struct {
  int32_t nr, nz;         /* cells in r and z                                */
  double R, L;            /* cylinder radius and height [m]                  */
  double xi_axis;         /* map parameter: r ~ sqrt(xi) below it, 0=uniform */
  double dt;              /* time step [s]                                   */
  double eps, mu;         /* permittivity, permeability of the gap           */
  int32_t n_drive;        /* harmonics on the drive gap edge (0..32)         */
  int32_t model;          /* ecpic_model                                     */
  double drive_amp[32];   /* V(t) = sum amp sin(2 pi freq t + phase) [V]     */
  double drive_freq[32];
  double drive_phase[32];
  double drive_t_end;     /* > 0: V(t) = 0 from this time on (a burst)       */
  double blocking_cap;    /* > 0: the generator V(t) reaches the powered
                             electrode through a blocking capacitor of this
                             capacitance [F] (Sec. 2.1, Eq. (6)).  The gap
                             then carries the electrode potential phi, which
                             the step iterates with the Picard iterates:
                             phi^{(k+1)} = V^{n+1} - (q^n + dt I_e^{(k)}) / C,
                             I_e the current the electrode sends into the
                             domain (EM: 2 pi r h^{n+1/2} of the gap cell
                             plus the gap edge's particle current; ES: the
                             plate nodes' field flux change over dt plus the
                             particle currents leaving them and the gap
                             edge's), and q^{n+1} = q^n + dt I_e of the
                             accepted iterate.  The residual is the larger of
                             the field update and |phi^{(k+1)} - phi^{(k)}|
                             over the sum of the drive amplitudes.  The plain
                             iteration contracts by about C_e / C (C_e the
                             electrode's capacitance to the domain, larger
                             with plasma): meant for C well above C_e.  Not
                             with the JFNK solver.  0 = the generator drives
                             the gap directly. */
  int32_t port_i;         /* > 0: the drive enters through a coaxial TEM port
                             (Sec. 2.1, Eqs. (5), (7)) instead of the gap:
                             a line filled with a dielectric of relative
                             permittivity port_eps meets the bottom wall over
                             the r-edges (i, 0), port_i <= i < nr
                             (1 <= port_i < nr); the powered electrode is the
                             wall r <= r(port_i).  EM: each port edge is a
                             free edge on the half cell above the wall, closed
                             by the line's wall field H_b (library state, zero
                             at create; ecpic_set_port_field), with the Mur
                             condition for the outgoing wave integrated over
                             the edge:
                               (u^{n+1} - u^n) + eta l (H_b^{n+1} - H_b^n)
                                 = kappa (phi^{n+1} - phi^n),
                             eta = sqrt(mu / (port_eps eps)), l the edge
                             length, kappa = ln(r_{i+1}/r_i) / ln(R/r_p) the
                             edge's share of the incoming TEM wave, phi the
                             electrode potential (the generator voltage, or
                             the blocking capacitor's electrode potential);
                             the power through the mouth is the drive's work
                             (w_drive).  ES: the port is the Dirichlet wall
                             with the static coaxial potential phi
                             ln(R/r)/ln(R/r_p) across the mouth (Sec. 2.2).
                             With the capacitor, I_e is Eq. (6)'s current
                             through the electrode's face r <= r_p (EM: the
                             Ampere loop 2 pi r h^{n+1/2} of the first port
                             cell).  Particles reaching the mouth stick to it:
                             they leave the plasma and their charge is
                             tallied on the wall nodes.  0 = the delta gap. */
  double port_eps;        /* relative permittivity of the port's line (> 0)  */
} ecpic_grid_desc;

typedef struct {
  double q, m;            /* charge [C], mass [kg]                           */
  double weight;          /* physical particles per macro-particle           */
  int64_t capacity;       /* maximum macro-particles held                    */
  int32_t mobile;         /* 0: frozen (not pushed, no current)              */
  int32_t sort_stride;    /* the sorts a step makes (ecpic_step_opts
                             sort_every) include this species at every
                             sort_stride-th of them, counted from step 0
                             (0 or 1: at every one): for a species that
                             hardly moves between sorts (cold ions), whose
                             order keeps.  ecpic_sort sorts every species.
                             Negative: EINVAL.                             */
} ecpic_species_desc;

/* Null-collision Monte Carlo (Sec. 2.1) with synthetic argon cross-sections:
 * e-Ar elastic, one excitation (11.5 eV), ionisation (15.76 eV); Ar+-Ar
 * charge exchange.  Random numbers: Philox4x64-10, key (seed, species id),
 * counter (particle id, step, block, 0). */
typedef struct {
  int32_t enabled;
  int32_t electron_sid, ion_sid;
  int32_t reserved;
  double n_gas, t_gas;    /* neutral density [m^-3] and temperature [K]      */
  double m_gas;           /* neutral mass [kg]                               */
  double eps_max_ev;      /* energy bound of the null-collision rate [eV]    */
  uint64_t seed;
} ecpic_mcc_desc;

typedef struct {
  double tol;             /* energy-norm relative update tolerance           */
  int32_t max_iter;       /* Picard iterations allowed (1..64)               */
  int32_t fixed_iter;     /* >0: exactly this many iterations (parity mode)  */
  int32_t sort_every;     /* counting sort by cell every k steps (0 = never) */
  int32_t use_nn;         /* 1: learned initial guess (see ecpic_nn_*)       */
  int32_t check_conservation; /* 1: fill gauss_max, continuity_max, q_max of
                             the step's statistics (one node-charge pass
                             over the particles per step, plus one at the
                             first checked step)                             */
  int32_t solver;         /* ecpic_solver: the nonlinear iteration            */
  int32_t krylov;         /* JFNK: GMRES iterations per Newton step, 1 up to
                             the space reserved with ECPIC_OPT_JFNK_KRYLOV
                             (all of them when fixed_iter > 0)               */
  double eta;             /* JFNK: GMRES stops once its residual estimate is
                             <= eta |F| (tolerance mode)                     */
} ecpic_step_opts;

/* The nonlinear iteration of the step (Sec. 2.1 names both).
 * ECPIC_SOLVER_PICARD: u^{(k+1)} = G(u^{(k)}), where G pushes every species
 * in (u^n + u^{(k)}) / 2, deposits, and solves the field equations.
 * ECPIC_SOLVER_JFNK: Newton on F(u) = u - G(u): J d = -F with J = I - G',
 * J v by the forward difference (G(u + e v) - G(u)) / e with
 * e = 1e-6 max(|u|, |F|) / |v| in the energy norm (G carries the
 * deposit's rounding and the 1e-14 inner-solve tolerance: a relative step of
 * sqrt(eps_mach) leaves the Krylov directions after the first mostly
 * noise), GMRES from
 * d = 0 (Arnoldi by classical Gram-Schmidt applied twice, energy inner
 * product, Givens rotations, no restart), and in tolerance mode the step
 * u + l d with l halved at most 8 times until |F| falls by 1 - 1e-4 l.
 * max_iter / fixed_iter count Newton residual evaluations; stats.iters
 * counts every push pass (each evaluation of G), stats.residual holds the
 * Newton residuals |F| / |G(u)|.  The accepted state is that of Picard:
 * fields G(u), particles pushed in (u^n + u) / 2. */
typedef enum { ECPIC_SOLVER_PICARD = 0, ECPIC_SOLVER_JFNK = 1 } ecpic_solver;

typedef struct {
  int32_t iters, converged;
  int32_t used_nn, nn_fallback;
  double residual[64];
  double ke[4];           /* kinetic energy per species at t^{n+1} [J]       */
  double we, wb;          /* electric and magnetic field energy [J]          */
  double w_particles;     /* work done on particles by the field [J]         */
  double w_field_io;      /* field-side energy exchange with the current [J] */
  double w_drive;         /* energy injected by the drive gap [J]            */
  double w_absorbed;      /* kinetic energy lost to the walls [J]            */
  double w_coll;          /* kinetic energy lost in collisions [J]           */
  int64_t n_alive[4];
  int64_t n_absorbed[4];
  int64_t n_coll[4];
  int64_t n_ionized;
  int64_t n_substeps, n_crossings, n_errors, n_over_range;
  double t;               /* time after the step [s]                         */
  int64_t step;           /* step counter after the step                     */
  /* With check_conservation (Sec. 2.1: the charge-conserving current keeps
   * Gauss's law once it holds).  Q = particle node charge (bilinear
   * weights) plus the wall charge on the wall nodes; div = net flux out of a
   * node's dual cell.  All in coulombs, maxima over nodes:                   */
  double continuity_max;  /* |Q^{n+1} - Q^n + dt div I| over every node, with
                             I the currents of the accepted iterate          */
  double gauss_max;       /* |(G - Q_p)^{n+1} - (G - Q_p)^n| over the nodes
                             off the conducting walls (0<=i<nr, 0<j<nz), G
                             = div of the displacement flux eps Ad u / l,
                             Ad the dual-face area of an edge of length l   */
  double q_max;           /* max |Q_p^{n+1}|, the scale of the two above     */
  int32_t newton_iters;   /* JFNK: Newton residual evaluations (entries of
                             residual[]); 0 for Picard                       */
  int32_t krylov_iters;   /* JFNK: GMRES iterations over the step            */
  double electrode_v;     /* blocking capacitor: electrode potential phi at
                             t^{n+1} [V] (else the generator voltage)        */
  double cap_charge;      /* blocking capacitor: its charge q^{n+1} [C]      */
  double w_gen;           /* blocking capacitor: the generator's work
                             dt V^{1/2} I_e [J] (= w_drive + the capacitor's
                             energy change)                                  */
  double port_v;          /* port: voltage across its mouth at t^{n+1}, the
                             sum of the port edges' voltages [V]             */
} ecpic_step_stats;

typedef struct ecpic_ctx ecpic_ctx;

/* Create a context for the grid (Sec. 2.1 mesh and TM field model) and
 * factorise the H_theta system.  hip_stream: a hipStream_t (NULL = default
 * stream).  Fields start at zero, t = 0, step = 0.  EINVAL on bad shapes or
 * non-positive constants, ENOMEM/EHIP on device failures.  Shapes: nr <=
 * 2048, nz <= 1024 and ceil(nr/4) * ceil(nz/32) <= 8192 (1024 x 1024 and
 * 2048 x 512 fit), the limits of the field solve's blocking and of the
 * kernels' per-row LDS arrays; EINVAL beyond. */
ecpic_status ecpic_create(const ecpic_grid_desc* grid, ecpic_precision prec, void* hip_stream,
                          ecpic_ctx** out);
ecpic_status ecpic_destroy(ecpic_ctx* ctx);

/* Add a species with room for desc->capacity macro-particles (at most 2^29
 * per species).  Up to 4 species.  *sid receives its index.  Its device
 * buffers come with the context's region (see the conventions).  EINVAL for
 * a bad descriptor, a fifth species, or a species added after a workspace
 * was bound; ENOMEM if a library allocation fails. */
ecpic_status ecpic_add_species(ecpic_ctx* ctx, const ecpic_species_desc* desc, int32_t* sid);

/* Bytes of device memory the context needs for its grid and the species
 * added so far (all particle buffers, fields, solver tables, queues and
 * scratch), as ecpic_bind_workspace expects them.  Host only. */
ecpic_status ecpic_workspace_size(const ecpic_ctx* ctx, size_t* bytes);

/* Give the context its device memory: ws (device, 256-byte aligned, at
 * least ecpic_workspace_size bytes) is owned by the caller, who keeps it
 * alive until ecpic_destroy and frees it afterwards; the library carves
 * every device array from it and allocates none of its own for them.  Must
 * come after the last ecpic_add_species and before any call that touches the
 * device.  The solver tables are uploaded and the state cleared here
 * (synchronises).  EINVAL if device memory is already in use or ws is
 * misaligned, ENOMEM if bytes is too small. */
ecpic_status ecpic_bind_workspace(ecpic_ctx* ctx, void* ws, size_t bytes);

/* Field arrays of the state in the caller's memory (device, FP64, layouts as
 * above). */
typedef struct {
  double *ur, *uz, *h;                /* u at t^n                            */
  double *ur_prev, *uz_prev, *h_prev; /* u at t^{n-1}                        */
} ecpic_field_view;

/* Keep the field state in the caller's arrays (six distinct device arrays,
 * owned by the caller and kept alive while bound): their current contents
 * become u^n and u^{n-1} (as ecpic_set_fields would set them, without a
 * copy), and every committed step leaves the new u^n and u^{n-1} in the same
 * arrays (a copy kernel per step), so the caller reads the state in place.
 * view = NULL unbinds: the state is copied back into the library's arrays
 * (synchronises).  EINVAL for a null or repeated array. */
ecpic_status ecpic_bind_fields(ecpic_ctx* ctx, const ecpic_field_view* view);

/* Replace the particles of a species.  r, z: physical positions [m] inside
 * (0,R]x(0,L); vr, vt, vz [m/s]; uid: identifiers (RNG counters).  All
 * (device), length n <= capacity.  Positions are mapped to logical (xi, eta)
 * on the device.  EINVAL if n exceeds the capacity. */
ecpic_status ecpic_load_particles(ecpic_ctx* ctx, int32_t sid, const double* r, const double* z,
                                  const double* vr, const double* vt, const double* vz,
                                  const uint64_t* uid, int64_t n);

/* Copy the live particles of a species, in storage order, as FP64 logical
 * positions and velocities (device outputs of length cap).  *n_out receives
 * the count (synchronises).  EINVAL if cap is too small. */
ecpic_status ecpic_read_particles(ecpic_ctx* ctx, int32_t sid, double* xi, double* eta,
                                  double* vr, double* vt, double* vz, uint64_t* uid, int64_t cap,
                                  int64_t* n_out);

/* Set the field state: u at t^n (ur, uz, h) and u at t^{n-1} for the
 * extrapolated guess (NULL: same as t^n), plus the clock.  (device) */
ecpic_status ecpic_set_fields(ecpic_ctx* ctx, const double* ur, const double* uz, const double* h,
                              const double* ur_prev, const double* uz_prev, double t, int64_t step);
ecpic_status ecpic_get_fields(ecpic_ctx* ctx, double* ur, double* uz, double* h);

/* The TEM port's wall field H_b at t^n (Sec. 2.1, Eq. (5); see port_i):
 * hb[nr] (host), entries i >= port_i used, the others ignored (set) or
 * zero (get).  The field solves and steps read it; a committed EM step
 * moves it to t^{n+1}.  EINVAL without a port.  (host, synchronises) */
ecpic_status ecpic_set_port_field(ecpic_ctx* ctx, const double* hb);
ecpic_status ecpic_get_port_field(ecpic_ctx* ctx, double* hb);

/* Set the frozen half-step field u^{n+1/2} used by ecpic_push_deposit. (device) */
ecpic_status ecpic_set_half_field(ecpic_ctx* ctx, const double* ur_half, const double* uz_half);

/* One pass of the implicit push (Eq. (4), mid-point centring, each orbit
 * split at every cell-face crossing) and charge-conserving deposit (Eq. (3),
 * spline order 1) of every mobile species in the current half-step field.
 * commit=0: particle state is read only and the currents I are recomputed;
 * commit=1: state written, wall absorption applied.  Ir, Iz: optional
 * (device) outputs receiving a copy of the currents.  EPUSH if a particle
 * failed (state left as far as it got). */
ecpic_status ecpic_push_deposit(ecpic_ctx* ctx, int32_t commit, double* Ir, double* Iz);

/* Stateless Crank-Nicolson solve of the TM equations (Eq. (2), mid-point
 * centring) from (ur0, uz0, h0) at time t with currents (Ir, Iz), writing the
 * fields at t+dt.  H_theta is the unknown; the drive gap edge takes
 * V(t+dt).  All arrays (device). */
ecpic_status ecpic_field_solve(ecpic_ctx* ctx, const double* ur0, const double* uz0,
                               const double* h0, const double* Ir, const double* Iz, double t,
                               double* ur1, double* uz1, double* h1);

/* The solve of ecpic_field_solve (same arguments, same results), for
 * callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation.  Its one scratch
 * array, the [nz][nr] transform intermediate, is a static device array of
 * the library (2^20 doubles, 8 MiB, on each GPU it runs on, held until the
 * process ends) instead of the context's region; the call allocates nothing
 * and needs nothing cleared (the solve writes every element it reads).
 * Limit: nr * nz <= 2^20 cells (EINVAL beyond), which every grid
 * ecpic_create accepts meets.  The context's device
 * memory must already be in place (after ecpic_bind_workspace or any
 * earlier call that touches the device): EINVAL otherwise.  Every call on
 * one GPU shares the array: calls that overlap on one GPU (different
 * streams, or contexts used from several threads) race. */
ecpic_status ecpic_field_solve_noalloc(ecpic_ctx* ctx, const double* ur0, const double* uz0,
                                       const double* h0, const double* Ir, const double* Iz,
                                       double t, double* ur1, double* uz1, double* h1);

/* One field iterate of the Picard loop: solve with the currents of the last
 * push_deposit, store u^{n+1,(k+1)}, h^{n+1,(k+1)} and the next half-step
 * field, and return r_k = |u^(k+1)-u^(k)|_E / |u^(k+1)|_E (synchronises). */
ecpic_status ecpic_field_iterate(ecpic_ctx* ctx, double* rel_update);

/* Null-collision Monte Carlo on the current velocities (Sec. 2.1), at the
 * given step index (RNG counter), in place.  ECAPACITY: an ionisation whose
 * electron-ion pair did not fit was not applied (its electron keeps its
 * velocity; every other collision was applied).  ERANGE: the collisions
 * were applied, and some particle's collision rate exceeded the
 * null-collision bound (raise eps_max_ev). */
ecpic_status ecpic_collide(ecpic_ctx* ctx, const ecpic_mcc_desc* mcc, int64_t step);

/* Collision model used by ecpic_step (NULL or enabled=0 turns MCC off). */
ecpic_status ecpic_set_mcc(ecpic_ctx* ctx, const ecpic_mcc_desc* mcc);

/* One implicit step: extrapolated (or learned) guess, Picard iterations of
 * push_deposit + field_iterate until r_k <= tol (or fixed_iter passes),
 * commit of the particles pushed in the accepted half-step field, MCC,
 * optional sort, field shift.  stats may be NULL.  A step that returns
 * ENOTCONV, ECAPACITY (an ionisation's electron-ion pair did not fit in a
 * species' capacity) or ERANGE (a particle's collision rate exceeded the
 * null-collision bound, eps_max_ev) is not committed: particles, counts,
 * fields, wall charge and clock are as before the call (stats are filled).
 * EPUSH: committed, with n_errors particles whose push failed. */
ecpic_status ecpic_step(ecpic_ctx* ctx, const ecpic_step_opts* opts, ecpic_step_stats* stats);

/* n_steps implicit steps with the same options, back to back in the library
 * (Sec. 2.1 per step, as ecpic_step).  Between steps the next step's
 * extrapolated guess is enqueued before the host reads the commit summary,
 * so the stream does not wait for the host.  Stops at the first step that
 * does not return ECPIC_OK and returns its status (ENOTCONV leaves that
 * step's state and fields untouched); *done (may be NULL) receives the
 * number of steps completed.  last (may be NULL) receives the statistics of
 * the last step (computing them costs a few reductions).  n_steps < 0 is
 * ECPIC_EINVAL; 0 does nothing. */
ecpic_status ecpic_run(ecpic_ctx* ctx, const ecpic_step_opts* opts, int32_t n_steps, int32_t* done,
                       ecpic_step_stats* last);

/* Counting sort of every species by cell (the order the fast pass's
 * per-block current tiles rely on), dropping absorbed particles.  Slots come
 * out in nondecreasing cell order; the order of the particles within a cell
 * is not specified (it depends on the order of device atomics).  Device
 * work on the context's stream; synchronises to read the new counts. */
ecpic_status ecpic_sort(ecpic_ctx* ctx);

/* Node charge of all species with logical bilinear weights into q (device,
 * [nr+1][nz+1]); wall charge absorbed so far into bot[nr+1], top[nr+1],
 * side[nz+1] (device, each optional). */
ecpic_status ecpic_node_charge(ecpic_ctx* ctx, double* q, double* bot, double* top, double* side);

/* Energies and counts of the current state (synchronises). */
ecpic_status ecpic_diagnostics(ecpic_ctx* ctx, ecpic_step_stats* stats);

/* Learned initial guess (not part of the paper: an initial guess for the
 * Picard iteration of Sec. 2.1, which still converges to the same tolerance).
 * A 4-layer 3x3 convolutional network, 6 -> 32 -> 32 -> 32 -> 2 channels,
 * ReLU between layers, zero padding, on the (nr+1) x (nz+1) canvas where
 * u_r[i][j], u_z[i][j] and h[i][j] sit at index (i, j) (zero elsewhere).
 * Input channels: u_r, u_z, h at t^n and u_r, u_z, h at t^n minus t^{n-1},
 * each divided by its scale.  Output channels: the corrections of the
 * extrapolated guess 2u^n - u^{n-1} of u_r and u_z at t^{n+1}, in units of
 * their scales, used on the interior r-edges (i < nr, 0 < j < nz) and the
 * z-edges off the PEC wall (i < nr, j < nz).
 * Weights: FP32 in the canonical layout, per layer W_l[cout][cin][3][3]
 * then b_l[cout], layers concatenated (ecpic_nn_param_count floats).  The
 * kernels round weights, inputs and activations to BF16 (nearest even) and
 * accumulate in FP32 on the matrix cores; biases stay FP32.
 * ecpic_nn_param_count returns the number of weights plus biases. */
int64_t ecpic_nn_param_count(void);
/* Install the network for ecpic_step with use_nn = 1: weights w (device,
 * FP32, copied) and scales norm (host, 8 floats: 6 input, 2 output, > 0).
 * w = NULL uninstalls it.  EINVAL on bad scales. */
ecpic_status ecpic_nn_set_weights(ecpic_ctx* ctx, const float* w, const float* norm);
/* Forward pass on a batch of canvases: x (device, [batch][6][nr+1][nz+1]
 * BF16 bit patterns, already scaled) into y (device, [batch][2][nr+1][nz+1]
 * FP32, in output-scale units).  Weights w as above (device, FP32). */
ecpic_status ecpic_nn_forward(ecpic_ctx* ctx, const float* w, const uint16_t* x, float* y,
                              int32_t batch);
/* Loss and gradient for training: mean over the batch and the valid output
 * positions of (y - t)^2, with t (device FP32, shaped like y); the gradient
 * of the loss with respect to every weight and bias goes to dw (device,
 * FP32, canonical layout), the loss to *loss (host, may be NULL).
 * Synchronises. */
ecpic_status ecpic_nn_grad(ecpic_ctx* ctx, const float* w, const uint16_t* x, const float* t,
                           int32_t batch, float* dw, float* loss);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, step count t >= 1, learning
 * rate lr > 0) in place on FP32 weights w with moments m, v (all device,
 * param_count floats) from the gradient dw. */
ecpic_status ecpic_nn_adam(ecpic_ctx* ctx, float* w, float* m, float* v, const float* dw,
                           float lr, int32_t t);

/* Kernel timing with HIP events recorded on the context stream around every
 * launch of the hot kernels (one record per launch), for measurement. */
typedef enum {
  ECPIC_K_PUSH = 0,         /* in-cell push + deposit of a Picard iteration,
                               all particles of one species                  */
  ECPIC_K_PUSH_SLOW = 1,    /* the same pass for the particles that cross
                               cell faces (split sub-steps)                  */
  ECPIC_K_COMMIT = 2,       /* committing in-cell push + absorption + MCC    */
  ECPIC_K_COMMIT_SLOW = 3,  /* committing push of the face-crossing ones     */
  ECPIC_K_FIELD = 4,        /* one field solve (rhs+DCT, scan, iDCT+recover) */
  ECPIC_K_SORT = 5,         /* counting sort of one species                  */
  ECPIC_K_PUSH_COMMIT = 6,  /* a Picard iteration's in-cell pass that also
                               commits (into the other particle buffer), run
                               when the residual trend predicts convergence */
  ECPIC_K_COUNT = 7
} ecpic_kernel_kind;

typedef struct {
  int64_t launches[ECPIC_K_COUNT];    /* timed launches                     */
  double ms[ECPIC_K_COUNT];           /* their summed event-measured times  */
  double bytes[ECPIC_K_COUNT];        /* their summed algorithmic HBM bytes */
  int64_t particles[ECPIC_K_COUNT];   /* their summed particles processed   */
  int64_t calls[ECPIC_K_COUNT];       /* every launch of an enabled kind,
                                         timed or not                       */
  int64_t call_particles[ECPIC_K_COUNT]; /* particles of those launches     */
} ecpic_profile;

/* Choose the kinds to time: bit k of kind_mask enables ECPIC_K_* kind k
 * (ECPIC_PROFILE_ALL = every kind, 0 = off).  Each timed launch costs two
 * event records on its stream, so a narrow mask perturbs the run least.
 * Launches of a speculative Picard iteration that turns out not to be needed
 * are not counted.  Any call clears the totals. */
#define ECPIC_PROFILE_ALL 0x7F
ecpic_status ecpic_set_profiling(ecpic_ctx* ctx, int32_t kind_mask);
/* Time only every `every`-th launch of each enabled kind (1, the default,
 * times all of them); `calls` and `call_particles` still count every launch.
 * Sampling keeps the event records from stretching a timed run.  every < 1
 * is ECPIC_EINVAL.  Clears the totals like ecpic_set_profiling. */
ecpic_status ecpic_set_profiling_every(ecpic_ctx* ctx, int32_t every);
/* Totals since profiling was turned on (synchronises). */
ecpic_status ecpic_get_profile(ecpic_ctx* ctx, ecpic_profile* out);

/* Switches: kernel builds (the results are the same to the inner-solve
 * tolerance; they exist for tuning and so that every compiled build can be
 * compared with the CPU reference at small sizes) and a test switch. */
typedef enum {
  ECPIC_OPT_QUEUE_WAVES = 0, /* the plain slow pass (face crossers, Eq. (4)
                                split at crossings): 0 = chosen by size (the
                                build for three wavefronts per SIMD from 16M
                                particles per pass, else two), 2 or 3 = that
                                build always                                 */
  ECPIC_OPT_NN_FORCE_FALLBACK = 1, /* test switch for the learned guess's
                                fallback: k >= 1 makes a step that uses the
                                learned guess treat residual k as not falling
                                (the fallback to the extrapolated guess is
                                then taken at iteration k, as for a real rise);
                                0 = off (the default)                        */
  ECPIC_OPT_JFNK_KRYLOV = 2  /* Krylov vectors reserved for the JFNK solver,
                                0..32 (default 0: JFNK unavailable).  Adds
                                (value + 7) field-sized vectors to the device
                                layout, so it must be set before the device
                                memory is set up (before ecpic_workspace_size
                                and ecpic_bind_workspace, or the first call
                                that touches the device); later: EINVAL      */
} ecpic_option;
/* Set a switch.  EINVAL for an unknown option or value. */
ecpic_status ecpic_set_option(ecpic_ctx* ctx, int32_t option, int64_t value);

const char* ecpic_last_error(const ecpic_ctx* ctx);
const char* ecpic_status_string(ecpic_status s);

#ifdef __cplusplus
}
#endif
#endif
