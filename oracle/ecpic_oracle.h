/*
 * ecpic_oracle.h -- plain FP64 CPU oracle of one implicit step of the
 * energy- and charge-conserving electromagnetic PIC/MCC method on an
 * axisymmetric r-z grid (Eremin et al., Sec. 2.1, Eqs. (1)-(4)).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.
 * Only the test-suite, the smoke check and the CPU-baseline timing may load
 * it.  It shares no source, header, table or constant with the HIP library.
 *
 * Conventions (all arrays are caller-owned host memory, row-major, FP64):
 *   ur[i][j], 0<=i<nr, 0<=j<=nz : voltage of the r-edge (i+1/2, j)  [V]
 *   uz[i][j], 0<=i<=nr, 0<=j<nz : voltage of the z-edge (i, j+1/2)  [V]
 *   h [i][j], 0<=i<nr, 0<=j<nz  : H_theta at the cell centre        [A/m]
 *   Ir, Iz have the shapes of ur, uz: current through the dual face [A]
 *   Node arrays (charge) are [nr+1][nz+1].
 * Logical particle positions xi in [0,nr], eta in [0,nz] are in cell units.
 */
#ifndef ECPIC_ORACLE_H
#define ECPIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OG_MAX_DRIVE 32

typedef struct {
  int32_t nr, nz;
  double R, L, xi_a;            /* radius, height [m]; axis map parameter   */
  double dt, eps, mu;           /* time step [s]; permittivity, permeability */
  int32_t n_drive;              /* number of drive harmonics on the gap edge
                                   (0..OG_MAX_DRIVE)                          */
  int32_t self_b;               /* test option: mu*h as B_theta on particles */
  double drive_amp[OG_MAX_DRIVE], drive_freq[OG_MAX_DRIVE], drive_phase[OG_MAX_DRIVE];
  double drive_t_end;           /* > 0: the drive is off from this time on    */
  double bz_ext;                /* test option: uniform external B_z [T]     */
  double er_ext;                /* test option: external E_r = er_ext*r/R    */
  double sub_tol;               /* inner fixed-point tolerance (0 -> 1e-14)  */
  int32_t push_only;            /* 1: no field solver (push passes only; the
                                   banded factorisation is skipped, and
                                   og_field_solve / og_step return -5)       */
  int32_t model;                /* OG_EM (Eq. (2)) or OG_ES (Eq. (8))        */
  double cap;                   /* > 0: the drive reaches the powered
                                   electrode through a blocking capacitor of
                                   this capacitance [F] (Eq. (6)); the gap
                                   voltage is then the electrode potential   */
  int32_t port_i;               /* > 0: the drive enters through a coaxial
                                   TEM port on the bottom wall, r-edges
                                   (i, 0) with port_i <= i < nr (the powered
                                   electrode is r <= r(port_i)); 0: the
                                   delta gap on the r-edge (nr-1, 0)         */
  double port_eps;              /* relative permittivity of the port's line */
} og_grid;

#define OG_EM 0
#define OG_ES 1

typedef struct {
  double q, m, w;               /* charge [C], mass [kg], macro weight       */
  int32_t mobile;               /* 0: frozen (not pushed, no current)        */
  int32_t mcc_role;             /* 0 none, 1 electron-Ar, 2 Ar+-Ar           */
  int64_t n, cap;               /* live count and capacity of the arrays     */
  double *xi, *eta, *vr, *vt, *vz;
  uint64_t *uid;
} og_species;

typedef struct {
  double *ur, *uz, *h;          /* fields at t^n                             */
  double *ur_prev, *uz_prev;    /* u at t^{n-1} (extrapolated guess)         */
  double *wall_bot, *wall_top;  /* absorbed charge per node, [nr+1]          */
  double *wall_side;            /* absorbed charge per node, [nz+1]          */
  double t;                     /* t^n [s]                                   */
  int64_t step;                 /* n                                         */
  double phi, phi_prev;         /* electrode potential at t^n, t^{n-1} [V]   */
  double q_cap;                 /* blocking-capacitor charge at t^n [C]      */
  double *hb;                   /* port: H_theta on the wall under every port
                                   edge at t^n, [nr] (entries i >= port_i)   */
} og_state;

typedef struct {
  double tol;                   /* relative energy-norm update tolerance     */
  int32_t max_iter;             /* Picard iterations (JFNK: Newton residual
                                   evaluations) allowed (<=64)               */
  int32_t fixed_iter;           /* >0: run exactly this many iterations      */
  int32_t solver;               /* OG_PICARD or OG_JFNK                      */
  int32_t krylov;               /* JFNK: GMRES iterations per Newton step
                                   (1..OG_MAX_KRYLOV; all of them when
                                   fixed_iter > 0)                           */
  double eta;                   /* JFNK: GMRES stops at eta * |F| (tolerance
                                   mode)                                     */
} og_opts;

#define OG_PICARD 0
#define OG_JFNK 1
#define OG_MAX_KRYLOV 32

typedef struct {
  int32_t enabled;
  int32_t electron_sid, ion_sid;
  int32_t pad;
  double n_gas, T_gas;          /* neutral density [m^-3], temperature [K]   */
  double m_gas;                 /* neutral mass [kg]                         */
  double eps_max_ev;            /* electron energy bound of nu_max [eV]      */
  uint64_t seed;
} og_mcc;

typedef struct {
  int32_t iters, converged;
  double residual[64];
  double ke[4];                 /* kinetic energy per species at t^{n+1} [J] */
  double we, wb;                /* field energies at t^{n+1} [J]             */
  double w_particles;           /* sum over pushes of work q E.dx  [J]       */
  double w_field_io;            /* dt * sum_int u^{1/2}.I (field side) [J]   */
  double w_drive;               /* energy injected by the drive edge [J]     */
  double w_absorbed;            /* kinetic energy lost to walls [J]          */
  double w_coll;                /* kinetic energy lost in collisions [J]     */
  int64_t n_absorbed[4];
  int64_t n_coll[4];            /* real collisions per species               */
  int64_t n_ionized;
  int64_t n_substeps, n_crossings, n_halvings, n_errors, n_capped;
  int64_t n_over_range;         /* particles beyond the nu_max bound         */
  int32_t newton_iters;         /* JFNK: Newton residual evaluations (the
                                   residual[] entries); iters counts every
                                   push pass of the iteration               */
  int32_t krylov_iters;         /* JFNK: GMRES iterations in all             */
  double phi;                   /* electrode potential at t^{n+1} [V]        */
  double q_cap;                 /* capacitor charge at t^{n+1} [C]           */
  double w_gen;                 /* generator work dt V^{1/2} I_e [J]         */
  double port_v;                /* port: voltage across the port's mouth at
                                   t^{n+1}, sum of its edge voltages [V]     */
} og_stats;

typedef struct og_ctx og_ctx;

/* Threads a push pass uses: 1, or the OpenMP thread count in the timing
 * build (libecpic_oracle_omp.so). */
int og_threads(void);

/* Setup: derived mesh quantities and the Cholesky factor of the H_theta
 * system (Sec. 2.1, Eq. (2) with mid-point centring).  Returns 0 or <0. */
int  og_create(const og_grid* g, og_ctx** out);
void og_destroy(og_ctx* c);

/* Mapping r(xi), J_r(xi) = dr/dxi, 1/J_r and its inverse xi(r). */
double og_r_of_xi(const og_ctx* c, double xi);
double og_jr_of_xi(const og_ctx* c, double xi);
double og_xi_of_r(const og_ctx* c, double r);
/* Geometric tables: rn[nr+1] (node radii), rh[nr] (cell-centre radii),
 * area_c[nr] (meridional cell area), wr[nr] = eps*A*_r/l_r for interior
 * r-edges, wz[nr] = eps*A*_z/dz, vol_c[nr] = 2*pi*rh*area_c. */
void og_tables(const og_ctx* c, double* rn, double* rh, double* area_c,
               double* wr, double* wz, double* vol_c);

/* Drive-gap voltage V(t) on the r-edge (nr-1, 0). */
double og_drive(const og_ctx* c, double t);

/* Discrete operators used by the invariant tests.
 *   og_curl_e : (C u)[cell] = uz[i+1][j]-uz[i][j]-ur[i][j+1]+ur[i][j]
 *   og_curl_h : circulation of h around every interior edge (K h), the
 *               right-hand side of Ampere's law before the current.
 *   og_div    : net outward flux of (ur-like, uz-like) edge fluxes per node. */
void og_curl_e(const og_ctx* c, const double* ur, const double* uz, double* ce);
void og_curl_h(const og_ctx* c, const double* h, double* kr, double* kz);
void og_div(const og_ctx* c, const double* fr, const double* fz, double* dnode);

/* Crank-Nicolson field update from t to t+dt with the given currents.
 * With a port, its wall field H_b at t comes from og_set_port_h (zero at
 * create), and the solve leaves H_b at t+dt for og_get_port_h. */
int og_field_solve(og_ctx* c, const double* ur0, const double* uz0,
                   const double* h0, const double* Ir, const double* Iz,
                   double t, double* ur1, double* uz1, double* h1);

/* Port (Sec. 2.1, Eqs. (5), (7)): the wall field H_b of the port edges,
 * [nr] with entries i >= port_i, in and out of og_field_solve; the TEM
 * share kappa[i] of the mouth voltage carried by port edge i (ln of its end
 * radii over ln(R / r_p)), and the electrostatic model's wall potential
 * profile prof[nr+1] (1 on the electrode, ln(R/r)/ln(R/r_p) across the
 * mouth).  Both do nothing without a port. */
void og_set_port_h(og_ctx* c, const double* hb);
void og_get_port_h(const og_ctx* c, double* hb);
void og_port_tables(const og_ctx* c, double* kappa, double* prof);

/* One pass of the implicit push + charge-conserving deposit of one species in
 * the frozen half-step field (ur_h, uz_h, h_h).  commit=0 leaves the state
 * untouched; commit=1 writes it, removes absorbed particles (order kept) and
 * tallies wall charge.  Currents are ADDED into Ir, Iz.  st may be NULL when
 * commit=0.  Returns 0, or the negative count of particles in error. */
int og_push_deposit(og_ctx* c, og_species* s, const double* ur_h,
                    const double* uz_h, const double* h_h, int commit,
                    double* Ir, double* Iz, og_state* st, og_stats* stats);

/* One implicit step: guess, Picard iterations, commit, MCC, field shift.
 * Returns 0, -4 when not converged within max_iter (nothing committed), or
 * another negative code on error. */
int og_step(og_ctx* c, og_state* st, og_species* sp, int32_t nsp,
            const og_mcc* mcc, const og_opts* o, og_stats* stats);

/* Null-collision Monte Carlo on the current state (velocities at t^{n+1}). */
int og_collide(og_ctx* c, og_species* sp, int32_t nsp, const og_mcc* mcc,
               int64_t step, og_stats* stats);
double og_nu_max(const og_mcc* mcc, int32_t role, double m_particle);
void og_cross_sections(double eps_ev, double* s_el, double* s_ex, double* s_iz);

/* Diagnostics. */
void   og_node_charge(const og_ctx* c, const og_species* sp, int32_t nsp, double* q);
void   og_gauss(const og_ctx* c, const double* ur, const double* uz, double* g);
double og_energy_e(const og_ctx* c, const double* ur, const double* uz);
double og_energy_b(const og_ctx* c, const double* h);
double og_energy_norm2(const og_ctx* c, const double* ur, const double* uz);
double og_kinetic(const og_species* s);

/* Counter-based generator: Philox4x64 with 10 rounds. */
void og_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
uint64_t og_child_uid(uint64_t parent, int64_t step);

#ifdef __cplusplus
}
#endif
#endif
