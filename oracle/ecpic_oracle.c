/*
 * ecpic_oracle.c -- plain FP64 CPU oracle of the implicit energy- and
 * charge-conserving electromagnetic PIC/MCC step on an axisymmetric r-z
 * grid, written from Eremin et al., "Modeling of very high frequency
 * large-electrode capacitively coupled plasmas with a fully electromagnetic
 * particle-in-cell code", Sec. 2.1.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline timing, never by the product path.  Single-threaded, particle
 * load order, no blocking or fusion beyond what the method states.  The
 * same source built with OpenMP (a second library, used only to time the
 * CPU baseline on all host cores) runs the particle loop of a push pass in
 * parallel, each thread into its own current arrays, summed in thread
 * order; everything else stays as written.
 *
 * What each part follows:
 *   mapping            Sec. 2.1 (separable r(xi), z(eta); r ~ sqrt(xi) near
 *                      the axis so that r*J_r is constant there)
 *   fields             Eq. (2) (TM set E_r, E_z, H_theta) on the Yee mesh,
 *                      in finite-integration form, mid-point centring
 *   current deposit    Eq. (3) with spline order m = 1, orbit-averaged over
 *                      each sub-step (charge-conserving, Sec. 2.1)
 *   particle push      Eq. (4) with mid-point centring, split at every
 *                      cell-face crossing (Sec. 2.1)
 *   nonlinear solve    Picard iteration of the coupled system (Sec. 2.1)
 *   collisions         null-collision Monte Carlo (Sec. 2.1) with synthetic
 *                      analytic argon cross-sections
 */
#include "ecpic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OG_PI 3.14159265358979323846
#define OG_QE 1.602176634e-19 /* elementary charge [C], CODATA 2018 */
#define OG_KB 1.380649e-23    /* Boltzmann constant [J/K]            */
#define OG_MAX_SUB 64         /* sub-steps per particle per step     */
#define OG_MAX_HALVE 20       /* halvings of a failing sub-step      */
#define OG_MAX_FP 50          /* fixed-point iterations per solve    */

struct og_ctx {
  og_grid g;
  double s;      /* radial scale: r = s*(xi+xi_a) in the linear part */
  double dz;     /* axial cell size (= J_z)                          */
  double *rn;    /* node radii r(i), nr+1                            */
  double *rh;    /* cell-centre radii r(i+1/2), nr                   */
  double *ell;   /* r-edge lengths r(i+1)-r(i), nr                   */
  double *area;  /* meridional cell area ell*dz, nr                  */
  double *azs;   /* dual area of a z-edge, nr (i<nr)                 */
  double *wr;    /* eps*A*_r/ell of an interior r-edge, nr           */
  double *wz;    /* eps*A*_z/dz of a z-edge, nr                      */
  int64_t ncell; /* nr*nz                                            */
  int64_t nunk;  /* unknowns of the factorised system: the cells     */
                 /* (EM) or the free nodes nr*(nz-1) (ES)            */
  int32_t band;  /* Cholesky half bandwidth (nz, or nz-1 for ES)     */
  double *chol;  /* banded lower factor, nunk*(band+1)               */
  double *rhs, *x, *tr, *tz; /* work                                 */
  int gap_set;              /* 1: the solves take the gap voltages below */
  double gap_now, gap_next; /* gap voltage at t^n and t^{n+1}            */
  /* TEM port (Sec. 2.1, Eqs. (5), (7)), edges (i, 0), ip <= i < nr */
  int ip;                   /* first port edge, 0: no port                */
  double eta_p;             /* wave impedance of the line sqrt(mu/eps_l)  */
  double *pk;               /* kappa: TEM share of the mouth voltage, nr  */
  double *pg;               /* 1 / (w_b/dt + M/(2 eta l)), nr             */
  double *pprof;            /* ES wall potential profile, nr+1            */
  double *hb0, *hb1;        /* H_b at t^n (input), t^{n+1} (last solve)   */
};

/* ------------------------------------------------------------------------ */
/* Mapping (Sec. 2.1: r = r(xi) with r ~ sqrt(xi) for a few points next to  */
/* the axis and r ~ xi elsewhere; C^1 two-piece reading).                   */
/* ------------------------------------------------------------------------ */
double og_r_of_xi(const og_ctx* c, double xi) {
  const double xa = c->g.xi_a, s = c->s;
  if (xi < xa) return 2.0 * s * sqrt(xi * xa);
  return s * (xi + xa);
}

double og_jr_of_xi(const og_ctx* c, double xi) {
  const double xa = c->g.xi_a, s = c->s;
  if (xi < xa) return s * sqrt(xa / xi);
  return s;
}

/* 1/J_r, finite (zero) on the axis of the square-root region. */
static double inv_jr(const og_ctx* c, double xi) {
  const double xa = c->g.xi_a, s = c->s;
  if (xi < xa) return sqrt(xi / xa) / s;
  return 1.0 / s;
}

double og_xi_of_r(const og_ctx* c, double r) {
  const double xa = c->g.xi_a, s = c->s;
  if (r < 2.0 * s * xa) return r * r / (4.0 * s * s * xa);
  return r / s - xa;
}

double og_drive(const og_ctx* c, double t) {
  double v = 0.0;
  if (c->g.drive_t_end > 0.0 && t >= c->g.drive_t_end) return 0.0;
  for (int k = 0; k < c->g.n_drive && k < OG_MAX_DRIVE; ++k)
    v += c->g.drive_amp[k] * sin(2.0 * OG_PI * c->g.drive_freq[k] * t + c->g.drive_phase[k]);
  return v;
}

/* ------------------------------------------------------------------------ */
/* Index helpers                                                             */
/* ------------------------------------------------------------------------ */
#define UR(i, j) ((int64_t)(i) * (nz + 1) + (j))
#define UZ(i, j) ((int64_t)(i) * nz + (j))
#define HC(i, j) ((int64_t)(i) * nz + (j))

/* ------------------------------------------------------------------------ */
/* Discrete operators of Eq. (2) in integral form                           */
/* ------------------------------------------------------------------------ */

/* Faraday: mu * A_c * dh/dt equals the circulation of E around the cell,
 * oriented so that mu dH/dt = dE_z/dr - dE_r/dz (Eq. (2), first line). */
void og_curl_e(const og_ctx* c, const double* ur, const double* uz, double* ce) {
  const int nr = c->g.nr, nz = c->g.nz;
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nz; ++j)
      ce[HC(i, j)] = uz[UZ(i + 1, j)] - uz[UZ(i, j)] - ur[UR(i, j + 1)] + ur[UR(i, j)];
}

/* Ampere: circulation of H_theta around the dual face of every edge.
 * r-edge: -2 pi r_{i+1/2} (h[i][j] - h[i][j-1])        (dual ring, -dH/dz)
 * z-edge:  2 pi (r_{i+1/2} h[i][j] - r_{i-1/2} h[i-1][j]) ((1/r) d(rH)/dr)
 * Boundary edges (PEC walls) get zero. */
void og_curl_h(const og_ctx* c, const double* h, double* kr, double* kz) {
  const int nr = c->g.nr, nz = c->g.nz;
  for (int i = 0; i < nr; ++i) {
    kr[UR(i, 0)] = 0.0;
    kr[UR(i, nz)] = 0.0;
    for (int j = 1; j < nz; ++j)
      kr[UR(i, j)] = -2.0 * OG_PI * c->rh[i] * (h[HC(i, j)] - h[HC(i, j - 1)]);
  }
  for (int i = 0; i <= nr; ++i)
    for (int j = 0; j < nz; ++j) {
      if (i == nr) { kz[UZ(i, j)] = 0.0; continue; }
      double v = 2.0 * OG_PI * c->rh[i] * h[HC(i, j)];
      if (i > 0) v -= 2.0 * OG_PI * c->rh[i - 1] * h[HC(i - 1, j)];
      kz[UZ(i, j)] = v;
    }
}

/* Net outward flux per node of edge fluxes fr (r-edges) and fz (z-edges). */
void og_div(const og_ctx* c, const double* fr, const double* fz, double* d) {
  const int nr = c->g.nr, nz = c->g.nz;
  for (int i = 0; i <= nr; ++i)
    for (int j = 0; j <= nz; ++j) {
      double v = 0.0;
      if (i < nr) v += fr[UR(i, j)];
      if (i > 0) v -= fr[UR(i - 1, j)];
      if (j < nz) v += fz[UZ(i, j)];
      if (j > 0) v -= fz[UZ(i, j - 1)];
      d[(int64_t)i * (nz + 1) + j] = v;
    }
}

static int is_int_r_edge(const og_ctx* c, int j) { return j > 0 && j < c->g.nz; }

/* ------------------------------------------------------------------------ */
/* Banded Cholesky of the SPD H_theta system                                 */
/* ------------------------------------------------------------------------ */
#define LB(k, d) c->chol[(int64_t)(k) * (b + 1) + (d)] /* L[k][k-d] */

static void add_entry(og_ctx* c, int64_t a, int64_t bcol, double v) {
  /* accumulate A[a][bcol] (lower triangle only) */
  const int b = c->band;
  if (bcol > a) { int64_t t = a; a = bcol; bcol = t; }
  LB(a, a - bcol) += v;
}

static int chol_factor(og_ctx* c);

static int factorize(og_ctx* c) {
  const int nr = c->g.nr, nz = c->g.nz, b = c->band;
  const int64_t N = c->ncell;
  const double dt = c->g.dt, mu = c->g.mu;
  memset(c->chol, 0, sizeof(double) * (size_t)N * (size_t)(b + 1));
  /* Assemble M (P + C D^-1 C^T M) with M = diag(2 pi r_{i+1/2}),
   * P = diag(2 mu A_c / dt), D = diag(2 eps A* / (l dt)) on interior edges.
   * The cells touching an edge e carry coefficients C[cell][e] = +-1. */
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nz; ++j) {
      const double m = 2.0 * OG_PI * c->rh[i];
      add_entry(c, HC(i, j), HC(i, j), m * 2.0 * mu * c->area[i] / dt);
    }
  /* interior r-edges (i, j), 1 <= j < nz: cell (i,j) has +1, cell (i,j-1) -1 */
  for (int i = 0; i < nr; ++i)
    for (int j = 1; j < nz; ++j) {
      const double dinv = dt / (2.0 * c->wr[i]);
      const double m = 2.0 * OG_PI * c->rh[i];
      const int64_t a = HC(i, j), bb = HC(i, j - 1);
      add_entry(c, a, a, m * m * dinv);
      add_entry(c, bb, bb, m * m * dinv);
      add_entry(c, a, bb, -m * m * dinv);
    }
  /* interior z-edges (i, j), 0 <= i < nr: cell (i-1,j) has +1, cell (i,j) -1 */
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nz; ++j) {
      const double dinv = dt / (2.0 * c->wz[i]);
      const double mi = 2.0 * OG_PI * c->rh[i];
      add_entry(c, HC(i, j), HC(i, j), mi * mi * dinv);
      if (i > 0) {
        const double mm = 2.0 * OG_PI * c->rh[i - 1];
        add_entry(c, HC(i - 1, j), HC(i - 1, j), mm * mm * dinv);
        add_entry(c, HC(i - 1, j), HC(i, j), -mm * mi * dinv);
      }
    }
  /* port edges: the eliminated half-face voltage couples the wall cell to
   * itself only */
  for (int i = c->ip; c->ip > 0 && i < nr; ++i) {
    const double m = 2.0 * OG_PI * c->rh[i];
    add_entry(c, HC(i, 0), HC(i, 0), 0.5 * m * m * c->pg[i]);
  }
  return chol_factor(c);
}

/* Electrostatic model (Sec. 2.2, Eq. (8)): the mapped Poisson operator on
 * the free nodes (i, j), 0 <= i < nr, 0 < j < nz, in finite-integration
 * form: (L phi)_n = sum over the edges e at node n of w_e (phi_n - phi_m),
 * with w_e = eps A*_e / l_e, so that L phi is the Gauss charge of the edge
 * voltages u = phi(start) - phi(end).  Plates, side wall and corners are
 * Dirichlet nodes. */
#define PN(i, j) ((int64_t)(i) * (nz - 1) + (j) - 1)

static int factorize_es(og_ctx* c) {
  const int nr = c->g.nr, nz = c->g.nz, b = c->band;
  const int64_t N = c->nunk;
  memset(c->chol, 0, sizeof(double) * (size_t)N * (size_t)(b + 1));
  /* r-edges (i, j) -> (i+1, j) of the free rows j */
  for (int i = 0; i < nr; ++i)
    for (int j = 1; j < nz; ++j) {
      const double w = c->wr[i];
      add_entry(c, PN(i, j), PN(i, j), w);
      if (i + 1 < nr) {
        add_entry(c, PN(i + 1, j), PN(i + 1, j), w);
        add_entry(c, PN(i, j), PN(i + 1, j), -w);
      }
    }
  /* z-edges (i, j) -> (i, j+1) */
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nz; ++j) {
      const double w = c->wz[i];
      const int lo_free = j >= 1, hi_free = j + 1 <= nz - 1;
      if (lo_free) add_entry(c, PN(i, j), PN(i, j), w);
      if (hi_free) add_entry(c, PN(i, j + 1), PN(i, j + 1), w);
      if (lo_free && hi_free) add_entry(c, PN(i, j), PN(i, j + 1), -w);
    }
  return chol_factor(c);
}

static int chol_factor(og_ctx* c) {
  const int b = c->band;
  const int64_t N = c->nunk;
  /* In-place Cholesky (row-oriented), L stored in the band. */
  for (int64_t k = 0; k < N; ++k) {
    const int64_t m0 = k - b > 0 ? k - b : 0;
    for (int64_t m = m0; m < k; ++m) {
      double s = LB(k, k - m);
      const int64_t p0 = (m - b > m0) ? m - b : m0;
      for (int64_t p = p0; p < m; ++p) s -= LB(k, k - p) * LB(m, m - p);
      LB(k, k - m) = s / LB(m, 0);
    }
    double s = LB(k, 0);
    for (int64_t p = m0; p < k; ++p) s -= LB(k, k - p) * LB(k, k - p);
    if (!(s > 0.0)) return -1;
    LB(k, 0) = sqrt(s);
  }
  return 0;
}

static void chol_solve(og_ctx* c, const double* rhs, double* x) {
  const int b = c->band;
  const int64_t N = c->nunk;
  for (int64_t k = 0; k < N; ++k) {
    double s = rhs[k];
    const int64_t p0 = k - b > 0 ? k - b : 0;
    for (int64_t p = p0; p < k; ++p) s -= LB(k, k - p) * x[p];
    x[k] = s / LB(k, 0);
  }
  for (int64_t k = N - 1; k >= 0; --k) {
    double s = x[k];
    const int64_t m1 = k + b < N - 1 ? k + b : N - 1;
    for (int64_t m = k + 1; m <= m1; ++m) s -= LB(m, m - k) * x[m];
    x[k] = s / LB(k, 0);
  }
}

/* ------------------------------------------------------------------------ */
/* Setup                                                                     */
/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* TEM port (Sec. 2.1, Eqs. (5), (7))                                        */
/* ------------------------------------------------------------------------ */
/* The drive enters through a coaxial line, filled with a dielectric of
 * permittivity eps_l = port_eps * eps, that meets the bottom wall over
 * r_p = r(ip) <= r <= R.  The powered electrode is the wall r <= r_p.  Each
 * port edge (i, 0), ip <= i < nr, is a free edge whose dual face is the half
 * cell above the wall (capacitance w_b = wr/2, the half face og_gauss
 * already uses), closed on the wall by the line's field H_b.  Ampere's law
 * on that half face reads
 *   w_b (u^{n+1} - u^n) / dt = -M (h^{n+1/2}(i,0) - H_b^{n+1/2}) - I_r(i,0),
 * with M = 2 pi r_{i+1/2}.  Eq. (5) is the Mur condition for the wave
 * leaving through the line; with the line's own Ampere law
 * (d_z H = -eps_l d_t E_r) it becomes d_t (E_r + eta H_b) = d_t (2 E_r^+),
 * eta = sqrt(mu / eps_l), where E_r^+ is the incoming wave.  Eq. (7) gives
 * that wave from the electrode potential: half of phi, with the TEM radial
 * profile 1/r, so that on edge i it carries kappa_i phi / 2 with
 * kappa_i = ln(r_{i+1} / r_i) / ln(R / r_p) (the kappa_i add up to one).
 * Integrated over the edge and centred in time:
 *   (u^{n+1} - u^n) + eta l_i (H_b^{n+1} - H_b^n) = kappa_i (phi^{n+1} - phi^n).
 * Eliminating H_b^{n+1/2} between the two:
 *   u^{n+1} - u^n = g_i (-M h^{n+1/2} + M H_b^n + a_i dphi - I_r(i,0)),
 *   g_i = 1 / (w_b / dt + M / (2 eta l_i)),  a_i = M kappa_i / (2 eta l_i),
 * so the cell (i, 0) of the H_theta system gains M^2 g_i / 2 on its
 * diagonal and the rest joins the right-hand side.  The line delivers
 * dt M H_b^{n+1/2} u^{n+1/2} per edge and step, and the discrete energy
 * balance holds with it exactly.  The condition constrains only changes:
 * a static voltage across the mouth (E_r with H_b = 0) is allowed, as in
 * the paper's differential form, so a dc self-bias is not drained.
 *
 * The electrostatic model takes the port as a Dirichlet wall with the
 * static coaxial potential: 1 on the electrode's nodes, ln(R/r)/ln(R/r_p)
 * on the mouth's (Sec. 2.2), times the electrode potential. */
static void port_tables(og_ctx* c) {
  const og_grid* g = &c->g;
  const int nr = g->nr, ip = g->port_i;
  c->ip = ip;
  /* the electrostatic wall profile of the gap model: the whole bottom wall
   * but its corner node with the side wall is powered */
  for (int i = 0; i <= nr; ++i) c->pprof[i] = (i < nr) ? 1.0 : 0.0;
  if (ip == 0) return;
  c->eta_p = sqrt(g->mu / (g->eps * g->port_eps));
  const double lnr = log(g->R / c->rn[ip]);
  for (int i = ip; i < nr; ++i) {
    const double M = 2.0 * OG_PI * c->rh[i];
    c->pk[i] = log(c->rn[i + 1] / c->rn[i]) / lnr;
    c->pg[i] = 1.0 / (0.5 * c->wr[i] / g->dt + M / (2.0 * c->eta_p * c->ell[i]));
  }
  for (int i = 0; i <= nr; ++i) c->pprof[i] = (i <= ip) ? 1.0 : log(g->R / c->rn[i]) / lnr;
  c->pprof[nr] = 0.0;
}

int og_create(const og_grid* g, og_ctx** out) {
  if (!g || !out || g->nr < 1 || g->nz < 1 || !(g->R > 0) || !(g->L > 0) ||
      !(g->dt > 0) || !(g->eps > 0) || !(g->mu > 0) || g->xi_a < 0 || g->xi_a > g->nr ||
      !(g->cap >= 0.0) ||
      (g->model != OG_EM && g->model != OG_ES) || (g->model == OG_ES && g->nz < 2) ||
      g->port_i < 0 || (g->port_i > 0 && (g->port_i >= g->nr || !(g->port_eps > 0.0))))
    return -1;
  og_ctx* c = (og_ctx*)calloc(1, sizeof(og_ctx));
  if (!c) return -2;
  c->g = *g;
  if (c->g.sub_tol <= 0) c->g.sub_tol = 1e-14;
  const int nr = g->nr, nz = g->nz;
  c->s = g->R / (nr + g->xi_a);
  c->dz = g->L / nz;
  c->rn = (double*)calloc(nr + 1, sizeof(double));
  c->rh = (double*)calloc(nr, sizeof(double));
  c->ell = (double*)calloc(nr, sizeof(double));
  c->area = (double*)calloc(nr, sizeof(double));
  c->azs = (double*)calloc(nr, sizeof(double));
  c->wr = (double*)calloc(nr, sizeof(double));
  c->wz = (double*)calloc(nr, sizeof(double));
  c->ncell = (int64_t)nr * nz;
  c->nunk = g->model == OG_ES ? (int64_t)nr * (nz - 1) : c->ncell;
  c->band = g->model == OG_ES ? nz - 1 : nz;
  c->chol = g->push_only ? (double*)malloc(sizeof(double))
                         : (double*)malloc(sizeof(double) * (size_t)c->ncell * (size_t)(nz + 1));
  c->rhs = (double*)malloc(sizeof(double) * (size_t)c->ncell);
  c->x = (double*)malloc(sizeof(double) * (size_t)c->ncell);
  c->tr = (double*)malloc(sizeof(double) * (size_t)nr * (nz + 1));
  c->tz = (double*)malloc(sizeof(double) * (size_t)(nr + 1) * nz);
  c->pk = (double*)calloc(nr, sizeof(double));
  c->pg = (double*)calloc(nr, sizeof(double));
  c->pprof = (double*)calloc(nr + 1, sizeof(double));
  c->hb0 = (double*)calloc(nr, sizeof(double));
  c->hb1 = (double*)calloc(nr, sizeof(double));
  if (!c->rn || !c->rh || !c->ell || !c->area || !c->azs || !c->wr || !c->wz ||
      !c->chol || !c->rhs || !c->x || !c->tr || !c->tz || !c->pk || !c->pg || !c->pprof ||
      !c->hb0 || !c->hb1) {
    og_destroy(c);
    return -2;
  }
  for (int i = 0; i <= nr; ++i) c->rn[i] = og_r_of_xi(c, (double)i);
  c->rn[nr] = g->R;
  for (int i = 0; i < nr; ++i) {
    c->rh[i] = og_r_of_xi(c, i + 0.5);
    c->ell[i] = c->rn[i + 1] - c->rn[i];
    c->area[i] = c->ell[i] * c->dz;
    const double rm = (i > 0) ? c->rh[i - 1] : 0.0;
    c->azs[i] = OG_PI * (c->rh[i] * c->rh[i] - rm * rm);
    c->wr[i] = g->eps * 2.0 * OG_PI * c->rh[i] * c->dz / c->ell[i];
    c->wz[i] = g->eps * c->azs[i] / c->dz;
  }
  port_tables(c);
  if (!g->push_only && (g->model == OG_ES ? factorize_es(c) : factorize(c)) != 0) {
    og_destroy(c);
    return -3;
  }
  *out = c;
  return 0;
}

void og_destroy(og_ctx* c) {
  if (!c) return;
  free(c->rn); free(c->rh); free(c->ell); free(c->area); free(c->azs);
  free(c->wr); free(c->wz); free(c->chol); free(c->rhs); free(c->x);
  free(c->tr); free(c->tz);
  free(c->pk); free(c->pg); free(c->pprof); free(c->hb0); free(c->hb1);
  free(c);
}

void og_set_port_h(og_ctx* c, const double* hb) {
  for (int i = c->ip; c->ip > 0 && i < c->g.nr; ++i) c->hb0[i] = hb[i];
}

void og_get_port_h(const og_ctx* c, double* hb) {
  for (int i = c->ip; c->ip > 0 && i < c->g.nr; ++i) hb[i] = c->hb1[i];
}

void og_port_tables(const og_ctx* c, double* kappa, double* prof) {
  if (c->ip == 0) return;
  for (int i = 0; i < c->g.nr; ++i) if (kappa) kappa[i] = c->pk[i];
  for (int i = 0; i <= c->g.nr; ++i) if (prof) prof[i] = c->pprof[i];
}

void og_tables(const og_ctx* c, double* rn, double* rh, double* area_c,
               double* wr, double* wz, double* vol_c) {
  const int nr = c->g.nr;
  for (int i = 0; i <= nr; ++i) if (rn) rn[i] = c->rn[i];
  for (int i = 0; i < nr; ++i) {
    if (rh) rh[i] = c->rh[i];
    if (area_c) area_c[i] = c->area[i];
    if (wr) wr[i] = c->wr[i];
    if (wz) wz[i] = c->wz[i];
    if (vol_c) vol_c[i] = 2.0 * OG_PI * c->rh[i] * c->area[i];
  }
}

/* ------------------------------------------------------------------------ */
/* Field solve: Crank-Nicolson form of Eq. (2) with H_theta the unknown      */
/* ------------------------------------------------------------------------ */
static void set_boundary(const og_ctx* c, double* ur, double* uz, double vd) {
  const int nr = c->g.nr, nz = c->g.nz;
  for (int i = 0; i < nr; ++i) {
    if (c->ip == 0 || i < c->ip) ur[UR(i, 0)] = 0.0; /* port edges are unknowns */
    ur[UR(i, nz)] = 0.0;
  }
  for (int j = 0; j < nz; ++j) uz[UZ(nr, j)] = 0.0;
  if (c->ip == 0) ur[UR(nr - 1, 0)] = vd; /* drive gap between powered plate and wall */
}

/* Electrostatic update (Sec. 2.2, Eq. (8)).  The deposit conserves charge,
 * so the node charge after the step is Q^n - dt div I, and Poisson's
 * equation for phi^{n+1} is the same as L (phi^{n+1} - phi^n) = -dt div I
 * with the plate potential's change on the powered plate's nodes (the
 * bottom nodes i < nr) and zero on the grounded ones.  Then
 * u^{n+1} = u^n + (dphi(start) - dphi(end)) on every edge, and h = 0. */
static void field_solve_es(og_ctx* c, const double* ur0, const double* uz0,
                           const double* Ir, const double* Iz, double t,
                           double* ur1, double* uz1, double* h1) {
  const int nr = c->g.nr, nz = c->g.nz;
  const double dt = c->g.dt;
  const double vnow = c->gap_set ? c->gap_now : og_drive(c, t);
  const double vnext = c->gap_set ? c->gap_next : og_drive(c, t + dt);
  const double dv = vnext - vnow;
  double* b = c->rhs;
  for (int i = 0; i < nr; ++i)
    for (int j = 1; j < nz; ++j) {
      double div = Ir[UR(i, j)] + Iz[UZ(i, j)] - Iz[UZ(i, j - 1)];
      if (i > 0) div -= Ir[UR(i - 1, j)];
      double v = -dt * div;
      if (j == 1) v += c->wz[i] * dv * c->pprof[i]; /* the powered wall below */
      b[PN(i, j)] = v;
    }
  chol_solve(c, b, c->x);
  /* dphi on every node, Dirichlet values included */
  const double* pw = c->pprof;
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j <= nz; ++j) {
      const double pa = (j == 0) ? dv * pw[i] : (j == nz ? 0.0 : c->x[PN(i, j)]);
      const double pb = (i + 1 == nr) ? 0.0
                                      : ((j == 0) ? dv * pw[i + 1] : (j == nz ? 0.0 : c->x[PN(i + 1, j)]));
      ur1[UR(i, j)] = ur0[UR(i, j)] + (pa - pb);
    }
  for (int i = 0; i <= nr; ++i)
    for (int j = 0; j < nz; ++j) {
      if (i == nr) { uz1[UZ(i, j)] = 0.0; continue; }
      const double pa = (j == 0) ? dv * pw[i] : c->x[PN(i, j)];
      const double pb = (j + 1 == nz) ? 0.0 : c->x[PN(i, j + 1)];
      uz1[UZ(i, j)] = uz0[UZ(i, j)] + (pa - pb);
    }
  set_boundary(c, ur1, uz1, vnext);
  for (int64_t k = 0; k < c->ncell; ++k) h1[k] = 0.0;
}

int og_field_solve(og_ctx* c, const double* ur0, const double* uz0, const double* h0,
                   const double* Ir, const double* Iz, double t,
                   double* ur1, double* uz1, double* h1) {
  if (c->g.push_only) return -5;
  if (c->g.model == OG_ES) {
    field_solve_es(c, ur0, uz0, Ir, Iz, t, ur1, uz1, h1);
    return 0;
  }
  const int nr = c->g.nr, nz = c->g.nz;
  const double dt = c->g.dt, mu = c->g.mu;
  const double vnow = c->gap_set ? c->gap_now : og_drive(c, t);
  const double vnext = c->gap_set ? c->gap_next : og_drive(c, t + dt);
  const double vh = 0.5 * (vnow + vnext);
  double* tr = c->tr;
  double* tz = c->tz;
  /* u0 - D^-1 I on interior edges, the half-step value on boundary edges */
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j <= nz; ++j)
      tr[UR(i, j)] = is_int_r_edge(c, j) ? ur0[UR(i, j)] - dt * Ir[UR(i, j)] / (2.0 * c->wr[i]) : 0.0;
  for (int i = 0; i <= nr; ++i)
    for (int j = 0; j < nz; ++j)
      tz[UZ(i, j)] = (i < nr) ? uz0[UZ(i, j)] - dt * Iz[UZ(i, j)] / (2.0 * c->wz[i]) : 0.0;
  const double dphi = vnext - vnow;
  if (c->ip == 0) {
    tr[UR(nr - 1, 0)] = vh;
  } else {
    /* port edges: u^n plus the h-free part of their half-step change */
    for (int i = c->ip; i < nr; ++i) {
      const double M = 2.0 * OG_PI * c->rh[i];
      const double a = M * c->pk[i] / (2.0 * c->eta_p * c->ell[i]);
      tr[UR(i, 0)] = ur0[UR(i, 0)] +
                     0.5 * c->pg[i] * (M * c->hb0[i] + a * dphi - Ir[UR(i, 0)]);
    }
  }
  og_curl_e(c, tr, tz, c->rhs);
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nz; ++j) {
      const double m = 2.0 * OG_PI * c->rh[i];
      c->rhs[HC(i, j)] = m * (2.0 * mu * c->area[i] / dt * h0[HC(i, j)] + c->rhs[HC(i, j)]);
    }
  chol_solve(c, c->rhs, c->x); /* x = h^{n+1/2} */
  /* recover u^{n+1/2} = u0 + D^-1 (K h^{1/2} - I), then the n+1 values */
  og_curl_h(c, c->x, tr, tz);
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j <= nz; ++j) {
      if (!is_int_r_edge(c, j)) continue;
      const double uh = ur0[UR(i, j)] + dt * (tr[UR(i, j)] - Ir[UR(i, j)]) / (2.0 * c->wr[i]);
      ur1[UR(i, j)] = 2.0 * uh - ur0[UR(i, j)];
    }
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nz; ++j) {
      const double uh = uz0[UZ(i, j)] + dt * (tz[UZ(i, j)] - Iz[UZ(i, j)]) / (2.0 * c->wz[i]);
      uz1[UZ(i, j)] = 2.0 * uh - uz0[UZ(i, j)];
    }
  for (int i = c->ip; c->ip > 0 && i < nr; ++i) {
    const double M = 2.0 * OG_PI * c->rh[i];
    const double a = M * c->pk[i] / (2.0 * c->eta_p * c->ell[i]);
    const double du = c->pg[i] * (-M * c->x[HC(i, 0)] + M * c->hb0[i] + a * dphi - Ir[UR(i, 0)]);
    ur1[UR(i, 0)] = ur0[UR(i, 0)] + du;
    c->hb1[i] = c->hb0[i] + (c->pk[i] * dphi - du) / (c->eta_p * c->ell[i]);
  }
  set_boundary(c, ur1, uz1, vnext);
  for (int64_t k = 0; k < c->ncell; ++k) h1[k] = 2.0 * c->x[k] - h0[k];
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Energies and norms                                                        */
/* ------------------------------------------------------------------------ */
double og_energy_norm2(const og_ctx* c, const double* ur, const double* uz) {
  const int nr = c->g.nr, nz = c->g.nz;
  double s = 0.0;
  for (int i = 0; i < nr; ++i)
    for (int j = 1; j < nz; ++j) s += c->wr[i] * ur[UR(i, j)] * ur[UR(i, j)];
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nz; ++j) s += c->wz[i] * uz[UZ(i, j)] * uz[UZ(i, j)];
  /* port edges: the half cell above the wall */
  for (int i = c->ip; c->ip > 0 && i < nr; ++i) s += 0.5 * c->wr[i] * ur[UR(i, 0)] * ur[UR(i, 0)];
  return s;
}

double og_energy_e(const og_ctx* c, const double* ur, const double* uz) {
  return 0.5 * og_energy_norm2(c, ur, uz);
}

double og_energy_b(const og_ctx* c, const double* h) {
  const int nr = c->g.nr, nz = c->g.nz;
  double s = 0.0;
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nz; ++j)
      s += 2.0 * OG_PI * c->rh[i] * c->area[i] * h[HC(i, j)] * h[HC(i, j)];
  return 0.5 * c->g.mu * s;
}

double og_kinetic(const og_species* s) {
  double e = 0.0;
  for (int64_t p = 0; p < s->n; ++p)
    e += s->vr[p] * s->vr[p] + s->vt[p] * s->vt[p] + s->vz[p] * s->vz[p];
  return 0.5 * s->m * s->w * e;
}

/* Node charge from logical bilinear weights S_1(xi-i) S_1(eta-j). */
void og_node_charge(const og_ctx* c, const og_species* sp, int32_t nsp, double* q) {
  const int nr = c->g.nr, nz = c->g.nz;
  memset(q, 0, sizeof(double) * (size_t)(nr + 1) * (nz + 1));
  for (int k = 0; k < nsp; ++k) {
    const og_species* s = &sp[k];
    const double qw = s->q * s->w;
    for (int64_t p = 0; p < s->n; ++p) {
      int i = (int)floor(s->xi[p]), j = (int)floor(s->eta[p]);
      if (i > nr - 1) i = nr - 1;
      if (j > nz - 1) j = nz - 1;
      if (i < 0) i = 0;
      if (j < 0) j = 0;
      const double a = s->xi[p] - i, bq = s->eta[p] - j;
      q[(int64_t)i * (nz + 1) + j] += qw * (1 - a) * (1 - bq);
      q[(int64_t)(i + 1) * (nz + 1) + j] += qw * a * (1 - bq);
      q[(int64_t)i * (nz + 1) + j + 1] += qw * (1 - a) * bq;
      q[(int64_t)(i + 1) * (nz + 1) + j + 1] += qw * a * bq;
    }
  }
}

/* Gauss: net outward displacement flux of every node dual cell. */
void og_gauss(const og_ctx* c, const double* ur, const double* uz, double* g) {
  const int nr = c->g.nr, nz = c->g.nz;
  double* fr = (double*)malloc(sizeof(double) * (size_t)nr * (nz + 1));
  double* fz = (double*)malloc(sizeof(double) * (size_t)(nr + 1) * nz);
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j <= nz; ++j) {
      /* dual face of an r-edge is halved on the z walls */
      const double f = (j == 0 || j == nz) ? 0.5 : 1.0;
      fr[UR(i, j)] = f * c->wr[i] * ur[UR(i, j)];
    }
  for (int i = 0; i <= nr; ++i)
    for (int j = 0; j < nz; ++j) fz[UZ(i, j)] = (i < nr) ? c->wz[i] * uz[UZ(i, j)] : 0.0;
  og_div(c, fr, fz, g);
  free(fr);
  free(fz);
}

/* ------------------------------------------------------------------------ */
/* Particle push: Eq. (4), mid-point centring, split at cell crossings       */
/* ------------------------------------------------------------------------ */
typedef struct { double xi, eta, vr, vt, vz; } pst;

typedef struct {
  const og_ctx* c;
  const double *ur, *uz, *hh; /* half-step fields */
  double qm;                  /* q/m              */
} pctx;

/* Cell of a coordinate; on a face, the side the motion goes to. */
static int cell_of(double x, double v, int n) {
  int i = (int)floor(x);
  if ((double)i == x && v < 0.0) i -= 1;
  if (i < 0) i = 0;
  if (i > n - 1) i = n - 1;
  return i;
}

static double clamp01(double a) { return a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a); }

/* Position equation of the mid-point rule in xi: xb = xi + (dtau/2) vb_r / J_r(xb).
 * Solved exactly: linear map part, or the square-root part as a quadratic in
 * sqrt(xb) (positive root), whichever is consistent. */
static double solve_xi_mid(const og_ctx* c, double xi, double vbr, double dtau) {
  const double xa = c->g.xi_a, s = c->s;
  const double xl = xi + 0.5 * dtau * vbr / s;
  if (xl >= xa) return xl;
  const double beta = 0.5 * dtau * vbr / (s * sqrt(xa));
  const double y = 0.5 * (beta + sqrt(beta * beta + 4.0 * xi));
  return y * y;
}

/* Acceleration at the mid-point (xb, eb) of cell (i,j) with mid velocity vb.
 * Returns the theta mid velocity consistent with the angular equation. */
typedef struct { double ar, az, vt_bar; int ok; } accel_t;

static accel_t mid_accel(const pctx* P, int i, int j, double xb, double eb,
                         double vbr, double vbz, double vt0, double dtau) {
  const og_ctx* c = P->c;
  const int nz = c->g.nz;
  accel_t A = {0, 0, 0, 1};
  const double rb = og_r_of_xi(c, xb);
  const double ijr = inv_jr(c, xb);
  const double a = clamp01(xb - i), bq = clamp01(eb - j);
  /* gather: adjoint of the deposit (logical S_0 along, S_1 across) */
  double er = ((1.0 - bq) * P->ur[UR(i, j)] + bq * P->ur[UR(i, j + 1)]) * ijr;
  double ez = ((1.0 - a) * P->uz[UZ(i, j)] + a * P->uz[UZ(i + 1, j)]) / c->dz;
  if (c->g.er_ext != 0.0) er += c->g.er_ext * rb / c->g.R;
  double bth = 0.0;
  if (c->g.self_b && P->hh) bth = c->g.mu * P->hh[HC(i, j)];
  const double bz = c->g.bz_ext;
  /* theta equation: vb_t (1 + dtau vb_r / (2 rb)) = v_t - (dtau/2) qm vb_r B_z */
  double num = vt0 - 0.5 * dtau * P->qm * vbr * bz;
  double vtb;
  if (rb > 0.0) {
    const double den = 1.0 + 0.5 * dtau * vbr / rb;
    if (!(den > 0.0)) { A.ok = 0; return A; }
    vtb = num / den;
    A.ar = P->qm * er + vtb * vtb / rb;
  } else {
    if (num != 0.0) { A.ok = 0; return A; }
    vtb = 0.0;
    A.ar = P->qm * er;
  }
  A.ar += P->qm * (vtb * bz - vbz * bth);
  A.az = P->qm * ez + P->qm * vbr * bth;
  A.vt_bar = vtb;
  if (!isfinite(A.ar) || !isfinite(A.az) || !isfinite(vtb)) A.ok = 0;
  return A;
}

/* Unconstrained mid-point sub-step of length dtau in cell (i,j).
 * Unknowns are the mid velocities; mid positions are solved exactly from them.
 * Returns 1 on convergence with (xb, eb, vb). */
static int solve_free(const pctx* P, int i, int j, const pst* p, double dtau,
                      double* xb, double* eb, double vb[3]) {
  const og_ctx* c = P->c;
  const double tol = c->g.sub_tol;
  double vr = p->vr, vt = p->vt, vz = p->vz;
  for (int it = 0; it < OG_MAX_FP; ++it) {
    const double x = solve_xi_mid(c, p->xi, vr, dtau);
    const double e = p->eta + 0.5 * dtau * vz / c->dz;
    if (!(x >= 0.0) || !isfinite(e)) return 0;
    accel_t A = mid_accel(P, i, j, x, e, vr, vz, p->vt, dtau);
    if (!A.ok) return 0;
    const double nvr = p->vr + 0.5 * dtau * A.ar;
    const double nvz = p->vz + 0.5 * dtau * A.az;
    const double nvt = A.vt_bar;
    const double scale = fabs(nvr) + fabs(nvt) + fabs(nvz);
    const double d = fmax(fabs(nvr - vr), fmax(fabs(nvt - vt), fabs(nvz - vz)));
    vr = nvr; vt = nvt; vz = nvz;
    if (d <= tol * scale) {
      *xb = solve_xi_mid(c, p->xi, vr, dtau);
      *eb = p->eta + 0.5 * dtau * vz / c->dz;
      vb[0] = vr; vb[1] = vt; vb[2] = vz;
      return (*xb >= 0.0) ? 1 : 0;
    }
  }
  return 0;
}

/* Smallest positive root of a/2 t^2 + v t - D = 0 (cancellation-free), or +inf. */
static double smallest_pos_root(double a, double v, double D) {
  const double A = 0.5 * a, B = v, C = -D;
  double best = INFINITY;
  if (A == 0.0) {
    if (B != 0.0) { const double t = -C / B; if (t > 0.0) best = t; }
    return best;
  }
  const double disc = B * B - 4.0 * A * C;
  if (disc < 0.0) return best;
  const double sq = sqrt(disc);
  const double q = -0.5 * (B + (B >= 0.0 ? sq : -sq));
  if (q != 0.0) {
    const double t1 = q / A, t2 = C / q;
    if (t1 > 0.0 && t1 < best) best = t1;
    if (t2 > 0.0 && t2 < best) best = t2;
  } else {
    /* B == 0 and C == 0: double root at 0 */
  }
  return best;
}

/* Constrained sub-step that ends exactly on face f of axis d (0: xi, 1: eta).
 * The crossed coordinate's mid value is (x_d + f)/2; the length dtau solves
 * the position equation as a quadratic in dtau given the mid acceleration.
 * Returns 1 on convergence; *capped = 1 if no root within dmax was found. */
static int solve_cross(const pctx* P, int i, int j, const pst* p, int d, double f,
                       double dmax, double dt0, const double vb0[3],
                       double* dtau_out, double* xb, double* eb, double vb[3], int* capped) {
  const og_ctx* c = P->c;
  const double tol = c->g.sub_tol;
  double vr = vb0[0], vt = vb0[1], vz = vb0[2];
  double dtau = dt0;
  *capped = 0;
  const double xd = (d == 0) ? p->xi : p->eta;
  const double xbar_d = 0.5 * (xd + f);
  const double Jd = (d == 0) ? 1.0 / inv_jr(c, xbar_d) : c->dz;
  const double D = (f == xd) ? 0.0 : (f - xd) * Jd; /* J_r is infinite on the axis */
  if (D == 0.0) {
    /* already on the face: leaving through it now if moving outward */
    const double v0d = (d == 0) ? p->vr : p->vz;
    const int lower = (d == 0) ? (f == (double)i) : (f == (double)j);
    if (lower ? (v0d < 0.0) : (v0d > 0.0)) {
      *dtau_out = 0.0;
      *xb = p->xi; *eb = p->eta;
      vb[0] = p->vr; vb[1] = p->vt; vb[2] = p->vz;
      return 1;
    }
  }
  for (int it = 0; it < OG_MAX_FP; ++it) {
    double x, e;
    if (d == 0) {
      x = xbar_d;
      e = p->eta + 0.5 * dtau * vz / c->dz;
    } else {
      e = xbar_d;
      x = solve_xi_mid(c, p->xi, vr, dtau);
    }
    if (!(x >= 0.0) || !isfinite(e)) return 0;
    accel_t A = mid_accel(P, i, j, x, e, vr, vz, p->vt, dtau);
    if (!A.ok) return 0;
    const double ad = (d == 0) ? A.ar : A.az;
    const double v0d = (d == 0) ? p->vr : p->vz;
    double nd = smallest_pos_root(ad, v0d, D);
    int cap = 0;
    if (!(nd <= dmax)) { nd = dmax; cap = 1; }
    const double nvr = p->vr + 0.5 * nd * A.ar;
    const double nvz = p->vz + 0.5 * nd * A.az;
    const double nvt = A.vt_bar;
    const double scale = fabs(nvr) + fabs(nvt) + fabs(nvz);
    const double dv = fmax(fabs(nvr - vr), fmax(fabs(nvt - vt), fabs(nvz - vz)));
    const double ddt = fabs(nd - dtau);
    vr = nvr; vt = nvt; vz = nvz; dtau = nd;
    if (dv <= tol * scale && ddt <= tol * dmax) {
      *capped = cap;
      *dtau_out = dtau;
      if (d == 0) {
        *xb = xbar_d;
        *eb = p->eta + 0.5 * dtau * vz / c->dz;
      } else {
        *eb = xbar_d;
        *xb = solve_xi_mid(c, p->xi, vr, dtau);
      }
      vb[0] = vr; vb[1] = vt; vb[2] = vz;
      return 1;
    }
  }
  return 0;
}

/* Charge-conserving deposit of one straight logical sub-step in cell (i,j):
 * Eq. (3) with m = 1 integrated along the sub-step (S_1 across at the
 * sub-step mid-point, S_0 along). */
static void deposit(const og_ctx* c, int i, int j, double x0, double e0, double x1,
                    double e1, double qw_dt, double* Ir, double* Iz) {
  const int nz = c->g.nz;
  const double dx = x1 - x0, de = e1 - e0;
  const double xm = 0.5 * (x0 + x1) - i, em = 0.5 * (e0 + e1) - j;
  Ir[UR(i, j)] += qw_dt * dx * (1.0 - em);
  Ir[UR(i, j + 1)] += qw_dt * dx * em;
  Iz[UZ(i, j)] += qw_dt * de * (1.0 - xm);
  Iz[UZ(i + 1, j)] += qw_dt * de * xm;
}

/* Work q*E.dx of one sub-step, the same sum the deposit gives against u. */
static double substep_work(const og_ctx* c, const pctx* P, int i, int j, double x0,
                           double e0, double x1, double e1, double qw) {
  const int nz = c->g.nz;
  const double dx = x1 - x0, de = e1 - e0;
  const double xm = 0.5 * (x0 + x1) - i, em = 0.5 * (e0 + e1) - j;
  return qw * (dx * ((1.0 - em) * P->ur[UR(i, j)] + em * P->ur[UR(i, j + 1)]) +
               de * ((1.0 - xm) * P->uz[UZ(i, j)] + xm * P->uz[UZ(i + 1, j)]));
}

enum { P_ALIVE = 0, P_ABSORBED = 1, P_ERROR = -1 };

typedef struct {
  int wall;       /* 0 none, 1 bottom (eta=0), 2 top (eta=nz), 3 side (xi=nr) */
  double xi, eta; /* where it hit */
} hit_t;

/* Push one particle over dt.  Deposits into Ir, Iz.  Returns P_* code. */
static int push_one(const pctx* P, pst* p, double qw, double* Ir, double* Iz,
                    og_stats* S, double* work, hit_t* hit) {
  const og_ctx* c = P->c;
  const int nr = c->g.nr, nz = c->g.nz;
  const double dt = c->g.dt;
  const double qw_dt = qw / dt;
  double tau = dt;
  int nsub = 0, ncut = 0; /* ncut: halvings after crossing solves that found no face */
  hit->wall = 0;
  while (tau > 0.0) {
    if (nsub >= OG_MAX_SUB) { if (S) S->n_errors++; return P_ERROR; }
    nsub++;
    const int i = cell_of(p->xi, p->vr, nr);
    const int j = cell_of(p->eta, p->vz, nz);
    double dtry = tau, xb = 0, eb = 0, vb[3];
    for (int k = 0; k < ncut; ++k) dtry *= 0.5;
    int ok = 0, nh = 0;
    for (nh = 0; nh <= OG_MAX_HALVE; ++nh) {
      ok = solve_free(P, i, j, p, dtry, &xb, &eb, vb);
      if (ok) break;
      dtry *= 0.5;
    }
    if (!ok) { if (S) S->n_errors++; return P_ERROR; }
    pst e;
    e.xi = 2.0 * xb - p->xi;
    e.eta = 2.0 * eb - p->eta;
    e.vr = 2.0 * vb[0] - p->vr;
    e.vt = 2.0 * vb[1] - p->vt;
    e.vz = 2.0 * vb[2] - p->vz;
    const int in_x = (e.xi >= i && e.xi <= i + 1);
    const int in_e = (e.eta >= j && e.eta <= j + 1);
    if (in_x && in_e) {
      if (S) { S->n_substeps++; S->n_halvings += nh + ncut; }
      ncut = 0;
      deposit(c, i, j, p->xi, p->eta, e.xi, e.eta, qw_dt, Ir, Iz);
      if (work) *work += substep_work(c, P, i, j, p->xi, p->eta, e.xi, e.eta, qw);
      *p = e;
      tau -= dtry;
      continue;
    }
    /* crossing: candidates are the violated axes */
    double best_t = INFINITY, bx = 0, be = 0, bv[3] = {0, 0, 0};
    int best_d = -1, best_cap = 0;
    double best_f = 0;
    for (int d = 0; d < 2; ++d) {
      double f;
      if (d == 0) {
        if (in_x) continue;
        f = (e.xi < i) ? (double)i : (double)(i + 1);
      } else {
        if (in_e) continue;
        f = (e.eta < j) ? (double)j : (double)(j + 1);
      }
      const double xd = (d == 0) ? p->xi : p->eta;
      const double xe = (d == 0) ? e.xi : e.eta;
      const double t0 = dtry * (f - xd) / (xe - xd);
      double tt, cx, ce, cv[3];
      int cap = 0;
      if (!solve_cross(P, i, j, p, d, f, dtry, t0, vb, &tt, &cx, &ce, cv, &cap)) continue;
      /* tie within 1e-15 dt: xi first (d=0 seen first, keep it) */
      if (best_d < 0 || tt < best_t - 1e-15 * dt) {
        best_t = tt; best_d = d; best_f = f; bx = cx; be = ce;
        bv[0] = cv[0]; bv[1] = cv[1]; bv[2] = cv[2]; best_cap = cap;
      }
    }
    if (best_d < 0) {
      /* the free orbit leaves the cell but no face can be reached
       * consistently (an orbit that turns at the face: the crossing solve
       * jumps between a root and none): take the sub-step again at half
       * the length (a new pass of the loop, counted like a sub-step) */
      if (ncut >= OG_MAX_HALVE) { if (S) S->n_errors++; return P_ERROR; }
      ncut++;
      continue;
    }
    if (S) { S->n_substeps++; S->n_halvings += nh + ncut; }
    ncut = 0;
    if (S) { S->n_crossings++; if (best_cap) S->n_capped++; }
    pst q;
    q.vr = 2.0 * bv[0] - p->vr;
    q.vt = 2.0 * bv[1] - p->vt;
    q.vz = 2.0 * bv[2] - p->vz;
    if (best_d == 0) {
      q.xi = best_f;
      q.eta = 2.0 * be - p->eta;
      if (q.eta < j) q.eta = j;          /* round-off clamp into the cell */
      if (q.eta > j + 1) q.eta = j + 1;
    } else {
      q.eta = best_f;
      q.xi = 2.0 * bx - p->xi;
      if (q.xi < i) q.xi = i;
      if (q.xi > i + 1) q.xi = i + 1;
    }
    deposit(c, i, j, p->xi, p->eta, q.xi, q.eta, qw_dt, Ir, Iz);
    if (work) *work += substep_work(c, P, i, j, p->xi, p->eta, q.xi, q.eta, qw);
    *p = q;
    tau -= best_t;
    if (best_d == 0 && best_f == (double)nr) { hit->wall = 3; hit->xi = p->xi; hit->eta = p->eta; return P_ABSORBED; }
    if (best_d == 1 && best_f == 0.0) { hit->wall = 1; hit->xi = p->xi; hit->eta = p->eta; return P_ABSORBED; }
    if (best_d == 1 && best_f == (double)nz) { hit->wall = 2; hit->xi = p->xi; hit->eta = p->eta; return P_ABSORBED; }
    if (best_d == 0 && best_f == 0.0) p->vr = -p->vr; /* axis: mirror */
  }
  return P_ALIVE;
}

static void tally_wall(const og_ctx* c, og_state* st, const hit_t* h, double qw) {
  const int nr = c->g.nr, nz = c->g.nz;
  if (!st) return;
  if (h->wall == 1 || h->wall == 2) {
    int i = (int)floor(h->xi);
    if (i > nr - 1) i = nr - 1;
    if (i < 0) i = 0;
    const double a = h->xi - i;
    double* w = (h->wall == 1) ? st->wall_bot : st->wall_top;
    if (w) { w[i] += qw * (1 - a); w[i + 1] += qw * a; }
  } else if (h->wall == 3) {
    int j = (int)floor(h->eta);
    if (j > nz - 1) j = nz - 1;
    if (j < 0) j = 0;
    const double b = h->eta - j;
    if (st->wall_side) { st->wall_side[j] += qw * (1 - b); st->wall_side[j + 1] += qw * b; }
  }
}

int og_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

#ifdef _OPENMP
/* The push pass with the particle loop split over the threads (timing
 * build): each thread pushes a contiguous range into its own currents and
 * counters, which are then summed in thread order; a commit then absorbs and
 * compacts in particle order, as the serial loop does. */
static int push_deposit_threads(og_ctx* c, og_species* s, const pctx* P, int commit,
                                double* Ir, double* Iz, og_state* st, og_stats* S) {
  const int nt = omp_get_max_threads();
  const int64_t nur = (int64_t)c->g.nr * (c->g.nz + 1), nuz = (int64_t)(c->g.nr + 1) * c->g.nz;
  const double qw = s->q * s->w;
  double* cur = (double*)calloc((size_t)nt * (size_t)(nur + nuz), sizeof(double));
  og_stats* ts = (og_stats*)calloc((size_t)nt, sizeof(og_stats));
  double* twork = (double*)calloc((size_t)nt, sizeof(double));
  int* terr = (int*)calloc((size_t)nt, sizeof(int));
  pst* res = commit ? (pst*)malloc(sizeof(pst) * (size_t)(s->n > 0 ? s->n : 1)) : NULL;
  int* rcs = commit ? (int*)malloc(sizeof(int) * (size_t)(s->n > 0 ? s->n : 1)) : NULL;
  hit_t* hits = commit ? (hit_t*)malloc(sizeof(hit_t) * (size_t)(s->n > 0 ? s->n : 1)) : NULL;
#pragma omp parallel
  {
    const int t = omp_get_thread_num();
    double* mr = cur + (int64_t)t * (nur + nuz);
    double* mz = mr + nur;
#pragma omp for schedule(static)
    for (int64_t k = 0; k < s->n; ++k) {
      pst p = {s->xi[k], s->eta[k], s->vr[k], s->vt[k], s->vz[k]};
      hit_t hit;
      const int rc = push_one(P, &p, qw, mr, mz, S ? &ts[t] : NULL, &twork[t], &hit);
      if (rc == P_ERROR) terr[t]++;
      if (commit) { res[k] = p; rcs[k] = rc; hits[k] = hit; }
    }
  }
  int nerr = 0;
  double work = 0.0;
  for (int t = 0; t < nt; ++t) {
    const double* mr = cur + (int64_t)t * (nur + nuz);
    for (int64_t e = 0; e < nur; ++e) Ir[e] += mr[e];
    for (int64_t e = 0; e < nuz; ++e) Iz[e] += mr[nur + e];
    nerr += terr[t];
    work += twork[t];
    if (S) {
      S->n_substeps += ts[t].n_substeps;
      S->n_crossings += ts[t].n_crossings;
      S->n_halvings += ts[t].n_halvings;
      S->n_errors += ts[t].n_errors;
      S->n_capped += ts[t].n_capped;
    }
  }
  if (commit) {
    int64_t out = 0;
    for (int64_t k = 0; k < s->n; ++k) {
      const pst p = res[k];
      if (rcs[k] == P_ABSORBED) {
        tally_wall(c, st, &hits[k], qw);
        if (S) S->w_absorbed += 0.5 * s->m * s->w * (p.vr * p.vr + p.vt * p.vt + p.vz * p.vz);
        continue;
      }
      s->xi[out] = p.xi; s->eta[out] = p.eta;
      s->vr[out] = p.vr; s->vt[out] = p.vt; s->vz[out] = p.vz;
      s->uid[out] = s->uid[k];
      out++;
    }
    if (S) S->w_particles += work;
    s->n = out;
  }
  free(cur); free(ts); free(twork); free(terr); free(res); free(rcs); free(hits);
  return -nerr;
}
#endif

int og_push_deposit(og_ctx* c, og_species* s, const double* ur_h, const double* uz_h,
                    const double* h_h, int commit, double* Ir, double* Iz,
                    og_state* st, og_stats* S) {
  if (!s->mobile) return 0;
#ifdef _OPENMP
  if (omp_get_max_threads() > 1) {
    pctx Pt = {c, ur_h, uz_h, h_h, s->q / s->m};
    return push_deposit_threads(c, s, &Pt, commit, Ir, Iz, st, S);
  }
#endif
  pctx P = {c, ur_h, uz_h, h_h, s->q / s->m};
  const double qw = s->q * s->w;
  int nerr = 0;
  int64_t out = 0;
  double work = 0.0;
  for (int64_t k = 0; k < s->n; ++k) {
    pst p = {s->xi[k], s->eta[k], s->vr[k], s->vt[k], s->vz[k]};
    hit_t hit;
    const int rc = push_one(&P, &p, qw, Ir, Iz, S, &work, &hit);
    if (rc == P_ERROR) nerr++;
    if (!commit) continue;
    if (rc == P_ABSORBED) {
      tally_wall(c, st, &hit, qw);
      if (S) {
        S->w_absorbed += 0.5 * s->m * s->w * (p.vr * p.vr + p.vt * p.vt + p.vz * p.vz);
      }
      continue;
    }
    s->xi[out] = p.xi; s->eta[out] = p.eta;
    s->vr[out] = p.vr; s->vt[out] = p.vt; s->vz[out] = p.vz;
    s->uid[out] = s->uid[k];
    out++;
  }
  if (commit) {
    if (S) S->w_particles += work;
    s->n = out;
  }
  return -nerr;
}

/* ------------------------------------------------------------------------ */
/* Counter-based RNG: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11)      */
/* ------------------------------------------------------------------------ */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  const __uint128_t p = (__uint128_t)a * (__uint128_t)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void og_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, x0, &hi0, &lo0);
    mulhilo64(M1, x2, &hi1, &lo1);
    const uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Identifier of a particle born at `step` from `parent`: the SplitMix64
 * finaliser (Steele, Lea, Flood 2014) of a Weyl-shifted parent id, with the
 * top bit set so that it never equals a loaded (0-based) identifier. */
uint64_t og_child_uid(uint64_t parent, int64_t step) {
  uint64_t z = parent + 0x9E3779B97F4A7C15ULL * (uint64_t)(step + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z = z ^ (z >> 31);
  return z | 0x8000000000000000ULL;
}

static double u01(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

typedef struct { double u[12]; } draws_t;

/* Uniform draws for particle uid of species sid at step: block b gives
 * draws 4b..4b+3 from counter (uid, step, b, 0), key (seed, sid). */
static void get_draws(uint64_t seed, int sid, uint64_t uid, int64_t step, int nblk, draws_t* D) {
  const uint64_t key[2] = {seed, (uint64_t)sid};
  for (int b = 0; b < nblk; ++b) {
    const uint64_t ctr[4] = {uid, (uint64_t)step, (uint64_t)b, 0};
    uint64_t o[4];
    og_philox4x64_10(ctr, key, o);
    for (int k = 0; k < 4; ++k) D->u[4 * b + k] = u01(o[k]);
  }
}

/* ------------------------------------------------------------------------ */
/* Synthetic analytic argon cross-sections (elastic, one excitation at       */
/* 11.5 eV, ionisation at 15.76 eV; Ar+ charge exchange), in m^2.            */
/* ------------------------------------------------------------------------ */
#define OG_EX_TH 11.5
#define OG_IZ_TH 15.76
#define OG_SIG_EL 1.0e-19
#define OG_SIG_EX 1.0e-20
#define OG_SIG_IZ 8.0e-20
#define OG_SIG_CX 5.0e-19

void og_cross_sections(double e, double* s_el, double* s_ex, double* s_iz) {
  *s_el = OG_SIG_EL;
  *s_ex = (e > OG_EX_TH) ? OG_SIG_EX * (1.0 - OG_EX_TH / e) : 0.0;
  if (e > OG_IZ_TH) {
    const double x = e / OG_IZ_TH;
    *s_iz = OG_SIG_IZ * log(x) / x;
  } else {
    *s_iz = 0.0;
  }
}

/* Null-collision bound: nu_max = 1.05 * n_g * max over a 2e5-point energy
 * grid up to eps_max of sigma_tot(eps) v(eps) (electrons), or n_g sigma_cx g_max
 * with g_max the relative speed of an ion of eps_max (ions). */
double og_nu_max(const og_mcc* m, int32_t role, double mp) {
  if (role == 1) {
    double best = 0.0;
    const int K = 200000;
    for (int k = 1; k <= K; ++k) {
      const double e = m->eps_max_ev * (double)k / (double)K;
      double a, b, cc;
      og_cross_sections(e, &a, &b, &cc);
      const double v = sqrt(2.0 * e * OG_QE / mp);
      const double f = (a + b + cc) * v;
      if (f > best) best = f;
    }
    return 1.05 * m->n_gas * best;
  }
  if (role == 2) {
    const double g = sqrt(2.0 * m->eps_max_ev * OG_QE / mp);
    return 1.05 * m->n_gas * OG_SIG_CX * g;
  }
  return 0.0;
}

static void iso_dir(double u1, double u2, double d[3]) {
  const double ct = 1.0 - 2.0 * u1;
  const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
  const double ph = 2.0 * OG_PI * u2;
  d[0] = st * cos(ph);
  d[1] = st * sin(ph);
  d[2] = ct;
}

static int append(og_species* s, double xi, double eta, double vr, double vt, double vz, uint64_t uid) {
  if (s->n >= s->cap) return -1;
  const int64_t k = s->n++;
  s->xi[k] = xi; s->eta[k] = eta; s->vr[k] = vr; s->vt[k] = vt; s->vz[k] = vz; s->uid[k] = uid;
  return 0;
}

int og_collide(og_ctx* c, og_species* sp, int32_t nsp, const og_mcc* m, int64_t step, og_stats* S) {
  if (!m || !m->enabled) return 0;
  const double dt = c->g.dt;
  int rc = 0;
  int64_t nstart[8];
  for (int sid = 0; sid < nsp && sid < 8; ++sid) nstart[sid] = sp[sid].n;
  for (int sid = 0; sid < nsp && sid < 8; ++sid) {
    og_species* s = &sp[sid];
    const int role = (sid == m->electron_sid) ? 1 : (sid == m->ion_sid ? 2 : 0);
    if (!role || !s->mobile) continue;
    const double numax = og_nu_max(m, role, s->m);
    const double pnull = 1.0 - exp(-numax * dt);
    const int64_t n0 = nstart[sid]; /* particles born this step do not collide */
    for (int64_t k = 0; k < n0; ++k) {
      draws_t D;
      get_draws(m->seed, sid, s->uid[k], step, 1, &D);
      if (!(D.u[0] < pnull)) continue;
      const double vr = s->vr[k], vt = s->vt[k], vz = s->vz[k];
      const double v2 = vr * vr + vt * vt + vz * vz;
      const double v = sqrt(v2);
      if (role == 1) {
        const double e = 0.5 * s->m * v2 / OG_QE;
        if (e > m->eps_max_ev) { if (S) S->n_over_range++; }
        double sel, sex, siz;
        og_cross_sections(e, &sel, &sex, &siz);
        const double nel = m->n_gas * sel * v, nex = m->n_gas * sex * v, niz = m->n_gas * siz * v;
        const double x = D.u[1] * numax;
        double d[3];
        iso_dir(D.u[2], D.u[3], d);
        const double ke0 = 0.5 * s->m * s->w * v2;
        if (x < nel) {
          const double cosx = (v > 0.0) ? (d[0] * vr + d[1] * vt + d[2] * vz) / v : 1.0;
          const double e1 = e * (1.0 - 2.0 * s->m / m->m_gas * (1.0 - cosx));
          const double v1 = sqrt(2.0 * e1 * OG_QE / s->m);
          s->vr[k] = v1 * d[0]; s->vt[k] = v1 * d[1]; s->vz[k] = v1 * d[2];
          if (S) { S->w_coll += ke0 - 0.5 * s->m * s->w * v1 * v1; S->n_coll[sid]++; }
        } else if (x < nel + nex) {
          const double e1 = e - OG_EX_TH;
          const double v1 = sqrt(2.0 * e1 * OG_QE / s->m);
          s->vr[k] = v1 * d[0]; s->vt[k] = v1 * d[1]; s->vz[k] = v1 * d[2];
          if (S) { S->w_coll += ke0 - 0.5 * s->m * s->w * v1 * v1; S->n_coll[sid]++; }
        } else if (x < nel + nex + niz) {
          draws_t E;
          get_draws(m->seed, sid, s->uid[k], step, 3, &E);
          const double er = e - OG_IZ_TH;
          const double e1 = E.u[4] * er, e2 = er - e1;
          const double v1 = sqrt(2.0 * e1 * OG_QE / s->m), v2n = sqrt(2.0 * e2 * OG_QE / s->m);
          double d2[3];
          iso_dir(E.u[5], E.u[6], d2);
          /* ion from the gas Maxwellian (Box-Muller) */
          og_species* ion = &sp[m->ion_sid];
          const double sg = sqrt(OG_KB * m->T_gas / ion->m);
          const double ra = sqrt(-2.0 * log(1.0 - E.u[7])), rb = sqrt(-2.0 * log(1.0 - E.u[9]));
          const double ivr = sg * ra * cos(2.0 * OG_PI * E.u[8]);
          const double ivt = sg * ra * sin(2.0 * OG_PI * E.u[8]);
          const double ivz = sg * rb * cos(2.0 * OG_PI * E.u[10]);
          const uint64_t nu = og_child_uid(s->uid[k], step);
          s->vr[k] = v1 * d[0]; s->vt[k] = v1 * d[1]; s->vz[k] = v1 * d[2];
          if (append(s, s->xi[k], s->eta[k], v2n * d2[0], v2n * d2[1], v2n * d2[2], nu) != 0 ||
              append(ion, s->xi[k], s->eta[k], ivr, ivt, ivz, nu) != 0) {
            rc = -6;
            continue;
          }
          if (S) {
            S->w_coll += ke0 - 0.5 * s->m * s->w * (v1 * v1 + v2n * v2n) -
                         0.5 * ion->m * ion->w * (ivr * ivr + ivt * ivt + ivz * ivz);
            S->n_coll[sid]++;
            S->n_ionized++;
          }
        }
      } else {
        /* Ar+ - Ar charge exchange: constant sigma, neutral from the gas
         * Maxwellian; accepted with probability n_g sigma g / nu_max. */
        draws_t E;
        get_draws(m->seed, sid, s->uid[k], step, 2, &E);
        const double sg = sqrt(OG_KB * m->T_gas / m->m_gas);
        const double ra = sqrt(-2.0 * log(1.0 - E.u[1])), rb = sqrt(-2.0 * log(1.0 - E.u[3]));
        const double nvr = sg * ra * cos(2.0 * OG_PI * E.u[2]);
        const double nvt = sg * ra * sin(2.0 * OG_PI * E.u[2]);
        const double nvz = sg * rb * cos(2.0 * OG_PI * E.u[4]);
        const double gr = vr - nvr, gt = vt - nvt, gz = vz - nvz;
        const double g = sqrt(gr * gr + gt * gt + gz * gz);
        const double nu = m->n_gas * OG_SIG_CX * g;
        if (nu > numax) { if (S) S->n_over_range++; }
        if (E.u[5] * numax < nu) {
          const double ke0 = 0.5 * s->m * s->w * v2;
          s->vr[k] = nvr; s->vt[k] = nvt; s->vz[k] = nvz;
          if (S) {
            S->w_coll += ke0 - 0.5 * s->m * s->w * (nvr * nvr + nvt * nvt + nvz * nvz);
            S->n_coll[sid]++;
          }
        }
      }
    }
  }
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Jacobian-free Newton-Krylov solve of the same system (Sec. 2.1 names     */
/* JFNK beside Picard).  The unknown is the edge-voltage iterate X = u^{n+1} */
/* and the residual F(X) = X - G(X), where G is one Picard map: push every   */
/* species in the half-step field (u^n + X)/2, deposit, and solve the field  */
/* equations from u^n with that current.  Newton: J d = -F with J = I - G',  */
/* J v taken by the forward difference (G(X + e v) - G(X)) / e, e =         */
/* 1e-6 max(|X|, |F|) / |v| in the energy norm (G carries the rounding of   */
/* the deposit and the 1e-14 inner-solve tolerance, so a difference over a  */
/* relative step of sqrt(eps_mach) is mostly noise beyond the first Krylov  */
/* direction; 1e-6 keeps that noise near 1e-8 of |v| while G is nearly      */
/* linear in u over such a step), and solved by                             */
/* GMRES (Arnoldi with modified Gram-Schmidt in the energy inner product,   */
/* Givens rotations), from d = 0, without restarts.  In tolerance mode the  */
/* step X + l d is taken with l halved (at most 8 times) until |F| falls by */
/* the factor 1 - 1e-4 l (backtracking); with a fixed count, l = 1.         */
/* ------------------------------------------------------------------------ */
#define OG_JF_DIFF 1e-6

typedef struct {
  og_ctx* c;
  og_state* st;
  og_species* sp;
  int32_t nsp;
  double *urh, *uzh, *hh, *Ir, *Iz; /* work: half field and currents */
  int64_t evals;
} jfnk_ctx;

/* energy inner product over the interior edges (the weights of the
 * residual norm); a vector is ur (nr*(nz+1)) followed by uz ((nr+1)*nz) */
static double wdot(const og_ctx* c, const double* a, const double* b) {
  const int nr = c->g.nr, nz = c->g.nz;
  const int64_t nur = (int64_t)nr * (nz + 1);
  double s = 0.0;
  for (int i = 0; i < nr; ++i)
    for (int j = 1; j < nz; ++j) s += c->wr[i] * a[UR(i, j)] * b[UR(i, j)];
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nz; ++j) s += c->wz[i] * a[nur + UZ(i, j)] * b[nur + UZ(i, j)];
  for (int i = c->ip; c->ip > 0 && i < nr; ++i) s += 0.5 * c->wr[i] * a[UR(i, 0)] * b[UR(i, 0)];
  return s;
}

/* G(X): the Picard map; X and the result are [ur | uz], h into gh */
static void picard_map(jfnk_ctx* J, const double* X, double* GX, double* gh) {
  og_ctx* c = J->c;
  const int nr = c->g.nr, nz = c->g.nz;
  const int64_t nur = (int64_t)nr * (nz + 1), nuz = (int64_t)(nr + 1) * nz;
  for (int64_t e = 0; e < nur; ++e) J->urh[e] = 0.5 * (J->st->ur[e] + X[e]);
  for (int64_t e = 0; e < nuz; ++e) J->uzh[e] = 0.5 * (J->st->uz[e] + X[nur + e]);
  memcpy(J->hh, J->st->h, sizeof(double) * c->ncell);
  memset(J->Ir, 0, sizeof(double) * nur);
  memset(J->Iz, 0, sizeof(double) * nuz);
  for (int s = 0; s < J->nsp; ++s)
    og_push_deposit(c, &J->sp[s], J->urh, J->uzh, J->hh, 0, J->Ir, J->Iz, NULL, NULL);
  og_field_solve(c, J->st->ur, J->st->uz, J->st->h, J->Ir, J->Iz, J->st->t, GX, GX + nur, gh);
  J->evals++;
}

/* Newton iterations from X (in place).  Returns 1 when converged (or the
 * fixed count is done), 0 otherwise; GX and gh hold G(X) of the accepted X,
 * and J->urh/uzh its half field. */
static int jfnk_solve(jfnk_ctx* J, const og_opts* o, double* X, double* GX, double* gh,
                      og_stats* S) {
  og_ctx* c = J->c;
  const int nr = c->g.nr, nz = c->g.nz;
  const int64_t n = (int64_t)nr * (nz + 1) + (int64_t)(nr + 1) * nz;
  const int m = o->krylov;
  const int fixed = o->fixed_iter > 0;
  const int nmax = fixed ? o->fixed_iter : o->max_iter;
  double* F = (double*)malloc(sizeof(double) * n);
  double* V = (double*)malloc(sizeof(double) * n * (m + 1));
  double* Y = (double*)malloc(sizeof(double) * n);
  double* GY = (double*)malloc(sizeof(double) * n);
  double* W = (double*)malloc(sizeof(double) * n);
  double* D = (double*)malloc(sizeof(double) * n);
  double* hy = (double*)malloc(sizeof(double) * c->ncell);
  double H[OG_MAX_KRYLOV + 1][OG_MAX_KRYLOV];
  double cs[OG_MAX_KRYLOV], sn[OG_MAX_KRYLOV], g[OG_MAX_KRYLOV + 1], y[OG_MAX_KRYLOV];
  int conv = 0;
  if (!F || !V || !Y || !GY || !W || !D || !hy) goto out;
  picard_map(J, X, GX, gh);
  for (int64_t e = 0; e < n; ++e) F[e] = X[e] - GX[e];
  double fn = sqrt(wdot(c, F, F)), gn = sqrt(wdot(c, GX, GX));
  for (int k = 0; k < nmax; ++k) {
    const double r = gn > 0.0 ? fn / gn : (fn > 0.0 ? INFINITY : 0.0);
    S->residual[k] = r;
    S->newton_iters = k + 1;
    if (fixed ? (k == nmax - 1) : (r <= o->tol)) { conv = 1; break; }
    if (!(fn > 0.0)) { conv = 1; break; }
    /* GMRES on J d = -F from d = 0 */
    const double xn = sqrt(wdot(c, X, X));
    const double eps = OG_JF_DIFF * (xn > fn ? xn : fn);
    for (int64_t e = 0; e < n; ++e) V[e] = -F[e] / fn;
    g[0] = fn;
    int used = 0;
    for (int j = 0; j < m; ++j) {
      double* vj = V + (int64_t)j * n;
      for (int64_t e = 0; e < n; ++e) Y[e] = X[e] + eps * vj[e];
      picard_map(J, Y, GY, hy);
      for (int64_t e = 0; e < n; ++e) W[e] = vj[e] - (GY[e] - GX[e]) / eps;
      for (int i = 0; i <= j; ++i) {
        const double* vi = V + (int64_t)i * n;
        H[i][j] = wdot(c, W, vi);
        for (int64_t e = 0; e < n; ++e) W[e] -= H[i][j] * vi[e];
      }
      H[j + 1][j] = sqrt(wdot(c, W, W));
      double* vn = V + (int64_t)(j + 1) * n;
      for (int64_t e = 0; e < n; ++e) vn[e] = H[j + 1][j] > 0.0 ? W[e] / H[j + 1][j] : 0.0;
      /* previous rotations on the new column, then its own */
      for (int i = 0; i < j; ++i) {
        const double a = H[i][j], b = H[i + 1][j];
        H[i][j] = cs[i] * a + sn[i] * b;
        H[i + 1][j] = -sn[i] * a + cs[i] * b;
      }
      const double a = H[j][j], b = H[j + 1][j];
      const double d = sqrt(a * a + b * b);
      cs[j] = d > 0.0 ? a / d : 1.0;
      sn[j] = d > 0.0 ? b / d : 0.0;
      H[j][j] = d;
      H[j + 1][j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      used = j + 1;
      S->krylov_iters++;
      if (!fixed && fabs(g[j + 1]) <= o->eta * fn) break;
    }
    /* back substitution: d = sum y_i V_i */
    for (int i = used - 1; i >= 0; --i) {
      double s = g[i];
      for (int q = i + 1; q < used; ++q) s -= H[i][q] * y[q];
      y[i] = s / H[i][i];
    }
    memset(D, 0, sizeof(double) * n);
    for (int i = 0; i < used; ++i) {
      const double* vi = V + (int64_t)i * n;
      for (int64_t e = 0; e < n; ++e) D[e] += y[i] * vi[e];
    }
    /* the step, backtracking in tolerance mode; the trial's map is the next
     * residual evaluation */
    double lam = 1.0;
    for (int ls = 0;; ++ls) {
      for (int64_t e = 0; e < n; ++e) Y[e] = X[e] + lam * D[e];
      picard_map(J, Y, GY, gh);
      for (int64_t e = 0; e < n; ++e) W[e] = Y[e] - GY[e];
      const double fy = sqrt(wdot(c, W, W));
      if (fixed || ls == 8 || fy <= (1.0 - 1e-4 * lam) * fn) {
        memcpy(X, Y, sizeof(double) * n);
        memcpy(GX, GY, sizeof(double) * n);
        memcpy(F, W, sizeof(double) * n);
        fn = fy;
        gn = sqrt(wdot(c, GX, GX));
        break;
      }
      lam *= 0.5;
    }
  }
out:
  free(F); free(V); free(Y); free(GY); free(W); free(D); free(hy);
  return conv;
}

/* ------------------------------------------------------------------------ */
/* Blocking capacitor (Sec. 2.1, Eq. (6)): the current I_e leaving the       */
/* powered electrode into the domain over the step, in the form the energy   */
/* balance of the drive takes (the drive's work is dt V_gap^{1/2} I_e):       */
/*   EM: 2 pi r_{nr-1/2} h^{n+1/2} of the gap cell + I_r of the gap edge;     */
/*   ES: the change of the field flux leaving the plate's nodes over dt, the  */
/*       particle current leaving them, and I_r of the gap edge;              */
/*   with a port (either model): the displacement plus conduction current     */
/*       through the z-edges of the electrode's face r <= r_p, as Eq. (6)     */
/*       writes it (in EM, 2 pi r h^{n+1/2} of the first port cell).          */
/* The electrode potential then follows from the capacitor charge:            */
/* phi^{n+1} = V^{n+1} - (q^n + dt I_e) / C, iterated with the Picard         */
/* iterates, and q^{n+1} = q^n + dt I_e for the accepted one.  The iteration */
/* is converged when the field update and the potential's change (relative  */
/* to the generator's amplitude) are both within the tolerance.              */
/* ------------------------------------------------------------------------ */
/* the scale of the circuit's part of the residual: the sum of the drive
 * amplitudes (1 V when there is none) */
static double circuit_scale(const og_ctx* c) {
  double s = 0.0;
  for (int k = 0; k < c->g.n_drive && k < OG_MAX_DRIVE; ++k) s += fabs(c->g.drive_amp[k]);
  return s > 0.0 ? s : 1.0;
}

static double electrode_current(const og_ctx* c, const og_state* st, const double* uz1,
                                const double* h1, const double* Ir, const double* Iz) {
  const int nr = c->g.nr, nz = c->g.nz;
  const double dt = c->g.dt;
  if (c->ip > 0) {
    /* Eq. (6) over the electrode's face r <= r_p: displacement plus
     * conduction current through the z-edges on its nodes */
    double s = 0.0;
    for (int i = 0; i <= c->ip; ++i)
      s += c->wz[i] * (uz1[UZ(i, 0)] - st->uz[UZ(i, 0)]) / dt + Iz[UZ(i, 0)];
    return s;
  }
  if (c->g.model == OG_ES) {
    double dq = 0.0, ip = 0.0;
    for (int i = 0; i < nr; ++i) {
      dq += c->wz[i] * (uz1[UZ(i, 0)] - st->uz[UZ(i, 0)]);
      ip += Iz[UZ(i, 0)];
    }
    return dq / dt + ip + Ir[UR(nr - 1, 0)];
  }
  const double hgap = 0.5 * (st->h[HC(nr - 1, 0)] + h1[HC(nr - 1, 0)]);
  return 2.0 * OG_PI * c->rh[nr - 1] * hgap + Ir[UR(nr - 1, 0)];
}

/* ------------------------------------------------------------------------ */
/* One implicit step (Picard iteration of the coupled system, Sec. 2.1)      */
/* ------------------------------------------------------------------------ */
int og_step(og_ctx* c, og_state* st, og_species* sp, int32_t nsp, const og_mcc* mcc,
            const og_opts* o, og_stats* S) {
  if (c->g.push_only) return -5;
  const int nr = c->g.nr, nz = c->g.nz;
  const int64_t nur = (int64_t)nr * (nz + 1), nuz = (int64_t)(nr + 1) * nz, nh = c->ncell;
  const double dt = c->g.dt, t = st->t;
  int rc = 0;
  if (nsp > 4 || nsp < 0) return -1;
  og_stats local;
  if (!S) S = &local;
  memset(S, 0, sizeof(*S));
  double* ur1 = (double*)malloc(sizeof(double) * nur);
  double* uz1 = (double*)malloc(sizeof(double) * nuz);
  double* h1 = (double*)malloc(sizeof(double) * nh);
  double* urn = (double*)malloc(sizeof(double) * nur);
  double* uzn = (double*)malloc(sizeof(double) * nuz);
  double* hn = (double*)malloc(sizeof(double) * nh);
  double* urh = (double*)malloc(sizeof(double) * nur);
  double* uzh = (double*)malloc(sizeof(double) * nuz);
  double* hh = (double*)malloc(sizeof(double) * nh);
  double* Ir = (double*)malloc(sizeof(double) * nur);
  double* Iz = (double*)malloc(sizeof(double) * nuz);
  double* dr_ = (double*)malloc(sizeof(double) * nur);
  double* dz_ = (double*)malloc(sizeof(double) * nuz);
  if (!ur1 || !uz1 || !h1 || !urn || !uzn || !hn || !urh || !uzh || !hh || !Ir || !Iz || !dr_ || !dz_) {
    rc = -2;
    goto done;
  }
  /* with a blocking capacitor the gap carries the electrode potential: phi^n
   * now, its extrapolation 2 phi^n - phi^{n-1} as the first iterate */
  const int circ = c->g.cap > 0.0;
  double phi_it = 2.0 * st->phi - st->phi_prev, phi_used = st->phi, ie = 0.0;
  set_boundary(c, st->ur, st->uz, circ ? st->phi : og_drive(c, t));
  /* guess: u^{n+1,(0)} = 2 u^n - u^{n-1}; boundary edges at t^{n+1} */
  for (int64_t k = 0; k < nur; ++k) ur1[k] = 2.0 * st->ur[k] - st->ur_prev[k];
  for (int64_t k = 0; k < nuz; ++k) uz1[k] = 2.0 * st->uz[k] - st->uz_prev[k];
  set_boundary(c, ur1, uz1, circ ? phi_it : og_drive(c, t + dt));
  memcpy(h1, st->h, sizeof(double) * nh);
  c->gap_set = circ;
  c->gap_now = st->phi;
  if (c->ip > 0) og_set_port_h(c, st->hb);
  int k;
  int kmax = o->fixed_iter > 0 ? o->fixed_iter : o->max_iter;
  if (kmax > 64) kmax = 64;
  S->converged = 0;
  if (o->solver == OG_JFNK) {
    if (o->krylov < 1 || o->krylov > OG_MAX_KRYLOV || c->g.self_b || circ) {
      rc = -1;
      goto done;
    }
    const int64_t nv = nur + nuz;
    double* X = (double*)malloc(sizeof(double) * nv);
    double* GX = (double*)malloc(sizeof(double) * nv);
    if (!X || !GX) { free(X); free(GX); rc = -2; goto done; }
    memcpy(X, ur1, sizeof(double) * nur);
    memcpy(X + nur, uz1, sizeof(double) * nuz);
    jfnk_ctx J = {c, st, sp, nsp, urh, uzh, hh, Ir, Iz, 0};
    og_opts oo = *o;
    oo.max_iter = kmax;
    const int ok = jfnk_solve(&J, &oo, X, GX, h1, S);
    /* the accepted iterate: fields G(X), particles pushed in (u^n + X)/2
     * (left in urh, uzh by the last evaluation of G at X) */
    memcpy(ur1, GX, sizeof(double) * nur);
    memcpy(uz1, GX + nur, sizeof(double) * nuz);
    free(X);
    free(GX);
    k = (int)J.evals;
    S->converged = ok;
    S->iters = k;
    if (!ok) { rc = -4; goto done; }
    goto accepted;
  }
  for (k = 0; k < kmax; ++k) {
    for (int64_t e = 0; e < nur; ++e) urh[e] = 0.5 * (st->ur[e] + ur1[e]);
    for (int64_t e = 0; e < nuz; ++e) uzh[e] = 0.5 * (st->uz[e] + uz1[e]);
    for (int64_t e = 0; e < nh; ++e) hh[e] = 0.5 * (st->h[e] + h1[e]);
    memset(Ir, 0, sizeof(double) * nur);
    memset(Iz, 0, sizeof(double) * nuz);
    for (int s = 0; s < nsp; ++s) og_push_deposit(c, &sp[s], urh, uzh, hh, 0, Ir, Iz, NULL, NULL);
    c->gap_next = phi_it;
    og_field_solve(c, st->ur, st->uz, st->h, Ir, Iz, t, urn, uzn, hn);
    if (circ) {
      ie = electrode_current(c, st, uzn, hn, Ir, Iz);
      phi_used = phi_it;
      phi_it = og_drive(c, t + dt) - (st->q_cap + dt * ie) / c->g.cap;
    }
    for (int64_t e = 0; e < nur; ++e) dr_[e] = urn[e] - ur1[e];
    for (int64_t e = 0; e < nuz; ++e) dz_[e] = uzn[e] - uz1[e];
    const double num = og_energy_norm2(c, dr_, dz_), den = og_energy_norm2(c, urn, uzn);
    double r = (den > 0.0) ? sqrt(num / den) : (num > 0.0 ? INFINITY : 0.0);
    if (circ) {
      /* the electrode potential's change, against the generator's amplitude */
      const double rc_ = fabs(phi_it - phi_used) / circuit_scale(c);
      if (rc_ > r) r = rc_;
    }
    S->residual[k] = r;
    memcpy(ur1, urn, sizeof(double) * nur);
    memcpy(uz1, uzn, sizeof(double) * nuz);
    memcpy(h1, hn, sizeof(double) * nh);
    if (o->fixed_iter <= 0 && r <= o->tol) { S->converged = 1; k++; break; }
  }
  S->iters = k;
  if (o->fixed_iter > 0) S->converged = 1;
  if (!S->converged) { rc = -4; goto done; }
accepted:
  /* commit the particles from the last push (field urh, uzh, hh) and
   * account the energy exchanged with the field on both sides */
  memset(Ir, 0, sizeof(double) * nur);
  memset(Iz, 0, sizeof(double) * nuz);
  for (int s = 0; s < nsp; ++s) {
    int64_t n_before = sp[s].n;
    const int e = og_push_deposit(c, &sp[s], urh, uzh, hh, 1, Ir, Iz, st, S);
    if (e < 0) rc = -5;
    S->n_absorbed[s] = n_before - sp[s].n;
  }
  {
    /* field side: dt * sum over interior edges of u^{1/2}_field . I, and the
     * drive: dt * (2 pi r h^{1/2} V^{1/2} + V^{1/2} I_gap) */
    double wio = 0.0;
    for (int i = 0; i < nr; ++i)
      for (int j = 1; j < nz; ++j) wio += 0.5 * (st->ur[UR(i, j)] + ur1[UR(i, j)]) * Ir[UR(i, j)];
    for (int i = c->ip; c->ip > 0 && i < nr; ++i)
      wio += 0.5 * (st->ur[UR(i, 0)] + ur1[UR(i, 0)]) * Ir[UR(i, 0)];
    for (int i = 0; i < nr; ++i)
      for (int j = 0; j < nz; ++j) wio += 0.5 * (st->uz[UZ(i, j)] + uz1[UZ(i, j)]) * Iz[UZ(i, j)];
    S->w_field_io = dt * wio;
    const double vgen = 0.5 * (og_drive(c, t) + og_drive(c, t + dt));
    const double vh = circ ? 0.5 * (st->phi + phi_used) : vgen;
    if (c->ip > 0 && c->g.model == OG_ES) {
      /* the source's work on the powered wall nodes (profile p): phi^{1/2}
       * times sum p (change of the node's Gauss charge, port edges with
       * their half faces, plus dt times the current leaving it) */
      double sq = 0.0;
      for (int i = 0; i <= nr; ++i) {
        double dg = 0.0, dv = 0.0;
        if (i < nr) {
          dg += c->wz[i] * (uz1[UZ(i, 0)] - st->uz[UZ(i, 0)]);
          dv += Iz[UZ(i, 0)] + Ir[UR(i, 0)];
          if (i >= c->ip) dg += 0.5 * c->wr[i] * (ur1[UR(i, 0)] - st->ur[UR(i, 0)]);
        }
        if (i > 0) {
          dv -= Ir[UR(i - 1, 0)];
          if (i - 1 >= c->ip) dg -= 0.5 * c->wr[i - 1] * (ur1[UR(i - 1, 0)] - st->ur[UR(i - 1, 0)]);
        }
        sq += c->pprof[i] * (dg + dt * dv);
      }
      S->w_drive = vh * sq;
    } else if (c->ip > 0) {
      /* the power the line delivers through the mouth: M H_b u per edge at
       * the half step (H_b at t^{n+1} from the solve of the accepted
       * iterate, the last one made) */
      double pw = 0.0;
      for (int i = c->ip; i < nr; ++i)
        pw += 2.0 * OG_PI * c->rh[i] * 0.5 * (st->hb[i] + c->hb1[i]) * 0.5 *
              (st->ur[UR(i, 0)] + ur1[UR(i, 0)]);
      S->w_drive = dt * pw;
    } else if (c->g.model == OG_ES) {
      /* the source's work: V^{1/2} times the charge it moves onto the
       * powered plate's nodes (the change of their field flux plus the
       * current leaving them into the domain), plus the gap edge's share */
      double dq = 0.0, ip = 0.0;
      for (int i = 0; i < nr; ++i) {
        dq += c->wz[i] * (uz1[UZ(i, 0)] - st->uz[UZ(i, 0)]);
        ip += Iz[UZ(i, 0)];
      }
      S->w_drive = vh * (dq + dt * ip) + dt * vh * Ir[UR(nr - 1, 0)];
    } else {
      const double hgap = 0.5 * (st->h[HC(nr - 1, 0)] + h1[HC(nr - 1, 0)]);
      S->w_drive = dt * (2.0 * OG_PI * c->rh[nr - 1] * hgap * vh + vh * Ir[UR(nr - 1, 0)]);
    }
    if (circ) S->w_gen = dt * vgen * ie;
  }
  if (mcc && mcc->enabled) {
    const int e = og_collide(c, sp, nsp, mcc, st->step, S);
    if (e < 0) rc = e;
  }
  memcpy(st->ur_prev, st->ur, sizeof(double) * nur);
  memcpy(st->uz_prev, st->uz, sizeof(double) * nuz);
  memcpy(st->ur, ur1, sizeof(double) * nur);
  memcpy(st->uz, uz1, sizeof(double) * nuz);
  memcpy(st->h, h1, sizeof(double) * nh);
  st->t = t + dt;
  st->step += 1;
  if (circ) {
    st->phi_prev = st->phi;
    st->phi = phi_used;
    st->q_cap += dt * ie;
  }
  if (c->ip > 0) {
    double v = 0.0;
    for (int i = c->ip; i < nr; ++i) {
      if (c->g.model == OG_EM) st->hb[i] = c->hb1[i];
      v += st->ur[UR(i, 0)];
    }
    S->port_v = v;
  }
  S->phi = st->phi;
  S->q_cap = st->q_cap;
  for (int s = 0; s < nsp; ++s) S->ke[s] = og_kinetic(&sp[s]);
  S->we = og_energy_e(c, st->ur, st->uz);
  S->wb = og_energy_b(c, st->h);
done:
  c->gap_set = 0;
  free(ur1); free(uz1); free(h1); free(urn); free(uzn); free(hn);
  free(urh); free(uzh); free(hh); free(Ir); free(Iz); free(dr_); free(dz_);
  return rc;
}
