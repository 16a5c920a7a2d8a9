/*
 * FP64 CPU oracle for the modal discontinuous-Galerkin Euler scheme of
 * Bauer et al., "Simulating Turbulence Using the Astrophysical Discontinuous
 * Galerkin Code TENET" (arXiv 1602.09079).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct
 * definition that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or constant with the GPU library.
 *
 * Every array is FP64 on the host.  State layout:
 *   y[i][l][z][y][x], x fastest; i = field (rho, m_x, m_y, m_z, E);
 *   l = mode index in the graded order listed by orc_mode_list().
 *
 * Parity status per function (pins live in tests/test_oracle_*.py):
 *   tables, projection, rhs, hllc, flux, dt, step, totals  -- pinned
 *   forcing table (OU + Helmholtz projection)               -- pinned (statistics, solenoidality)
 *   restriction                                             -- pinned (exactness, conservation)
 *   MLP forward/backward/Adam                               -- pinned (finite differences, textbook Adam)
 *   positivity limiter, GLL rules, limited dt               -- pinned (closed-form cases, invariants)
 *   closure features / correction                           -- pinned (neighbour order, closed-form outputs,
 *                                                              fallback, zero-sum mean rows)
 */
#ifndef DG_ORACLE_H
#define DG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t k;          /* polynomial degree, 0..3 */
    int32_t n[3];       /* cells per axis */
    double box[3];      /* box lengths; cells are box[a]/n[a] wide */
    double gamma;       /* adiabatic index */
    double cfl;         /* Courant factor C of Sec. 2.4 */
    int32_t riemann;    /* numerical flux: 0 HLLC (Toro ch. 10), 1 exact Riemann solver (Toro ch. 4) */
} orc_cfg;

typedef struct {
    int32_t nmodes;          /* number of Fourier modes in the table */
    const int32_t *nvec;     /* [nmodes][3] integer wave vectors */
    const double *ahat;      /* [nmodes][3][2] complex amplitude (re, im) per component */
} orc_forcing;

/* ---- Sec. 2.1: basis ---- */
int    orc_nmodes(int k);
void   orc_mode_list(int k, int32_t *uvw);                 /* [N][3] degrees (u,v,w) */
void   orc_gauss_legendre(int n, double *x, double *w);   /* n-point rule on [-1,1] */
double orc_pleg(int u, double x);                         /* scaled Legendre sqrt(2u+1) P_u */
double orc_dpleg(int u, double x);                        /* its derivative */
void   orc_basis(int k, const double xi[3], double *phi);          /* [N] */
void   orc_basis_grad(int k, const double xi[3], double *dphi);    /* [3][N] */

/* ---- Sec. 2.2: initial conditions by Gauss-quadrature L2 projection ----
 * qp: point values [5][c][b][a][cell] at the (k+1)^3 Gauss points of every
 * cell (a,b,c = Gauss index along x,y,z).  y: [5][N][cell]. */
void orc_project(const orc_cfg *cfg, const double *qp, double *y);
/* point coordinates of the Gauss points in cell-relative units: the x-coordinate
 * of Gauss index a in cell ix is (ix + (1 + xi_a)/2) * box/n */

/* ---- Sec. 2.3: the operator ---- */
void orc_euler_flux(const double q[5], int axis, double gamma, double F[5]);
void orc_hllc(const double qL[5], const double qR[5], int axis, double gamma, double F[5]);
void orc_exact_riemann(const double qL[5], const double qR[5], int axis, double gamma, double F[5]);
/* r = R(y) with dy/dt + R(y) = 0 (eq. dg:eqn:time); frc may be NULL */
void orc_rhs(const orc_cfg *cfg, const double *y, const orc_forcing *frc, double *r);
/* R at listed cells only (cell = (z*ny + y)*nx + x); r: [ncells_list][5][N] */
void orc_rhs_cells(const orc_cfg *cfg, const double *y, const orc_forcing *frc, int64_t ncells_list,
                   const int64_t *cells, double *r);

/* ---- Sec. 2.4: time step from cell means, global minimum ---- */
double orc_dt(const orc_cfg *cfg, const double *y);

/* ---- Sec. 2.3: SSP-RK3 in Shu-Osher form.  dt <= 0 selects the CFL time step
 * of Sec. 2.4 at the start of every step.  t is advanced by the steps taken. */
void orc_step(const orc_cfg *cfg, double *y, double dt, int nsteps, double *t,
              const orc_forcing *frc);
/* a single stage: out = a*y0 + b*(yin - dt*R(yin)) */
void orc_stage(const orc_cfg *cfg, const double *y0, const double *yin, double a, double b,
               double dt, const orc_forcing *frc, double *out);

/* conserved totals sum_K |K| w_{i,0}^K (pairwise summation) */
void orc_totals(const orc_cfg *cfg, const double *y, double out[5]);

/* ---- Sec. 3.1: driving field ----
 * acceleration at physical point x: a_c(x) = sum_m Re(ahat_{m,c} exp(2 pi i n_m.x/L)) */
void orc_accel(const orc_forcing *frc, const double box[3], const double x[3], double a[3]);
/* One Ornstein-Uhlenbeck update of the complex amplitudes followed by the
 * Helmholtz (solenoidal) projection and the paraboloid amplitude profile.
 * theta: [nmodes][3][2] OU state (updated in place); z: [nmodes][3][2] standard
 * normal draws; f = exp(-dt/t_s); sigma: OU standard deviation; a0: overall
 * amplitude; kmin/kmax: band in units of 2 pi / L.  ahat out: [nmodes][3][2]. */
void orc_ou_update(int32_t nmodes, const int32_t *nvec, double *theta, const double *z,
                   double f, double sigma, double a0, double kmin, double kmax, double *ahat);

/* ---- Sec. 2.5: positivity limiter (Zhang and Shu) ----
 * Points S = S_x u S_y u S_z: the m GLL nodes along one axis (m = 2 for k <= 1,
 * 3 for k = 2, 3, 4 for k = 4: the fewest with 2m - 3 >= k) times the k+1 Gauss
 * nodes along the other two.  Per cell:
 * theta_1 = min(|(rhobar - eps)/(rhobar - rho_min)|, 1) over S scales the
 * density's modes l >= 1; then theta_2 = min over S of tau, tau = 1 where
 * P >= eps, else the root of P(qbar + tau (q - qbar)) = eps (the garbled
 * printed form read as Zhang-Shu's), scales every field's modes l >= 1.
 * y is limited in place; theta (may be NULL) receives [cell][2] = (th1, th2). */
int    orc_limiter_m(int k);
void   orc_gll(int m, double *x, double *w);
int    orc_limiter_points(int k, double *pts);
/* rel > 0 raises the targets to max(eps, rel rhobar) and max(eps, rel (gamma-1) Ebar) per cell
 * (single-precision storage); rel = 0 is the plain limiter */
void   orc_limit(const orc_cfg *cfg, double *y, double eps, double rel, double *theta);
/* dt of the limited scheme: C min(1/(2k+1), w_hat_1/2) / max rate */
double orc_dt_limited(const orc_cfg *cfg, const double *y);
/* SSP-RK3 with the limiter applied to each stage's input (y^n in place for stage 1) */
void   orc_step_limited(const orc_cfg *cfg, double *y, double dt, int nsteps, double *t, const orc_forcing *frc,
                        double eps);

/* ---- Sec. 3.2: isothermal reset and the dissipated energy ----
 * After a time step the specific internal energy
 *   eps(rho) = cs^2/(gamma-1) (rho/rho0)^(gamma-1)
 * is imposed at the (k+1)^3 Gauss points of every cell: the energy weights become
 *   w_E,l = (1/8) sum_q (|m_q|^2/(2 rho_q) + rho_q eps(rho_q)) phi_l(xi_q) omega_q
 * with rho_q, m_q from the cell's current weights (rho and m unchanged).
 * Returns the dissipated energy sum_K |K| (rhoe_before - rhoe_after), where per
 * cell rhoe = w_E,0 - |w_m,0|^2 / (2 w_rho,0) (the cell-mean internal energy). */
double orc_isothermal_reset(const orc_cfg *cfg, double *y, double cs, double rho0);
/* nsteps SSP-RK3 steps, each followed by the reset; with limit != 0 the limiter (eps, rel = 0)
 * is applied to every stage input as in orc_step_limited and once more after the reset, and the
 * limited time step is used.  dissipated (may be NULL) accumulates the reset's return values. */
void orc_step_isothermal(const orc_cfg *cfg, double *y, double dt, int nsteps, double *t,
                         const orc_forcing *frc, double cs, double rho0, int limit, double eps,
                         double *dissipated);

/* ---- closure support (not in the paper) ---- */
/* exact L2 restriction of a degree-kf state on (2n)^3 cells onto degree-kc on n^3 cells */
void orc_restrict(int kf, int kc, const int32_t nc[3], const double *yf, double *yc);
/* 140-128-128-20 tanh MLP: see orc_mlp_* in dg_oracle.c for the parameter layout */
void orc_mlp_forward(int nin, int nh1, int nh2, int nout, const double *params,
                     int batch, const double *x, double *h1, double *h2, double *yout);
double orc_mlp_loss_grad(int nin, int nh1, int nh2, int nout, const double *params,
                         int batch, const double *x, const double *target, double *grad);
void orc_adam(int nparams, double *params, const double *grad, double *m, double *v,
              int step, double lr, double beta1, double beta2, double eps);

/* Per-cell closure.  A cell's features are the weights of itself and of its
 * -x, +x, -y, +y, -z, +z neighbours: feat[cell][j][i][l], 7*5*N values (140 at
 * k=1).  The network sees (feat - feat_mean)/feat_std; its output o (nout =
 * 5N, ordered [i][l]) gives the correction c = out_scale * o, added to the
 * time derivative: dy/dt = -R(y) + c.  A cell with any o_j non-finite or
 * |o_j| > out_bound_j gets c = 0 (the plain operator).  Afterwards the l = 0
 * rows of c are shifted to zero sum over cells per field (totals conserved). */
typedef struct {
    int32_t nin, nh1, nh2, nout;
    const double *params;      /* orc_mlp_* layout */
    const double *feat_mean;   /* [nin] */
    const double *feat_std;    /* [nin] */
    const double *out_scale;   /* [nout] */
    const double *out_bound;   /* [nout] */
} orc_closure;
void orc_closure_features(const orc_cfg *cfg, const double *y, double *feat);   /* [ncells][7*5*N] */
/* corr: state layout; returns the number of cells that fell back */
int64_t orc_closure_correction(const orc_cfg *cfg, const double *y, const orc_closure *clo, double *corr);

#ifdef __cplusplus
}
#endif
#endif
