/*
 * FP64 CPU oracle: a plain, slow, literal implementation of the modal DG
 * scheme of Bauer et al. (arXiv 1602.09079), Sec. 2, and of its driving
 * source term, Sec. 3.1.
 *
 * TEST INFRASTRUCTURE ONLY -- the reference that the GPU library is checked
 * against.  Nothing in the product path may load it.  It shares no code with
 * the GPU library: its quadrature comes from Newton iteration on Legendre
 * polynomials and its basis from the Bonnet recurrence, its operator is the
 * paper's dense per-cell / per-face quadrature sums.  Each cell evaluates the
 * numerical flux of its six faces from the two traces, in the +axis
 * orientation, so both cells of a face use the same value.
 *
 * Readings of the paper used here (where it is silent or garbled):
 *  - basis normalised so that (1/8) int phi_l phi_m dxi = delta_lm, i.e. the
 *    scaled Legendre polynomial is sqrt(2u+1) P_u and phi_0 = 1 (Sec. 2.1,
 *    "orthonormal" together with w_{0,0} being the cell mean);
 *  - mode order graded by total degree d = 0..k, then u descending, then v
 *    descending, w = d-u-v (Sec. 2.1 lists the set but not its order);
 *  - ideal-gas Euler flux, p = (gamma-1)(E - |m|^2/(2 rho)) (Sec. 2.3 names
 *    F_alpha but does not write it out);
 *  - the surface sum uses the basis at the face point and the outward normal
 *    (eq. dg:eqn:surface_int prints phi_l at the volume point);
 *  - HLLC with Davis wave-speed estimates (Toro, Riemann Solvers and Numerical
 *    Methods for Fluid Dynamics, ch. 10); S* >= 0 takes the left star state;
 *  - time step from the cell-mean conserved variables (Sec. 2.4);
 *  - driving acceleration a_c(x) = sum_m Re(ahat_{m,c} e^{2 pi i n_m.x/L}),
 *    momentum source rho*a and energy source m.a, both projected with the
 *    volume Gauss rule (Sec. 3.1).
 */
#include "dg_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NF 5
#define KMAX 4
#define NMAX 35          /* N(4) */
#define GMAX (KMAX + 2)  /* Gauss points per axis handled here */

/* ------------------------------------------------------------------ */
/* Sec. 2.1: basis                                                      */
/* ------------------------------------------------------------------ */

int orc_nmodes(int k) { return (k + 1) * (k + 2) * (k + 3) / 6; }

void orc_mode_list(int k, int32_t *uvw)
{
    int l = 0;
    for (int d = 0; d <= k; d++)
        for (int u = d; u >= 0; u--)
            for (int v = d - u; v >= 0; v--) {
                uvw[3 * l + 0] = u;
                uvw[3 * l + 1] = v;
                uvw[3 * l + 2] = d - u - v;
                l++;
            }
}

/* unscaled Legendre P_n(x) and P_{n-1}(x) by the Bonnet recurrence */
static void legendre_pair(int n, double x, double *pn, double *pnm1)
{
    double p0 = 1.0, p1 = x;
    if (n == 0) { *pn = 1.0; *pnm1 = 0.0; return; }
    for (int m = 1; m < n; m++) {
        double p2 = ((2.0 * m + 1.0) * x * p1 - m * p0) / (m + 1.0);
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;
    *pnm1 = p0;
}

void orc_gauss_legendre(int n, double *x, double *w)
{
    /* roots of P_n by Newton's method, weights 2 / ((1 - x^2) P_n'(x)^2) */
    for (int i = 0; i < n; i++) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double pn, pm;
            legendre_pair(n, z, &pn, &pm);
            dp = n * (z * pn - pm) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (fabs(dz) < 1e-17) break;
        }
        double pn, pm;
        legendre_pair(n, z, &pn, &pm);
        dp = n * (z * pn - pm) / (z * z - 1.0);
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

double orc_pleg(int u, double x)
{
    double pn, pm;
    legendre_pair(u, x, &pn, &pm);
    return sqrt(2.0 * u + 1.0) * pn;
}

double orc_dpleg(int u, double x)
{
    /* P_u' = P_{u-2}' + (2u - 1) P_{u-1} */
    double d[KMAX + 3];
    d[0] = 0.0;
    if (u >= 1) d[1] = 1.0;
    for (int m = 2; m <= u; m++) {
        double pn, pm;
        legendre_pair(m - 1, x, &pn, &pm);
        d[m] = d[m - 2] + (2.0 * m - 1.0) * pn;
    }
    return sqrt(2.0 * u + 1.0) * d[u];
}

void orc_basis(int k, const double xi[3], double *phi)
{
    int32_t uvw[3 * NMAX];
    int N = orc_nmodes(k);
    orc_mode_list(k, uvw);
    for (int l = 0; l < N; l++)
        phi[l] = orc_pleg(uvw[3 * l], xi[0]) * orc_pleg(uvw[3 * l + 1], xi[1]) *
                 orc_pleg(uvw[3 * l + 2], xi[2]);
}

void orc_basis_grad(int k, const double xi[3], double *dphi)
{
    int32_t uvw[3 * NMAX];
    int N = orc_nmodes(k);
    orc_mode_list(k, uvw);
    for (int l = 0; l < N; l++) {
        int u = uvw[3 * l], v = uvw[3 * l + 1], w = uvw[3 * l + 2];
        dphi[0 * N + l] = orc_dpleg(u, xi[0]) * orc_pleg(v, xi[1]) * orc_pleg(w, xi[2]);
        dphi[1 * N + l] = orc_pleg(u, xi[0]) * orc_dpleg(v, xi[1]) * orc_pleg(w, xi[2]);
        dphi[2 * N + l] = orc_pleg(u, xi[0]) * orc_pleg(v, xi[1]) * orc_dpleg(w, xi[2]);
    }
}

/* ------------------------------------------------------------------ */
/* per-degree tables of basis values at the Gauss points                */
/* ------------------------------------------------------------------ */

typedef struct {
    int k, N, n, Q, P;                /* P = n*n points per face */
    double xg[GMAX], wg[GMAX];
    double *phi_v;                    /* [Q][N]  volume point q = (c*n + b)*n + a */
    double *dphi_v;                   /* [3][Q][N] */
    double *w_v;                      /* [Q] */
    double *phi_f;                    /* [3 axes][2 sides][P][N]; side 0 = xi_axis=-1 */
    double *w_f;                      /* [P] */
} tables;

static void face_point(int axis, int side, int p, int n, const double *xg, double xi[3])
{
    /* face points enumerate the two remaining axes in increasing axis order,
     * the first of them fastest */
    int i0 = p % n, i1 = p / n;
    int o0 = (axis == 0) ? 1 : 0;
    int o1 = (axis == 2) ? 1 : 2;
    xi[axis] = side ? 1.0 : -1.0;
    xi[o0] = xg[i0];
    xi[o1] = xg[i1];
}

static void tables_init(tables *t, int k)
{
    t->k = k;
    t->N = orc_nmodes(k);
    t->n = k + 1;
    t->Q = t->n * t->n * t->n;
    t->P = t->n * t->n;
    orc_gauss_legendre(t->n, t->xg, t->wg);
    int N = t->N, n = t->n, Q = t->Q, P = t->P;
    t->phi_v = malloc(sizeof(double) * Q * N);
    t->dphi_v = malloc(sizeof(double) * 3 * Q * N);
    t->w_v = malloc(sizeof(double) * Q);
    t->phi_f = malloc(sizeof(double) * 6 * P * N);
    t->w_f = malloc(sizeof(double) * P);
    double dbuf[3 * NMAX];
    for (int c = 0; c < n; c++)
        for (int b = 0; b < n; b++)
            for (int a = 0; a < n; a++) {
                int q = (c * n + b) * n + a;
                double xi[3] = {t->xg[a], t->xg[b], t->xg[c]};
                orc_basis(k, xi, t->phi_v + q * N);
                orc_basis_grad(k, xi, dbuf);
                for (int al = 0; al < 3; al++)
                    for (int l = 0; l < N; l++) t->dphi_v[(al * Q + q) * N + l] = dbuf[al * N + l];
                t->w_v[q] = t->wg[a] * t->wg[b] * t->wg[c];
            }
    for (int axis = 0; axis < 3; axis++)
        for (int side = 0; side < 2; side++)
            for (int p = 0; p < P; p++) {
                double xi[3];
                face_point(axis, side, p, n, t->xg, xi);
                orc_basis(k, xi, t->phi_f + ((axis * 2 + side) * P + p) * N);
            }
    for (int p = 0; p < P; p++) t->w_f[p] = t->wg[p % n] * t->wg[p / n];
}

static void tables_free(tables *t)
{
    free(t->phi_v);
    free(t->dphi_v);
    free(t->w_v);
    free(t->phi_f);
    free(t->w_f);
}

static inline size_t ncells_of(const orc_cfg *c) { return (size_t)c->n[0] * c->n[1] * c->n[2]; }

/* ------------------------------------------------------------------ */
/* Sec. 2.2: projection of point values                                */
/* ------------------------------------------------------------------ */

void orc_project(const orc_cfg *cfg, const double *qp, double *y)
{
    tables t;
    tables_init(&t, cfg->k);
    size_t nc = ncells_of(cfg);
    int N = t.N, Q = t.Q;
#pragma omp parallel for schedule(static)
    for (size_t K = 0; K < nc; K++)
        for (int i = 0; i < NF; i++)
            for (int l = 0; l < N; l++) {
                double s = 0.0;
                for (int q = 0; q < Q; q++)
                    s += qp[((size_t)i * Q + q) * nc + K] * t.phi_v[q * N + l] * t.w_v[q];
                y[((size_t)i * N + l) * nc + K] = s / 8.0;
            }
    tables_free(&t);
}

/* ------------------------------------------------------------------ */
/* Sec. 2.3: Euler flux and the HLLC numerical flux                    */
/* ------------------------------------------------------------------ */

static inline double pressure(const double q[5], double gamma)
{
    double ke = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
    return (gamma - 1.0) * (q[4] - ke);
}

void orc_euler_flux(const double q[5], int axis, double gamma, double F[5])
{
    double p = pressure(q, gamma);
    double un = q[1 + axis] / q[0];
    F[0] = q[1 + axis];
    F[1] = q[1] * un;
    F[2] = q[2] * un;
    F[3] = q[3] * un;
    F[1 + axis] += p;
    F[4] = (q[4] + p) * un;
}

static void star_state(const double q[5], int axis, double p, double S, double Ss, double U[5])
{
    double rho = q[0], un = q[1 + axis] / rho;
    double fac = rho * (S - un) / (S - Ss);
    U[0] = fac;
    for (int j = 0; j < 3; j++) U[1 + j] = fac * q[1 + j] / rho;
    U[1 + axis] = fac * Ss;
    U[4] = fac * (q[4] / rho + (Ss - un) * (Ss + p / (rho * (S - un))));
}

void orc_hllc(const double qL[5], const double qR[5], int axis, double gamma, double F[5])
{
    double pL = pressure(qL, gamma), pR = pressure(qR, gamma);
    double uL = qL[1 + axis] / qL[0], uR = qR[1 + axis] / qR[0];
    double cL = sqrt(gamma * pL / qL[0]), cR = sqrt(gamma * pR / qR[0]);
    double SL = fmin(uL - cL, uR - cR);
    double SR = fmax(uL + cL, uR + cR);
    double Ss = (pR - pL + qL[0] * uL * (SL - uL) - qR[0] * uR * (SR - uR)) /
                (qL[0] * (SL - uL) - qR[0] * (SR - uR));
    double FK[5], US[5];
    if (SL >= 0.0) {
        orc_euler_flux(qL, axis, gamma, F);
    } else if (Ss >= 0.0) {
        orc_euler_flux(qL, axis, gamma, FK);
        star_state(qL, axis, pL, SL, Ss, US);
        for (int i = 0; i < 5; i++) F[i] = FK[i] + SL * (US[i] - qL[i]);
    } else if (SR > 0.0) {
        orc_euler_flux(qR, axis, gamma, FK);
        star_state(qR, axis, pR, SR, Ss, US);
        for (int i = 0; i < 5; i++) F[i] = FK[i] + SR * (US[i] - qR[i]);
    } else {
        orc_euler_flux(qR, axis, gamma, F);
    }
}

/* Exact Riemann solver (the alternative numerical flux of Sec. 2.3), after Toro, Riemann
 * Solvers and Numerical Methods for Fluid Dynamics, ch. 4: the star pressure is the root of
 * f_L(p) + f_R(p) + (u_R - u_L) = 0 with the shock (Rankine-Hugoniot) or rarefaction
 * (isentropic) branch of each side, found here by bisection (slow, obviously convergent: f is
 * increasing in p); the similarity solution is sampled on the face (x/t = 0) and its Euler
 * flux returned.  Tangential velocities travel with the contact.  When the data generate
 * vacuum (2(c_L + c_R)/(gamma-1) <= u_R - u_L) the vacuum solution is sampled. */
static double wave_f(double p, double rK, double pK, double cK, double gamma)
{
    if (p > pK) {
        double A = 2.0 / ((gamma + 1.0) * rK), B = (gamma - 1.0) / (gamma + 1.0) * pK;
        return (p - pK) * sqrt(A / (p + B));
    }
    return 2.0 * cK / (gamma - 1.0) * (pow(p / pK, (gamma - 1.0) / (2.0 * gamma)) - 1.0);
}

/* primitive state (rho, u_normal, p) at x/t = 0 of the fan on side K (sign = -1 left, +1 right) */
static void fan_state(double rK, double uK, double pK, double cK, double gamma, double sign, double W[3])
{
    double g1 = gamma - 1.0, gp = gamma + 1.0;
    double c = 2.0 / gp - sign * g1 / (gp * cK) * uK;
    W[0] = rK * pow(c, 2.0 / g1);
    W[1] = 2.0 / gp * (-sign * cK + g1 / 2.0 * uK);
    W[2] = pK * pow(c, 2.0 * gamma / g1);
}

void orc_exact_riemann(const double qL[5], const double qR[5], int axis, double gamma, double F[5])
{
    double rL = qL[0], rR = qR[0];
    double uL = qL[1 + axis] / rL, uR = qR[1 + axis] / rR;
    double pL = pressure(qL, gamma), pR = pressure(qR, gamma);
    double cL = sqrt(gamma * pL / rL), cR = sqrt(gamma * pR / rR);
    double g1 = gamma - 1.0, gp = gamma + 1.0;
    double W[3];      /* rho, u_normal, p on the face */
    const double *qt; /* side whose tangential velocities are carried */
    if (2.0 * (cL + cR) / g1 <= uR - uL) {
        /* vacuum between two rarefactions */
        double sL = uL + 2.0 * cL / g1, sR = uR - 2.0 * cR / g1;
        if (0.0 <= sL) {
            qt = qL;
            if (0.0 <= uL - cL) { W[0] = rL; W[1] = uL; W[2] = pL; }
            else fan_state(rL, uL, pL, cL, gamma, -1.0, W);
        } else if (0.0 >= sR) {
            qt = qR;
            if (0.0 >= uR + cR) { W[0] = rR; W[1] = uR; W[2] = pR; }
            else fan_state(rR, uR, pR, cR, gamma, 1.0, W);
        } else {
            qt = qL;
            W[0] = 0.0; W[1] = 0.0; W[2] = 0.0;
        }
    } else {
        /* star pressure by bisection on the increasing function f */
        double lo = 0.0, hi = fmax(pL, pR);
        double du = uR - uL;
        while (wave_f(hi, rL, pL, cL, gamma) + wave_f(hi, rR, pR, cR, gamma) + du < 0.0) hi *= 2.0;
        for (int it = 0; it < 200; it++) {
            double mid = 0.5 * (lo + hi);
            if (mid == lo || mid == hi) break;
            if (wave_f(mid, rL, pL, cL, gamma) + wave_f(mid, rR, pR, cR, gamma) + du < 0.0) lo = mid;
            else hi = mid;
        }
        double ps = 0.5 * (lo + hi);
        double us = 0.5 * (uL + uR) + 0.5 * (wave_f(ps, rR, pR, cR, gamma) - wave_f(ps, rL, pL, cL, gamma));
        if (0.0 <= us) {
            qt = qL;
            if (ps > pL) { /* left shock */
                double S = uL - cL * sqrt(gp / (2.0 * gamma) * ps / pL + g1 / (2.0 * gamma));
                if (0.0 <= S) { W[0] = rL; W[1] = uL; W[2] = pL; }
                else { W[0] = rL * (ps / pL + g1 / gp) / (g1 / gp * ps / pL + 1.0); W[1] = us; W[2] = ps; }
            } else { /* left rarefaction */
                double head = uL - cL, tail = us - cL * pow(ps / pL, g1 / (2.0 * gamma));
                if (0.0 <= head) { W[0] = rL; W[1] = uL; W[2] = pL; }
                else if (0.0 >= tail) { W[0] = rL * pow(ps / pL, 1.0 / gamma); W[1] = us; W[2] = ps; }
                else fan_state(rL, uL, pL, cL, gamma, -1.0, W);
            }
        } else {
            qt = qR;
            if (ps > pR) { /* right shock */
                double S = uR + cR * sqrt(gp / (2.0 * gamma) * ps / pR + g1 / (2.0 * gamma));
                if (0.0 >= S) { W[0] = rR; W[1] = uR; W[2] = pR; }
                else { W[0] = rR * (ps / pR + g1 / gp) / (g1 / gp * ps / pR + 1.0); W[1] = us; W[2] = ps; }
            } else { /* right rarefaction */
                double head = uR + cR, tail = us + cR * pow(ps / pR, g1 / (2.0 * gamma));
                if (0.0 >= head) { W[0] = rR; W[1] = uR; W[2] = pR; }
                else if (0.0 <= tail) { W[0] = rR * pow(ps / pR, 1.0 / gamma); W[1] = us; W[2] = ps; }
                else fan_state(rR, uR, pR, cR, gamma, 1.0, W);
            }
        }
    }
    /* Euler flux of the face state, tangential velocities from side qt */
    double v[3];
    for (int a = 0; a < 3; a++) v[a] = qt[1 + a] / qt[0];
    v[axis] = W[1];
    double E = W[2] / g1 + 0.5 * W[0] * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    F[0] = W[0] * W[1];
    for (int a = 0; a < 3; a++) F[1 + a] = W[0] * W[1] * v[a];
    F[1 + axis] += W[2];
    F[4] = W[1] * (E + W[2]);
}

static void face_flux(const orc_cfg *cfg, const double qL[5], const double qR[5], int axis, double F[5])
{
    if (cfg->riemann == 1) orc_exact_riemann(qL, qR, axis, cfg->gamma, F);
    else orc_hllc(qL, qR, axis, cfg->gamma, F);
}

/* ------------------------------------------------------------------ */
/* Sec. 3.1: driving acceleration                                      */
/* ------------------------------------------------------------------ */

void orc_accel(const orc_forcing *frc, const double box[3], const double x[3], double a[3])
{
    a[0] = a[1] = a[2] = 0.0;
    for (int m = 0; m < frc->nmodes; m++) {
        const int32_t *nv = frc->nvec + 3 * m;
        double th = 2.0 * M_PI * (nv[0] * x[0] / box[0] + nv[1] * x[1] / box[1] + nv[2] * x[2] / box[2]);
        double cs = cos(th), sn = sin(th);
        for (int c = 0; c < 3; c++) {
            double re = frc->ahat[(m * 3 + c) * 2], im = frc->ahat[(m * 3 + c) * 2 + 1];
            a[c] += re * cs - im * sn;
        }
    }
}

void orc_ou_update(int32_t nmodes, const int32_t *nvec, double *theta, const double *z,
                   double f, double sigma, double a0, double kmin, double kmax, double *ahat)
{
    double kc = 0.5 * (kmin + kmax), hw = 0.5 * (kmax - kmin);
    for (int m = 0; m < nmodes; m++) {
        /* OU step on the six real components of the complex vector amplitude */
        for (int j = 0; j < 6; j++)
            theta[6 * m + j] = f * theta[6 * m + j] + sigma * sqrt(1.0 - f * f) * z[6 * m + j];
        const int32_t *nv = nvec + 3 * m;
        double kk = (double)nv[0] * nv[0] + (double)nv[1] * nv[1] + (double)nv[2] * nv[2];
        double kn = sqrt(kk);
        double amp = 1.0 - ((kn - kc) / hw) * ((kn - kc) / hw);
        if (amp < 0.0) amp = 0.0;
        /* Helmholtz projection (delta_ij - k_i k_j / |k|^2) on real and imaginary parts */
        for (int part = 0; part < 2; part++) {
            double t[3], out[3];
            for (int c = 0; c < 3; c++) t[c] = theta[6 * m + 2 * c + part];
            for (int i = 0; i < 3; i++) {
                out[i] = t[i];
                for (int j = 0; j < 3; j++) out[i] -= nv[i] * (double)nv[j] / kk * t[j];
            }
            for (int c = 0; c < 3; c++) ahat[6 * m + 2 * c + part] = a0 * amp * out[c];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Sec. 2.3: R(y)                                                      */
/* ------------------------------------------------------------------ */

static inline size_t cell_index(const orc_cfg *c, long ix, long iy, long iz)
{
    long nx = c->n[0], ny = c->n[1], nz = c->n[2];
    ix = ((ix % nx) + nx) % nx;
    iy = ((iy % ny) + ny) % ny;
    iz = ((iz % nz) + nz) % nz;
    return ((size_t)iz * ny + iy) * nx + ix;
}

static void eval_at(const double *y, size_t nc, size_t K, int N, const double *phi, double q[5])
{
    for (int i = 0; i < NF; i++) {
        double s = 0.0;
        for (int l = 0; l < N; l++) s += y[((size_t)i * N + l) * nc + K] * phi[l];
        q[i] = s;
    }
}

/* R of one cell K: out[i][l].  The numerical flux of a face is a function of
 * the two traces only, evaluated in the +axis orientation (left = the cell on
 * the -axis side), so the two cells sharing a face receive the same value. */
static void cell_rhs(const orc_cfg *cfg, const tables *t, const double *y, size_t K, const orc_forcing *frc,
                     double out[NF][NMAX])
{
    const int N = t->N, Q = t->Q, P = t->P, n = t->n;
    const size_t nc = ncells_of(cfg);
    const double g = cfg->gamma;
    double dx[3], s[3];
    for (int a = 0; a < 3; a++) {
        dx[a] = cfg->box[a] / cfg->n[a];
        s[a] = 1.0 / (4.0 * dx[a]); /* (dx^2/4) / |K| of eqs. dg:eqn:volume_int and dg:eqn:surface_int */
    }
    long ix = K % cfg->n[0], iy = (K / cfg->n[0]) % cfg->n[1], iz = K / ((size_t)cfg->n[0] * cfg->n[1]);
    double vol[NF][NMAX], surf[NF][NMAX], src[NF][NMAX];
    memset(vol, 0, sizeof vol);
    memset(surf, 0, sizeof surf);
    memset(src, 0, sizeof src);
    /* volume integral, eq. dg:eqn:volume_int */
    for (int q = 0; q < Q; q++) {
        double qv[5];
        eval_at(y, nc, K, N, t->phi_v + q * N, qv);
        for (int al = 0; al < 3; al++) {
            double F[5];
            orc_euler_flux(qv, al, g, F);
            for (int i = 0; i < NF; i++)
                for (int l = 0; l < N; l++) vol[i][l] += s[al] * F[i] * t->dphi_v[(al * Q + q) * N + l] * t->w_v[q];
        }
        if (frc) {
            /* driving source, Sec. 3.1: (0, rho a, m.a) projected with the volume rule */
            int a = q % n, b = (q / n) % n, c = q / (n * n);
            double xq[3] = {(ix + 0.5 * (1.0 + t->xg[a])) * dx[0], (iy + 0.5 * (1.0 + t->xg[b])) * dx[1],
                            (iz + 0.5 * (1.0 + t->xg[c])) * dx[2]};
            double acc[3];
            orc_accel(frc, cfg->box, xq, acc);
            double S[5] = {0.0, qv[0] * acc[0], qv[0] * acc[1], qv[0] * acc[2],
                           qv[1] * acc[0] + qv[2] * acc[1] + qv[3] * acc[2]};
            for (int i = 0; i < NF; i++)
                for (int l = 0; l < N; l++) src[i][l] += S[i] * t->phi_v[q * N + l] * t->w_v[q] / 8.0;
        }
    }
    /* surface integral, eq. dg:eqn:surface_int, outward normal */
    for (int axis = 0; axis < 3; axis++) {
        size_t Km = cell_index(cfg, ix - (axis == 0), iy - (axis == 1), iz - (axis == 2));
        size_t Kp = cell_index(cfg, ix + (axis == 0), iy + (axis == 1), iz + (axis == 2));
        for (int p = 0; p < P; p++) {
            const double *php = t->phi_f + ((axis * 2 + 1) * P + p) * N;
            const double *phm = t->phi_f + ((axis * 2 + 0) * P + p) * N;
            double qa[5], qb[5], Fp[5], Fm[5];
            eval_at(y, nc, K, N, php, qa);  /* my trace on the + face */
            eval_at(y, nc, Kp, N, phm, qb); /* right neighbour's trace on its - face */
            face_flux(cfg, qa, qb, axis, Fp);
            eval_at(y, nc, Km, N, php, qa); /* left neighbour's trace on its + face */
            eval_at(y, nc, K, N, phm, qb);  /* my trace on the - face */
            face_flux(cfg, qa, qb, axis, Fm);
            for (int i = 0; i < NF; i++)
                for (int l = 0; l < N; l++) surf[i][l] += s[axis] * (Fp[i] * php[l] - Fm[i] * phm[l]) * t->w_f[p];
        }
    }
    for (int i = 0; i < NF; i++)
        for (int l = 0; l < N; l++) out[i][l] = surf[i][l] - vol[i][l] - src[i][l];
}

void orc_rhs(const orc_cfg *cfg, const double *y, const orc_forcing *frc, double *r)
{
    tables t;
    tables_init(&t, cfg->k);
    const size_t nc = ncells_of(cfg);
    const int N = t.N;
#pragma omp parallel for schedule(static)
    for (size_t K = 0; K < nc; K++) {
        double o[NF][NMAX];
        cell_rhs(cfg, &t, y, K, frc, o);
        for (int i = 0; i < NF; i++)
            for (int l = 0; l < N; l++) r[((size_t)i * N + l) * nc + K] = o[i][l];
    }
    tables_free(&t);
}

void orc_rhs_cells(const orc_cfg *cfg, const double *y, const orc_forcing *frc, int64_t ncells_list,
                   const int64_t *cells, double *r)
{
    tables t;
    tables_init(&t, cfg->k);
    const int N = t.N;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < ncells_list; j++) {
        double o[NF][NMAX];
        cell_rhs(cfg, &t, y, (size_t)cells[j], frc, o);
        for (int i = 0; i < NF; i++)
            for (int l = 0; l < N; l++) r[((size_t)j * NF + i) * N + l] = o[i][l];
    }
    tables_free(&t);
}

/* ------------------------------------------------------------------ */
/* Sec. 2.4: time step                                                 */
/* ------------------------------------------------------------------ */

double orc_dt(const orc_cfg *cfg, const double *y)
{
    int N = orc_nmodes(cfg->k);
    size_t nc = ncells_of(cfg);
    double dx[3];
    for (int a = 0; a < 3; a++) dx[a] = cfg->box[a] / cfg->n[a];
    double rmax = 0.0;
#pragma omp parallel for reduction(max : rmax) schedule(static)
    for (size_t K = 0; K < nc; K++) {
        double q[5];
        for (int i = 0; i < NF; i++) q[i] = y[((size_t)i * N + 0) * nc + K];
        double p = pressure(q, cfg->gamma);
        double c = sqrt(cfg->gamma * p / q[0]);
        double rate = 0.0;
        for (int a = 0; a < 3; a++) rate += (fabs(q[1 + a] / q[0]) + c) / dx[a];
        if (rate > rmax) rmax = rate;
    }
    return cfg->cfl / (2.0 * cfg->k + 1.0) / rmax;
}

/* ------------------------------------------------------------------ */
/* Sec. 2.3: SSP-RK3                                                   */
/* ------------------------------------------------------------------ */

void orc_stage(const orc_cfg *cfg, const double *y0, const double *yin, double a, double b,
               double dt, const orc_forcing *frc, double *out)
{
    size_t ns = (size_t)NF * orc_nmodes(cfg->k) * ncells_of(cfg);
    double *r = malloc(sizeof(double) * ns);
    orc_rhs(cfg, yin, frc, r);
#pragma omp parallel for schedule(static)
    for (size_t j = 0; j < ns; j++) out[j] = a * y0[j] + b * (yin[j] - dt * r[j]);
    free(r);
}

void orc_step(const orc_cfg *cfg, double *y, double dt, int nsteps, double *t, const orc_forcing *frc)
{
    size_t ns = (size_t)NF * orc_nmodes(cfg->k) * ncells_of(cfg);
    double *y1 = malloc(sizeof(double) * ns), *y2 = malloc(sizeof(double) * ns);
    for (int it = 0; it < nsteps; it++) {
        double h = dt > 0.0 ? dt : orc_dt(cfg, y);
        orc_stage(cfg, y, y, 0.0, 1.0, h, frc, y1);             /* y1 = y0 - dt R(y0) */
        orc_stage(cfg, y, y1, 0.75, 0.25, h, frc, y2);          /* y2 = 3/4 y0 + 1/4 (y1 - dt R(y1)) */
        orc_stage(cfg, y, y2, 1.0 / 3.0, 2.0 / 3.0, h, frc, y); /* y3 = 1/3 y0 + 2/3 (y2 - dt R(y2)) */
        if (t) *t += h;
    }
    free(y1);
    free(y2);
}

/* ------------------------------------------------------------------ */
/* conserved totals                                                    */
/* ------------------------------------------------------------------ */

static double pairwise_sum(const double *a, size_t n)
{
    if (n <= 8) {
        double s = 0.0;
        for (size_t i = 0; i < n; i++) s += a[i];
        return s;
    }
    size_t h = n / 2;
    return pairwise_sum(a, h) + pairwise_sum(a + h, n - h);
}

void orc_totals(const orc_cfg *cfg, const double *y, double out[5])
{
    int N = orc_nmodes(cfg->k);
    size_t nc = ncells_of(cfg);
    double vol = (cfg->box[0] / cfg->n[0]) * (cfg->box[1] / cfg->n[1]) * (cfg->box[2] / cfg->n[2]);
    for (int i = 0; i < NF; i++) out[i] = vol * pairwise_sum(y + (size_t)i * N * nc, nc);
}

/* ------------------------------------------------------------------ */
/* closure support: restriction and a textbook tanh MLP                */
/* ------------------------------------------------------------------ */

void orc_restrict(int kf, int kc, const int32_t nc3[3], const double *yf, double *yc)
{
    /* w^C_l = (1/|C|) int_C q_f phi^C_l dV, integrated child by child with a
     * Gauss rule exact for degree kf + kc */
    int Nf = orc_nmodes(kf), Nc = orc_nmodes(kc);
    int m = (kf + kc) / 2 + 1;
    double xg[GMAX], wg[GMAX];
    orc_gauss_legendre(m, xg, wg);
    long NX = nc3[0], NY = nc3[1], NZ = nc3[2];
    size_t ncc = (size_t)NX * NY * NZ, ncf = ncc * 8;
    long FX = 2 * NX, FY = 2 * NY;
#pragma omp parallel for schedule(static)
    for (size_t C = 0; C < ncc; C++) {
        long X = C % NX, Y = (C / NX) % NY, Z = C / ((size_t)NX * NY);
        double acc[NF][NMAX];
        memset(acc, 0, sizeof acc);
        for (int ch = 0; ch < 8; ch++) {
            int dxo = ch & 1, dyo = (ch >> 1) & 1, dzo = ch >> 2;
            size_t Kf = ((size_t)(2 * Z + dzo) * FY + (2 * Y + dyo)) * FX + (2 * X + dxo);
            for (int c = 0; c < m; c++)
                for (int b = 0; b < m; b++)
                    for (int a = 0; a < m; a++) {
                        double xf[3] = {xg[a], xg[b], xg[c]};
                        double xcrs[3] = {-0.5 + dxo + 0.5 * xg[a], -0.5 + dyo + 0.5 * xg[b], -0.5 + dzo + 0.5 * xg[c]};
                        double phf[NMAX], phc[NMAX], q[5];
                        orc_basis(kf, xf, phf);
                        orc_basis(kc, xcrs, phc);
                        eval_at(yf, ncf, Kf, Nf, phf, q);
                        double w = wg[a] * wg[b] * wg[c] / 64.0;
                        for (int i = 0; i < NF; i++)
                            for (int l = 0; l < Nc; l++) acc[i][l] += q[i] * phc[l] * w;
                    }
        }
        for (int i = 0; i < NF; i++)
            for (int l = 0; l < Nc; l++) yc[((size_t)i * Nc + l) * ncc + C] = acc[i][l];
    }
}

/* parameter layout: W1[nh1][nin] b1[nh1] W2[nh2][nh1] b2[nh2] W3[nout][nh2] b3[nout] */
void orc_mlp_forward(int nin, int nh1, int nh2, int nout, const double *params, int batch,
                     const double *x, double *h1, double *h2, double *yout)
{
    const double *W1 = params, *b1 = W1 + (size_t)nh1 * nin;
    const double *W2 = b1 + nh1, *b2 = W2 + (size_t)nh2 * nh1;
    const double *W3 = b2 + nh2, *b3 = W3 + (size_t)nout * nh2;
#pragma omp parallel for schedule(static)
    for (int s = 0; s < batch; s++) {
        const double *xs = x + (size_t)s * nin;
        double *a1 = h1 + (size_t)s * nh1, *a2 = h2 + (size_t)s * nh2, *ys = yout + (size_t)s * nout;
        for (int j = 0; j < nh1; j++) {
            double z = b1[j];
            for (int i = 0; i < nin; i++) z += W1[(size_t)j * nin + i] * xs[i];
            a1[j] = tanh(z);
        }
        for (int j = 0; j < nh2; j++) {
            double z = b2[j];
            for (int i = 0; i < nh1; i++) z += W2[(size_t)j * nh1 + i] * a1[i];
            a2[j] = tanh(z);
        }
        for (int j = 0; j < nout; j++) {
            double z = b3[j];
            for (int i = 0; i < nh2; i++) z += W3[(size_t)j * nh2 + i] * a2[i];
            ys[j] = z;
        }
    }
}

/* loss = mean over batch and outputs of (y - target)^2; grad has the params layout */
double orc_mlp_loss_grad(int nin, int nh1, int nh2, int nout, const double *params, int batch,
                         const double *x, const double *target, double *grad)
{
    size_t np = (size_t)nh1 * nin + nh1 + (size_t)nh2 * nh1 + nh2 + (size_t)nout * nh2 + nout;
    const double *W2 = params + (size_t)nh1 * nin + nh1;
    const double *W3 = W2 + (size_t)nh2 * nh1 + nh2;
    double *h1 = malloc(sizeof(double) * batch * nh1), *h2 = malloc(sizeof(double) * batch * nh2);
    double *yo = malloc(sizeof(double) * batch * nout);
    orc_mlp_forward(nin, nh1, nh2, nout, params, batch, x, h1, h2, yo);
    memset(grad, 0, sizeof(double) * np);
    double *gW1 = grad, *gb1 = gW1 + (size_t)nh1 * nin, *gW2 = gb1 + nh1, *gb2 = gW2 + (size_t)nh2 * nh1;
    double *gW3 = gb2 + nh2, *gb3 = gW3 + (size_t)nout * nh2;
    double loss = 0.0, scale = 2.0 / ((double)batch * nout);
    double d3[64], d2[512], d1[512];
    for (int s = 0; s < batch; s++) {
        const double *xs = x + (size_t)s * nin, *a1 = h1 + (size_t)s * nh1, *a2 = h2 + (size_t)s * nh2;
        for (int j = 0; j < nout; j++) {
            double e = yo[(size_t)s * nout + j] - target[(size_t)s * nout + j];
            loss += e * e;
            d3[j] = scale * e;
        }
        for (int i = 0; i < nh2; i++) {
            double acc = 0.0;
            for (int j = 0; j < nout; j++) acc += W3[(size_t)j * nh2 + i] * d3[j];
            d2[i] = acc * (1.0 - a2[i] * a2[i]);
        }
        for (int i = 0; i < nh1; i++) {
            double acc = 0.0;
            for (int j = 0; j < nh2; j++) acc += W2[(size_t)j * nh1 + i] * d2[j];
            d1[i] = acc * (1.0 - a1[i] * a1[i]);
        }
        for (int j = 0; j < nout; j++) {
            gb3[j] += d3[j];
            for (int i = 0; i < nh2; i++) gW3[(size_t)j * nh2 + i] += d3[j] * a2[i];
        }
        for (int j = 0; j < nh2; j++) {
            gb2[j] += d2[j];
            for (int i = 0; i < nh1; i++) gW2[(size_t)j * nh1 + i] += d2[j] * a1[i];
        }
        for (int j = 0; j < nh1; j++) {
            gb1[j] += d1[j];
            for (int i = 0; i < nin; i++) gW1[(size_t)j * nin + i] += d1[j] * xs[i];
        }
    }
    free(h1);
    free(h2);
    free(yo);
    return loss / ((double)batch * nout);
}

void orc_adam(int nparams, double *params, const double *grad, double *m, double *v, int step,
              double lr, double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, step), c2 = 1.0 - pow(beta2, step);
    for (int j = 0; j < nparams; j++) {
        m[j] = beta1 * m[j] + (1.0 - beta1) * grad[j];
        v[j] = beta2 * v[j] + (1.0 - beta2) * grad[j] * grad[j];
        double mh = m[j] / c1, vh = v[j] / c2;
        params[j] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------ */
/* Learned closure (not in the paper): features and correction          */
/* ------------------------------------------------------------------ */

/* the seven cells whose weights form a cell's features: itself, then its
 * -x, +x, -y, +y, -z, +z neighbours (periodic) */
static const int nb_off[7][3] = {{0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};

void orc_closure_features(const orc_cfg *cfg, const double *y, double *feat)
{
    int N = orc_nmodes(cfg->k);
    size_t nc = ncells_of(cfg);
    long nx = cfg->n[0], ny = cfg->n[1];
    int nin = 7 * NF * N;
#pragma omp parallel for schedule(static)
    for (size_t K = 0; K < nc; K++) {
        long ix = K % nx, iy = (K / nx) % ny, iz = K / ((size_t)nx * ny);
        for (int j = 0; j < 7; j++) {
            size_t Kn = cell_index(cfg, ix + nb_off[j][0], iy + nb_off[j][1], iz + nb_off[j][2]);
            for (int i = 0; i < NF; i++)
                for (int l = 0; l < N; l++)
                    feat[K * nin + (size_t)(j * NF + i) * N + l] = y[((size_t)i * N + l) * nc + Kn];
        }
    }
}

int64_t orc_closure_correction(const orc_cfg *cfg, const double *y, const orc_closure *clo, double *corr)
{
    int N = orc_nmodes(cfg->k);
    size_t nc = ncells_of(cfg);
    int nin = clo->nin, nh1 = clo->nh1, nh2 = clo->nh2, nout = clo->nout;
    double *feat = malloc(sizeof(double) * nc * nin);
    double *h1 = malloc(sizeof(double) * nc * nh1), *h2 = malloc(sizeof(double) * nc * nh2);
    double *o = malloc(sizeof(double) * nc * nout);
    orc_closure_features(cfg, y, feat);
    /* standardised features, then the network */
    for (size_t K = 0; K < nc; K++)
        for (int f = 0; f < nin; f++)
            feat[K * nin + f] = (feat[K * nin + f] - clo->feat_mean[f]) / clo->feat_std[f];
    orc_mlp_forward(nin, nh1, nh2, nout, clo->params, (int)nc, feat, h1, h2, o);
    /* correction = scale * output, or nothing for a cell with any output
     * non-finite or beyond its bound (the plain operator is kept there) */
    int64_t fallbacks = 0;
    for (size_t K = 0; K < nc; K++) {
        int bad = 0;
        for (int j = 0; j < nout; j++) {
            double v = o[K * nout + j];
            if (!isfinite(v) || fabs(v) > clo->out_bound[j]) bad = 1;
        }
        fallbacks += bad;
        for (int i = 0; i < NF; i++)
            for (int l = 0; l < N; l++) {
                int j = i * N + l;
                corr[((size_t)i * N + l) * nc + K] = bad ? 0.0 : clo->out_scale[j] * o[K * nout + j];
            }
    }
    /* the cell-mean rows are shifted to zero sum per field, so the closure
     * leaves the conserved totals unchanged */
    for (int i = 0; i < NF; i++) {
        double *row = corr + (size_t)i * N * nc;
        double s = pairwise_sum(row, nc) / (double)nc;
        for (size_t K = 0; K < nc; K++) row[K] -= s;
    }
    free(feat);
    free(h1);
    free(h2);
    free(o);
    return fallbacks;
}

/* ------------------------------------------------------------------ */
/* Sec. 2.5: positivity limiter                                         */
/* ------------------------------------------------------------------ */

/* m GLL nodes per axis, the fewest whose rule is exact for degree k (2m - 3 >= k): the paper's
 * first weights are 1 (m = 2) for second order and 1/3 (m = 3) for third and fourth order; k = 4
 * takes m = 4 by the same exactness condition */
int orc_limiter_m(int k) { return k <= 1 ? 2 : (k <= 3 ? 3 : 4); }

void orc_gll(int m, double *x, double *w)
{
    /* Gauss-Lobatto-Legendre rules with 2, 3 and 4 points on [-1, 1] (closed forms; the
     * interior nodes of the 4-point rule are the roots of P_3'(x) = (15 x^2 - 3) / 2) */
    if (m == 2) {
        x[0] = -1.0; x[1] = 1.0;
        w[0] = 1.0; w[1] = 1.0;
    } else if (m == 4) {
        const double a = 1.0 / sqrt(5.0);
        x[0] = -1.0; x[1] = -a; x[2] = a; x[3] = 1.0;
        w[0] = 1.0 / 6.0; w[1] = 5.0 / 6.0; w[2] = 5.0 / 6.0; w[3] = 1.0 / 6.0;
    } else {
        x[0] = -1.0; x[1] = 0.0; x[2] = 1.0;
        w[0] = 1.0 / 3.0; w[1] = 4.0 / 3.0; w[2] = 1.0 / 3.0;
    }
}

/* the points of S = S_x u S_y u S_z: along one axis the m GLL nodes, along the
 * other two the k+1 Gauss nodes; returns the count, fills pts[count][3] */
int orc_limiter_points(int k, double *pts)
{
    int n = k + 1, m = orc_limiter_m(k), c = 0;
    double xg[GMAX], wg[GMAX], xl[4], wl[4];
    orc_gauss_legendre(n, xg, wg);
    orc_gll(m, xl, wl);
    for (int a = 0; a < 3; a++)
        for (int r = 0; r < m; r++)
            for (int s = 0; s < n; s++)
                for (int t = 0; t < n; t++) {
                    double *p = pts + 3 * c++;
                    int o1 = a == 0 ? 1 : 0, o2 = a == 2 ? 1 : 2;
                    p[a] = xl[r];
                    p[o1] = xg[s];
                    p[o2] = xg[t];
                }
    return c;
}

/* the unique root in (0, 1) of P(qbar + tau (q - qbar)) = eps, where P is concave
 * along the segment, positive above eps at tau = 0 and below it at tau = 1;
 * bisection to the end of double precision.  A mean already at or below eps
 * gives 0. */
static double tau_root(const double qbar[5], const double q[5], double gamma, double eps)
{
    double lo = 0.0, hi = 1.0, s[5];
    if (!(pressure(qbar, gamma) > eps)) return 0.0;
    for (int it = 0; it < 200; it++) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        for (int i = 0; i < NF; i++) s[i] = qbar[i] + mid * (q[i] - qbar[i]);
        if (s[0] > 0.0 && pressure(s, gamma) >= eps) lo = mid;
        else hi = mid;
    }
    return lo;
}

void orc_limit(const orc_cfg *cfg, double *y, double eps, double rel, double *theta)
{
    int k = cfg->k, N = orc_nmodes(k);
    size_t nc = ncells_of(cfg);
    double pts[3 * 3 * 4 * GMAX * GMAX];
    int np = orc_limiter_points(k, pts);
    double *phi = malloc(sizeof(double) * np * N);
    for (int p = 0; p < np; p++) orc_basis(k, pts + 3 * p, phi + (size_t)p * N);
#pragma omp parallel for schedule(static)
    for (size_t K = 0; K < nc; K++) {
        double w[NF][NMAX];
        for (int i = 0; i < NF; i++)
            for (int l = 0; l < N; l++) w[i][l] = y[((size_t)i * N + l) * nc + K];
        /* density: theta_1 from the minimum over S */
        double rmin = w[0][0];
        for (int p = 0; p < np; p++) {
            double r = 0.0;
            for (int l = 0; l < N; l++) r += w[0][l] * phi[(size_t)p * N + l];
            if (r < rmin) rmin = r;
        }
        double rbar = w[0][0];
        /* targets: eps, raised to rel times the cell's mean density / (gamma-1) times its mean
         * energy for storage whose rounding would otherwise undo the limiting */
        double eps_r = fmax(eps, rel * rbar), eps_p = fmax(eps, rel * (cfg->gamma - 1.0) * w[4][0]);
        double th1 = rbar == rmin ? 1.0 : fmin(fabs((rbar - eps_r) / (rbar - rmin)), 1.0);
        for (int l = 1; l < N; l++) w[0][l] *= th1;
        /* pressure: theta_2 = min over S of tau */
        double qbar[5], th2 = 1.0;
        for (int i = 0; i < NF; i++) qbar[i] = w[i][0];
        for (int p = 0; p < np; p++) {
            double q[5];
            for (int i = 0; i < NF; i++) {
                double s = 0.0;
                for (int l = 0; l < N; l++) s += w[i][l] * phi[(size_t)p * N + l];
                q[i] = s;
            }
            if (!(q[0] > 0.0 && pressure(q, cfg->gamma) >= eps_p)) {
                double t = tau_root(qbar, q, cfg->gamma, eps_p);
                if (t < th2) th2 = t;
            }
        }
        for (int i = 0; i < NF; i++)
            for (int l = 1; l < N; l++) w[i][l] *= th2;
        for (int i = 0; i < NF; i++)
            for (int l = 0; l < N; l++) y[((size_t)i * N + l) * nc + K] = w[i][l];
        if (theta) {
            theta[2 * K] = th1;
            theta[2 * K + 1] = th2;
        }
    }
    free(phi);
}

double orc_dt_limited(const orc_cfg *cfg, const double *y)
{
    double xl[4], wl[4];
    orc_gll(orc_limiter_m(cfg->k), xl, wl);
    double f = fmin(1.0 / (2.0 * cfg->k + 1.0), 0.5 * wl[0]);
    return orc_dt(cfg, y) * (2.0 * cfg->k + 1.0) * f;
}

void orc_step_limited(const orc_cfg *cfg, double *y, double dt, int nsteps, double *t, const orc_forcing *frc,
                      double eps)
{
    size_t ns = (size_t)NF * orc_nmodes(cfg->k) * ncells_of(cfg);
    double *y1 = malloc(sizeof(double) * ns), *y2 = malloc(sizeof(double) * ns);
    for (int it = 0; it < nsteps; it++) {
        orc_limit(cfg, y, eps, 0.0, NULL);  /* the stage input of stage 1 is y^n itself */
        double h = dt > 0.0 ? dt : orc_dt_limited(cfg, y);
        orc_stage(cfg, y, y, 0.0, 1.0, h, frc, y1);
        orc_limit(cfg, y1, eps, 0.0, NULL);
        orc_stage(cfg, y, y1, 0.75, 0.25, h, frc, y2);
        orc_limit(cfg, y2, eps, 0.0, NULL);
        orc_stage(cfg, y, y2, 1.0 / 3.0, 2.0 / 3.0, h, frc, y);
        if (t) *t += h;
    }
    free(y1);
    free(y2);
}

/* ------------------------------------------------------------------ */
/* Sec. 3.2: isothermal reset                                          */
/* ------------------------------------------------------------------ */

static double mean_internal(const double *y, int N, size_t nc, size_t K)
{
    double r = y[((size_t)0 * N) * nc + K];
    double mx = y[((size_t)1 * N) * nc + K], my = y[((size_t)2 * N) * nc + K], mz = y[((size_t)3 * N) * nc + K];
    double E = y[((size_t)4 * N) * nc + K];
    return E - 0.5 * (mx * mx + my * my + mz * mz) / r;
}

double orc_isothermal_reset(const orc_cfg *cfg, double *y, double cs, double rho0)
{
    tables t;
    tables_init(&t, cfg->k);
    size_t nc = ncells_of(cfg);
    int N = t.N, Q = t.Q;
    double vol = cfg->box[0] * cfg->box[1] * cfg->box[2] / (double)nc;
    double gm1 = cfg->gamma - 1.0;
    double *dis = malloc(sizeof(double) * nc);
#pragma omp parallel for schedule(static)
    for (size_t K = 0; K < nc; K++) {
        double before = mean_internal(y, N, nc, K);
        double e[GMAX * GMAX * GMAX];
        for (int q = 0; q < Q; q++) {
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            for (int i = 0; i < 4; i++)
                for (int l = 0; l < N; l++) v[i] += y[((size_t)i * N + l) * nc + K] * t.phi_v[q * N + l];
            double rho = v[0];
            double eps = cs * cs / gm1 * pow(rho / rho0, gm1);
            e[q] = 0.5 * (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / rho + rho * eps;
        }
        for (int l = 0; l < N; l++) {
            double s = 0.0;
            for (int q = 0; q < Q; q++) s += e[q] * t.phi_v[q * N + l] * t.w_v[q];
            y[((size_t)4 * N + l) * nc + K] = s / 8.0;
        }
        dis[K] = vol * (before - mean_internal(y, N, nc, K));
    }
    double total = 0.0;
    for (size_t K = 0; K < nc; K++) total += dis[K];
    free(dis);
    tables_free(&t);
    return total;
}

void orc_step_isothermal(const orc_cfg *cfg, double *y, double dt, int nsteps, double *t,
                         const orc_forcing *frc, double cs, double rho0, int limit, double eps,
                         double *dissipated)
{
    for (int it = 0; it < nsteps; it++) {
        if (limit)
            orc_step_limited(cfg, y, dt, 1, t, frc, eps);
        else
            orc_step(cfg, y, dt, 1, t, frc);
        double d = orc_isothermal_reset(cfg, y, cs, rho0);
        if (dissipated) *dissipated += d;
        if (limit) orc_limit(cfg, y, eps, 0.0, NULL);
    }
}
