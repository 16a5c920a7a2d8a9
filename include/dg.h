/*
 * dg.h -- C ABI of libdgmi.so, an MI355X (gfx950) implementation of the
 * modal discontinuous-Galerkin operator for the 3D ideal-gas Euler equations
 * on a periodic Cartesian mesh, and of the SSP-RK3 stages that call it, as
 * stated in Bauer et al., "Simulating Turbulence Using the Astrophysical
 * Discontinuous Galerkin Code TENET" (arXiv 1602.09079), Sec. 2 and 3.1.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * State.  A state holds the weights w_{i,l}^K of Sec. 2 (the expansion of the
 *   five conserved fields in the orthonormal scaled-Legendre basis of Sec.
 *   2.1).  Element order is y[z][y][i][l][x] with x fastest: for every row of
 *   cells (fixed y, z) the 5 N(k) rows of that row's weights form one
 *   contiguous slab.  i = 0..4 is (rho, m_x, m_y, m_z, E); l = 0..N(k)-1 runs
 *   over the modes of total degree <= k, graded by degree d = 0..k, then u
 *   descending, then v descending, w = d-u-v (k=1: (000),(100),(010),(001)).
 *   Mode 0 is the cell mean.
 *   The basis is normalised so that (1/8) int_{[-1,1]^3} phi_l phi_m = delta_lm.
 * Storage type.  double for DG_FP64, float for DG_FP32, DG_BF16 and
 *   DG_BF16X3 (the last two differ only in how the contractions run).
 * Memory.  Every void* state, point-value or output argument is DEVICE memory
 *   owned by the caller (for instance a torch tensor's data_ptr()), at least
 *   the stated number of elements, naturally aligned.  Pointers typed
 *   int32_t* / double* / float* that are not states are HOST memory and are
 *   copied before the call returns.
 * Streams.  All device work is enqueued on the HIP stream given to dg_init;
 *   calls return without waiting unless stated ("synchronises").
 * Errors.  Every call returns a dg_status; nothing aborts or throws across
 *   the ABI.  On DG_ERR_HIP or DG_ERR_ARG the message is available from
 *   dg_error_string(ctx).  Inputs are never modified on error (y in dg_step
 *   excepted).  A ctx is not thread-safe.
 */
#ifndef DG_H
#define DG_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_ctx dg_ctx;

typedef enum {
    DG_OK = 0,
    DG_ERR_ARG = 1,          /* invalid argument or configuration */
    DG_ERR_UNSUPPORTED = 2,  /* valid but not built (e.g. k outside 1..3) */
    DG_ERR_HIP = 3,          /* a HIP runtime call failed */
    DG_ERR_RANGE = 4,        /* non-physical state detected (DG_CHECK_RANGE) */
    DG_ERR_STATE = 5         /* call out of order (e.g. forcing flag without a table) */
} dg_status;

typedef enum {
    DG_FP64 = 0,    /* FP64 storage, FP64 arithmetic, FP64 MFMA contractions */
    DG_FP32 = 1,    /* FP32 storage, FP32 arithmetic, FP32 MFMA contractions */
    DG_BF16 = 2,    /* FP32 storage and pointwise arithmetic; contractions on BF16 MFMA with FP32 accumulation */
    DG_BF16X3 = 3   /* as DG_BF16, each contraction operand split into two BF16 parts (3 MFMA products) */
} dg_precision;

enum {
    DG_FORCING = 1u,      /* add the driving source term of Sec. 3.1 (needs dg_set_forcing) */
    DG_CHECK_RANGE = 4u   /* dg_step checks cell means for rho>0, p>0, finite after each step */
};

typedef struct {
    int32_t k;          /* polynomial degree; this build supports 1, 2, 3 */
    int32_t n[3];       /* cells per axis, each >= 2 */
    double box[3];      /* box lengths (> 0); cell widths are box[a]/n[a] */
    double gamma;       /* adiabatic index, > 1 */
    double cfl;         /* Courant factor C of Sec. 2.4, in (0, 1] */
    int32_t precision;  /* a dg_precision value */
    uint32_t flags;     /* DG_FORCING | DG_CHECK_RANGE */
} dg_config;

/* Validate cfg, build the quadrature/basis tables on the host (Sec. 2.1-2.2),
 * upload them and allocate the context's small device slots (dt, time,
 * partial sums).  hip_stream: a hipStream_t (NULL = default stream).
 * DG_ERR_ARG and no context for: k < 1, any n < 2, box <= 0, gamma <= 1,
 * cfl outside (0, 1], unknown precision or flags.  DG_ERR_UNSUPPORTED for k > 3
 * or a slab (5 N(k) n[0] elements) of 2 GiB or more. */
dg_status dg_init(const dg_config *cfg, void *hip_stream, dg_ctx **out);

/* Release the context and its device memory.  NULL is accepted. */
dg_status dg_destroy(dg_ctx *ctx);

/* Number of state elements: 5 * N(k) * n[0] * n[1] * n[2]. */
size_t dg_state_count(const dg_ctx *ctx);

/* Bytes of caller-provided workspace dg_step needs: two stage buffers. */
size_t dg_workspace_bytes(const dg_ctx *ctx);

/* Initial conditions by L2 projection, Sec. 2.2 (last equation):
 *   w_{i,l}^K = (1/8) sum_q q_i(x_q) phi_l(xi_q) omega_q over (k+1)^3 Gauss points.
 * qp: DEVICE, storage type, [5][c][b][a][z][y][x] point values; (a,b,c) is
 *   the Gauss index along (x,y,z) and the point of index a in cell ix sits at
 *   x = (ix + (1 + xi_a)/2) * box[0]/n[0] (xi from dg_gauss_nodes).
 * y: DEVICE, dg_state_count elements (output). */
dg_status dg_project(dg_ctx *ctx, const void *qp, void *y);

/* r = R(y), the spatial operator of eq. dg:eqn:time (dw/dt + R = 0): the
 * volume integral (eq. dg:eqn:volume_int), the HLLC surface integral
 * (eq. dg:eqn:surface_int) and, with DG_FORCING, minus the driving source
 * of Sec. 3.1, all divided by the cell volume.  y, r: DEVICE, distinct. */
dg_status dg_rhs(dg_ctx *ctx, const void *y, void *r);

/* One SSP-RK stage (Sec. 2.3):  out = a*y0 + b*(yin - dt*R(yin)).
 * dt > 0 is used as given; dt <= 0 uses the CFL time step last computed by
 * dg_step/dg_dt on the device.  out may alias y0 (not yin).  a == 0 skips y0. */
dg_status dg_stage(dg_ctx *ctx, const void *y0, const void *yin, void *out, double a, double b,
                   double dt);

/* CFL time step of Sec. 2.4 from the cell means, minimum over all cells,
 * evaluated in FP64:  dt = C/(2k+1) / max_K sum_a (|v_a| + c)/dx_a.
 * dt: HOST (output).  Synchronises the stream. */
dg_status dg_dt(dg_ctx *ctx, const void *y, double *dt);

/* nsteps SSP-RK3 steps in Shu-Osher form (Sec. 2.3) on y, in place.
 * work: DEVICE, dg_workspace_bytes bytes (holds y^(1), y^(2)).
 * dt > 0: fixed step.  dt <= 0: the CFL step of Sec. 2.4, computed on the
 * device at the start of every step (no host synchronisation per step).
 * t_inout: HOST, may be NULL; advanced by the total time stepped (with
 * dt <= 0 this synchronises once at the end of the call).
 * DG_ERR_RANGE (only with DG_CHECK_RANGE): y holds the end of the failing step. */
dg_status dg_step(dg_ctx *ctx, void *y, void *work, double dt, int32_t nsteps, double *t_inout);

/* Conserved totals sum_K |K| w_{i,0}^K for the five fields, in FP64 with a
 * fixed summation order (bitwise reproducible).  out: HOST [5].  Synchronises. */
dg_status dg_totals(dg_ctx *ctx, const void *y, double out[5]);

/* Driving acceleration of Sec. 3.1 as a Fourier sum:
 *   a_c(x) = sum_m Re( ahat[m][c] * exp(2 pi i sum_a nvec[m][a] x_a / box[a]) ).
 * nvec: HOST [nmodes][3]; ahat: HOST [nmodes][3][2] (re, im); copied.
 * 0 <= nmodes <= 256.  Takes effect for the calls enqueued after it. */
dg_status dg_set_forcing(dg_ctx *ctx, int32_t nmodes, const int32_t *nvec, const double *ahat);

/* Host-only helper (no ctx, no device): one Ornstein-Uhlenbeck update of the
 * driving amplitudes (Sec. 3.1), theta <- f theta + sigma sqrt(1-f^2) z on
 * the six real parts of every mode, followed by the solenoidal projection
 * (delta_ij - n_i n_j/|n|^2) and the paraboloid profile
 * max(0, 1 - ((|n| - (kmin+kmax)/2) / ((kmax-kmin)/2))^2) times a0.
 * theta: HOST [nmodes][3][2] in/out; z: HOST standard normals, same shape;
 * ahat: HOST output, same shape. */
dg_status dg_ou_update(int32_t nmodes, const int32_t *nvec, double *theta, const double *z, double f,
                       double sigma, double a0, double kmin, double kmax, double *ahat);

/* Host-only helpers for callers that sample fields at the Gauss points. */
int32_t dg_nmodes(int32_t k);                      /* N(k) = (k+1)(k+2)(k+3)/6, Sec. 2.1 */
dg_status dg_gauss_nodes(int32_t n, double *xi);   /* n-point Gauss-Legendre nodes on [-1,1], 1 <= n <= 5, ascending */

/* Last error message of ctx ("" if none); a static string for ctx == NULL. */
const char *dg_error_string(const dg_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
