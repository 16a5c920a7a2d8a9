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
    DG_ERR_UNSUPPORTED = 2,  /* valid but not built (e.g. k > 4) */
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
    DG_CLOSURE = 2u,      /* k = 1 only: add the learned closure correction (needs dg_set_closure) */
    DG_CHECK_RANGE = 4u,  /* dg_step checks cell means for rho>0, p>0, finite after each step */
    DG_LIMIT = 8u,        /* positivity limiter of Sec. 2.5 on every stage input (see dg_limiter_stats) */
    DG_ISOTHERMAL = 16u,  /* dg_step: isothermal reset of Sec. 3.2 after every step (needs dg_set_isothermal) */
    DG_EXACT_RIEMANN = 32u, /* face flux from the exact Riemann solver instead of HLLC (see below) */
    DG_ZHALO = 64u        /* the mesh is one z slab of a larger periodic one: halo planes (dg_set_halo) */
};

typedef struct {
    int32_t k;          /* polynomial degree 0..4: 0 first-order finite volume, 1..3 the MFMA stage kernel,
                           4 the quadrature-form kernel (FP64 and FP32 storage only) */
    int32_t n[3];       /* cells per axis, each >= 2 */
    double box[3];      /* box lengths (> 0); cell widths are box[a]/n[a] */
    double gamma;       /* adiabatic index, > 1 */
    double cfl;         /* Courant factor C of Sec. 2.4, in (0, 1] */
    int32_t precision;  /* a dg_precision value */
    uint32_t flags;     /* DG_FORCING | DG_CLOSURE | DG_CHECK_RANGE | DG_LIMIT | DG_ISOTHERMAL | DG_EXACT_RIEMANN | DG_ZHALO */
} dg_config;

/* Validate cfg, build the quadrature/basis tables on the host (Sec. 2.1-2.2),
 * upload them and allocate the context's small device slots (dt, time,
 * partial sums).  hip_stream: a hipStream_t (NULL = default stream).
 * DG_ERR_ARG and no context for: k < 0, any n < 2, box <= 0, gamma <= 1,
 * cfl outside (0, 1], unknown precision or flags.  DG_ERR_UNSUPPORTED for k > 4,
 * k = 4 with DG_BF16 or DG_BF16X3, DG_CLOSURE with k != 1, or a slab (5 N(k) n[0]
 * elements) of 2 GiB or more.  With DG_LIMIT the limiter's point set has m = 2, 3, 3, 4
 * Gauss-Lobatto nodes per axis for k = 1, 2, 3, 4 (Sec. 2.5). */
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

/* The state in the canonical order y_c[i][l][z][y][x] (field, mode, then the mesh with x fastest:
 * one contiguous plane of cells per (field, mode)), converted to (import) or from (export) the
 * order y[z][y][i][l][x] that every other entry point takes.  The internal order keeps a row's
 * 5 N(k) weight rows together for the stage kernels' loads; the canonical one is the natural
 * order of the weights w_{i,l}^K of Sec. 2.  canon, y: DEVICE, dg_state_count elements of the
 * storage type, distinct (not in place).  DG_ERR_ARG on NULL or identical pointers. */
dg_status dg_state_import(dg_ctx *ctx, const void *canon, void *y);
dg_status dg_state_export(dg_ctx *ctx, const void *y, void *canon);

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
 * 0 <= nmodes <= 256.  The field is constant until the next call (the driving
 * is piecewise constant in time), so it is evaluated here once, in FP64, at
 * every volume Gauss point of every cell, and cached on the device in the
 * storage type (3 (k+1)^3 values per cell; the first call allocates the
 * cache).  The stages read the cache.  Synchronises. */
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

/* ---------------------------------------------------------------------------
 * Learned closure (an addition to the paper's scheme, for under-resolved k = 1
 * runs).  A cell's 140 features are the weights of the cell and of its -x,
 * +x, -y, +y, -z, +z neighbours (periodic), ordered feat[j][i][l] (neighbour j,
 * field i, mode l).  A 140-128-128-20 network with tanh hidden layers maps
 * (feat - feat_mean) / feat_std to o (20 values ordered [i][l]); the
 * correction is c = out_scale * o and the scheme becomes dy/dt = -R(y) + c,
 * i.e. dg_rhs returns R - c and the stages use it.  A cell with any o_j
 * non-finite or |o_j| > out_bound_j keeps the plain operator (c = 0 for that
 * cell, counted as a fallback).  The mode-0 rows of c are then shifted by
 * their mean over the mesh, per field, so the conserved totals are unchanged.
 * Inference runs in FP32 (FP32 matrix cores) in every precision tier.
 * ------------------------------------------------------------------------- */

/* Install the network (DG_CLOSURE contexts only; DG_ERR_STATE otherwise).
 * HOST arrays, copied: params [dg_mlp_nparams({140,128,128,20})] in the layout
 * W1[128][140] b1[128] W2[128][128] b2[128] W3[20][128] b3[20]; feat_mean,
 * feat_std [140] (std > 0); out_scale, out_bound [20] (bound >= 0).  The first
 * call allocates the correction buffer (one state).  Synchronises. */
dg_status dg_set_closure(dg_ctx *ctx, const float *params, const float *feat_mean, const float *feat_std,
                         const float *out_scale, const float *out_bound);

/* Cells that fell back since the previous call (summed over every closure
 * evaluation, one per R evaluation), then reset.  count: HOST.  Synchronises. */
dg_status dg_closure_fallbacks(dg_ctx *ctx, int64_t *count);

/* Training data.  feat: DEVICE float [ncells][7][5][N] (raw, unstandardised)
 * features of state y (any k).  Cells in x-fastest order (z, y, x). */
dg_status dg_closure_features(dg_ctx *ctx, const void *y, float *feat);

/* target[cell][i][l] = r_coarse - r_fine_restricted (DEVICE float
 * [ncells][5N]); both inputs are states of ctx's shape, e.g. R_c(P y_f) and
 * P R_f(y_f), whose difference is the correction a closure should supply. */
dg_status dg_closure_targets(dg_ctx *ctx, const void *r_coarse, const void *r_fine_restricted, float *target);

/* Exact L2 restriction onto ctx's mesh and degree (the coarse side): yf is a
 * degree-kf state on the mesh with twice as many cells per axis (cell
 * (2X+dx, 2Y+dy, 2Z+dz) is a child of coarse cell (X, Y, Z)); yc = the
 * projection of the piecewise polynomial onto degree ctx.k, computed child by
 * child with a Gauss rule exact for degree kf + k.  Linear, so it also
 * restricts time derivatives.  k <= kf <= 3.  yf, yc: DEVICE, storage type of
 * ctx.  The first call per kf allocates a small table. */
dg_status dg_restrict(dg_ctx *ctx, int32_t kf, const void *yf, void *yc);

/* ---- Dense tanh networks for the closure's training (no context) --------
 * shape = {nin, nh1, nh2, nout}; params layout W1[nh1][nin] b1 W2[nh2][nh1] b2
 * W3[nout][nh2] b3 (row-major), FP32, DEVICE.  All products on the FP32 matrix
 * cores.  work: DEVICE, dg_mlp_workspace_bytes(shape, batch) bytes.
 * hip_stream: the stream all work is enqueued on (NULL = default). */
size_t dg_mlp_nparams(const int32_t shape[4]);
size_t dg_mlp_workspace_bytes(const int32_t shape[4], int32_t batch);

/* y[s][j] = network(x[rows[s]])_j for s < batch.  x: DEVICE [nsamples][nin];
 * rows: DEVICE int32 [batch] sample indices, or NULL for rows 0..batch-1;
 * y: DEVICE [batch][nout]. */
dg_status dg_mlp_forward(const int32_t shape[4], const float *params, int32_t batch, const float *x,
                         const int32_t *rows, float *y, void *work, void *hip_stream);

/* Mean-squared error over the batch and the outputs, and its gradient:
 * loss = mean_{s,j} (y_sj - target[rows[s]][j])^2; grad (DEVICE, params
 * layout) = d loss / d params, summed over the batch in a fixed order.
 * noise_std > 0 adds noise_std * N(0,1) to every input of the batch (input
 * noise for robustness), drawn from a counter-based generator keyed by seed
 * and the element's position in the batch, so a (seed, rows) pair always
 * draws the same noise.  loss: DEVICE double, or NULL. */
dg_status dg_mlp_loss_grad(const int32_t shape[4], const float *params, int32_t batch, const float *x,
                           const float *target, const int32_t *rows, float noise_std, uint64_t seed, float *grad,
                           double *loss, void *work, void *hip_stream);

/* One Adam step (Kingma and Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).  All DEVICE
 * FP32 arrays of nparams entries, updated in place; step >= 1. */
dg_status dg_adam(int64_t nparams, float *params, const float *grad, float *m, float *v, int32_t step, double lr,
                  double beta1, double beta2, double eps, void *hip_stream);

/* Column statistics of x (DEVICE float [rows][cols], cols <= 256), in FP64 with
 * a fixed summation order: mean, standard deviation about the mean, root mean
 * square about zero, max |x|.  Outputs: DEVICE double [cols] each.  work:
 * DEVICE, dg_column_stats_workspace_bytes(cols) bytes. */
size_t dg_column_stats_workspace_bytes(int32_t cols);
dg_status dg_column_stats(const float *x, int64_t rows, int32_t cols, double *mean, double *stdev, double *rms,
                          double *maxabs, void *work, void *hip_stream);

/* dg_column_stats without a workspace, for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid allocation).  The same kernels and
 * the same results, bit for bit; the partial sums live in a static device array of the library
 * (1024 x 160 x 3 doubles, 3.75 MiB per GPU, held until the process ends), found once per device
 * on its first call.  cols <= 160 (DG_ERR_ARG beyond, with the reason in dg_error_string(NULL)).
 * Allocates nothing.  Every call on one GPU uses that GPU's one array: calls that overlap on a GPU
 * (other streams, other threads) race and must be ordered by the caller.  Nothing in the array
 * needs to start at zero: each call writes every partial it reads. */
dg_status dg_column_stats_noalloc(const float *x, int64_t rows, int32_t cols, double *mean, double *stdev,
                                  double *rms, double *maxabs, void *hip_stream);

/* x[r][c] = (x[r][c] - shift[c]) / scale[c] in place.  shift, scale: DEVICE double [cols]. */
dg_status dg_standardize(float *x, int64_t rows, int32_t cols, const double *shift, const double *scale,
                         void *hip_stream);

/* ---------------------------------------------------------------------------
 * Positivity limiter (Sec. 2.5, Zhang and Shu), enabled by DG_LIMIT.
 * Applied to the input of every stage (dg_rhs, dg_stage, each stage of
 * dg_step), IN PLACE: the caller's y / yin is replaced by its limited value
 * (for dg_step: y^n before the time step is computed, then y^(1), y^(2)).
 * Points S: along one axis the m GLL nodes (m = 2 for k = 1, m = 3 for
 * k = 2, 3: -1, 0, 1; m = 4 for k = 4: -1, -1/sqrt(5), 1/sqrt(5), 1; the fewest
 * nodes whose rule is exact for degree k), along the other two the k+1 Gauss
 * nodes, for each axis.
 * Per cell, eps = 1e-13: theta_1 = min(|(rhobar - eps)/(rhobar - rho_min)|, 1)
 * scales the density's modes l >= 1; then theta_2 = min over S of tau, tau = 1
 * where P >= eps (and rho > 0), else the root in (0, 1) of
 * P(qbar + tau (q - qbar)) = eps found by Newton-Raphson, scales the modes
 * l >= 1 of every field.  Cell means are never changed.  FP32-storage tiers
 * raise the targets per cell to max(eps, 2^-20 rhobar) for the density and
 * max(eps, 2^-20 (gamma-1) Ebar) for the pressure, above the rounding of the
 * stored weights, which would otherwise undo the limiting.  With DG_LIMIT the CFL
 * step becomes C min(1/(2k+1), w_hat_1/2) / max rate, w_hat_1 the first GLL
 * weight (1 for k = 1, 1/3 for k = 2, 3, 1/6 for k = 4).  Computed in the storage
 * precision (FP32 for the FP32-storage tiers).
 *
 * Cells changed by the limiter since the previous call, then reset.
 * count: HOST.  Synchronises.  0 without DG_LIMIT. */
dg_status dg_limiter_stats(dg_ctx *ctx, int64_t *count);

/* Host-only helpers for callers that sample fields at the Gauss points. */
int32_t dg_nmodes(int32_t k);                      /* N(k) = (k+1)(k+2)(k+3)/6, Sec. 2.1 */
dg_status dg_gauss_nodes(int32_t n, double *xi);   /* n-point Gauss-Legendre nodes on [-1,1], 1 <= n <= 5, ascending */

/* Last error message of ctx ("" if none).  ctx == NULL: why the calling thread's last dg_init
 * or dg_column_stats_noalloc failed (the rejected argument, or the failing HIP call's error), or
 * a fixed message if neither has failed.  The string stays valid until the thread's next call of
 * either. */
const char *dg_error_string(const dg_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Isothermal reset and dissipation measurement (Sec. 3.2).
 * The gas is an ideal gas with gamma close to 1 (the paper: 1.01); after each
 * step the specific internal energy is reset to
 *   eps(rho) = cs^2/(gamma-1) (rho/rho0)^(gamma-1)
 * at the (k+1)^3 Gauss points of every cell, and the energy weights become
 *   w_E,l = (1/8) sum_q (|m_q|^2/(2 rho_q) + rho_q eps(rho_q)) phi_l(xi_q) omega_q
 * (rho_q, m_q from the current weights; the density and momentum weights are
 * unchanged).  The dissipated energy of a reset is
 *   sum_K |K| (rhoe_before - rhoe_after),  rhoe = w_E,0 - |w_m,0|^2/(2 w_rho,0),
 * accumulated on the device in FP64 with a fixed summation order.  The
 * arithmetic at the points runs in the storage precision.  With DG_ISOTHERMAL
 * dg_step resets after every step and then, with DG_LIMIT, applies the
 * positivity limiter to the reset state.
 *
 * Set the reset's sound speed cs and reference density rho0 (both finite and
 * > 0, else DG_ERR_ARG); allocates the partial-sum buffer on the first call. */
dg_status dg_set_isothermal(dg_ctx *ctx, double cs, double rho0);

/* One reset of y (DEVICE, in place), as dg_step does after a step; adds to the
 * dissipation account.  DG_ERR_STATE before dg_set_isothermal.  Asynchronous. */
dg_status dg_isothermal_reset(dg_ctx *ctx, void *y);

/* Dissipated energy accumulated since the previous call (0 if none), then reset.
 * out: HOST.  Synchronises. */
dg_status dg_dissipated(dg_ctx *ctx, double *out);

/* ---------------------------------------------------------------------------
 * Turbulence diagnostics (Sec. 3.3, 4.1, 4.4).  The DG polynomials are sampled
 * on a sub-cell grid: each cell is split into S equal parts per axis (the paper
 * uses S = 4) and evaluated at the part centres xi_j = -1 + (2j+1)/S, giving
 * M_a = S n[a] points per axis; grid point X sits at x = (X + 1/2) box[a]/M_a.
 * Point values are computed in the storage precision, 1 <= S <= 4 (else
 * DG_ERR_ARG).  The first call allocates a small device buffer.
 *
 * The five conserved fields on the grid.  out: DEVICE, storage type,
 * [5][M_z][M_y][M_x] (5 M_x M_y M_z elements).  Asynchronous. */
dg_status dg_sample(dg_ctx *ctx, const void *y, int32_t S, void *out);

/* Bytes of the workspace dg_velocity_spectrum needs: one real-to-complex FFT
 * buffer of M^2 * 2(M/2+1) elements of the storage type (M = S n). */
size_t dg_spectrum_workspace_bytes(const dg_ctx *ctx, int32_t S);

/* Shell power spectrum of the velocity v = m/rho (Sec. 3.3), cubic meshes only
 * (equal n and box on every axis, else DG_ERR_UNSUPPORTED):
 *   P(s) = sum_i sum_{n: nearest integer to |n| is s} |v_hat_i(n)|^2 / M^6,
 *   v_hat_i(n) = sum_X v_i(X) exp(-2 pi i n.X/M),
 * so that sum_s P(s) is the grid mean of |v|^2; E(k) = P(s) box/(2 pi) at
 * k = 2 pi s / box.  The transforms are hipFFT real-to-complex (FP32 for the
 * FP32-storage tiers, FP64 for DG_FP64; the plan is made on the first call and
 * kept); shells are summed in FP64 in a fixed order (bitwise reproducible, and a
 * shell's value does not depend on nbins).  out: HOST double [nbins], 1 <= nbins <= 4096, shells >= nbins are
 * dropped.  work: DEVICE, dg_spectrum_workspace_bytes(ctx, S).  Synchronises. */
dg_status dg_velocity_spectrum(dg_ctx *ctx, const void *y, int32_t S, int32_t nbins, double *out, void *work);

/* Density PDF (Sec. 4.4): counts of log10(rho) at the sampled points in nbins
 * equal bins of [lo, hi); counts[0]: points below lo, with rho <= 0 or not
 * finite; counts[nbins+1]: points at or above hi.  counts: HOST int64
 * [nbins + 2], 1 <= nbins <= 4096, lo < hi finite.  Exact integer counts (the
 * bin of a point is decided in the storage precision).  Synchronises. */
dg_status dg_density_pdf(dg_ctx *ctx, const void *y, int32_t S, double lo, double hi, int32_t nbins,
                         int64_t *counts);

/* rms Mach number (Sec. 4.1): sqrt of the mean over the sampled points of
 * |v|^2 / c^2, c^2 = gamma p / rho, summed in FP64 in a fixed order.
 * out: HOST.  Synchronises. */
dg_status dg_rms_mach(dg_ctx *ctx, const void *y, int32_t S, double *out);

/* ---------------------------------------------------------------------------
 * DG_EXACT_RIEMANN: the numerical flux of eq. dg:eqn:surface_int comes from the
 * exact solution of each face's Riemann problem (the alternative to HLLC that
 * Sec. 2.3 names; Toro, Riemann Solvers and Numerical Methods for Fluid
 * Dynamics, ch. 4): the star pressure from the shock / rarefaction wave curves
 * by Newton iteration from the primitive-variable estimate (one more step after
 * the first whose relative change is below 1e-8 FP64 / 1e-4 otherwise; 24 at most), the solution sampled at the face and its
 * Euler flux taken, tangential velocities from the side of the contact the face
 * lies on; vacuum-generating data are sampled from the two rarefactions.  The
 * rest of the scheme is unchanged.  Computed in the tier's pointwise precision
 * (FP32 for the FP32-storage tiers).  Costs more than HLLC (iterations,
 * divergent lanes). */

/* ---------------------------------------------------------------------------
 * One GPU's share of a mesh split into z slabs (the way the method shards:
 * every stage needs one ghost layer of the neighbouring slabs, Sec. 2.3).
 * With DG_ZHALO the stage kernels take the cells below z = 0 and above
 * z = n[2] - 1 from two halo planes instead of wrapping periodically; x and y
 * stay periodic.  A halo plane is one z plane of a state, [y][i][l][x]
 * (dg_plane_count elements of the storage type): the neighbouring slab's top
 * plane below, its bottom plane above.  Since the state is stored
 * [z][y][i][l][x], a slab's boundary plane is contiguous and is sent as is
 * (no packing).  The caller refreshes the halo planes before every stage
 * (dg_rhs, dg_stage; dg_step cannot exchange between its stages and returns
 * DG_ERR_UNSUPPORTED for a slab: drive the stages with dg_stage) and reduces
 * the CFL rate across slabs (dg_dt per slab, then the minimum).  The slab's box[2] is its own extent (the whole
 * box's times n[2] / nz_global).  DG_ZHALO with DG_CLOSURE: DG_ERR_UNSUPPORTED.
 *
 * Elements of one z plane: 5 N(k) n[0] n[1]. */
size_t dg_plane_count(const dg_ctx *ctx);

/* The halo planes (DEVICE, caller-owned, read by every later stage launch).
 * DG_ERR_STATE without DG_ZHALO; a stage without halo planes set returns
 * DG_ERR_STATE. */
dg_status dg_set_halo(dg_ctx *ctx, const void *lo, const void *hi);

/* The z-chunk length of the stage sweep of k = 1..3 (the cells along z one work item of the
 * stage kernel covers, carrying the z-face flux from cell to cell); 0 restores the length
 * dg_init chose for the device.  The result does not depend on it, bit for bit (a test checks
 * that); it exists for that check and for tuning.  DG_ERR_ARG unless 0 <= len <= n[2]. */
dg_status dg_set_zchunk(dg_ctx *ctx, int32_t len);

/* The slab's place in the whole mesh for the driving field: its first plane
 * is global plane z0 of nz_global (default 0 of n[2]).  Call before
 * dg_set_forcing.  DG_ERR_ARG unless 0 <= z0 and z0 + n[2] <= nz_global. */
dg_status dg_set_slab(dg_ctx *ctx, int32_t z0, int32_t nz_global);

#ifdef __cplusplus
}
#endif
#endif
