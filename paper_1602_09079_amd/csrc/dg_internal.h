// Internal declarations shared by the host half (dg_host.cpp) and the kernels
// (dg_kernels.hip) of libdgmi.so.  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "dg.h"

namespace dgmi {

constexpr int NF = 5;          // conserved fields
constexpr int BLK = 16;        // cells per MFMA column tile (one x-run)
constexpr int BLK_INNER = 14;  // cells of a block whose result is kept; columns 0 and 15 are x-halo
constexpr int MAX_FORCING_MODES = 256;  // accepted by dg_set_forcing


inline int nmodes_of(int k) { return (k + 1) * (k + 2) * (k + 3) / 6; }

// Row of a 16x16 MFMA output tile held by lane group g (= lane/16) in result
// register r.  FP32/BF16 accumulators: 4g + r.  FP64 (16x16x4f64): g + 4r.
inline int out_row(int prec, int g, int r) { return prec == DG_FP64 ? g + 4 * r : 4 * g + r; }

// index of mode (u, v, w) in the graded order (total degree, then u descending, then v descending)
template <int K>
__host__ __device__ constexpr int mode_of(int u, int v, int w) {
    int l = 0;
    for (int d = 0; d <= K; d++)
        for (int a = d; a >= 0; a--)
            for (int b = d - a; b >= 0; b--) {
                if (a == u && b == v && d - a - b == w) return l;
                l++;
            }
    return -1;
}
static_assert(mode_of<3>(0, 0, 0) == 0 && mode_of<3>(1, 0, 0) == 1 && mode_of<3>(0, 0, 1) == 3 &&
                  mode_of<3>(1, 1, 0) == 5 && mode_of<3>(3, 0, 0) == 10 && mode_of<3>(0, 0, 3) == 19,
              "graded mode order");

// Mode assignment shared by every product: lane group g owns the modes
// g*spl .. g*spl + spl - 1 (spl = ceil(N/4)), mode slot s = 0..spl-1.  Slot s is
// the K-step s (FP32/FP64) or value s (BF16) of the B operands of GEMM1/GEMM3,
// and the result register r of row tile rt with s = 4 rt + r of GEMM2/4/5, so
// the weights a lane loads as product inputs are the modes of the result rows
// it receives.  Returns N for an unused slot.
__host__ __device__ constexpr int mode_slots(int N) { return (N + 3) / 4; }
__host__ __device__ constexpr int slot_mode(int N, int g, int s) {
    return (s < mode_slots(N) && g * mode_slots(N) + s < N) ? g * mode_slots(N) + s : N;
}

// ---- the k = 3 stage kernel of the BF16-product tiers (stage_k3.hip): 16-cell x-blocks on
// 64-byte boundaries, every product a 16x16x32 BF16 matrix-core operation.
// Slot s (0..4) of lane group g (0..3) holds one mode, for the B operands of the products with
// the weights (contraction index 8g + s) and for the result rows (row tile s / 4, register s % 4).
// Slot 4 holds the four modes (0,0,w): their x and y derivatives vanish, so the volume product of
// the x and y fluxes needs the first row tile only.
__host__ __device__ constexpr int k3_slot_mode(int g, int s) {
    return s == 4 ? (g == 0 ? 0 : g == 1 ? 3 : g == 2 ? 9 : 19)
                  : (g == 0 ? (s == 0 ? 1 : s == 1 ? 2 : s == 2 ? 4 : 5)
                     : g == 1 ? (s == 0 ? 6 : s == 1 ? 7 : s == 2 ? 8 : 10)
                     : g == 2 ? (s == 0 ? 11 : s == 1 ? 12 : s == 2 ? 13 : 14)
                              : (s == 0 ? 15 : s == 1 ? 16 : s == 2 ? 17 : 18));
}
// A-operand fragments (64 lanes x 8 BF16 = 1 KiB each) of one table set, in this order:
// T1[t] (phi at the 16 volume points of z-node t), T3[f] (phi at the 16 points of face f),
// T2A[t] (x and y derivative tables of z-node t), T2B[t][rt] (z derivative and source tables),
// T4[a][rt] (lift of the - and + face of axis a).  BF16X3 appends the lo set.
constexpr int K3_FRAG = 1024;
constexpr int K3_T1 = 0, K3_T3 = 4, K3_T2A = 10, K3_T2B = 14, K3_T4 = 22, K3_NFRAG = 28;
constexpr int K3_SET = K3_NFRAG * K3_FRAG;
// After the LDS sets, read through the caches: the mass flux's volume term as mode-to-mode
// fragments (x, y and z derivative in the first row tile, z in the second), hi then lo set in
// BF16X3, each fragment two 1 KiB halves in FP32
constexpr int K3_NS = 4;
constexpr int K3_BLK = 16;           // cells per x-block
constexpr int K3_DKS = 2;            // K steps (of 4) of the driving product: wave numbers |n_x| <= 3
// driving factor table per (z, y) row of cells: [component][z-node][K step][lane] floats
__host__ __device__ inline long long k3_drive_row_floats(int dks) { return 3LL * 4 * dks * 64; }

// k = 4 stage kernel (stage_k4.hip): A-operand fragments of its 16x16x4 / 4x4x1 products
// (64 values each, in the storage precision), in this order: PHI[t][s] (values at the 16 points
// of volume tile t, K step s over the modes), GRAD[t][d][rt][s] (minus the weighted
// d-derivatives, result row tile rt, K step s over the tile's points), TRACE[f][ft][s] (values at
// the 16 points of face tile ft of face f), LIFT[f][rt][s] (K step s over the face's 32 rows),
// then SRC[t][rt][s] (minus the weighted basis / 8, read only with the driving).
constexpr int K4_BLK = 16;  // cells per x-block
// x-degree of mode l in the graded order of the basis (total degree d, then the x-degree
// descending, then the y-degree descending)
__host__ __device__ constexpr int graded_mode_u(int l) {
    int n = 0;
    for (int d = 0; d < 16; d++)
        for (int a = d; a >= 0; a--)
            for (int b = d - a; b >= 0; b--) {
                if (n == l) return a;
                n++;
            }
    return -1;
}
constexpr int K4_PHI = 0, K4_GRAD = K4_PHI + 8 * 9, K4_TRACE = K4_GRAD + 8 * 3 * 3 * 4, K4_LIFT = K4_TRACE + 6 * 2 * 9,
              K4_SRC = K4_LIFT + 6 * 3 * 8, K4_NFRAG = K4_SRC + 8 * 3 * 4;
// LDS of the kernel: FP32 the fragments before SRC, FP64 (8-byte values) the GRAD fragments
constexpr int k4_lds_bytes(int prec) { return prec == DG_FP64 ? (K4_TRACE - K4_GRAD) * 64 * 8 : K4_SRC * 64 * 4; }

// Stage kernel launch shape.  FP32-storage tiers: workgroups of 8 waves that own
// 8 consecutive y rows of one x-block and sweep z together, sharing y-face traces
// and fluxes through LDS.  FP64: workgroups of 4 independent waves.
constexpr int YROWS = 8;
constexpr int K3_GHOST_BYTES = YROWS * 4 * 64 * 4;  // k = 3 x-face ghost cells: 4 copies of 64 lanes per wave
inline int stage_block_threads(int prec) { return prec == DG_FP64 ? 256 : 64 * YROWS; }
inline int stage_rows_per_item(int prec) { return prec == DG_FP64 ? 1 : YROWS; }
// LDS bytes of one y-face exchange region: a slot of 5 fields x 4 values x 64 lanes per wave
inline size_t stage_exchange_bytes(int prec) { return prec == DG_FP64 ? 0 : (size_t)YROWS * NF * 4 * 64 * 4; }
// the two end rows of a workgroup's y group, prefetched into LDS: the mean and the mode slots of
// every field per lane (FP32 storage)
inline size_t stage_endrow_bytes(int prec, int k) {
    return prec == DG_FP64 ? 0 : (size_t)2 * NF * (1 + (nmodes_of(k) + 3) / 4) * 64 * 4;
}

// Geometry of the MFMA operand tables for one (k, precision).  A "fragment" is
// what the 64 lanes feed to one MFMA as its A operand.  GEMM1/3/4 use the wide
// MFMA (K = 4 for FP32/FP64, K = 32 for BF16: kpl values per lane); GEMM2/5
// (contractions over the volume points, fed straight from GEMM1's results) use
// K = 4 / K = 16 (kpl2 values per lane) so that one 16-point tile is one chunk.
struct TableLayout {
    int k, prec;
    int N, n, Q, P;
    int kpl, kpl2;   // operand values per lane: (1, 1) for FP32/FP64, (8, 4) for BF16
    int kstep;       // K extent of the wide MFMA (4 or 32)
    int ks1;         // K steps over the modes
    int rt1;         // volume-point row tiles, ceil(Q/16)
    int rt2;         // mode row tiles of the result, ceil(N/16)
    int nc2;         // chunks over the volume points: rt1*4 (kpl2 = 1) or rt1 (kpl2 = 4)
    int nc4;         // chunks over the six faces: 24 (kpl = 1) or 3 (kpl = 8)
    size_t elem;     // bytes per table element
    size_t fb1, fb2; // bytes per fragment of the wide / narrow tables
    size_t o1, o2, o3, o4, o5, set_bytes;  // byte offsets of the five tables in one set
    int ntab;        // 1, or 2 for split (hi, lo) BF16 tables (the lo set follows)
    size_t bytes() const { return set_bytes * ntab; }
};

TableLayout make_layout(int k, int prec);
struct GaussNodes {
    double x[5];
};
// elements of the driving acceleration cache per (z, y) row of cells: 3 components x 16 ceil(Q/16) points x nx
inline long long accel_slab_elems(int k, int nx) {
    if (k == 0) return 3LL * nx;  // k = 0: [component][x], the cell centre only
    const int Q = (k + 1) * (k + 1) * (k + 1);
    return (long long)((Q + 15) / 16) * 16 * 3 * nx;
}
constexpr double LIMIT_EPS = 1e-13;  // minimum density and pressure of the positivity limiter
// FP32 storage: the targets are raised to 2^-20 times the cell's mean density / (gamma-1) x mean energy
constexpr double LIMIT_REL_FP32 = 1.0 / 1048576.0;
hipError_t launch_limit(int k, int prec, void *y, const double *tab, int np, long long nc, int nx, double gamma,
                        double eps, unsigned long long *count, hipStream_t s);
// isothermal reset of Sec. 3.2: energy weights re-projected in place; the dissipated energy
// (FP64, fixed order) is added to *acc.  partials: reset_partials(nc) doubles.
struct Leg1D {
    double p[5][5];  // p[u][a]: scaled Legendre polynomial of degree u at Gauss node a (k+1 nodes)
    double w[5];     // Gauss weights
};
long long reset_partials(long long nc);

// ---- turbulence diagnostics (Sec. 3.3, 4.1, 4.4) on the S^3 sub-cell grid
constexpr int DIAG_MAX_S = 4;        // sub-cell points per axis
constexpr int DIAG_MAX_BINS = 4096;  // spectrum shells / PDF bins
struct SampleArgs {
    const void *y;
    long long nc;
    int nx, ny;
    int what;             // 0: the five conserved fields; 1..3: velocity component what-1; 4: statistics
    void *out;            // grid (what 0..3): [field][Z][Y][X] with the pitches below
    long long px, py, pf; // row, plane and field pitches of out, in elements
    double gamma;
    double lo, hi;        // PDF range of log10(rho); nbins > 0 enables the PDF
    int nbins;
    unsigned long long *counts;  // [nbins + 2]
    double *mach_partials;       // per block sum of |v|^2/c^2 over the block's points, or nullptr
};
long long sample_blocks(long long nc);
hipError_t launch_sample(int k, int S, int prec, const SampleArgs &a, const Leg1D &L, hipStream_t s);
// bins[s] += scale * weight * |c|^2 over an R2C spectrum [M][M][M/2+1] (interleaved complex)
hipError_t launch_shells(int prec, const void *spec, int M, int nbins, double scale, double *bins, hipStream_t s);
hipError_t launch_fill_zero(unsigned long long *p, long long n, hipStream_t s);
hipError_t launch_sum_into(const double *p, long long n, double *acc, hipStream_t s);
hipError_t launch_reset(int k, int prec, void *y, const Leg1D &L, long long nc, int nx, double gm1, double ce,
                        double rho0, double vol, double *partials, double *acc, hipStream_t s);
hipError_t launch_accel_cache(int k, int prec, const double *modes, int nmodes, int nx, int ny, int nz, long long nc,
                              const GaussNodes &xg, int z0, int nzg, void *out, hipStream_t s);

struct StageArgs {
    const void *yin;
    const void *y0;
    void *out;
    const void *tables;   // device copy of the fragment tables (staged into LDS by each workgroup)
    const double *rate;   // device max CFL rate slot, or nullptr to use dt
    double *tacc;         // device time accumulator, advanced by dt when non-null
    double dt, a, b;
    double dtfac;         // C / (2k+1)
    double gamma;
    int nx, ny, nz;
    int nbx;              // x-blocks per row
    int zlen;             // cells per z chunk swept by one wave
    long long nitems;     // work items: nbx * ceil(ny / rows per item) * ceil(nz / zlen)
    int ex_off;           // LDS byte offset of the y-face trace slots
    int ex_off2;          // LDS byte offset of the y-face flux slots (== ex_off: shared, ex_single = 1)
    int ex_single;
    int ex_off3;          // LDS byte offset of the end-row buffers, or -1 when they do not fit
    int ex_off4;          // k = 3 BF16 tiers: LDS byte offset of the x-face ghost-cell copies
    long long ncells;
    int mode;             // 0: out = R(yin); 1: out = a*y0 + b*(yin - dt*R(yin))
    int forcing;          // 1: add the driving source
    const void *acache;   // driving acceleration at the volume points (layout of accel_load)
    double h[3];          // cell widths
    const void *corr;     // closure correction c (state layout) or nullptr: R <- R - (c - cmean on mode 0)
    const double *cmean;  // [5] mean of c's mode-0 rows per field
    int riemann;          // face flux: 0 HLLC, 1 exact Riemann solver
    const void *halo_lo;  // z slab: the plane below z = 0 and the plane above z = nz - 1 ([y][i][l][x]),
    const void *halo_hi;  // or nullptr (periodic in z)
    // k = 3 BF16-tier kernel: the driving as a product (per-row factor table, per-x phases)
    const float *dtab;    // [z][y] rows of k3_drive_row_floats(dks)
    const float *dcs;     // [x][dks][4]: cos / sin of the x phases of the wave numbers n_x
    int dks;              // K steps (of 4) of the driving product
};

hipError_t launch_stage(int k, int prec, const StageArgs &a, int grid, int lds_bytes, hipStream_t s);
hipError_t launch_relayout(int prec, const void *src, void *dst, int nfm, int nx, int ny, int nz, int to_canonical,
                           hipStream_t s);
hipError_t set_stage_attributes(int k, int prec, int lds_bytes);
// the k = 3 BF16-tier kernel (stage_k3.hip)
hipError_t launch_stage_k3(int prec, const StageArgs &a, int grid, int lds_bytes, hipStream_t s);
hipError_t set_stage_k3_attributes(int prec, int lds_bytes);
hipError_t stage_k3_occupancy(int prec, int lds_bytes, int *per_cu);
hipError_t launch_stage_k4(int prec, const StageArgs &a, int grid, hipStream_t s);
hipError_t set_stage_k4_attributes(int prec);
// driving factor table of the k = 3 kernel: modes [m][9] as for the cache (n as doubles, then
// Re/Im of the three components), wave vectors with n_x >= 0
hipError_t launch_drive_table_k3(const double *modes, int nmodes, int dks, int ny, int nz, const GaussNodes &xg,
                                 int nx, int z0, int nzg, float *out, hipStream_t s);

hipError_t launch_project(int k, int prec, const void *qp, void *y, const double *ptab, long long ncells, int nx,
                          hipStream_t s);
hipError_t launch_cfl(int prec, const void *y, int N, int nx, long long ncells, double gamma, const double h[3],
                      double *rate_slot, double *zero_slot, hipStream_t s);
hipError_t launch_totals(int prec, const void *y, int N, int nx, long long ncells, double vol, double *partials,
                         int nparts, double *out, hipStream_t s);
hipError_t launch_range_check(int prec, const void *y, int N, int nx, long long ncells, double gamma, int *flag,
                              hipStream_t s);

// ---- learned closure (k = 1): 140 -> 128 -> 128 -> 20, tanh
constexpr int CL_ROWS = NF * 4;         // weight rows per cell at k = 1
constexpr int CL_NIN = 7 * CL_ROWS;     // self and six face neighbours
constexpr int CL_NH = 128;
constexpr int CL_NOUT = CL_ROWS;
constexpr long long CL_NPARAMS = (long long)CL_NH * CL_NIN + CL_NH + CL_NH * CL_NH + CL_NH + CL_NOUT * CL_NH + CL_NOUT;

struct ClosureArgs {
    const void *y;
    void *corr;
    const float *params;   // W1 b1 W2 b2 W3 b3, W row-major [out][in]
    const float *fmean;    // [CL_NIN]
    const float *fistd;    // [CL_NIN] 1 / std
    const float *oscale;   // [CL_NOUT]
    const float *obound;   // [CL_NOUT]
    double *partials;      // [waves of the grid][5]
    unsigned long long *fallbacks;
    unsigned long long *done;  // workgroups finished (zero between launches)
    double *cmean;         // [5]
    int nx, ny, nz;
    long long ncells;
};
hipError_t launch_closure(int prec, const ClosureArgs &a, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long *p, hipStream_t s);
hipError_t launch_features(int prec, const void *y, float *feat, int N, int nx, int ny, int nz, long long nc,
                           hipStream_t s);
hipError_t launch_targets(int prec, const void *rc, const void *prf, float *out, int N, int nx, long long nc,
                          hipStream_t s);
hipError_t launch_restrict(int prec, const void *yf, void *yc, const double *M, int Nf, int Nc, int NX, int NY, int NZ,
                           hipStream_t s);

// ---- training kernels
enum { EP_NONE = 0, EP_TANH = 1, EP_DTANH = 2 };
struct GemmArgs {
    const float *A, *B;
    float *C;
    const float *bias;  // [M] or nullptr
    const float *E;     // EP_DTANH: tanh outputs, C's strides
    int M, N, K;
    long long sam, sak, sbk, sbn, scm, scn;
    int ep;
};
hipError_t launch_gemm(const GemmArgs &a, hipStream_t s);
hipError_t launch_rowsum(const float *X, int M, int N, float *out, hipStream_t s);
hipError_t launch_gather(const float *X, int cols, const int *rows, int batch, float *Xb, hipStream_t s,
                         float noise = 0.0f, unsigned long long seed = 0);
hipError_t launch_mse(const float *Y, const float *T, float *dY, long long n, double *loss, hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, long long n, int step, double lr, double b1,
                       double b2, double eps, hipStream_t s);
hipError_t launch_colstats(const float *x, long long rows, int cols, double *part, int nchunks, double *mean,
                           double *stdv, double *rms, double *maxabs, hipStream_t s);
hipError_t launch_standardize(float *x, long long rows, int cols, const double *shift, const double *scale,
                              hipStream_t s);
// the message dg_error_string(NULL) returns on the calling thread (calls without a context)
void set_call_error(const char *msg);

}  // namespace dgmi

struct dg_ctx {
    dg_config cfg;
    hipStream_t stream;
    int N, n, Q, P;
    long long ncells;
    double h[3];
    dgmi::TableLayout lay;
    void *tables = nullptr;        // MFMA fragment tables
    double *ptab = nullptr;        // projection table [Q][N] = phi_l(xi_q) w_q / 8
    double *slots = nullptr;       // [0],[1]: max CFL rate (alternating), [2]: time, [3]: scratch
    int *flag = nullptr;           // range-check flag
    double *partials = nullptr;    // totals partial sums
    int nparts = 0;
    double *fmodes = nullptr;      // forcing mode table [MAX_FORCING_MODES][9]
    void *acache = nullptr;        // driving acceleration at the volume points (storage type)
    // k = 3 in the FP32-storage tiers runs stage_k3_kernel (16-cell x-blocks, driving as a product)
    bool k3x = false;
    bool k4m = false;  // k = 4 in FP32 / FP64: the matrix-core kernel of stage_k4.hip
    float *dtab = nullptr;         // its driving factor table, per (z, y) row
    float *dcs = nullptr;          // cos / sin of the x phases, per x
    int dks = 0;                   // K steps of the driving product
    int nfmodes = 0;
    bool have_forcing = false;
    int grid = 0;
    int zlen = 1;                  // z chunk length of the stage sweep
    int zlen_auto = 1;             // the length dg_init chose (dg_set_zchunk(ctx, 0) restores it)
    int ex_off = 0;                // LDS offsets of the y-face trace and flux regions (after the tables)
    int ex_off2 = 0;
    int ex_off3 = -1;              // LDS offset of the end-row buffers (-1: not used)
    int ex_off4 = -1;              // LDS offset of the x-face ghost-cell copies (k = 3 BF16 tiers)
    // z slab of a larger periodic mesh (DG_ZHALO): halo planes and the slab's place for the driving
    const void *halo_lo = nullptr, *halo_hi = nullptr;
    int slab_z0 = 0, slab_nz = 0;
    int cur_slot = 1;              // slot holding the latest CFL rate
    int lds = 0;
    long long step_count = 0;
    // closure (DG_CLOSURE)
    float *clo = nullptr;                 // params, fmean, fistd, oscale, obound
    void *corr = nullptr;                 // correction, state layout
    double *clo_partials = nullptr;       // per-wave mean-row sums; then [5] means
    unsigned long long *clo_fallbacks = nullptr;
    bool have_closure = false;
    double *restrict_tab[4] = {nullptr, nullptr, nullptr, nullptr};  // per fine degree: [8][N][Nf]
    // positivity limiter (DG_LIMIT)
    double *limtab = nullptr;              // phi_l at the limiter points [np][N]
    int limnp = 0;
    unsigned long long *limcount = nullptr;  // cells changed by the limiter since the last query
    // isothermal reset (Sec. 3.2; dg_set_isothermal)
    dgmi::Leg1D leg1d{};                   // 1D Legendre values and weights at the Gauss nodes
    double *iso_partials = nullptr;        // per-block dissipated energy
    double iso_cs = 0.0, iso_rho0 = 0.0;
    bool have_iso = false;
    // diagnostics (dg_sample, dg_velocity_spectrum, dg_density_pdf, dg_rms_mach)
    void *fft = nullptr;                   // hipFFT plan (R2C / D2Z, fft_m^3), made on first use
    int fft_m = 0;
    double *diag_bins = nullptr;           // [DIAG_MAX_BINS] shell sums, then [DIAG_MAX_BINS + 2] counts
    double *diag_partials = nullptr;       // per-block Mach sums, then the total
    std::string err;
};
