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

// The driving acceleration at the volume points is one more MFMA product over
// KF contraction slots (the real and imaginary parts of KF/2 Fourier modes).
inline int forcing_slots(int prec) { return (prec == DG_BF16 || prec == DG_BF16X3) ? 96 : 88; }

inline int nmodes_of(int k) { return (k + 1) * (k + 2) * (k + 3) / 6; }

// Row of a 16x16 MFMA output tile held by lane group g (= lane/16) in result
// register r.  FP32/BF16 accumulators: 4g + r.  FP64 (16x16x4f64): g + 4r.
inline int out_row(int prec, int g, int r) { return prec == DG_FP64 ? g + 4 * r : 4 * g + r; }

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
size_t forcing_table_bytes(const TableLayout &L);
std::vector<char> build_forcing_table(const TableLayout &L, const int n[3], int nmodes, const int32_t *nvec);

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
    long long nitems;     // work items: nbx * ny * ceil(nz / zlen)
    long long ncells;
    int mode;             // 0: out = R(yin); 1: out = a*y0 + b*(yin - dt*R(yin))
    int forcing;          // 1: add the driving source
    const double *fmodes; // device mode table [KF/2][9]: n_x, n_y, n_z, then Re/Im of ahat_x, ahat_y, ahat_z
    int nfmodes;
    double h[3];          // cell widths
};

hipError_t launch_stage(int k, int prec, const StageArgs &a, int grid, int lds_bytes, hipStream_t s);
hipError_t set_stage_attributes(int k, int prec, int lds_bytes);
int stage_block_threads();

hipError_t launch_project(int k, int prec, const void *qp, void *y, const double *ptab, long long ncells, int nx,
                          hipStream_t s);
hipError_t launch_cfl(int prec, const void *y, int N, int nx, long long ncells, double gamma, const double h[3],
                      double *rate_slot, double *zero_slot, hipStream_t s);
hipError_t launch_totals(int prec, const void *y, int N, int nx, long long ncells, double vol, double *partials,
                         int nparts, double *out, hipStream_t s);
hipError_t launch_range_check(int prec, const void *y, int N, int nx, long long ncells, double gamma, int *flag,
                              hipStream_t s);

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
    double *fmodes = nullptr;      // forcing mode table (zero padded to KF/2 modes)
    size_t f6_bytes = 0;           // bytes of the forcing point table (after the operator tables)
    int nfmodes = 0;
    bool have_forcing = false;
    int grid = 0;
    int zlen = 1;                  // z chunk length of the stage sweep
    int cur_slot = 1;              // slot holding the latest CFL rate
    int lds = 0;
    long long step_count = 0;
    std::string err;
};
