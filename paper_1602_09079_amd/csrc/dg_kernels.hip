// HIP kernels of libdgmi.so for gfx950 (MI355X).
//
// The fused SSP stage kernel evaluates the modal DG operator of Bauer et al.
// (arXiv 1602.09079), Sec. 2.3, for blocks of 16 cells that are consecutive in
// x.  Every basis contraction is a dense GEMM over cells on the matrix cores:
//
//   GEMM1  q(xi_q)        = Phi[q][l]         * w[l][cell]      (modal -> volume points)
//   GEMM2  R[l]          += -s_a dPhi_a[l][q] * F_a(q)[q][cell]  (volume integral, eq. dg:eqn:volume_int)
//   GEMM3  q(face point)  = Phif[p][l]        * w[l][cell]      (traces on the six faces)
//   GEMM4  R[l]          += s_a (+-) Phif[l][p] * Fhat[p][cell]  (surface lift, eq. dg:eqn:surface_int)
//   GEMM5  R[l]          -= Phi[l][q] w_q/8   * S(q)[q][cell]    (driving source, Sec. 3.1)
//
// Cells are the 16 columns of each MFMA tile.  The result registers of GEMM1
// and GEMM3 are used directly as B operands of GEMM2 and GEMM4: the contraction
// index of the tables is permuted on the host to match the output lane layout,
// so no data is moved between the chained products.  The Euler flux and the HLLC
// Riemann solver run on the vector ALUs in that same lane layout.
//
// Faces: the x-neighbour of a column is the adjacent lane of its 16-lane row
// (DPP row shifts); a block's columns 0 and 15 are halo cells whose results are
// discarded, so consecutive blocks overlap by two cells.  The y- and z-neighbour
// traces are computed from the neighbouring blocks' weights (loaded through L2)
// with the same GEMM3 tables, so each face flux is computed from bitwise
// identical inputs on both sides and the scheme stays conservative to round-off.
//
// Persistent grid: each wave loops over blocks; the block range is split into 8
// contiguous parts, one per XCD (workgroup id modulo 8), so that the y/z
// neighbours a wave reads were recently loaded into the same XCD's L2.

#include "dg_internal.h"

#include <type_traits>

namespace dgmi {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

template <int K>
struct Dims {
    static constexpr int N = (K + 1) * (K + 2) * (K + 3) / 6;
    static constexpr int n = K + 1;
    static constexpr int Q = n * n * n;
    static constexpr int P = n * n;
};

// ------------------------------------------------------------------ precision policies

template <int PREC>
struct Prec;

template <>
struct Prec<DG_FP64> {
    using S = double;  // storage
    using C = double;  // pointwise arithmetic
    using Acc = d4;
    static constexpr int KPL = 1, KSTEP = 4;
    struct AF { double v; };
    struct BF { double v; };
    __device__ static AF lda(const char *lds, int frag, int lane) {
        return AF{reinterpret_cast<const double *>(lds)[frag * 64 + lane]};
    }
    __device__ static Acc mma(Acc c, AF a, BF b) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a.v, b.v, c, 0, 0, 0); }
    __device__ static int orow(int g, int r) { return g + 4 * r; }
    __device__ static BF mkb(const C *v) { return BF{v[0]}; }
    __device__ static C rcp(C x) { return 1.0 / x; }
    __device__ static C sqrt_(C x) { return __builtin_sqrt(x); }
};

template <>
struct Prec<DG_FP32> {
    using S = float;
    using C = float;
    using Acc = f4;
    static constexpr int KPL = 1, KSTEP = 4;
    struct AF { float v; };
    struct BF { float v; };
    __device__ static AF lda(const char *lds, int frag, int lane) {
        return AF{reinterpret_cast<const float *>(lds)[frag * 64 + lane]};
    }
    __device__ static Acc mma(Acc c, AF a, BF b) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a.v, b.v, c, 0, 0, 0); }
    __device__ static int orow(int g, int r) { return 4 * g + r; }
    __device__ static BF mkb(const C *v) { return BF{v[0]}; }
    __device__ static C rcp(C x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static C sqrt_(C x) { return __builtin_amdgcn_sqrtf(x); }
};

template <>
struct Prec<DG_BF16> {
    using S = float;
    using C = float;
    using Acc = f4;
    static constexpr int KPL = 8, KSTEP = 32;
    struct AF { bf8 v; };
    struct BF { bf8 v; };
    __device__ static AF lda(const char *lds, int frag, int lane) {
        return AF{reinterpret_cast<const bf8 *>(lds)[frag * 64 + lane]};
    }
    __device__ static Acc mma(Acc c, AF a, BF b) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, c, 0, 0, 0); }
    __device__ static int orow(int g, int r) { return 4 * g + r; }
    __device__ static BF mkb(const C *v) {
        BF b;
#pragma unroll
        for (int j = 0; j < 8; j++) b.v[j] = (__bf16)v[j];
        return b;
    }
    __device__ static C rcp(C x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static C sqrt_(C x) { return __builtin_amdgcn_sqrtf(x); }
};

// FP32-grade contractions from BF16 matrix cores: x = hi + lo with hi = bf16(x),
// lo = bf16(x - hi); a*b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b (lo_a lo_b dropped).
template <>
struct Prec<DG_BF16X3> {
    using S = float;
    using C = float;
    using Acc = f4;
    static constexpr int KPL = 8, KSTEP = 32;
    struct AF { bf8 hi, lo; };
    struct BF { bf8 hi, lo; };
    static constexpr int HALF_OFFSET_FRAGS = 0;  // lo tables follow the hi tables (offset passed at run time)
    __device__ static AF lda2(const char *lds, int frag, int lane, int lo_off) {
        const bf8 *t = reinterpret_cast<const bf8 *>(lds);
        return AF{t[frag * 64 + lane], t[(lo_off + frag) * 64 + lane]};
    }
    __device__ static Acc mma(Acc c, AF a, BF b) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b.hi, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.lo, c, 0, 0, 0);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.hi, c, 0, 0, 0);
    }
    __device__ static int orow(int g, int r) { return 4 * g + r; }
    __device__ static BF mkb(const C *v) {
        BF b;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            __bf16 h = (__bf16)v[j];
            b.hi[j] = h;
            b.lo[j] = (__bf16)(v[j] - (float)h);
        }
        return b;
    }
    __device__ static C rcp(C x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static C sqrt_(C x) { return __builtin_amdgcn_sqrtf(x); }
};

// ------------------------------------------------------------------ lane exchange

__device__ inline float dpp_shr1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, true));
}
__device__ inline float dpp_shl1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x101, 0xf, 0xf, true));
}
__device__ inline double dpp_shr1(double v) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x111, 0xf, 0xf, true);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x111, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double dpp_shl1(double v) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x101, 0xf, 0xf, true);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x101, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ------------------------------------------------------------------ pointwise physics

// Ideal-gas Euler flux along the three axes at one point, Sec. 2.3.
template <class PR, class C>
__device__ inline void euler_flux3(const C q[5], C g1, C F[3][5]) {
    C inv = PR::rcp(q[0]);
    C u = q[1] * inv, v = q[2] * inv, w = q[3] * inv;
    C p = g1 * (q[4] - C(0.5) * (q[1] * u + q[2] * v + q[3] * w));
    C ep = q[4] + p;
    F[0][0] = q[1]; F[0][1] = q[1] * u + p; F[0][2] = q[2] * u; F[0][3] = q[3] * u; F[0][4] = ep * u;
    F[1][0] = q[2]; F[1][1] = q[1] * v;     F[1][2] = q[2] * v + p; F[1][3] = q[3] * v; F[1][4] = ep * v;
    F[2][0] = q[3]; F[2][1] = q[1] * w;     F[2][2] = q[2] * w; F[2][3] = q[3] * w + p; F[2][4] = ep * w;
}

// HLLC numerical flux across a face normal to AXIS, left state qL, right state
// qR (Toro, Riemann Solvers and Numerical Methods for Fluid Dynamics, ch. 10,
// Davis wave-speed bounds).  S* >= 0 takes the left star state.  Written without
// branches: the side K is selected first and only its flux and star state are formed.
template <class PR, int AXIS, class C>
__device__ inline void hllc(const C qL[5], const C qR[5], C gam, C F[5]) {
    const C g1 = gam - C(1);
    C iL = PR::rcp(qL[0]), iR = PR::rcp(qR[0]);
    C uL = qL[1 + AXIS] * iL, uR = qR[1 + AXIS] * iR;
    C pL = g1 * (qL[4] - C(0.5) * (qL[1] * qL[1] + qL[2] * qL[2] + qL[3] * qL[3]) * iL);
    C pR = g1 * (qR[4] - C(0.5) * (qR[1] * qR[1] + qR[2] * qR[2] + qR[3] * qR[3]) * iR);
    C cL = PR::sqrt_(gam * pL * iL), cR = PR::sqrt_(gam * pR * iR);
    C SL = __builtin_fmin(uL - cL, uR - cR);
    C SR = __builtin_fmax(uL + cL, uR + cR);
    C dL = qL[0] * (SL - uL), dR = qR[0] * (SR - uR);
    C Ss = (pR - pL + qL[1 + AXIS] * (SL - uL) - qR[1 + AXIS] * (SR - uR)) / (dL - dR);
    bool left = (Ss >= C(0)) || (SL >= C(0));
    C q[5];
#pragma unroll
    for (int i = 0; i < 5; i++) q[i] = left ? qL[i] : qR[i];
    C iK = left ? iL : iR, uK = left ? uL : uR, pK = left ? pL : pR, SK = left ? SL : SR, dK = left ? dL : dR;
    // physical flux of side K
    C FK[5];
    FK[0] = q[1 + AXIS];
#pragma unroll
    for (int j = 0; j < 3; j++) FK[1 + j] = q[1 + j] * uK;
    FK[1 + AXIS] += pK;
    FK[4] = (q[4] + pK) * uK;
    // star state of side K
    C fac = dK / (SK - Ss);
    C U[5];
    U[0] = fac;
#pragma unroll
    for (int j = 0; j < 3; j++) U[1 + j] = fac * q[1 + j] * iK;
    U[1 + AXIS] = fac * Ss;
    U[4] = fac * (q[4] * iK + (Ss - uK) * (Ss + pK / dK));
    bool plain = (SL >= C(0)) || (!left && SR <= C(0));
#pragma unroll
    for (int i = 0; i < 5; i++) F[i] = plain ? FK[i] : FK[i] + SK * (U[i] - q[i]);
}

// ------------------------------------------------------------------ the fused stage kernel

template <int K, int PREC>
struct StageCfg {
    using D = Dims<K>;
    using PR = Prec<PREC>;
    static constexpr int N = D::N, Q = D::Q, P = D::P;
    static constexpr int KPL = PR::KPL, KSTEP = PR::KSTEP;
    static constexpr int KS1 = (N + KSTEP - 1) / KSTEP;
    static constexpr int RT1 = KPL == 8 ? 2 * ((Q + 31) / 32) : (Q + 15) / 16;
    static constexpr int RT2 = (N + 15) / 16;
    static constexpr int NC2 = KPL == 8 ? RT1 / 2 : RT1 * 4;
    static constexpr int NC4 = KPL == 8 ? 3 : 24;
    static constexpr int OFF1 = 0;
    static constexpr int OFF2 = OFF1 + RT1 * KS1;
    static constexpr int OFF3 = OFF2 + RT2 * 3 * NC2;
    static constexpr int OFF4 = OFF3 + 6 * KS1;
    static constexpr int OFF5 = OFF4 + RT2 * NC4;
    static constexpr int NFRAG = OFF5 + RT2 * NC2;
};

template <int PREC>
struct TabReader {
    const char *lds;
    int lane;
    int lo_off;
    __device__ typename Prec<PREC>::AF operator()(int frag) const {
        if constexpr (PREC == DG_BF16X3)
            return Prec<PREC>::lda2(lds, frag, lane, lo_off);
        else
            return Prec<PREC>::lda(lds, frag, lane);
    }
};

constexpr int STAGE_THREADS = 256;

template <int K, int PREC>
__global__ __launch_bounds__(STAGE_THREADS) void stage_kernel(StageArgs a) {
    using SC = StageCfg<K, PREC>;
    using PR = typename SC::PR;
    using C = typename PR::C;
    using S = typename PR::S;
    using Acc = typename PR::Acc;
    using BF = typename PR::BF;
    constexpr int N = SC::N, Q = SC::Q, P = SC::P;
    constexpr int KPL = SC::KPL, KSTEP = SC::KSTEP, KS1 = SC::KS1;
    constexpr int RT1 = SC::RT1, RT2 = SC::RT2, NC2 = SC::NC2, NC4 = SC::NC4;

    extern __shared__ __attribute__((aligned(16))) char lds[];
    {
        // stage the fragment tables into LDS
        constexpr int ntab = PREC == DG_BF16X3 ? 2 : 1;
        constexpr size_t esz = PREC == DG_FP64 ? 8 : (PREC == DG_FP32 ? 4 : 2);
        constexpr size_t bytes = (size_t)SC::NFRAG * 64 * KPL * esz * ntab;
        const int4 *src = reinterpret_cast<const int4 *>(a.tables);
        int4 *dst = reinterpret_cast<int4 *>(lds);
        for (size_t j = threadIdx.x; j < bytes / 16; j += STAGE_THREADS) dst[j] = src[j];
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15;
    const int g = lane >> 4;
    const TabReader<PREC> T{lds, lane, SC::NFRAG};

    const C gam = (C)a.gamma;
    const C g1 = gam - C(1);
    double dtd = a.dt;
    if (a.rate) dtd = a.dtfac / a.rate[0];
    const C dt = (C)dtd;
    if (a.tacc && blockIdx.x == 0 && threadIdx.x == 0) a.tacc[0] += dtd;
    const S *__restrict__ yin = reinterpret_cast<const S *>(a.yin);
    const S *__restrict__ y0 = reinterpret_cast<const S *>(a.y0);
    S *out = reinterpret_cast<S *>(a.out);
    const long long nc = a.ncells;
    const int nx = a.nx, ny = a.ny, nz = a.nz;

    // XCD-aware assignment of blocks to waves
    const int nxcd = gridDim.x < 8 ? (int)gridDim.x : 8;
    const int xcd = blockIdx.x % nxcd;
    const int wgs_x = (gridDim.x - xcd + nxcd - 1) / nxcd;
    const long long wid = (long long)(blockIdx.x / nxcd) * (STAGE_THREADS / 64) + wave;
    const long long wcount = (long long)wgs_x * (STAGE_THREADS / 64);
    const long long b_lo = a.nblocks * xcd / nxcd, b_hi = a.nblocks * (xcd + 1) / nxcd;

    for (long long blk = b_lo + wid; blk < b_hi; blk += wcount) {
        const int bx = (int)(blk % a.nbx);
        const long long rest = blk / a.nbx;
        const int iy = (int)(rest % ny);
        const int iz = (int)(rest / ny);
        const int xraw = BLK_INNER * bx - 1 + col;          // may be -1 or >= nx: periodic wrap
        const int xc = (xraw % nx + nx) % nx;
        const long long rowbase = ((long long)iz * ny + iy) * nx;
        const long long cell = rowbase + xc;

        auto load_w = [&](long long cidx, BF w[NF][KS1]) {
#pragma unroll
            for (int i = 0; i < NF; i++)
#pragma unroll
                for (int s = 0; s < KS1; s++) {
                    C v[KPL];
#pragma unroll
                    for (int j = 0; j < KPL; j++) {
                        const int m = s * KSTEP + g * KPL + j;
                        v[j] = m < N ? (C)yin[((long long)i * N + m) * nc + cidx] : C(0);
                    }
                    w[i][s] = PR::mkb(v);
                }
        };
        auto trace = [&](const BF w[NF][KS1], int face, Acc tr[NF]) {
#pragma unroll
            for (int i = 0; i < NF; i++) tr[i] = Acc{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KS1; s++) {
                const auto A = T(SC::OFF3 + face * KS1 + s);
#pragma unroll
                for (int i = 0; i < NF; i++) tr[i] = PR::mma(tr[i], A, w[i][s]);
            }
        };

        BF w[NF][KS1];
        load_w(cell, w);

        Acc acc[NF][RT2];
#pragma unroll
        for (int i = 0; i < NF; i++)
#pragma unroll
            for (int rt = 0; rt < RT2; rt++) acc[i][rt] = Acc{0, 0, 0, 0};

        // ---------------- volume integral: GEMM1 -> flux -> GEMM2
        if constexpr (KPL == 1) {
#pragma unroll
            for (int t = 0; t < RT1; t++) {
                Acc d[NF];
#pragma unroll
                for (int i = 0; i < NF; i++) d[i] = Acc{0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < KS1; s++) {
                    const auto A = T(SC::OFF1 + t * KS1 + s);
#pragma unroll
                    for (int i = 0; i < NF; i++) d[i] = PR::mma(d[i], A, w[i][s]);
                }
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const bool valid = 16 * t + PR::orow(g, r) < Q;
                    C q[5], F[3][5];
#pragma unroll
                    for (int i = 0; i < 5; i++) q[i] = valid ? d[i][r] : C(1);
                    euler_flux3<PR>(q, g1, F);
#pragma unroll
                    for (int al = 0; al < 3; al++)
#pragma unroll
                        for (int i = 0; i < 5; i++) F[al][i] = valid ? F[al][i] : C(0);
#pragma unroll
                    for (int rt = 0; rt < RT2; rt++)
#pragma unroll
                        for (int al = 0; al < 3; al++) {
                            const auto A = T(SC::OFF2 + (rt * 3 + al) * NC2 + t * 4 + r);
#pragma unroll
                            for (int i = 0; i < NF; i++) acc[i][rt] = PR::mma(acc[i][rt], A, PR::mkb(&F[al][i]));
                        }
                }
            }
        } else {
#pragma unroll
            for (int tp = 0; tp < RT1 / 2; tp++) {
                C Fv[3][5][8];
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const int t = 2 * tp + h;
                    Acc d[NF];
#pragma unroll
                    for (int i = 0; i < NF; i++) d[i] = Acc{0, 0, 0, 0};
                    const auto A = T(SC::OFF1 + t * KS1);
#pragma unroll
                    for (int i = 0; i < NF; i++) d[i] = PR::mma(d[i], A, w[i][0]);
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const bool valid = 16 * t + PR::orow(g, r) < Q;
                        C q[5], F[3][5];
#pragma unroll
                        for (int i = 0; i < 5; i++) q[i] = valid ? d[i][r] : C(1);
                        euler_flux3<PR>(q, g1, F);
#pragma unroll
                        for (int al = 0; al < 3; al++)
#pragma unroll
                            for (int i = 0; i < 5; i++) Fv[al][i][4 * h + r] = valid ? F[al][i] : C(0);
                    }
                }
#pragma unroll
                for (int rt = 0; rt < RT2; rt++)
#pragma unroll
                    for (int al = 0; al < 3; al++) {
                        const auto A = T(SC::OFF2 + (rt * 3 + al) * NC2 + tp);
#pragma unroll
                        for (int i = 0; i < NF; i++) acc[i][rt] = PR::mma(acc[i][rt], A, PR::mkb(Fv[al][i]));
                    }
            }
        }

        // ---------------- surface integral: traces -> HLLC -> lift, one axis at a time
        auto lift = [&](int axis, const C Fm[NF][4], const C Fp[NF][4]) {
            if constexpr (KPL == 1) {
#pragma unroll
                for (int side = 0; side < 2; side++)
#pragma unroll
                    for (int r = 0; r < 4; r++)
#pragma unroll
                        for (int rt = 0; rt < RT2; rt++) {
                            const auto A = T(SC::OFF4 + rt * NC4 + (2 * axis + side) * 4 + r);
#pragma unroll
                            for (int i = 0; i < NF; i++)
                                acc[i][rt] = PR::mma(acc[i][rt], A, PR::mkb(side ? &Fp[i][r] : &Fm[i][r]));
                        }
            } else {
#pragma unroll
                for (int rt = 0; rt < RT2; rt++) {
                    const auto A = T(SC::OFF4 + rt * NC4 + axis);
#pragma unroll
                    for (int i = 0; i < NF; i++) {
                        C v[8];
#pragma unroll
                        for (int r = 0; r < 4; r++) {
                            v[r] = Fm[i][r];
                            v[4 + r] = Fp[i][r];
                        }
                        acc[i][rt] = PR::mma(acc[i][rt], A, PR::mkb(v));
                    }
                }
            }
        };
        auto riemann = [&](auto axis_c, const Acc tl[NF], const Acc tr_[NF], C Fo[NF][4]) {
            constexpr int AX = decltype(axis_c)::value;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const bool valid = PR::orow(g, r) < P;
                C qL[5], qR[5], F[5];
#pragma unroll
                for (int i = 0; i < 5; i++) {
                    qL[i] = valid ? (C)tl[i][r] : C(1);
                    qR[i] = valid ? (C)tr_[i][r] : C(1);
                }
                if (!valid) { qL[4] = qR[4] = C(2); }
                hllc<PR, AX>(qL, qR, gam, F);
#pragma unroll
                for (int i = 0; i < 5; i++) Fo[i][r] = valid ? F[i] : C(0);
            }
        };

        // x faces: left neighbour's + trace comes from the adjacent lane
        {
            Acc tm[NF], tp[NF];
            trace(w, 0, tm);
            trace(w, 1, tp);
            Acc tl[NF];
#pragma unroll
            for (int i = 0; i < NF; i++)
#pragma unroll
                for (int r = 0; r < 4; r++) tl[i][r] = dpp_shr1((C)tp[i][r]);
            C Fm[NF][4], Fp[NF][4];
            riemann(std::integral_constant<int, 0>{}, tl, tm, Fm);
#pragma unroll
            for (int i = 0; i < NF; i++)
#pragma unroll
                for (int r = 0; r < 4; r++) Fp[i][r] = dpp_shl1(Fm[i][r]);
            lift(0, Fm, Fp);
        }
        // y faces
        {
            C Fm[NF][4], Fp[NF][4];
            {
                BF wn[NF][KS1];
                load_w(((long long)iz * ny + (iy + ny - 1) % ny) * nx + xc, wn);
                Acc tn[NF], tm[NF];
                trace(wn, 3, tn);
                trace(w, 2, tm);
                riemann(std::integral_constant<int, 1>{}, tn, tm, Fm);
            }
            {
                BF wn[NF][KS1];
                load_w(((long long)iz * ny + (iy + 1) % ny) * nx + xc, wn);
                Acc tn[NF], tp[NF];
                trace(wn, 2, tn);
                trace(w, 3, tp);
                riemann(std::integral_constant<int, 1>{}, tp, tn, Fp);
            }
            lift(1, Fm, Fp);
        }
        // z faces
        {
            C Fm[NF][4], Fp[NF][4];
            {
                BF wn[NF][KS1];
                load_w(((long long)((iz + nz - 1) % nz) * ny + iy) * nx + xc, wn);
                Acc tn[NF], tm[NF];
                trace(wn, 5, tn);
                trace(w, 4, tm);
                riemann(std::integral_constant<int, 2>{}, tn, tm, Fm);
            }
            {
                BF wn[NF][KS1];
                load_w(((long long)((iz + 1) % nz) * ny + iy) * nx + xc, wn);
                Acc tn[NF], tp[NF];
                trace(wn, 4, tn);
                trace(w, 5, tp);
                riemann(std::integral_constant<int, 2>{}, tp, tn, Fp);
            }
            lift(2, Fm, Fp);
        }

        // ---------------- combine and store the interior columns
        const bool keep = col >= 1 && col <= BLK_INNER && xraw < nx && xraw >= 0 && (BLK_INNER * bx + col - 1) < nx;
        if (keep) {
#pragma unroll
            for (int rt = 0; rt < RT2; rt++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int m = 16 * rt + PR::orow(g, r);
                    if (m < N) {
#pragma unroll
                        for (int i = 0; i < NF; i++) {
                            const long long idx = ((long long)i * N + m) * nc + cell;
                            const C R = (C)acc[i][rt][r];
                            if (a.mode == 0) {
                                out[idx] = (S)R;
                            } else {
                                const C yv = (C)yin[idx];
                                const C base = (C)a.b * (yv - dt * R);
                                out[idx] = (S)(a.a != 0.0 ? (C)a.a * (C)y0[idx] + base : base);
                            }
                        }
                    }
                }
        }
    }
}

template <int K, int PREC>
static hipError_t launch_stage_t(const StageArgs &a, int grid, int lds_bytes, hipStream_t s) {
    hipLaunchKernelGGL((stage_kernel<K, PREC>), dim3(grid), dim3(STAGE_THREADS), lds_bytes, s, a);
    return hipGetLastError();
}

template <int K, int PREC>
static hipError_t set_attr_t(int lds_bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&stage_kernel<K, PREC>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}

#define DG_DISPATCH(k, prec, CALL, ARGS)                                             \
    switch (k * 10 + prec) {                                                          \
        case 10: return CALL<1, DG_FP64> ARGS; case 11: return CALL<1, DG_FP32> ARGS;   \
        case 12: return CALL<1, DG_BF16> ARGS; case 13: return CALL<1, DG_BF16X3> ARGS; \
        case 20: return CALL<2, DG_FP64> ARGS; case 21: return CALL<2, DG_FP32> ARGS;   \
        case 22: return CALL<2, DG_BF16> ARGS; case 23: return CALL<2, DG_BF16X3> ARGS; \
        case 30: return CALL<3, DG_FP64> ARGS; case 31: return CALL<3, DG_FP32> ARGS;   \
        case 32: return CALL<3, DG_BF16> ARGS; case 33: return CALL<3, DG_BF16X3> ARGS; \
        default: return hipErrorInvalidValue;                                         \
    }

hipError_t launch_stage(int k, int prec, const StageArgs &a, int grid, int lds_bytes, hipStream_t s) {
    DG_DISPATCH(k, prec, launch_stage_t, (a, grid, lds_bytes, s))
}

hipError_t set_stage_attributes(int k, int prec, int lds_bytes) {
    DG_DISPATCH(k, prec, set_attr_t, (lds_bytes))
}

int stage_block_threads() { return STAGE_THREADS; }

template <int K, int PREC>
static hipError_t occ_t(int lds_bytes, int *per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, stage_kernel<K, PREC>, STAGE_THREADS, lds_bytes);
}

}  // namespace dgmi

hipError_t stage_occupancy(int k, int prec, int lds_bytes, int *per_cu) {
    using namespace dgmi;
    DG_DISPATCH(k, prec, occ_t, (lds_bytes, per_cu))
}

namespace dgmi {

// ------------------------------------------------------------------ projection (Sec. 2.2)

template <int K, class S>
__global__ void project_kernel(const S *__restrict__ qp, S *__restrict__ y, const double *__restrict__ ptab,
                               long long nc) {
    constexpr int N = Dims<K>::N, Q = Dims<K>::Q;
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= nc) return;
    for (int i = 0; i < NF; i++) {
        double s[N];
#pragma unroll
        for (int l = 0; l < N; l++) s[l] = 0.0;
        for (int q = 0; q < Q; q++) {
            const double v = (double)qp[((long long)i * Q + q) * nc + cell];
#pragma unroll
            for (int l = 0; l < N; l++) s[l] += v * ptab[q * N + l];
        }
#pragma unroll
        for (int l = 0; l < N; l++) y[((long long)i * N + l) * nc + cell] = (S)s[l];
    }
}

template <int K>
static hipError_t launch_project_k(int prec, const void *qp, void *y, const double *ptab, long long nc,
                                   hipStream_t s) {
    const int th = 256;
    const long long nb = (nc + th - 1) / th;
    if (prec == DG_FP64)
        hipLaunchKernelGGL((project_kernel<K, double>), dim3(nb), dim3(th), 0, s, (const double *)qp, (double *)y,
                           ptab, nc);
    else
        hipLaunchKernelGGL((project_kernel<K, float>), dim3(nb), dim3(th), 0, s, (const float *)qp, (float *)y, ptab,
                           nc);
    return hipGetLastError();
}

hipError_t launch_project(int k, int prec, const void *qp, void *y, const double *ptab, long long nc,
                          hipStream_t s) {
    switch (k) {
        case 1: return launch_project_k<1>(prec, qp, y, ptab, nc, s);
        case 2: return launch_project_k<2>(prec, qp, y, ptab, nc, s);
        case 3: return launch_project_k<3>(prec, qp, y, ptab, nc, s);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ CFL reduction (Sec. 2.4)

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

template <class S>
__global__ void cfl_kernel(const S *__restrict__ y, int N, long long nc, double gamma, double hx, double hy,
                           double hz, double *rate_slot, double *zero_slot) {
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double rate = 0.0;
    if (cell < nc) {
        const double rho = (double)y[(0LL * N) * nc + cell];
        const double mx = (double)y[(1LL * N) * nc + cell];
        const double my = (double)y[(2LL * N) * nc + cell];
        const double mz = (double)y[(3LL * N) * nc + cell];
        const double E = (double)y[(4LL * N) * nc + cell];
        const double inv = 1.0 / rho;
        const double p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my + mz * mz) * inv);
        const double c = sqrt(gamma * p * inv);
        rate = (fabs(mx * inv) + c) / hx + (fabs(my * inv) + c) / hy + (fabs(mz * inv) + c) / hz;
        if (!(rate >= 0.0)) rate = __builtin_inf();  // non-physical cell: force dt -> 0
    }
    rate = wave_max(rate);
    if ((threadIdx.x & 63) == 0)
        atomicMax(reinterpret_cast<unsigned long long *>(rate_slot), (unsigned long long)__double_as_longlong(rate));
    if (blockIdx.x == 0 && threadIdx.x == 0 && zero_slot) *zero_slot = 0.0;
}

hipError_t launch_cfl(int prec, const void *y, int N, long long nc, double gamma, const double h[3],
                      double *rate_slot, double *zero_slot, hipStream_t s) {
    const int th = 256;
    const long long nb = (nc + th - 1) / th;
    if (prec == DG_FP64)
        hipLaunchKernelGGL((cfl_kernel<double>), dim3(nb), dim3(th), 0, s, (const double *)y, N, nc, gamma, h[0], h[1],
                           h[2], rate_slot, zero_slot);
    else
        hipLaunchKernelGGL((cfl_kernel<float>), dim3(nb), dim3(th), 0, s, (const float *)y, N, nc, gamma, h[0], h[1],
                           h[2], rate_slot, zero_slot);
    return hipGetLastError();
}

// ------------------------------------------------------------------ conserved totals (fixed order)

constexpr int TOT_THREADS = 256;

template <class S>
__global__ void totals_pass1(const S *__restrict__ y, int N, long long nc, double *partials, int nparts) {
    __shared__ double red[TOT_THREADS];
    const long long chunk = (nc + nparts - 1) / nparts;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = lo + chunk < nc ? lo + chunk : nc;
    for (int i = 0; i < NF; i++) {
        double s = 0.0;
        for (long long c = lo + threadIdx.x; c < hi; c += TOT_THREADS) s += (double)y[((long long)i * N) * nc + c];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = TOT_THREADS / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) partials[(long long)i * nparts + blockIdx.x] = red[0];
        __syncthreads();
    }
}

__global__ void totals_pass2(const double *partials, int nparts, double vol, double *out) {
    __shared__ double red[TOT_THREADS];
    for (int i = 0; i < NF; i++) {
        double s = 0.0;
        for (int j = threadIdx.x; j < nparts; j += TOT_THREADS) s += partials[(long long)i * nparts + j];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = TOT_THREADS / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[i] = vol * red[0];
        __syncthreads();
    }
}

hipError_t launch_totals(int prec, const void *y, int N, long long nc, double vol, double *partials, int nparts,
                         double *out, hipStream_t s) {
    if (prec == DG_FP64)
        hipLaunchKernelGGL((totals_pass1<double>), dim3(nparts), dim3(TOT_THREADS), 0, s, (const double *)y, N, nc,
                           partials, nparts);
    else
        hipLaunchKernelGGL((totals_pass1<float>), dim3(nparts), dim3(TOT_THREADS), 0, s, (const float *)y, N, nc,
                           partials, nparts);
    hipLaunchKernelGGL(totals_pass2, dim3(1), dim3(TOT_THREADS), 0, s, partials, nparts, vol, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ range check

template <class S>
__global__ void range_kernel(const S *__restrict__ y, int N, long long nc, double gamma, int *flag) {
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= nc) return;
    const double rho = (double)y[(0LL * N) * nc + cell];
    const double mx = (double)y[(1LL * N) * nc + cell];
    const double my = (double)y[(2LL * N) * nc + cell];
    const double mz = (double)y[(3LL * N) * nc + cell];
    const double E = (double)y[(4LL * N) * nc + cell];
    const double p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my + mz * mz) / rho);
    const bool ok = rho > 0.0 && p > 0.0 && __builtin_isfinite(p) && __builtin_isfinite(rho);
    if (!ok) atomicOr(flag, 1);
}

hipError_t launch_range_check(int prec, const void *y, int N, long long nc, double gamma, int *flag,
                              hipStream_t s) {
    const int th = 256;
    const long long nb = (nc + th - 1) / th;
    if (prec == DG_FP64)
        hipLaunchKernelGGL((range_kernel<double>), dim3(nb), dim3(th), 0, s, (const double *)y, N, nc, gamma, flag);
    else
        hipLaunchKernelGGL((range_kernel<float>), dim3(nb), dim3(th), 0, s, (const float *)y, N, nc, gamma, flag);
    return hipGetLastError();
}

}  // namespace dgmi
