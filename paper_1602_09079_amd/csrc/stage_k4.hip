// The SSP stage kernel for k = 4 (N = 35 modes, 5^3 volume points, 5^2 points per face) in FP32
// and FP64 on the matrix cores: the quadrature form of the volume and surface integrals (Bauer et
// al., arXiv 1602.09079, Sec. 2.3, eqs. dg:eqn:volume_int and dg:eqn:surface_int, the driving
// source of Sec. 3.1, the Shu-Osher combine of the SSP-RK3 step), with the cells of an x-block as
// the columns of 16x16x4 FP32 / FP64 MFMAs and the basis tables as their A operands:
//
// - One wave per x-block: 16 consecutive cells of a (z, y) row, all updated.  Lane (g, c) holds
//   cell c and, of every field, the modes 4s + g, s = 0..8 (the B operand of the K step s of every
//   product over the modes).  The x faces on the block's edges take the cell before and the cell
//   after from one extra "ghost" product (column 0: the cell before; column 15: the cell after
//   with its odd-x-degree modes negated, which turns the +x trace table into the -x one); the
//   16 points of column 15's +x face are gathered into the lanes of columns 12..15 and solved in
//   one pass.  A ragged last block takes its right neighbour from the wrapped column after the
//   last valid one.
// - Volume, one tile of 16 points at a time: point values (8 tiles of 16 rows over the 125
//   points, 9 K steps), the Euler fluxes and the driving source at the lane's 4 points, then
//   their contraction with the weighted gradients and basis (K = the tile's 16 points, 4 steps).
// - Result rows: the mode of each row is chosen so that register r of lane group g' of row tile t
//   is mode 16t + 4r + g', the modes the lane holds (FP32 results: row 4g' + r; FP64: row g' + 4r).
//   FP32: the last tile (modes 32..34, one row per lane group) runs as 4x4x1 products of 16 blocks
//   (a quarter of the cost) summed across the lane groups at the end.
// - Faces, one tile of 16 points at a time (2 tiles over the 25 points): the traces of the cell
//   and of its neighbour on the face, the Riemann flux at the lane's 4 points, the lift (K = the
//   32 face rows, 8 steps).  x faces: the neighbour is the next column (DPP row shifts), each
//   face inside the block solved once; the block-edge faces and the y and z faces (whose
//   neighbours' traces come from their weights) are solved by both of their cells with the same
//   arithmetic, so that they get the same flux.
// - Padding rows repeat the last point in the trace and value tables (a valid state) and are zero
//   in the tables that take their results, so they add nothing.
// - FP32: the value, gradient, trace and lift tables (153 KiB) sit in LDS, shared by the eight
//   waves (two per SIMD) of the one workgroup per compute unit, the source tables (24 KiB, read
//   only with the driving) through the caches.  FP64: the gradient tables (144 KiB) sit in LDS,
//   the rest is read through the caches, and one wave per SIMD holds the weights and results in
//   512 registers.
//   The waves take x-blocks independently (no barrier after the table copy).

#include "dg_device.h"

namespace dgmi {

namespace {

constexpr int K4_NM = 35, K4_E = NF * K4_NM;
constexpr int k4_threads(int prec) { return prec == DG_FP64 ? 256 : 512; }

// DPP row shifts within 16-lane rows: row_shl:1 (lane c <- lane c + 1), row_shr:1 (lane c <- c - 1)
template <int CTRL>
__device__ inline float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ inline double dpp(double v) {
    const u2 h = __builtin_bit_cast(u2, v);
    const u2 o = {(unsigned)__builtin_amdgcn_update_dpp(0, (int)h.x, CTRL, 0xf, 0xf, true),
                  (unsigned)__builtin_amdgcn_update_dpp(0, (int)h.y, CTRL, 0xf, 0xf, true)};
    return __builtin_bit_cast(double, o);
}
template <int N, class T>
__device__ inline T shl(T v) {
    return dpp<0x100 + N>(v);
}
template <int N, class T>
__device__ inline T shr(T v) {
    return dpp<0x110 + N>(v);
}
// modes with odd x-degree: bit l (k = 4, 35 modes)
constexpr unsigned long long k4_oddu_mask() {
    unsigned long long m = 0;
    for (int l = 0; l < 35; l++)
        if (graded_mode_u(l) & 1) m |= 1ull << l;
    return m;
}
__device__ inline f4 mfma16(float x, float y, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0); }
__device__ inline d4 mfma16(double x, double y, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0); }
// the last row tile: FP32 4x4x1 products of 16 blocks, FP64 a full 16x16x4 product
__device__ inline f4 mfma_last(float x, float y, f4 c) { return __builtin_amdgcn_mfma_f32_4x4x1f32(x, y, c, 0, 0, 0); }
__device__ inline d4 mfma_last(double x, double y, d4 c) { return mfma16(x, y, c); }

}  // namespace

template <int PREC, bool FORCE, int RS>
__global__ __launch_bounds__(k4_threads(PREC))
__attribute__((amdgpu_waves_per_eu(PREC == DG_FP64 ? 1 : 2, PREC == DG_FP64 ? 1 : 2))) void stage_k4_kernel(StageArgs a) {
    constexpr bool F64 = PREC == DG_FP64;
    constexpr int THREADS = k4_threads(PREC);
    using PR = Prec<PREC>;
    using C = typename PR::C;
    using Acc = typename PR::Acc;
    constexpr int ESZ = sizeof(C);
    // the fragments staged in LDS: FP32 all before the source tables, FP64 the gradient tables
    constexpr int L0 = F64 ? K4_GRAD : 0, L1 = F64 ? K4_TRACE : K4_SRC;
    extern __shared__ __attribute__((aligned(16))) char lds[];
    {
        const int4 *src = reinterpret_cast<const int4 *>(static_cast<const char *>(a.tables) + (size_t)L0 * 64 * ESZ);
        int4 *dst = reinterpret_cast<int4 *>(lds);
        for (int j = threadIdx.x; j < (L1 - L0) * 64 * ESZ / 16; j += THREADS) dst[j] = src[j];
        __syncthreads();
    }
    const C *ltab = reinterpret_cast<const C *>(lds);
    const C *gtab = static_cast<const C *>(a.tables);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col = lane & 15;
    const int g = lane >> 4;
    const C gam = (C)a.gamma, g1 = gam - C(1);
    double dtd = a.dt;
    if (a.rate) dtd = a.dtfac / a.rate[0];
    const C dt = (C)dtd;
    if (a.tacc && blockIdx.x == 0 && threadIdx.x == 0) a.tacc[0] += dtd;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long long slabn = (long long)K4_E * nx;  // elements per (z, y) row of cells
    const C *yin = static_cast<const C *>(a.yin);
    const C *y0 = static_cast<const C *>(a.y0);
    C *out = static_cast<C *>(a.out);
    const unsigned mstride = (unsigned)nx * ESZ;  // bytes between modes

    // A operand of one product step (a fragment: one value per lane).  The lane offset is made
    // opaque at each use, so that the compiler forms no per-fragment address to keep (and spill)
    // across the sweep: LDS reads take the fragment as an immediate offset, the lift table's
    // buffer loads as a uniform one
    auto lane_off = [&]() {
        int o = lane;
        asm volatile("" : "+v"(o));
        return o;
    };
    const auto trs = slab_rsrc(gtab, (long long)K4_NFRAG * 64, 0);
    auto A = [&](int frag) -> C {
        if (frag >= L0 && frag < L1) return ltab[(frag - L0) * 64 + lane_off()];
        return bload(C(0), trs, (unsigned)lane_off() * ESZ, (unsigned)frag * 64u * ESZ);
    };
    // the weights of the block in row r of base (modes 4s + g of cell column col at x)
    auto load_b = [&](const C *base, long long r, unsigned xb, C b[NF][9]) {
        const auto rs = slab_rsrc(base, slabn, r);
        const unsigned vo = (unsigned)g * mstride + xb;
#pragma unroll
        for (int i = 0; i < NF; i++)
#pragma unroll
            for (int s = 0; s < 9; s++) b[i][s] = bload(C(0), rs, vo, (unsigned)(i * K4_NM + 4 * s) * mstride);
    };
    // the neighbouring block across a y or z face (the z ends of a slab: the halo planes)
    auto load_nb = [&](int iy, int iz, unsigned xb, C b[NF][9]) {
        iy = iy < 0 ? iy + ny : (iy >= ny ? iy - ny : iy);
        if (a.halo_lo && iz < 0)
            load_b(static_cast<const C *>(a.halo_lo), iy, xb, b);
        else if (a.halo_hi && iz >= nz)
            load_b(static_cast<const C *>(a.halo_hi), iy, xb, b);
        else
            load_b(yin, (long long)(iz < 0 ? iz + nz : (iz >= nz ? iz - nz : iz)) * ny + iy, xb, b);
    };
    // traces of a block on face f, face tile ft (register r: face row 16 ft + 4 g + r in FP32,
    // 16 ft + g + 4 r in FP64)
    auto trace = [&](int f, int ft, const C b[NF][9], C tr[NF][4]) {
        Acc t[NF];
#pragma unroll
        for (int i = 0; i < NF; i++) t[i] = Acc{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 9; s++) {
            const C av = A(K4_TRACE + (f * 2 + ft) * 9 + s);
#pragma unroll
            for (int i = 0; i < NF; i++) t[i] = mfma16(av, b[i][s], t[i]);
        }
#pragma unroll
        for (int i = 0; i < NF; i++)
#pragma unroll
            for (int r = 0; r < 4; r++) tr[i][r] = t[i][r];
    };
    auto riemann = [&](auto axis_c, const C tl[NF][4], const C tr_[NF][4], C Fo[NF][4]) {
        constexpr int AX = decltype(axis_c)::value;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            C qL[5], qR[5], F[5];
#pragma unroll
            for (int i = 0; i < 5; i++) {
                qL[i] = tl[i][r];
                qR[i] = tr_[i][r];
            }
            if constexpr (RS == 1)
                exact_rs<PR, AX>(qL, qR, gam, F);
            else
                hllc<PR, AX>(qL, qR, gam, F);
#pragma unroll
            for (int i = 0; i < 5; i++) Fo[i][r] = F[i];
        }
    };
    // lift of the flux at face tile ft of face f (K steps 4 ft .. 4 ft + 3)
    auto lift = [&](int f, int ft, const C F[NF][4], Acc acc[NF][3]) {
#pragma unroll
        for (int rt = 0; rt < 3; rt++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const C av = A(K4_LIFT + (f * 3 + rt) * 8 + 4 * ft + r);
#pragma unroll
                for (int i = 0; i < NF; i++)
                    acc[i][rt] = rt < 2 ? mfma16(av, F[i][r], acc[i][rt]) : mfma_last(av, F[i][r], acc[i][rt]);
            }
    };
    // FP32: the last row tile's result (4x4x1 blocks: register r of lane group g holds group g's
    // part of mode 32 + r) summed over the lane groups into register 0 (mode 32 + g)
    auto tile_sum = [&](Acc c) -> Acc {
        const bool hi2 = (g & 2) != 0, odd = (g & 1) != 0;
        const C k0 = hi2 ? c[2] : c[0], k1 = hi2 ? c[3] : c[1];
        const C s0 = hi2 ? c[0] : c[2], s1 = hi2 ? c[1] : c[3];
        const C h0 = k0 + __shfl_xor(s0, 32), h1 = k1 + __shfl_xor(s1, 32);
        const C keep = odd ? h1 : h0, send = odd ? h0 : h1;
        c[0] = keep + __shfl_xor(send, 16);
        return c;
    };

    const int nbx = (nx + K4_BLK - 1) / K4_BLK;
    const long long nitems = (long long)nbx * ny * nz;
    for (long long item = (long long)blockIdx.x * (THREADS / 64) + wave; item < nitems;
         item += (long long)gridDim.x * (THREADS / 64)) {
        const int bx = (int)(item % nbx);
        const long long row = item / nbx;
        const int iy = (int)(row % ny), iz = (int)(row / ny);
        const int x0 = bx * K4_BLK;
        const int vc = nx - x0 < K4_BLK ? nx - x0 : K4_BLK;  // valid columns of the block
        int x = x0 + col;
        const bool store = col < vc;
        x = x >= nx ? x % nx : x;  // a ragged block's column vc holds the wrapped right neighbour
        const unsigned xb = (unsigned)x * ESZ;

        C b[NF][9];
        load_b(yin, row, xb, b);
        Acc acc[NF][3];
#pragma unroll
        for (int i = 0; i < NF; i++)
#pragma unroll
            for (int rt = 0; rt < 3; rt++) acc[i][rt] = Acc{0, 0, 0, 0};

        // ---- volume: one tile of 16 points at a time (register r: point 16 t + 4 g + r in FP32,
        // 16 t + g + 4 r in FP64, the layout of the driving cache)
        const Acc *ac = FORCE ? reinterpret_cast<const Acc *>(a.acache) + row * (96LL * nx) : nullptr;
#pragma unroll 1
        for (int t = 0; t < 8; t++) {
            Acc d[NF];
#pragma unroll
            for (int i = 0; i < NF; i++) d[i] = Acc{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < 9; s++) {
                const C av = A(K4_PHI + t * 9 + s);
#pragma unroll
                for (int i = 0; i < NF; i++) d[i] = mfma16(av, b[i][s], d[i]);
            }
            Acc acv[3];
            if constexpr (FORCE) {
#pragma unroll
                for (int c = 0; c < 3; c++) acv[c] = ac[((t * 3 + c) * 4 + g) * nx + x];
            }
            C rho[4], u[4], v[4], w[4], p[4], ep[4];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                rho[r] = d[0][r];
                const C inv = PR::rcp(rho[r]);
                u[r] = d[1][r] * inv;
                v[r] = d[2][r] * inv;
                w[r] = d[3][r] * inv;
                p[r] = g1 * (d[4][r] - C(0.5) * (d[1][r] * u[r] + d[2][r] * v[r] + d[3][r] * w[r]));
                ep[r] = d[4][r] + p[r];
            }
            // the three directional fluxes, each contracted with its gradient table
#pragma unroll
            for (int dd = 0; dd < 3; dd++) {
                C F[NF][4];
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const C vel = dd == 0 ? u[r] : (dd == 1 ? v[r] : w[r]);
                    F[0][r] = d[1 + dd][r];
                    F[1][r] = d[1][r] * vel + (dd == 0 ? p[r] : C(0));
                    F[2][r] = d[2][r] * vel + (dd == 1 ? p[r] : C(0));
                    F[3][r] = d[3][r] * vel + (dd == 2 ? p[r] : C(0));
                    F[4][r] = ep[r] * vel;
                }
#pragma unroll
                for (int rt = 0; rt < 3; rt++)
#pragma unroll
                    for (int s = 0; s < 4; s++) {
                        const C av = A(K4_GRAD + ((t * 3 + dd) * 3 + rt) * 4 + s);
#pragma unroll
                        for (int i = 0; i < NF; i++)
                            acc[i][rt] = rt < 2 ? mfma16(av, F[i][s], acc[i][rt]) : mfma_last(av, F[i][s], acc[i][rt]);
                    }
            }
            if constexpr (FORCE) {
                C S[4][4];  // rho a_c and m . a at the points
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    S[0][r] = rho[r] * acv[0][r];
                    S[1][r] = rho[r] * acv[1][r];
                    S[2][r] = rho[r] * acv[2][r];
                    S[3][r] = d[1][r] * acv[0][r] + d[2][r] * acv[1][r] + d[3][r] * acv[2][r];
                }
#pragma unroll
                for (int rt = 0; rt < 3; rt++)
#pragma unroll
                    for (int s = 0; s < 4; s++) {
                        const C av = A(K4_SRC + (t * 3 + rt) * 4 + s);
#pragma unroll
                        for (int c = 0; c < 4; c++)
                            acc[1 + c][rt] =
                                rt < 2 ? mfma16(av, S[c][s], acc[1 + c][rt]) : mfma_last(av, S[c][s], acc[1 + c][rt]);
                    }
            }
        }

        // phase boundaries: the memory clobber keeps each phase's loads in it (hoisted loads hold
        // registers across the phases before them)
        asm volatile("" ::: "memory");
        // ---- x faces: the - face of column c between columns c - 1 and c; the + face of c is the
        // - face of c + 1.  The cells before and after the block from one "ghost" product: column 0
        // holds the cell before, column 15 the cell after with its odd-x-degree modes negated, which
        // turns the +x trace table into the -x one
        C tg[2][NF][4];
        {
            C bg[NF][9];
            const int xa = x0 == 0 ? nx - 1 : x0 - 1, xr = x0 + K4_BLK;
            const int xz = col < 8 ? xa : (xr >= nx ? xr % nx : xr);
            load_b(yin, row, (unsigned)xz * ESZ, bg);
            constexpr unsigned long long odd = k4_oddu_mask();
#pragma unroll
            for (int s = 0; s < 9; s++) {
                const bool neg = col >= 8 && ((odd >> (4 * s + g)) & 1ull);
#pragma unroll
                for (int i = 0; i < NF; i++) bg[i][s] = neg ? -bg[i][s] : bg[i][s];
            }
            trace(1, 0, bg, tg[0]);
            trace(1, 1, bg, tg[1]);
        }
        const bool full = vc == K4_BLK;
#pragma unroll
        for (int ft = 0; ft < 2; ft++) {
            C tl[NF][4], fo[5];
            {
                C tp[NF][4];
                trace(1, ft, b, tp);
                if (full) {
                    // the + face of column 15: its 4 points of this lane group, one per lane of
                    // columns 12..15, solved in one pass
                    C ql[5], qr[5];
#pragma unroll
                    for (int i = 0; i < NF; i++) {
                        const C l1 = shl<1>(tp[i][1]), l2 = shl<2>(tp[i][2]), l3 = shl<3>(tp[i][3]);
                        const C r1 = shl<1>(tg[ft][i][1]), r2 = shl<2>(tg[ft][i][2]), r3 = shl<3>(tg[ft][i][3]);
                        const C dflt = i == 0 ? C(1) : (i == 4 ? C(2) : C(0));  // lanes without a point
                        ql[i] = col == 15 ? tp[i][0] : (col == 14 ? l1 : (col == 13 ? l2 : (col == 12 ? l3 : dflt)));
                        qr[i] = col == 15 ? tg[ft][i][0] : (col == 14 ? r1 : (col == 13 ? r2 : (col == 12 ? r3 : dflt)));
                    }
                    if constexpr (RS == 1)
                        exact_rs<PR, 0>(ql, qr, gam, fo);
                    else
                        hllc<PR, 0>(ql, qr, gam, fo);
                }
#pragma unroll
                for (int i = 0; i < NF; i++)
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const C sh = shr<1>(tp[i][r]);  // DPP outside any select: every lane active
                        tl[i][r] = col == 0 ? tg[ft][i][r] : sh;
                    }
            }
            C Fm[NF][4];
            {
                C tr[NF][4];
                trace(0, ft, b, tr);
                riemann(std::integral_constant<int, 0>{}, tl, tr, Fm);
            }
            lift(0, ft, Fm, acc);
#pragma unroll
            for (int i = 0; i < NF; i++) {
#pragma unroll
                for (int r = 0; r < 4; r++) Fm[i][r] = shl<1>(Fm[i][r]);  // the + face: column c + 1's - face
                if (full) {
                    const C f1 = shr<1>(fo[i]), f2 = shr<2>(fo[i]), f3 = shr<3>(fo[i]);
                    if (col == 15) {
                        Fm[i][0] = fo[i];
                        Fm[i][1] = f1;
                        Fm[i][2] = f2;
                        Fm[i][3] = f3;
                    }
                }
            }
            lift(1, ft, Fm, acc);
        }
        // ---- y and z faces: side 0 the - face (the neighbour on the left), side 1 the + face
        auto face = [&](auto axis_c, int side) {
            constexpr int AX = decltype(axis_c)::value;
            const int f = 2 * AX + side;
            asm volatile("" ::: "memory");
            C tn[2][NF][4];
            {
                C bn[NF][9];
                const int dy = AX == 1 ? (side ? 1 : -1) : 0, dz = AX == 2 ? (side ? 1 : -1) : 0;
                load_nb(iy + dy, iz + dz, xb, bn);
                trace(f ^ 1, 0, bn, tn[0]);
                trace(f ^ 1, 1, bn, tn[1]);
            }
#pragma unroll
            for (int ft = 0; ft < 2; ft++) {
                C to[NF][4], F[NF][4];
                trace(f, ft, b, to);
                if (side)
                    riemann(axis_c, to, tn[ft], F);
                else
                    riemann(axis_c, tn[ft], to, F);
                lift(f, ft, F, acc);
            }
        };
        face(std::integral_constant<int, 1>{}, 0);
        face(std::integral_constant<int, 1>{}, 1);
        face(std::integral_constant<int, 2>{}, 0);
        face(std::integral_constant<int, 2>{}, 1);

        asm volatile("" ::: "memory");
        // ---- combine and store: result register r of row tile t is mode 16 t + 4 r + g, which
        // this lane holds in b[i][4 t + r]
        if constexpr (!F64) {
#pragma unroll
            for (int i = 0; i < NF; i++) acc[i][2] = tile_sum(acc[i][2]);
        }
        if (store) {
            const auto ro = slab_rsrc(out, slabn, row);
            const unsigned vo = (unsigned)g * mstride + xb;
            if (a.mode == 0) {
#pragma unroll
                for (int i = 0; i < NF; i++)
#pragma unroll
                    for (int s = 0; s < 9; s++) {
                        if (s == 8 && g == 3) continue;
                        bstore(acc[i][s / 4][s % 4], ro, vo, (unsigned)(i * K4_NM + 4 * s) * mstride);
                    }
            } else {
                const C ca = (C)a.a, cb = (C)a.b;
                const bool with_y0 = a.a != 0.0;
                const auto r0 = slab_rsrc(with_y0 ? y0 : yin, slabn, row);
#pragma unroll
                for (int i = 0; i < NF; i++)
#pragma unroll
                    for (int s = 0; s < 9; s++) {
                        if (s == 8 && g == 3) continue;
                        const unsigned so = (unsigned)(i * K4_NM + 4 * s) * mstride;
                        const C base = cb * (b[i][s] - dt * acc[i][s / 4][s % 4]);
                        const C res = with_y0 ? ca * bload(C(0), r0, vo, so) + base : base;
                        bstore(res, ro, vo, so);
                    }
            }
        }
    }
}

template <int PREC, bool FORCE, int RS>
static const void *k4_fn() {
    return reinterpret_cast<const void *>(&stage_k4_kernel<PREC, FORCE, RS>);
}

template <int PREC>
static hipError_t launch_k4_t(const StageArgs &a, int grid, hipStream_t s) {
    constexpr int T = k4_threads(PREC);
    const int lds = k4_lds_bytes(PREC);
    if (a.riemann == 1) {
        if (a.forcing)
            hipLaunchKernelGGL((stage_k4_kernel<PREC, true, 1>), dim3(grid), dim3(T), lds, s, a);
        else
            hipLaunchKernelGGL((stage_k4_kernel<PREC, false, 1>), dim3(grid), dim3(T), lds, s, a);
    } else {
        if (a.forcing)
            hipLaunchKernelGGL((stage_k4_kernel<PREC, true, 0>), dim3(grid), dim3(T), lds, s, a);
        else
            hipLaunchKernelGGL((stage_k4_kernel<PREC, false, 0>), dim3(grid), dim3(T), lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_stage_k4(int prec, const StageArgs &a, int grid, hipStream_t s) {
    if (prec == DG_FP32) return launch_k4_t<DG_FP32>(a, grid, s);
    if (prec == DG_FP64) return launch_k4_t<DG_FP64>(a, grid, s);
    return hipErrorInvalidValue;
}

template <int PREC>
static hipError_t set_attr_k4_t() {
    const void *fns[] = {k4_fn<PREC, false, 0>(), k4_fn<PREC, true, 0>(), k4_fn<PREC, false, 1>(),
                         k4_fn<PREC, true, 1>()};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, k4_lds_bytes(PREC));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t set_stage_k4_attributes(int prec) {
    if (prec == DG_FP32) return set_attr_k4_t<DG_FP32>();
    if (prec == DG_FP64) return set_attr_k4_t<DG_FP64>();
    return hipErrorInvalidValue;
}

}  // namespace dgmi
