// HIP kernels of libdgmi.so for gfx950 (MI355X).
//
// The fused SSP stage kernel evaluates the modal DG operator of Bauer et al.
// (arXiv 1602.09079), Sec. 2.3, on blocks of 16 cells that are consecutive in
// x.  Every basis contraction is a dense GEMM over cells on the matrix cores:
//
//   GEMM1  q(xi_q)        = Phi[q][l]           * w[l][cell]        (modal -> volume points)
//   GEMM2  R[l]          += -s_a dPhi_a[l][q] w_q * (F_a(q) - F_a(qbar))  (eq. dg:eqn:volume_int)
//   GEMM3  q(face point)  = Phif[p][l]          * w[l][cell]        (traces on the six faces)
//   GEMM4  R[l]          += s_a (+-) Phif[l][p] w_p * (Fhat - F_a(qbar))  (eq. dg:eqn:surface_int)
//   GEMM5  R[l]          -= Phi[l][q] w_q / 8   * S(q)              (driving source, Sec. 3.1)
//
// The 16 cells are the columns of each MFMA tile.  The result registers of
// GEMM1 and GEMM3 are fed directly as B operands of GEMM2 and GEMM4: the
// contraction index of the tables is permuted on the host to match the result
// lane layout, so no data moves between the chained products.  The Euler flux
// and the HLLC Riemann solver run on the vector ALUs in that same layout.
//
// Deviation form: mode 0 (the cell mean qbar) is kept out of the products and
// added back in full precision, and the cell-mean flux F(qbar) is subtracted from
// every volume and face flux before projection.  The subtracted terms cancel
// exactly because the Gauss rules integrate the basis derivatives and the face
// traces exactly, so the operator is unchanged while reduced-precision rounding
// acts on the in-cell variation instead of the mean.
//
// Faces: the x-neighbour of a column is the adjacent lane of its 16-lane row
// (DPP row shifts); columns 0 and 15 of a block are halo cells whose results are
// discarded (consecutive blocks overlap by two cells).  Each wave sweeps a chunk
// of blocks along z, loading block z+1 while it computes block z; the flux on
// the face between them is computed once and carried to the next step.  The
// y-neighbour traces come from the neighbouring rows' weights (through L2) with
// the same GEMM3 tables, so a face flux is computed from bitwise identical inputs
// on both sides.
//
// Persistent grid: the work items (x-block, y row, z chunk) are split into 8
// contiguous ranges, one per XCD (workgroup id modulo 8), so the rows a wave
// reads as y-neighbours were recently loaded into the same XCD's L2.

#include <type_traits>

#include "dg_device.h"

namespace dgmi {

// ------------------------------------------------------------------ table geometry (matches make_layout)

template <int K, int PREC>
struct StageCfg {
    using D = Dims<K>;
    using PR = Prec<PREC>;
    static constexpr int N = D::N, Q = D::Q, P = D::P;
    static constexpr int KPL = PR::KPL, KPL2 = PR::KPL2, KSTEP = PR::KSTEP;
    static constexpr int KS1 = (N + KSTEP - 1) / KSTEP;
    static constexpr int RT1 = (Q + 15) / 16;
    static constexpr int RT2 = (N + 15) / 16;
    static constexpr int NC2 = KPL2 == 4 ? RT1 : RT1 * 4;
    static constexpr int NC4 = KPL2 == 4 ? 6 : 24;
    static constexpr int FB1 = 64 * KPL * PR::ESZ, FB2 = 64 * KPL2 * PR::ESZ;
    static constexpr int O1 = 0;
    static constexpr int O2 = O1 + RT1 * KS1 * FB1;
    static constexpr int O3 = O2 + RT2 * 3 * NC2 * FB2;
    static constexpr int O4 = O3 + 6 * KS1 * FB1;
    static constexpr int O5 = O4 + RT2 * NC4 * FB2;
    static constexpr int SET = O5 + RT2 * NC2 * FB2;
    static constexpr int NTAB = PREC == DG_BF16X3 ? 2 : 1;
    static constexpr bool QFULL = (Q % 16) == 0;  // no padded volume rows
    static constexpr bool PFULL = P == 16;        // no padded face rows
};

// Reads A-operand fragments from the LDS copy of the tables.  refresh() hides the
// lane offset from loop-invariant code motion so fragments are re-read where they
// are used instead of being hoisted into (and exhausting) the register file.
template <int K, int PREC>
struct TabReader {
    using SC = StageCfg<K, PREC>;
    using PR = Prec<PREC>;
    const char *lds;
    int off1, off2;  // this lane's byte offset inside a wide / narrow fragment
    __device__ void refresh() {
        asm volatile("" : "+v"(off1));
        asm volatile("" : "+v"(off2));
    }
    __device__ typename PR::AF wide(int byte) const {
        if constexpr (PREC == DG_BF16X3)
            return typename PR::AF{*reinterpret_cast<const bf8 *>(lds + byte + off1),
                                   *reinterpret_cast<const bf8 *>(lds + SC::SET + byte + off1)};
        else
            return PR::lda(lds + byte + off1);
    }
    __device__ typename PR::AF2 narrow(int byte) const {
        if constexpr (PREC == DG_BF16X3)
            return typename PR::AF2{*reinterpret_cast<const bf4 *>(lds + byte + off2),
                                    *reinterpret_cast<const bf4 *>(lds + SC::SET + byte + off2)};
        else
            return PR::lda2(lds + byte + off2);
    }
    __device__ typename PR::AF t1(int t, int s) const { return wide(SC::O1 + (t * SC::KS1 + s) * SC::FB1); }
    __device__ typename PR::AF2 t2(int rt, int al, int c) const {
        return narrow(SC::O2 + ((rt * 3 + al) * SC::NC2 + c) * SC::FB2);
    }
    __device__ typename PR::AF t3(int f, int s) const { return wide(SC::O3 + (f * SC::KS1 + s) * SC::FB1); }
    __device__ typename PR::AF2 t4(int rt, int c) const { return narrow(SC::O4 + (rt * SC::NC4 + c) * SC::FB2); }
    __device__ typename PR::AF2 t5(int rt, int c) const { return narrow(SC::O5 + (rt * SC::NC2 + c) * SC::FB2); }
};

// Workgroup size: 8 waves sharing y faces (FP32-storage tiers), 4 independent waves (FP64).
template <int PREC>
constexpr int stage_threads() { return PREC == DG_FP64 ? 256 : 64 * YROWS; }

// Waves per SIMD the stage kernel is compiled for (register budget 512 / this):
// two for the FP32-storage tiers, one for FP64, whose doubles need the full file.
template <int PREC>
constexpr int stage_waves_per_eu() { return PREC == DG_FP64 ? 1 : 2; }

// The weights of one block of 16 cells in B-operand layout, without mode 0,
// plus the cell means in full precision.
template <int K, int PREC>
struct Blk {
    // FP32/FP64: the B operands are the weights themselves.  BF16 tiers: the raw weights of the
    // lane's mode slots; the (split) BF16 operands are formed where they are used, which keeps
    // fewer registers live than holding the converted copy, and keeps the FP32 values for the combine.
    static constexpr bool RAW = Prec<PREC>::KPL != 1;
    typename Prec<PREC>::BF w[NF][RAW ? 1 : StageCfg<K, PREC>::KS1];
    typename Prec<PREC>::C v[NF][RAW ? mode_slots(Dims<K>::N) : 1];
    typename Prec<PREC>::C qbar[NF];
};


// Acceleration cache: per slab [tile t][component c][lane group g][x][r] holds a_c at volume
// point 16 t + orow(g, r) of cell x, so a lane reads its 4 values of a tile with one 16-byte load.
__device__ inline void accel_load(__amdgpu_buffer_rsrc_t r, unsigned off, float v[4]) {
    // the whole 16-byte vector is reinterpreted at once (casting its elements one by one lets the
    // compiler narrow the load to one dword)
    const f4 w = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
#pragma unroll
    for (int j = 0; j < 4; j++) v[j] = w[j];
}
__device__ inline void accel_load(__amdgpu_buffer_rsrc_t r, unsigned off, double v[4]) {
    typedef double dv2 __attribute__((ext_vector_type(2)));
    const dv2 w0 = __builtin_bit_cast(dv2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    const dv2 w1 = __builtin_bit_cast(dv2, __builtin_amdgcn_raw_buffer_load_b128(r, off + 16, 0, 0));
    v[0] = w0[0];
    v[1] = w0[1];
    v[2] = w1[0];
    v[3] = w1[1];
}

template <int K, int PREC, bool FORCE, int RS>
__global__ __launch_bounds__(stage_threads<PREC>()) __attribute__((amdgpu_waves_per_eu(stage_waves_per_eu<PREC>(), stage_waves_per_eu<PREC>()))) void stage_kernel(StageArgs a) {
    using SC = StageCfg<K, PREC>;
    using PR = typename SC::PR;
    using C = typename PR::C;
    using S = typename PR::S;
    using Acc = typename PR::Acc;
    using B = Blk<K, PREC>;
    constexpr int N = SC::N, Q = SC::Q, P = SC::P;
    constexpr int KPL = SC::KPL, KPL2 = SC::KPL2, KSTEP = SC::KSTEP, KS1 = SC::KS1;
    constexpr int RT1 = SC::RT1, RT2 = SC::RT2;
    constexpr int SPL = mode_slots(N);               // mode slots per lane group
    constexpr int THREADS = stage_threads<PREC>();
    constexpr bool YSH = PREC != DG_FP64;             // workgroup rows share y faces through LDS
    static_assert(KPL == 1 ? KS1 == SPL : (KS1 == 1 && SPL <= KPL), "mode slots must fit the B operands");
    static_assert(4 * RT2 >= SPL, "mode slots must fit the result rows");

    extern __shared__ __attribute__((aligned(16))) char lds[];
    {
        const int bytes = SC::SET * SC::NTAB;
        const int4 *src = reinterpret_cast<const int4 *>(a.tables);
        int4 *dst = reinterpret_cast<int4 *>(lds);
        for (int j = threadIdx.x; j < bytes / 16; j += THREADS) dst[j] = src[j];
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    // LDS exchange addresses: one lane base, made opaque at each use, plus immediate offsets (the
    // compiler would otherwise hoist a register per element out of the sweep and spill them)
    auto lane_base = [&]() {
        int o = lane;
        asm volatile("" : "+v"(o));
        return o;
    };
    const int col = lane & 15;
    const int g = lane >> 4;
    TabReader<K, PREC> T{lds, lane * KPL * PR::ESZ, lane * KPL2 * PR::ESZ};

    const C gam = (C)a.gamma;
    const C g1 = gam - C(1);
    double dtd = a.dt;
    if (a.rate) dtd = a.dtfac / a.rate[0];
    const C dt = (C)dtd;
    if (a.tacc && blockIdx.x == 0 && threadIdx.x == 0) a.tacc[0] += dtd;
    const S *yin = reinterpret_cast<const S *>(a.yin);
    const S *y0 = reinterpret_cast<const S *>(a.y0);
    S *out = reinterpret_cast<S *>(a.out);
    const long long nc = a.ncells;
    const long long slabn = (long long)NF * N * a.nx;  // elements per (z, y) slab
    const long long aslab = (long long)RT1 * 16 * 3 * a.nx;  // elements per slab of the acceleration cache
    const unsigned nxu = (unsigned)a.nx;
    const int nx = a.nx, ny = a.ny, nz = a.nz;

    // ---------------- building blocks
    // Per-lane byte offsets of the rows this lane feeds to the B operand: the
    // modes of its slots (slot_mode); unused slots are clamped to the last mode
    // and meet zero table entries, as does mode 0 (the mean enters apart).
    // The same rows are the ones this lane's results belong to.
    unsigned boff[KS1][KPL];
    unsigned xoff = 0;
    const unsigned esz = (unsigned)sizeof(S);
    const unsigned fbytes = (unsigned)N * nxu * esz;  // one field of a slab
    auto set_lane_offsets = [&](int xc) {
        xoff = (unsigned)xc * esz;
#pragma unroll
        for (int s = 0; s < KS1; s++)
#pragma unroll
            for (int j = 0; j < KPL; j++) {
                const int m = KPL == 1 ? slot_mode(N, g, s) : slot_mode(N, g, j);
                boff[s][j] = (unsigned)(m < N ? m : N - 1) * nxu * esz + xoff;
            }
    };
    // the block of slab r (wave-uniform) whose first column is at x = xc
    auto load_from = [&](const S *base, long long r, B &b) {
        const auto rs = slab_rsrc(base, slabn, r);
#pragma unroll
        for (int i = 0; i < NF; i++) {
            const unsigned so = (unsigned)i * fbytes;
            b.qbar[i] = (C)bload(S(), rs, xoff, so);
            if constexpr (B::RAW) {
#pragma unroll
                for (int s = 0; s < SPL; s++) b.v[i][s] = (C)bload(S(), rs, boff[0][s], so);
            } else {
#pragma unroll
                for (int s = 0; s < KS1; s++) {
                    C v[KPL];
#pragma unroll
                    for (int j = 0; j < KPL; j++) v[j] = (C)bload(S(), rs, boff[s][j], so);
                    b.w[i][s] = PR::mkb(v);
                }
            }
        }
    };
    auto load = [&](long long r, B &b) { load_from(yin, r, b); };
    // the block in z plane zz of y row yy: across the ends of a z slab from the halo planes (one
    // plane of the neighbouring slab each, [y][i][l][x]) when they are given, else periodic
    auto loadz = [&](int yy, int zz, B &b) {
        yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
        if (a.halo_lo && zz < 0)
            load_from(static_cast<const S *>(a.halo_lo), yy, b);
        else if (a.halo_hi && zz >= nz)
            load_from(static_cast<const S *>(a.halo_hi), yy, b);
        else
            load_from(yin, (long long)(zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz)) * ny + yy, b);
    };
    // end rows of the y group (waves 0 and nact-1): copied into LDS by buffer loads one step ahead
    constexpr int ERV = NF * (1 + SPL);  // values per lane of a block: the mean and the slots, per field
    const bool erows = YSH && a.ex_off3 >= 0;
    C *ex_e = reinterpret_cast<C *>(lds + (a.ex_off3 >= 0 ? a.ex_off3 : 0));
    // the block of slab r copied into LDS buffer e (0: the row below the group, 1: the row above)
    auto load_lds = [&](long long r, int e) {
      if constexpr (YSH) {
        const auto rs = slab_rsrc(yin, slabn, r);
        C *dst = ex_e + e * ERV * 64;
#pragma unroll
        for (int i = 0; i < NF; i++) {
            const int so = (int)((unsigned)i * fbytes);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rs, (__attribute__((address_space(3))) void *)(dst + (i * (1 + SPL)) * 64), (int)sizeof(S), xoff, so, 0,
                0);
#pragma unroll
            for (int s = 0; s < SPL; s++) {
                const unsigned vo = KPL == 1 ? boff[s][0] : boff[0][s];
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rs, (__attribute__((address_space(3))) void *)(dst + (i * (1 + SPL) + 1 + s) * 64), (int)sizeof(S),
                    vo, so, 0, 0);
            }
        }
      }
    };
    auto read_lds = [&](int e, B &b) {
      if constexpr (YSH) {
        // vmcnt(0): the copies have landed (the compiler does not track them); the memory clobber keeps
        // the LDS reads below the wait
        __builtin_amdgcn_s_waitcnt(0x0F70);
        asm volatile("" ::: "memory");
        const C *src = ex_e + e * ERV * 64 + lane_base();
#pragma unroll
        for (int i = 0; i < NF; i++) {
            b.qbar[i] = src[(i * (1 + SPL)) * 64];
#pragma unroll
            for (int s = 0; s < SPL; s++) {
                const C v = src[(i * (1 + SPL) + 1 + s) * 64];
                if constexpr (B::RAW) {
                    b.v[i][s] = v;
                } else {
                    C vv[KPL];
                    vv[0] = v;
                    b.w[i][s] = PR::mkb(vv);
                }
            }
        }
      }
    };
    // B operand of field i, K-step s of a block (converted here for the BF16 tiers)
    auto bop = [&](const B &b, int i, int s) -> typename PR::BF {
        if constexpr (B::RAW) {
            // an empty asm on the copies keeps each use's conversion from being merged with the
            // others (which would hold the converted copy live across the whole step)
            C v[KPL];
#pragma unroll
            for (int j = 0; j < KPL; j++) {
                v[j] = j < SPL ? b.v[i][j] : C(0);
                if (j < SPL) asm volatile("" : "+v"(v[j]));
            }
            return PR::mkb(v);
        } else {
            return b.w[i][s];
        }
    };
    auto trace = [&](const B &b, int face, C tr[NF][4]) {
        Acc t[NF];
#pragma unroll
        for (int i = 0; i < NF; i++) t[i] = Acc{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS1; s++) {
            const auto A = T.t3(face, s);
#pragma unroll
            for (int i = 0; i < NF; i++) t[i] = PR::mma(t[i], A, bop(b, i, s));
        }
#pragma unroll
        for (int i = 0; i < NF; i++)
#pragma unroll
            for (int r = 0; r < 4; r++) tr[i][r] = (C)t[i][r] + b.qbar[i];
    };
    auto riemann = [&](auto axis_c, const C tl[NF][4], const C tr_[NF][4], C Fo[NF][4]) {
        constexpr int AX = decltype(axis_c)::value;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const bool valid = SC::PFULL || PR::orow(g, r) < P;
            C qL[5], qR[5], F[5];
#pragma unroll
            for (int i = 0; i < 5; i++) {
                qL[i] = valid ? tl[i][r] : C(i == 0 ? 1 : (i == 4 ? 2 : 0));
                qR[i] = valid ? tr_[i][r] : C(i == 0 ? 1 : (i == 4 ? 2 : 0));
            }
            if constexpr (RS == 1)
                exact_rs<PR, AX>(qL, qR, gam, F);
            else
                hllc<PR, AX>(qL, qR, gam, F);
#pragma unroll
            for (int i = 0; i < 5; i++) Fo[i][r] = F[i];
        }
    };
    // the cell-mean flux along one axis (recomputed where needed, to save registers)
    auto mean_flux = [&](const B &b, int axis, C Fb[5]) {
        C F3[3][5];
        euler_flux3<PR>(b.qbar, g1, F3);
#pragma unroll
        for (int i = 0; i < 5; i++) Fb[i] = F3[axis][i];
    };
    // lift of one face flux (face = 2*axis + side) minus the cell-mean flux, GEMM4
    auto lift = [&](int face, const B &b, const C Fh[NF][4], Acc acc[NF][RT2]) {
        C Fb[5];
        mean_flux(b, face >> 1, Fb);
        C v[NF][4];
#pragma unroll
        for (int i = 0; i < NF; i++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const bool valid = SC::PFULL || PR::orow(g, r) < P;
                v[i][r] = valid ? Fh[i][r] - Fb[i] : C(0);
            }
        if constexpr (KPL2 == 1) {
#pragma unroll
            for (int r = 0; r < 4; r++)
#pragma unroll
                for (int rt = 0; rt < RT2; rt++) {
                    const auto A = T.t4(rt, face * 4 + r);
#pragma unroll
                    for (int i = 0; i < NF; i++) acc[i][rt] = PR::mma2(acc[i][rt], A, PR::mkb2(&v[i][r]));
                }
        } else {
#pragma unroll
            for (int i = 0; i < NF; i++) {
                const auto bf = PR::mkb2(v[i]);
#pragma unroll
                for (int rt = 0; rt < RT2; rt++) acc[i][rt] = PR::mma2(acc[i][rt], T.t4(rt, face), bf);
            }
        }
    };
    // volume integral: GEMM1 -> flux deviation -> GEMM2, one 16-point tile at a time; with the
    // driving (Sec. 3.1) the source S = (0, rho a, m.a) at the same points is projected by GEMM5
    // (T5 = -phi w / 8), a(x_q) read from the acceleration cache of the row (slab ar)
    // this lane's 4 points of tile t: a_c at point 16 t + orow(g, r); the offset passes an empty asm
    // so the loads are issued where this is called, not hoisted for every tile
    auto accel_tile = [&](__amdgpu_buffer_rsrc_t ar, int t, C av[3][4]) {
        unsigned ao = ((t * 3) * 4 + g) * nxu * 4 * esz + xoff * 4;
        asm volatile("" : "+v"(ao));
#pragma unroll
        for (int c = 0; c < 3; c++) accel_load(ar, ao + c * 4 * nxu * 4 * esz, av[c]);
    };
    // av holds tile 0 on entry (loaded early by the caller); tile t + 1 is requested once tile t's
    // source is done, so its latency hides behind tile t's fluxes
    auto volume = [&](const B &b, Acc acc[NF][RT2], __amdgpu_buffer_rsrc_t ar, C av[3][4]) {
        C Fb[3][5];
        euler_flux3<PR>(b.qbar, g1, Fb);
#pragma unroll
        for (int t = 0; t < RT1; t++) {
            Acc d[NF];
#pragma unroll
            for (int i = 0; i < NF; i++) d[i] = Acc{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KS1; s++) {
                const auto A = T.t1(t, s);
#pragma unroll
                for (int i = 0; i < NF; i++) d[i] = PR::mma(d[i], A, bop(b, i, s));
            }
            // primitive quantities at this lane's 4 points of the tile
            C mx[4], my[4], mz[4], ep[4], vel[3][4], p[4], rho_pt[4];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const bool valid = SC::QFULL || 16 * t + PR::orow(g, r) < Q;
                C q[5];
#pragma unroll
                for (int i = 0; i < 5; i++) q[i] = valid ? (C)d[i][r] + b.qbar[i] : b.qbar[i];
                const C inv = PR::rcp(q[0]);
                rho_pt[r] = q[0];
                mx[r] = q[1]; my[r] = q[2]; mz[r] = q[3];
                vel[0][r] = q[1] * inv; vel[1][r] = q[2] * inv; vel[2][r] = q[3] * inv;
                p[r] = g1 * (q[4] - C(0.5) * (q[1] * vel[0][r] + q[2] * vel[1][r] + q[3] * vel[2][r]));
                ep[r] = q[4] + p[r];
            }
            if constexpr (FORCE) {
                C Sv[4][4];
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const bool valid = SC::QFULL || 16 * t + PR::orow(g, r) < Q;
                    const C rho = rho_pt[r];
                    Sv[0][r] = valid ? rho * av[0][r] : C(0);
                    Sv[1][r] = valid ? rho * av[1][r] : C(0);
                    Sv[2][r] = valid ? rho * av[2][r] : C(0);
                    Sv[3][r] = valid ? mx[r] * av[0][r] + my[r] * av[1][r] + mz[r] * av[2][r] : C(0);
                }
                if constexpr (KPL2 == 1) {
#pragma unroll
                    for (int r = 0; r < 4; r++)
#pragma unroll
                        for (int rt = 0; rt < RT2; rt++) {
                            const auto A = T.t5(rt, t * 4 + r);
#pragma unroll
                            for (int i = 1; i < NF; i++)
                                acc[i][rt] = PR::mma2(acc[i][rt], A, PR::mkb2(&Sv[i - 1][r]));
                        }
                } else {
#pragma unroll
                    for (int i = 1; i < NF; i++) {
                        const auto bf = PR::mkb2(Sv[i - 1]);
#pragma unroll
                        for (int rt = 0; rt < RT2; rt++) acc[i][rt] = PR::mma2(acc[i][rt], T.t5(rt, t), bf);
                    }
                }
                if (t + 1 < RT1) accel_tile(ar, t + 1, av);
            }
#pragma unroll
            for (int al = 0; al < 3; al++) {
                C F[5][4];
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const bool valid = SC::QFULL || 16 * t + PR::orow(g, r) < Q;
                    C f[5];
                    f[0] = al == 0 ? mx[r] : (al == 1 ? my[r] : mz[r]);
                    f[1] = mx[r] * vel[al][r];
                    f[2] = my[r] * vel[al][r];
                    f[3] = mz[r] * vel[al][r];
                    f[1 + al] += p[r];
                    f[4] = ep[r] * vel[al][r];
#pragma unroll
                    for (int i = 0; i < 5; i++) F[i][r] = valid ? f[i] - Fb[al][i] : C(0);
                }
                if constexpr (KPL2 == 1) {
#pragma unroll
                    for (int r = 0; r < 4; r++)
#pragma unroll
                        for (int rt = 0; rt < RT2; rt++) {
                            const auto A = T.t2(rt, al, t * 4 + r);
#pragma unroll
                            for (int i = 0; i < NF; i++) acc[i][rt] = PR::mma2(acc[i][rt], A, PR::mkb2(&F[i][r]));
                        }
                } else {
#pragma unroll
                    for (int i = 0; i < NF; i++) {
                        const auto bf = PR::mkb2(F[i]);
#pragma unroll
                        for (int rt = 0; rt < RT2; rt++) acc[i][rt] = PR::mma2(acc[i][rt], T.t2(rt, al, t), bf);
                    }
                }
            }
        }
    };

    // y-face exchange in LDS (after the tables): a trace region and a flux region of one slot per
    // wave (5 x 4 values per lane).  When the two regions do not both fit, they coincide and two
    // more barriers order the reuse (a.ex_single).
    C *ex_t = reinterpret_cast<C *>(lds + a.ex_off);
    // BF16 tiers: y0 of up to four slots travels through the trace region (see the second y-face
    // barrier).  The FP32 tier keeps register loads: there the extra live range costs spills.
    constexpr int DMA_SL = SPL < 4 ? SPL : 4;  // slots of y0 that fit a wave's part of the trace region
    constexpr bool DMA = YSH && (PREC == DG_BF16 || PREC == DG_BF16X3);
    const bool dma_y0 = DMA && !a.ex_single && a.mode != 0 && a.a != 0.0;
    C *ex_f = reinterpret_cast<C *>(lds + a.ex_off2);
    auto ex_put = [&](C *ex, int slot, const C v[NF][4]) {
        C *p = ex + slot * NF * 4 * 64 + lane_base();
#pragma unroll
        for (int i = 0; i < NF; i++)
#pragma unroll
            for (int r = 0; r < 4; r++) p[(i * 4 + r) * 64] = v[i][r];
    };
    auto ex_get = [&](const C *ex, int slot, C v[NF][4]) {
        const C *p = ex + slot * NF * 4 * 64 + lane_base();
#pragma unroll
        for (int i = 0; i < NF; i++)
#pragma unroll
            for (int r = 0; r < 4; r++) v[i][r] = p[(i * 4 + r) * 64];
    };

    // ---------------- work items: (x-block, y row or group of YROWS rows, z chunk), x-block fastest.
    // YSH: one item per workgroup, wave w takes row iy0 + w; otherwise one item per wave.
    constexpr int ROWS = YSH ? YROWS : 1;
    constexpr int IPW = YSH ? 1 : THREADS / 64;  // items a workgroup holds at once
    const int nyg = (ny + ROWS - 1) / ROWS;
    const int nxcd = gridDim.x < 8 ? (int)gridDim.x : 8;
    const int xcd = blockIdx.x % nxcd;
    const int wgs_x = (gridDim.x - xcd + nxcd - 1) / nxcd;
    const long long wid = (long long)(blockIdx.x / nxcd) * IPW + (YSH ? 0 : wave);
    const long long wcount = (long long)wgs_x * IPW;
    const long long i_lo = a.nitems * xcd / nxcd, i_hi = a.nitems * (xcd + 1) / nxcd;

    for (long long item = i_lo + wid; item < i_hi; item += wcount) {
        const int bx = (int)(item % a.nbx);
        const long long rest = item / a.nbx;
        const int iy0 = (int)(rest % nyg) * ROWS;
        const int zc = (int)(rest / nyg);
        const int nact = ny - iy0 < ROWS ? ny - iy0 : ROWS;  // rows of this item (the last group may be short)
        const int wrow = YSH ? wave : 0;
        const bool act = wrow < nact;                          // inactive waves compute a valid row, store nothing
        const int iy = act ? iy0 + wrow : iy0;
        const int z0 = zc * a.zlen;
        const int z1 = z0 + a.zlen < nz ? z0 + a.zlen : nz;
        const int xraw = BLK_INNER * bx - 1 + col;  // -1 .. : periodic wrap
        const int xc = (xraw % nx + nx) % nx;
        const bool keep = col >= 1 && col <= BLK_INNER && xraw < nx;
        set_lane_offsets(xc);
        auto cidx = [&](int yy, int zz) -> long long {  // slab index (wave-uniform), periodic
            yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
            zz = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
            return (long long)zz * ny + yy;
        };

        if (erows && act) {
            if (wrow == 0) load_lds(cidx(iy0 - 1, z0), 0);
            if (wrow == nact - 1) load_lds(cidx(iy0 + nact, z0), 1);
        }
        T.refresh();
        B cur;
        load(cidx(iy, z0), cur);
        C Fz[NF][4];  // flux on the -z face of the current block
        {
            B prv;
            loadz(iy, z0 - 1, prv);
            C tp[NF][4], tm[NF][4];
            trace(prv, 5, tp);
            trace(cur, 4, tm);
            riemann(std::integral_constant<int, 2>{}, tp, tm, Fz);
        }
        for (int z = z0; z < z1; z++) {
            T.refresh();
            Acc acc[NF][RT2];
#pragma unroll
            for (int i = 0; i < NF; i++)
#pragma unroll
                for (int rt = 0; rt < RT2; rt++) acc[i][rt] = Acc{0, 0, 0, 0};
            C av[3][4];  // driving acceleration of the current tile (FORCE)
            const auto ar = slab_rsrc(reinterpret_cast<const S *>(a.acache), aslab, cidx(iy, z));
            if constexpr (FORCE) accel_tile(ar, 0, av);
            lift(4, cur, Fz, acc);  // -z face: flux carried from the previous step
            B nxt;
            loadz(iy, z + 1, nxt);
            volume(cur, acc, ar, av);
            if constexpr (YSH) {
                // y faces shared by the rows of the workgroup: each face flux is solved once, by the
                // row below it; the faces at the group's ends use the neighbour rows' weights
                {
                    C tm[NF][4];
                    trace(cur, 2, tm);
                    if (a.ex_single) __syncthreads();  // the previous step's flux reads are done
                    ex_put(ex_t, wrow, tm);
                    if (wrow == 0) {
                        C Fm[NF][4];
                        {
                            C tb[NF][4];
                            {
                                B nb;
                                if (erows) {
                                    read_lds(0, nb);
                                    trace(nb, 3, tb);
                                    if (z + 1 < z1) load_lds(cidx(iy0 - 1, z + 1), 0);  // reads consumed above
                                } else {
                                    load(cidx(iy0 - 1, z), nb);
                                    trace(nb, 3, tb);
                                }
                            }
                            riemann(std::integral_constant<int, 1>{}, tb, tm, Fm);
                        }
                        lift(2, cur, Fm, acc);
                    }
                }
                __syncthreads();
                // the younger wave of each SIMD (rows w + 4) leads from here to the end of the step
                // (by default the older one wins issue and then waits at the next barrier)
                if (wave >= 4) __builtin_amdgcn_s_setprio(2);
                {
                    C Fp[NF][4];
                    {
                        C tp[NF][4], ta[NF][4];
                        trace(cur, 3, tp);
                        if (wrow == nact - 1) {
                            B nb;
                            if (erows) {
                                read_lds(1, nb);
                                trace(nb, 2, ta);
                                if (z + 1 < z1) load_lds(cidx(iy0 + nact, z + 1), 1);  // reads consumed above
                            } else {
                                load(cidx(iy0 + nact, z), nb);
                                trace(nb, 2, ta);
                            }
                        } else {
                            ex_get(ex_t, wrow + 1 < ROWS ? wrow + 1 : wrow, ta);
                        }
                        riemann(std::integral_constant<int, 1>{}, tp, ta, Fp);
                    }
                    lift(3, cur, Fp, acc);
                    if (a.ex_single) __syncthreads();  // every trace has been read
                    ex_put(ex_f, wrow, Fp);
                }
                __syncthreads();
                // the trace region is free until the next step's puts: the stage-combine input y0 of
                // this wave's slots (four at most) is copied into its part by the load unit now, so the
                // round trip hides behind the remaining faces
                if (DMA && dma_y0 && act) {
                    const auto r0 = slab_rsrc(y0, slabn, cidx(iy, z));
#pragma unroll
                    for (int u = 0; u < DMA_SL; u++) {
                        unsigned eo = KPL == 1 ? boff[u][0] : boff[0][u];
#pragma unroll
                        for (int i = 0; i < NF; i++)
                            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                                r0, (__attribute__((address_space(3))) void *)(ex_t + ((wrow * NF + i) * 4 + u) * 64),
                                (int)sizeof(S), eo, (int)((unsigned)i * fbytes), 0, 0);
                    }
                }
                if (wrow > 0) {
                    C Fm[NF][4];
                    ex_get(ex_f, wrow - 1, Fm);
                    lift(2, cur, Fm, acc);
                }
            } else {  // y faces: neighbour rows' traces from their weights
                C Fh[NF][4];
                {
                    C tn[NF][4];
                    {
                        B nb;
                        load(cidx(iy - 1, z), nb);
                        trace(nb, 3, tn);
                    }
                    C tm[NF][4];
                    trace(cur, 2, tm);
                    riemann(std::integral_constant<int, 1>{}, tn, tm, Fh);
                }
                lift(2, cur, Fh, acc);
                {
                    C tn[NF][4];
                    {
                        B nb;
                        load(cidx(iy + 1, z), nb);
                        trace(nb, 2, tn);
                    }
                    C tp[NF][4];
                    trace(cur, 3, tp);
                    riemann(std::integral_constant<int, 1>{}, tp, tn, Fh);
                }
                lift(3, cur, Fh, acc);
            }
            // x faces after the y faces: with the +z face they cover the round trip of the y0 copy
            // issued after the second barrier, and the waves reach the first barrier sooner
            {  // x faces: the left neighbour's + trace sits in the adjacent lane
                C tl[NF][4], Fh[NF][4];
                {
                    C tp[NF][4];
                    trace(cur, 1, tp);
#pragma unroll
                    for (int i = 0; i < NF; i++)
#pragma unroll
                        for (int r = 0; r < 4; r++) tl[i][r] = dpp_shr1(tp[i][r]);
                }
                {
                    C tm[NF][4];
                    trace(cur, 0, tm);
                    riemann(std::integral_constant<int, 0>{}, tl, tm, Fh);
                }
                lift(0, cur, Fh, acc);
                // the + face flux of a column is the - face flux of its right neighbour
#pragma unroll
                for (int i = 0; i < NF; i++)
#pragma unroll
                    for (int r = 0; r < 4; r++) Fh[i][r] = dpp_shl1(Fh[i][r]);
                lift(1, cur, Fh, acc);
            }
            {  // +z face with block z+1; its flux is the -z flux of the next step
                C tp[NF][4], tm[NF][4];
                trace(cur, 5, tp);
                trace(nxt, 4, tm);
                riemann(std::integral_constant<int, 2>{}, tp, tm, Fz);
                lift(5, cur, Fz, acc);
            }
            // combine and store the interior columns; result slot s = 4 rt + r is mode slot_mode(N, g, s),
            // the mode this lane loaded in slot s, so the FP32/FP64 stage input is still in registers.
            // The slots go in groups whose loads are all issued before the group's first store:
            // vector stores count in the same wait counter as loads, so a load placed after a store
            // waits for it, and interleaving them one by one would serialise the round trips.
            if (keep && act) {
                const long long rz = cidx(iy, z);
                const auto ro = slab_rsrc(out, slabn, rz);
                const bool comb = a.mode != 0;
                const bool with0 = comb && a.a != 0.0;
                constexpr bool CLO = K == 1;  // the closure exists for k = 1 only
                constexpr int EG = PREC != DG_FP64 ? SPL : 2;  // slots per group
#pragma unroll
                for (int s0 = 0; s0 < SPL; s0 += EG) {
                    // the row offsets pass an empty asm here so the group's loads are not hoisted
                    unsigned eo[EG];
#pragma unroll
                    for (int u = 0; u < EG; u++) {
                        const int sl = s0 + u < SPL ? s0 + u : SPL - 1;
                        eo[u] = KPL == 1 ? boff[sl][0] : boff[0][sl];
                        asm volatile("" : "+v"(eo[u]));
                    }
                    C y0v[NF][EG], cv[NF][EG];
                    if (DMA && dma_y0) {
                        // slots past the copied ones are loaded here
#pragma unroll
                        for (int u = 0; u < EG; u++)
                            if (s0 + u >= DMA_SL) {
                                const auto r0 = slab_rsrc(y0, slabn, rz);
#pragma unroll
                                for (int i = 0; i < NF; i++) y0v[i][u] = (C)bload(S(), r0, eo[u], (unsigned)i * fbytes);
                            }
                        // vmcnt(0): the copies into LDS have landed (the compiler does not track them);
                        // the memory clobber keeps the LDS reads below the wait
                        __builtin_amdgcn_s_waitcnt(0x0F70);
                        asm volatile("" ::: "memory");
                        const C *y0s = ex_t + wrow * NF * 4 * 64 + lane_base();
#pragma unroll
                        for (int u = 0; u < EG; u++)
                            if (s0 + u < DMA_SL) {
#pragma unroll
                                for (int i = 0; i < NF; i++) y0v[i][u] = y0s[(i * 4 + s0 + u) * 64];
                            }
                    } else if (with0) {
                        const auto r0 = slab_rsrc(y0, slabn, rz);
#pragma unroll
                        for (int u = 0; u < EG; u++)
#pragma unroll
                            for (int i = 0; i < NF; i++) y0v[i][u] = (C)bload(S(), r0, eo[u], (unsigned)i * fbytes);
                    }
                    if constexpr (CLO) {
                        if (a.corr) {  // learned closure: dy/dt = -R + c
                            const auto rcr = slab_rsrc(reinterpret_cast<const S *>(a.corr), slabn, rz);
#pragma unroll
                            for (int u = 0; u < EG; u++)
#pragma unroll
                                for (int i = 0; i < NF; i++) cv[i][u] = (C)bload(S(), rcr, eo[u], (unsigned)i * fbytes);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < EG; u++) {
                        const int sl = s0 + u;
                        if (sl >= SPL) break;
                        const int rt = sl / 4, r = sl % 4;
                        const int m = slot_mode(N, g, sl);
                        if (m < N) {
#pragma unroll
                            for (int i = 0; i < NF; i++) {
                                const unsigned so = (unsigned)i * fbytes;
                                C R = (C)acc[i][rt][r];
                                if constexpr (CLO)
                                    if (a.corr) R -= cv[i][u] - (m == 0 ? (C)a.cmean[i] : C(0));
                                if (!comb) {
                                    bstore((S)R, ro, eo[u] + so);
                                } else {
                                    C y1;
                                    if constexpr (KPL == 1)
                                        y1 = m == 0 ? cur.qbar[i] : (C)cur.w[i][sl].v;
                                    else
                                        y1 = m == 0 ? cur.qbar[i] : cur.v[i][sl];
                                    const C base = (C)a.b * (y1 - dt * R);
                                    const C res = with0 ? (C)a.a * y0v[i][u] + base : base;
                                    bstore((S)res, ro, eo[u] + so);
                                }
                            }
                        }
                    }
                }
            }
            if (YSH && wave >= 4) __builtin_amdgcn_s_setprio(0);
            cur = nxt;
        }
    }
}

// k = 0: one weight per field, and the scheme is first-order Godunov finite volume:
// R = sum_a (Fhat(q, q_{+a}) - Fhat(q_{-a}, q)) / h_a minus the source at the cell centre (the
// single Gauss point).  One thread per cell, workgroups of 64 x 4 cells in x and y: each cell
// solves its +x and +y faces and shares them through LDS with the cell that needs them as its -x
// or -y face (the same inputs and arithmetic, so the same bits as solving it there); faces on the
// tile's low edges and the z faces are solved by both of their cells.  No products.
constexpr int FV_TX = 64, FV_TY = 4, FV_THREADS = FV_TX * FV_TY;

template <int PREC, bool FORCE, int RS>
__global__ __launch_bounds__(FV_THREADS) void fv_stage_kernel(StageArgs a) {
    using PR = Prec<PREC>;
    using S = typename PR::S;
    using C = typename PR::C;
    __shared__ C fx[FV_TY][FV_TX][NF], fy[FV_TY][FV_TX][NF];  // each cell's +x and +y face fluxes
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int tx = threadIdx.x % FV_TX, ty = threadIdx.x / FV_TX;
    const int ntx = (nx + FV_TX - 1) / FV_TX, nty = (ny + FV_TY - 1) / FV_TY;
    const long long bid = blockIdx.x;
    const int bx = (int)(bid % ntx);
    const long long bzy = bid / ntx;
    const int by = (int)(bzy % nty), iz = (int)(bzy / nty);
    const int ix = bx * FV_TX + tx, iy = by * FV_TY + ty;
    const bool act = ix < nx && iy < ny;
    double dtd = a.dt;
    if (a.rate) dtd = a.dtfac / a.rate[0];
    if (a.tacc && blockIdx.x == 0 && threadIdx.x == 0) a.tacc[0] += dtd;
    const long long row = (long long)iz * ny + iy;
    const S *yin = static_cast<const S *>(a.yin);
    auto load = [&](int x, int yy, int zz, C q[5]) {
        x = x < 0 ? x + nx : (x >= nx ? x - nx : x);
        yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
        const S *src = yin;
        if (a.halo_lo && zz < 0) {  // across the ends of a z slab: the halo planes
            src = static_cast<const S *>(a.halo_lo);
            zz = 0;
        } else if (a.halo_hi && zz >= nz) {
            src = static_cast<const S *>(a.halo_hi);
            zz = 0;
        } else {
            zz = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
        }
        const long long b = ((long long)zz * ny + yy) * NF * nx + x;
#pragma unroll
        for (int i = 0; i < NF; i++) q[i] = (C)src[b + (long long)i * nx];
    };
    const C gam = (C)a.gamma;
    auto flux = [&](auto axis_c, const C qL[5], const C qR[5], C F[5]) {
        constexpr int AX = decltype(axis_c)::value;
        if constexpr (RS == 1)
            exact_rs<PR, AX>(qL, qR, gam, F);
        else
            hllc<PR, AX>(qL, qR, gam, F);
    };
    C q[5] = {1, 0, 0, 0, 1}, R[5] = {0, 0, 0, 0, 0};
    C Fpx[5], Fpy[5];
    if (act) {
        load(ix, iy, iz, q);
        C qn[5];
        load(ix + 1, iy, iz, qn);
        flux(std::integral_constant<int, 0>{}, q, qn, Fpx);
        load(ix, iy + 1, iz, qn);
        flux(std::integral_constant<int, 1>{}, q, qn, Fpy);
#pragma unroll
        for (int i = 0; i < NF; i++) {
            fx[ty][tx][i] = Fpx[i];
            fy[ty][tx][i] = Fpy[i];
        }
    }
    __syncthreads();
    if (!act) return;
    C Fmx[5], Fmy[5];
    if (tx > 0) {  // the -x neighbour is the thread to the left (same row, ix - 1 >= 0)
#pragma unroll
        for (int i = 0; i < NF; i++) Fmx[i] = fx[ty][tx - 1][i];
    } else {
        C qm[5];
        load(ix - 1, iy, iz, qm);
        flux(std::integral_constant<int, 0>{}, qm, q, Fmx);
    }
    if (ty > 0) {  // the -y neighbour is the thread below (iy - 1 >= 0)
#pragma unroll
        for (int i = 0; i < NF; i++) Fmy[i] = fy[ty - 1][tx][i];
    } else {
        C qm[5];
        load(ix, iy - 1, iz, qm);
        flux(std::integral_constant<int, 1>{}, qm, q, Fmy);
    }
    {
        const C ih = (C)(1.0 / a.h[0]);
#pragma unroll
        for (int i = 0; i < NF; i++) R[i] += (Fpx[i] - Fmx[i]) * ih;
    }
    {
        const C ih = (C)(1.0 / a.h[1]);
#pragma unroll
        for (int i = 0; i < NF; i++) R[i] += (Fpy[i] - Fmy[i]) * ih;
    }
    {
        C qm[5], qp[5], Fm[5], Fp[5];
        load(ix, iy, iz - 1, qm);
        load(ix, iy, iz + 1, qp);
        flux(std::integral_constant<int, 2>{}, qm, q, Fm);
        flux(std::integral_constant<int, 2>{}, q, qp, Fp);
        const C ih = (C)(1.0 / a.h[2]);
#pragma unroll
        for (int i = 0; i < NF; i++) R[i] += (Fp[i] - Fm[i]) * ih;
    }
    if constexpr (FORCE) {
        // the driving acceleration at the cell centre, from the k = 0 cache layout [component][x]
        const S *ac = static_cast<const S *>(a.acache) + row * (3LL * nx) + ix;
        C sE = 0;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const C av = (C)ac[(long long)c * nx];
            R[1 + c] -= q[0] * av;
            sE += q[1 + c] * av;
        }
        R[4] -= sE;
    }
    S *out = static_cast<S *>(a.out);
    const S *y0 = static_cast<const S *>(a.y0);
    const long long b = row * NF * nx + ix;
    const C dt = (C)dtd;
#pragma unroll
    for (int i = 0; i < NF; i++) {
        const long long j = b + (long long)i * nx;
        if (a.mode == 0) {
            out[j] = (S)R[i];
        } else {
            const C base = (C)a.b * (q[i] - dt * R[i]);
            out[j] = (S)(a.a != 0.0 ? (C)a.a * (C)y0[j] + base : base);
        }
    }
}

template <int PREC>
static hipError_t launch_fv_t(const StageArgs &a, hipStream_t s) {
    const long long nb = (long long)((a.nx + FV_TX - 1) / FV_TX) * ((a.ny + FV_TY - 1) / FV_TY) * a.nz;
    if (a.riemann == 1) {
        if (a.forcing) hipLaunchKernelGGL((fv_stage_kernel<PREC, true, 1>), dim3(nb), dim3(FV_THREADS), 0, s, a);
        else hipLaunchKernelGGL((fv_stage_kernel<PREC, false, 1>), dim3(nb), dim3(FV_THREADS), 0, s, a);
    } else {
        if (a.forcing) hipLaunchKernelGGL((fv_stage_kernel<PREC, true, 0>), dim3(nb), dim3(FV_THREADS), 0, s, a);
        else hipLaunchKernelGGL((fv_stage_kernel<PREC, false, 0>), dim3(nb), dim3(FV_THREADS), 0, s, a);
    }
    return hipGetLastError();
}

template <int K, int PREC>
static hipError_t launch_stage_t(const StageArgs &a, int grid, int lds_bytes, hipStream_t s) {
    constexpr int T = stage_threads<PREC>();
    if (a.riemann == 1) {
        if (a.forcing)
            hipLaunchKernelGGL((stage_kernel<K, PREC, true, 1>), dim3(grid), dim3(T), lds_bytes, s, a);
        else
            hipLaunchKernelGGL((stage_kernel<K, PREC, false, 1>), dim3(grid), dim3(T), lds_bytes, s, a);
    } else {
        if (a.forcing)
            hipLaunchKernelGGL((stage_kernel<K, PREC, true, 0>), dim3(grid), dim3(T), lds_bytes, s, a);
        else
            hipLaunchKernelGGL((stage_kernel<K, PREC, false, 0>), dim3(grid), dim3(T), lds_bytes, s, a);
    }
    return hipGetLastError();
}

template <int K, int PREC>
static hipError_t set_attr_t(int lds_bytes) {
    const void *fns[] = {reinterpret_cast<const void *>(&stage_kernel<K, PREC, false, 0>),
                         reinterpret_cast<const void *>(&stage_kernel<K, PREC, true, 0>),
                         reinterpret_cast<const void *>(&stage_kernel<K, PREC, false, 1>),
                         reinterpret_cast<const void *>(&stage_kernel<K, PREC, true, 1>)};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
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
    if (k == 0) {
        switch (prec) {
            case DG_FP64: return launch_fv_t<DG_FP64>(a, s);
            case DG_FP32: return launch_fv_t<DG_FP32>(a, s);
            case DG_BF16: return launch_fv_t<DG_BF16>(a, s);
            case DG_BF16X3: return launch_fv_t<DG_BF16X3>(a, s);
            default: return hipErrorInvalidValue;
        }
    }
    DG_DISPATCH(k, prec, launch_stage_t, (a, grid, lds_bytes, s))
}

hipError_t set_stage_attributes(int k, int prec, int lds_bytes) {
    DG_DISPATCH(k, prec, set_attr_t, (lds_bytes))
}

template <int K, int PREC>
static hipError_t occ_t(int lds_bytes, int *per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, stage_kernel<K, PREC, true, 0>, stage_threads<PREC>(),
                                                        lds_bytes);
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
                               long long nc, int nx) {
    constexpr int N = Dims<K>::N, Q = Dims<K>::Q;
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= nc) return;
    const long long r = cell / nx;
    const int x = (int)(cell - r * nx);
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
        for (int l = 0; l < N; l++) y[((r * NF + i) * N + l) * nx + x] = (S)s[l];
    }
}

template <int K>
static hipError_t launch_project_k(int prec, const void *qp, void *y, const double *ptab, long long nc, int nx,
                                   hipStream_t s) {
    const int th = 256;
    const long long nb = (nc + th - 1) / th;
    if (prec == DG_FP64)
        hipLaunchKernelGGL((project_kernel<K, double>), dim3(nb), dim3(th), 0, s, (const double *)qp, (double *)y,
                           ptab, nc, nx);
    else
        hipLaunchKernelGGL((project_kernel<K, float>), dim3(nb), dim3(th), 0, s, (const float *)qp, (float *)y, ptab,
                           nc, nx);
    return hipGetLastError();
}

hipError_t launch_project(int k, int prec, const void *qp, void *y, const double *ptab, long long nc, int nx,
                          hipStream_t s) {
    switch (k) {
        case 0: return launch_project_k<0>(prec, qp, y, ptab, nc, nx, s);
        case 1: return launch_project_k<1>(prec, qp, y, ptab, nc, nx, s);
        case 2: return launch_project_k<2>(prec, qp, y, ptab, nc, nx, s);
        case 3: return launch_project_k<3>(prec, qp, y, ptab, nc, nx, s);
        case 4: return launch_project_k<4>(prec, qp, y, ptab, nc, nx, s);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ state relayout at the boundary

// Between the canonical order [i][l][z][y][x] and the internal order [z][y][i][l][x]: both keep x
// fastest, so every row of nx weights moves whole.  One workgroup per row, the row's x values
// across the threads (coalesced reads and writes); a data move bound by HBM bandwidth.
template <class S>
__global__ __launch_bounds__(256) void relayout_kernel(const S *__restrict__ src, S *__restrict__ dst, int nfm,
                                                       int ny, int nz, int nx, int to_canonical) {
    const long long rows = (long long)nfm * ny * nz;
    for (long long r = blockIdx.x; r < rows; r += gridDim.x) {
        // r numbers the rows in internal order: ((z ny + y) nfm + f), f = i N + l
        const int f = (int)(r % nfm);
        const long long zy = r / nfm;
        const long long rc = (long long)f * ny * nz + zy;  // the same row in canonical order
        const long long si = (to_canonical ? r : rc) * nx, di = (to_canonical ? rc : r) * nx;
        for (int x = threadIdx.x; x < nx; x += blockDim.x) dst[di + x] = src[si + x];
    }
}

hipError_t launch_relayout(int prec, const void *src, void *dst, int nfm, int nx, int ny, int nz, int to_canonical,
                           hipStream_t s) {
    const long long rows = (long long)nfm * ny * nz;
    const unsigned grid = (unsigned)std::min<long long>(rows, 1LL << 20);
    if (prec == DG_FP64)
        hipLaunchKernelGGL(relayout_kernel<double>, dim3(grid), dim3(256), 0, s, static_cast<const double *>(src),
                           static_cast<double *>(dst), nfm, ny, nz, nx, to_canonical);
    else
        hipLaunchKernelGGL(relayout_kernel<float>, dim3(grid), dim3(256), 0, s, static_cast<const float *>(src),
                           static_cast<float *>(dst), nfm, ny, nz, nx, to_canonical);
    return hipGetLastError();
}

// ------------------------------------------------------------------ driving acceleration cache (Sec. 3.1)

// a_c(x_q) = sum_m Re(ahat_{m,c} exp(2 pi i n_m . x_q / L)) at every volume point of every
// cell, in the layout the stage kernel reads (see accel_load).  One workgroup per (row of cells,
// y node, z node): the y and z part of each mode's phase is shared by the whole row, so
// P_{m,c} = ahat_{m,c} exp(2 pi i (n_y Y + n_z Z)) is formed once into LDS; each thread then takes
// points along x, where the modes (sorted by n_x on the host) need one exp(2 pi i n_x X) per
// distinct n_x.  Phases are reduced to one turn and their sine and cosine taken in FP64.  Rows of
// the layout past the last point are zero.  k = 0 (the finite-volume kernel) takes a compact
// layout instead: per row of cells [component][x], the cell centre only.
constexpr int ACC_THREADS = 256;

template <int K, class S>
__global__ __launch_bounds__(ACC_THREADS) void accel_cache_kernel(const double *__restrict__ modes, int nmodes,
                                                                  int nx, int ny, int nz, GaussNodes xg, int z0,
                                                                  int nzg, S *__restrict__ out) {
    constexpr int n = K + 1, Q = n * n * n, RT1 = (Q + 15) / 16;
    constexpr bool F64 = sizeof(S) == 8;
    __shared__ double P[MAX_FORCING_MODES][3][2];
    const long long items = (long long)ny * nz * n * n;
    const long long aslab = K == 0 ? 3LL * nx : (long long)RT1 * 16 * 3 * nx;
    for (long long it = blockIdx.x; it < items; it += gridDim.x) {
        const long long row = it / (n * n);
        const int qbc = (int)(it - row * (n * n)), qb = qbc % n, qc = qbc / n;
        const int iy = (int)(row % ny), iz = (int)(row / ny);
        const double Y = (iy + 0.5 * (1.0 + xg.x[qb])) / ny, Z = (z0 + iz + 0.5 * (1.0 + xg.x[qc])) / nzg;
        for (int m = threadIdx.x; m < nmodes; m += ACC_THREADS) {
            const double *md = modes + 9 * m;
            double ph = md[1] * Y + md[2] * Z;
            ph -= floor(ph);
            double sn, cs;
            sincospi(2.0 * ph, &sn, &cs);
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const double re = md[3 + 2 * c], im = md[4 + 2 * c];
                P[m][c][0] = re * cs - im * sn;
                P[m][c][1] = re * sn + im * cs;
            }
        }
        __syncthreads();
        S *orow = out + row * aslab;
        for (int j = threadIdx.x; j < n * nx; j += ACC_THREADS) {
            const int qa = j / nx, ix = j - qa * nx;  // consecutive threads: consecutive cells
            const double X = (ix + 0.5 * (1.0 + xg.x[qa])) / nx;
            double acc[3] = {0.0, 0.0, 0.0};
            double er = 1.0, ei = 0.0, nprev = 0.0;
            for (int m = 0; m < nmodes; m++) {
                const double n0 = modes[9 * m];
                if (m == 0 || n0 != nprev) {
                    double ph = n0 * X;
                    ph -= floor(ph);
                    sincospi(2.0 * ph, &ei, &er);
                    nprev = n0;
                }
#pragma unroll
                for (int c = 0; c < 3; c++) acc[c] += P[m][c][0] * er - P[m][c][1] * ei;
            }
            if constexpr (K == 0) {  // the finite-volume kernel's compact layout [component][x]
#pragma unroll
                for (int c = 0; c < 3; c++) orow[(long long)c * nx + ix] = (S)acc[c];
                continue;
            }
            const int rho = qa + n * qb + n * n * qc;
            const int t = rho / 16, rr = rho % 16;
            const int g = F64 ? rr % 4 : rr / 4, r = F64 ? rr / 4 : rr % 4;  // result lane group and register
#pragma unroll
            for (int c = 0; c < 3; c++) orow[(((long long)(t * 3 + c) * 4 + g) * nx + ix) * 4 + r] = (S)acc[c];
        }
        if (K > 0 && qbc == 0 && RT1 * 16 > Q) {  // the padding rows of the last tile
            for (int j = threadIdx.x; j < (RT1 * 16 - Q) * nx; j += ACC_THREADS) {
                const int rho = Q + j / nx, ix = j % nx;
                const int t = rho / 16, rr = rho % 16;
                const int g = F64 ? rr % 4 : rr / 4, r = F64 ? rr / 4 : rr % 4;
#pragma unroll
                for (int c = 0; c < 3; c++) orow[(((long long)(t * 3 + c) * 4 + g) * nx + ix) * 4 + r] = S(0);
            }
        }
        __syncthreads();  // P is rewritten for the next item
    }
}

template <int K>
static hipError_t launch_accel_k(int prec, const double *modes, int nmodes, int nx, int ny, int nz, long long nc,
                                 const GaussNodes &xg, int z0, int nzg, void *out, hipStream_t s) {
    (void)nc;
    const long long items = (long long)ny * nz * (K + 1) * (K + 1);
    const long long nb = items < (1LL << 30) ? items : (1LL << 30);
    if (prec == DG_FP64)
        hipLaunchKernelGGL((accel_cache_kernel<K, double>), dim3(nb), dim3(ACC_THREADS), 0, s, modes, nmodes, nx, ny,
                           nz, xg, z0, nzg, (double *)out);
    else
        hipLaunchKernelGGL((accel_cache_kernel<K, float>), dim3(nb), dim3(ACC_THREADS), 0, s, modes, nmodes, nx, ny,
                           nz, xg, z0, nzg, (float *)out);
    return hipGetLastError();
}

hipError_t launch_accel_cache(int k, int prec, const double *modes, int nmodes, int nx, int ny, int nz, long long nc,
                              const GaussNodes &xg, int z0, int nzg, void *out, hipStream_t s) {
    switch (k) {
        case 0: return launch_accel_k<0>(prec, modes, nmodes, nx, ny, nz, nc, xg, z0, nzg, out, s);
        case 1: return launch_accel_k<1>(prec, modes, nmodes, nx, ny, nz, nc, xg, z0, nzg, out, s);
        case 2: return launch_accel_k<2>(prec, modes, nmodes, nx, ny, nz, nc, xg, z0, nzg, out, s);
        case 3: return launch_accel_k<3>(prec, modes, nmodes, nx, ny, nz, nc, xg, z0, nzg, out, s);
        case 4: return launch_accel_k<4>(prec, modes, nmodes, nx, ny, nz, nc, xg, z0, nzg, out, s);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ positivity limiter (Sec. 2.5)

// One thread per cell, in the storage precision.  The state is read once; it is
// written back only for the cells the limiter changes.  tab[p][l] = phi_l at the
// limiter points (the m GLL nodes along one axis times the k+1 Gauss nodes along
// the other two, for each axis).
template <int K, class S>
__global__ __launch_bounds__(256) void limit_kernel(S *__restrict__ y, const double *__restrict__ tab, int np,
                                                    long long nc, int nx, double gamma, double eps, double rel,
                                                    unsigned long long *count) {
    constexpr int N = Dims<K>::N;
    using C = S;
    extern __shared__ __attribute__((aligned(16))) char lsm[];
    C *lt = reinterpret_cast<C *>(lsm);
    for (int j = threadIdx.x; j < (np + 1) * N; j += blockDim.x) lt[j] = (C)tab[j];
    __syncthreads();
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= nc) return;
    const long long r = cell / nx;
    const long long base = r * (long long)NF * N * nx + (cell - r * nx);
    C w[NF][N];
#pragma unroll
    for (int i = 0; i < NF; i++)
#pragma unroll
        for (int l = 0; l < N; l++) w[i][l] = y[base + (long long)(i * N + l) * nx];
    const C g1 = (C)(gamma - 1.0), ep = (C)eps;
    {
        // Sufficient test first: with D_i = sum_l |u_il| max_S |phi_l| bounding |q_i - qbar_i| on the
        // point set, rho >= rbar - D_0 and p >= (gamma-1)(Ebar - D_4 - |m|^2_max / (2 rho_min)) there.
        // When both bounds clear the targets by more than the rounding of either evaluation, every
        // point passes, both scaling factors are 1 and the cell is left as it is.
        C dv[NF];
#pragma unroll
        for (int i = 0; i < NF; i++) {
            C a = 0;
#pragma unroll
            for (int l = 1; l < N; l++) a += __builtin_fabs(w[i][l]) * lt[np * N + l];
            dv[i] = a;
        }
        constexpr C u = sizeof(C) == 8 ? C(1.2e-16) : C(6e-8);  // unit roundoff
        const C rb = w[0][0];
        const C tr = (C)rel * rb > ep ? (C)rel * rb : ep;
        const C tp = (C)rel * g1 * w[4][0] > ep ? (C)rel * g1 * w[4][0] : ep;
        const C rlo = rb - dv[0];
        C m2 = 0;
#pragma unroll
        for (int i = 1; i < 4; i++) {
            const C mm = __builtin_fabs(w[i][0]) + dv[i];
            m2 += mm * mm;
        }
        const C kin = C(0.5) * m2 / rlo;
        const C el = w[4][0] - dv[4];
        const C plo = g1 * (el - kin);
        const C slack = C(256) * u * (rb + dv[0]);
        const C pslack = C(256) * u * g1 * (__builtin_fabs(w[4][0]) + dv[4] + kin);
        if (rlo > C(2) * tr + slack && plo > C(2) * tp + pslack) return;
    }
    // density: theta_1 from the minimum over the points
    C rmin = w[0][0];
    for (int p = 0; p < np; p++) {
        C v = 0;
#pragma unroll
        for (int l = 0; l < N; l++) v += w[0][l] * lt[p * N + l];
        rmin = v < rmin ? v : rmin;
    }
    const C rbar = w[0][0];
    // targets raised to rel x the cell's mean density / (gamma-1) x its mean energy where the
    // storage's rounding (FP32) would otherwise undo the limiting
    const C ep_r = (C)rel * rbar > ep ? (C)rel * rbar : ep;
    const C ep_p = (C)rel * g1 * w[4][0] > ep ? (C)rel * g1 * w[4][0] : ep;
    C th1 = C(1);
    if (rbar != rmin) {
        const C t = __builtin_fabs((rbar - ep_r) / (rbar - rmin));
        th1 = t < C(1) ? t : C(1);
    }
#pragma unroll
    for (int l = 1; l < N; l++) w[0][l] *= th1;
    // pressure: theta_2 = min over the points of tau, the root of P(qbar + tau (q - qbar)) = eps
    // (Newton-Raphson on rho P - eps rho, a quadratic in tau, kept inside its bracket)
    const C qb[5] = {w[0][0], w[1][0], w[2][0], w[3][0], w[4][0]};
    auto gfun = [&](const C d[5], C t, C &dg) {
        const C rr = qb[0] + t * d[0], mx = qb[1] + t * d[1], my = qb[2] + t * d[2], mz = qb[3] + t * d[3],
                ee = qb[4] + t * d[4];
        dg = g1 * (d[0] * ee + rr * d[4] - (mx * d[1] + my * d[2] + mz * d[3])) - ep_p * d[0];
        return g1 * (rr * ee - C(0.5) * (mx * mx + my * my + mz * mz)) - ep_p * rr;
    };
    C th2 = C(1);
    for (int p = 0; p < np; p++) {
        C q[5];
#pragma unroll
        for (int i = 0; i < NF; i++) {
            C v = 0;
#pragma unroll
            for (int l = 0; l < N; l++) v += w[i][l] * lt[p * N + l];
            q[i] = v;
        }
        const C pr = g1 * (q[4] - C(0.5) * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
        if (q[0] > C(0) && pr >= ep_p) continue;
        C d[5];
#pragma unroll
        for (int i = 0; i < 5; i++) d[i] = q[i] - qb[i];
        C dg0, dg1;
        const C g0 = gfun(d, C(0), dg0);
        C tau = C(0);
        if (g0 > C(0)) {
            const C gone = gfun(d, C(1), dg1);
            C lo = C(0), hi = C(1);
            C t = gone < C(0) ? g0 / (g0 - gone) : C(1);
            for (int it = 0; it < 60; it++) {
                C dv;
                const C v = gfun(d, t, dv);
                if (v >= C(0)) lo = t;
                else hi = t;
                C tn = dv != C(0) ? t - v / dv : C(0.5) * (lo + hi);
                if (!(tn > lo && tn < hi)) tn = C(0.5) * (lo + hi);
                if (tn == t || hi - lo <= C(4) * __builtin_fabs(t) * (sizeof(C) == 8 ? C(2.3e-16) : C(1.2e-7))) break;
                t = tn;
            }
            tau = lo;
        }
        th2 = tau < th2 ? tau : th2;
    }
    if (th1 < C(1) || th2 < C(1)) {
#pragma unroll
        for (int i = 0; i < NF; i++)
#pragma unroll
            for (int l = 1; l < N; l++) y[base + (long long)(i * N + l) * nx] = w[i][l] * th2;
        atomicAdd(count, 1ull);
    }
}

template <int K>
static hipError_t launch_limit_k(int prec, void *y, const double *tab, int np, long long nc, int nx, double gamma,
                                 double eps, unsigned long long *count, hipStream_t s) {
    const long long nb = (nc + 255) / 256;
    const int N = Dims<K>::N;
    if (prec == DG_FP64) {
        const int bytes = (np + 1) * N * 8;  // k = 4: 84 KB, above the default dynamic LDS limit
        if (bytes > 65536) {
            const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&limit_kernel<K, double>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((limit_kernel<K, double>), dim3(nb), dim3(256), bytes, s, (double *)y, tab, np, nc, nx,
                           gamma, eps, 0.0, count);
    } else
        hipLaunchKernelGGL((limit_kernel<K, float>), dim3(nb), dim3(256), (np + 1) * N * 4, s, (float *)y, tab, np, nc, nx,
                           gamma, eps, LIMIT_REL_FP32, count);
    return hipGetLastError();
}

hipError_t launch_limit(int k, int prec, void *y, const double *tab, int np, long long nc, int nx, double gamma,
                        double eps, unsigned long long *count, hipStream_t s) {
    switch (k) {
        case 0: return launch_limit_k<0>(prec, y, tab, np, nc, nx, gamma, eps, count, s);
        case 1: return launch_limit_k<1>(prec, y, tab, np, nc, nx, gamma, eps, count, s);
        case 2: return launch_limit_k<2>(prec, y, tab, np, nc, nx, gamma, eps, count, s);
        case 3: return launch_limit_k<3>(prec, y, tab, np, nc, nx, gamma, eps, count, s);
        case 4: return launch_limit_k<4>(prec, y, tab, np, nc, nx, gamma, eps, count, s);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ isothermal reset (Sec. 3.2)

// rho^(gamma-1) / rho0^(gamma-1): FP32 through the hardware base-2 logarithm and exponential,
// FP64 through pow
__device__ inline float pow_d(float x, float p) { return __builtin_amdgcn_exp2f(p * __builtin_amdgcn_logf(x)); }
__device__ inline double pow_d(double x, double p) { return pow(x, p); }
// 1/x in the precision of C (FP32: the hardware reciprocal, not an IEEE division)
__device__ inline float rcp_d(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp_d(double x) { return 1.0 / x; }

constexpr int RESET_THREADS = 256;

// One thread per cell (x consecutive over the lanes), one z slice of the Gauss grid at a time.
// rho and m at the slice's points by sum factorisation over the tensor-product Legendre factors
// (z, then y, then x), the energy density |m|^2/(2 rho) + rho eps(rho), eps = ce (rho/rho0)^(gamma-1)
// with ce = cs^2/(gamma-1), projected back in the reverse order (x, y, then z into the modes).
// The block's sum of |K| (rhoe_before - rhoe_after) (cell means, FP64) goes to partials[block].
template <int K, class S>
__global__ __launch_bounds__(RESET_THREADS) void reset_kernel(S *__restrict__ y, Leg1D L, long long nc, int nx,
                                                              double gm1, double ce, double rho0, double vol,
                                                              double *__restrict__ partials) {
    constexpr int N = Dims<K>::N, n = K + 1;
    using C = S;
    __shared__ double red[RESET_THREADS];
    C P[K + 1][n], WP[K + 1][n];
#pragma unroll
    for (int u = 0; u <= K; u++)
#pragma unroll
        for (int a = 0; a < n; a++) {
            P[u][a] = (C)L.p[u][a];
            WP[u][a] = (C)(L.w[a] * L.p[u][a]);
        }
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double dis = 0.0;
    if (cell < nc) {
        const long long r = cell / nx;
        const long long base = r * (long long)NF * N * nx + (cell - r * nx);
        C wt[4][N];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int l = 0; l < N; l++) wt[i][l] = y[base + (long long)(i * N + l) * nx];
        const C e_old = y[base + (long long)(4 * N) * nx];
        C acc[N];
#pragma unroll
        for (int l = 0; l < N; l++) acc[l] = 0;
        const C g = (C)gm1, cc = (C)ce, ir0 = C(1) / (C)rho0;
#pragma unroll
        for (int c = 0; c < n; c++) {
            // one field's values at the slice's points (z, then y, then x factor)
            auto eval = [&](int i, C q[n][n]) {
                C t1[K + 1][K + 1];
#pragma unroll
                for (int u = 0; u <= K; u++)
#pragma unroll
                    for (int v = 0; u + v <= K; v++) {
                        C t = 0;
#pragma unroll
                        for (int w = 0; u + v + w <= K; w++) t += wt[i][mode_of<K>(u, v, w)] * P[w][c];
                        t1[u][v] = t;
                    }
                C t2[K + 1][n];
#pragma unroll
                for (int u = 0; u <= K; u++)
#pragma unroll
                    for (int b = 0; b < n; b++) {
                        C t = 0;
#pragma unroll
                        for (int v = 0; u + v <= K; v++) t += t1[u][v] * P[v][b];
                        t2[u][b] = t;
                    }
#pragma unroll
                for (int b = 0; b < n; b++)
#pragma unroll
                    for (int a = 0; a < n; a++) {
                        C t = 0;
#pragma unroll
                        for (int u = 0; u <= K; u++) t += t2[u][b] * P[u][a];
                        q[b][a] = t;
                    }
            };
            C rho[n][n], m2[n][n], qm[n][n];
            eval(0, rho);
#pragma unroll
            for (int i = 1; i < 4; i++) {
                eval(i, qm);
#pragma unroll
                for (int b = 0; b < n; b++)
#pragma unroll
                    for (int a = 0; a < n; a++) m2[b][a] = (i == 1 ? C(0) : m2[b][a]) + qm[b][a] * qm[b][a];
            }
            C e[n][n];
#pragma unroll
            for (int b = 0; b < n; b++)
#pragma unroll
                for (int a = 0; a < n; a++)
                    e[b][a] = C(0.5) * m2[b][a] * rcp_d(rho[b][a]) + cc * rho[b][a] * pow_d(rho[b][a] * ir0, g);
            C s1[K + 1][n];
#pragma unroll
            for (int u = 0; u <= K; u++)
#pragma unroll
                for (int b = 0; b < n; b++) {
                    C t = 0;
#pragma unroll
                    for (int a = 0; a < n; a++) t += WP[u][a] * e[b][a];
                    s1[u][b] = t;
                }
#pragma unroll
            for (int u = 0; u <= K; u++)
#pragma unroll
                for (int v = 0; u + v <= K; v++) {
                    C t = 0;
#pragma unroll
                    for (int b = 0; b < n; b++) t += WP[v][b] * s1[u][b];
#pragma unroll
                    for (int w = 0; u + v + w <= K; w++) acc[mode_of<K>(u, v, w)] += C(0.125) * WP[w][c] * t;
                }
        }
#pragma unroll
        for (int l = 0; l < N; l++) y[base + (long long)(4 * N + l) * nx] = acc[l];
        const double rb = (double)wt[0][0], kin = 0.5 * ((double)wt[1][0] * (double)wt[1][0] +
                                                         (double)wt[2][0] * (double)wt[2][0] +
                                                         (double)wt[3][0] * (double)wt[3][0]) / rb;
        dis = vol * (((double)e_old - kin) - ((double)acc[0] - kin));
    }
    red[threadIdx.x] = dis;
    __syncthreads();
    for (int h = RESET_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// acc += sum of p[0..n) in a fixed order (one workgroup: contiguous chunks per thread, then a tree)
__global__ __launch_bounds__(256) void sum_into_kernel(const double *__restrict__ p, long long n, double *acc) {
    __shared__ double red[256];
    const long long ch = (n + 255) / 256;
    const long long lo = threadIdx.x * ch, hi = lo + ch < n ? lo + ch : n;
    double s = 0.0;
    for (long long j = lo; j < hi; j++) s += p[j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *acc += red[0];
}

long long reset_partials(long long nc) { return (nc + RESET_THREADS - 1) / RESET_THREADS; }

hipError_t launch_sum_into(const double *p, long long n, double *acc, hipStream_t s) {
    hipLaunchKernelGGL(sum_into_kernel, dim3(1), dim3(256), 0, s, p, n, acc);
    return hipGetLastError();
}

template <int K>
static hipError_t launch_reset_k(int prec, void *y, const Leg1D &L, long long nc, int nx, double gm1, double ce,
                                 double rho0, double vol, double *partials, double *acc, hipStream_t s) {
    const long long nb = reset_partials(nc);
    if (prec == DG_FP64)
        hipLaunchKernelGGL((reset_kernel<K, double>), dim3(nb), dim3(RESET_THREADS), 0, s, (double *)y, L, nc, nx,
                           gm1, ce, rho0, vol, partials);
    else
        hipLaunchKernelGGL((reset_kernel<K, float>), dim3(nb), dim3(RESET_THREADS), 0, s, (float *)y, L, nc, nx, gm1,
                           ce, rho0, vol, partials);
    hipLaunchKernelGGL(sum_into_kernel, dim3(1), dim3(256), 0, s, partials, nb, acc);
    return hipGetLastError();
}

hipError_t launch_reset(int k, int prec, void *y, const Leg1D &L, long long nc, int nx, double gm1, double ce,
                        double rho0, double vol, double *partials, double *acc, hipStream_t s) {
    switch (k) {
        case 0: return launch_reset_k<0>(prec, y, L, nc, nx, gm1, ce, rho0, vol, partials, acc, s);
        case 1: return launch_reset_k<1>(prec, y, L, nc, nx, gm1, ce, rho0, vol, partials, acc, s);
        case 2: return launch_reset_k<2>(prec, y, L, nc, nx, gm1, ce, rho0, vol, partials, acc, s);
        case 3: return launch_reset_k<3>(prec, y, L, nc, nx, gm1, ce, rho0, vol, partials, acc, s);
        case 4: return launch_reset_k<4>(prec, y, L, nc, nx, gm1, ce, rho0, vol, partials, acc, s);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ CFL reduction (Sec. 2.4)

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// index of mode 0 of field i of a cell in the [z][y][i][l][x] layout
__device__ inline long long mean_index(long long cell, int i, int N, int nx) {
    const long long r = cell / nx;
    return ((r * NF + i) * N) * nx + (cell - r * nx);
}

// Grid-stride over the cells with a fixed grid: each thread keeps the largest rate of its cells, the
// workgroup reduces them (wave shuffles, then LDS), and one atomic max per workgroup goes to the slot
// (a per-wave atomic on one address serialised ~260k atomics per call at 256^3).
constexpr int CFL_THREADS = 256, CFL_BLOCKS = 2048;

template <class S>
__global__ __launch_bounds__(CFL_THREADS) void cfl_kernel(const S *__restrict__ y, int N, int nx, long long nc,
                                                          double gamma, double hx, double hy, double hz,
                                                          double *rate_slot, double *zero_slot) {
    __shared__ double wmax[CFL_THREADS / 64];
    double rate = 0.0;
    for (long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x; cell < nc;
         cell += (long long)gridDim.x * blockDim.x) {
        const double rho = (double)y[mean_index(cell, 0, N, nx)];
        const double mx = (double)y[mean_index(cell, 1, N, nx)];
        const double my = (double)y[mean_index(cell, 2, N, nx)];
        const double mz = (double)y[mean_index(cell, 3, N, nx)];
        const double E = (double)y[mean_index(cell, 4, N, nx)];
        const double inv = 1.0 / rho;
        const double p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my + mz * mz) * inv);
        const double c = sqrt(gamma * p * inv);
        double r = (fabs(mx * inv) + c) / hx + (fabs(my * inv) + c) / hy + (fabs(mz * inv) + c) / hz;
        if (!(r >= 0.0)) r = __builtin_inf();  // non-physical cell: force dt -> 0
        rate = fmax(rate, r);
    }
    rate = wave_max(rate);
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = rate;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = wmax[0];
        for (int w = 1; w < CFL_THREADS / 64; w++) m = fmax(m, wmax[w]);
        // the bit patterns of non-negative doubles order like their values
        atomicMax(reinterpret_cast<unsigned long long *>(rate_slot), (unsigned long long)__double_as_longlong(m));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && zero_slot) *zero_slot = 0.0;
}

hipError_t launch_cfl(int prec, const void *y, int N, int nx, long long nc, double gamma, const double h[3],
                      double *rate_slot, double *zero_slot, hipStream_t s) {
    long long nb = (nc + CFL_THREADS - 1) / CFL_THREADS;
    if (nb > CFL_BLOCKS) nb = CFL_BLOCKS;
    if (prec == DG_FP64)
        hipLaunchKernelGGL((cfl_kernel<double>), dim3(nb), dim3(CFL_THREADS), 0, s, (const double *)y, N, nx, nc, gamma,
                           h[0], h[1], h[2], rate_slot, zero_slot);
    else
        hipLaunchKernelGGL((cfl_kernel<float>), dim3(nb), dim3(CFL_THREADS), 0, s, (const float *)y, N, nx, nc, gamma,
                           h[0], h[1], h[2], rate_slot, zero_slot);
    return hipGetLastError();
}

// ------------------------------------------------------------------ conserved totals (fixed order)

constexpr int TOT_THREADS = 256;

template <class S>
__global__ void totals_pass1(const S *__restrict__ y, int N, int nx, long long nc, double *partials, int nparts) {
    __shared__ double red[TOT_THREADS];
    const long long chunk = (nc + nparts - 1) / nparts;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = lo + chunk < nc ? lo + chunk : nc;
    for (int i = 0; i < NF; i++) {
        double s = 0.0;
        for (long long c = lo + threadIdx.x; c < hi; c += TOT_THREADS) s += (double)y[mean_index(c, i, N, nx)];
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

hipError_t launch_totals(int prec, const void *y, int N, int nx, long long nc, double vol, double *partials,
                         int nparts, double *out, hipStream_t s) {
    if (prec == DG_FP64)
        hipLaunchKernelGGL((totals_pass1<double>), dim3(nparts), dim3(TOT_THREADS), 0, s, (const double *)y, N, nx, nc,
                           partials, nparts);
    else
        hipLaunchKernelGGL((totals_pass1<float>), dim3(nparts), dim3(TOT_THREADS), 0, s, (const float *)y, N, nx, nc,
                           partials, nparts);
    hipLaunchKernelGGL(totals_pass2, dim3(1), dim3(TOT_THREADS), 0, s, partials, nparts, vol, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ range check

template <class S>
__global__ void range_kernel(const S *__restrict__ y, int N, int nx, long long nc, double gamma, int *flag) {
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= nc) return;
    const double rho = (double)y[mean_index(cell, 0, N, nx)];
    const double mx = (double)y[mean_index(cell, 1, N, nx)];
    const double my = (double)y[mean_index(cell, 2, N, nx)];
    const double mz = (double)y[mean_index(cell, 3, N, nx)];
    const double E = (double)y[mean_index(cell, 4, N, nx)];
    const double p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my + mz * mz) / rho);
    const bool ok = rho > 0.0 && p > 0.0 && __builtin_isfinite(p) && __builtin_isfinite(rho);
    if (!ok) atomicOr(flag, 1);
}

hipError_t launch_range_check(int prec, const void *y, int N, int nx, long long nc, double gamma, int *flag,
                              hipStream_t s) {
    const int th = 256;
    const long long nb = (nc + th - 1) / th;
    if (prec == DG_FP64)
        hipLaunchKernelGGL((range_kernel<double>), dim3(nb), dim3(th), 0, s, (const double *)y, N, nx, nc, gamma, flag);
    else
        hipLaunchKernelGGL((range_kernel<float>), dim3(nb), dim3(th), 0, s, (const float *)y, N, nx, nc, gamma, flag);
    return hipGetLastError();
}

}  // namespace dgmi
