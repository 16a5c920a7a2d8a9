// The SSP stage kernel for k = 3 (N = 20 modes, 4^3 volume points, 4^2 points per face) in the
// tiers with FP32 storage: DG_BF16 (one BF16 product), DG_BF16X3 (each operand split x = hi + lo,
// three BF16 products: FP32-grade) and DG_FP32 (FP32 products).  It evaluates the same operator as
// stage_kernel in dg_kernels.hip (Bauer et al., arXiv 1602.09079, Sec. 2.3, eqs.
// dg:eqn:volume_int and dg:eqn:surface_int, the driving source of Sec. 3.1, the Shu-Osher
// combine of the SSP-RK3 step), organised for gfx950:
//
// - x-blocks of 16 cells that start on 64-byte boundaries, no halo columns.  The x faces inside a
//   block are solved by lanes of one 16-lane row (DPP shifts); the face on the block's low edge
//   uses the +x trace of the cell before it and, for full blocks, the face on the high edge the
//   -x trace of the cell after it, both from one extra product ("ghost" product: column 0 holds
//   the cell before, column 15 the cell after with its odd-u modes negated, which turns the +x
//   trace table into the -x one).  The high edge's 16 points are gathered into 16 lanes and
//   solved in one pass.  Ragged last blocks take their right neighbour from the wrapped column
//   after the last valid one.
// - Every product is a K = 32 chunk: one 16x16x32 BF16 MFMA, or in FP32 eight 16x16x4 steps
//   (steps whose operand half is zero are skipped; the second row tile, one useful row per lane
//   group, runs as 4x4x1 products of 16 blocks, a quarter of the cost).  The volume contraction
//   pairs the x and y fluxes of a z-node's 16 points in one K = 32 chunk and the z flux with the
//   driving source in another; the lift pairs the - and + face of an axis.  The mode order of the result rows
//   (k3_slot_mode) puts the four modes (0,0,w) in the second row tile, whose x and y derivative
//   tables vanish, so the x/y chunk needs one row tile.
// - The symmetric momentum flux m_a m_b / rho is formed and split once for both of its uses.  The
//   lo part of a split is x - hi formed by a BF16 dot product with (-1, 0) (exact).
// - The driving acceleration at the volume points is itself a product:
//   a_c(x) = sum_{n_x >= 0} Re(H_{c,n_x}(point) exp(2 pi i n_x ix / nx)), with H per (z, y) row of
//   cells (the y, z and in-cell x phases of the modes, built once per driving update in FP64) as
//   the A operand and cos / sin of the cell's x phase as the B operand of FP32 16x16x4 MFMAs.
// - y faces shared by the 8 rows of a workgroup through LDS (each face solved once), the z face
//   carried along the z sweep, as in stage_kernel.
// - No register spills in the z sweep: loads complete in order, so a spill reload waits for every
//   copy and prefetch in flight before it.  LDS is addressed from one opaque lane base plus
//   immediate offsets, nothing is held in registers across the barriers, and the copies into
//   LDS are waited for with exact counts.
// - The two waves of a SIMD (rows w and w + 4) take turns to lead (issue priority), so that they
//   reach the barriers together.

#include <type_traits>

#include "dg_device.h"

namespace dgmi {

namespace {

constexpr int K3_THREADS = 64 * YROWS;
constexpr int NSL = 5;  // mode slots per lane group

typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// B operand of one K = 32 chunk: 8 values per lane, as BF16 (hi, and lo for BF16X3) or, for FP32,
// as floats (element j is the operand of the chunk's j-th 16x16x4 FP32 product)
template <int P>
struct Op;
template <>
struct Op<DG_BF16X3> {
    bf8 hi, lo;
};
template <>
struct Op<DG_BF16> {
    bf8 hi;
};
template <>
struct Op<DG_FP32> {
    float v[8];
};

// half of a B operand: four values as two packed BF16 pairs (hi, and lo for BF16X3), or floats
template <int P>
struct H4 {
    unsigned hi[2];
    unsigned lo[P == DG_BF16X3 ? 2 : 1];
};
template <>
struct H4<DG_FP32> {
    float v[4];
};

__device__ inline unsigned pk_bf16(float a, float b) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector((fv2){a, b}, bv2));  // v_cvt_pk_bf16_f32
}

// x = hi + lo: hi = bf16(x) (round to nearest even); lo = bf16(x - hi), with x - hi (exact) from
// a BF16 dot product of the packed hi pair with (-1, 0) or (0, -1) accumulated onto x.  The two
// constant pairs are passed in scalar registers: written as literals, the compiler encodes (-1, 0)
// as the inline constant -1.0, which the hardware applies to the other half of the pair (every
// result wrong, measured on gfx950); the register operands give x - hi exactly.
struct SplitConst {
    unsigned m0, m1;  // BF16 pairs (-1, 0) and (0, -1)
};
__device__ inline SplitConst split_const() {
    SplitConst c{0x0000BF80u, 0xBF800000u};
    asm volatile("" : "+s"(c.m0));
    asm volatile("" : "+s"(c.m1));
    return c;
}
template <bool X3>
__device__ inline void split_pair(float a, float b, unsigned &hi, unsigned &lo, const SplitConst &k) {
    const bv2 h = __builtin_convertvector((fv2){a, b}, bv2);
    hi = __builtin_bit_cast(unsigned, h);
    if constexpr (X3) {
        const float la = __builtin_amdgcn_fdot2_f32_bf16(h, __builtin_bit_cast(bv2, k.m0), a, false);
        const float lb = __builtin_amdgcn_fdot2_f32_bf16(h, __builtin_bit_cast(bv2, k.m1), b, false);
        lo = pk_bf16(la, lb);
    }
}
template <int P>
__device__ inline H4<P> split4(const float v[4], const SplitConst &k) {
    H4<P> o;
    if constexpr (P == DG_FP32) {
#pragma unroll
        for (int r = 0; r < 4; r++) o.v[r] = v[r];
    } else {
        constexpr bool X3 = P == DG_BF16X3;
        unsigned l0 = 0, l1 = 0;
        split_pair<X3>(v[0], v[1], o.hi[0], l0, k);
        split_pair<X3>(v[2], v[3], o.hi[1], l1, k);
        if constexpr (X3) {
            o.lo[0] = l0;
            o.lo[1] = l1;
        }
    }
    return o;
}
template <int P>
__device__ inline Op<P> join(const H4<P> &a, const H4<P> &b) {
    Op<P> o;
    if constexpr (P == DG_FP32) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
            o.v[r] = a.v[r];
            o.v[4 + r] = b.v[r];
        }
    } else {
        o.hi = __builtin_bit_cast(bf8, (u4v){a.hi[0], a.hi[1], b.hi[0], b.hi[1]});
        if constexpr (P == DG_BF16X3) o.lo = __builtin_bit_cast(bf8, (u4v){a.lo[0], a.lo[1], b.lo[0], b.lo[1]});
    }
    return o;
}
template <int P>
__device__ inline H4<P> zero4() {
    H4<P> o;
    if constexpr (P == DG_FP32) {
#pragma unroll
        for (int r = 0; r < 4; r++) o.v[r] = 0.0f;
    } else {
        o.hi[0] = o.hi[1] = 0u;
        if constexpr (P == DG_BF16X3) o.lo[0] = o.lo[1] = 0u;
    }
    return o;
}

// The weights of a block of 16 cells: the means (mode 0, full precision) and the raw values of
// the lane's five mode slots.  Their BF16 operands are formed per use (once for the four volume
// nodes, once per pair of faces): kept for the whole step, the split copies would take the
// registers that the second wave per SIMD needs.
struct Blk3 {
    float qbar[NF];
    float v[NF][NSL];
};

// the B operand of one field of a block: slots 0..4 at contraction indices 8g + 0..4, 5..7 zero
template <int P>
__device__ inline Op<P> weights_op(const float v[NSL], const SplitConst &k) {
    Op<P> op;
    if constexpr (P == DG_FP32) {
#pragma unroll
        for (int s = 0; s < 8; s++) op.v[s] = s < NSL ? v[s] : 0.0f;
    } else {
        constexpr bool X3 = P == DG_BF16X3;
        unsigned h0, h1, h2, l0 = 0, l1 = 0, l2 = 0;
        split_pair<X3>(v[0], v[1], h0, l0, k);
        split_pair<X3>(v[2], v[3], h1, l1, k);
        {  // slot 4 with a zero: one split
            const bv2 h = __builtin_convertvector((fv2){v[4], 0.0f}, bv2);
            h2 = __builtin_bit_cast(unsigned, h);
            if constexpr (X3)
                l2 = pk_bf16(__builtin_amdgcn_fdot2_f32_bf16(h, __builtin_bit_cast(bv2, k.m0), v[4], false), 0.0f);
        }
        op.hi = __builtin_bit_cast(bf8, (u4v){h0, h1, h2, 0u});
        if constexpr (X3) op.lo = __builtin_bit_cast(bf8, (u4v){l0, l1, l2, 0u});
    }
    return op;
}

// DPP row shifts within 16-lane rows: row_shl:n (lane c <- lane c + n), row_shr:n (lane c <- c - n)
template <int N>
__device__ inline float shl(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x100 + N, 0xf, 0xf, true));
}
template <int N>
__device__ inline float shr(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 + N, 0xf, 0xf, true));
}

// s_waitcnt immediates (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
constexpr int wait_vm(int n) { return (n & 15) | ((n >> 4) << 14) | 0x0F70; }
constexpr int WAIT_LGKM0 = 0xC07F;

// Barrier for data exchanged through LDS only: this wave's LDS accesses have completed, then the
// workgroup meets.  Unlike __syncthreads it does not wait for outstanding global loads and stores
// (the copies requested one step ahead stay in flight); what the load unit copies into LDS is read
// only by the wave that requested it, after its own wait.
__device__ inline void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(WAIT_LGKM0);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

}  // namespace

template <int PREC, bool FORCE, int RS>
__global__ __launch_bounds__(K3_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void stage_k3_kernel(StageArgs a) {
    constexpr bool X3 = PREC == DG_BF16X3;
    using PR = Prec<PREC>;
    using C = float;
    using Acc = f4;
    using B3 = Blk3;
    using HH = H4<PREC>;
    using OP = Op<PREC>;

    extern __shared__ __attribute__((aligned(16))) char lds[];
    {
        constexpr int bytes = K3_SET * (PREC == DG_BF16 ? 1 : 2);
        const int4 *src = reinterpret_cast<const int4 *>(a.tables);
        int4 *dst = reinterpret_cast<int4 *>(lds);
        for (int j = threadIdx.x; j < bytes / 16; j += K3_THREADS) dst[j] = src[j];
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int col = lane & 15;
    const int g = lane >> 4;
    const SplitConst sk = split_const();
    // this lane's byte offset in a fragment; the empty asm keeps fragment reads where they are used
    int toff = lane * 16;
    auto refresh = [&]() { asm volatile("" : "+v"(toff)); };
    // LDS accesses address one lane base plus immediate offsets: the lane index is made opaque at
    // each use, so that the compiler does not hoist a register per element out of the sweep (and
    // spill them: a spill reload waits for every load in flight)
    auto lane_base = [&]() {
        int o = lane;
        asm volatile("" : "+v"(o));
        return o;
    };
    // one K = 32 chunk; FP32: steps j0 .. j1 - 1 of its eight 16x16x4 products (the others have a
    // zero operand), the A values of steps 4h .. 4h + 3 one 16-byte read at half h of the fragment
    // LDS destination of a copy by the load unit (M0): a wave-uniform base made opaque at each use,
    // so that the compiler adds the copy's immediate offset there instead of keeping one scalar
    // register per copy across the sweep (they spill into vector lanes and come back by readlane)
    typedef __attribute__((address_space(3))) C lds_c;
    auto lds_dst = [](C *p) -> lds_c * {
        lds_c *q = (lds_c *)p;
        asm volatile("" : "+s"(q));
        return q;
    };
    auto mma = [&](Acc c, int frag, const OP &b, int j0 = 0, int j1 = 8) -> Acc {
        if constexpr (PREC == DG_FP32) {
#pragma unroll
            for (int h = 0; h < 2; h++) {
                if (4 * h >= j1 || 4 * h + 4 <= j0) continue;
                const f4 af = *reinterpret_cast<const f4 *>(lds + (2 * frag + h) * K3_FRAG + toff);
#pragma unroll
                for (int r = 0; r < 4; r++)
                    if (4 * h + r >= j0 && 4 * h + r < j1)
                        c = __builtin_amdgcn_mfma_f32_16x16x4f32(af[r], b.v[4 * h + r], c, 0, 0, 0);
            }
            return c;
        } else {
            const bf8 ah = *reinterpret_cast<const bf8 *>(lds + frag * K3_FRAG + toff);
            if constexpr (X3) {
                const bf8 al = *reinterpret_cast<const bf8 *>(lds + K3_SET + frag * K3_FRAG + toff);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b.hi, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b.lo, c, 0, 0, 0);
            }
            return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b.hi, c, 0, 0, 0);
        }
    };
    // the second row tile of a chunk (one useful row per lane group: slot 4).  FP32: 4x4x1 products
    // of 16 blocks, block 4g + c (this lane: g = lane / 16, c = (lane % 16) / 4) taking cells
    // 4c .. 4c + 3 and contraction index 8g + j; register r of lane l then holds the part from
    // lane group l / 16 of row 4r (slot 4 of lane group r) for cell l % 16, summed by tile1_sum.
    // A quarter of the 16x16x4 products' cost.
    auto mma1 = [&](Acc c, int frag, const OP &b, int j0 = 0, int j1 = 8) -> Acc {
        if constexpr (PREC == DG_FP32) {
#pragma unroll
            for (int h = 0; h < 2; h++) {
                if (4 * h >= j1 || 4 * h + 4 <= j0) continue;
                const f4 af = *reinterpret_cast<const f4 *>(lds + (2 * frag + h) * K3_FRAG + toff);
#pragma unroll
                for (int r = 0; r < 4; r++)
                    if (4 * h + r >= j0 && 4 * h + r < j1)
                        c = __builtin_amdgcn_mfma_f32_4x4x1f32(af[r], b.v[4 * h + r], c, 0, 0, 0);
            }
            return c;
        } else {
            return mma(c, frag, b, j0, j1);
        }
    };
    // the mass flux's volume term: fragment sf of the mode-to-mode tables after the LDS sets, read
    // through the caches (A operands requested by sload, used by smma)
    constexpr unsigned SOFF = (unsigned)K3_SET * (PREC == DG_BF16 ? 1u : 2u);
    constexpr unsigned STOT = SOFF + (unsigned)K3_NS * K3_FRAG * (PREC == DG_BF16 ? 1u : 2u);
    struct SFrag {
        bf8 hi, lo;
        f4 v;
        float v4;
    };
    auto sload = [&](int sf) -> SFrag {
        const auto rs = slab_rsrc(reinterpret_cast<const unsigned *>(a.tables), (long long)(STOT / 4u), 0);
        const unsigned vo = (unsigned)lane_base() * 16u;
        SFrag o;
        if constexpr (PREC == DG_FP32) {
            const unsigned so = SOFF + 2u * (unsigned)sf * K3_FRAG;
            o.v = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, so, 0));
            o.v4 = bload(0.0f, rs, vo, so + K3_FRAG);
        } else {
            o.hi = __builtin_bit_cast(bf8, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, SOFF + (unsigned)sf * K3_FRAG, 0));
            if constexpr (X3)
                o.lo = __builtin_bit_cast(
                    bf8, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, SOFF + (unsigned)(K3_NS + sf) * K3_FRAG, 0));
        }
        return o;
    };
    auto smma = [&](Acc c, const SFrag &f, const OP &b, bool tile1) -> Acc {
        if constexpr (PREC == DG_FP32) {
#pragma unroll
            for (int r = 0; r < 4; r++)
                c = tile1 ? __builtin_amdgcn_mfma_f32_4x4x1f32(f.v[r], b.v[r], c, 0, 0, 0)
                          : __builtin_amdgcn_mfma_f32_16x16x4f32(f.v[r], b.v[r], c, 0, 0, 0);
            return tile1 ? __builtin_amdgcn_mfma_f32_4x4x1f32(f.v4, b.v[4], c, 0, 0, 0)
                         : __builtin_amdgcn_mfma_f32_16x16x4f32(f.v4, b.v[4], c, 0, 0, 0);
        } else {
            if constexpr (X3) {
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.lo, b.hi, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.hi, b.lo, c, 0, 0, 0);
            }
            return __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.hi, b.hi, c, 0, 0, 0);
        }
    };
    // FP32: the second row tile's result in register 0 (slot 4): this lane group's row summed over
    // the four lane groups' parts (two exchange steps, each lane keeping half of what remains)
    auto tile1_sum = [&](Acc c) -> Acc {
        const bool hi2 = (g & 2) != 0, odd = (g & 1) != 0;
        const C k0 = hi2 ? c[2] : c[0], k1 = hi2 ? c[3] : c[1];
        const C s0 = hi2 ? c[0] : c[2], s1 = hi2 ? c[1] : c[3];
        const C h0 = k0 + __shfl_xor(s0, 32), h1 = k1 + __shfl_xor(s1, 32);
        const C keep = odd ? h1 : h0, send = odd ? h0 : h1;
        c[0] = keep + __shfl_xor(send, 16);
        return c;
    };

    const C gam = (C)a.gamma;
    const C g1 = gam - C(1);
    double dtd = a.dt;
    if (a.rate) dtd = a.dtfac / a.rate[0];
    const C dt = (C)dtd;
    if (a.tacc && blockIdx.x == 0 && threadIdx.x == 0) a.tacc[0] += dtd;
    const float *yin = reinterpret_cast<const float *>(a.yin);
    const float *y0 = reinterpret_cast<const float *>(a.y0);
    float *out = reinterpret_cast<float *>(a.out);
    constexpr int N = 20;
    const long long slabn = (long long)NF * N * a.nx;  // elements per (z, y) slab
    const unsigned nxu = (unsigned)a.nx;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const unsigned fbytes = (unsigned)N * nxu * 4u;  // one field of a slab

    // per-lane byte offsets of the mode rows of this lane's slots (column offset added per item)
    unsigned roff[NSL];
#pragma unroll
    for (int s = 0; s < NSL; s++) roff[s] = (unsigned)k3_slot_mode(g, s) * nxu * 4u;
    // the -x trace of a cell is the +x trace table applied to the weights with the odd-u modes
    // negated: the sign bits of this lane's slots (k = 3 graded order: u = 1 or 3 for these modes)
    unsigned oddu = 0;
#pragma unroll
    for (int s = 0; s < NSL; s++) {
        const int m = k3_slot_mode(g, s);
        const bool odd = m == 1 || m == 5 || m == 6 || m == 10 || m == 13 || m == 14 || m == 15;
        if (odd) oddu |= 1u << s;
    }

    unsigned xoff = 0;
    auto load_from = [&](const float *base, long long r, B3 &b) {
        const auto rs = slab_rsrc(base, slabn, r);
#pragma unroll
        for (int i = 0; i < NF; i++) {
            const unsigned so = (unsigned)i * fbytes;
            b.qbar[i] = bload(0.0f, rs, xoff, so);
#pragma unroll
            for (int s = 0; s < NSL; s++) b.v[i][s] = bload(0.0f, rs, roff[s] + xoff, so);
        }
    };
    auto loadz = [&](int yy, int zz, B3 &b) {
        yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
        if (a.halo_lo && zz < 0)
            load_from(static_cast<const float *>(a.halo_lo), yy, b);
        else if (a.halo_hi && zz >= nz)
            load_from(static_cast<const float *>(a.halo_hi), yy, b);
        else
            load_from(yin, (long long)(zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz)) * ny + yy, b);
    };

    // end rows of the y group, copied into LDS by the load unit one z step ahead
    constexpr int ERV = NF * (1 + NSL);
    C *ex_e = reinterpret_cast<C *>(lds + a.ex_off3);
    auto load_lds = [&](long long r, int e) {
        const auto rs = slab_rsrc(yin, slabn, r);
        lds_c *dst = lds_dst(ex_e + e * ERV * 64);
#pragma unroll
        for (int i = 0; i < NF; i++) {
            const int so = (int)((unsigned)i * fbytes);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)(dst + (i * (1 + NSL)) * 64),
                                                     4, xoff, so, 0, 0);
#pragma unroll
            for (int s = 0; s < NSL; s++)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rs, (__attribute__((address_space(3))) void *)(dst + (i * (1 + NSL) + 1 + s) * 64), 4,
                    roff[s] + xoff, so, 0, 0);
        }
    };
    // the operand of field i of a block where it is used: an empty asm on the inputs keeps the
    // conversions of different uses from being merged (and held across the step)
    auto wop = [&](const B3 &b, int i) -> OP {
        C v[NSL];
#pragma unroll
        for (int s = 0; s < NSL; s++) {
            v[s] = b.v[i][s];
            if constexpr (PREC != DG_FP32) asm volatile("" : "+v"(v[s]));
        }
        return weights_op<PREC>(v, sk);
    };
    // traces of a block on face f (GEMM3), mean added back in full precision
    auto trace = [&](int f, const B3 &b, C tr[NF][4]) {
#pragma unroll
        for (int i = 0; i < NF; i++) {
            const Acc t = mma(Acc{0, 0, 0, 0}, K3_T3 + f, wop(b, i), 0, NSL);
#pragma unroll
            for (int r = 0; r < 4; r++) tr[i][r] = t[r] + b.qbar[i];
        }
    };
    // two faces of one block from one operand per field
    auto trace2 = [&](int f1, int f2, const B3 &b, C tr1[NF][4], C tr2[NF][4]) {
#pragma unroll
        for (int i = 0; i < NF; i++) {
            const OP op = wop(b, i);
            const Acc t1 = mma(Acc{0, 0, 0, 0}, K3_T3 + f1, op, 0, NSL);
            const Acc t2 = mma(Acc{0, 0, 0, 0}, K3_T3 + f2, op, 0, NSL);
#pragma unroll
            for (int r = 0; r < 4; r++) {
                tr1[i][r] = t1[r] + b.qbar[i];
                tr2[i][r] = t2[r] + b.qbar[i];
            }
        }
    };
    // the trace on face f of the end row copied into LDS buffer e
    auto trace_lds = [&](int f, int e, C tr[NF][4]) {
        // the copies have landed (the compiler does not track them): requests complete in order,
        // and the 30 loads of a block and 4 ghost copies, at least, were issued after them (one
        // step ahead: the next block's loads and the end-of-step ghost copies; before the first
        // step: the first block's and the one before it); the memory clobber keeps the LDS reads
        // below the wait
        __builtin_amdgcn_s_waitcnt(wait_vm(NF * (1 + NSL) + 4));
        asm volatile("" ::: "memory");
        const C *src = ex_e + e * ERV * 64 + lane_base();
        B3 b;
#pragma unroll
        for (int i = 0; i < NF; i++) {
            b.qbar[i] = src[(i * (1 + NSL)) * 64];
#pragma unroll
            for (int s = 0; s < NSL; s++) b.v[i][s] = src[(i * (1 + NSL) + 1 + s) * 64];
        }
        trace(f, b, tr);
    };
    // The ghost cells of the x faces (the cell before the block and the cell after it), copied into
    // LDS by the load unit one z step ahead, four 64-lane copies per wave: lane (g, c) copies for
    // lane group g a value of the cell before (c < 8) or after (c >= 8); with c8 = c % 8, copy k
    // holds value c8 of field k for c8 < 6 and value 4 (c8 - 6) + k of field 4 for c8 = 6, 7, value
    // 0 being the field's mean and value s + 1 its slot s (values 6 and 7 repeat the mean).
    // x0: the block's first cell (wave-uniform).
    C *ex_g = reinterpret_cast<C *>(lds + a.ex_off4) + wave * 4 * 64;
    auto ghost_dma = [&](long long r, int x0) {
        const auto rs = slab_rsrc(yin, slabn, r);
        const int xr = x0 + K3_BLK;
        const unsigned xgl = (unsigned)(x0 == 0 ? nx - 1 : x0 - 1) * 4u, xgr = (unsigned)(xr >= nx ? xr - nx : xr) * 4u;
        // lane values made opaque here: the offsets are formed at each use instead of being kept
        // in registers across the sweep
        int ln = lane;
        asm volatile("" : "+v"(ln));
        const unsigned cx = (ln & 15) < 8 ? xgl : xgr;
        const int c8 = ln & 7;
        const bool f4 = c8 >= 6;
        lds_c *gdst = lds_dst(ex_g);
        asm volatile("" ::: "memory");
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int m = f4 ? 4 * (c8 - 6) + k : c8;
            unsigned row = 0;  // the value's mode row: this lane group's slot rows
#pragma unroll
            for (int s2 = 0; s2 < NSL; s2++) row = m == s2 + 1 ? roff[s2] : row;
            const unsigned fo = f4 ? 4u * fbytes : (unsigned)k * fbytes;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)(gdst + k * 64), 4,
                                                     row + cx + fo, 0, 0, 0);
        }
        asm volatile("" ::: "memory");
    };
    // this lane's ghost cell (column 0: the cell before, column 15 of a full block: the cell after,
    // odd-u modes negated); other lanes get values they do not use
    auto ghost_read = [&](bool after, B3 &gb) {
        int o = 16 * g + (after ? 8 : 0);
        asm volatile("" : "+v"(o));
        const C *src = ex_g + o;
        // value m of field i: copy i, lane m (fields 0..3); copy m % 4, lane 6 + m / 4 (field 4)
        auto at = [&](int i, int m) { return i < 4 ? src[i * 64 + m] : src[(m % 4) * 64 + 6 + m / 4]; };
#pragma unroll
        for (int i = 0; i < NF; i++) {
            gb.qbar[i] = at(i, 0);
#pragma unroll
            for (int s2 = 0; s2 < NSL; s2++) {
                const C vv = at(i, 1 + s2);
                gb.v[i][s2] = (after && ((oddu >> s2) & 1u)) ? -vv : vv;
            }
        }
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
    // the cell-mean flux along one axis
    auto mean_flux = [&](const B3 &b, int axis, C Fb[5]) {
        C F3[3][5];
        euler_flux3<PR>(b.qbar, g1, F3);
#pragma unroll
        for (int i = 0; i < 5; i++) Fb[i] = F3[axis][i];
    };
    // lift (GEMM4) of the flux deviations on the - face (Fm) and + face (Fp) of an axis; a null
    // side contributes nothing
    auto lift = [&](int axis, const B3 &b, const C (*Fm)[4], const C (*Fp)[4], Acc acc[NF][2]) {
        C Fb[5];
        mean_flux(b, axis, Fb);
#pragma unroll
        for (int i = 0; i < NF; i++) {
            HH hm = zero4<PREC>(), hp = zero4<PREC>();
            if (Fm) {
                C v[4];
#pragma unroll
                for (int r = 0; r < 4; r++) v[r] = Fm[i][r] - Fb[i];
                hm = split4<PREC>(v, sk);
            }
            if (Fp) {
                C v[4];
#pragma unroll
                for (int r = 0; r < 4; r++) v[r] = Fp[i][r] - Fb[i];
                hp = split4<PREC>(v, sk);
            }
            const OP op = join<PREC>(hm, hp);
            const int j0 = Fm ? 0 : 4, j1 = Fp ? 8 : 4;
            acc[i][0] = mma(acc[i][0], K3_T4 + 2 * axis, op, j0, j1);
            acc[i][1] = mma1(acc[i][1], K3_T4 + 2 * axis + 1, op, j0, j1);
        }
    };

    // volume integral and driving source (GEMM1 -> fluxes -> GEMM2), one z-node (16 points) at a
    // time; the driving acceleration of the node from its own product (A: the row's factor table)
    constexpr int dks = K3_DKS;
    float csv[K3_DKS];  // B operand of the driving product: cos / sin of the x phases
    auto volume = [&](const B3 &b, Acc acc[NF][2], const float *drow) {
        C Fb[3][5];
        euler_flux3<PR>(b.qbar, g1, Fb);
        float hn[3][K3_DKS];  // the driving factors of the next node, requested one node ahead
        if constexpr (FORCE) {
#pragma unroll
            for (int c = 0; c < 3; c++)
#pragma unroll
                for (int s = 0; s < K3_DKS; s++) hn[c][s] = drow[(c * 4 * K3_DKS + s) * 64 + lane];
        }
        SFrag sfr[K3_NS];
#pragma unroll
        for (int sf = 0; sf < K3_NS; sf++) sfr[sf] = sload(sf);
        // the weights' operands, formed once for the four nodes
        OP w5[NF];
        {
#pragma unroll
            for (int i = 0; i < NF; i++) w5[i] = wop(b, i);
        }
        // mass: its flux deviation is the momentum deviation, a polynomial of the cell's modes, so
        // its volume term is a fixed matrix on the momentum weights (the quadrature integrates
        // the products exactly)
        acc[0][0] = smma(acc[0][0], sfr[0], w5[1], false);
        acc[0][0] = smma(acc[0][0], sfr[1], w5[2], false);
        acc[0][0] = smma(acc[0][0], sfr[2], w5[3], false);
        acc[0][1] = smma(acc[0][1], sfr[3], w5[3], true);
#pragma unroll
        for (int t = 0; t < 4; t++) {
            refresh();
            Acc d[NF];
#pragma unroll
            for (int i = 0; i < NF; i++) d[i] = mma(Acc{0, 0, 0, 0}, K3_T1 + t, w5[i], 0, NSL);
            // the driving acceleration of the node (issued after the x/y chunk, below)
            Acc av[3] = {Acc{0, 0, 0, 0}, Acc{0, 0, 0, 0}, Acc{0, 0, 0, 0}};
            float ha[3][K3_DKS];
            if constexpr (FORCE) {
#pragma unroll
                for (int c = 0; c < 3; c++)
#pragma unroll
                    for (int s = 0; s < K3_DKS; s++) {
                        ha[c][s] = hn[c][s];
                        if (t + 1 < 4) hn[c][s] = drow[((c * 4 + t + 1) * K3_DKS + s) * 64 + lane];
                    }
            }
            // point values and primitive quantities at this lane's 4 points of the node
            C rho[4], mx[4], my[4], mz[4], u[4], v[4], w[4], p[4], ep[4];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                rho[r] = d[0][r] + b.qbar[0];
                mx[r] = d[1][r] + b.qbar[1];
                my[r] = d[2][r] + b.qbar[2];
                mz[r] = d[3][r] + b.qbar[3];
                const C E = d[4][r] + b.qbar[4];
                const C inv = PR::rcp(rho[r]);
                u[r] = mx[r] * inv;
                v[r] = my[r] * inv;
                w[r] = mz[r] * inv;
                p[r] = g1 * (E - C(0.5) * (mx[r] * u[r] + my[r] * v[r] + mz[r] * w[r]));
                ep[r] = E + p[r];
            }
            // flux deviations F(q) - F(qbar) of the momentum and energy (the mass term is above);
            // m_a m_b / rho is formed once for both uses
            C tmp[4];
            HH hxy, hxz, hyz;
            {
#pragma unroll
                for (int r = 0; r < 4; r++) tmp[r] = mx[r] * u[r] + p[r] - Fb[0][1];
                const HH hxx = split4<PREC>(tmp, sk);
#pragma unroll
                for (int r = 0; r < 4; r++) tmp[r] = mx[r] * v[r] - Fb[1][1];
                hxy = split4<PREC>(tmp, sk);
                acc[1][0] = mma(acc[1][0], K3_T2A + t, join<PREC>(hxx, hxy));
            }
            {
#pragma unroll
                for (int r = 0; r < 4; r++) tmp[r] = my[r] * v[r] + p[r] - Fb[1][2];
                const HH hyy = split4<PREC>(tmp, sk);
                acc[2][0] = mma(acc[2][0], K3_T2A + t, join<PREC>(hxy, hyy));
            }
            {
#pragma unroll
                for (int r = 0; r < 4; r++) tmp[r] = mx[r] * w[r] - Fb[2][1];
                hxz = split4<PREC>(tmp, sk);
#pragma unroll
                for (int r = 0; r < 4; r++) tmp[r] = my[r] * w[r] - Fb[2][2];
                hyz = split4<PREC>(tmp, sk);
                acc[3][0] = mma(acc[3][0], K3_T2A + t, join<PREC>(hxz, hyz));
            }
            {
#pragma unroll
                for (int r = 0; r < 4; r++) tmp[r] = ep[r] * u[r] - Fb[0][4];
                const HH hxe = split4<PREC>(tmp, sk);
#pragma unroll
                for (int r = 0; r < 4; r++) tmp[r] = ep[r] * v[r] - Fb[1][4];
                const HH hye = split4<PREC>(tmp, sk);
                acc[4][0] = mma(acc[4][0], K3_T2A + t, join<PREC>(hxe, hye));
            }
            if constexpr (FORCE) {
#pragma unroll
                for (int c = 0; c < 3; c++)
#pragma unroll
                    for (int s = 0; s < K3_DKS; s++)
                        av[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ha[c][s], csv[s], av[c], 0, 0, 0);
            }
            // chunk (z, source): S = (0, rho a, m.a) at the points
            auto chunk_b = [&](int i, const HH &hz, const HH &hs) {
                const OP op = join<PREC>(hz, hs);
                const int j1 = FORCE && i > 0 ? 8 : 4;  // the source half is zero otherwise
                acc[i][0] = mma(acc[i][0], K3_T2B + 2 * t, op, 0, j1);
                acc[i][1] = mma1(acc[i][1], K3_T2B + 2 * t + 1, op, 0, j1);
            };
            {
                HH hs = zero4<PREC>();
                if constexpr (FORCE) {
#pragma unroll
                    for (int r = 0; r < 4; r++) tmp[r] = rho[r] * av[0][r];
                    hs = split4<PREC>(tmp, sk);
                }
                chunk_b(1, hxz, hs);
            }
            {
                HH hs = zero4<PREC>();
                if constexpr (FORCE) {
#pragma unroll
                    for (int r = 0; r < 4; r++) tmp[r] = rho[r] * av[1][r];
                    hs = split4<PREC>(tmp, sk);
                }
                chunk_b(2, hyz, hs);
            }
            {
#pragma unroll
                for (int r = 0; r < 4; r++) tmp[r] = mz[r] * w[r] + p[r] - Fb[2][3];
                const HH hzz = split4<PREC>(tmp, sk);
                HH hs = zero4<PREC>();
                if constexpr (FORCE) {
#pragma unroll
                    for (int r = 0; r < 4; r++) tmp[r] = rho[r] * av[2][r];
                    hs = split4<PREC>(tmp, sk);
                }
                chunk_b(3, hzz, hs);
            }
            {
#pragma unroll
                for (int r = 0; r < 4; r++) tmp[r] = ep[r] * w[r] - Fb[2][4];
                const HH hze = split4<PREC>(tmp, sk);
                HH hs = zero4<PREC>();
                if constexpr (FORCE) {
#pragma unroll
                    for (int r = 0; r < 4; r++) tmp[r] = mx[r] * av[0][r] + my[r] * av[1][r] + mz[r] * av[2][r];
                    hs = split4<PREC>(tmp, sk);
                }
                chunk_b(4, hze, hs);
            }
        }
    };

    // y-face exchange in LDS: a trace region and a flux region of one slot per wave
    C *ex_t = reinterpret_cast<C *>(lds + a.ex_off);
    C *ex_f = reinterpret_cast<C *>(lds + a.ex_off2);
    const bool dma_y0 = a.mode != 0 && a.a != 0.0;  // stages 2 and 3 read y0
    auto ex_put = [&](C *ex, int slot, const C vv[NF][4]) {
        C *p = ex + slot * NF * 4 * 64 + lane_base();
#pragma unroll
        for (int i = 0; i < NF; i++)
#pragma unroll
            for (int r = 0; r < 4; r++) p[(i * 4 + r) * 64] = vv[i][r];
    };
    auto ex_get = [&](const C *ex, int slot, C vv[NF][4]) {
        const C *p = ex + slot * NF * 4 * 64 + lane_base();
#pragma unroll
        for (int i = 0; i < NF; i++)
#pragma unroll
            for (int r = 0; r < 4; r++) vv[i][r] = p[(i * 4 + r) * 64];
    };

    // ---------------- work items: (x-block, group of YROWS rows, z chunk), x-block fastest
    const int nyg = (ny + YROWS - 1) / YROWS;
    const int nxcd = gridDim.x < 8 ? (int)gridDim.x : 8;
    const int xcd = blockIdx.x % nxcd;
    const int wgs_x = (gridDim.x - xcd + nxcd - 1) / nxcd;
    const long long wid = (long long)(blockIdx.x / nxcd);
    const long long wcount = (long long)wgs_x;
    const long long i_lo = a.nitems * xcd / nxcd, i_hi = a.nitems * (xcd + 1) / nxcd;

    for (long long item = i_lo + wid; item < i_hi; item += wcount) {
        const int bx = (int)(item % a.nbx);
        const long long rest = item / a.nbx;
        const int iy0 = (int)(rest % nyg) * YROWS;
        const int zc = (int)(rest / nyg);
        const int nact = ny - iy0 < YROWS ? ny - iy0 : YROWS;  // rows of this item
        const int wrow = wave;
        const bool act = wrow < nact;  // inactive waves compute a valid row, store nothing
        const int iy = act ? iy0 + wrow : iy0;
        const int z0 = zc * a.zlen;
        const int z1 = z0 + a.zlen < nz ? z0 + a.zlen : nz;
        const int x0 = K3_BLK * bx;
        const int vc = nx - x0 < K3_BLK ? nx - x0 : K3_BLK;  // valid columns (wave-uniform)
        const int xraw = x0 + col;
        const int xc = xraw < nx ? xraw : xraw % nx;          // columns past the mesh wrap
        const bool keep = col < vc;
        xoff = (unsigned)xc * 4u;
        // the ghost columns: column 0 reads the cell before the block, column 15 (full blocks)
        // the cell after it
        const bool gl = col == 0, gr = col == 15 && vc == K3_BLK;
        if constexpr (FORCE) {
#pragma unroll
            for (int s = 0; s < K3_DKS; s++) csv[s] = a.dcs[((long long)xc * K3_DKS + s) * 4 + g];
        }
        auto cidx = [&](int yy, int zz) -> long long {  // slab index (wave-uniform), periodic
            yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
            zz = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
            return (long long)zz * ny + yy;
        };

        // the host guarantees the end-row and ghost regions (a.ex_off3, a.ex_off4 >= 0)
        ghost_dma(cidx(iy, z0), x0);
        if (act) {
            if (wrow == 0) load_lds(cidx(iy0 - 1, z0), 0);
            if (wrow == nact - 1) load_lds(cidx(iy0 + nact, z0), 1);
        }
        refresh();
        B3 cur;
        loadz(iy, z0, cur);
        C Fz[NF][4];  // flux on the -z face of the current block
        {
            C tp[NF][4], tm[NF][4];
            {
                B3 prv;
                loadz(iy, z0 - 1, prv);
                trace(5, prv, tp);
            }
            trace(4, cur, tm);
            riemann(std::integral_constant<int, 2>{}, tp, tm, Fz);
        }
        for (int z = z0; z < z1; z++) {
            refresh();
            // lane offsets made opaque once per step: the addresses derived from them are formed where
            // they are used instead of being hoisted out of the loop (and spilled)
            asm volatile("" : "+v"(xoff));
#pragma unroll
            for (int s2 = 0; s2 < NSL; s2++) asm volatile("" : "+v"(roff[s2]));
            Acc acc[NF][2];
#pragma unroll
            for (int i = 0; i < NF; i++) acc[i][0] = acc[i][1] = Acc{0, 0, 0, 0};
            lift(2, cur, Fz, nullptr, acc);  // -z face: flux carried from the previous step
            const float *drow = FORCE ? a.dtab + cidx(iy, z) * k3_drive_row_floats(K3_DKS) : nullptr;
            volume(cur, acc, drow);
            C y044 = C(0);  // slot 4 of field 4 of y0 (stages 2 and 3)
            // x faces: own traces, the ghost cells' traces, the -x face of every column (its left
            // neighbour's +x trace in the adjacent lane), the +x flux from the right neighbour's -x
            // flux, and for a full block the face on its high edge.  In BF16X3 with the driving the
            // older wave of each SIMD (rows 0..3) forms them before the first y-face barrier, where
            // it would otherwise wait for its partner, and the younger one after the y lift; the
            // other kernels (measured slower that way) form them after the y lift in every wave
            constexpr bool XEARLY = PREC == DG_BF16X3 && FORCE;
            auto xfaces = [&](bool early) {
                {
                    C tl[NF][4], Fxp[NF][4], tm[NF][4];
                    {
                        C tp[NF][4], tg[NF][4];
                        {
                            // the ghost cells from their copy in LDS.  The copies were requested in the
                            // previous step (or before the first) and requests complete in order: after
                            // the y lift the 30 loads of the next block and, in stages 2 and 3, the 20
                            // copies of y0 were issued after them; before the first barrier fewer
                            // requests follow them, so that wave waits for all
                            if (early)
                                __builtin_amdgcn_s_waitcnt(wait_vm(0));
                            else if (dma_y0 && act)
                                __builtin_amdgcn_s_waitcnt(wait_vm(NF * (1 + NSL) + NF * 4));
                            else
                                __builtin_amdgcn_s_waitcnt(wait_vm(NF * (1 + NSL)));
                            asm volatile("" ::: "memory");
                            B3 gb;
                            ghost_read(gr, gb);
                            trace(1, gb, tg);  // column 0: +x trace of the cell before; 15: -x trace after
                        }
                        // the copies read above have been used: until the combine, their slots take slot 4
                        // of y0 for fields 0..3 (stages 2 and 3); field 4's is loaded into a register
                        __builtin_amdgcn_s_waitcnt(WAIT_LGKM0);
                        if (dma_y0 && act) {
                            const auto r0 = slab_rsrc(y0, slabn, cidx(iy, z));
                            lds_c *gdst = lds_dst(ex_g);
                            asm volatile("" ::: "memory");
    #pragma unroll
                            for (int i = 0; i < 4; i++)
                                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                                    r0, (__attribute__((address_space(3))) void *)(gdst + i * 64), 4, roff[4] + xoff,
                                    (int)((unsigned)i * fbytes), 0, 0);
                            asm volatile("" ::: "memory");
                            y044 = bload(0.0f, r0, roff[4] + xoff, 4u * fbytes);
                        }
                        trace2(1, 0, cur, tp, tm);  // both x traces of the block from one operand
                        if (vc == K3_BLK) {
                            // the 16 points of column 15's +x face, one per lane of columns 12..15
                            C ql[5], qr[5], fo[5];
    #pragma unroll
                            for (int i = 0; i < NF; i++) {
                                // the DPP moves first, with every lane active, then the selects
                                const C l1 = shl<1>(tp[i][1]), l2 = shl<2>(tp[i][2]), l3 = shl<3>(tp[i][3]);
                                const C r1 = shl<1>(tg[i][1]), r2 = shl<2>(tg[i][2]), r3 = shl<3>(tg[i][3]);
                                const C dflt = i == 0 ? C(1) : (i == 4 ? C(2) : C(0));  // lanes without a point
                                ql[i] = col == 15 ? tp[i][0] : (col == 14 ? l1 : (col == 13 ? l2 : (col == 12 ? l3 : dflt)));
                                qr[i] = col == 15 ? tg[i][0] : (col == 14 ? r1 : (col == 13 ? r2 : (col == 12 ? r3 : dflt)));
                            }
                            if constexpr (RS == 1)
                                exact_rs<PR, 0>(ql, qr, gam, fo);
                            else
                                hllc<PR, 0>(ql, qr, gam, fo);
    #pragma unroll
                            for (int i = 0; i < NF; i++) {
                                Fxp[i][0] = fo[i];
                                Fxp[i][1] = shr<1>(fo[i]);
                                Fxp[i][2] = shr<2>(fo[i]);
                                Fxp[i][3] = shr<3>(fo[i]);
                            }
                        }
    #pragma unroll
                        for (int i = 0; i < NF; i++)
    #pragma unroll
                            for (int r = 0; r < 4; r++) {
                                const C sh = shr<1>(tp[i][r]);  // DPP outside any select: every lane active
                                tl[i][r] = gl ? tg[i][r] : sh;
                            }
                    }
                    C Fxm[NF][4];
                    riemann(std::integral_constant<int, 0>{}, tl, tm, Fxm);
                    // the + face flux of a column is the - face flux of its right neighbour; column 15
                    // of a full block keeps the flux of its high edge
                    const bool edge = vc == K3_BLK && col == 15;
    #pragma unroll
                    for (int i = 0; i < NF; i++)
    #pragma unroll
                        for (int r = 0; r < 4; r++) {
                            const C sh = shl<1>(Fxm[i][r]);
                            Fxp[i][r] = edge ? Fxp[i][r] : sh;
                        }
                    lift(0, cur, Fxm, Fxp, acc);
                }
            };
            // y faces shared by the rows of the workgroup: each face flux is solved once, by the
            // row below it; the faces at the group's ends use the neighbour rows' weights.  Row 0's
            // -y face is solved by four waves of SIMDs 1 and 2, one result register each (row 0
            // and the top row trace the end rows, on SIMDs 0 and 3), from row 0's -y trace in its
            // trace slot and the end row's +y trace in flux slot YROWS - 1 (no row's flux goes
            // there); the flux goes back into row 0's trace slot, which no other row reads, so
            // that nothing is held in registers across the two barriers
            C Fyp[NF][4];  // +y face flux of this row
            C tp[NF][4];   // +y trace, formed with the -y one from the same operands
            {
                C tm[NF][4];
                trace2(2, 3, cur, tm, tp);
                if (wrow == 0) {
                    C tb[NF][4];
                    trace_lds(3, 0, tb);
                    if (z + 1 < z1) load_lds(cidx(iy0 - 1, z + 1), 0);  // reads consumed above
                    ex_put(ex_f, YROWS - 1, tb);
                }
                ex_put(ex_t, wrow, tm);
            }
            if (XEARLY && wave < 4) xfaces(true);
            lds_barrier();
            // Issue priority: the two waves of a SIMD are rows w and w + 4.  By default the older
            // one (w < 4) wins issue, runs ahead through the faces and then waits at the next
            // barrier while its partner finishes alone; the younger one leads from here to the end
            // of the step, the older one the volume term, so the two reach the barriers together
            if (wave >= 4) __builtin_amdgcn_s_setprio(2);
            {
                C ta[NF][4];
                if (wrow == nact - 1) {
                    trace_lds(2, 1, ta);
                    if (z + 1 < z1) load_lds(cidx(iy0 + nact, z + 1), 1);  // reads consumed above
                } else {
                    ex_get(ex_t, wrow + 1 < YROWS ? wrow + 1 : wrow, ta);
                }
                riemann(std::integral_constant<int, 1>{}, tp, ta, Fyp);
                if (wrow < YROWS - 1) ex_put(ex_f, wrow, Fyp);  // the top row's flux has no reader here
                if (wave == 1 || wave == 2 || wave == 5 || wave == 6) {  // row 0's -y face, register r
                    const int r = wave == 1 ? 0 : (wave == 5 ? 1 : (wave == 2 ? 2 : 3));
                    C *pt = ex_t + r * 64 + lane_base();
                    const C *pb = ex_f + ((YROWS - 1) * NF * 4 + r) * 64 + lane_base();
                    C qL[5], qR[5], F[5];
#pragma unroll
                    for (int i = 0; i < NF; i++) {
                        qL[i] = pb[i * 4 * 64];
                        qR[i] = pt[i * 4 * 64];
                    }
                    if constexpr (RS == 1)
                        exact_rs<PR, 1>(qL, qR, gam, F);
                    else
                        hllc<PR, 1>(qL, qR, gam, F);
#pragma unroll
                    for (int i = 0; i < NF; i++) pt[i * 4 * 64] = F[i];
                }
            }
            lds_barrier();
            // the stage-combine input y0 (stages 2 and 3): slots 0..3 copied by the load unit into
            // this wave's trace slot (free until the next step's puts), requested now, so the round
            // trip hides behind the remaining faces; slot 4 is loaded into registers before the last
            // lift (held from here it would be spilled)
            auto y0_copy = [&]() {
                if (dma_y0 && act) {
                    const auto r0 = slab_rsrc(y0, slabn, cidx(iy, z));
                    lds_c *ydst = lds_dst(ex_t + wrow * NF * 4 * 64);
#pragma unroll
                    for (int u = 0; u < 4; u++)
#pragma unroll
                        for (int i = 0; i < NF; i++)
                            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                                r0, (__attribute__((address_space(3))) void *)(ydst + (i * 4 + u) * 64), 4,
                                roff[u] + xoff, (int)((unsigned)i * fbytes), 0, 0);
                }
            };
            C Fym[NF][4];  // -y face flux of this row: the +y flux of the row below, or row 0's own
            ex_get(wrow > 0 ? ex_f : ex_t, wrow > 0 ? wrow - 1 : 0, Fym);
            // the reads above have returned before the copy of y0 overwrites this wave's trace slot
            __builtin_amdgcn_s_waitcnt(WAIT_LGKM0);
            y0_copy();
            lift(1, cur, Fym, Fyp, acc);
            B3 nxt;
            loadz(iy, z + 1, nxt);
            if (!XEARLY || wave >= 4) xfaces(false);
            {  // +z face with block z+1; its flux is the -z flux of the next step
                C tp[NF][4], tm[NF][4];
                trace(5, cur, tp);
                trace(4, nxt, tm);
                riemann(std::integral_constant<int, 2>{}, tp, tm, Fz);
                lift(2, cur, nullptr, Fz, acc);
            }
            if constexpr (PREC == DG_FP32) {
#pragma unroll
                for (int i = 0; i < NF; i++) acc[i][1] = tile1_sum(acc[i][1]);
            }
            // combine and store; result slot s (row tile s / 4, register s % 4) is the mode this
            // lane loaded in slot s, so the stage input is still in registers.  The coefficients are
            // uniform: one branch-free path per kind of stage
            if (keep && act) {
                const long long rz = cidx(iy, z);
                const auto ro = slab_rsrc(out, slabn, rz);
                if (a.mode == 0) {
#pragma unroll
                    for (int i = 0; i < NF; i++)
#pragma unroll
                        for (int s = 0; s < NSL; s++) bstore(acc[i][s / 4][s % 4], ro, roff[s] + xoff, (unsigned)i * fbytes);
                } else {
                    const C ca = (C)a.a, cb = (C)a.b;
                    C y0v[NF][NSL];
                    if (dma_y0) {
                        // slots 0..3 were copied into this wave's trace slot after the y faces, slot 4 of
                        // fields 0..3 into its ghost slots after the ghost cells were read; vmcnt(0):
                        // the copies have landed (the compiler does not track them); the memory clobber
                        // keeps the LDS reads below the wait
                        __builtin_amdgcn_s_waitcnt(wait_vm(0));
                        asm volatile("" ::: "memory");
                        const C *y0s = ex_t + wrow * NF * 4 * 64 + lane_base();
                        const C *y0g = ex_g + lane_base();
#pragma unroll
                        for (int i = 0; i < NF; i++)
#pragma unroll
                            for (int s = 0; s < 4; s++) y0v[i][s] = y0s[(i * 4 + s) * 64];
#pragma unroll
                        for (int i = 0; i < 4; i++) y0v[i][4] = y0g[i * 64];
                        y0v[4][4] = y044;
                    } else {
#pragma unroll
                        for (int i = 0; i < NF; i++)
#pragma unroll
                            for (int s = 0; s < NSL; s++) y0v[i][s] = C(0);
                    }
#pragma unroll
                    for (int i = 0; i < NF; i++)
#pragma unroll
                        for (int s = 0; s < NSL; s++) {
                            const C res = ca * y0v[i][s] + cb * (cur.v[i][s] - dt * acc[i][s / 4][s % 4]);
                            bstore(res, ro, roff[s] + xoff, (unsigned)i * fbytes);
                        }
                }
            }
            // the next step's ghost cells, now that the combine has read slot 4 of y0 from their slots
            if (z + 1 < z1) {
                __builtin_amdgcn_s_waitcnt(WAIT_LGKM0);
                ghost_dma(cidx(iy, z + 1), x0);
            }
            if (wave >= 4) __builtin_amdgcn_s_setprio(0);
            cur = nxt;
        }
    }
}

// ------------------------------------------------------------------ driving factor table

// H_{c,n_x}(point) = sum over the modes with wave-number n_x (>= 0) of ahat_{m,c}
// exp(2 pi i (n_y Y + n_z Z)) exp(2 pi i n_x (1 + xi_a) / (2 nx)), at the 64 volume points of a
// cell of row (y, z) (Y, Z the points' coordinates, xi_a the point's x node), in FP64, stored as
// the A operand of the stage kernel's 16x16x4 FP32 product: for z-node t and K step s, lane L
// holds point 16 t + L % 16 and contraction index k = 4 s + L / 16 (k = 2 n_x: Re H,
// k = 2 n_x + 1: -Im H).
__global__ __launch_bounds__(256) void drive_table_k3_kernel(const double *__restrict__ modes, int nmodes, int dks,
                                                             int ny, int nz, GaussNodes xg, int nx, int z0, int nzg,
                                                             float *__restrict__ out) {
    const long long rowf = k3_drive_row_floats(dks);
    const long long total = (long long)ny * nz * rowf;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        const long long row = e / rowf;
        const int j = (int)(e - row * rowf);
        const int L = j % 64, s = (j / 64) % dks, t = (j / (64 * dks)) % 4, c = j / (64 * dks * 4);
        const int m = L % 16, k = 4 * s + L / 16;
        const int qa = m % 4, qb = m / 4, qc = t;
        const int iy = (int)(row % ny), iz = (int)(row / ny);
        const double Y = (iy + 0.5 * (1.0 + xg.x[qb])) / ny, Z = (z0 + iz + 0.5 * (1.0 + xg.x[qc])) / nzg;
        const double dx = 0.5 * (1.0 + xg.x[qa]) / nx;
        const int nxw = k / 2;
        double hr = 0.0, hi = 0.0;
        for (int md = 0; md < nmodes; md++) {
            const double *q = modes + 9 * md;
            if ((int)q[0] != nxw) continue;
            double ph = q[1] * Y + q[2] * Z + q[0] * dx;
            ph -= floor(ph);
            double sn, cs;
            sincospi(2.0 * ph, &sn, &cs);
            const double re = q[3 + 2 * c], im = q[4 + 2 * c];
            hr += re * cs - im * sn;
            hi += re * sn + im * cs;
        }
        out[e] = (float)((k & 1) ? -hi : hr);
    }
}

hipError_t launch_drive_table_k3(const double *modes, int nmodes, int dks, int ny, int nz, const GaussNodes &xg,
                                 int nx, int z0, int nzg, float *out, hipStream_t s) {
    const long long total = (long long)ny * nz * k3_drive_row_floats(dks);
    const long long nb = std::min<long long>((total + 255) / 256, 1LL << 20);
    hipLaunchKernelGGL(drive_table_k3_kernel, dim3((unsigned)nb), dim3(256), 0, s, modes, nmodes, dks, ny, nz, xg, nx,
                       z0, nzg, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ launch

template <int PREC>
static hipError_t launch_k3_t(const StageArgs &a, int grid, int lds_bytes, hipStream_t s) {
    if (a.riemann == 1) {
        if (a.forcing)
            hipLaunchKernelGGL((stage_k3_kernel<PREC, true, 1>), dim3(grid), dim3(K3_THREADS), lds_bytes, s, a);
        else
            hipLaunchKernelGGL((stage_k3_kernel<PREC, false, 1>), dim3(grid), dim3(K3_THREADS), lds_bytes, s, a);
    } else {
        if (a.forcing)
            hipLaunchKernelGGL((stage_k3_kernel<PREC, true, 0>), dim3(grid), dim3(K3_THREADS), lds_bytes, s, a);
        else
            hipLaunchKernelGGL((stage_k3_kernel<PREC, false, 0>), dim3(grid), dim3(K3_THREADS), lds_bytes, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_stage_k3(int prec, const StageArgs &a, int grid, int lds_bytes, hipStream_t s) {
    if (prec == DG_BF16X3) return launch_k3_t<DG_BF16X3>(a, grid, lds_bytes, s);
    if (prec == DG_BF16) return launch_k3_t<DG_BF16>(a, grid, lds_bytes, s);
    if (prec == DG_FP32) return launch_k3_t<DG_FP32>(a, grid, lds_bytes, s);
    return hipErrorInvalidValue;
}

template <int PREC>
static hipError_t set_attr_k3_t(int lds_bytes) {
    const void *fns[] = {reinterpret_cast<const void *>(&stage_k3_kernel<PREC, false, 0>),
                         reinterpret_cast<const void *>(&stage_k3_kernel<PREC, true, 0>),
                         reinterpret_cast<const void *>(&stage_k3_kernel<PREC, false, 1>),
                         reinterpret_cast<const void *>(&stage_k3_kernel<PREC, true, 1>)};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t set_stage_k3_attributes(int prec, int lds_bytes) {
    if (prec == DG_BF16X3) return set_attr_k3_t<DG_BF16X3>(lds_bytes);
    if (prec == DG_BF16) return set_attr_k3_t<DG_BF16>(lds_bytes);
    if (prec == DG_FP32) return set_attr_k3_t<DG_FP32>(lds_bytes);
    return hipErrorInvalidValue;
}

hipError_t stage_k3_occupancy(int prec, int lds_bytes, int *per_cu) {
    if (prec == DG_BF16X3)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, stage_k3_kernel<DG_BF16X3, true, 0>, K3_THREADS,
                                                            lds_bytes);
    if (prec == DG_BF16)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, stage_k3_kernel<DG_BF16, true, 0>, K3_THREADS,
                                                            lds_bytes);
    if (prec == DG_FP32)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, stage_k3_kernel<DG_FP32, true, 0>, K3_THREADS,
                                                            lds_bytes);
    return hipErrorInvalidValue;
}

}  // namespace dgmi
