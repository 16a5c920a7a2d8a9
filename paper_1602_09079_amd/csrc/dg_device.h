// Device helpers shared by the stage kernels of libdgmi.so (dg_kernels.hip, stage_k3.hip):
// vector types, BF16 operand splits, the precision policies of the matrix-core products, DPP
// lane shifts, the pointwise physics (ideal-gas Euler flux, HLLC and exact Riemann fluxes) and
// buffer access to (z, y) slabs of the state.  Not part of the ABI.
#pragma once
#include "dg_internal.h"

namespace dgmi {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef float fv2 __attribute__((ext_vector_type(2)));
typedef __bf16 bv2 __attribute__((ext_vector_type(2)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

// round-to-nearest-even float -> bf16 conversion of pairs (one v_cvt_pk_bf16_f32 each)
template <int L, class V>
__device__ inline void to_bf16(const float *v, V &out) {
#pragma unroll
    for (int j = 0; j < L; j += 2) {
        const bv2 h = __builtin_convertvector((fv2){v[j], v[j + 1]}, bv2);
        out[j] = h[0];
        out[j + 1] = h[1];
    }
}
// x = hi + lo split: hi = bf16(x), lo = bf16(x - hi)
template <int L, class V>
__device__ inline void to_bf16x2(const float *v, V &hi, V &lo) {
#pragma unroll
    for (int j = 0; j < L; j += 2) {
        const bv2 h = __builtin_convertvector((fv2){v[j], v[j + 1]}, bv2);
        const fv2 hf = __builtin_convertvector(h, fv2);
        const bv2 l = __builtin_convertvector((fv2){v[j] - hf[0], v[j + 1] - hf[1]}, bv2);
        hi[j] = h[0];
        hi[j + 1] = h[1];
        lo[j] = l[0];
        lo[j + 1] = l[1];
    }
}

template <int K>
struct Dims {
    static constexpr int N = (K + 1) * (K + 2) * (K + 3) / 6;
    static constexpr int n = K + 1;
    static constexpr int Q = n * n * n;
    static constexpr int P = n * n;
};

// ------------------------------------------------------------------ precision policies
//
// S: storage type; C: pointwise arithmetic; Acc: MFMA accumulator.
// AF/BF: wide A/B operands (GEMM1/3/4), AF2/BF2: narrow ones (GEMM2/5).

template <int PREC>
struct Prec;

template <>
struct Prec<DG_FP64> {
    using S = double;
    using C = double;
    using Acc = d4;
    static constexpr int KPL = 1, KPL2 = 1, KSTEP = 4, ESZ = 8;
    struct AF { double v; };
    using AF2 = AF;
    struct BF { double v; };
    using BF2 = BF;
    __device__ static AF lda(const char *p) { return AF{*reinterpret_cast<const double *>(p)}; }
    __device__ static AF2 lda2(const char *p) { return lda(p); }
    __device__ static Acc mma(Acc c, AF a, BF b) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a.v, b.v, c, 0, 0, 0); }
    __device__ static Acc mma2(Acc c, AF2 a, BF2 b) { return mma(c, a, b); }
    __device__ static int orow(int g, int r) { return g + 4 * r; }
    __device__ static BF mkb(const C *v) { return BF{v[0]}; }
    __device__ static BF2 mkb2(const C *v) { return BF{v[0]}; }
    __device__ static C rcp(C x) { return 1.0 / x; }
    __device__ static C sqrt_(C x) { return __builtin_sqrt(x); }
};

template <>
struct Prec<DG_FP32> {
    using S = float;
    using C = float;
    using Acc = f4;
    static constexpr int KPL = 1, KPL2 = 1, KSTEP = 4, ESZ = 4;
    struct AF { float v; };
    using AF2 = AF;
    struct BF { float v; };
    using BF2 = BF;
    __device__ static AF lda(const char *p) { return AF{*reinterpret_cast<const float *>(p)}; }
    __device__ static AF2 lda2(const char *p) { return lda(p); }
    __device__ static Acc mma(Acc c, AF a, BF b) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a.v, b.v, c, 0, 0, 0); }
    __device__ static Acc mma2(Acc c, AF2 a, BF2 b) { return mma(c, a, b); }
    __device__ static int orow(int g, int r) { return 4 * g + r; }
    __device__ static BF mkb(const C *v) { return BF{v[0]}; }
    __device__ static BF2 mkb2(const C *v) { return BF{v[0]}; }
    __device__ static C rcp(C x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static C sqrt_(C x) { return __builtin_amdgcn_sqrtf(x); }
};

template <>
struct Prec<DG_BF16> {
    using S = float;
    using C = float;
    using Acc = f4;
    static constexpr int KPL = 8, KPL2 = 4, KSTEP = 32, ESZ = 2;
    struct AF { bf8 v; };
    struct AF2 { bf4 v; };
    struct BF { bf8 v; };
    struct BF2 { bf4 v; };
    __device__ static AF lda(const char *p) { return AF{*reinterpret_cast<const bf8 *>(p)}; }
    __device__ static AF2 lda2(const char *p) { return AF2{*reinterpret_cast<const bf4 *>(p)}; }
    __device__ static Acc mma(Acc c, AF a, BF b) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, c, 0, 0, 0); }
    __device__ static Acc mma2(Acc c, AF2 a, BF2 b) {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a.v), __builtin_bit_cast(s4, b.v), c, 0,
                                                          0, 0);
    }
    __device__ static int orow(int g, int r) { return 4 * g + r; }
    __device__ static BF mkb(const C *v) {
        BF b;
        to_bf16<8>(v, b.v);
        return b;
    }
    __device__ static BF2 mkb2(const C *v) {
        BF2 b;
        to_bf16<4>(v, b.v);
        return b;
    }
    __device__ static C rcp(C x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static C sqrt_(C x) { return __builtin_amdgcn_sqrtf(x); }
};

// FP32-grade contractions on BF16 matrix cores: x = hi + lo with hi = bf16(x),
// lo = bf16(x - hi); a*b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b (lo_a lo_b dropped,
// relative size 2^-18).  The lo tables follow the hi tables at +LO bytes.
template <>
struct Prec<DG_BF16X3> {
    using S = float;
    using C = float;
    using Acc = f4;
    static constexpr int KPL = 8, KPL2 = 4, KSTEP = 32, ESZ = 2;
    struct AF { bf8 hi, lo; };
    struct AF2 { bf4 hi, lo; };
    struct BF { bf8 hi, lo; };
    struct BF2 { bf4 hi, lo; };
    static __device__ inline int lo_bytes();
    __device__ static Acc mma(Acc c, AF a, BF b) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b.hi, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.lo, c, 0, 0, 0);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.hi, c, 0, 0, 0);
    }
    __device__ static Acc mma2(Acc c, AF2 a, BF2 b) {
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a.lo), __builtin_bit_cast(s4, b.hi), c, 0,
                                                       0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a.hi), __builtin_bit_cast(s4, b.lo), c, 0,
                                                       0, 0);
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a.hi), __builtin_bit_cast(s4, b.hi), c,
                                                          0, 0, 0);
    }
    __device__ static int orow(int g, int r) { return 4 * g + r; }
    __device__ static BF mkb(const C *v) {
        BF b;
        to_bf16x2<8>(v, b.hi, b.lo);
        return b;
    }
    __device__ static BF2 mkb2(const C *v) {
        BF2 b;
        to_bf16x2<4>(v, b.hi, b.lo);
        return b;
    }
    __device__ static C rcp(C x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static C sqrt_(C x) { return __builtin_amdgcn_sqrtf(x); }
};

// ------------------------------------------------------------------ lane exchange (DPP row shifts)

__device__ inline float dpp_shr1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, true));
}
__device__ inline float dpp_shl1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x101, 0xf, 0xf, true));
}
__device__ inline double dpp_shr1(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x111, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x111, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double dpp_shl1(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x101, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x101, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ------------------------------------------------------------------ pointwise physics

// Ideal-gas Euler flux along the three axes at one point, Sec. 2.3.
template <class PR, class C>
__device__ inline void euler_flux3(const C q[5], C g1, C F[3][5]) {
    const C inv = PR::rcp(q[0]);
    const C u = q[1] * inv, v = q[2] * inv, w = q[3] * inv;
    const C p = g1 * (q[4] - C(0.5) * (q[1] * u + q[2] * v + q[3] * w));
    const C ep = q[4] + p;
    F[0][0] = q[1]; F[0][1] = q[1] * u + p; F[0][2] = q[2] * u; F[0][3] = q[3] * u; F[0][4] = ep * u;
    F[1][0] = q[2]; F[1][1] = q[1] * v;     F[1][2] = q[2] * v + p; F[1][3] = q[3] * v; F[1][4] = ep * v;
    F[2][0] = q[3]; F[2][1] = q[1] * w;     F[2][2] = q[2] * w; F[2][3] = q[3] * w + p; F[2][4] = ep * w;
}

// HLLC numerical flux across a face normal to AXIS, left state qL, right state
// qR (Toro, Riemann Solvers and Numerical Methods for Fluid Dynamics, ch. 10:
// Davis wave-speed bounds; the star flux F*_K = F_K + S_K (U*_K - U_K) of the star-state
// form, written as
//   F*_K = F_K + S_K / (S_K - S*) (S* U_K - F_K + p* D*),  D* = (0, n, S*),
//   p* = p_K + rho_K (S_K - u_K)(S* - u_K)).  S* >= 0 takes the left star state.
// Branch-free: side K is selected first, only its flux is formed; where the face lies
// outside the star region the coefficient of the correction is zero.
template <class PR, int AXIS, class C>
__device__ inline void hllc(const C qL[5], const C qR[5], C gam, C F[5]) {
    const C g1 = gam - C(1);
    const C iL = PR::rcp(qL[0]), iR = PR::rcp(qR[0]);
    const C uL = qL[1 + AXIS] * iL, uR = qR[1 + AXIS] * iR;
    const C pL = g1 * (qL[4] - C(0.5) * (qL[1] * qL[1] + qL[2] * qL[2] + qL[3] * qL[3]) * iL);
    const C pR = g1 * (qR[4] - C(0.5) * (qR[1] * qR[1] + qR[2] * qR[2] + qR[3] * qR[3]) * iR);
    const C cL = PR::sqrt_(gam * pL * iL), cR = PR::sqrt_(gam * pR * iR);
    const C SL = __builtin_fmin(uL - cL, uR - cR);
    const C SR = __builtin_fmax(uL + cL, uR + cR);
    const C sL = SL - uL, sR = SR - uR;
    const C dL = qL[0] * sL, dR = qR[0] * sR;
    const C Ss = (pR - pL + qL[1 + AXIS] * sL - qR[1 + AXIS] * sR) * PR::rcp(dL - dR);
    const bool left = (Ss >= C(0)) || (SL >= C(0));
    C q[5];
#pragma unroll
    for (int i = 0; i < 5; i++) q[i] = left ? qL[i] : qR[i];
    const C uK = left ? uL : uR, pK = left ? pL : pR, SK = left ? SL : SR, dK = left ? dL : dR;
    C FK[5];
    FK[0] = q[1 + AXIS];
#pragma unroll
    for (int j = 0; j < 3; j++) FK[1 + j] = q[1 + j] * uK;
    FK[1 + AXIS] += pK;
    FK[4] = (q[4] + pK) * uK;
    const bool plain = (SL >= C(0)) || (!left && SR <= C(0));
    const C pst = pK + dK * (Ss - uK);
    const C cf = plain ? C(0) : SK * PR::rcp(SK - Ss);
    C t[5];
#pragma unroll
    for (int i = 0; i < 5; i++) t[i] = Ss * q[i] - FK[i];
    t[1 + AXIS] += pst;
    t[4] += pst * Ss;
#pragma unroll
    for (int i = 0; i < 5; i++) F[i] = FK[i] + cf * t[i];
}

// x^y for x > 0 in the precision of C (FP32: hardware base-2 logarithm and exponential)
__device__ inline float powpos(float x, float y) { return __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(x)); }
__device__ inline double powpos(double x, double y) { return pow(x, y); }

// Exact Riemann solver (the alternative to HLLC; Toro, Riemann Solvers and Numerical Methods
// for Fluid Dynamics, ch. 4) across a face normal to AXIS.  The star pressure p* is the root of
// f_L(p) + f_R(p) + u_R - u_L, each f_K the shock branch (p > p_K) or the rarefaction branch,
// found by Newton from the primitive-variable estimate, kept positive; the wave pattern is
// sampled at x/t = 0 and the Euler flux of that state returned, the tangential velocities
// taken from the side of the contact the face lies on.  Vacuum-generating data (2(c_L + c_R)/
// (gamma-1) <= u_R - u_L) are sampled from the two rarefactions and the vacuum between them.
template <class PR, int AXIS, class C>
__device__ inline void exact_rs(const C qL[5], const C qR[5], C gam, C F[5]) {
    // quotients as products with reciprocals (PR::rcp: the hardware reciprocal in the FP32 tiers,
    // 1/x in FP64); the ones of gamma alone are wave-uniform
    const C g1 = gam - C(1), gp = gam + C(1), z = g1 * PR::rcp(C(2) * gam);
    const C g1i = PR::rcp(g1), gpi = PR::rcp(gp);
    const C iL = PR::rcp(qL[0]), iR = PR::rcp(qR[0]);
    const C rL = qL[0], rR = qR[0];
    const C uL = qL[1 + AXIS] * iL, uR = qR[1 + AXIS] * iR;
    const C pL = g1 * (qL[4] - C(0.5) * (qL[1] * qL[1] + qL[2] * qL[2] + qL[3] * qL[3]) * iL);
    const C pR = g1 * (qR[4] - C(0.5) * (qR[1] * qR[1] + qR[2] * qR[2] + qR[3] * qR[3]) * iR);
    const C cL = PR::sqrt_(gam * pL * iL), cR = PR::sqrt_(gam * pR * iR);
    const C ipL = PR::rcp(pL), ipR = PR::rcp(pR);
    // f_K and its derivative (shock: A_K = 2 / ((gamma + 1) rho_K), B_K = (gamma - 1) / (gamma + 1) p_K)
    auto wave = [&](C p, C iK, C pK, C ipK, C cK, C &df) -> C {
        if (p > pK) {
            const C A = C(2) * gpi * iK, Bk = g1 * gpi * pK;
            const C ipb = PR::rcp(p + Bk);
            const C sq = PR::sqrt_(A * ipb);
            df = sq * (C(1) - C(0.5) * (p - pK) * ipb);
            return (p - pK) * sq;
        }
        const C pr = p * ipK;
        const C t = powpos(pr, z);
        df = t * PR::rcp(pr * cK) * iK;
        return C(2) * cK * g1i * (t - C(1));
    };
    C W0, W1, W2;  // face state: rho, normal velocity, pressure
    bool from_left;
    const C du = uR - uL;
    auto fan = [&](C rK, C uK, C pK, C cK, C sgn) {  // sgn = -1 left fan, +1 right fan
        const C c = C(2) * gpi - sgn * g1 * gpi * PR::rcp(cK) * uK;
        W0 = rK * powpos(c, C(2) * g1i);
        W1 = C(2) * gpi * (-sgn * cK + C(0.5) * g1 * uK);
        W2 = pK * powpos(c, C(2) * gam * g1i);
    };
    if (C(2) * (cL + cR) * g1i <= du) {
        const C sL = uL + C(2) * cL * g1i, sR = uR - C(2) * cR * g1i;
        if (C(0) <= sL) {
            from_left = true;
            if (C(0) <= uL - cL) { W0 = rL; W1 = uL; W2 = pL; }
            else fan(rL, uL, pL, cL, C(-1));
        } else if (C(0) >= sR) {
            from_left = false;
            if (C(0) >= uR + cR) { W0 = rR; W1 = uR; W2 = pR; }
            else fan(rR, uR, pR, cR, C(1));
        } else {
            from_left = true;
            W0 = C(0); W1 = C(0); W2 = C(0);
        }
    } else {
        const C tiny = (sizeof(C) == 8 ? C(1e-300) : C(1e-30));
        C p = C(0.5) * (pL + pR) - C(0.125) * du * (rL + rR) * (cL + cR);
        p = p > tiny ? p : tiny;
        // Newton converges quadratically: the error after a step is about the square of the step
        // (relative), so a step below tol2 (about the square root of the unit roundoff, with a
        // margin for the curvature of f) leaves p at rounding, and the iteration stops there
        const C tol2 = sizeof(C) == 8 ? C(1e-9) : C(2.5e-5);
        C fl = 0, fr = 0, sl = 0, sr = 0, pold = p;  // the last evaluation: f_L, f_R, their slopes, at pold
        for (int it = 0; it < 24; it++) {
            C dfL, dfR;
            const C a = wave(p, iL, pL, ipL, cL, dfL), b = wave(p, iR, pR, ipR, cR, dfR);
            C pn = p - (a + b + du) * PR::rcp(dfL + dfR);
            pn = pn > tiny ? pn : C(0.1) * p;
            const C ch = __builtin_fabs(pn - p) * PR::rcp(pn + p);
            fl = a; fr = b; sl = dfL; sr = dfR; pold = p;
            p = pn;
            if (ch <= tol2) break;
        }
        // u* from f_R(p*) - f_L(p*), each one step of size below tol2 from its last evaluation: the
        // first-order update is exact to rounding
        const C dp = p - pold;
        const C us = C(0.5) * (uL + uR) + C(0.5) * ((fr + sr * dp) - (fl + sl * dp));
        from_left = C(0) <= us;
        const C rK = from_left ? rL : rR, uK = from_left ? uL : uR, pK = from_left ? pL : pR;
        const C cK = from_left ? cL : cR, sg = from_left ? C(-1) : C(1);
        const C ppK = p * (from_left ? ipL : ipR);  // p* / p_K
        // in the frame mirrored for the right side, every test reads as for the left side
        if (p > pK) {
            const C h2g = C(0.5) * PR::rcp(gam);
            const C S = uK + sg * cK * PR::sqrt_(gp * h2g * ppK + g1 * h2g);
            if (sg * S <= C(0)) { W0 = rK; W1 = uK; W2 = pK; }
            else {
                W0 = rK * (ppK + g1 * gpi) * PR::rcp(g1 * gpi * ppK + C(1));
                W1 = us; W2 = p;
            }
        } else {
            const C head = uK + sg * cK;
            const C tail = us + sg * cK * powpos(ppK, z);
            if (sg * head <= C(0)) { W0 = rK; W1 = uK; W2 = pK; }
            else if (sg * tail >= C(0)) { W0 = rK * powpos(ppK, PR::rcp(gam)); W1 = us; W2 = p; }
            else fan(rK, uK, pK, cK, sg);
        }
    }
    const C *qt = from_left ? qL : qR;
    const C it = from_left ? iL : iR;
    C v[3];
#pragma unroll
    for (int a = 0; a < 3; a++) v[a] = qt[1 + a] * it;
    v[AXIS] = W1;
    const C E = W2 * g1i + C(0.5) * W0 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const C mflux = W0 * W1;
    F[0] = mflux;
#pragma unroll
    for (int a = 0; a < 3; a++) F[1 + a] = mflux * v[a];
    F[1 + AXIS] += W2;
    F[4] = W1 * (E + W2);
}

// Buffer access to one (z, y) slab of a state: the state is stored
// [z][y][i][l][x], so the 5 N rows of a y-row of cells (one per field and mode)
// are one contiguous slab.  A resource per slab (base, size in bytes), a per-lane
// byte offset in a VGPR (mode row and x) and a wave-uniform byte offset in an
// SGPR (field).  All offsets the kernel forms lie inside the slab.
constexpr int BUF_DWORD3 = 0x00020000;  // 32-bit data format (gfx9 family)

// The base is passed through an opaque copy so the resource is rebuilt (a few
// scalar instructions) where it is used instead of being kept live in SGPRs.
template <class S>
__device__ inline __amdgpu_buffer_rsrc_t slab_rsrc(const S *base, long long slab_elems, long long r) {
    const S *p = base + r * slab_elems;
    asm volatile("" : "+s"(p));
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<S *>(p), (short)0,
                                             (int)(unsigned)(slab_elems * (long long)sizeof(S)), BUF_DWORD3);
}
__device__ inline float bload(float, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ inline double bload(double, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ inline void bstore(float v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff = 0) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, 0);
}
__device__ inline void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff = 0) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, 0);
}

}  // namespace dgmi
