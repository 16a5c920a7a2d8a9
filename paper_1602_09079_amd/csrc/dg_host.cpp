// Host half of libdgmi.so: configuration checks, quadrature and basis tables
// (Sec. 2.1-2.2 of arXiv 1602.09079) and the C ABI declared in include/dg.h.
//
// The tables come from closed forms: Gauss-Legendre nodes and weights for
// n <= 5 and the explicit Legendre polynomials of degree <= 4.  They are
// rearranged on the host into the per-lane operand order of the MFMA
// instructions the stage kernel issues, so that the kernel's loads from LDS are
// contiguous and the chained products need no data movement.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dg_internal.h"

using namespace dgmi;

namespace {

// ---------------------------------------------------------------- closed-form quadrature

bool gauss_rule(int n, double *x, double *w) {
    switch (n) {
        case 1: x[0] = 0.0; w[0] = 2.0; return true;
        case 2: {
            const double a = 1.0 / std::sqrt(3.0);
            x[0] = -a; x[1] = a; w[0] = w[1] = 1.0;
            return true;
        }
        case 3: {
            const double a = std::sqrt(0.6);
            x[0] = -a; x[1] = 0.0; x[2] = a;
            w[0] = w[2] = 5.0 / 9.0; w[1] = 8.0 / 9.0;
            return true;
        }
        case 4: {
            const double r = 2.0 / 7.0 * std::sqrt(6.0 / 5.0);
            const double xi = std::sqrt(3.0 / 7.0 - r), xo = std::sqrt(3.0 / 7.0 + r);
            const double wi = (18.0 + std::sqrt(30.0)) / 36.0, wo = (18.0 - std::sqrt(30.0)) / 36.0;
            x[0] = -xo; x[1] = -xi; x[2] = xi; x[3] = xo;
            w[0] = wo; w[1] = wi; w[2] = wi; w[3] = wo;
            return true;
        }
        case 5: {
            const double r = 2.0 * std::sqrt(10.0 / 7.0);
            const double xi = std::sqrt(5.0 - r) / 3.0, xo = std::sqrt(5.0 + r) / 3.0;
            const double wi = (322.0 + 13.0 * std::sqrt(70.0)) / 900.0, wo = (322.0 - 13.0 * std::sqrt(70.0)) / 900.0;
            x[0] = -xo; x[1] = -xi; x[2] = 0.0; x[3] = xi; x[4] = xo;
            w[0] = wo; w[1] = wi; w[2] = 128.0 / 225.0; w[3] = wi; w[4] = wo;
            return true;
        }
        default: return false;
    }
}

// Gauss-Lobatto nodes per axis of the limiter's point set (Sec. 2.5): the fewest whose rule is
// exact for degree k (2m - 3 >= k), which gives the paper's first weights 1 (second order) and
// 1/3 (third and fourth order), and 1/6 at k = 4
int limiter_gll_points(int k) { return k <= 1 ? 2 : (k <= 3 ? 3 : 4); }

// explicit Legendre polynomials P_u and derivatives, u <= 4, times sqrt(2u+1)
double leg(int u, double x) {
    double p;
    switch (u) {
        case 0: p = 1.0; break;
        case 1: p = x; break;
        case 2: p = 0.5 * (3.0 * x * x - 1.0); break;
        case 3: p = 0.5 * (5.0 * x * x * x - 3.0 * x); break;
        default: p = 0.125 * (35.0 * x * x * x * x - 30.0 * x * x + 3.0); break;
    }
    return std::sqrt(2.0 * u + 1.0) * p;
}
double dleg(int u, double x) {
    double p;
    switch (u) {
        case 0: p = 0.0; break;
        case 1: p = 1.0; break;
        case 2: p = 3.0 * x; break;
        case 3: p = 0.5 * (15.0 * x * x - 3.0); break;
        default: p = 0.5 * (35.0 * x * x * x - 15.0 * x); break;
    }
    return std::sqrt(2.0 * u + 1.0) * p;
}

struct Basis {
    int k, N, n, Q, P;
    double xg[5], wg[5];
    std::vector<int> u, v, w;  // degrees per mode
    explicit Basis(int k_) : k(k_), N(nmodes_of(k_)), n(k_ + 1), Q(n * n * n), P(n * n) {
        gauss_rule(n, xg, wg);
        for (int d = 0; d <= k; d++)          // graded by total degree,
            for (int a = d; a >= 0; a--)      // then x-degree descending,
                for (int b = d - a; b >= 0; b--) {  // then y-degree descending
                    u.push_back(a);
                    v.push_back(b);
                    w.push_back(d - a - b);
                }
    }
    void point(int q, double xi[3]) const {  // volume point q = (c n + b) n + a
        xi[0] = xg[q % n];
        xi[1] = xg[(q / n) % n];
        xi[2] = xg[q / (n * n)];
    }
    double weight(int q) const { return wg[q % n] * wg[(q / n) % n] * wg[q / (n * n)]; }
    void face_point(int face, int p, double xi[3]) const {
        // face = 2*axis + side; points run over the other two axes, lower axis fastest
        const int axis = face / 2;
        const int o0 = axis == 0 ? 1 : 0, o1 = axis == 2 ? 1 : 2;
        xi[axis] = (face & 1) ? 1.0 : -1.0;
        xi[o0] = xg[p % n];
        xi[o1] = xg[p / n];
    }
    double face_weight(int p) const { return wg[p % n] * wg[p / n]; }
    double phi(int l, const double xi[3]) const { return leg(u[l], xi[0]) * leg(v[l], xi[1]) * leg(w[l], xi[2]); }
    double dphi(int l, int a, const double xi[3]) const {
        return (a == 0 ? dleg(u[l], xi[0]) : leg(u[l], xi[0])) * (a == 1 ? dleg(v[l], xi[1]) : leg(v[l], xi[1])) *
               (a == 2 ? dleg(w[l], xi[2]) : leg(w[l], xi[2]));
    }
};

uint16_t bf16_rne(float f) {
    uint32_t b;
    std::memcpy(&b, &f, 4);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}
float bf16_to_float(uint16_t h) {
    uint32_t b = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}

// Build the MFMA operand tables.  A fragment holds, for each of the 64 lanes,
// the values that lane feeds to one MFMA as its A operand: row = lane % 16,
// contraction index = (lane / 16) * kpl + j.  Contraction indices over volume
// or face points are permuted to match the lane layout of the MFMA results that
// are fed as B operands (see out_row).
std::vector<char> build_tables(const TableLayout &L, const double s[3]) {
    const Basis B(L.k);
    const int N = L.N, Q = L.Q, P = L.P;
    // values in FP64, one vector per table: [frag][lane][j]
    std::vector<double> t1((size_t)L.rt1 * L.ks1 * 64 * L.kpl, 0.0), t2((size_t)L.rt2 * 3 * L.nc2 * 64 * L.kpl2, 0.0),
        t3((size_t)6 * L.ks1 * 64 * L.kpl, 0.0), t4((size_t)L.rt2 * L.nc4 * 64 * L.kpl2, 0.0),
        t5((size_t)L.rt2 * L.nc2 * 64 * L.kpl2, 0.0);
    auto vol_point = [&](int chunk, int g, int j) {  // volume point at contraction slot (g, j) of a chunk
        if (L.kpl2 == 1) return 16 * (chunk / 4) + out_row(L.prec, g, chunk % 4);
        return 16 * chunk + out_row(L.prec, g, j);
    };
    auto face_slot = [&](int chunk, int g, int j, int &face) {  // (face, point) at slot (g, j)
        if (L.kpl2 == 1) {
            face = chunk / 4;
            return out_row(L.prec, g, chunk % 4);
        }
        face = chunk;
        return out_row(L.prec, g, j);
    };
    double xi[3];
    // mode of B-operand value (K-step st, lane group g, value j) of GEMM1/GEMM3
    auto in_mode = [&](int st, int g, int j) {
        return L.kpl == 1 ? slot_mode(N, g, st) : (st == 0 ? slot_mode(N, g, j) : N);
    };
    // mode of result row rho of GEMM2/4/5: the row lands in lane group g, register r of tile rho/16
    auto row_mode = [&](int rho) {
        const int rr = rho % 16;
        const int g = L.prec == DG_FP64 ? rr % 4 : rr / 4, r = L.prec == DG_FP64 ? rr / 4 : rr % 4;
        return slot_mode(N, g, 4 * (rho / 16) + r);
    };
    for (int lane = 0; lane < 64; lane++) {
        const int row = lane % 16, g = lane / 16;
        for (int j = 0; j < L.kpl; j++) {
            for (int t = 0; t < L.rt1; t++)  // T1: Phi[q][m]
                for (int st = 0; st < L.ks1; st++) {
                    const int q = 16 * t + row, m = in_mode(st, g, j);
                    if (q < Q && m >= 1 && m < N) {  // mode 0 (the mean) is added apart
                        B.point(q, xi);
                        t1[(((size_t)t * L.ks1 + st) * 64 + lane) * L.kpl + j] = B.phi(m, xi);
                    }
                }
            for (int f = 0; f < 6; f++)  // T3: Phi[face point][m]
                for (int st = 0; st < L.ks1; st++) {
                    const int p = row, m = in_mode(st, g, j);
                    if (p < P && m >= 1 && m < N) {  // mode 0 (the mean) is added apart
                        B.face_point(f, p, xi);
                        t3[(((size_t)f * L.ks1 + st) * 64 + lane) * L.kpl + j] = B.phi(m, xi);
                    }
                }
        }
        for (int j = 0; j < L.kpl2; j++) {
            for (int rt = 0; rt < L.rt2; rt++)  // T4: s_a (+-1) Phi[m][face point] w_p, outward normal
                for (int c = 0; c < L.nc4; c++) {
                    int f;
                    const int p = face_slot(c, g, j, f);
                    const int m = row_mode(16 * rt + row);
                    if (p < P && m < N) {
                        B.face_point(f, p, xi);
                        const double sg = (f & 1) ? 1.0 : -1.0;
                        t4[(((size_t)rt * L.nc4 + c) * 64 + lane) * L.kpl2 + j] = s[f / 2] * sg * B.phi(m, xi) * B.face_weight(p);
                    }
                }
            for (int rt = 0; rt < L.rt2; rt++)
                for (int c = 0; c < L.nc2; c++) {
                    const int m = row_mode(16 * rt + row), q = vol_point(c, g, j);
                    if (q < Q && m < N) {
                        B.point(q, xi);
                        for (int a = 0; a < 3; a++)  // T2: -s_a dPhi_a[m][q] w_q
                            t2[((((size_t)rt * 3 + a) * L.nc2 + c) * 64 + lane) * L.kpl2 + j] =
                                -s[a] * B.dphi(m, a, xi) * B.weight(q);
                        // T5: -Phi[m][q] w_q / 8 (source projection)
                        t5[(((size_t)rt * L.nc2 + c) * 64 + lane) * L.kpl2 + j] = -B.phi(m, xi) * B.weight(q) / 8.0;
                    }
                }
        }
    }
    std::vector<char> blob(L.bytes(), 0);
    auto put = [&](const std::vector<double> &v, size_t off) {
        const size_t cnt = v.size();
        if (L.prec == DG_FP64) {
            std::memcpy(blob.data() + off, v.data(), cnt * 8);
        } else if (L.prec == DG_FP32) {
            float *o = reinterpret_cast<float *>(blob.data() + off);
            for (size_t i = 0; i < cnt; i++) o[i] = (float)v[i];
        } else {
            uint16_t *hi = reinterpret_cast<uint16_t *>(blob.data() + off);
            uint16_t *lo = reinterpret_cast<uint16_t *>(blob.data() + L.set_bytes + off);
            for (size_t i = 0; i < cnt; i++) {
                const uint16_t h = bf16_rne((float)v[i]);
                hi[i] = h;
                if (L.ntab == 2) lo[i] = bf16_rne((float)(v[i] - (double)bf16_to_float(h)));
            }
        }
    };
    put(t1, L.o1);
    put(t2, L.o2);
    put(t3, L.o3);
    put(t4, L.o4);
    put(t5, L.o5);
    return blob;
}

// Tables of the k = 3 FP32-storage stage kernel (stage_k3.hip), in its fragment order (K3_T1 ..
// K3_T4, 1 KiB each in BF16): lane L feeds row L % 16 and contraction indices 8 (L / 16) + j, j = 0..7.
// Products with the weights: index 8g + s is the mode of slot s of lane group g (k3_slot_mode),
// s < 5; mode 0 (the mean, added apart) and indices 8g + 5..7 are zero.  Products over points:
// index 8g + j is the result register j % 4 of lane group g of the preceding product, i.e. point
// 4g + j % 4 of the node (volume) or face, and j / 4 selects the first or second table of the
// chunk (x / y derivative; z derivative / source; - face / + face).  Result row 4g' + r' of row
// tile rt is slot 4 rt + r' of lane group g' (row tile 1: r' = 0 only).  After the LDS sets come
// the K3_NS mode-to-mode fragments of the mass flux's volume term (products with the momentum
// weights): the gradient tables contracted with the point values over the 64 volume points.
std::vector<char> build_tables_k3(int prec, const double s[3]) {
    const Basis B(3);
    std::vector<double> t((size_t)K3_NFRAG * 64 * 8, 0.0);
    auto at = [&](int frag, int lane, int j) -> double & { return t[((size_t)frag * 64 + lane) * 8 + j]; };
    std::vector<double> sm((size_t)K3_NS * 64 * 8, 0.0);
    auto rowmode = [](int rt, int row) {
        const int gg = row / 4, rr = row % 4;
        return rt == 0 ? k3_slot_mode(gg, rr) : (rr == 0 ? k3_slot_mode(gg, 4) : -1);
    };
    double xi[3];
    for (int lane = 0; lane < 64; lane++) {
        const int row = lane % 16, g = lane / 16;
        for (int j = 0; j < 8; j++) {
            const int m = j < 5 ? k3_slot_mode(g, j) : -1;
            const int pnt = 4 * g + (j % 4), half = j / 4;
            for (int tn = 0; tn < 4; tn++) {
                if (m > 0) {  // T1: phi at the node's volume points
                    B.point(16 * tn + row, xi);
                    at(K3_T1 + tn, lane, j) = B.phi(m, xi);
                }
                const int q = 16 * tn + pnt;
                B.point(q, xi);
                const int ma = rowmode(0, row);  // T2A: x and y derivatives, first row tile
                at(K3_T2A + tn, lane, j) = -s[half] * B.dphi(ma, half, xi) * B.weight(q);
                for (int rt = 0; rt < 2; rt++) {  // T2B: z derivative, then the source
                    const int mb = rowmode(rt, row);
                    if (mb < 0) continue;
                    at(K3_T2B + 2 * tn + rt, lane, j) =
                        half == 0 ? -s[2] * B.dphi(mb, 2, xi) * B.weight(q) : -B.phi(mb, xi) * B.weight(q) / 8.0;
                }
            }
            for (int f = 0; f < 6; f++)  // T3: phi at the face's points
                if (m > 0) {
                    B.face_point(f, row, xi);
                    at(K3_T3 + f, lane, j) = B.phi(m, xi);
                }
            // S: the mass flux's volume term from the momentum weights, sum over the 64 volume
            // points of -s_a dphi_a[mb](x_q) w_q phi[m](x_q)
            if (m > 0)
                for (int sf = 0; sf < K3_NS; sf++) {
                    const int ax = sf < 3 ? sf : 2, rt = sf < 3 ? 0 : 1;
                    const int mb = rowmode(rt, row);
                    if (mb < 0) continue;
                    double acc = 0.0;
                    for (int q = 0; q < 64; q++) {
                        B.point(q, xi);
                        acc += -s[ax] * B.dphi(mb, ax, xi) * B.weight(q) * B.phi(m, xi);
                    }
                    sm[((size_t)sf * 64 + lane) * 8 + j] = acc;
                }
            for (int ax = 0; ax < 3; ax++)  // T4: lift with the outward sign, - face then + face
                for (int rt = 0; rt < 2; rt++) {
                    const int mb = rowmode(rt, row);
                    if (mb < 0) continue;
                    const int f = 2 * ax + half;
                    B.face_point(f, pnt, xi);
                    at(K3_T4 + 2 * ax + rt, lane, j) = s[ax] * (half ? 1.0 : -1.0) * B.phi(mb, xi) * B.face_weight(pnt);
                }
        }
    }
    if (prec == DG_FP32) {
        // FP32: value j of lane l of a fragment is the A operand of step j of the chunk's eight
        // 16x16x4 products; stored [frag][j / 4][lane][j % 4] (one 16-byte read per four steps).
        // The second row tiles (one useful row per lane group) run as 4x4x1 products of 16
        // blocks: block 4g + c (lanes 4(4g + c) .. + 3) holds cells 4c .. 4c + 3 and contraction
        // index 8g + j, and its row i is row 4i of the tile, so lane l takes the value of lane
        // 4 (l % 4) + 16 (l / 16)
        std::vector<char> blob((size_t)K3_SET * 2 + (size_t)K3_NS * 2 * K3_FRAG, 0);
        float *f = reinterpret_cast<float *>(blob.data());
        for (int frag = 0; frag < K3_NFRAG + K3_NS; frag++) {
            const bool tile1 = (frag >= K3_T2B && frag < K3_T4 && (frag - K3_T2B) % 2 == 1) ||
                               (frag >= K3_T4 && frag < K3_NFRAG && (frag - K3_T4) % 2 == 1) ||
                               frag == K3_NFRAG + 3;
            for (int lane = 0; lane < 64; lane++) {
                const int src = tile1 ? 4 * (lane % 4) + 16 * (lane / 16) : lane;
                for (int j = 0; j < 8; j++)
                    f[((size_t)(2 * frag + j / 4) * 64 + lane) * 4 + j % 4] =
                        (float)(frag < K3_NFRAG ? at(frag, src, j) : sm[((size_t)(frag - K3_NFRAG) * 64 + src) * 8 + j]);
            }
        }
        return blob;
    }
    const int ntab = prec == DG_BF16X3 ? 2 : 1;
    constexpr size_t SB = (size_t)K3_NS * K3_FRAG;
    std::vector<char> blob(((size_t)K3_SET + SB) * ntab, 0);
    uint16_t *hi = reinterpret_cast<uint16_t *>(blob.data());
    uint16_t *lo = reinterpret_cast<uint16_t *>(blob.data() + K3_SET);
    for (size_t i = 0; i < t.size(); i++) {
        const uint16_t h = bf16_rne((float)t[i]);
        hi[i] = h;
        if (ntab == 2) lo[i] = bf16_rne((float)(t[i] - (double)bf16_to_float(h)));
    }
    uint16_t *shi = reinterpret_cast<uint16_t *>(blob.data() + (size_t)K3_SET * ntab);
    uint16_t *slo = reinterpret_cast<uint16_t *>(blob.data() + (size_t)K3_SET * ntab + SB);
    for (size_t i = 0; i < sm.size(); i++) {
        const uint16_t h = bf16_rne((float)sm[i]);
        shi[i] = h;
        if (ntab == 2) slo[i] = bf16_rne((float)(sm[i] - (double)bf16_to_float(h)));
    }
    return blob;
}

// Tables of the k = 4 matrix-core stage kernel (stage_k4.hip), K4_NFRAG fragments of 64 values
// in the storage precision, in the order of dg_internal.h.  Lane L feeds row L % 16 and K index
// L / 16 of a 16x16x4 product; in FP32 the last result tile (modes 32..34) runs as 4x4x1 products
// of 16 blocks, where lane L feeds row L % 4 of its block.  Cell c's weights are the B operand with
// mode 4s + g at K step s in lane group g.  A result lands in register r of lane group g from row
// 4g + r (FP32) or g + 4r (FP64); the row of mode 16 rt + 4 r + g is chosen so that lane group g
// gets the modes it holds.  The point and face-point products take K index g at step s to be the
// point in register s of lane group g of the product that made it.  Padding rows: the value and
// trace tables repeat the last point, the tables that take their results are zero there.
std::vector<char> build_tables_k4(int prec, const double s[3]) {
    const Basis B(4);
    constexpr int N = 35, Q = 125, P = 25;
    const bool f64 = prec == DG_FP64;
    std::vector<double> f((size_t)K4_NFRAG * 64, 0.0);
    auto at = [&](int frag, int lane) -> double & { return f[(size_t)frag * 64 + lane]; };
    // result row R of a 16x16 tile -> (lane group, register)
    auto grp = [&](int R) { return f64 ? R % 4 : R / 4; };
    auto reg = [&](int R) { return f64 ? R / 4 : R % 4; };
    auto rowmode = [&](int lane, int rt) {
        if (rt == 2 && !f64) return 32 + lane % 4;
        const int R = lane % 16;
        return 16 * rt + 4 * reg(R) + grp(R);
    };
    // the row of register r of lane group g
    auto row_of = [&](int g, int r) { return f64 ? g + 4 * r : 4 * g + r; };
    double xi[3];
    for (int lane = 0; lane < 64; lane++) {
        const int g = lane / 16;
        for (int t = 0; t < 8; t++) {
            const int qv = std::min(16 * t + lane % 16, Q - 1);  // the row's point (padding: the last)
            B.point(qv, xi);
            for (int st = 0; st < 9; st++) {
                const int l = 4 * st + g;
                if (l < N) at(K4_PHI + t * 9 + st, lane) = B.phi(l, xi);
            }
            for (int st = 0; st < 4; st++) {
                const int q = 16 * t + row_of(g, st);  // the K index's point
                if (q >= Q) continue;
                B.point(q, xi);
                for (int rt = 0; rt < 3; rt++) {
                    const int l = rowmode(lane, rt);
                    if (l >= N) continue;
                    for (int d = 0; d < 3; d++)
                        at(K4_GRAD + ((t * 3 + d) * 3 + rt) * 4 + st, lane) = -s[d] * B.weight(q) * B.dphi(l, d, xi);
                    at(K4_SRC + (t * 3 + rt) * 4 + st, lane) = -B.weight(q) * B.phi(l, xi) / 8.0;
                }
            }
        }
        for (int fc = 0; fc < 6; fc++) {
            for (int ft = 0; ft < 2; ft++) {
                B.face_point(fc, std::min(16 * ft + lane % 16, P - 1), xi);
                for (int st = 0; st < 9; st++) {
                    const int l = 4 * st + g;
                    if (l < N) at(K4_TRACE + (fc * 2 + ft) * 9 + st, lane) = B.phi(l, xi);
                }
            }
            for (int st = 0; st < 8; st++) {
                const int p = 16 * (st / 4) + row_of(g, st % 4);
                if (p >= P) continue;
                B.face_point(fc, p, xi);
                const double c = ((fc & 1) ? 1.0 : -1.0) * s[fc / 2] * B.face_weight(p);
                for (int rt = 0; rt < 3; rt++) {
                    const int l = rowmode(lane, rt);
                    if (l < N) at(K4_LIFT + (fc * 3 + rt) * 8 + st, lane) = c * B.phi(l, xi);
                }
            }
        }
    }
    std::vector<char> blob;
    if (f64) {
        blob.resize(f.size() * 8);
        std::memcpy(blob.data(), f.data(), blob.size());
    } else {
        std::vector<float> h(f.begin(), f.end());
        blob.resize(h.size() * 4);
        std::memcpy(blob.data(), h.data(), blob.size());
    }
    return blob;
}

const char *kNoCtx = "invalid or NULL dg_ctx";
// why the calling thread's last dg_init failed (no context survives to hold it)
thread_local std::string g_init_err;

dg_status hip_fail(dg_ctx *c, hipError_t e, const char *what) {
    if (c) c->err = std::string(what) + ": " + hipGetErrorString(e);
    return DG_ERR_HIP;
}

#define HIPCHK(ctx, call)                                      \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

size_t elem_bytes(const dg_ctx *c) { return c->cfg.precision == DG_FP64 ? 8 : 4; }

// C / (2k+1) (Sec. 2.4); with the positivity limiter C min(1/(2k+1), w_hat_1/2) (Sec. 2.5)
double dt_factor(const dg_ctx *c) {
    double f = 1.0 / (2.0 * c->cfg.k + 1.0);
    if (c->cfg.flags & DG_LIMIT) {
        const int m = limiter_gll_points(c->cfg.k);  // first Gauss-Lobatto weight: 1, 1/3, 1/6
        f = std::min(f, 0.5 * (m == 2 ? 1.0 : (m == 3 ? 1.0 / 3.0 : 1.0 / 6.0)));
    }
    return c->cfg.cfl * f;
}

}  // namespace

namespace dgmi {

TableLayout make_layout(int k, int prec) {
    TableLayout L{};
    L.k = k;
    L.prec = prec;
    L.N = nmodes_of(k);
    L.n = k + 1;
    L.Q = L.n * L.n * L.n;
    L.P = L.n * L.n;
    const bool bf = prec == DG_BF16 || prec == DG_BF16X3;
    L.kpl = bf ? 8 : 1;
    L.kpl2 = bf ? 4 : 1;
    L.kstep = 4 * L.kpl;
    L.ks1 = (L.N + L.kstep - 1) / L.kstep;
    L.rt1 = (L.Q + 15) / 16;
    L.rt2 = (L.N + 15) / 16;
    L.nc2 = bf ? L.rt1 : L.rt1 * 4;
    L.nc4 = bf ? 6 : 24;
    L.elem = prec == DG_FP64 ? 8 : (prec == DG_FP32 ? 4 : 2);
    L.fb1 = (size_t)64 * L.kpl * L.elem;
    L.fb2 = (size_t)64 * L.kpl2 * L.elem;
    L.o1 = 0;
    L.o2 = L.o1 + (size_t)L.rt1 * L.ks1 * L.fb1;
    L.o3 = L.o2 + (size_t)L.rt2 * 3 * L.nc2 * L.fb2;
    L.o4 = L.o3 + (size_t)6 * L.ks1 * L.fb1;
    L.o5 = L.o4 + (size_t)L.rt2 * L.nc4 * L.fb2;
    L.set_bytes = L.o5 + (size_t)L.rt2 * L.nc2 * L.fb2;
    L.ntab = prec == DG_BF16X3 ? 2 : 1;
    return L;
}

}  // namespace dgmi

hipError_t stage_occupancy(int k, int prec, int lds_bytes, int *blocks_per_cu);

// ====================================================================== ABI

extern "C" {

int32_t dg_nmodes(int32_t k) { return k >= 0 ? nmodes_of(k) : 0; }

dg_status dg_gauss_nodes(int32_t n, double *xi) {
    double w[5];
    if (!xi || n < 1 || n > 5) return DG_ERR_ARG;
    gauss_rule(n, xi, w);
    return DG_OK;
}

}  // extern "C"

void dgmi::set_call_error(const char *msg) { g_init_err = msg; }

extern "C" {

const char *dg_error_string(const dg_ctx *ctx) {
    if (ctx) return ctx->err.c_str();
    return g_init_err.empty() ? kNoCtx : g_init_err.c_str();
}

dg_status dg_init(const dg_config *cfg, void *hip_stream, dg_ctx **out) {
    g_init_err.clear();
    auto reject = [](dg_status st, const char *why) {
        g_init_err = std::string("dg_init: ") + why;
        return st;
    };
    if (!cfg || !out) return reject(DG_ERR_ARG, "NULL cfg or out");
    *out = nullptr;
    if (cfg->k < 0) return reject(DG_ERR_ARG, "k < 0");
    for (int a = 0; a < 3; a++)
        if (cfg->n[a] < 2 || !(cfg->box[a] > 0.0) || !std::isfinite(cfg->box[a]))
            return reject(DG_ERR_ARG, "n < 2 or box not positive and finite");
    if (!(cfg->gamma > 1.0) || !std::isfinite(cfg->gamma)) return reject(DG_ERR_ARG, "gamma <= 1");
    if (!(cfg->cfl > 0.0 && cfg->cfl <= 1.0)) return reject(DG_ERR_ARG, "cfl outside (0, 1]");
    if (cfg->precision < DG_FP64 || cfg->precision > DG_BF16X3) return reject(DG_ERR_ARG, "unknown precision");
    if (cfg->flags &
        ~(uint32_t)(DG_FORCING | DG_CLOSURE | DG_CHECK_RANGE | DG_LIMIT | DG_ISOTHERMAL | DG_EXACT_RIEMANN |
                    DG_ZHALO))
        return reject(DG_ERR_ARG, "unknown flags");
    if (cfg->k > 4) return reject(DG_ERR_UNSUPPORTED, "k > 4");
    // k = 4 runs the matrix-core kernel of stage_k4.hip: FP64 and FP32 storage
    if (cfg->k == 4 && cfg->precision != DG_FP64 && cfg->precision != DG_FP32)
        return reject(DG_ERR_UNSUPPORTED, "k = 4 takes FP64 or FP32 storage only");
    if ((cfg->flags & DG_CLOSURE) && cfg->k != 1) return reject(DG_ERR_UNSUPPORTED, "DG_CLOSURE needs k = 1");
    if ((cfg->flags & DG_CLOSURE) && (cfg->flags & DG_ZHALO))
        return reject(DG_ERR_UNSUPPORTED, "DG_CLOSURE with DG_ZHALO");
    {
        // the stage kernel addresses one (z, y) slab of 5 N(k) rows of n[0] cells with 32-bit offsets
        const double slab_bytes = 5.0 * nmodes_of(cfg->k) * cfg->n[0] * (cfg->precision == DG_FP64 ? 8.0 : 4.0);
        if (slab_bytes >= 2147483648.0) return reject(DG_ERR_UNSUPPORTED, "a (z, y) row of the state is 2 GiB or more");
    }
    const long long ncells = (long long)cfg->n[0] * cfg->n[1] * cfg->n[2];
    if ((long long)cfg->n[0] > (1LL << 30) || ncells > (1LL << 40)) return reject(DG_ERR_ARG, "mesh too large");

    dg_ctx *c = new (std::nothrow) dg_ctx();
    if (!c) return reject(DG_ERR_HIP, "out of host memory");
    c->cfg = *cfg;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->N = nmodes_of(cfg->k);
    c->n = cfg->k + 1;
    c->Q = c->n * c->n * c->n;
    c->P = c->n * c->n;
    c->ncells = ncells;
    double s[3];
    for (int a = 0; a < 3; a++) {
        c->h[a] = cfg->box[a] / cfg->n[a];
        s[a] = 1.0 / (4.0 * c->h[a]);  // (dx^2/4) / |K| of eqs. dg:eqn:volume_int and dg:eqn:surface_int
    }
    auto fail = [&](dg_status st) {
        if (st == DG_ERR_HIP) {
            const hipError_t e = hipGetLastError();
            g_init_err = std::string("dg_init: HIP call failed: ") + hipGetErrorName(e) + ", " + hipGetErrorString(e);
        } else {
            g_init_err = "dg_init: the stage kernel's LDS exceeds the device's";
        }
        dg_destroy(c);
        return st;
    };
    // k = 3 in the FP32-storage tiers: the kernel of stage_k3.hip; k = 4: stage_k4.hip
    c->k3x = cfg->k == 3 && cfg->precision != DG_FP64;
    c->k4m = cfg->k == 4;
    if (cfg->k >= 1) {  // k = 0 runs the finite-volume kernel, which needs no product tables
        std::vector<char> blob;
        if (c->k4m) {
            blob = build_tables_k4(cfg->precision, s);
        } else if (c->k3x) {
            c->lay = make_layout(cfg->k, cfg->precision);
            blob = build_tables_k3(cfg->precision, s);
        } else {
            c->lay = make_layout(cfg->k, cfg->precision);
            blob = build_tables(c->lay, s);
        }
        if (hipMalloc(&c->tables, blob.size()) != hipSuccess) return fail(DG_ERR_HIP);
        if (hipMemcpy(c->tables, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess)
            return fail(DG_ERR_HIP);
    }
    // projection table: phi_l(xi_q) w_q / 8
    {
        const Basis B(cfg->k);
        std::vector<double> pt((size_t)c->Q * c->N);
        double xi[3];
        for (int q = 0; q < c->Q; q++) {
            B.point(q, xi);
            for (int l = 0; l < c->N; l++) pt[(size_t)q * c->N + l] = B.phi(l, xi) * B.weight(q) / 8.0;
        }
        if (hipMalloc(&c->ptab, pt.size() * 8) != hipSuccess) return fail(DG_ERR_HIP);
        if (hipMemcpy(c->ptab, pt.data(), pt.size() * 8, hipMemcpyHostToDevice) != hipSuccess) return fail(DG_ERR_HIP);
        for (int u = 0; u <= cfg->k; u++)
            for (int a = 0; a < c->n; a++) c->leg1d.p[u][a] = leg(u, B.xg[a]);
        for (int a = 0; a < c->n; a++) c->leg1d.w[a] = B.wg[a];
    }
    if (cfg->flags & DG_LIMIT) {
        // phi_l at the limiter points: GLL nodes along one axis, Gauss nodes along the others
        const Basis B(cfg->k);
        const int m = limiter_gll_points(cfg->k);
        const double a5 = 1.0 / std::sqrt(5.0);
        const double xl2[2] = {-1.0, 1.0}, xl3[3] = {-1.0, 0.0, 1.0}, xl4[4] = {-1.0, -a5, a5, 1.0};
        const double *xl = m == 2 ? xl2 : (m == 3 ? xl3 : xl4);
        std::vector<double> lt;
        for (int a = 0; a < 3; a++)
            for (int r = 0; r < m; r++)
                for (int s2 = 0; s2 < c->n; s2++)
                    for (int t = 0; t < c->n; t++) {
                        double xi[3];
                        const int o1 = a == 0 ? 1 : 0, o2 = a == 2 ? 1 : 2;
                        xi[a] = xl[r];
                        xi[o1] = B.xg[s2];
                        xi[o2] = B.xg[t];
                        for (int l = 0; l < c->N; l++) lt.push_back(B.phi(l, xi));
                    }
        c->limnp = 3 * m * c->n * c->n;
        // then max over the points of |phi_l| (mode 0 unused): bounds the deviation from the mean
        for (int l = 0; l < c->N; l++) {
            double mx = 0.0;
            for (int p = 0; l > 0 && p < c->limnp; p++) mx = std::max(mx, std::fabs(lt[(size_t)p * c->N + l]));
            lt.push_back(mx);
        }
        if (hipMalloc(&c->limtab, lt.size() * sizeof(double)) != hipSuccess ||
            hipMemcpy(c->limtab, lt.data(), lt.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMalloc(&c->limcount, sizeof(unsigned long long)) != hipSuccess ||
            hipMemset(c->limcount, 0, sizeof(unsigned long long)) != hipSuccess)
            return fail(DG_ERR_HIP);
    }
    c->nparts = 1024;
    if (hipMalloc(&c->slots, 8 * sizeof(double)) != hipSuccess) return fail(DG_ERR_HIP);
    if (hipMemset(c->slots, 0, 8 * sizeof(double)) != hipSuccess) return fail(DG_ERR_HIP);
    if (hipMalloc(&c->flag, sizeof(int)) != hipSuccess) return fail(DG_ERR_HIP);
    if (hipMalloc(&c->partials, (size_t)(NF * c->nparts + 8) * sizeof(double)) != hipSuccess) return fail(DG_ERR_HIP);
    if (c->k4m) {  // one workgroup per compute unit (the tables fill its LDS)
        int dev = 0, ncu = 0, per_cu = 0;
        if (set_stage_k4_attributes(cfg->precision) != hipSuccess || hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return fail(DG_ERR_HIP);
        per_cu = 1;
        c->grid = ncu * per_cu;
        *out = c;
        return DG_OK;
    }
    if (cfg->k == 0) {  // launch shape set by its launcher
        c->grid = (int)std::min<long long>((ncells + 255) / 256, 1LL << 30);
        *out = c;
        return DG_OK;
    }
    {
        int dev0 = 0, maxlds = 0;
        if (hipGetDevice(&dev0) != hipSuccess ||
            hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev0) != hipSuccess)
            return fail(DG_ERR_HIP);
        // separate y-face trace and flux regions when both fit, else one shared region
        const int exb = (int)stage_exchange_bytes(cfg->precision);
        c->ex_off = c->k3x ? K3_SET * (cfg->precision == DG_BF16 ? 1 : 2) : (int)c->lay.bytes();
        c->ex_off2 = c->ex_off + exb;
        c->lds = c->ex_off + 2 * exb;
        if (c->lds > maxlds) {
            c->ex_off2 = c->ex_off;
            c->lds = c->ex_off + exb;
        }
        if (c->lds > maxlds) return fail(DG_ERR_UNSUPPORTED);
        if (c->k3x && c->ex_off2 == c->ex_off) return fail(DG_ERR_UNSUPPORTED);  // it needs both regions
        const int erb = (int)stage_endrow_bytes(cfg->precision, cfg->k);
        if (erb > 0 && c->lds + erb <= maxlds) {
            c->ex_off3 = c->lds;
            c->lds += erb;
        }
        if (c->k3x) {  // it also needs the end rows and the ghost-cell copies
            if (c->ex_off3 < 0 || c->lds + K3_GHOST_BYTES > maxlds) return fail(DG_ERR_UNSUPPORTED);
            c->ex_off4 = c->lds;
            c->lds += K3_GHOST_BYTES;
        }
    }
    if ((c->k3x ? set_stage_k3_attributes(cfg->precision, c->lds)
                : set_stage_attributes(cfg->k, cfg->precision, c->lds)) != hipSuccess)
        return fail(DG_ERR_HIP);
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(DG_ERR_HIP);
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return fail(DG_ERR_HIP);
    if ((c->k3x ? stage_k3_occupancy(cfg->precision, c->lds, &per_cu)
                : stage_occupancy(cfg->k, cfg->precision, c->lds, &per_cu)) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    // z chunk length: the resident item slots take the items in rounds, and an item costs its
    // planes plus about one plane of start-up (the -z face of its first plane, the look-ahead
    // that is not yet overlapped); pick the length (at most 32) that minimises
    // rounds x (length + 1), the longer one on ties
    const long long nbx = c->k3x ? (cfg->n[0] + K3_BLK - 1) / K3_BLK : (cfg->n[0] + BLK_INNER - 1) / BLK_INNER;
    const int rows = stage_rows_per_item(cfg->precision);
    const int items_per_wg = rows == 1 ? stage_block_threads(cfg->precision) / 64 : 1;  // one item per wave or per workgroup
    const long long nyg = (cfg->n[1] + rows - 1) / rows;
    const long long resident = std::max(1LL, (long long)per_cu * ncu * items_per_wg);
    long long zl = 1, best = -1;
    for (long long l = 1; l <= std::min(32LL, (long long)cfg->n[2]); l++) {
        const long long nch = (cfg->n[2] + l - 1) / l;
        const long long len = (cfg->n[2] + nch - 1) / nch;  // equal chunks
        if (len != l) continue;
        const long long rounds = (nbx * nyg * nch + resident - 1) / resident;
        const long long cost = rounds * (len + 1);
        if (best < 0 || cost <= best) {
            best = cost;
            zl = len;
        }
    }
    c->zlen = (int)zl;
    c->zlen_auto = c->zlen;
    const long long nitems = nbx * nyg * ((cfg->n[2] + zl - 1) / zl);
    long long grid = (long long)per_cu * ncu;
    grid = std::min(grid, (nitems + items_per_wg - 1) / items_per_wg);
    if (grid >= 8) grid -= grid % 8;
    c->grid = (int)std::max(1LL, grid);
    *out = c;
    return DG_OK;
}

dg_status dg_destroy(dg_ctx *c) {
    if (!c) return DG_OK;
    void *bufs[] = {c->tables, c->ptab,      c->slots,        c->flag,     c->partials,     c->fmodes,
                    c->acache, c->limtab,    c->iso_partials, c->limcount, c->clo,
                    c->corr,   c->clo_partials, c->clo_fallbacks, c->restrict_tab[0], c->restrict_tab[1],
                    c->restrict_tab[2], c->restrict_tab[3]};
    for (void *b : bufs)
        if (b) (void)hipFree(b);  // release what was allocated; a failure here has no remedy
    if (c->dtab) (void)hipFree(c->dtab);
    if (c->dcs) (void)hipFree(c->dcs);
    if (c->diag_bins) (void)hipFree(c->diag_bins);
    if (c->diag_partials) (void)hipFree(c->diag_partials);
    if (c->fft) (void)hipfftDestroy(static_cast<hipfftHandle>(c->fft));
    delete c;
    return DG_OK;
}

size_t dg_state_count(const dg_ctx *c) { return c ? (size_t)NF * c->N * (size_t)c->ncells : 0; }

size_t dg_workspace_bytes(const dg_ctx *c) { return c ? 2 * dg_state_count(c) * elem_bytes(c) : 0; }

static dg_status relayout(dg_ctx *c, const void *src, void *dst, int to_canonical, const char *name) {
    if (!c) return DG_ERR_ARG;
    if (!src || !dst || src == dst) {
        c->err = std::string(name) + ": NULL or identical pointers (the conversion is not in place)";
        return DG_ERR_ARG;
    }
    HIPCHK(c, launch_relayout(c->cfg.precision, src, dst, NF * nmodes_of(c->cfg.k), c->cfg.n[0], c->cfg.n[1],
                              c->cfg.n[2], to_canonical, c->stream));
    return DG_OK;
}

dg_status dg_state_import(dg_ctx *c, const void *canon, void *y) {
    return relayout(c, canon, y, 0, "dg_state_import");
}

dg_status dg_state_export(dg_ctx *c, const void *y, void *canon) {
    return relayout(c, y, canon, 1, "dg_state_export");
}

dg_status dg_project(dg_ctx *c, const void *qp, void *y) {
    if (!c) return DG_ERR_ARG;
    if (!qp || !y) {
        c->err = "dg_project: NULL pointer";
        return DG_ERR_ARG;
    }
    HIPCHK(c, launch_project(c->cfg.k, c->cfg.precision, qp, y, c->ptab, c->ncells, c->cfg.n[0], c->stream));
    return DG_OK;
}

}  // extern "C"

namespace {

dg_status run_stage(dg_ctx *c, const void *y0, const void *yin, void *out, double a, double b, double dt, int mode,
                    bool advance_time, bool limit_input = true) {
    if ((c->cfg.flags & DG_FORCING) && !c->have_forcing) {
        c->err = "DG_FORCING set but dg_set_forcing was not called";
        return DG_ERR_STATE;
    }
    if ((c->cfg.flags & DG_CLOSURE) && !c->have_closure) {
        c->err = "DG_CLOSURE set but dg_set_closure was not called";
        return DG_ERR_STATE;
    }
    if ((c->cfg.flags & DG_ZHALO) && !c->halo_lo) {
        c->err = "DG_ZHALO set but dg_set_halo was not called";
        return DG_ERR_STATE;
    }
    StageArgs s{};
    if ((c->cfg.flags & DG_LIMIT) && limit_input)  // Sec. 2.5: the stage input is limited in place
        HIPCHK(c, launch_limit(c->cfg.k, c->cfg.precision, const_cast<void *>(yin), c->limtab, c->limnp, c->ncells,
                               c->cfg.n[0], c->cfg.gamma, LIMIT_EPS, c->limcount, c->stream));
    if (c->cfg.flags & DG_CLOSURE) {
        // the correction of the stage input, then the stage that applies it
        ClosureArgs ca{};
        ca.y = yin;
        ca.corr = c->corr;
        ca.params = c->clo;
        ca.fmean = c->clo + CL_NPARAMS;
        ca.fistd = ca.fmean + CL_NIN;
        ca.oscale = ca.fistd + CL_NIN;
        ca.obound = ca.oscale + CL_NOUT;
        ca.partials = c->clo_partials + NF;
        ca.fallbacks = c->clo_fallbacks;
        ca.done = c->clo_fallbacks + 1;
        ca.cmean = c->clo_partials;
        ca.nx = c->cfg.n[0];
        ca.ny = c->cfg.n[1];
        ca.nz = c->cfg.n[2];
        ca.ncells = c->ncells;
        HIPCHK(c, launch_closure(c->cfg.precision, ca, c->stream));
        s.corr = c->corr;
        s.cmean = c->clo_partials;
    }
    s.yin = yin;
    s.y0 = y0 ? y0 : yin;
    s.out = out;
    s.tables = c->tables;
    s.rate = (mode == 1 && dt <= 0.0) ? c->slots + c->cur_slot : nullptr;
    s.tacc = advance_time ? c->slots + 2 : nullptr;
    s.dt = dt;
    s.a = a;
    s.b = b;
    s.dtfac = dt_factor(c);
    s.gamma = c->cfg.gamma;
    s.nx = c->cfg.n[0];
    s.ny = c->cfg.n[1];
    s.nz = c->cfg.n[2];
    s.nbx = c->k3x ? (c->cfg.n[0] + K3_BLK - 1) / K3_BLK : (c->cfg.n[0] + BLK_INNER - 1) / BLK_INNER;
    s.zlen = c->zlen;
    {
        const int rows = stage_rows_per_item(c->cfg.precision);
        s.nitems = (long long)s.nbx * ((s.ny + rows - 1) / rows) * ((s.nz + c->zlen - 1) / c->zlen);
    }
    s.ex_off = c->ex_off;
    s.ex_off2 = c->ex_off2;
    s.ex_single = c->ex_off2 == c->ex_off ? 1 : 0;
    s.ex_off3 = c->ex_off3;
    s.ex_off4 = c->ex_off4;
    s.ncells = c->ncells;
    s.mode = mode;
    s.forcing = (c->cfg.flags & DG_FORCING) ? 1 : 0;
    s.riemann = (c->cfg.flags & DG_EXACT_RIEMANN) ? 1 : 0;
    s.halo_lo = c->halo_lo;
    s.halo_hi = c->halo_hi;
    s.acache = c->acache;
    for (int i = 0; i < 3; i++) s.h[i] = c->h[i];
    s.dtab = c->dtab;
    s.dcs = c->dcs;
    s.dks = c->dks;
    if (c->k3x)
        HIPCHK(c, launch_stage_k3(c->cfg.precision, s, c->grid, c->lds, c->stream));
    else if (c->k4m)
        HIPCHK(c, launch_stage_k4(c->cfg.precision, s, c->grid, c->stream));
    else
        HIPCHK(c, launch_stage(c->cfg.k, c->cfg.precision, s, c->grid, c->lds, c->stream));
    return DG_OK;
}

// CFL rate into the free slot; it becomes the current one.
dg_status run_cfl(dg_ctx *c, const void *y) {
    const int nxt = 1 - c->cur_slot;
    HIPCHK(c, launch_cfl(c->cfg.precision, y, c->N, c->cfg.n[0], c->ncells, c->cfg.gamma, c->h, c->slots + nxt,
                         c->slots + c->cur_slot, c->stream));
    c->cur_slot = nxt;
    return DG_OK;
}

}  // namespace

extern "C" {

dg_status dg_rhs(dg_ctx *c, const void *y, void *r) {
    if (!c) return DG_ERR_ARG;
    if (!y || !r || y == r) {
        c->err = "dg_rhs: NULL or aliased pointers";
        return DG_ERR_ARG;
    }
    return run_stage(c, nullptr, y, r, 0.0, 1.0, 0.0, 0, false);
}

dg_status dg_stage(dg_ctx *c, const void *y0, const void *yin, void *out, double a, double b, double dt) {
    if (!c) return DG_ERR_ARG;
    if (!yin || !out || out == yin || (a != 0.0 && !y0)) {
        c->err = "dg_stage: NULL or aliased pointers";
        return DG_ERR_ARG;
    }
    return run_stage(c, y0, yin, out, a, b, dt, 1, false);
}

dg_status dg_dt(dg_ctx *c, const void *y, double *dt) {
    if (!c) return DG_ERR_ARG;
    if (!y || !dt) {
        c->err = "dg_dt: NULL pointer";
        return DG_ERR_ARG;
    }
    dg_status st = run_cfl(c, y);
    if (st != DG_OK) return st;
    double rate = 0.0;
    HIPCHK(c, hipMemcpyAsync(&rate, c->slots + c->cur_slot, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *dt = dt_factor(c) / rate;
    return DG_OK;
}

static hipError_t run_reset(dg_ctx *c, void *y) {
    const double gm1 = c->cfg.gamma - 1.0;
    return launch_reset(c->cfg.k, c->cfg.precision, y, c->leg1d, c->ncells, c->cfg.n[0], gm1,
                        c->iso_cs * c->iso_cs / gm1, c->iso_rho0, c->h[0] * c->h[1] * c->h[2], c->iso_partials,
                        c->slots + 4, c->stream);
}

dg_status dg_set_isothermal(dg_ctx *c, double cs, double rho0) {
    if (!c) return DG_ERR_ARG;
    if (!(cs > 0.0) || !(rho0 > 0.0) || !std::isfinite(cs) || !std::isfinite(rho0)) {
        c->err = "dg_set_isothermal: cs and rho0 must be finite and > 0";
        return DG_ERR_ARG;
    }
    if (!c->iso_partials && hipMalloc(&c->iso_partials, reset_partials(c->ncells) * sizeof(double)) != hipSuccess) {
        c->iso_partials = nullptr;
        c->err = "dg_set_isothermal: hipMalloc failed";
        return DG_ERR_HIP;
    }
    c->iso_cs = cs;
    c->iso_rho0 = rho0;
    c->have_iso = true;
    return DG_OK;
}

dg_status dg_isothermal_reset(dg_ctx *c, void *y) {
    if (!c) return DG_ERR_ARG;
    if (!y) {
        c->err = "dg_isothermal_reset: NULL pointer";
        return DG_ERR_ARG;
    }
    if (!c->have_iso) {
        c->err = "dg_isothermal_reset: dg_set_isothermal has not been called";
        return DG_ERR_STATE;
    }
    HIPCHK(c, run_reset(c, y));
    return DG_OK;
}

dg_status dg_dissipated(dg_ctx *c, double *out) {
    if (!c) return DG_ERR_ARG;
    if (!out) {
        c->err = "dg_dissipated: NULL pointer";
        return DG_ERR_ARG;
    }
    HIPCHK(c, hipMemcpyAsync(out, c->slots + 4, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, launch_zero_u64(reinterpret_cast<unsigned long long *>(c->slots + 4), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DG_OK;
}

dg_status dg_step(dg_ctx *c, void *y, void *work, double dt, int32_t nsteps, double *t_inout) {
    if (!c) return DG_ERR_ARG;
    if (!y || !work || nsteps < 0) {
        c->err = "dg_step: NULL pointer or negative step count";
        return DG_ERR_ARG;
    }
    if ((c->cfg.flags & DG_ISOTHERMAL) && !c->have_iso) {
        c->err = "dg_step: DG_ISOTHERMAL needs dg_set_isothermal first";
        return DG_ERR_STATE;
    }
    if (c->cfg.flags & DG_ZHALO) {  // the halo planes must be refreshed between the stages
        c->err = "dg_step: a z slab (DG_ZHALO) is stepped stage by stage with dg_stage";
        return DG_ERR_UNSUPPORTED;
    }
    const size_t sb = dg_state_count(c) * elem_bytes(c);
    void *w1 = work;
    void *w2 = static_cast<char *>(work) + sb;
    const bool dev_dt = !(dt > 0.0);
    if (dev_dt && t_inout) {
        double t0 = 0.0;
        HIPCHK(c, hipMemcpyAsync(c->slots + 2, &t0, sizeof(double), hipMemcpyHostToDevice, c->stream));
    }
    const bool check = (c->cfg.flags & DG_CHECK_RANGE) != 0;
    for (int it = 0; it < nsteps; it++) {
        dg_status st;
        const bool lim = (c->cfg.flags & DG_LIMIT) != 0;
        if (lim)  // y^n is limited before its time step is taken (it is the first stage's input)
            HIPCHK(c, launch_limit(c->cfg.k, c->cfg.precision, y, c->limtab, c->limnp, c->ncells, c->cfg.n[0],
                                   c->cfg.gamma, LIMIT_EPS, c->limcount, c->stream));
        if (dev_dt && (st = run_cfl(c, y)) != DG_OK) return st;
        if ((st = run_stage(c, y, y, w1, 0.0, 1.0, dt, 1, false, false)) != DG_OK) return st;
        if ((st = run_stage(c, y, w1, w2, 0.75, 0.25, dt, 1, false)) != DG_OK) return st;
        if ((st = run_stage(c, y, w2, y, 1.0 / 3.0, 2.0 / 3.0, dt, 1, dev_dt && t_inout)) != DG_OK) return st;
        if (c->cfg.flags & DG_ISOTHERMAL) {  // Sec. 3.2: reset after the step, then the limiter
            HIPCHK(c, run_reset(c, y));
            if (lim)
                HIPCHK(c, launch_limit(c->cfg.k, c->cfg.precision, y, c->limtab, c->limnp, c->ncells, c->cfg.n[0],
                                       c->cfg.gamma, LIMIT_EPS, c->limcount, c->stream));
        }
        if (check) {
            int flag = 0;
            HIPCHK(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
            HIPCHK(c, launch_range_check(c->cfg.precision, y, c->N, c->cfg.n[0], c->ncells, c->cfg.gamma, c->flag, c->stream));
            HIPCHK(c, hipMemcpyAsync(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            if (flag) {
                if (t_inout && !dev_dt) *t_inout += dt * (it + 1);
                c->err = "non-physical cell mean (rho <= 0, p <= 0 or non-finite) after step " + std::to_string(it + 1);
                return DG_ERR_RANGE;
            }
        }
    }
    if (t_inout) {
        if (dev_dt) {
            double tt = 0.0;
            HIPCHK(c, hipMemcpyAsync(&tt, c->slots + 2, sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            *t_inout += tt;
        } else {
            *t_inout += dt * nsteps;
        }
    }
    return DG_OK;
}

dg_status dg_totals(dg_ctx *c, const void *y, double out[5]) {
    if (!c) return DG_ERR_ARG;
    if (!y || !out) {
        c->err = "dg_totals: NULL pointer";
        return DG_ERR_ARG;
    }
    const double vol = c->h[0] * c->h[1] * c->h[2];
    double *dres = c->partials + (size_t)NF * c->nparts;
    HIPCHK(c, launch_totals(c->cfg.precision, y, c->N, c->cfg.n[0], c->ncells, vol, c->partials, c->nparts, dres, c->stream));
    HIPCHK(c, hipMemcpyAsync(out, dres, NF * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DG_OK;
}

dg_status dg_set_forcing(dg_ctx *c, int32_t nmodes, const int32_t *nvec, const double *ahat) {
    if (!c) return DG_ERR_ARG;
    if (nmodes < 0 || nmodes > MAX_FORCING_MODES || (nmodes > 0 && (!nvec || !ahat))) {
        c->err = "dg_set_forcing: bad mode count or NULL table";
        return DG_ERR_ARG;
    }
    if (!(c->cfg.flags & DG_FORCING)) {
        c->err = "dg_set_forcing: context was created without DG_FORCING";
        return DG_ERR_STATE;
    }
    // device mode table per mode: n_x, n_y, n_z (as doubles), then Re/Im of the three components;
    // sorted by n_x so that the cache kernel forms one x phase per distinct n_x
    std::vector<int> order(nmodes);
    for (int m = 0; m < nmodes; m++) order[m] = m;
    std::stable_sort(order.begin(), order.end(), [&](int p, int q) { return nvec[3 * p] < nvec[3 * q]; });
    std::vector<double> t((size_t)MAX_FORCING_MODES * 9, 0.0);
    for (int j = 0; j < nmodes; j++) {
        const int m = order[j];
        for (int a = 0; a < 3; a++) t[9 * j + a] = (double)nvec[3 * m + a];
        for (int i = 0; i < 6; i++) t[9 * j + 3 + i] = ahat[6 * m + i];
    }
    if (c->k3x) {
        // the k = 3 kernel forms the acceleration as a product: wave vectors with n_x >= 0
        // (n -> -n with the conjugate amplitude gives the same real field), their y, z and in-cell
        // x phases per (z, y) row in a table, the x phase of the cell per x
        int nxmax = 0;
        for (int j = 0; j < nmodes; j++) {
            if (t[9 * j] < 0.0) {
                for (int a = 0; a < 3; a++) t[9 * j + a] = -t[9 * j + a];
                for (int cc = 0; cc < 3; cc++) t[9 * j + 4 + 2 * cc] = -t[9 * j + 4 + 2 * cc];
            }
            nxmax = std::max(nxmax, (int)t[9 * j]);
        }
        if (2 * (nxmax + 1) > 4 * K3_DKS) {
            c->err = "dg_set_forcing: the k = 3 BF16 tiers take driving wave numbers |n_x| <= 3";
            return DG_ERR_UNSUPPORTED;
        }
        const int dks = K3_DKS;
        if (c->dtab && dks != c->dks) {
            (void)hipFree(c->dtab);
            (void)hipFree(c->dcs);
            c->dtab = nullptr;
            c->dcs = nullptr;
        }
        const int nx = c->cfg.n[0];
        if (!c->dtab) {
            HIPCHK(c, hipMalloc(&c->dtab, (size_t)k3_drive_row_floats(dks) * c->cfg.n[1] * c->cfg.n[2] * sizeof(float)));
            HIPCHK(c, hipMalloc(&c->dcs, (size_t)nx * dks * 4 * sizeof(float)));
        }
        c->dks = dks;
        std::vector<float> cs((size_t)nx * dks * 4);
        for (int x = 0; x < nx; x++)
            for (int k = 0; k < 4 * dks; k++) {
                const int w = k / 2;
                double ph = (double)w * x / nx;
                ph -= std::floor(ph);
                cs[(size_t)x * dks * 4 + k] = (float)((k & 1) ? std::sin(2.0 * M_PI * ph) : std::cos(2.0 * M_PI * ph));
            }
        if (!c->fmodes) HIPCHK(c, hipMalloc(&c->fmodes, t.size() * sizeof(double)));
        HIPCHK(c, hipMemcpyAsync(c->fmodes, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->dcs, cs.data(), cs.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
        GaussNodes xg{};
        double wg[5];
        gauss_rule(c->n, xg.x, wg);
        HIPCHK(c, launch_drive_table_k3(c->fmodes, nmodes, dks, c->cfg.n[1], c->cfg.n[2], xg, nx, c->slab_z0,
                                        c->slab_nz > 0 ? c->slab_nz : c->cfg.n[2], c->dtab, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->nfmodes = nmodes;
        c->have_forcing = true;
        return DG_OK;
    }
    if (!c->fmodes) HIPCHK(c, hipMalloc(&c->fmodes, t.size() * sizeof(double)));
    if (!c->acache)
        HIPCHK(c, hipMalloc(&c->acache, (size_t)accel_slab_elems(c->cfg.k, c->cfg.n[0]) * c->cfg.n[1] * c->cfg.n[2] *
                                            elem_bytes(c)));
    HIPCHK(c, hipMemcpyAsync(c->fmodes, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    GaussNodes xg{};
    double wg[5];
    gauss_rule(c->n, xg.x, wg);
    HIPCHK(c, launch_accel_cache(c->cfg.k, c->cfg.precision, c->fmodes, nmodes, c->cfg.n[0], c->cfg.n[1], c->cfg.n[2],
                                 c->ncells, xg, c->slab_z0, c->slab_nz > 0 ? c->slab_nz : c->cfg.n[2], c->acache,
                                 c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->nfmodes = nmodes;
    c->have_forcing = true;
    return DG_OK;
}

dg_status dg_ou_update(int32_t nmodes, const int32_t *nvec, double *theta, const double *z, double f, double sigma,
                       double a0, double kmin, double kmax, double *ahat) {
    if (nmodes < 0 || (nmodes > 0 && (!nvec || !theta || !z || !ahat))) return DG_ERR_ARG;
    if (!(f >= 0.0 && f <= 1.0) || !(kmax > kmin)) return DG_ERR_ARG;
    const double mid = 0.5 * (kmin + kmax), half = 0.5 * (kmax - kmin);
    const double kick = sigma * std::sqrt(1.0 - f * f);
    for (int m = 0; m < nmodes; m++) {
        double *th = theta + 6 * m;
        for (int j = 0; j < 6; j++) th[j] = f * th[j] + kick * z[6 * m + j];
        const double n0 = nvec[3 * m], n1 = nvec[3 * m + 1], n2 = nvec[3 * m + 2];
        const double nn = n0 * n0 + n1 * n1 + n2 * n2;
        double prof = 0.0;
        if (nn > 0.0) {
            const double d = (std::sqrt(nn) - mid) / half;
            prof = std::max(0.0, 1.0 - d * d);
        }
        for (int part = 0; part < 2; part++) {
            const double vx = th[part], vy = th[2 + part], vz = th[4 + part];
            const double dot = nn > 0.0 ? (n0 * vx + n1 * vy + n2 * vz) / nn : 0.0;
            ahat[6 * m + 0 + part] = a0 * prof * (vx - n0 * dot);
            ahat[6 * m + 2 + part] = a0 * prof * (vy - n1 * dot);
            ahat[6 * m + 4 + part] = a0 * prof * (vz - n2 * dot);
        }
    }
    return DG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- learned closure and its training

extern "C" {

dg_status dg_set_closure(dg_ctx *c, const float *params, const float *feat_mean, const float *feat_std,
                         const float *out_scale, const float *out_bound) {
    if (!c) return DG_ERR_ARG;
    if (!(c->cfg.flags & DG_CLOSURE)) {
        c->err = "dg_set_closure: the context was created without DG_CLOSURE";
        return DG_ERR_STATE;
    }
    if (!params || !feat_mean || !feat_std || !out_scale || !out_bound) {
        c->err = "dg_set_closure: NULL pointer";
        return DG_ERR_ARG;
    }
    std::vector<float> blob((size_t)CL_NPARAMS + 2 * CL_NIN + 2 * CL_NOUT);
    std::memcpy(blob.data(), params, sizeof(float) * CL_NPARAMS);
    float *fm = blob.data() + CL_NPARAMS, *fi = fm + CL_NIN, *os = fi + CL_NIN, *ob = os + CL_NOUT;
    for (int f = 0; f < CL_NIN; f++) {
        if (!(feat_std[f] > 0.0f) || !std::isfinite(feat_std[f]) || !std::isfinite(feat_mean[f])) {
            c->err = "dg_set_closure: feat_std must be positive and finite, feat_mean finite";
            return DG_ERR_ARG;
        }
        fm[f] = feat_mean[f];
        fi[f] = 1.0f / feat_std[f];
    }
    for (int j = 0; j < CL_NOUT; j++) {
        if (!std::isfinite(out_scale[j]) || !(out_bound[j] >= 0.0f)) {
            c->err = "dg_set_closure: out_scale must be finite and out_bound >= 0";
            return DG_ERR_ARG;
        }
        os[j] = out_scale[j];
        ob[j] = out_bound[j];
    }
    if (!c->clo) {
        const long long nwaves = (c->ncells + 15) / 16;
        if (hipMalloc(&c->clo, blob.size() * sizeof(float)) != hipSuccess ||
            hipMalloc(&c->corr, dg_state_count(c) * elem_bytes(c)) != hipSuccess ||
            hipMalloc(&c->clo_partials, (size_t)(nwaves + 9) * NF * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->clo_fallbacks, 2 * sizeof(unsigned long long)) != hipSuccess) {
            c->err = "dg_set_closure: device allocation failed";
            return DG_ERR_HIP;
        }
        HIPCHK(c, launch_zero_u64(c->clo_fallbacks, c->stream));
        HIPCHK(c, launch_zero_u64(c->clo_fallbacks + 1, c->stream));  // the inference's finished-workgroup count
    }
    // the copy is ordered after the work already enqueued on the stream
    HIPCHK(c, hipMemcpyAsync(c->clo, blob.data(), blob.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->have_closure = true;
    return DG_OK;
}

dg_status dg_closure_fallbacks(dg_ctx *c, int64_t *count) {
    if (!c) return DG_ERR_ARG;
    if (!count) {
        c->err = "dg_closure_fallbacks: NULL pointer";
        return DG_ERR_ARG;
    }
    if (!c->have_closure) {
        *count = 0;
        return DG_OK;
    }
    unsigned long long v = 0;
    HIPCHK(c, hipMemcpyAsync(&v, c->clo_fallbacks, sizeof v, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, launch_zero_u64(c->clo_fallbacks, c->stream));
    *count = (int64_t)v;
    return DG_OK;
}

dg_status dg_closure_features(dg_ctx *c, const void *y, float *feat) {
    if (!c) return DG_ERR_ARG;
    if (!y || !feat) {
        c->err = "dg_closure_features: NULL pointer";
        return DG_ERR_ARG;
    }
    HIPCHK(c, launch_features(c->cfg.precision, y, feat, c->N, c->cfg.n[0], c->cfg.n[1], c->cfg.n[2], c->ncells,
                              c->stream));
    return DG_OK;
}

dg_status dg_closure_targets(dg_ctx *c, const void *r_coarse, const void *r_fine_restricted, float *target) {
    if (!c) return DG_ERR_ARG;
    if (!r_coarse || !r_fine_restricted || !target) {
        c->err = "dg_closure_targets: NULL pointer";
        return DG_ERR_ARG;
    }
    HIPCHK(c, launch_targets(c->cfg.precision, r_coarse, r_fine_restricted, target, c->N, c->cfg.n[0], c->ncells,
                             c->stream));
    return DG_OK;
}

dg_status dg_restrict(dg_ctx *c, int32_t kf, const void *yf, void *yc) {
    if (!c) return DG_ERR_ARG;
    if (kf < c->cfg.k || kf > 3) {
        c->err = "dg_restrict: need k <= kf <= 3";
        return kf > 3 ? DG_ERR_UNSUPPORTED : DG_ERR_ARG;
    }
    if (!yf || !yc || yf == yc) {
        c->err = "dg_restrict: NULL or aliased pointers";
        return DG_ERR_ARG;
    }
    const int Nf = nmodes_of(kf), Nc = c->N;
    if (!c->restrict_tab[kf]) {
        // M[ch][l][m] = (1/64) sum_q phi^f_m(xi_q) phi^c_l(xi^c(xi_q)) w_q over a Gauss rule of the
        // child exact for degree kf + kc; child ch = (dz dy dx) bits, xi^c = -1/2 + d + xi/2
        const Basis Bf(kf), Bc(c->cfg.k);
        const int nq = (kf + c->cfg.k) / 2 + 1;
        double xg[5], wg[5];
        gauss_rule(nq, xg, wg);
        std::vector<double> M((size_t)8 * Nc * Nf, 0.0);
        for (int ch = 0; ch < 8; ch++) {
            const int d[3] = {ch & 1, (ch >> 1) & 1, ch >> 2};
            for (int qc = 0; qc < nq; qc++)
                for (int qb = 0; qb < nq; qb++)
                    for (int qa = 0; qa < nq; qa++) {
                        const double xf[3] = {xg[qa], xg[qb], xg[qc]};
                        double xcs[3];
                        for (int a = 0; a < 3; a++) xcs[a] = -0.5 + d[a] + 0.5 * xf[a];
                        const double w = wg[qa] * wg[qb] * wg[qc] / 64.0;
                        for (int l = 0; l < Nc; l++) {
                            const double pc = Bc.phi(l, xcs) * w;
                            for (int m = 0; m < Nf; m++) M[((size_t)ch * Nc + l) * Nf + m] += pc * Bf.phi(m, xf);
                        }
                    }
        }
        double *dM = nullptr;
        HIPCHK(c, hipMalloc(&dM, M.size() * sizeof(double)));
        c->restrict_tab[kf] = dM;
        HIPCHK(c, hipMemcpy(dM, M.data(), M.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    HIPCHK(c, launch_restrict(c->cfg.precision, yf, yc, c->restrict_tab[kf], Nf, Nc, c->cfg.n[0], c->cfg.n[1],
                              c->cfg.n[2], c->stream));
    return DG_OK;
}

// ---- MLP training (no context): the caller's stream and workspace

static bool mlp_shape_ok(const int32_t *sh) {
    return sh && sh[0] >= 1 && sh[1] >= 1 && sh[2] >= 1 && sh[3] >= 1 && sh[0] <= 4096 && sh[1] <= 4096 &&
           sh[2] <= 4096 && sh[3] <= 4096;
}

size_t dg_mlp_nparams(const int32_t shape[4]) {
    if (!mlp_shape_ok(shape)) return 0;
    const size_t a = shape[0], b = shape[1], cc = shape[2], d = shape[3];
    return b * a + b + cc * b + cc + d * cc + d;
}

size_t dg_mlp_workspace_bytes(const int32_t shape[4], int32_t batch) {
    if (!mlp_shape_ok(shape) || batch < 1) return 0;
    const size_t B = batch;
    // Xb, H1, H2, Y, Tb, dY, D2, D1 (feature-major) and a loss slot
    return sizeof(float) * B * ((size_t)shape[0] + 2 * shape[1] + 2 * shape[2] + 3 * shape[3]) + 64;
}

namespace {
struct MlpWork {
    float *Xb, *H1, *H2, *Y, *Tb, *dY, *D2, *D1;
};
MlpWork carve(const int32_t *sh, int B, void *work) {
    float *p = static_cast<float *>(work);
    MlpWork w;
    w.Xb = p; p += (size_t)sh[0] * B;
    w.H1 = p; p += (size_t)sh[1] * B;
    w.D1 = p; p += (size_t)sh[1] * B;
    w.H2 = p; p += (size_t)sh[2] * B;
    w.D2 = p; p += (size_t)sh[2] * B;
    w.Y = p; p += (size_t)sh[3] * B;
    w.Tb = p; p += (size_t)sh[3] * B;
    w.dY = p;
    return w;
}
// C[M][B] = act(W[M][K] X[K][B] + b), feature-major activations
hipError_t dense(const float *W, const float *b, const float *X, float *C, int M, int K, int B, int ep,
                 hipStream_t s) {
    GemmArgs g{};
    g.A = W; g.B = X; g.C = C; g.bias = b; g.E = nullptr;
    g.M = M; g.N = B; g.K = K;
    g.sam = K; g.sak = 1; g.sbk = B; g.sbn = 1; g.scm = B; g.scn = 1;
    g.ep = ep;
    return launch_gemm(g, s);
}
hipError_t mlp_fwd(const int32_t *sh, const float *P, int B, const MlpWork &w, hipStream_t s) {
    const int nin = sh[0], h1 = sh[1], h2 = sh[2], no = sh[3];
    const float *W1 = P, *b1 = W1 + (size_t)h1 * nin, *W2 = b1 + h1, *b2 = W2 + (size_t)h2 * h1;
    const float *W3 = b2 + h2, *b3 = W3 + (size_t)no * h2;
    hipError_t e;
    if ((e = dense(W1, b1, w.Xb, w.H1, h1, nin, B, EP_TANH, s)) != hipSuccess) return e;
    if ((e = dense(W2, b2, w.H1, w.H2, h2, h1, B, EP_TANH, s)) != hipSuccess) return e;
    return dense(W3, b3, w.H2, w.Y, no, h2, B, EP_NONE, s);
}
}  // namespace

dg_status dg_mlp_forward(const int32_t shape[4], const float *params, int32_t batch, const float *x, const int32_t *rows,
                         float *y, void *work, void *hip_stream) {
    if (!mlp_shape_ok(shape) || batch < 1 || !params || !x || !y || !work) return DG_ERR_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const MlpWork w = carve(shape, batch, work);
    if (launch_gather(x, shape[0], rows, batch, w.Xb, s) != hipSuccess) return DG_ERR_HIP;
    if (mlp_fwd(shape, params, batch, w, s) != hipSuccess) return DG_ERR_HIP;
    // y[s][j] = Y[j][s]: the gather kernel with the roles of rows and columns swapped transposes
    if (launch_gather(w.Y, batch, nullptr, shape[3], y, s) != hipSuccess) return DG_ERR_HIP;
    return DG_OK;
}

dg_status dg_mlp_loss_grad(const int32_t shape[4], const float *params, int32_t batch, const float *x,
                           const float *target, const int32_t *rows, float noise_std, uint64_t seed, float *grad,
                           double *loss, void *work, void *hip_stream) {
    if (!mlp_shape_ok(shape) || batch < 1 || !params || !x || !target || !grad || !work || !(noise_std >= 0.0f))
        return DG_ERR_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const int nin = shape[0], h1 = shape[1], h2 = shape[2], no = shape[3], B = batch;
    const MlpWork w = carve(shape, B, work);
    const float *W2 = params + (size_t)h1 * nin + h1, *W3 = W2 + (size_t)h2 * h1 + h2;
    float *gW1 = grad, *gb1 = gW1 + (size_t)h1 * nin, *gW2 = gb1 + h1, *gb2 = gW2 + (size_t)h2 * h1;
    float *gW3 = gb2 + h2, *gb3 = gW3 + (size_t)no * h2;
    auto ok = [](hipError_t e) { return e == hipSuccess; };
    if (!ok(launch_gather(x, nin, rows, B, w.Xb, s, noise_std, (unsigned long long)seed)) ||
        !ok(launch_gather(target, no, rows, B, w.Tb, s)) ||
        !ok(mlp_fwd(shape, params, B, w, s)) || !ok(launch_mse(w.Y, w.Tb, w.dY, (long long)no * B, loss, s)))
        return DG_ERR_HIP;
    // weight gradients: gW = D A^T (contraction over the batch); bias gradients: row sums of D
    auto wgrad = [&](const float *D, const float *Aact, float *gW, int M, int K) {
        GemmArgs g{};
        g.A = D; g.B = Aact; g.C = gW; g.M = M; g.N = K; g.K = B;
        g.sam = B; g.sak = 1; g.sbk = 1; g.sbn = B; g.scm = K; g.scn = 1;
        g.ep = EP_NONE;
        return launch_gemm(g, s);
    };
    // back-propagated signal: D_prev = (W^T D) * (1 - H_prev^2)
    auto bprop = [&](const float *W, const float *D, const float *Hp, float *Dp, int Mout, int Kin) {
        GemmArgs g{};
        g.A = W; g.B = D; g.C = Dp; g.E = Hp; g.M = Kin; g.N = B; g.K = Mout;
        g.sam = 1; g.sak = Kin; g.sbk = B; g.sbn = 1; g.scm = B; g.scn = 1;
        g.ep = EP_DTANH;
        return launch_gemm(g, s);
    };
    if (!ok(wgrad(w.dY, w.H2, gW3, no, h2)) || !ok(launch_rowsum(w.dY, no, B, gb3, s)) ||
        !ok(bprop(W3, w.dY, w.H2, w.D2, no, h2)) || !ok(wgrad(w.D2, w.H1, gW2, h2, h1)) ||
        !ok(launch_rowsum(w.D2, h2, B, gb2, s)) || !ok(bprop(W2, w.D2, w.H1, w.D1, h2, h1)) ||
        !ok(wgrad(w.D1, w.Xb, gW1, h1, nin)) || !ok(launch_rowsum(w.D1, h1, B, gb1, s)))
        return DG_ERR_HIP;
    return DG_OK;
}

dg_status dg_adam(int64_t nparams, float *params, const float *grad, float *m, float *v, int32_t step, double lr,
                  double beta1, double beta2, double eps, void *hip_stream) {
    if (nparams < 1 || !params || !grad || !m || !v || step < 1 || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) ||
        !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
        return DG_ERR_ARG;
    if (launch_adam(params, grad, m, v, nparams, step, lr, beta1, beta2, eps, reinterpret_cast<hipStream_t>(hip_stream)) !=
        hipSuccess)
        return DG_ERR_HIP;
    return DG_OK;
}

size_t dg_column_stats_workspace_bytes(int32_t cols) { return cols < 1 ? 0 : (size_t)1024 * cols * 3 * sizeof(double); }

dg_status dg_column_stats(const float *x, int64_t rows, int32_t cols, double *mean, double *stdev, double *rms,
                          double *maxabs, void *work, void *hip_stream) {
    if (!x || rows < 1 || cols < 1 || cols > 256 || !mean || !stdev || !rms || !maxabs || !work) return DG_ERR_ARG;
    const int nchunks = (int)std::min<int64_t>(1024, rows);
    if (launch_colstats(x, rows, cols, static_cast<double *>(work), nchunks, mean, stdev, rms, maxabs,
                        reinterpret_cast<hipStream_t>(hip_stream)) != hipSuccess)
        return DG_ERR_HIP;
    return DG_OK;
}

dg_status dg_standardize(float *x, int64_t rows, int32_t cols, const double *shift, const double *scale,
                         void *hip_stream) {
    if (!x || rows < 1 || cols < 1 || !shift || !scale) return DG_ERR_ARG;
    if (launch_standardize(x, rows, cols, shift, scale, reinterpret_cast<hipStream_t>(hip_stream)) != hipSuccess)
        return DG_ERR_HIP;
    return DG_OK;
}

}  // extern "C"

extern "C" dg_status dg_limiter_stats(dg_ctx *c, int64_t *count) {
    if (!c) return DG_ERR_ARG;
    if (!count) {
        c->err = "dg_limiter_stats: NULL pointer";
        return DG_ERR_ARG;
    }
    *count = 0;
    if (!c->limcount) return DG_OK;
    unsigned long long v = 0;
    HIPCHK(c, hipMemcpyAsync(&v, c->limcount, sizeof v, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, launch_zero_u64(c->limcount, c->stream));
    *count = (int64_t)v;
    return DG_OK;
}

// ------------------------------------------------------------------ diagnostics (Sec. 3.3, 4.1, 4.4)

static dg_status diag_begin(dg_ctx *c, const void *y, int S, const char *who, Leg1D *L) {
    if (!y) {
        c->err = std::string(who) + ": NULL pointer";
        return DG_ERR_ARG;
    }
    if (S < 1 || S > DIAG_MAX_S) {
        c->err = std::string(who) + ": S must be in 1.." + std::to_string(DIAG_MAX_S);
        return DG_ERR_ARG;
    }
    if (!c->diag_bins) {
        if (hipMalloc(&c->diag_bins, (2 * DIAG_MAX_BINS + 2) * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->diag_partials, (sample_blocks(c->ncells) + 1) * sizeof(double)) != hipSuccess) {
            c->err = std::string(who) + ": hipMalloc failed";
            return DG_ERR_HIP;
        }
    }
    // scaled Legendre polynomials at the centres of the S equal parts of [-1, 1]
    *L = Leg1D{};
    for (int u = 0; u <= c->cfg.k; u++)
        for (int a = 0; a < S; a++) L->p[u][a] = leg(u, -1.0 + (2.0 * a + 1.0) / S);
    return DG_OK;
}

static SampleArgs sample_args(const dg_ctx *c, const void *y, int what) {
    SampleArgs a{};
    a.y = y;
    a.nc = c->ncells;
    a.nx = c->cfg.n[0];
    a.ny = c->cfg.n[1];
    a.what = what;
    a.gamma = c->cfg.gamma;
    return a;
}

dg_status dg_sample(dg_ctx *c, const void *y, int32_t S, void *out) {
    if (!c) return DG_ERR_ARG;
    Leg1D L;
    dg_status st = diag_begin(c, y, S, "dg_sample", &L);
    if (st != DG_OK) return st;
    if (!out) {
        c->err = "dg_sample: NULL pointer";
        return DG_ERR_ARG;
    }
    SampleArgs a = sample_args(c, y, 0);
    a.out = out;
    a.px = (long long)S * c->cfg.n[0];
    a.py = a.px * S * c->cfg.n[1];
    a.pf = a.py * S * c->cfg.n[2];
    HIPCHK(c, launch_sample(c->cfg.k, S, c->cfg.precision, a, L, c->stream));
    return DG_OK;
}

static bool cubic(const dg_ctx *c) {
    return c->cfg.n[0] == c->cfg.n[1] && c->cfg.n[1] == c->cfg.n[2] && c->cfg.box[0] == c->cfg.box[1] &&
           c->cfg.box[1] == c->cfg.box[2];
}

size_t dg_spectrum_workspace_bytes(const dg_ctx *c, int32_t S) {
    if (!c || S < 1 || S > DIAG_MAX_S) return 0;
    const size_t M = (size_t)S * c->cfg.n[0];
    return M * M * 2 * (M / 2 + 1) * elem_bytes(c);
}

dg_status dg_velocity_spectrum(dg_ctx *c, const void *y, int32_t S, int32_t nbins, double *out, void *work) {
    if (!c) return DG_ERR_ARG;
    Leg1D L;
    dg_status st = diag_begin(c, y, S, "dg_velocity_spectrum", &L);
    if (st != DG_OK) return st;
    if (!out || !work || nbins < 1 || nbins > DIAG_MAX_BINS) {
        c->err = "dg_velocity_spectrum: NULL pointer or nbins outside 1.." + std::to_string(DIAG_MAX_BINS);
        return DG_ERR_ARG;
    }
    if (!cubic(c)) {
        c->err = "dg_velocity_spectrum: needs the same cell count and box length on every axis";
        return DG_ERR_UNSUPPORTED;
    }
    const int M = S * c->cfg.n[0];
    const bool f64 = c->cfg.precision == DG_FP64;
    if (c->fft && c->fft_m != M) {
        (void)hipfftDestroy(static_cast<hipfftHandle>(c->fft));
        c->fft = nullptr;
    }
    if (!c->fft) {
        hipfftHandle h = nullptr;
        if (hipfftPlan3d(&h, M, M, M, f64 ? HIPFFT_D2Z : HIPFFT_R2C) != HIPFFT_SUCCESS) {
            c->err = "dg_velocity_spectrum: hipfftPlan3d failed";
            return DG_ERR_HIP;
        }
        c->fft = h;
        c->fft_m = M;
    }
    hipfftHandle h = static_cast<hipfftHandle>(c->fft);
    if (hipfftSetStream(h, c->stream) != HIPFFT_SUCCESS) {
        c->err = "dg_velocity_spectrum: hipfftSetStream failed";
        return DG_ERR_HIP;
    }
    HIPCHK(c, launch_fill_zero(reinterpret_cast<unsigned long long *>(c->diag_bins), nbins, c->stream));
    const double scale = 1.0 / ((double)M * M * M * (double)M * M * M);
    for (int comp = 1; comp <= 3; comp++) {
        SampleArgs a = sample_args(c, y, comp);
        a.out = work;
        a.px = 2LL * (M / 2 + 1);  // rows padded for the in-place real-to-complex transform
        a.py = a.px * M;
        HIPCHK(c, launch_sample(c->cfg.k, S, c->cfg.precision, a, L, c->stream));
        const hipfftResult r = f64 ? hipfftExecD2Z(h, (hipfftDoubleReal *)work, (hipfftDoubleComplex *)work)
                                   : hipfftExecR2C(h, (hipfftReal *)work, (hipfftComplex *)work);
        if (r != HIPFFT_SUCCESS) {
            c->err = "dg_velocity_spectrum: FFT execution failed";
            return DG_ERR_HIP;
        }
        HIPCHK(c, launch_shells(c->cfg.precision, work, M, nbins, scale, c->diag_bins, c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(out, c->diag_bins, nbins * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DG_OK;
}

dg_status dg_density_pdf(dg_ctx *c, const void *y, int32_t S, double lo, double hi, int32_t nbins, int64_t *counts) {
    if (!c) return DG_ERR_ARG;
    Leg1D L;
    dg_status st = diag_begin(c, y, S, "dg_density_pdf", &L);
    if (st != DG_OK) return st;
    if (!counts || nbins < 1 || nbins > DIAG_MAX_BINS || !std::isfinite(lo) || !std::isfinite(hi) || !(lo < hi)) {
        c->err = "dg_density_pdf: NULL pointer, nbins outside 1.." + std::to_string(DIAG_MAX_BINS) +
                 " or an invalid range";
        return DG_ERR_ARG;
    }
    unsigned long long *dc = reinterpret_cast<unsigned long long *>(c->diag_bins + DIAG_MAX_BINS);
    HIPCHK(c, launch_fill_zero(dc, nbins + 2, c->stream));
    SampleArgs a = sample_args(c, y, 4);
    a.lo = lo;
    a.hi = hi;
    a.nbins = nbins;
    a.counts = dc;
    HIPCHK(c, launch_sample(c->cfg.k, S, c->cfg.precision, a, L, c->stream));
    static_assert(sizeof(int64_t) == sizeof(unsigned long long), "count width");
    HIPCHK(c, hipMemcpyAsync(counts, dc, (nbins + 2) * sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DG_OK;
}

dg_status dg_rms_mach(dg_ctx *c, const void *y, int32_t S, double *out) {
    if (!c) return DG_ERR_ARG;
    Leg1D L;
    dg_status st = diag_begin(c, y, S, "dg_rms_mach", &L);
    if (st != DG_OK) return st;
    if (!out) {
        c->err = "dg_rms_mach: NULL pointer";
        return DG_ERR_ARG;
    }
    const long long nb = sample_blocks(c->ncells);
    SampleArgs a = sample_args(c, y, 4);
    a.mach_partials = c->diag_partials;
    HIPCHK(c, launch_sample(c->cfg.k, S, c->cfg.precision, a, L, c->stream));
    double *tot = c->diag_partials + nb;
    HIPCHK(c, launch_fill_zero(reinterpret_cast<unsigned long long *>(tot), 1, c->stream));
    HIPCHK(c, launch_sum_into(c->diag_partials, nb, tot, c->stream));
    double v = 0.0;
    HIPCHK(c, hipMemcpyAsync(&v, tot, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *out = std::sqrt(v / ((double)c->ncells * S * S * S));
    return DG_OK;
}

// ------------------------------------------------------------------ z slabs (one GPU's share of a split mesh)

size_t dg_plane_count(const dg_ctx *c) {
    return c ? (size_t)NF * c->N * c->cfg.n[0] * c->cfg.n[1] : 0;
}

dg_status dg_set_halo(dg_ctx *c, const void *lo, const void *hi) {
    if (!c) return DG_ERR_ARG;
    if (!(c->cfg.flags & DG_ZHALO)) {
        c->err = "dg_set_halo: the context was made without DG_ZHALO";
        return DG_ERR_STATE;
    }
    if (!lo || !hi) {
        c->err = "dg_set_halo: NULL pointer";
        return DG_ERR_ARG;
    }
    c->halo_lo = lo;
    c->halo_hi = hi;
    return DG_OK;
}

dg_status dg_set_zchunk(dg_ctx *c, int32_t len) {
    if (!c) return DG_ERR_ARG;
    if (len < 0 || len > c->cfg.n[2]) {
        c->err = "dg_set_zchunk: need 0 <= len <= n[2]";
        return DG_ERR_ARG;
    }
    c->zlen = len == 0 ? c->zlen_auto : len;
    return DG_OK;
}

dg_status dg_set_slab(dg_ctx *c, int32_t z0, int32_t nz_global) {
    if (!c) return DG_ERR_ARG;
    if (z0 < 0 || nz_global < c->cfg.n[2] || z0 + c->cfg.n[2] > nz_global) {
        c->err = "dg_set_slab: need 0 <= z0 and z0 + n[2] <= nz_global";
        return DG_ERR_ARG;
    }
    c->slab_z0 = z0;
    c->slab_nz = nz_global;
    return DG_OK;
}
