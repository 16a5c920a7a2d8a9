// HIP kernels of the learned closure and of its training (gfx950).
//
// The closure is not part of the paper: an under-resolved k = 1 run is
// corrected toward high-resolution DG data restricted to its mesh.  A cell's
// features are the weights of itself and its six face neighbours (7 x 5 x 4 =
// 140 values); a 140-128-128-20 tanh network maps their standardised values to
// the 20 standardised entries of a correction of the time derivative,
// dy/dt = -R(y) + c.  A cell whose output is non-finite or outside the trained
// range keeps the plain operator (c = 0).  The mean rows of c are shifted to
// zero sum over the mesh so the conserved totals are untouched.
//
// Every dense product (inference and training) runs on the FP32 matrix cores
// (v_mfma_f32_16x16x4_f32, exact products, FP32 accumulation).
//
// Restriction (training data): the exact L2 projection of a degree-kf state on
// (2n)^3 cells onto degree kc on n^3 cells, a fixed linear map per child cell
// built on the host from the library's own basis and Gauss rules.

#include <algorithm>
#include <mutex>
#include <string>

#include "dg_internal.h"

namespace dgmi {

typedef float f4c __attribute__((ext_vector_type(4)));

// closure inference: 8 waves per workgroup; the weight fragments in LDS (floats)
constexpr int CL_THREADS = 512;
constexpr int CL_W1F = 8 * 35 * 64;     // layer 1: 8 output tiles x 35 K steps
constexpr int CL_W2F = 8 * 4 * 8 * 64;  // layer 2: 32 K steps x 8 output tiles
constexpr int CL_W3F = 8 * 4 * 2 * 64;  // layer 3: 32 K steps x 2 output tiles (rows 20..31 zero)
constexpr int CL_LDS = (CL_W1F + CL_W2F + CL_W3F) * 4;

__device__ inline f4c mfma4(float a, float b, f4c c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// tanh for the inference activations from the identity tanh x = sign(x) (1 - e) / (1 + e),
// e = exp(-2|x|) in (0, 1] (no overflow), with the hardware base-2 exponential and reciprocal:
// absolute error a few 1e-7, which the FP32 accumulations that follow do not resolve
__device__ inline float tanh_act(float x) {
    const float e = __builtin_amdgcn_exp2f(-2.0f * 1.4426950408889634f * __builtin_fabsf(x));
    return __builtin_copysignf((1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e), x);
}

// ------------------------------------------------------------------ inference

// A persistent grid of one 8-wave workgroup per compute unit: the workgroup
// first copies the three weight matrices into LDS in the order the MFMA A
// operand takes them (a fragment of 64 floats per K step and output tile,
// lane l at position l: conflict-free 4-byte reads), 151 KB, then each wave
// takes groups of 16 consecutive cells in turn.  Read from L2 for every group
// instead, the weights cost about 600 loads per group and wave.
//
// A wave evaluates 16 consecutive cells (the MFMA columns).  MFMA lane
// layout (16x16x4, FP32): lane l feeds A[l%16][l/16] and B[l/16][l%16] and
// receives C[4(l/16) + r][l%16], r = 0..3.
//  * layer 1: K-step s = 5 j + i (neighbour j, field i), lane group g = mode l,
//    so the feature index j*20 + i*4 + l is 4 s + g, the order of the features;
//  * layers 2 and 3: K-step (t, r) feeds hidden unit 16 t + 4 g + r, which is
//    exactly what lane group g received in register r of tile t, so the
//    hidden activations never leave the registers;
//  * output tile 0 row 4 g + r is field g, mode r; tile 1 rows 16..19 are
//    field 4 (lane group 0).
template <class S>
__global__ __launch_bounds__(CL_THREADS) void closure_kernel(ClosureArgs a) {
    extern __shared__ float wl[];
    {
        const float *W1 = a.params;
        const float *W2 = W1 + CL_NH * CL_NIN + CL_NH;
        const float *W3 = W2 + CL_NH * CL_NH + CL_NH;
        for (int e = threadIdx.x; e < CL_W1F; e += CL_THREADS) {  // [t][s][lane]
            const int l = e & 63, s = (e >> 6) % 35, t = (e >> 6) / 35;
            wl[e] = W1[(16 * t + (l & 15)) * CL_NIN + 4 * s + (l >> 4)];
        }
        for (int e = threadIdx.x; e < CL_W2F; e += CL_THREADS) {  // [t][r][u][lane]
            const int l = e & 63, u = (e >> 6) & 7, r = (e >> 9) & 3, t = e >> 11;
            wl[CL_W1F + e] = W2[(16 * u + (l & 15)) * CL_NH + 16 * t + 4 * (l >> 4) + r];
        }
        for (int e = threadIdx.x; e < CL_W3F; e += CL_THREADS) {  // [t][r][tile][lane], rows past 20 zero
            const int l = e & 63, tile = (e >> 6) & 1, r = (e >> 7) & 3, t = e >> 9;
            const int row = 16 * tile + (l & 15);
            wl[CL_W1F + CL_W2F + e] = row < CL_NOUT ? W3[row * CL_NH + 16 * t + 4 * (l >> 4) + r] : 0.0f;
        }
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int col = lane & 15;
    const int g = lane >> 4;
    const long long ntasks = (a.ncells + 15) / 16;
    double s0 = 0.0, s4 = 0.0;  // this wave's sums of the mean-row corrections, in task order
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long long slabn = (long long)CL_ROWS * nx;  // 5 fields x 4 modes rows per slab
    const S *y = reinterpret_cast<const S *>(a.y);
    // offsets of the 7 cells whose weights are this lane's features in task w (column col)
    auto task_bases = [&](long long w, long long base[7]) {
        const long long c0 = w * 16;
        const long long cell = c0 + col < a.ncells ? c0 + col : a.ncells - 1;
        const int x = (int)(cell % nx);
        const long long rr = cell / nx;
        const int yy = (int)(rr % ny), zz = (int)(rr / ny);
        auto at = [&](int dx, int dy, int dz) -> long long {
            int xi = x + dx, yi = yy + dy, zi = zz + dz;
            xi = xi < 0 ? xi + nx : (xi >= nx ? xi - nx : xi);
            yi = yi < 0 ? yi + ny : (yi >= ny ? yi - ny : yi);
            zi = zi < 0 ? zi + nz : (zi >= nz ? zi - nz : zi);
            return ((long long)zi * ny + yi) * slabn + xi;
        };
        base[0] = at(0, 0, 0);
        base[1] = at(-1, 0, 0);
        base[2] = at(1, 0, 0);
        base[3] = at(0, -1, 0);
        base[4] = at(0, 1, 0);
        base[5] = at(0, 0, -1);
        base[6] = at(0, 0, 1);
    };
    // the raw features of task w (value s: field s % 5, mode g, of cell s / 5 of the 7), requested
    // one task ahead, after the layer that used the previous ones
    float fv[35];
    auto load_feat = [&](long long w) {
        long long bs[7];
        task_bases(w, bs);
    #pragma unroll
        for (int s = 0; s < 35; s++) fv[s] = (float)y[bs[s / 5] + (long long)((s % 5) * 4 + g) * nx];
    };
    const long long wstride = (long long)gridDim.x * (CL_THREADS / 64);
    long long wave0 = (long long)blockIdx.x * (CL_THREADS / 64) + (threadIdx.x >> 6);
    if (wave0 < ntasks) load_feat(wave0);
    for (long long wave = wave0; wave < ntasks; wave += wstride) {
        const long long cell0 = wave * 16;
        const bool live = cell0 + col < a.ncells;
        long long base[7];
        task_bases(wave, base);
        const float *b1 = a.params + CL_NH * CL_NIN;
        const float *b2 = b1 + CL_NH + CL_NH * CL_NH;
        const float *b3 = b2 + CL_NH + CL_NOUT * CL_NH;
        // the fragments at this lane: an opaque lane base plus immediate offsets (not a register per
        // fragment hoisted out of the loop)
        int lb = lane;
        asm volatile("" : "+v"(lb));
        const float *w1l = wl + lb, *w2l = wl + CL_W1F + lb, *w3l = wl + CL_W1F + CL_W2F + lb;

        // layer 1: 140 -> 128
        f4c h1[8];
    #pragma unroll
        for (int t = 0; t < 8; t++) h1[t] = f4c{0, 0, 0, 0};
    #pragma unroll
        for (int s = 0; s < 35; s++) {
            const int f = 4 * s + g;
            const float b = (fv[s] - a.fmean[f]) * a.fistd[f];
    #pragma unroll
            for (int t = 0; t < 8; t++) h1[t] = mfma4(w1l[(t * 35 + s) * 64], b, h1[t]);
        }
    #pragma unroll
        for (int t = 0; t < 8; t++)
    #pragma unroll
            for (int r = 0; r < 4; r++) h1[t][r] = tanh_act(h1[t][r] + b1[16 * t + 4 * g + r]);

        asm volatile("" ::: "memory");
        if (wave + wstride < ntasks) load_feat(wave + wstride);
        asm volatile("" ::: "memory");
        // layer 2: 128 -> 128
        f4c h2[8];
    #pragma unroll
        for (int t = 0; t < 8; t++) h2[t] = f4c{0, 0, 0, 0};
    #pragma unroll
        for (int t = 0; t < 8; t++)
    #pragma unroll
            for (int r = 0; r < 4; r++) {
    #pragma unroll
                for (int u = 0; u < 8; u++) h2[u] = mfma4(w2l[((t * 4 + r) * 8 + u) * 64], h1[t][r], h2[u]);
            }
    #pragma unroll
        for (int t = 0; t < 8; t++)
    #pragma unroll
            for (int r = 0; r < 4; r++) h2[t][r] = tanh_act(h2[t][r] + b2[16 * t + 4 * g + r]);

        // layer 3: 128 -> 20 (rows 20..31 of tile 1 are zero)
        f4c o[2] = {f4c{0, 0, 0, 0}, f4c{0, 0, 0, 0}};
    #pragma unroll
        for (int t = 0; t < 8; t++)
    #pragma unroll
            for (int r = 0; r < 4; r++) {
                o[0] = mfma4(w3l[((t * 4 + r) * 2) * 64], h2[t][r], o[0]);
                o[1] = mfma4(w3l[((t * 4 + r) * 2 + 1) * 64], h2[t][r], o[1]);
            }
        // output entries held by this lane: tile 0 rows 4g+r (field g), tile 1 rows 16+r (lane group 0)
        bool bad = false;
    #pragma unroll
        for (int r = 0; r < 4; r++) {
            const int j0 = 4 * g + r;
            o[0][r] += b3[j0];
            bad |= !(__builtin_fabsf(o[0][r]) <= a.obound[j0]);  // also true for NaN
            if (g == 0) {
                o[1][r] += b3[16 + r];
                bad |= !(__builtin_fabsf(o[1][r]) <= a.obound[16 + r]);
            }
        }
        // a cell falls back if any of its 20 outputs is out of range: OR over the 4 lane groups
        int bi = bad ? 1 : 0;
        bi |= __shfl_xor(bi, 16, 64);
        bi |= __shfl_xor(bi, 32, 64);
        bad = bi != 0;
        S *corr = reinterpret_cast<S *>(a.corr);
        double m0 = 0.0, m4 = 0.0;  // this lane's mean-row corrections (field g; field 4 on group 0)
    #pragma unroll
        for (int r = 0; r < 4; r++) {
            const int j0 = 4 * g + r;
            const float c0 = bad ? 0.0f : a.oscale[j0] * o[0][r];
            if (live) corr[base[0] + (long long)j0 * nx] = (S)c0;
            if (r == 0) m0 = live ? (double)(S)c0 : 0.0;
            if (g == 0) {
                const float c1 = bad ? 0.0f : a.oscale[16 + r] * o[1][r];
                if (live) corr[base[0] + (long long)(16 + r) * nx] = (S)c1;
                if (r == 0) m4 = live ? (double)(S)c1 : 0.0;
            }
        }
        // per-wave sums of the mean rows over the 16 columns, fixed order
    #pragma unroll
        for (int off = 8; off >= 1; off >>= 1) {
            m0 += __shfl_xor(m0, off, 16);
            m4 += __shfl_xor(m4, off, 16);
        }
        s0 += m0;
        s4 += m4;
        const unsigned long long fb = __ballot(bad && live && g == 0);
        if (lane == 0 && fb) atomicAdd(a.fallbacks, (unsigned long long)__popcll(fb));
    }
    // one partial per wave of the grid; the last workgroup to finish forms the means from them in a
    // fixed order (and resets the counter for the next launch), so no second kernel is launched
    const long long gw = (long long)blockIdx.x * (CL_THREADS / 64) + (threadIdx.x >> 6);
    if (col == 0) {
        a.partials[gw * NF + g] = s0;
        if (g == 0) a.partials[gw * NF + 4] = s4;
    }
    __threadfence();
    __syncthreads();
    __shared__ int last;
    if (threadIdx.x == 0) last = atomicAdd(a.done, 1ull) == (unsigned long long)gridDim.x - 1 ? 1 : 0;
    __syncthreads();
    if (!last) return;
    __threadfence();
    double *red = reinterpret_cast<double *>(wl);  // the weights are no longer read
    const long long nparts = (long long)gridDim.x * (CL_THREADS / 64);
    for (int i = 0; i < NF; i++) {
        double sum = 0.0;
        for (long long w = threadIdx.x; w < nparts; w += CL_THREADS)
            sum += __hip_atomic_load(a.partials + w * NF + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        red[threadIdx.x] = sum;
        __syncthreads();
        for (int h = CL_THREADS / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) a.cmean[i] = red[0] / (double)a.ncells;
        __syncthreads();
    }
    if (threadIdx.x == 0) __hip_atomic_store(a.done, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

hipError_t launch_closure(int prec, const ClosureArgs &a, hipStream_t s) {
    const long long nwaves = (a.ncells + 15) / 16;
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const void *fn = prec == DG_FP64 ? reinterpret_cast<const void *>(&closure_kernel<double>)
                                     : reinterpret_cast<const void *>(&closure_kernel<float>);
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, CL_LDS);
    if (e != hipSuccess) return e;
    // one workgroup per compute unit (the weights fill its LDS), no more than there are groups
    const long long nb = std::min<long long>((nwaves + CL_THREADS / 64 - 1) / (CL_THREADS / 64), std::max(ncu, 1));
    if (prec == DG_FP64)
        hipLaunchKernelGGL((closure_kernel<double>), dim3(nb), dim3(CL_THREADS), CL_LDS, s, a);
    else
        hipLaunchKernelGGL((closure_kernel<float>), dim3(nb), dim3(CL_THREADS), CL_LDS, s, a);
    return hipGetLastError();
}

__global__ void zero_u64_kernel(unsigned long long *p) { *p = 0ull; }

hipError_t launch_zero_u64(unsigned long long *p, hipStream_t s) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, p);
    return hipGetLastError();
}

// ------------------------------------------------------------------ training data

// feat[cell][j][i][l] = y of neighbour j (self, -x, +x, -y, +y, -z, +z), field i, mode l
template <class S>
__global__ void features_kernel(const S *__restrict__ y, float *__restrict__ feat, int N, int nx, int ny, int nz,
                                long long nc) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nc * 7) return;
    const long long cell = id / 7;
    const int j = (int)(id - cell * 7);
    const int dx[7] = {0, -1, 1, 0, 0, 0, 0}, dy[7] = {0, 0, 0, -1, 1, 0, 0}, dz[7] = {0, 0, 0, 0, 0, -1, 1};
    int x = (int)(cell % nx);
    const long long r = cell / nx;
    int yy = (int)(r % ny), zz = (int)(r / ny);
    x = (x + dx[j] + nx) % nx;
    yy = (yy + dy[j] + ny) % ny;
    zz = (zz + dz[j] + nz) % nz;
    const long long b = ((long long)zz * ny + yy) * (long long)NF * N * nx + x;
    float *o = feat + (cell * 7 + j) * (long long)NF * N;
    for (int q = 0; q < NF * N; q++) o[q] = (float)y[b + (long long)q * nx];
}

// target[cell][i][l] = rc - prf (state layout in, sample rows out)
template <class S>
__global__ void targets_kernel(const S *__restrict__ rc, const S *__restrict__ prf, float *__restrict__ out, int N,
                               int nx, long long nc) {
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= nc) return;
    const long long r = cell / nx;
    const long long b = r * (long long)NF * N * nx + (cell - r * nx);
    for (int q = 0; q < NF * N; q++)
        out[cell * NF * N + q] = (float)((double)rc[b + (long long)q * nx] - (double)prf[b + (long long)q * nx]);
}

hipError_t launch_features(int prec, const void *y, float *feat, int N, int nx, int ny, int nz, long long nc,
                           hipStream_t s) {
    const long long nb = (nc * 7 + 255) / 256;
    if (prec == DG_FP64)
        hipLaunchKernelGGL((features_kernel<double>), dim3(nb), dim3(256), 0, s, (const double *)y, feat, N, nx, ny, nz,
                           nc);
    else
        hipLaunchKernelGGL((features_kernel<float>), dim3(nb), dim3(256), 0, s, (const float *)y, feat, N, nx, ny, nz,
                           nc);
    return hipGetLastError();
}

hipError_t launch_targets(int prec, const void *rc, const void *prf, float *out, int N, int nx, long long nc,
                          hipStream_t s) {
    const long long nb = (nc + 255) / 256;
    if (prec == DG_FP64)
        hipLaunchKernelGGL((targets_kernel<double>), dim3(nb), dim3(256), 0, s, (const double *)rc,
                           (const double *)prf, out, N, nx, nc);
    else
        hipLaunchKernelGGL((targets_kernel<float>), dim3(nb), dim3(256), 0, s, (const float *)rc, (const float *)prf,
                           out, N, nx, nc);
    return hipGetLastError();
}

// exact L2 restriction: yc[C][i][l] = sum over children ch and fine modes m of M[ch][l][m] yf[child][i][m]
template <class S>
__global__ void restrict_kernel(const S *__restrict__ yf, S *__restrict__ yc, const double *__restrict__ M, int Nf,
                                int Nc, int NX, int NY, int NZ) {
    const long long ncc = (long long)NX * NY * NZ;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= ncc * NF) return;
    const long long C = id / NF;
    const int i = (int)(id - C * NF);
    const int X = (int)(C % NX);
    const long long rc = C / NX;
    const int Y = (int)(rc % NY), Z = (int)(rc / NY);
    const int FX = 2 * NX, FY = 2 * NY;
    double acc[35];
    for (int l = 0; l < Nc; l++) acc[l] = 0.0;
    for (int ch = 0; ch < 8; ch++) {
        const int fx = 2 * X + (ch & 1), fy = 2 * Y + ((ch >> 1) & 1), fz = 2 * Z + (ch >> 2);
        const long long b = (((long long)fz * FY + fy) * NF + i) * (long long)Nf * FX + fx;
        const double *Mc = M + (long long)ch * Nc * Nf;
        for (int m = 0; m < Nf; m++) {
            const double v = (double)yf[b + (long long)m * FX];
            for (int l = 0; l < Nc; l++) acc[l] += Mc[l * Nf + m] * v;
        }
    }
    const long long bc = ((long long)Z * NY + Y) * NF * (long long)Nc * NX + (long long)i * Nc * NX + X;
    for (int l = 0; l < Nc; l++) yc[bc + (long long)l * NX] = (S)acc[l];
}

hipError_t launch_restrict(int prec, const void *yf, void *yc, const double *M, int Nf, int Nc, int NX, int NY, int NZ,
                           hipStream_t s) {
    const long long n = (long long)NX * NY * NZ * NF;
    const long long nb = (n + 255) / 256;
    if (prec == DG_FP64)
        hipLaunchKernelGGL((restrict_kernel<double>), dim3(nb), dim3(256), 0, s, (const double *)yf, (double *)yc, M, Nf,
                           Nc, NX, NY, NZ);
    else
        hipLaunchKernelGGL((restrict_kernel<float>), dim3(nb), dim3(256), 0, s, (const float *)yf, (float *)yc, M, Nf,
                           Nc, NX, NY, NZ);
    return hipGetLastError();
}

// ------------------------------------------------------------------ training: dense products

// C[m][n] = sum_k A[m][k] B[k][n] with arbitrary strides, one 16x16 tile per
// wave, 2x2 waves per workgroup; epilogue: + bias[m], then tanh (EP_TANH) or
// times (1 - E[m][n]^2) (EP_DTANH, the tanh derivative at output E).
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs a) {
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int col = lane & 15, g = lane >> 4;
    const int m0 = blockIdx.y * 32 + (w >> 1) * 16;
    const int n0 = blockIdx.x * 32 + (w & 1) * 16;
    if (m0 >= a.M || n0 >= a.N) return;  // wave-uniform
    const int am = m0 + col, bn = n0 + col;
    const bool arow = am < a.M, bcol = bn < a.N;
    const float *A = a.A + (arow ? (long long)am * a.sam : 0);
    const float *B = a.B + (bcol ? (long long)bn * a.sbn : 0);
    f4c acc = f4c{0, 0, 0, 0};
    for (int k0 = 0; k0 < a.K; k0 += 4) {
        const int k = k0 + g;
        const bool kin = k < a.K;
        const float av = (arow && kin) ? A[(long long)k * a.sak] : 0.0f;
        const float bv = (bcol && kin) ? B[(long long)k * a.sbk] : 0.0f;
        acc = mfma4(av, bv, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const int m = m0 + 4 * g + r, n = n0 + col;
        if (m < a.M && n < a.N) {
            float v = acc[r];
            if (a.bias) v += a.bias[m];
            if (a.ep == EP_TANH) v = tanhf(v);
            if (a.ep == EP_DTANH) {
                const float e = a.E[(long long)m * a.scm + (long long)n * a.scn];
                v *= 1.0f - e * e;
            }
            a.C[(long long)m * a.scm + (long long)n * a.scn] = v;
        }
    }
}

hipError_t launch_gemm(const GemmArgs &a, hipStream_t s) {
    dim3 grid((a.N + 31) / 32, (a.M + 31) / 32);
    hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// out[m] = sum_n X[m][n] (row-major, n fastest), fixed summation order
__global__ __launch_bounds__(256) void rowsum_kernel(const float *X, int N, float *out) {
    __shared__ double red[256];
    const float *x = X + (long long)blockIdx.x * N;
    double s = 0.0;
    for (int n = threadIdx.x; n < N; n += 256) s += x[n];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = (float)red[0];
}

hipError_t launch_rowsum(const float *X, int M, int N, float *out, hipStream_t s) {
    hipLaunchKernelGGL(rowsum_kernel, dim3(M), dim3(256), 0, s, X, N, out);
    return hipGetLastError();
}

// Counter-based standard normal draw for element `idx` of stream `seed`: the
// SplitMix64 output function (Steele, Lea and Flood, 2014) of the counter gives
// two 32-bit uniforms, the Box-Muller transform a normal deviate.
__device__ inline float normal_draw(unsigned long long seed, unsigned long long idx) {
    unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (idx + 1ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const float u1 = ((float)(unsigned)(z >> 40) + 1.0f) * (1.0f / 16777216.0f);  // (0, 1]
    const float u2 = (float)(unsigned)(z & 0xffffffull) * (1.0f / 16777216.0f);   // [0, 1)
    return sqrtf(-2.0f * logf(u1)) * __builtin_amdgcn_cosf(u2);  // cos(2 pi u2): argument in revolutions
}

// Xb[k][s] = X[rows[s]][k] (+ noise * N(0,1)) (feature-major batch), rows == nullptr: row s
__global__ void gather_kernel(const float *X, int cols, const int *rows, int batch, float *Xb, float noise,
                              unsigned long long seed) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long long)cols * batch) return;
    const int s = (int)(id % batch);
    const int k = (int)(id / batch);
    const long long r = rows ? rows[s] : s;
    float v = X[r * cols + k];
    if (noise != 0.0f) v += noise * normal_draw(seed, (unsigned long long)id);
    Xb[id] = v;
}

hipError_t launch_gather(const float *X, int cols, const int *rows, int batch, float *Xb, hipStream_t s, float noise,
                         unsigned long long seed) {
    const long long n = (long long)cols * batch;
    hipLaunchKernelGGL(gather_kernel, dim3((n + 255) / 256), dim3(256), 0, s, X, cols, rows, batch, Xb, noise, seed);
    return hipGetLastError();
}

// MSE over batch x nout: dY = 2 (Y - T) / (batch nout), loss = mean (Y - T)^2
// (Y, T, dY feature-major [nout][batch]); one workgroup, fixed order
__global__ __launch_bounds__(256) void mse_kernel(const float *Y, const float *T, float *dY, long long n, double *loss) {
    __shared__ double red[256];
    const float sc = (float)(2.0 / (double)n);
    double s = 0.0;
    for (long long j = threadIdx.x; j < n; j += 256) {
        const float e = Y[j] - T[j];
        s += (double)e * (double)e;
        dY[j] = sc * e;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) *loss = red[0] / (double)n;
}

hipError_t launch_mse(const float *Y, const float *T, float *dY, long long n, double *loss, hipStream_t s) {
    hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(256), 0, s, Y, T, dY, n, loss);
    return hipGetLastError();
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, long long n, int step, double lr, double b1,
                            double b2, double eps) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    const float gj = g[j];
    const float mj = (float)b1 * m[j] + (float)(1.0 - b1) * gj;
    const float vj = (float)b2 * v[j] + (float)(1.0 - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    p[j] -= (float)lr * (mj / (float)c1) / (sqrtf(vj / (float)c2) + (float)eps);
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, long long n, int step, double lr, double b1,
                       double b2, double eps, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, step, lr, b1, b2, eps);
    return hipGetLastError();
}

// ------------------------------------------------------------------ column statistics

// pass 1 (what = 0): per chunk of rows, sum, sum of squares and max |x| per column;
// pass 3 (what = 1): per chunk, sum of (x - mean)^2.  Column c is thread c.
__global__ __launch_bounds__(256) void colstat_pass(const float *x, long long rows, int cols, long long chunk,
                                                    const double *mean, double *part, int what) {
    const int c = threadIdx.x;
    if (c >= cols) return;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = lo + chunk < rows ? lo + chunk : rows;
    double s = 0.0, s2 = 0.0, mx = 0.0;
    if (what == 0) {
        for (long long r = lo; r < hi; r++) {
            const double v = x[r * cols + c];
            s += v;
            s2 += v * v;
            mx = fmax(mx, fabs(v));
        }
        double *p = part + ((long long)blockIdx.x * cols + c) * 3;
        p[0] = s;
        p[1] = s2;
        p[2] = mx;
    } else {
        const double mu = mean[c];
        for (long long r = lo; r < hi; r++) {
            const double d = x[r * cols + c] - mu;
            s += d * d;
        }
        part[((long long)blockIdx.x * cols + c) * 3] = s;
    }
}

// pass 2 (what = 0): mean, rms, maxabs; pass 4 (what = 1): std
__global__ __launch_bounds__(256) void colstat_final(const double *part, int nchunks, long long rows, int cols,
                                                     double *mean, double *stdv, double *rms, double *maxabs,
                                                     int what) {
    const int c = threadIdx.x;
    if (c >= cols) return;
    double s = 0.0, s2 = 0.0, mx = 0.0;
    for (int b = 0; b < nchunks; b++) {
        const double *p = part + ((long long)b * cols + c) * 3;
        s += p[0];
        if (what == 0) {
            s2 += p[1];
            mx = fmax(mx, p[2]);
        }
    }
    if (what == 0) {
        mean[c] = s / (double)rows;
        rms[c] = sqrt(s2 / (double)rows);
        maxabs[c] = mx;
    } else {
        stdv[c] = sqrt(s / (double)rows);
    }
}

hipError_t launch_colstats(const float *x, long long rows, int cols, double *part, int nchunks, double *mean,
                           double *stdv, double *rms, double *maxabs, hipStream_t s) {
    const long long chunk = (rows + nchunks - 1) / nchunks;
    hipLaunchKernelGGL(colstat_pass, dim3(nchunks), dim3(256), 0, s, x, rows, cols, chunk, (const double *)nullptr,
                       part, 0);
    hipLaunchKernelGGL(colstat_final, dim3(1), dim3(256), 0, s, (const double *)part, nchunks, rows, cols, mean, stdv,
                       rms, maxabs, 0);
    hipLaunchKernelGGL(colstat_pass, dim3(nchunks), dim3(256), 0, s, x, rows, cols, chunk, (const double *)mean, part,
                       1);
    hipLaunchKernelGGL(colstat_final, dim3(1), dim3(256), 0, s, (const double *)part, nchunks, rows, cols, mean, stdv,
                       rms, maxabs, 1);
    return hipGetLastError();
}

// x[r][c] = (x[r][c] - shift[c]) / scale[c]
__global__ void standardize_kernel(float *x, long long n, int cols, const double *shift, const double *scale) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int c = (int)(j % cols);
    x[j] = (float)(((double)x[j] - shift[c]) / scale[c]);
}

hipError_t launch_standardize(float *x, long long rows, int cols, const double *shift, const double *scale,
                              hipStream_t s) {
    const long long n = rows * cols;
    hipLaunchKernelGGL(standardize_kernel, dim3((n + 255) / 256), dim3(256), 0, s, x, n, cols, shift, scale);
    return hipGetLastError();
}

// ------------------------------------------------------------------ allocation-free column statistics

// The scratch of dg_column_stats_noalloc: the per-chunk partial sums of the column statistics
// (chunk, column, 3), in a file-scope device array, one copy per GPU, held until the process ends.
// Host code never uses the array's name as an address: it takes the address that
// hipGetSymbolAddress returns for the current device, once per device, and passes that.
constexpr int NOALLOC_MAX_COLS = 160;   // 140 closure features, with room to spare
constexpr int NOALLOC_CHUNKS = 1024;    // the chunking of dg_column_stats: the same bits
static __device__ __align__(256) double scratch[(size_t)NOALLOC_CHUNKS * NOALLOC_MAX_COLS * 3];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

// the current device's copy of the scratch array (looked up on the device's first call)
static hipError_t scratch_address(double **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace dgmi

extern "C" dg_status dg_column_stats_noalloc(const float *x, int64_t rows, int32_t cols, double *mean, double *stdev,
                                             double *rms, double *maxabs, void *hip_stream) {
    using namespace dgmi;
    if (!x || rows < 1 || cols < 1 || !mean || !stdev || !rms || !maxabs) {
        set_call_error("dg_column_stats_noalloc: NULL pointer, rows < 1 or cols < 1");
        return DG_ERR_ARG;
    }
    if (cols > NOALLOC_MAX_COLS) {
        set_call_error("dg_column_stats_noalloc: cols > 160, the columns its static scratch holds "
                       "(dg_column_stats takes up to 256 with a workspace)");
        return DG_ERR_ARG;
    }
    double *part = nullptr;
    hipError_t e = scratch_address(&part);
    if (e == hipSuccess) {
        const int nchunks = (int)(rows < NOALLOC_CHUNKS ? rows : NOALLOC_CHUNKS);
        e = launch_colstats(x, rows, cols, part, nchunks, mean, stdev, rms, maxabs,
                            reinterpret_cast<hipStream_t>(hip_stream));
    }
    if (e != hipSuccess) {
        set_call_error((std::string("dg_column_stats_noalloc: ") + hipGetErrorString(e)).c_str());
        return DG_ERR_HIP;
    }
    return DG_OK;
}
