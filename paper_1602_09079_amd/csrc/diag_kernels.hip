// Turbulence diagnostics of arXiv 1602.09079 on the GPU: sub-cell sampling of the
// DG polynomials (Sec. 4: slices and PDFs use 4^3 points per cell), the shell
// power spectrum of the velocity (Sec. 3.3), the log-density PDF (Sec. 4.4) and
// the rms Mach number (Sec. 4.1).
#include <hip/hip_runtime.h>

#include "dg_internal.h"

namespace dgmi {

constexpr int SAMPLE_THREADS = 256;

long long sample_blocks(long long nc) { return (nc + SAMPLE_THREADS - 1) / SAMPLE_THREADS; }

__device__ inline float log10_d(float x) { return log10f(x); }
__device__ inline double log10_d(double x) { return log10(x); }

// One thread per cell (x consecutive over the lanes).  The cell is split into S equal parts per
// axis; per z slice of the S^3 part centres the five fields are evaluated by sum factorisation
// over the 1D Legendre factors at the centres (z, then y, then x).  Grid point (X, Y, Z) =
// (S ix + a, S iy + b, S iz + c).
template <int K, int S, class C>
__global__ __launch_bounds__(SAMPLE_THREADS) void sample_kernel(SampleArgs A, Leg1D L) {
    constexpr int N = (K + 1) * (K + 2) * (K + 3) / 6;
    __shared__ double red[SAMPLE_THREADS];
    __shared__ unsigned int hist[DIAG_MAX_BINS + 2];
    const bool stats = A.what == 4;
    if (stats && A.nbins > 0) {
        for (int j = threadIdx.x; j < A.nbins + 2; j += blockDim.x) hist[j] = 0u;
        __syncthreads();
    }
    C P[K + 1][S];
#pragma unroll
    for (int u = 0; u <= K; u++)
#pragma unroll
        for (int a = 0; a < S; a++) P[u][a] = (C)L.p[u][a];
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double msum = 0.0;
    if (cell < A.nc) {
        const C *y = static_cast<const C *>(A.y);
        const long long r = cell / A.nx;
        const int ix = (int)(cell - r * A.nx);
        const int iy = (int)(r % A.ny);
        const int iz = (int)(r / A.ny);
        const long long base = r * (long long)NF * N * A.nx + ix;
        C wt[NF][N];
#pragma unroll
        for (int i = 0; i < NF; i++)
#pragma unroll
            for (int l = 0; l < N; l++) wt[i][l] = y[base + (long long)(i * N + l) * A.nx];
        const C g = (C)A.gamma;
#pragma unroll
        for (int c = 0; c < S; c++) {
            auto eval = [&](int i, C q[S][S]) {
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
                C t2[K + 1][S];
#pragma unroll
                for (int u = 0; u <= K; u++)
#pragma unroll
                    for (int b = 0; b < S; b++) {
                        C t = 0;
#pragma unroll
                        for (int v = 0; u + v <= K; v++) t += t1[u][v] * P[v][b];
                        t2[u][b] = t;
                    }
#pragma unroll
                for (int b = 0; b < S; b++)
#pragma unroll
                    for (int a = 0; a < S; a++) {
                        C t = 0;
#pragma unroll
                        for (int u = 0; u <= K; u++) t += t2[u][b] * P[u][a];
                        q[b][a] = t;
                    }
            };
            const long long Z = (long long)iz * S + c;
            if (A.what == 0) {
                C *o = static_cast<C *>(A.out);
#pragma unroll
                for (int i = 0; i < NF; i++) {
                    C q[S][S];
                    eval(i, q);
#pragma unroll
                    for (int b = 0; b < S; b++)
#pragma unroll
                        for (int a = 0; a < S; a++)
                            o[i * A.pf + Z * A.py + (long long)(iy * S + b) * A.px + (long long)ix * S + a] = q[b][a];
                }
            } else if (A.what <= 3) {
                C *o = static_cast<C *>(A.out);
                C rho[S][S], m[S][S];
                eval(0, rho);
#pragma unroll
                for (int i = 1; i < 4; i++)  // compile-time field index: the weights stay in registers
                    if (i == A.what) eval(i, m);
#pragma unroll
                for (int b = 0; b < S; b++)
#pragma unroll
                    for (int a = 0; a < S; a++)
                        o[Z * A.py + (long long)(iy * S + b) * A.px + (long long)ix * S + a] = m[b][a] / rho[b][a];
            } else {
                C rho[S][S], m2[S][S], e[S][S], qm[S][S];
                eval(0, rho);
                eval(4, e);
#pragma unroll
                for (int i = 1; i < 4; i++) {
                    eval(i, qm);
#pragma unroll
                    for (int b = 0; b < S; b++)
#pragma unroll
                        for (int a = 0; a < S; a++) m2[b][a] = (i == 1 ? C(0) : m2[b][a]) + qm[b][a] * qm[b][a];
                }
#pragma unroll
                for (int b = 0; b < S; b++)
#pragma unroll
                    for (int a = 0; a < S; a++) {
                        const C rh = rho[b][a];
                        if (A.mach_partials) {
                            // |v|^2 / c^2 = |m|^2 / (gamma rho p), p = (gamma-1)(E - |m|^2/(2 rho))
                            const C p = (g - C(1)) * (e[b][a] - C(0.5) * m2[b][a] / rh);
                            msum += (double)(m2[b][a] / (g * rh * p));
                        }
                        if (A.nbins > 0) {
                            int bin;
                            if (!(rh > C(0)) || !(rh < __builtin_huge_valf())) {
                                bin = 0;
                            } else {
                                const double x = (double)log10_d(rh);
                                if (x < A.lo) bin = 0;
                                else if (x >= A.hi) bin = A.nbins + 1;
                                else {
                                    int bb = (int)floor((x - A.lo) / (A.hi - A.lo) * A.nbins);
                                    bin = 1 + (bb < A.nbins - 1 ? bb : A.nbins - 1);
                                }
                            }
                            atomicAdd(&hist[bin], 1u);
                        }
                    }
            }
        }
    }
    if (stats) {
        if (A.mach_partials) {
            red[threadIdx.x] = msum;
            __syncthreads();
            for (int h = SAMPLE_THREADS / 2; h > 0; h >>= 1) {
                if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
                __syncthreads();
            }
            if (threadIdx.x == 0) A.mach_partials[blockIdx.x] = red[0];
        }
        if (A.nbins > 0) {
            __syncthreads();
            for (int j = threadIdx.x; j < A.nbins + 2; j += blockDim.x)
                if (hist[j]) atomicAdd(&A.counts[j], (unsigned long long)hist[j]);
        }
    }
}

template <int K, int S>
static hipError_t launch_sample_ks(int prec, const SampleArgs &a, const Leg1D &L, hipStream_t s) {
    const long long nb = sample_blocks(a.nc);
    if (prec == DG_FP64)
        hipLaunchKernelGGL((sample_kernel<K, S, double>), dim3(nb), dim3(SAMPLE_THREADS), 0, s, a, L);
    else
        hipLaunchKernelGGL((sample_kernel<K, S, float>), dim3(nb), dim3(SAMPLE_THREADS), 0, s, a, L);
    return hipGetLastError();
}

template <int K>
static hipError_t launch_sample_k(int S, int prec, const SampleArgs &a, const Leg1D &L, hipStream_t s) {
    switch (S) {
        case 1: return launch_sample_ks<K, 1>(prec, a, L, s);
        case 2: return launch_sample_ks<K, 2>(prec, a, L, s);
        case 3: return launch_sample_ks<K, 3>(prec, a, L, s);
        case 4: return launch_sample_ks<K, 4>(prec, a, L, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sample(int k, int S, int prec, const SampleArgs &a, const Leg1D &L, hipStream_t s) {
    switch (k) {
        case 0: return launch_sample_k<0>(S, prec, a, L, s);
        case 1: return launch_sample_k<1>(S, prec, a, L, s);
        case 2: return launch_sample_k<2>(S, prec, a, L, s);
        case 3: return launch_sample_k<3>(S, prec, a, L, s);
        case 4: return launch_sample_k<4>(S, prec, a, L, s);
        default: return hipErrorInvalidValue;
    }
}

// Shell power of an R2C spectrum [M][M][Mh], Mh = M/2 + 1 (interleaved complex).  Element
// (kz, ky, kx) has wave vector (kx, ky or ky - M, kz or kz - M); it stands for itself and, for
// 0 < kx < M/2 (or kx > 0 when M is odd), for its conjugate at -n as well (weight 2).  The shell
// is the integer nearest to |n|, found in integer arithmetic: s = r + [4 |n|^2 >= (2r + 1)^2],
// r = floor(sqrt(|n|^2)).
__device__ inline long long shell_of(long long n2) {
    long long r = (long long)sqrt((double)n2);
    while (r * r > n2) r--;
    while ((r + 1) * (r + 1) <= n2) r++;
    return r + (4 * n2 >= (2 * r + 1) * (2 * r + 1) ? 1 : 0);
}

// smallest kx >= 0 whose shell (with n_y^2 + n_z^2 = c) is at least s: the shell is nondecreasing
// in kx, so the kx of one shell form one interval of a row
__device__ inline long long first_kx(long long c, long long s) {
    const double t = ((double)s - 0.5) * ((double)s - 0.5) - (double)c;
    long long x = t > 0.0 ? (long long)sqrt(t) : 0;
    while (x > 0 && shell_of((x - 1) * (x - 1) + c) >= s) x--;
    while (shell_of(x * x + c) < s) x++;
    return x;
}

// One workgroup per shell s < nbins, no atomics: the pairs (n_y, n_z) of the square |n_y|, |n_z| <=
// s + 1 are dealt to the threads in a fixed order, each thread adds the kx interval of shell s of
// each of its rows in order, and the workgroup adds the threads' sums in a fixed tree; the shell's
// bin then takes the sum (the three velocity components in turn, in stream order).  Bitwise
// reproducible.
template <class C>
__global__ __launch_bounds__(256) void shells_kernel(const C *__restrict__ spec, int M, int nbins, double scale,
                                                     double *__restrict__ bins) {
    __shared__ double red[256];
    const long long s = blockIdx.x;
    const long long Mh = M / 2 + 1;
    const long long nlo = -((M - 1) / 2), nhi = M / 2;  // signed wave numbers of a full axis
    const long long R = s + 1 < nhi ? s + 1 : nhi;
    const long long side = 2 * R + 1;
    double acc = 0.0;
    for (long long p = threadIdx.x; p < side * side; p += blockDim.x) {
        const long long ny = p % side - R, nz = p / side - R;
        if (ny < nlo || nz < nlo) continue;
        const long long c = ny * ny + nz * nz;
        if (shell_of(c) > s) continue;
        const long long a0 = first_kx(c, s);
        long long a1 = first_kx(c, s + 1) - 1;
        if (a1 > Mh - 1) a1 = Mh - 1;
        const long long ky = ny >= 0 ? ny : ny + M, kz = nz >= 0 ? nz : nz + M;
        const C *row = spec + 2 * ((kz * M + ky) * Mh);
        for (long long kx = a0; kx <= a1; kx++) {
            const double re = (double)row[2 * kx], im = (double)row[2 * kx + 1];
            const bool self_conj = kx == 0 || (M % 2 == 0 && kx == M / 2);
            acc += (re * re + im * im) * (self_conj ? 1.0 : 2.0);
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) bins[s] += red[0] * scale;
}

hipError_t launch_shells(int prec, const void *spec, int M, int nbins, double scale, double *bins, hipStream_t s) {
    if (prec == DG_FP64)
        hipLaunchKernelGGL(shells_kernel<double>, dim3(nbins), dim3(256), 0, s, (const double *)spec, M, nbins, scale,
                           bins);
    else
        hipLaunchKernelGGL(shells_kernel<float>, dim3(nbins), dim3(256), 0, s, (const float *)spec, M, nbins, scale,
                           bins);
    return hipGetLastError();
}

__global__ void fill_zero_kernel(unsigned long long *p, long long n) {
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (long long)gridDim.x * blockDim.x)
        p[j] = 0ull;
}

hipError_t launch_fill_zero(unsigned long long *p, long long n, hipStream_t s) {
    long long nb = (n + 255) / 256;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(nb), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace dgmi
