// Streaming vector kernels for the Krylov solver and the tuner.
//
// Reductions are deterministic: a fixed grid of kRedBlocks x kRedThreads
// threads accumulates in FP64 with a grid-stride loop, each block writes one
// partial, and a single block adds the partials in a fixed order.  Scalars
// (alpha, beta, norms) stay on the device between kernels, so a CG
// iteration needs no host round trip.
#include "blas.h"

namespace mfhex {

namespace {

template <typename T>
__device__ __forceinline__ double ld(const T *p, int64_t i) { return (double)p[i]; }

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

__device__ __forceinline__ double block_max(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    return sh[0];
}

template <typename TA, typename TB>
__global__ void __launch_bounds__(kRedThreads) k_dot(const TA *__restrict__ a, const TB *__restrict__ b, int64_t n,
                                                     double *__restrict__ partial)
{
    __shared__ double sh[kRedThreads];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads)
        s += ld(a, i) * ld(b, i);
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kRedThreads) k_finalize(const double *__restrict__ partial, double *__restrict__ sc,
                                                          int op, int k, double *__restrict__ hist, int hist_len)
{
    __shared__ double sh[kRedThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) s += partial[i];
    s = block_sum(s, sh);
    if (threadIdx.x != 0) return;
    if (op == kFinStore) {
        sc[k] = s;
    } else if (op == kFinAlpha) {
        sc[kScPAp] = s;
        const double al = sc[kScRR] / s;
        if (!(s > 0.0) || !isfinite(al)) {
            sc[kScFlag] = 1.0;
            sc[kScAlpha] = 0.0;
        } else {
            sc[kScAlpha] = al;
        }
    } else if (op == kFinBeta) {
        const double rr = sc[kScRR];
        sc[kScRRPrev] = rr;
        sc[kScRRNew] = s;
        sc[kScBeta] = (rr > 0.0) ? s / rr : 0.0;
        sc[kScRR] = s;
        if (!isfinite(s)) sc[kScFlag] = 1.0;
        if (hist && k >= 0 && k < hist_len) hist[k] = sqrt(s);
    } else if (op == kFinAlphaPre) {
        sc[kScPAp] = s;
        const double al = sc[kScRZ] / s;
        if (!(s > 0.0) || !isfinite(al)) {
            sc[kScFlag] = 1.0;
            sc[kScAlpha] = 0.0;
        } else {
            sc[kScAlpha] = al;
        }
    }
}

// Preconditioned beta step: partial[0..) holds r.r, partial[kRedBlocks..) holds r.z.
__global__ void __launch_bounds__(kRedThreads) k_finalize_beta_pre(const double *__restrict__ partial,
                                                                   double *__restrict__ sc, int k,
                                                                   double *__restrict__ hist, int hist_len)
{
    __shared__ double sh[kRedThreads];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) {
        a += partial[i];
        b += partial[kRedBlocks + i];
    }
    a = block_sum(a, sh);
    __syncthreads();
    b = block_sum(b, sh);
    if (threadIdx.x != 0) return;
    const double rz = sc[kScRZ];
    sc[kScRRPrev] = sc[kScRR];
    sc[kScRRNew] = a;
    sc[kScRR] = a;
    sc[kScRZPrev] = rz;
    sc[kScBeta] = (rz > 0.0) ? b / rz : 0.0;
    sc[kScRZ] = b;
    if (!isfinite(a) || !isfinite(b)) sc[kScFlag] = 1.0;
    if (hist && k >= 0 && k < hist_len) hist[k] = sqrt(a);
}

// x += alpha p; r -= alpha Ap; partial sums of r.r.  x is FP64; r, p, Ap in T.
template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_update_xr(double *__restrict__ x, T *__restrict__ r,
                                                           const T *__restrict__ p, const T *__restrict__ Ap,
                                                           const double *__restrict__ sc, int64_t n,
                                                           double *__restrict__ partial)
{
    __shared__ double sh[kRedThreads];
    const double al = sc[kScAlpha];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads) {
        x[i] += al * (double)p[i];
        const T ri = (T)((double)r[i] - al * (double)Ap[i]);
        r[i] = ri;
        s += (double)ri * (double)ri;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// x += alpha p; r -= alpha Ap; z = dinv r; partial sums of r.r and r.z.
template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_update_xrz(double *__restrict__ x, T *__restrict__ r,
                                                            const T *__restrict__ p, const T *__restrict__ Ap,
                                                            const T *__restrict__ dinv, T *__restrict__ z,
                                                            const double *__restrict__ sc, int64_t n,
                                                            double *__restrict__ partial)
{
    __shared__ double sh[kRedThreads];
    const double al = sc[kScAlpha];
    double srr = 0.0, srz = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads) {
        x[i] += al * (double)p[i];
        const T ri = (T)((double)r[i] - al * (double)Ap[i]);
        const T zi = (T)((double)dinv[i] * (double)ri);
        r[i] = ri;
        z[i] = zi;
        srr += (double)ri * (double)ri;
        srz += (double)ri * (double)zi;
    }
    srr = block_sum(srr, sh);
    __syncthreads();
    srz = block_sum(srz, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = srr;
        partial[kRedBlocks + blockIdx.x] = srz;
    }
}

// z = dinv r; partial sums of r.z.
template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_precond(const T *__restrict__ r, const T *__restrict__ dinv,
                                                         T *__restrict__ z, int64_t n, double *__restrict__ partial)
{
    __shared__ double sh[kRedThreads];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads) {
        const T zi = (T)((double)dinv[i] * (double)r[i]);
        z[i] = zi;
        s += (double)r[i] * (double)zi;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void k_jacobi_inverse(const double *__restrict__ d, double *__restrict__ dinv64, float *__restrict__ dinv32,
                                 int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads) {
        const double v = d[i] > 0.0 ? 1.0 / d[i] : 0.0;
        dinv64[i] = v;
        if (dinv32) dinv32[i] = (float)v;
    }
}

template <typename T>
__global__ void k_update_p(const T *__restrict__ r, T *__restrict__ p, const double *__restrict__ sc, int64_t n)
{
    const double be = sc[kScBeta];
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads)
        p[i] = (T)((double)r[i] + be * (double)p[i]);
}

// r = b - Ax (Ax may be null: r = b) into r64 and/or r32; partial sums of r.r (FP64 r).
__global__ void __launch_bounds__(kRedThreads) k_residual(const double *__restrict__ b, const double *__restrict__ Ax,
                                                          double *__restrict__ r64, float *__restrict__ r32, int64_t n,
                                                          double *__restrict__ partial)
{
    __shared__ double sh[kRedThreads];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads) {
        const double ri = Ax ? b[i] - Ax[i] : b[i];
        if (r64) r64[i] = ri;
        if (r32) r32[i] = (float)ri;
        s += ri * ri;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename TS, typename TD>
__global__ void k_copy(const TS *__restrict__ s, TD *__restrict__ d, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads)
        d[i] = (TD)s[i];
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Zero fill as a kernel rather than a runtime memset, so that the asynchronous entry points stay
// safe to record into a graph.
// 16-byte stores for the bulk, then the last (bytes mod 16) / 4 words
__global__ void k_zero16(uint4 *__restrict__ p, int64_t n, uint32_t *__restrict__ tail, int ntail)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t i = t; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = make_uint4(0u, 0u, 0u, 0u);
    if (t < ntail) tail[t] = 0u;
}

__global__ void k_zero4(uint32_t *__restrict__ p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k_fill_uniform(double *__restrict__ x, int64_t n, uint64_t seed)
{
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads) {
        const uint64_t z = splitmix64(seed * 0x632be59bd9b4e019ull + (uint64_t)i);
        x[i] = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
    }
}

template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_maxdiff(const T *__restrict__ a, const T *__restrict__ b, int64_t n,
                                                         double *__restrict__ partial)
{
    __shared__ double sh[kRedThreads];
    double d = 0.0, m = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads) {
        const double ai = a[i], bi = b[i];
        d = fmax(d, fabs(ai - bi));
        m = fmax(m, fabs(bi));
        if (ai != ai) d = INFINITY;
    }
    d = block_max(d, sh);
    __syncthreads();
    m = block_max(m, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = d;
        partial[kRedBlocks + blockIdx.x] = m;
    }
}

__global__ void __launch_bounds__(kRedThreads) k_maxfinal(const double *__restrict__ partial, double *__restrict__ out2)
{
    __shared__ double sh[kRedThreads];
    double d = 0.0, m = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) {
        d = fmax(d, partial[i]);
        m = fmax(m, partial[kRedBlocks + i]);
    }
    d = block_max(d, sh);
    __syncthreads();
    m = block_max(m, sh);
    if (threadIdx.x == 0) {
        out2[0] = d;
        out2[1] = m;
    }
}

}  // namespace

#define GRID dim3(kRedBlocks), dim3(kRedThreads), 0, s

hipError_t launch_dot(const void *a, int pa, const void *b, int pb, int64_t n, double *partial, hipStream_t s)
{
    if (pa == MFHEX_F64 && pb == MFHEX_F64)
        hipLaunchKernelGGL((k_dot<double, double>), GRID, (const double *)a, (const double *)b, n, partial);
    else if (pa == MFHEX_F32 && pb == MFHEX_F32)
        hipLaunchKernelGGL((k_dot<float, float>), GRID, (const float *)a, (const float *)b, n, partial);
    else if (pa == MFHEX_F64)
        hipLaunchKernelGGL((k_dot<double, float>), GRID, (const double *)a, (const float *)b, n, partial);
    else
        hipLaunchKernelGGL((k_dot<float, double>), GRID, (const float *)a, (const double *)b, n, partial);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partial, double *sc, int op, int k, double *hist, int hist_len,
                           hipStream_t s)
{
    if (op == kFinBetaPre)
        hipLaunchKernelGGL(k_finalize_beta_pre, dim3(1), dim3(kRedThreads), 0, s, partial, sc, k, hist, hist_len);
    else
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedThreads), 0, s, partial, sc, op, k, hist, hist_len);
    return hipGetLastError();
}

hipError_t launch_update_xrz(double *x, void *r, const void *p, const void *Ap, const void *dinv, void *z, int prec,
                             const double *sc, int64_t n, double *partial, hipStream_t s)
{
    if (prec == MFHEX_F64)
        hipLaunchKernelGGL(k_update_xrz<double>, GRID, x, (double *)r, (const double *)p, (const double *)Ap,
                           (const double *)dinv, (double *)z, sc, n, partial);
    else
        hipLaunchKernelGGL(k_update_xrz<float>, GRID, x, (float *)r, (const float *)p, (const float *)Ap,
                           (const float *)dinv, (float *)z, sc, n, partial);
    return hipGetLastError();
}

hipError_t launch_precond(const void *r, const void *dinv, void *z, int prec, int64_t n, double *partial,
                          hipStream_t s)
{
    if (prec == MFHEX_F64)
        hipLaunchKernelGGL(k_precond<double>, GRID, (const double *)r, (const double *)dinv, (double *)z, n, partial);
    else
        hipLaunchKernelGGL(k_precond<float>, GRID, (const float *)r, (const float *)dinv, (float *)z, n, partial);
    return hipGetLastError();
}

hipError_t launch_jacobi_inverse(const double *d, double *dinv64, float *dinv32, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_jacobi_inverse, GRID, d, dinv64, dinv32, n);
    return hipGetLastError();
}

hipError_t launch_update_xr(double *x, void *r, const void *p, const void *Ap, int prec, const double *sc, int64_t n,
                            double *partial, hipStream_t s)
{
    if (prec == MFHEX_F64)
        hipLaunchKernelGGL(k_update_xr<double>, GRID, x, (double *)r, (const double *)p, (const double *)Ap, sc, n,
                           partial);
    else
        hipLaunchKernelGGL(k_update_xr<float>, GRID, x, (float *)r, (const float *)p, (const float *)Ap, sc, n,
                           partial);
    return hipGetLastError();
}

hipError_t launch_update_p(const void *r, void *p, int prec, const double *sc, int64_t n, hipStream_t s)
{
    if (prec == MFHEX_F64)
        hipLaunchKernelGGL(k_update_p<double>, GRID, (const double *)r, (double *)p, sc, n);
    else
        hipLaunchKernelGGL(k_update_p<float>, GRID, (const float *)r, (float *)p, sc, n);
    return hipGetLastError();
}

hipError_t launch_residual(const double *b, const double *Ax, double *r64, float *r32, int64_t n, double *partial,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_residual, GRID, b, Ax, r64, r32, n, partial);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, int ps, void *dst, int pd, int64_t n, hipStream_t s)
{
    if (ps == MFHEX_F64 && pd == MFHEX_F64)
        hipLaunchKernelGGL((k_copy<double, double>), GRID, (const double *)src, (double *)dst, n);
    else if (ps == MFHEX_F64 && pd == MFHEX_F32)
        hipLaunchKernelGGL((k_copy<double, float>), GRID, (const double *)src, (float *)dst, n);
    else if (ps == MFHEX_F32 && pd == MFHEX_F64)
        hipLaunchKernelGGL((k_copy<float, double>), GRID, (const float *)src, (double *)dst, n);
    else
        hipLaunchKernelGGL((k_copy<float, float>), GRID, (const float *)src, (float *)dst, n);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s)
{
    if (bytes % 4) return hipErrorInvalidValue;
    if (bytes == 0) return hipSuccess;
    const bool wide = (uintptr_t)p % 16 == 0;
    const int64_t n = (int64_t)(wide ? bytes / 16 : bytes / 4);
    const int64_t blocks = n < 256 ? 1 : (n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536;
    if (wide)
        hipLaunchKernelGGL(k_zero16, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<uint4 *>(p), n,
                           reinterpret_cast<uint32_t *>(static_cast<char *>(p) + 16 * n), (int)(bytes % 16 / 4));
    else
        hipLaunchKernelGGL(k_zero4, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<uint32_t *>(p), n);
    return hipGetLastError();
}

hipError_t launch_fill_uniform(double *x, int64_t n, uint64_t seed, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_uniform, GRID, x, n, seed);
    return hipGetLastError();
}

hipError_t launch_relmaxdiff(const void *a, const void *b, int64_t n, int prec, double *partial, double *out2,
                             hipStream_t s)
{
    if (prec == MFHEX_F64)
        hipLaunchKernelGGL(k_maxdiff<double>, GRID, (const double *)a, (const double *)b, n, partial);
    else
        hipLaunchKernelGGL(k_maxdiff<float>, GRID, (const float *)a, (const float *)b, n, partial);
    hipLaunchKernelGGL(k_maxfinal, dim3(1), dim3(kRedThreads), 0, s, partial, out2);
    return hipGetLastError();
}

}  // namespace mfhex
