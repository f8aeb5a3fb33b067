// p-multigrid transfer and smoother kernels.
//
// Prolongation P maps a coarse field to its values at the fine nodes: in
// every element the coarse nodal values are interpolated to the fine
// Gauss-Lobatto nodes by the tensor product of the 1D interpolation matrix
// I1 [P_f][P_c] (three 1D contractions, sum factorization as in Sec. 1).  A
// fine node shared by m elements receives the same value from each of them,
// so every element adds it with weight 1/m: the sum is exactly P x_c.  The
// restriction adds I1^T (w r_f) per element with the same weights w = 1/m,
// which is exactly P^T r_f.  m is known from the node's position on the
// structured mesh (2 per direction in which it lies on a face between two
// elements).  Masked (Dirichlet) nodes are skipped on both levels.
#include "blas.h"
#include "mg.h"

namespace mfhex {

namespace {

constexpr int kTransferThreads = 128;

// Weight 1/m of local node (i, j, k) of element (ex, ey, ez) with P nodes per direction.
__device__ __forceinline__ double share_weight(int i, int j, int k, int P, int ex, int ey, int ez, int nex, int ney,
                                               int nez)
{
    const int mx = ((i == 0 && ex > 0) || (i == P - 1 && ex < nex - 1)) ? 2 : 1;
    const int my = ((j == 0 && ey > 0) || (j == P - 1 && ey < ney - 1)) ? 2 : 1;
    const int mz = ((k == 0 && ez > 0) || (k == P - 1 && ez < nez - 1)) ? 2 : 1;
    return 1.0 / (mx * my * mz);
}

template <int PF, int PC, int DIR, typename T>
__global__ void __launch_bounds__(kTransferThreads)
k_transfer(int nex, int ney, int nez, const int32_t *__restrict__ off_f, const int32_t *__restrict__ off_c,
           const T *__restrict__ I1, const T *__restrict__ src, T *__restrict__ dst)
{
    constexpr int NT = kTransferThreads;
    constexpr int F3 = PF * PF * PF, C3 = PC * PC * PC;
    // DIR 0 (prolong): a = coarse [k][j][i] -> b [k][j][I] -> c [k][J][I] -> fine [K][J][I]
    // DIR 1 (restrict): a = fine [K][J][I] -> b [K][J][i] -> c [K][j][i] -> coarse [k][j][i]
    constexpr int NA = DIR == 0 ? C3 : F3;
    constexpr int NB = DIR == 0 ? PC * PC * PF : PF * PF * PC;
    constexpr int NC = DIR == 0 ? PC * PF * PF : PF * PC * PC;
    __shared__ T sI[PF * PC], sa[NA], sb[NB], sc[NC];
    const int tid = threadIdx.x;
    const int64_t e = blockIdx.x;
    const int ex = (int)(e % nex), ey = (int)((e / nex) % ney), ez = (int)(e / ((int64_t)nex * ney));
    for (int t = tid; t < PF * PC; t += NT) sI[t] = I1[t];
    if constexpr (DIR == 0) {
        for (int t = tid; t < C3; t += NT) {
            const int32_t o = off_c[e * C3 + t];
            sa[t] = o >= 0 ? src[o] : T(0);
        }
    } else {
        for (int t = tid; t < F3; t += NT) {
            const int32_t o = off_f[e * F3 + t];
            const int i = t % PF, j = (t / PF) % PF, k = t / (PF * PF);
            sa[t] = o >= 0 ? T(share_weight(i, j, k, PF, ex, ey, ez, nex, ney, nez)) * src[o] : T(0);
        }
    }
    __syncthreads();
    // x: DIR 0: b[k][j][I] = sum_i I[I][i] a[k][j][i];  DIR 1: b[K][J][i] = sum_I I[I][i] a[K][J][I]
    constexpr int NIX = DIR == 0 ? PC : PF, NOX = DIR == 0 ? PF : PC;
    for (int t = tid; t < NB; t += NT) {
        const int o = t % NOX, rest = t / NOX;
        T s = T(0);
        for (int i = 0; i < NIX; ++i)
            s += (DIR == 0 ? sI[o * PC + i] : sI[i * PC + o]) * sa[i + NIX * rest];
        sb[t] = s;
    }
    __syncthreads();
    // y: contract the middle index
    constexpr int NX = NOX;                     // extent of the (already contracted) fastest index
    constexpr int NIY = DIR == 0 ? PC : PF, NOY = DIR == 0 ? PF : PC;
    for (int t = tid; t < NC; t += NT) {
        const int a = t % NX, o = (t / NX) % NOY, z = t / (NX * NOY);
        T s = T(0);
        for (int j = 0; j < NIY; ++j)
            s += (DIR == 0 ? sI[o * PC + j] : sI[j * PC + o]) * sb[a + NX * (j + NIY * z)];
        sc[t] = s;
    }
    __syncthreads();
    // z: contract the slowest index and add to the destination
    constexpr int NIZ = DIR == 0 ? PC : PF, NOZ = DIR == 0 ? PF : PC, NXY = NX * NOY;
    for (int t = tid; t < NOZ * NXY; t += NT) {
        const int ab = t % NXY, o = t / NXY;
        T s = T(0);
        for (int k = 0; k < NIZ; ++k) s += (DIR == 0 ? sI[o * PC + k] : sI[k * PC + o]) * sc[ab + NXY * k];
        if constexpr (DIR == 0) {
            const int32_t of = off_f[e * F3 + t];
            if (of >= 0) {
                const int i = t % PF, j = (t / PF) % PF, k = t / (PF * PF);
                unsafeAtomicAdd(&dst[of], T(share_weight(i, j, k, PF, ex, ey, ez, nex, ney, nez)) * s);
            }
        } else {
            const int32_t oc = off_c[e * C3 + t];
            if (oc >= 0) unsafeAtomicAdd(&dst[oc], s);
        }
    }
}

template <int PF, int PC, typename T>
hipError_t transfer_t(const TransferLaunch &t)
{
    const int64_t nelem = (int64_t)t.nex * t.ney * t.nez;
    const T *I1 = static_cast<const T *>(t.I1), *src = static_cast<const T *>(t.src);
    T *dst = static_cast<T *>(t.dst);
    if (t.dir == 0)
        hipLaunchKernelGGL((k_transfer<PF, PC, 0, T>), dim3((unsigned)nelem), dim3(kTransferThreads), 0, t.stream,
                           t.nex, t.ney, t.nez, t.off_f, t.off_c, I1, src, dst);
    else
        hipLaunchKernelGGL((k_transfer<PF, PC, 1, T>), dim3((unsigned)nelem), dim3(kTransferThreads), 0, t.stream,
                           t.nex, t.ney, t.nez, t.off_f, t.off_c, I1, src, dst);
    return hipGetLastError();
}

template <int PF, int PC>
hipError_t transfer_pf(const TransferLaunch &t)
{
    return t.prec == MFHEX_F32 ? transfer_t<PF, PC, float>(t) : transfer_t<PF, PC, double>(t);
}

#define GRID dim3(kRedBlocks), dim3(kRedThreads), 0, s

template <typename T>
__global__ void k_cheb_init(const T *__restrict__ b, const T *__restrict__ Ax, const T *__restrict__ dinv,
                            T *__restrict__ x, T *__restrict__ r, T *__restrict__ d, T inv_theta, int zero_x, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads) {
        const T ri = dinv[i] * (Ax ? b[i] - Ax[i] : b[i]);
        r[i] = ri;
        d[i] = ri * inv_theta;
        if (zero_x) x[i] = T(0);
    }
}

template <typename T>
__global__ void k_cheb_step(T *__restrict__ x, T *__restrict__ d, T *__restrict__ r, const T *__restrict__ Ad,
                            const T *__restrict__ dinv, T cd, T cr, int last, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads) {
        const T di = d[i];
        x[i] += di;
        if (!last) {
            const T ri = r[i] - dinv[i] * Ad[i];
            r[i] = ri;
            d[i] = cd * di + cr * ri;
        }
    }
}

template <typename T>
__global__ void k_mg_residual(const T *__restrict__ b, const T *__restrict__ Ax, T *__restrict__ r, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads)
        r[i] = b[i] - Ax[i];
}

__global__ void k_mask_scale(double *__restrict__ v, const double *__restrict__ dinv, double scale, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads)
        v[i] = dinv[i] > 0.0 ? (scale != 0.0 ? v[i] * scale : v[i]) : 0.0;
}

__global__ void k_scale_by(const double *__restrict__ a, const double *__restrict__ dinv, double *__restrict__ out,
                           int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads)
        out[i] = dinv[i] * a[i];
}

__global__ void __launch_bounds__(kRedThreads) k_dot_dinv(const double *__restrict__ v, const double *__restrict__ dinv,
                                                          int64_t n, double *__restrict__ partial)
{
    __shared__ double sh[kRedThreads];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads)
        if (dinv[i] > 0.0) s += v[i] * v[i] / dinv[i];
    sh[threadIdx.x] = s;
    __syncthreads();
#pragma unroll
    for (int st = kRedThreads / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

}  // namespace

hipError_t launch_transfer(const TransferLaunch &t)
{
    // coarse order max(1, pf / 2)
    switch (t.pf) {
    case 2: return t.pc == 1 ? transfer_pf<3, 2>(t) : hipErrorInvalidValue;
    case 3: return t.pc == 1 ? transfer_pf<4, 2>(t) : hipErrorInvalidValue;
    case 4: return t.pc == 2 ? transfer_pf<5, 3>(t) : hipErrorInvalidValue;
    case 5: return t.pc == 2 ? transfer_pf<6, 3>(t) : hipErrorInvalidValue;
    case 6: return t.pc == 3 ? transfer_pf<7, 4>(t) : hipErrorInvalidValue;
    case 7: return t.pc == 3 ? transfer_pf<8, 4>(t) : hipErrorInvalidValue;
    case 8: return t.pc == 4 ? transfer_pf<9, 5>(t) : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cheb_init(const void *b, const void *Ax, const void *dinv, void *x, void *r, void *d,
                            double inv_theta, bool zero_x, int prec, int64_t n, hipStream_t s)
{
    if (prec == MFHEX_F32)
        hipLaunchKernelGGL(k_cheb_init<float>, GRID, (const float *)b, (const float *)Ax, (const float *)dinv,
                           (float *)x, (float *)r, (float *)d, (float)inv_theta, zero_x ? 1 : 0, n);
    else
        hipLaunchKernelGGL(k_cheb_init<double>, GRID, (const double *)b, (const double *)Ax, (const double *)dinv,
                           (double *)x, (double *)r, (double *)d, inv_theta, zero_x ? 1 : 0, n);
    return hipGetLastError();
}

hipError_t launch_cheb_step(void *x, void *d, void *r, const void *Ad, const void *dinv, double cd, double cr,
                            bool last, int prec, int64_t n, hipStream_t s)
{
    if (prec == MFHEX_F32)
        hipLaunchKernelGGL(k_cheb_step<float>, GRID, (float *)x, (float *)d, (float *)r, (const float *)Ad,
                           (const float *)dinv, (float)cd, (float)cr, last ? 1 : 0, n);
    else
        hipLaunchKernelGGL(k_cheb_step<double>, GRID, (double *)x, (double *)d, (double *)r, (const double *)Ad,
                           (const double *)dinv, cd, cr, last ? 1 : 0, n);
    return hipGetLastError();
}

hipError_t launch_mg_residual(const void *b, const void *Ax, void *r, int prec, int64_t n, hipStream_t s)
{
    if (prec == MFHEX_F32)
        hipLaunchKernelGGL(k_mg_residual<float>, GRID, (const float *)b, (const float *)Ax, (float *)r, n);
    else
        hipLaunchKernelGGL(k_mg_residual<double>, GRID, (const double *)b, (const double *)Ax, (double *)r, n);
    return hipGetLastError();
}

hipError_t launch_mask_scale(double *v, const double *dinv, double scale, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_mask_scale, GRID, v, dinv, scale, n);
    return hipGetLastError();
}

hipError_t launch_scale_by(const double *a, const double *dinv, double *out, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_by, GRID, a, dinv, out, n);
    return hipGetLastError();
}

hipError_t launch_dot_dinv(const double *v, const double *dinv, int64_t n, double *partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_dinv, GRID, v, dinv, n, partial);
    return hipGetLastError();
}

}  // namespace mfhex
