// Fused matrix-free operator kernels for gfx950, templated on the 1D sizes.
//
// One thread block holds `epb` elements; each element gets Q*Q threads.  The
// element vector never leaves the chip: restriction (gather), the 1D basis
// contractions along x, y, z, the pointwise geometric factors and the
// transposed contractions run back to back in LDS and registers, and the
// result is scatter-added into the output with hardware atomics.  This is
// the operator-level fused form of Sec. 2 (w_L = A_L u_L with A^e = D^T G^e D,
// the tensor derivatives D_r, D_s, D_t and six symmetric factors) with the
// sum factorization of Sec. 1; the fusion of restriction, basis and
// pointwise stages into one kernel follows the discussion of generated fused
// operator kernels in Sec. 3.
//
// Contraction scheme ("pencils"): a 1D contraction along one axis is done by
// threads that each own one full line (pencil) along that axis: the thread
// reads the line from LDS into registers, multiplies by the small 1D matrix
// (uniform across the block, so it sits in scalar registers / the scalar
// cache), and writes the result line back in place.  LDS traffic is one read
// per input and one write per output instead of one read per multiply-add.
// The LDS array of an element is [c][b][a] with a fixed odd row pitch, so
// lines along x (thread stride = pitch), y and z (thread stride 1) are
// bank-conflict free, and every contraction can run in place.
//
// Diffusion with Gauss points (q = p+2): values are interpolated to the
// points along x, y, z (B), the reference gradient is taken with the
// collocated derivative on the points (D, q x q), the 3x3 symmetric factors
// are applied, and the transposes run in reverse order.  With Gauss-Lobatto
// points collocated at the nodes (q = p+1) B is the identity and only D
// remains.  Mass: interpolate, scale by w detJ, interpolate back.
#pragma once

#include "mfhex_internal.h"

namespace mfhex {

template <int Q>
struct Lds {
    static constexpr int PITCH = lds_pitch(Q);
    static constexpr int PLANE = PITCH * Q;
    static constexpr int BUF = lds_buf(Q);
};

// 1D matrices passed by value as a kernel argument (constant, uniform).
template <int P, int Q, typename T>
struct BasisArg {
    T B[Q * P];  // B[a*P + i]: node i -> point a
    T D[Q * Q];  // D[a*Q + b]: derivative at point a of the point-b Lagrange polynomial
};

// Blocks are dealt to the 8 XCDs round-robin; renumber them so that each XCD
// works on one contiguous range of elements (neighbouring elements share
// nodes, so their gathers and scatter-adds stay in that XCD's L2).
__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t nb)
{
    const int64_t x = bid % kNumXcd, i = bid / kNumXcd;
    const int64_t q = nb / kNumXcd, r = nb % kNumXcd;
    return x * q + (x < r ? x : r) + i;
}

// Contraction along x (axis 0) of lines (i1, i2), i1 < N1, i2 < N2:
// dst[o] = sum_i M(o, i) src[i]; M(o,i) = M[o*LDM + i], or M[i*LDM + o] when TR.
template <int NI, int NO, int N1, int N2, bool TR, int LDM, int Q, typename T>
__device__ __forceinline__ void pencil_x(const T *src, T *dst, const T *__restrict__ M, int lt)
{
    using L = Lds<Q>;
    if (lt < N1 * N2) {
        const int i1 = lt % N1, i2 = lt / N1;
        const int base = L::PITCH * i1 + L::PLANE * i2;
        T v[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) v[i] = src[base + i];
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            T acc = T(0);
#pragma unroll
            for (int i = 0; i < NI; ++i) acc += (TR ? M[i * LDM + o] : M[o * LDM + i]) * v[i];
            dst[base + o] = acc;
        }
    }
}

// Contraction along y (axis 1) of lines (i0, i2), i0 < N0, i2 < N2.
template <int NI, int NO, int N0, int N2, bool TR, int LDM, int Q, typename T>
__device__ __forceinline__ void pencil_y(const T *src, T *dst, const T *__restrict__ M, int lt)
{
    using L = Lds<Q>;
    if (lt < N0 * N2) {
        const int i0 = lt % N0, i2 = lt / N0;
        const int base = i0 + L::PLANE * i2;
        T v[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) v[i] = src[base + L::PITCH * i];
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            T acc = T(0);
#pragma unroll
            for (int i = 0; i < NI; ++i) acc += (TR ? M[i * LDM + o] : M[o * LDM + i]) * v[i];
            dst[base + L::PITCH * o] = acc;
        }
    }
}

// Restriction: element values into s0[k][j][i] (zero at masked nodes).
template <int P, int Q, int NOFF, typename T>
__device__ __forceinline__ void gather(T *s0, const int32_t (&off)[NOFF], const T *__restrict__ x, int nvec,
                                       int v, int lt)
{
    using L = Lds<Q>;
    constexpr int Q2 = Q * Q, P3 = P * P * P;
#pragma unroll
    for (int r = 0; r < NOFF; ++r) {
        const int t = lt + r * Q2;
        if (t < P3) {
            const int i = t % P, j = (t / P) % P, k = t / (P * P);
            const int32_t o = off[r];
            s0[i + L::PITCH * j + L::PLANE * k] = o >= 0 ? x[(int64_t)o * nvec + v] : T(0);
        }
    }
}

// Transposed restriction: y[node] += s0[k][j][i] for unmasked nodes.
template <int P, int Q, int NOFF, typename T>
__device__ __forceinline__ void scatter_add(const T *s0, const int32_t (&off)[NOFF], T *__restrict__ y, int nvec,
                                            int v, int lt)
{
    using L = Lds<Q>;
    constexpr int Q2 = Q * Q, P3 = P * P * P;
#pragma unroll
    for (int r = 0; r < NOFF; ++r) {
        const int t = lt + r * Q2;
        if (t < P3 && off[r] >= 0) {
            const int i = t % P, j = (t / P) % P, k = t / (P * P);
            unsafeAtomicAdd(&y[(int64_t)off[r] * nvec + v], s0[i + L::PITCH * j + L::PLANE * k]);
        }
    }
}

// Gathered element in s0 -> values at the points of column (a, b) in col[].
// For Gauss points the x and y interpolations run as pencils through LDS and
// the z interpolation in registers.  Ends without a trailing barrier.
template <int P, int Q, bool COLLOC, typename T>
__device__ __forceinline__ void interp_to_column(T *s0, const BasisArg<P, Q, T> &bas, int lt, int a, int b,
                                                 T (&col)[Q])
{
    using L = Lds<Q>;
    if constexpr (!COLLOC) {
        pencil_x<P, Q, P, P, false, P, Q>(s0, s0, bas.B, lt);
        __syncthreads();
        pencil_y<P, Q, Q, P, false, P, Q>(s0, s0, bas.B, lt);
        __syncthreads();
        T in[P];
#pragma unroll
        for (int k = 0; k < P; ++k) in[k] = s0[a + L::PITCH * b + L::PLANE * k];
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            T acc = T(0);
#pragma unroll
            for (int k = 0; k < P; ++k) acc += bas.B[c * P + k] * in[k];
            col[c] = acc;
        }
    } else {
#pragma unroll
        for (int c = 0; c < Q; ++c) col[c] = s0[a + L::PITCH * b + L::PLANE * c];
    }
}

// Column (a, b) of point values -> transposed interpolation back to the
// element's nodes, left in s0[k][j][i].  Ends with a barrier.
template <int P, int Q, bool COLLOC, typename T>
__device__ __forceinline__ void column_to_nodes(T *s0, const BasisArg<P, Q, T> &bas, int lt, int a, int b,
                                                const T (&col)[Q])
{
    using L = Lds<Q>;
    if constexpr (!COLLOC) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            T acc = T(0);
#pragma unroll
            for (int c = 0; c < Q; ++c) acc += bas.B[c * P + k] * col[c];
            s0[a + L::PITCH * b + L::PLANE * k] = acc;
        }
        __syncthreads();
        pencil_y<Q, P, Q, P, true, P, Q>(s0, s0, bas.B, lt);
        __syncthreads();
        pencil_x<Q, P, P, P, true, P, Q>(s0, s0, bas.B, lt);
        __syncthreads();
    } else {
#pragma unroll
        for (int c = 0; c < Q; ++c) s0[a + L::PITCH * b + L::PLANE * c] = col[c];
        __syncthreads();
    }
}

// Gathered element in s0 -> reference gradient at every point: d/dr in s1,
// d/ds in s2 (both [c][b][a]), d/dt of column (a, b) in dz[].  Ends with a
// barrier.  s0 then holds the point values.
template <int P, int Q, bool COLLOC, typename T>
__device__ __forceinline__ void gradient(T *s0, T *s1, T *s2, const BasisArg<P, Q, T> &bas, int lt, int a, int b,
                                         T (&dz)[Q])
{
    using L = Lds<Q>;
    T col[Q];
    interp_to_column<P, Q, COLLOC, T>(s0, bas, lt, a, b, col);
#pragma unroll
    for (int c = 0; c < Q; ++c) {
        T acc = T(0);
#pragma unroll
        for (int d = 0; d < Q; ++d) acc += bas.D[c * Q + d] * col[d];
        dz[c] = acc;
    }
    if constexpr (!COLLOC) {
#pragma unroll
        for (int c = 0; c < Q; ++c) s0[a + L::PITCH * b + L::PLANE * c] = col[c];
        __syncthreads();
    }
    pencil_x<Q, Q, Q, Q, false, Q, Q>(s0, s1, bas.D, lt);
    pencil_y<Q, Q, Q, Q, false, Q, Q>(s0, s2, bas.D, lt);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// y += A x  (mass / diffusion), or y += B^T (w detJ f) for the load vector.
// ---------------------------------------------------------------------------
template <int P, int Q, bool COLLOC, int MODE, bool VARK, typename T>
__global__ void __launch_bounds__(kMaxThreads)
k_apply(const BasisArg<P, Q, T> bas, const int64_t nelem, const int nvec, const int32_t *__restrict__ offsets,
        const T *__restrict__ qdata, const double *__restrict__ kappa, const double *__restrict__ wdet,
        const T *__restrict__ x, T *__restrict__ y)
{
    constexpr int Q2 = Q * Q, Q3 = Q2 * Q, P3 = P * P * P;
    constexpr int NOFF = (P3 + Q2 - 1) / Q2;
    constexpr int NBUF = apply_nbuf(MODE);
    using L = Lds<Q>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *const sm = reinterpret_cast<T *>(smem_raw);
    const int epb = blockDim.x / Q2;
    const int el = threadIdx.x / Q2, lt = threadIdx.x - el * Q2;
    T *const s0 = sm + (size_t)el * NBUF * L::BUF;
    T *const s1 = s0 + L::BUF;
    T *const s2 = s1 + L::BUF;
    const int64_t e = xcd_block(blockIdx.x, gridDim.x) * epb + el;
    const bool valid = e < nelem;
    const int a = lt % Q, b = lt / Q;

    int32_t off[NOFF];
#pragma unroll
    for (int r = 0; r < NOFF; ++r) {
        const int t = lt + r * Q2;
        off[r] = (valid && t < P3) ? offsets[e * P3 + t] : -1;
    }

    for (int v = 0; v < nvec; ++v) {
        T col[Q];
        if constexpr (MODE == kRhs) {
            const double *f = reinterpret_cast<const double *>(x);
#pragma unroll
            for (int c = 0; c < Q; ++c) {
                const int64_t pt = e * Q3 + a + Q * b + Q2 * c;
                col[c] = valid ? T(wdet[pt] * f[pt]) : T(0);
            }
        } else if constexpr (MODE == kMass) {
            gather<P, Q, NOFF, T>(s0, off, x, nvec, v, lt);
            __syncthreads();
            interp_to_column<P, Q, COLLOC, T>(s0, bas, lt, a, b, col);
            const T *qd = qdata + e * Q3;
#pragma unroll
            for (int c = 0; c < Q; ++c) {
                const int pt = a + Q * b + Q2 * c;
                const T w = valid ? __builtin_nontemporal_load(&qd[pt]) : T(0);
                col[c] *= w;
            }
        } else {  // diffusion
            gather<P, Q, NOFF, T>(s0, off, x, nvec, v, lt);
            __syncthreads();
            T dz[Q];
            gradient<P, Q, COLLOC, T>(s0, s1, s2, bas, lt, a, b, dz);
            // The point values in s0 are no longer needed: park d/dt there so
            // the pointwise loop below carries no register arrays.
#pragma unroll
            for (int c = 0; c < Q; ++c) s0[a + L::PITCH * b + L::PLANE * c] = dz[c];
            const T *qd = qdata + e * (kQdDiff * Q3);
#pragma unroll 2
            for (int c = 0; c < Q; ++c) {
                const int pt = a + Q * b + Q2 * c;
                const int ls = a + L::PITCH * b + L::PLANE * c;
                T g[kQdDiff];
#pragma unroll
                for (int m = 0; m < kQdDiff; ++m) g[m] = valid ? __builtin_nontemporal_load(&qd[m * Q3 + pt]) : T(0);
                if constexpr (VARK) {
                    const T kap = valid ? T(kappa[e * Q3 + pt]) : T(0);
#pragma unroll
                    for (int m = 0; m < kQdDiff; ++m) g[m] *= kap;
                }
                const T ur = s1[ls], us = s2[ls], ut = s0[ls];
                s1[ls] = g[0] * ur + g[5] * us + g[4] * ut;
                s2[ls] = g[5] * ur + g[1] * us + g[3] * ut;
                s0[ls] = g[4] * ur + g[3] * us + g[2] * ut;
            }
            // transposed t-derivative of the own column (no barrier needed)
#pragma unroll
            for (int c = 0; c < Q; ++c) dz[c] = s0[a + L::PITCH * b + L::PLANE * c];
#pragma unroll
            for (int c = 0; c < Q; ++c) {
                T acc = T(0);
#pragma unroll
                for (int d = 0; d < Q; ++d) acc += bas.D[d * Q + c] * dz[d];
                col[c] = acc;
            }
            __syncthreads();
            pencil_x<Q, Q, Q, Q, true, Q, Q>(s1, s1, bas.D, lt);
            pencil_y<Q, Q, Q, Q, true, Q, Q>(s2, s2, bas.D, lt);
            __syncthreads();
#pragma unroll
            for (int c = 0; c < Q; ++c) {
                const int ls = a + L::PITCH * b + L::PLANE * c;
                col[c] += s1[ls] + s2[ls];
            }
        }
        column_to_nodes<P, Q, COLLOC, T>(s0, bas, lt, a, b, col);
        if (valid) scatter_add<P, Q, NOFF, T>(s0, off, y, nvec, v, lt);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Coefficient gradient g[e][pt] = (Dhat r)^T G0 (Dhat u) at every point.
// ---------------------------------------------------------------------------
template <int P, int Q, bool COLLOC>
__global__ void __launch_bounds__(kMaxThreads)
k_kgrad(const BasisArg<P, Q, double> bas, const int64_t nelem, const int32_t *__restrict__ offsets,
        const double *__restrict__ qdata, const double *__restrict__ u, const double *__restrict__ r,
        double *__restrict__ g)
{
    using T = double;
    constexpr int Q2 = Q * Q, Q3 = Q2 * Q, P3 = P * P * P;
    constexpr int NOFF = (P3 + Q2 - 1) / Q2;
    using L = Lds<Q>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *const sm = reinterpret_cast<T *>(smem_raw);
    const int epb = blockDim.x / Q2;
    const int el = threadIdx.x / Q2, lt = threadIdx.x - el * Q2;
    T *const s0 = sm + (size_t)el * 3 * L::BUF;
    T *const s1 = s0 + L::BUF;
    T *const s2 = s1 + L::BUF;
    const int64_t e = xcd_block(blockIdx.x, gridDim.x) * epb + el;
    const bool valid = e < nelem;
    const int a = lt % Q, b = lt / Q;

    int32_t off[NOFF];
#pragma unroll
    for (int rr = 0; rr < NOFF; ++rr) {
        const int t = lt + rr * Q2;
        off[rr] = (valid && t < P3) ? offsets[e * P3 + t] : -1;
    }
    T ur[Q], us[Q], ut[Q];
    gather<P, Q, NOFF, T>(s0, off, u, 1, 0, lt);
    __syncthreads();
    gradient<P, Q, COLLOC, T>(s0, s1, s2, bas, lt, a, b, ut);
#pragma unroll
    for (int c = 0; c < Q; ++c) {
        const int ls = a + L::PITCH * b + L::PLANE * c;
        ur[c] = s1[ls];
        us[c] = s2[ls];
    }
    __syncthreads();
    T rt[Q];
    gather<P, Q, NOFF, T>(s0, off, r, 1, 0, lt);
    __syncthreads();
    gradient<P, Q, COLLOC, T>(s0, s1, s2, bas, lt, a, b, rt);
    if (!valid) return;  // no barrier follows
    const T *qd = qdata + e * (kQdDiff * Q3);
#pragma unroll
    for (int c = 0; c < Q; ++c) {
        const int pt = a + Q * b + Q2 * c;
        const int ls = a + L::PITCH * b + L::PLANE * c;
        T gm[kQdDiff];
#pragma unroll
        for (int m = 0; m < kQdDiff; ++m) gm[m] = __builtin_nontemporal_load(&qd[m * Q3 + pt]);
        const T vr = gm[0] * ur[c] + gm[5] * us[c] + gm[4] * ut[c];
        const T vs = gm[5] * ur[c] + gm[1] * us[c] + gm[3] * ut[c];
        const T vt = gm[4] * ur[c] + gm[3] * us[c] + gm[2] * ut[c];
        __builtin_nontemporal_store(s1[ls] * vr + s2[ls] * vs + rt[c] * vt, &g[e * Q3 + pt]);
    }
}

// ---------------------------------------------------------------------------
// Host launchers for one (P, Q) pair.
// ---------------------------------------------------------------------------
template <int P, int Q, typename T>
static BasisArg<P, Q, T> make_basis_arg(const Basis1D &b)
{
    BasisArg<P, Q, T> o;
    for (int i = 0; i < Q * P; ++i) o.B[i] = T(b.B[i]);
    for (int i = 0; i < Q * Q; ++i) o.D[i] = T(b.D[i]);
    return o;
}

template <typename K>
static hipError_t prepare_lds(K kernel, size_t lds)
{
    if (lds > 65536) return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return hipSuccess;
}

template <int P, int Q, bool COLLOC, int MODE, bool VARK, typename T>
static hipError_t launch_apply_t(const ApplyLaunch &a)
{
    const auto bas = make_basis_arg<P, Q, T>(*a.basis);
    const int64_t nblk = (a.v.nelem + a.epb - 1) / a.epb;
    const size_t lds = (size_t)a.epb * apply_nbuf(MODE) * Lds<Q>::BUF * sizeof(T);
    auto kern = k_apply<P, Q, COLLOC, MODE, VARK, T>;
    hipError_t err = prepare_lds(kern, lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(a.epb * Q * Q), lds, a.stream, bas, a.v.nelem, a.nvec,
                       a.v.offsets, static_cast<const T *>(a.v.qdata), a.v.kappa, a.wdet,
                       static_cast<const T *>(a.x), static_cast<T *>(a.y));
    return hipGetLastError();
}

template <int P, int Q, bool COLLOC>
static hipError_t launch_apply_pq(const ApplyLaunch &a)
{
    if (a.mode == kRhs) return launch_apply_t<P, Q, COLLOC, kRhs, false, double>(a);
    if (a.prec == MFHEX_F32) {
        if (a.mode == kMass) return launch_apply_t<P, Q, COLLOC, kMass, false, float>(a);
        return launch_apply_t<P, Q, COLLOC, kDiff, false, float>(a);
    }
    if (a.mode == kMass) return launch_apply_t<P, Q, COLLOC, kMass, false, double>(a);
    if (a.vark) return launch_apply_t<P, Q, COLLOC, kDiff, true, double>(a);
    return launch_apply_t<P, Q, COLLOC, kDiff, false, double>(a);
}

template <int P, int Q, bool COLLOC>
static hipError_t launch_kgrad_pq(const KgradLaunch &a)
{
    const auto bas = make_basis_arg<P, Q, double>(*a.basis);
    const int64_t nblk = (a.v.nelem + a.epb - 1) / a.epb;
    const size_t lds = (size_t)a.epb * 3 * Lds<Q>::BUF * sizeof(double);
    auto kern = k_kgrad<P, Q, COLLOC>;
    hipError_t err = prepare_lds(kern, lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(a.epb * Q * Q), lds, a.stream, bas, a.v.nelem,
                       a.v.offsets, static_cast<const double *>(a.v.qdata), a.u, a.r, a.g);
    return hipGetLastError();
}

}  // namespace mfhex

// Instantiate the launchers of order N (P = N+1): Gauss q = N+2, Lobatto q = N+1.
#define MFHEX_DEFINE_ORDER(N)                                                                          \
    namespace mfhex {                                                                                  \
    hipError_t launch_apply_p##N(const ApplyLaunch &a)                                                 \
    {                                                                                                  \
        if (a.basis->colloc) return launch_apply_pq<N + 1, N + 1, true>(a);                            \
        return launch_apply_pq<N + 1, N + 2, false>(a);                                                \
    }                                                                                                  \
    hipError_t launch_kgrad_p##N(const KgradLaunch &a)                                                 \
    {                                                                                                  \
        if (a.basis->colloc) return launch_kgrad_pq<N + 1, N + 1, true>(a);                            \
        return launch_kgrad_pq<N + 1, N + 2, false>(a);                                                \
    }                                                                                                  \
    }
