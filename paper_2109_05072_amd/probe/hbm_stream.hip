// Streaming kernels that measure the HBM bandwidth the operator kernels can
// hope for on this GPU: a read-only sweep (sum of every element), a copy and a
// fill, each with 16-byte accesses, several loads in flight per lane and an
// optional non-temporal form.  The caller times them with events on `stream`.
// Built as its own small library (libhbmprobe.so), apart from the operator
// library: it is a measuring instrument, not part of the operator.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace {

// two doubles as a native vector type (the non-temporal builtins take those, not HIP's dbl2 struct)
typedef double dbl2 __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;
constexpr int kUnroll = 4;  // 16-byte loads in flight per lane

template <bool NT>
__device__ __forceinline__ dbl2 ld(const dbl2 *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool NT>
__device__ __forceinline__ void st(dbl2 *p, dbl2 v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// partial[blockIdx.x] = sum of the block's share of src[0..n).
template <bool NT>
__global__ void __launch_bounds__(kThreads) k_read(const double *__restrict__ src, int64_t n, double *__restrict__ partial)
{
    const dbl2 *s2 = reinterpret_cast<const dbl2 *>(src);
    const int64_t n2 = n / 2;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    double acc = 0.0;
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < n2; i += kUnroll * stride) {
        dbl2 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = ld<NT>(s2 + i + u * stride);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc += v[u].x + v[u].y;
    }
    for (; i < n2; i += stride) {
        const dbl2 v = ld<NT>(s2 + i);
        acc += v.x + v.y;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) acc += src[n - 1];
    __shared__ double sh[kThreads];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w /= 2) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

template <bool NT>
__global__ void __launch_bounds__(kThreads) k_copy(const double *__restrict__ src, double *__restrict__ dst, int64_t n)
{
    const dbl2 *s2 = reinterpret_cast<const dbl2 *>(src);
    dbl2 *d2 = reinterpret_cast<dbl2 *>(dst);
    const int64_t n2 = n / 2;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < n2; i += kUnroll * stride) {
        dbl2 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = ld<NT>(s2 + i + u * stride);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) st<NT>(d2 + i + u * stride, v[u]);
    }
    for (; i < n2; i += stride) st<NT>(d2 + i, ld<NT>(s2 + i));
    if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) dst[n - 1] = src[n - 1];
}

template <bool NT>
__global__ void __launch_bounds__(kThreads) k_fill(double *__restrict__ dst, int64_t n, double v)
{
    dbl2 *d2 = reinterpret_cast<dbl2 *>(dst);
    const int64_t n2 = n / 2;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    const dbl2 w = {v, v};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n2; i += stride) st<NT>(d2 + i, w);
    if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) dst[n - 1] = v;
}

}  // namespace

extern "C" {

// kind: 0 read (partial[nblocks] receives block sums), 1 copy src -> dst, 2 fill dst with 1.0.
// nontemporal: 1 uses non-temporal loads and stores.  Pointers 16-byte aligned, n elements
// (FP64).  Returns the hipError_t of the launch.
int hbm_stream(int kind, int nontemporal, const double *src, double *dst, int64_t n, double *partial, int nblocks,
               void *stream)
{
    if (n <= 0 || nblocks <= 0 || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return (int)hipErrorInvalidValue;
    if ((kind == 0 && (!src || !partial)) || (kind == 1 && (!src || !dst)) || (kind == 2 && !dst) || kind < 0 ||
        kind > 2)
        return (int)hipErrorInvalidValue;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 g((unsigned)nblocks), b(kThreads);
    if (kind == 0) {
        if (nontemporal) hipLaunchKernelGGL(k_read<true>, g, b, 0, s, src, n, partial);
        else hipLaunchKernelGGL(k_read<false>, g, b, 0, s, src, n, partial);
    } else if (kind == 1) {
        if (nontemporal) hipLaunchKernelGGL(k_copy<true>, g, b, 0, s, src, dst, n);
        else hipLaunchKernelGGL(k_copy<false>, g, b, 0, s, src, dst, n);
    } else {
        if (nontemporal) hipLaunchKernelGGL(k_fill<true>, g, b, 0, s, dst, n, 1.0);
        else hipLaunchKernelGGL(k_fill<false>, g, b, 0, s, dst, n, 1.0);
    }
    return (int)hipGetLastError();
}

}  // extern "C"
