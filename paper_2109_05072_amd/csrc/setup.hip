// Setup kernels: quadrature data (geometric factors) and coordinates.
//
// Stored per point (Sec. 2, the six symmetric geometric factors of
// A^e = D^T G^e D; geometry in geom.hpp):
//   diffusion: G = w adj(J) adj(J)^T / detJ in Voigt order rr, ss, tt, st, rt, rs
//   mass:      w detJ
#include "geom.hpp"

namespace mfhex {

namespace {

struct Rule1D {
    double x[kMaxQ];
    double w[kMaxQ];
};


__global__ void k_qdata(int32_t nex, int32_t ney, int32_t nez, int Q, Rule1D rule, const double *__restrict__ vert,
                        int kind, double *__restrict__ q64, float *__restrict__ q32, double *__restrict__ wdet,
                        int32_t *__restrict__ bad)
{
    const int Q3 = Q * Q * Q;
    const int64_t nelem = (int64_t)nex * ney * nez;
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid >= nelem * Q3) return;
    const int64_t e = gid / Q3;
    const int pt = (int)(gid - e * Q3);
    const int a = pt % Q, b = (pt / Q) % Q, c = pt / (Q * Q);
    Elem8 el;
    load_elem(vert, e, nex, ney, el);
    double jr[3], js[3], jt[3], g[kQdDiff];
    jacobian_cols(el, rule.x[a], rule.x[b], rule.x[c], jr, js, jt);
    const double w = rule.w[a] * rule.w[b] * rule.w[c];
    const double det = diffusion_factors(jr, js, jt, w, g);
    if (!(det > 0.0)) atomicOr(bad, 1);
    if (!q64) {
        // factors evaluated in the apply kernel: only the Jacobian check (and w detJ)
    } else if (kind == MFHEX_DIFFUSION) {
        double *o = q64 + e * (kQdDiff * Q3) + pt;
#pragma unroll
        for (int m = 0; m < kQdDiff; ++m) o[m * Q3] = g[m];
        if (q32) {
            float *o32 = q32 + e * (kQdDiff * Q3) + pt;
#pragma unroll
            for (int m = 0; m < kQdDiff; ++m) o32[m * Q3] = (float)g[m];
        }
    } else {
        q64[e * Q3 + pt] = w * det;
        if (q32) q32[e * Q3 + pt] = (float)(w * det);
    }
    if (wdet) wdet[e * Q3 + pt] = w * det;
}

__global__ void k_qpoint_coords(int32_t nex, int32_t ney, int32_t nez, int Q, Rule1D rule,
                                const double *__restrict__ vert, double *__restrict__ xyz)
{
    const int Q3 = Q * Q * Q;
    const int64_t nelem = (int64_t)nex * ney * nez;
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid >= nelem * Q3) return;
    const int64_t e = gid / Q3;
    const int pt = (int)(gid - e * Q3);
    Elem8 el;
    load_elem(vert, e, nex, ney, el);
    double x[3];
    map_point(el, rule.x[pt % Q], rule.x[(pt / Q) % Q], rule.x[pt / (Q * Q)], x);
#pragma unroll
    for (int d = 0; d < 3; ++d) xyz[3 * gid + d] = x[d];
}

__global__ void k_node_coords(int32_t nex, int32_t ney, int32_t nez, int p, Rule1D nodes,
                              const double *__restrict__ vert, double *__restrict__ xyz)
{
    const int64_t nx = (int64_t)p * nex + 1, ny = (int64_t)p * ney + 1, nz = (int64_t)p * nez + 1;
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid >= nx * ny * nz) return;
    const int64_t I = gid % nx, J = (gid / nx) % ny, K = gid / (nx * ny);
    int64_t ex = I / p, ey = J / p, ez = K / p;
    ex = ex < nex ? ex : nex - 1;
    ey = ey < ney ? ey : ney - 1;
    ez = ez < nez ? ez : nez - 1;
    Elem8 el;
    load_elem(vert, ex + nex * (ey + (int64_t)ney * ez), nex, ney, el);
    double x[3];
    map_point(el, nodes.x[I - p * ex], nodes.x[J - p * ey], nodes.x[K - p * ez], x);
#pragma unroll
    for (int d = 0; d < 3; ++d) xyz[3 * gid + d] = x[d];
}

// Element restriction of a structured mesh: off[e][i + P(j + P k)] = global
// node of local node (i, j, k), or -1 for a Dirichlet boundary node.
__global__ void k_offsets(int32_t nex, int32_t ney, int32_t nez, int p, int dirichlet, int32_t *__restrict__ off)
{
    const int P = p + 1, P3 = P * P * P;
    const int64_t nelem = (int64_t)nex * ney * nez;
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid >= nelem * P3) return;
    const int64_t e = gid / P3;
    const int t = (int)(gid - e * P3);
    const int64_t ex = e % nex, ey = (e / nex) % ney, ez = e / ((int64_t)nex * ney);
    const int64_t I = p * ex + t % P, J = p * ey + (t / P) % P, K = p * ez + t / (P * P);
    const int64_t lx = (int64_t)p * nex, ly = (int64_t)p * ney, lz = (int64_t)p * nez;
    const bool bnd = I == 0 || I == lx || J == 0 || J == ly || K == 0 || K == lz;
    off[gid] = (dirichlet && bnd) ? -1 : (int32_t)(I + (lx + 1) * (J + (ly + 1) * K));
}

// Deterministic transposed restriction: node n = (I, J, K) lies in the elements
// ex in {I/p - 1 (when I is a multiple of p and > 0), I/p (when < nex)}, and
// likewise in y and z, at local index I - p ex; their values are summed in
// increasing element order (z, then y, then x), so the result does not depend
// on the order in which the elements were computed.  One thread per (node,
// vector) pair.
template <typename T>
__global__ void k_det_assemble(int32_t nex, int32_t ney, int32_t nez, int p, int dirichlet, int nvec,
                               const T *__restrict__ ebuf, T *__restrict__ y, int add)
{
    const int64_t lx = (int64_t)p * nex, ly = (int64_t)p * ney, lz = (int64_t)p * nez;
    const int64_t nn = (lx + 1) * (ly + 1) * (lz + 1);
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid >= nn * nvec) return;
    const int64_t n = gid / nvec;
    const int v = (int)(gid - n * nvec);
    const int64_t I = n % (lx + 1), J = (n / (lx + 1)) % (ly + 1), K = n / ((lx + 1) * (ly + 1));
    const bool bnd = I == 0 || I == lx || J == 0 || J == ly || K == 0 || K == lz;
    if (dirichlet && bnd) {
        if (!add) y[gid] = T(0);
        return;
    }
    const int P = p + 1, P3 = P * P * P;
    // candidate element coordinates per direction, ascending: (I - 1)/p when I is an inner multiple of p, then I/p
    auto cand = [p](int64_t I, int64_t ne, int64_t c[2]) {
        int m = 0;
        if (I % p == 0 && I > 0) c[m++] = I / p - 1;
        if (I / p < ne) c[m++] = I / p;
        return m;
    };
    int64_t cx[2], cy[2], cz[2];
    const int mx = cand(I, nex, cx), my = cand(J, ney, cy), mz = cand(K, nez, cz);
    T sum = T(0);
    for (int a = 0; a < mz; ++a)
        for (int b = 0; b < my; ++b)
            for (int c = 0; c < mx; ++c) {
                const int64_t e = cx[c] + nex * (cy[b] + (int64_t)ney * cz[a]);
                const int loc = (int)(I - p * cx[c]) + P * ((int)(J - p * cy[b]) + P * (int)(K - p * cz[a]));
                sum += ebuf[(e * P3 + loc) * nvec + v];
            }
    y[gid] = add ? y[gid] + sum : sum;
}

Rule1D quad_rule(const Basis1D &b)
{
    Rule1D r{};
    for (int i = 0; i < b.Q; ++i) {
        r.x[i] = b.xq[i];
        r.w[i] = b.wq[i];
    }
    return r;
}

unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_qdata(const GeomLaunch &g, int kind, double *q64, float *q32, double *wdet, int32_t *bad)
{
    const int64_t n = (int64_t)g.nex * g.ney * g.nez * g.q * g.q * g.q;
    hipLaunchKernelGGL(k_qdata, dim3(nblocks(n, 256)), dim3(256), 0, g.stream, g.nex, g.ney, g.nez, g.q,
                       quad_rule(*g.basis), g.vert, kind, q64, q32, wdet, bad);
    return hipGetLastError();
}

hipError_t launch_offsets(const GeomLaunch &g, int dirichlet, int32_t *off)
{
    const int P = g.p + 1;
    const int64_t n = (int64_t)g.nex * g.ney * g.nez * P * P * P;
    hipLaunchKernelGGL(k_offsets, dim3(nblocks(n, 256)), dim3(256), 0, g.stream, g.nex, g.ney, g.nez, g.p, dirichlet,
                       off);
    return hipGetLastError();
}

hipError_t launch_det_assemble(const GeomLaunch &g, int dirichlet, int nvec, int prec, const void *ebuf, void *y,
                               bool add)
{
    const int64_t n = (int64_t)(g.p * g.nex + 1) * (g.p * g.ney + 1) * (g.p * g.nez + 1) * nvec;
    if (prec == MFHEX_F32)
        hipLaunchKernelGGL(k_det_assemble<float>, dim3(nblocks(n, 256)), dim3(256), 0, g.stream, g.nex, g.ney, g.nez,
                           g.p, dirichlet, nvec, static_cast<const float *>(ebuf), static_cast<float *>(y), (int)add);
    else
        hipLaunchKernelGGL(k_det_assemble<double>, dim3(nblocks(n, 256)), dim3(256), 0, g.stream, g.nex, g.ney,
                           g.nez, g.p, dirichlet, nvec, static_cast<const double *>(ebuf), static_cast<double *>(y),
                           (int)add);
    return hipGetLastError();
}

hipError_t launch_qpoint_coords(const GeomLaunch &g, double *xyz)
{
    const int64_t n = (int64_t)g.nex * g.ney * g.nez * g.q * g.q * g.q;
    hipLaunchKernelGGL(k_qpoint_coords, dim3(nblocks(n, 256)), dim3(256), 0, g.stream, g.nex, g.ney, g.nez, g.q,
                       quad_rule(*g.basis), g.vert, xyz);
    return hipGetLastError();
}

hipError_t launch_node_coords(const GeomLaunch &g, double *xyz)
{
    const int64_t n = (int64_t)(g.p * g.nex + 1) * (g.p * g.ney + 1) * (g.p * g.nez + 1);
    Rule1D nodes{};
    for (int i = 0; i <= g.p; ++i) nodes.x[i] = g.basis->nodes[i];
    hipLaunchKernelGGL(k_node_coords, dim3(nblocks(n, 256)), dim3(256), 0, g.stream, g.nex, g.ney, g.nez, g.p,
                       nodes, g.vert, xyz);
    return hipGetLastError();
}

}  // namespace mfhex
