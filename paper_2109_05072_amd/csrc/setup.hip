// Setup kernels: quadrature data (geometric factors) and coordinates.
//
// Each hexahedron is the trilinear image of [-1,1]^3 through its 8 vertices.
// The Jacobian columns are written as averages of the element's edge
// vectors, e.g. dx/dr = 1/8 sum over the four x-edges of
// (1 +- s)(1 +- t) (X_hi - X_lo); the adjugate rows are the cross products
// of the columns, so J^{-1} = [ (j_s x j_t); (j_t x j_r); (j_r x j_s) ] / detJ
// with detJ = j_r . (j_s x j_t).  Stored per point (Sec. 2, the six symmetric
// geometric factors of A^e = D^T G^e D):
//   diffusion: G = w adj(J) adj(J)^T / detJ in Voigt order rr, ss, tt, st, rt, rs
//   mass:      w detJ
#include "mfhex_internal.h"

namespace mfhex {

namespace {

struct Rule1D {
    double x[kMaxQ];
    double w[kMaxQ];
};

struct Elem8 {
    double X[8][3];  // vertex (dx, dy, dz) at index dx + 2 dy + 4 dz
};

__device__ __forceinline__ void load_elem(const double *__restrict__ vert, int64_t e, int nex, int ney, Elem8 &el)
{
    const int64_t ex = e % nex, ey = (e / nex) % ney, ez = e / ((int64_t)nex * ney);
    const int64_t vx = nex + 1, vy = ney + 1;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int64_t id = (ex + (v & 1)) + vx * ((ey + ((v >> 1) & 1)) + vy * (ez + ((v >> 2) & 1)));
#pragma unroll
        for (int d = 0; d < 3; ++d) el.X[v][d] = vert[3 * id + d];
    }
}

__device__ __forceinline__ void map_point(const Elem8 &el, double r, double s, double t, double x[3])
{
    const double h[2][3] = {{0.5 * (1 - r), 0.5 * (1 - s), 0.5 * (1 - t)}, {0.5 * (1 + r), 0.5 * (1 + s), 0.5 * (1 + t)}};
#pragma unroll
    for (int d = 0; d < 3; ++d) x[d] = 0.0;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const double n = h[v & 1][0] * h[(v >> 1) & 1][1] * h[(v >> 2) & 1][2];
#pragma unroll
        for (int d = 0; d < 3; ++d) x[d] += n * el.X[v][d];
    }
}

// Jacobian columns jr = dx/dr, js = dx/ds, jt = dx/dt from edge vectors.
__device__ __forceinline__ void jacobian_cols(const Elem8 &el, double r, double s, double t, double jr[3],
                                              double js[3], double jt[3])
{
    const double sm[2] = {1 - s, 1 + s}, tm[2] = {1 - t, 1 + t}, rm[2] = {1 - r, 1 + r};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double ar = 0, as = 0, at = 0;
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int w = 0; w < 2; ++w) {
                // x-edges: vary dx at fixed (dy = u, dz = w)
                ar += sm[u] * tm[w] * (el.X[1 + 2 * u + 4 * w][d] - el.X[0 + 2 * u + 4 * w][d]);
                // y-edges: vary dy at fixed (dx = u, dz = w)
                as += rm[u] * tm[w] * (el.X[u + 2 + 4 * w][d] - el.X[u + 0 + 4 * w][d]);
                // z-edges: vary dz at fixed (dx = u, dy = w)
                at += rm[u] * sm[w] * (el.X[u + 2 * w + 4][d] - el.X[u + 2 * w + 0][d]);
            }
        jr[d] = 0.125 * ar;
        js[d] = 0.125 * as;
        jt[d] = 0.125 * at;
    }
}

__device__ __forceinline__ void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

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
    double jr[3], js[3], jt[3], ar[3], as[3], at[3];
    jacobian_cols(el, rule.x[a], rule.x[b], rule.x[c], jr, js, jt);
    cross(js, jt, ar);  // adjugate rows
    cross(jt, jr, as);
    cross(jr, js, at);
    const double det = dot3(jr, ar);
    const double w = rule.w[a] * rule.w[b] * rule.w[c];
    if (!(det > 0.0)) atomicOr(bad, 1);
    if (kind == MFHEX_DIFFUSION) {
        const double f = w / det;
        const double g[kQdDiff] = {f * dot3(ar, ar), f * dot3(as, as), f * dot3(at, at),
                                   f * dot3(as, at), f * dot3(ar, at), f * dot3(ar, as)};
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
