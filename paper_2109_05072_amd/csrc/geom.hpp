// Trilinear hexahedron geometry shared by the set-up kernels (stored
// geometric factors) and the diffusion kernel that evaluates the factors in
// place; both use these expressions, so both produce the same factors.
//
// Each hexahedron is the trilinear image of [-1,1]^3 through its 8 vertices.
// The Jacobian columns are averages of the element's edge vectors, e.g.
// dx/dr = 1/8 sum over the four x-edges of (1 +- s)(1 +- t) (X_hi - X_lo), so
// dx/dr depends on (s, t) only, dx/ds on (r, t) and dx/dt on (r, s).  The
// adjugate rows are the cross products of the columns, so
// J^{-1} = [ (j_s x j_t); (j_t x j_r); (j_r x j_s) ] / detJ with
// detJ = j_r . (j_s x j_t), and the six symmetric factors of A^e = D^T G^e D
// (Sec. 2) are G = w adj(J) adj(J)^T / detJ in Voigt order rr, ss, tt, st, rt, rs.
#pragma once

#include "mfhex_internal.h"

namespace mfhex {

struct Elem8 {
    double X[8][3];  // vertex (dx, dy, dz) at index dx + 2 dy + 4 dz
};

// Vertex index of corner v (dx + 2 dy + 4 dz) of element e on the structured vertex grid.
__device__ __forceinline__ int64_t elem_vertex(int64_t e, int nex, int ney, int v)
{
    const int64_t ex = e % nex, ey = (e / nex) % ney, ez = e / ((int64_t)nex * ney);
    const int64_t vx = nex + 1, vy = ney + 1;
    return (ex + (v & 1)) + vx * ((ey + ((v >> 1) & 1)) + vy * (ez + ((v >> 2) & 1)));
}

__device__ __forceinline__ void load_elem(const double *__restrict__ vert, int64_t e, int nex, int ney, Elem8 &el)
{
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int64_t id = elem_vertex(e, nex, ney, v);
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

// One Jacobian column: DIR 0: dx/dr at (s, t) = (u, w); DIR 1: dx/ds at (r, t);
// DIR 2: dx/dt at (r, s).  X(v) returns coordinate d of corner v.
template <int DIR, typename VX>
__device__ __forceinline__ void jacobian_col(VX X, double u, double w, double j[3])
{
    const double um[2] = {1 - u, 1 + u}, wm[2] = {1 - w, 1 + w};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double acc = 0;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                // edges along DIR at fixed values a, b of the other two corner bits
                const int lo = DIR == 0 ? 2 * a + 4 * b : DIR == 1 ? a + 4 * b : a + 2 * b;
                const int hi = lo + (DIR == 0 ? 1 : DIR == 1 ? 2 : 4);
                acc += um[a] * wm[b] * (X(hi, d) - X(lo, d));
            }
        j[d] = 0.125 * acc;
    }
}

// Jacobian columns jr = dx/dr, js = dx/ds, jt = dx/dt at (r, s, t).
__device__ __forceinline__ void jacobian_cols(const Elem8 &el, double r, double s, double t, double jr[3],
                                              double js[3], double jt[3])
{
    auto X = [&](int v, int d) { return el.X[v][d]; };
    jacobian_col<0>(X, s, t, jr);
    jacobian_col<1>(X, r, t, js);
    jacobian_col<2>(X, r, s, jt);
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

// detJ and the six diffusion factors (weight w) from the Jacobian columns.
__device__ __forceinline__ double diffusion_factors(const double jr[3], const double js[3], const double jt[3], double w,
                                                    double g[kQdDiff])
{
    double ar[3], as[3], at[3];
    cross(js, jt, ar);  // adjugate rows
    cross(jt, jr, as);
    cross(jr, js, at);
    const double det = dot3(jr, ar);
    const double f = w / det;
    g[0] = f * dot3(ar, ar);
    g[1] = f * dot3(as, as);
    g[2] = f * dot3(at, at);
    g[3] = f * dot3(as, at);
    g[4] = f * dot3(ar, at);
    g[5] = f * dot3(ar, as);
    return det;
}

}  // namespace mfhex
