// Tetrahedral P_p diffusion operator: set-up and fused apply kernels.
//
// Apply (Sec. 2.1 libCEED and Sec. 2.2 MAGMA: the non-tensor basis action as a matrix product over
// elements).  One wavefront owns 16 elements; the kWaves wavefronts of a
// thread group stage the basis fragments of each block of 16 quadrature
// points b in LDS together (coalesced copies shared by 4 x 16 elements,
// fetched one phase ahead), then each:
//   phase 1, U_d = G_d X on the FP64 matrix cores: A = the basis-gradient rows
//     of the block (16 points x 4 basis functions per step, a pre-swizzled
//     fragment of 64 consecutive doubles), B = the 16 elements' gathered
//     values (4 basis functions x 16 elements per step, kept in registers for
//     the whole element group);
//   pointwise, in the result registers: v = D_q u with the symmetric factor
//     D_q = w |det J| J^-1 J^-T of each (point, element);
//   phase 2, Y^T += V_d^T G_d: result register r of every lane holds the
//     points 16b + 4r + (0..3) of one element (the matrix-core result
//     layout), which is exactly the A operand of a 4-deep step over those
//     points, so the products feed the transposed contraction with no data
//     movement; B = the gradient rows of the same 4 points (pre-swizzled).
// The 16 x P element results then go to the nodes with FP64 atomics.
#include "mfhex_internal.h"
#include "tet.h"

namespace mfhex {
namespace tet {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Kuhn tetrahedron t: axis permutation; vertex k is the cube corner sum_{m<k} e_{pi[m]}.
__device__ __forceinline__ void kuhn_perm(int t, int &a0, int &a1, int &a2)
{
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    a0 = perms[t][0];
    a1 = perms[t][1];
    a2 = perms[t][2];
}

// Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous range of element groups.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nb)
{
    const int64_t x = bid % kNumXcd, i = bid / kNumXcd;
    const int64_t q = nb / kNumXcd, r = nb % kNumXcd;
    return x * q + (x < r ? x : r) + i;
}

// offsets[g][n][16]: global lattice node of basis function n of element 16 g + j (-1: masked / none).
__global__ void k_tet_offsets(int p, int P, int nex, int ney, int nez, int dirichlet, int64_t nelem, int64_t total,
                              const int32_t *__restrict__ lattice, int32_t *__restrict__ offsets)
{
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int j = (int)(idx % kGroup);
    const int n = (int)((idx / kGroup) % P);
    const int64_t e = (idx / ((int64_t)kGroup * P)) * kGroup + j;
    int32_t o = -1;
    if (e < nelem) {
        const int64_t cube = e / 6;
        const int t = (int)(e % 6);
        const int ex = (int)(cube % nex), ey = (int)((cube / nex) % ney), ez = (int)(cube / ((int64_t)nex * ney));
        int a0, a1, a2;
        kuhn_perm(t, a0, a1, a2);
        const int n1 = lattice[4 * n], n2 = lattice[4 * n + 1], n3 = lattice[4 * n + 2];
        // lattice offset n1 v1 + n2 v2 + n3 v3 with v1 = e_a0, v2 = e_a0 + e_a1, v3 = (1,1,1)
        int a[3] = {n3, n3, n3};
        a[a0] += n1 + n2;
        a[a1] += n2;
        (void)a2;
        const int nx = p * nex + 1, ny = p * ney + 1, nz = p * nez + 1;
        const int I = p * ex + a[0], J = p * ey + a[1], K = p * ez + a[2];
        const bool bnd = I == 0 || I == nx - 1 || J == 0 || J == ny - 1 || K == 0 || K == nz - 1;
        if (!(dirichlet && bnd)) o = I + nx * (J + ny * K);
    }
    offsets[idx] = o;
}

// qdata[g][m][6][16] = w_m |det J| J^-1 J^-T = w_m adj(J) adj(J)^T / |det J| (xx, yy, zz, yz, xz, xy).
// Element of column j of group g (-1: empty column).
__device__ __forceinline__ int64_t group_element(int64_t g, int j, bool pairs, int nex, int ney, int64_t nelem)
{
    if (!pairs) {
        const int64_t e = g * kGroup + j;
        return e < nelem ? e : -1;
    }
    const int npx = (nex + 1) / 2;
    const int px = (int)(g % npx);
    const int64_t row = g / npx;  // ey + ney ez
    const int cx = 2 * px + j / 6;
    if (j >= 12 || cx >= nex) return -1;
    return 6 * (cx + (int64_t)nex * row) + j % 6;
}

__global__ void k_tet_qdata(int Q, int nex, int ney, int pairs, int64_t nelem, int64_t nslots,
                            const double *__restrict__ vert, const double *__restrict__ wq, double *__restrict__ qdata,
                            int *__restrict__ bad)
{
    const int64_t slot = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (slot >= nslots) return;
    const int64_t g = slot / kGroup;
    const int j = (int)(slot % kGroup);
    const int64_t e = group_element(g, j, pairs != 0, nex, ney, nelem);
    double M[6] = {0, 0, 0, 0, 0, 0};
    if (e >= 0) {
        const int64_t cube = e / 6;
        const int t = (int)(e % 6);
        const int ex = (int)(cube % nex), ey = (int)((cube / nex) % ney), ez = (int)(cube / ((int64_t)nex * ney));
        int a0, a1, a2;
        kuhn_perm(t, a0, a1, a2);
        int c[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 1}};
        c[1][a0] = 1;
        c[2][a0] = 1;
        c[2][a1] = 1;
        (void)a2;
        double X[4][3];
        for (int v = 0; v < 4; ++v) {
            const int64_t vid = (ex + c[v][0]) + (int64_t)(nex + 1) * ((ey + c[v][1]) + (int64_t)(ney + 1) * (ez + c[v][2]));
            for (int d = 0; d < 3; ++d) X[v][d] = vert[3 * vid + d];
        }
        double Jm[3][3];  // J[row = physical dir][col = reference dir]
        for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc) Jm[r][cc] = X[cc + 1][r] - X[0][r];
        // adjugate: adj(J)[i][k] = cofactor(J)[k][i]
        double A[3][3];
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) {
                const int r0 = (k + 1) % 3, r1 = (k + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
                A[i][k] = Jm[r0][c0] * Jm[r1][c1] - Jm[r0][c1] * Jm[r1][c0];
            }
        const double det = Jm[0][0] * A[0][0] + Jm[0][1] * A[1][0] + Jm[0][2] * A[2][0];
        if (!(det != 0.0) || !isfinite(det)) bad[0] = 1;
        const double s = 1.0 / fabs(det);
        // (adj adj^T)[a][b] = sum_i adj[a][i] adj[b][i]
        auto aa = [&](int x, int y) { return (A[x][0] * A[y][0] + A[x][1] * A[y][1] + A[x][2] * A[y][2]) * s; };
        M[0] = aa(0, 0);
        M[1] = aa(1, 1);
        M[2] = aa(2, 2);
        M[3] = aa(1, 2);
        M[4] = aa(0, 2);
        M[5] = aa(0, 1);
    }
    double *qd = qdata + (size_t)g * Q * 6 * kGroup + j;
    for (int m = 0; m < Q; ++m) {
        const double w = wq[m];
        for (int f = 0; f < 6; ++f) qd[((size_t)m * 6 + f) * kGroup] = w * M[f];
    }
}

// LDS: the gradient fragments of one point block, shared by the kWaves element groups of the thread group.
constexpr size_t frag_block_doubles(const Dims &D) { return (size_t)3 * (D.Pk / 4) * 64 + (size_t)12 * (D.Pn / 16) * 64; }

// Pair groups: lattice-block coordinates (bx, by, bz) in [0, 2p] x [0, p] x [0, p] of basis
// function n of column j (tetrahedron j % 6 of hexahedron j / 6 of the pair).
__device__ __forceinline__ void pair_block_coords(int p, int j, const int32_t *__restrict__ lattice, int n, int &bx,
                                                  int &by, int &bz)
{
    int a0, a1, a2;
    kuhn_perm(j % 6, a0, a1, a2);
    (void)a2;
    const int n1 = lattice[4 * n], n2 = lattice[4 * n + 1], n3 = lattice[4 * n + 2];
    int a[3] = {n3, n3, n3};
    a[a0] += n1 + n2;
    a[a1] += n2;
    bx = (j / 6) * p + a[0];
    by = a[1];
    bz = a[2];
}

// Global lattice node of block node (bx, by, bz) of pair (px, row), -1 if masked or past the mesh.
__device__ __forceinline__ int32_t pair_node(int p, int nex, int ney, int nez, int dirichlet, int px, int64_t row,
                                             int bx, int by, int bz)
{
    const int nx = p * nex + 1, ny = p * ney + 1, nz = p * nez + 1;
    const int ey = (int)(row % ney), ez = (int)(row / ney);
    const int I = 2 * p * px + bx, J = p * ey + by, K = p * ez + bz;
    if (I >= nx) return -1;
    if (dirichlet && (I == 0 || I == nx - 1 || J == 0 || J == ny - 1 || K == 0 || K == nz - 1)) return -1;
    return I + nx * (J + ny * K);
}

template <int p, int q>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(p == 4 ? 3 : 2)))
k_tet_apply(int64_t ngroups, int nex, int ney, int nez, int dirichlet, const int32_t *__restrict__ lattice,
            const double *__restrict__ afrag, const double *__restrict__ bfrag, const int32_t *__restrict__ offsets,
            const double *__restrict__ qdata, const double *__restrict__ x, double *__restrict__ y)
{
    constexpr Dims D = dims(p, q);
    constexpr int P = D.P, Q = D.Q, NS = D.Pk / 4, NT = D.Pn / 16, NB = D.Qp / 16;
    constexpr int AL = 3 * NS * 64, BL = 12 * NT * 64, FL = AL + BL;
    constexpr bool PAIRS = pair_groups(p);
    constexpr int NBLK = pair_block_nodes(p), BXN = 2 * p + 1, BYN = p + 1;
    extern __shared__ __align__(16) double sfrag[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x / 64;
    const int64_t g0 = xcd_remap(blockIdx.x, gridDim.x) * kWaves + wave;  // wavefront-uniform
    // every wavefront takes part in the staging and its barriers; one past the last group computes on
    // the last group's data and stores nothing
    const bool active = g0 < ngroups;
    const int64_t g = active ? g0 : ngroups - 1;
    const int el = lane % 16, kq = lane / 16;
    const int32_t *off = PAIRS ? nullptr : offsets + (size_t)g * P * kGroup;
    // pair groups: pair coordinates, whether column el holds an element, this wavefront's block sums
    const int npx = (nex + 1) / 2;
    const int px = (int)(g % npx);
    const int64_t row = g / npx;
    const bool col_ok = el < 12 && 2 * px + el / 6 < nex;
    double *const sblk = sfrag + FL + wave * round_up(NBLK, 2);
    if constexpr (PAIRS)
        for (int i = lane; i < NBLK; i += 64) sblk[i] = 0.0;

    // B operand of phase 1: lane holds X[basis 4s + kq][element el] for every step s
    // (branch-free: every load is issued, from a clamped index, and the value selected afterwards, so
    // the loads of all steps are in flight together instead of one round trip per step)
    double xf[NS];
    int32_t xo[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int n = 4 * s + kq;
        if constexpr (PAIRS) {
            int bx, by, bz;
            pair_block_coords(p, el, lattice, n < P ? n : P - 1, bx, by, bz);
            const int32_t o = pair_node(p, nex, ney, nez, dirichlet, px, row, bx, by, bz);
            xo[s] = col_ok && n < P ? o : -1;
        } else {
            const int32_t o = __builtin_nontemporal_load(&off[(n < P ? n : P - 1) * kGroup + el]);
            xo[s] = n < P ? o : -1;
        }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const double v = x[xo[s] >= 0 ? xo[s] : 0];
        xf[s] = xo[s] >= 0 ? v : 0.0;
    }
    d4 yacc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) yacc[t] = d4{0.0, 0.0, 0.0, 0.0};

    const double *qg = qdata + (size_t)g * Q * 6 * kGroup + el;
    // staging is software-pipelined: the B fragments of block b travel (global -> registers) during
    // phase 1, the A fragments of block b+1 during phase 2; each lands in LDS at the next barrier
    constexpr int NTH = 64 * kWaves, RA = (AL + NTH - 1) / NTH, RB = (BL + NTH - 1) / NTH;
    double *const sA = sfrag, *const sB = sfrag + AL;
    const int tid = threadIdx.x;
    double stage[RA > RB ? RA : RB];
#pragma unroll
    for (int k = 0; k < RA; ++k)
        if (tid + k * NTH < AL) sA[tid + k * NTH] = afrag[tid + k * NTH];
    __syncthreads();
    for (int b = 0; b < NB; ++b) {
        // this lane's factors for the block (issued first: their latency overlaps phase 1)
        double qv[4][6];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = 16 * b + 4 * r + kq;
            const double *qd = qg + (size_t)(m < Q ? m : Q - 1) * 6 * kGroup;
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                const double v = __builtin_nontemporal_load(&qd[f * kGroup]);
                qv[r][f] = m < Q ? v : 0.0;
            }
        }
        {
            const double *bb = bfrag + (size_t)b * BL;
#pragma unroll
            for (int k = 0; k < RB; ++k) stage[k] = tid + k * NTH < BL ? bb[tid + k * NTH] : 0.0;
        }
        const double *A = sA + lane;
        d4 u[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) u[d] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int d = 0; d < 3; ++d) u[d] = mma(A[(d * NS + s) * 64], xf[s], u[d]);
        // pointwise: register r <-> point 16 b + 4 r + kq of element el
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double xx = qv[r][0], yy = qv[r][1], zz = qv[r][2], yz = qv[r][3], xz = qv[r][4], xy = qv[r][5];
            const double ur = u[0][r], us = u[1][r], ut = u[2][r];
            u[0][r] = xx * ur + xy * us + xz * ut;
            u[1][r] = xy * ur + yy * us + yz * ut;
            u[2][r] = xz * ur + yz * us + zz * ut;
        }
#pragma unroll
        for (int k = 0; k < RB; ++k)
            if (tid + k * NTH < BL) sB[tid + k * NTH] = stage[k];
        __syncthreads();  // B fragments of b in LDS; every wavefront is done with the A fragments of b
        if (b + 1 < NB) {
            const double *ab = afrag + (size_t)(b + 1) * AL;
#pragma unroll
            for (int k = 0; k < RA; ++k) stage[k] = tid + k * NTH < AL ? ab[tid + k * NTH] : 0.0;
        }
        const double *Bf = sB + lane;
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int t = 0; t < NT; ++t) yacc[t] = mma(u[d][r], Bf[((d * 4 + r) * NT + t) * 64], yacc[t]);
        if (b + 1 < NB) {
#pragma unroll
            for (int k = 0; k < RA; ++k)
                if (tid + k * NTH < AL) sA[tid + k * NTH] = stage[k];
        }
        __syncthreads();  // A fragments of b+1 in LDS; every wavefront is done with the B fragments of b
    }
    if (!active) return;
    // result register r of tile t: element 4 r + kq, basis function 16 t + el
    if constexpr (PAIRS) {
        // sum the pair's 12 element results over its lattice block on chip, then one atomic per node
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int n = 16 * t + el;
            if (n < P) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = 4 * r + kq;
                    if (j < 12 && 2 * px + j / 6 < nex) {
                        int bx, by, bz;
                        pair_block_coords(p, j, lattice, n, bx, by, bz);
                        atomicAdd(&sblk[bx + BXN * (by + BYN * bz)], yacc[t][r]);
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int i = lane; i < NBLK; i += 64) {
            const int bx = i % BXN, by = (i / BXN) % BYN, bz = i / (BXN * BYN);
            const int32_t o = pair_node(p, nex, ney, nez, dirichlet, px, row, bx, by, bz);
            if (o >= 0) unsafeAtomicAdd(&y[o], sblk[i]);
        }
    } else {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int n = 16 * t + el;
            if (n < P) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int32_t o = off[n * kGroup + 4 * r + kq];
                    if (o >= 0) unsafeAtomicAdd(&y[o], yacc[t][r]);
                }
            }
        }
    }
}

template <int p, int q>
hipError_t apply_pq(const TetLaunch &a)
{
    const int64_t nblk = (a.ngroups + kWaves - 1) / kWaves;
    const size_t lds = (frag_block_doubles(dims(p, q)) + (pair_groups(p) ? kWaves * round_up(pair_block_nodes(p), 2) : 0)) *
                       sizeof(double);
    auto kern = k_tet_apply<p, q>;
    if (lds > 65536) {
        const hipError_t e =
            hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(64 * kWaves), lds, a.stream, a.ngroups, a.nex, a.ney, a.nez,
                       a.dirichlet, a.lattice, a.afrag, a.bfrag, a.offsets, a.qdata, a.x, a.y);
    return hipGetLastError();
}

template <int p>
hipError_t apply_p(const TetLaunch &a)
{
    if (a.q == p) return apply_pq<p, p>(a);
    if (a.q == p + 1) return apply_pq<p, p + 1>(a);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_tet_setup(const TetSetupLaunch &s)
{
    const int P = n_basis(s.p), Q = s.q * s.q * s.q;
    const bool pairs = pair_groups(s.p);
    const int64_t total = s.ngroups * P * kGroup, nslots = s.ngroups * kGroup;
    if (!pairs) {
        hipLaunchKernelGGL(k_tet_offsets, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s.stream, s.p, P, s.nex,
                           s.ney, s.nez, s.dirichlet, s.nelem, total, s.lattice, s.offsets);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_tet_qdata, dim3((unsigned)((nslots + 127) / 128)), dim3(128), 0, s.stream, Q, s.nex, s.ney,
                       pairs ? 1 : 0, s.nelem, nslots, s.vert, s.wq, s.qdata, s.bad);
    return hipGetLastError();
}

hipError_t launch_tet_apply(const TetLaunch &a)
{
    switch (a.p) {
    case 1: return apply_p<1>(a);
    case 2: return apply_p<2>(a);
    case 3: return apply_p<3>(a);
    case 4: return apply_p<4>(a);
    case 5: return apply_p<5>(a);
    case 6: return apply_p<6>(a);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tet
}  // namespace mfhex
