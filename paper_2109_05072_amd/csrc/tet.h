// Tetrahedral P_p diffusion operator: the non-tensor basis path of Sec. 2.1 (libCEED) and
// Sec. 2.2 (its MAGMA / vendor-BLAS backend): the full basis-gradient matrix of one
// element is applied to all elements at once as a matrix product, here on
// the FP64 matrix cores.  Shared between the host set-up (tet.cpp) and the
// kernels (tet_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mfhex {
namespace tet {

constexpr int kMaxP = 6;
constexpr int kGroup = 16;       // elements per wavefront (the N extent of one matrix-core tile)
constexpr int kWaves = 4;        // wavefronts per thread group
constexpr int n_basis(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
// Low orders group elements by pairs of x-adjacent hexahedra (their 12 tetrahedra in columns 0..11
// of the wavefront's 16): the pair's element results are summed on chip over its
// (2p+1) x (p+1) x (p+1) lattice block before one global atomic per block node, and the
// restriction is computed from the block coordinates instead of read.  (At p = 2 each lattice node
// is shared by about 7 tetrahedra; per-element atomics dominate there.)
constexpr bool pair_groups(int p) { return p <= 3; }
constexpr int pair_block_nodes(int p) { return (2 * p + 1) * (p + 1) * (p + 1); }
constexpr int round_up(int n, int m) { return (n + m - 1) / m * m; }

// Sizes of one (p, q) instance: P basis functions, Q = q^3 points, padded to
// the matrix-core tile (points to 16, basis functions to 4 as a contraction
// extent and to 16 as an output extent).
struct Dims {
    int p, q, P, Q, Qp, Pk, Pn;
};
constexpr Dims dims(int p, int q)
{
    return Dims{p, q, n_basis(p), q * q * q, round_up(q * q * q, 16), round_up(n_basis(p), 4), round_up(n_basis(p), 16)};
}

// Device tables (element counts, doubles unless noted):
//   afrag [Qp/16][3][Pk/4][64]: lane l of step s of point block b holds G_d[16b + l%16][4s + l/16]
//   bfrag [Qp/16][3][4][Pn/16][64]: lane l of (b, d, r, t) holds G_d[16b + 4r + l/16][16t + l%16]
// with G_d[k][n] = d phi_n / d xi_d at point k (0 outside the Q x P matrix).
// Matrix-core operand layout of the 16x16x4 FP64 product D += A B (wave64):
// lane l supplies A[l%16][l/16] and B[l/16][l%16], and its result register r
// is D[4r + l/16][l%16] (checked on gfx950 with distinct entries).
constexpr size_t afrag_len(const Dims &D) { return (size_t)(D.Qp / 16) * 3 * (D.Pk / 4) * 64; }
constexpr size_t bfrag_len(const Dims &D) { return (size_t)(D.Qp / 16) * 3 * 4 * (D.Pn / 16) * 64; }

struct TetLaunch {
    int p, q;
    int nex, ney, nez, dirichlet;   // pair groups: the mesh, for the computed restriction
    int64_t nelem, ngroups;
    const int32_t *lattice;         // [P][4]: n1, n2, n3 of each basis function's node
    const double *afrag, *bfrag;
    const int32_t *offsets;  // [ngroups][P][16], -1 = masked node or no element (not with pair groups)
    const double *qdata;     // [ngroups][Q][6][16]: w |det J| J^-1 J^-T (xx, yy, zz, yz, xz, xy)
    const double *x;
    double *y;
    hipStream_t stream;
};

struct TetSetupLaunch {
    int p, q, nex, ney, nez, dirichlet;
    int64_t nelem, ngroups;
    const double *vert;     // [(nex+1)(ney+1)(nez+1)][3]
    const int32_t *lattice; // [P][4]: n1, n2, n3 of each basis function's node
    const double *wq;       // [Q] reference rule weights
    int32_t *offsets;
    double *qdata;
    int *bad;               // set to 1 when an element has det J <= 0 in absolute terms
    hipStream_t stream;
};

hipError_t launch_tet_setup(const TetSetupLaunch &s);
hipError_t launch_tet_apply(const TetLaunch &a);

}  // namespace tet
}  // namespace mfhex
