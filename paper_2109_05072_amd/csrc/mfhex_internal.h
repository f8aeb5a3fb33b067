// Internal declarations shared by the host runtime (*.cpp) and the kernels (*.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/mfhex.h"

namespace mfhex {

constexpr int kMaxP = 9;   // nodes per direction (p = 8)
constexpr int kMaxQ = 10;  // quadrature points per direction (q = p + 2)
constexpr int kQdDiff = 6; // symmetric geometric factors per point (Voigt rr, ss, tt, st, rt, rs)
constexpr int kNumXcd = 8; // MI355X: 8 accelerator complex dies, blocks dealt round-robin

// 1D data of one operator, FP64 (host master copy) and FP32.
struct Basis1D {
    int P = 0, Q = 0;
    bool colloc = false;             // Q == P and points == nodes (B = I)
    double nodes[kMaxP];             // Gauss-Lobatto nodes
    double xq[kMaxQ], wq[kMaxQ];     // quadrature points / weights
    double B[kMaxQ * kMaxP];         // B[a*P + i] = l_i(xq_a)
    double D[kMaxQ * kMaxQ];         // D[a*Q + b] = derivative at point a of the Lagrange
                                     // polynomial through the points that is 1 at point b
    double Gn[kMaxQ * kMaxP];        // Gn[a*P + i] = l_i'(xq_a)   (direct, for checks)
};

// Host side of the basis construction (basis.cpp).
int build_basis(int p, int q, int quad, Basis1D *out, std::string *err);
int gauss_rule(int n, double *x, double *w);
int lobatto_rule(int n, double *x, double *w);

// Kernel arguments common to the operator kernels.
struct OpView {
    int64_t nelem;
    int32_t nex, ney, nez, p, q;
    int64_t nnodes;
    const int32_t *offsets;  // [E][P^3], -1 = masked node
    const void *qdata;       // [E][g][Q^3] in the apply precision
    const double *kappa;     // [E][Q^3] or null
};

enum Mode : int { kMass = 0, kDiff = 1, kRhs = 2 };

// Launch configuration of the apply: the variant (elements and threads per
// thread group, vectors per chunk) and, for the mass operator, the number of
// consecutive element groups one thread group pipelines through.
constexpr int kMaxChain = 64;
struct LaunchCfg {
    int variant = 0;
    int chain = 1;
};

struct ApplyLaunch {
    OpView v;
    int P, colloc;
    const void *basis_dev; // device basis block (B, B^T, D, D^T) in the apply precision
    int prec;             // MFHEX_F64 / MFHEX_F32
    int mode;             // kMass / kDiff / kRhs
    int vark;             // multiply the factors by kappa
    int nvec;
    int variant;          // launch variant (elements and threads per group)
    int chain;            // mass: element groups per thread group (software pipeline depth), >= 1
    int otf;              // diffusion FP64: geometric factors evaluated in the kernel from the vertices
    const double *vert;   // device vertex coordinates [(nex+1)(ney+1)(nez+1)][3] (otf)
    const void *x;        // input (for kRhs: the per-point f, FP64)
    void *y;              // output (accumulated)
    const double *wdet;   // kRhs: w*detJ per point
    void *ebuf;           // deterministic scatter: element values [E][P^3][nvec] (null: atomics into y)
    hipStream_t stream;
};

// Diagonal of the assembled operator (FP64), accumulated into d.
struct DiagLaunch {
    OpView v;  // FP64 factors
    int P, colloc, mode, vark;
    const double *basis_dev;
    double *d;
    hipStream_t stream;
};

struct KgradLaunch {
    OpView v;
    int P, colloc;
    const double *basis_dev;
    const double *u, *r;
    double *g;
    hipStream_t stream;
};

// LDS layout of one element's working array: [c][b][a] with an odd row pitch so
// that pencils along any axis hit distinct banks; q = 10 keeps the pitch of 10,
// which fits a split group's four arrays in 32 KB, five groups per CU (4% faster
// than pitch 11 for the prefetching split group in same-box A/B, where the
// padding left room for four).
constexpr int lds_pitch(int Q) { return (Q % 2 == 0 && Q != 10) ? Q + 1 : Q; }
constexpr int lds_buf(int Q) { return lds_pitch(Q) * Q * Q; }
constexpr int apply_nbuf(int mode, bool split = false) { return mode == 1 ? (split ? 4 : 3) : 1; }
// Split stages of the diffusion kernel: with G elements and one vector per
// group of NT >= 256 threads whose widest contraction (G Q^2 lines) fits in
// half the group, the two halves (two wavefronts each) share every contraction:
// each takes half of the output rows, and independent contractions run side
// by side, so no wavefront of the group sits out a contraction stage.  A
// fourth LDS array lets every such stage write a different array than it
// reads.  (Measured on MI355X: 2% faster at q = 10 with 256 threads; with 128
// threads the extra registers cost one wave per SIMD and 6% at q = 8.)
constexpr bool split_stages(int Q, int mode, int G, int NT, int VC)
{
    return mode == 1 && VC == 1 && NT >= 256 && 2 * G * Q * Q <= NT;
}

// Launch variants of the fused kernels for q points per direction: G
// elements per thread group of NT threads; variant 0 is the default.
// Variants 0..4 carry one vector at a time through the element (rows: Q = 2
// .. 10; variant 0 is the measured best on MI355X for one vector); variants
// 5..8 carry a chunk of VC = 2, 4, 8, 16 vectors of a multi-vector together
// (one element per group), sharing the geometric factors and reading /
// writing each node's chunk as one contiguous run.  Variants 9..14 are the
// factored-gradient kernel (below); 15 and 16 are chunks of 4 and 8 vectors
// whose collocated gradient contractions run on the FP64 matrix cores.
constexpr int kNumVariants = 17;
// At q = 6 and 7 variant 4 fills the lanes: every contraction of the diffusion
// kernel runs over G q^2 lines (q^2 = 36, 49), so 7 and 5 elements per
// 256-thread group give 252 and 245 lines, where groups of 1 or 2 elements
// leave 44-62% of the lanes idle.
// Late factor loads: at q = 7 and 9 variant 2 and at q = 8 and 10 variants 4 and 2 load each
// point's geometric factors in the pointwise stage (the listed number of points at a time)
// instead of at the start of the element group.  The prefetched factors of a lane's points hold
// 6 x 2 registers per point (8 points per lane at q = 10 with 128 threads: 96 registers) through
// every forward contraction; loaded late they are live in the pointwise stage only, so more
// wavefronts fit on a SIMD (q = 7..9, two points at a time: 64-72 registers instead of 120-142)
// while the loads' latency is no longer hidden by the contractions.  At q = 10 this was 6% faster
// on one box and 5% slower on another against variant 0 with 128 threads.  With 256 threads
// (split stages) the late loads are the q = 9 and 10 defaults: 68 and 81 registers instead of 101
// and 126, so that five to six groups fit per CU (at q = 10 with the unpadded row pitch, which
// puts the four arrays of a group in 32 KB); same-box A/B, one element per group: q = 9 6%
// faster than the best prefetching variant, q = 10 11%.
constexpr int kVarG[9][5] = {
    {16, 8, 32, 16, 32}, {8, 4, 16, 8, 16}, {4, 2, 8, 4, 8}, {4, 2, 5, 2, 8}, {1, 3, 1, 2, 7},
    {1, 2, 1, 4, 5},     {1, 2, 1, 2, 1},   {2, 1, 1, 1, 1}, {1, 1, 1, 1, 2}};
constexpr int kVarNT[9][5] = {
    {64, 64, 64, 128, 128},  {64, 64, 64, 128, 128},  {64, 64, 64, 128, 128},
    {128, 64, 256, 128, 256}, {64, 256, 128, 128, 256}, {64, 128, 64, 256, 256},
    {128, 256, 64, 128, 128}, {256, 128, 128, 256, 256}, {256, 128, 128, 256, 256}};
// points per factor-load batch in the pointwise stage (0: factors prefetched at the group start)
constexpr int kVarLate[9][5] = {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}, {0, 0, 2, 0, 0}, {0, 2, 0, 0, 0},
                                {0, 0, 3, 3, 0}, {0, 2, 0, 0, 2}, {0, 0, 2, 0, 2}, {0, 0, 4, 2, 0}};
constexpr int variant_late(int Q, int v) { return v < 5 ? kVarLate[Q - 2][v] : 0; }
// of those, points per lane whose factors are still prefetched at the group start (the rest load late)
constexpr int kVarPre[9][5] = {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0},
                               {0, 0, 3, 3, 0}, {0, 0, 0, 0, 2}, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};
constexpr int variant_pre(int Q, int v) { return v < 5 ? kVarPre[Q - 2][v] : 0; }
constexpr bool variant_mx(int v) { return v >= 15; }
constexpr int variant_vc(int v)
{
    return v == 15 ? 4 : v == 16 ? 8 : v < 5 || v >= 9 ? 1 : v == 5 ? 2 : v == 6 ? 4 : v == 7 ? 8 : 16;
}
// Variants 9 .. 14: the factored-gradient diffusion kernel (Gauss points, one vector at a time;
// k_apply_gf): 9 .. 13 take the (elements, threads) pairs below per q and load the geometric
// factors at the start of the element group; 14 is variant 9 loading them in the middle of the
// forward stages (fewer registers held through the first contractions).
constexpr int kGfG[9][5] = {{16, 8, 32, 16, 8}, {16, 8, 32, 16, 8}, {8, 4, 16, 8, 4}, {8, 4, 2, 8, 4},
                            {4, 2, 8, 4, 2},    {2, 1, 4, 2, 1},    {1, 2, 4, 1, 2}, {1, 1, 2, 2, 1},
                            {1, 1, 2, 2, 1}};
constexpr int kGfNT[9][5] = {{128, 64, 256, 256, 128}, {128, 64, 256, 256, 128}, {128, 64, 256, 256, 128},
                             {256, 128, 64, 128, 64},  {128, 64, 256, 256, 128}, {128, 64, 256, 64, 128},
                             {64, 128, 256, 128, 64},  {128, 64, 256, 128, 256}, {128, 64, 256, 128, 256}};
constexpr bool variant_gf(int v) { return v >= 9 && v <= 14; }
constexpr bool gf_prefetch(int v) { return v != 14; }
constexpr int gf_slot(int v) { return v == 14 ? 0 : v - 9; }
// The mass operator keeps one LDS array per element instead of three and has
// far less work per element, so at low order its single-vector variants
// carry more elements per group.
constexpr int mass_group_scale(int Q) { return Q <= 4 ? 4 : Q <= 6 ? 2 : 1; }
constexpr int variant_g(int Q, int v, int mode = 1)
{
    return variant_gf(v) ? kGfG[Q - 2][gf_slot(v)] : v < 5 ? kVarG[Q - 2][v] * (mode == 1 ? 1 : mass_group_scale(Q)) : 1;
}
constexpr int variant_nt(int Q, int v)
{
    return variant_gf(v) ? kGfNT[Q - 2][gf_slot(v)]
           : v < 5       ? kVarNT[Q - 2][v]
                         : (Q * Q * variant_vc(v) <= 64 ? 64 : Q * Q * variant_vc(v) <= 128 ? 128 : 256);
}
// Dynamic LDS bytes of one group of the fused apply.
// In-kernel geometric factors: per element its 8 vertices (24 doubles) and
// the three Jacobian-column tables (3 x Q^2 columns of 3), plus the 1D rule.
constexpr int otf_lds_doubles(int Q, int G) { return G * (24 + 9 * Q * Q) + 2 * Q; }

constexpr bool variant_split(int Q, int v, int mode)
{
    return !variant_gf(v) && split_stages(Q, mode, variant_g(Q, v, mode), variant_nt(Q, v), variant_vc(v));
}
// Multi-vector chunks of the diffusion kernel add their results to y in runs of at least 64 bytes
// per node (8 FP64 or 16 FP32 vectors) when a launch has more vectors than one chunk: y is
// node-major, and a chunk of fewer vectors would leave partly written lines in the L2 between
// chunks, which go back to HBM as 32-byte partial writes.  The element values of all but the last
// chunk of a run wait in LDS ([P^3][run - VC]), next to the element's restriction offsets ([P^3]
// int32).  A launch whose vectors fit one chunk adds them directly.
constexpr int scatter_run(int vc, int elem_bytes) { return vc * elem_bytes >= 64 ? vc : 64 / elem_bytes; }
constexpr bool staged_scatter(int mode, int vc, int elem_bytes)
{
    return mode == 1 && vc > 1 && scatter_run(vc, elem_bytes) > vc;
}
constexpr size_t apply_lds(int P, int Q, int mode, int elem_bytes, int v, bool otf = false, bool stage = false)
{
    const int vc = variant_vc(v);
    const size_t p3 = (size_t)P * P * P;
    return (size_t)variant_g(Q, v, mode) * vc * apply_nbuf(mode, variant_split(Q, v, mode)) * lds_buf(Q) * elem_bytes +
           (otf ? (size_t)otf_lds_doubles(Q, variant_g(Q, v, mode)) * 8 : 0) +
           (stage && staged_scatter(mode, vc, elem_bytes) ? p3 * (scatter_run(vc, elem_bytes) - vc) * elem_bytes + p3 * 4
                                                          : 0);
}
// Largest dynamic LDS of one thread group (gfx950 has 160 KB per CU; above 64 KB the kernel is
// launched with a raised limit).  96 KB admits 8-vector chunks at q = 7, 4-vector chunks at q = 9
// and 16-vector chunks at q = 6 while still leaving room for a second group on the CU.
constexpr size_t kMaxLds = 98304;
constexpr size_t kLdsTwoGroups = 81920;  // at most this much LDS leaves room for two thread groups per CU

// Single-vector launch defaults per q (index q-2): the variant and, for the
// mass operator, the pipeline depth measured fastest (median of interleaved
// timings at about 1e7 DOFs on perturbed box meshes, Gauss q = p+2); orders
// not measured there keep variant 0.
constexpr int kDefVariantDiff[9] = {0, 0, 0, 4, 4, 4, 0, 4, 3};
// FP32 diffusion (the operator inside mixed-precision CG): half the register and LDS footprint
// favours two-element groups at q = 8 (20-27% faster than the FP64 choice at 1e7 and 3e7 nodes);
// the lane-filling groups of q = 6 and 7 are 6% and 6-12% faster than the earlier two-element
// choices; at q = 9 the best choice changes with the mesh size; q = 9 and 10 keep the one-element
// groups that prefetch their factors (the late-factor groups that are the FP64 defaults there
// were measured in FP64 only).
constexpr int kDefVariantDiff32[9] = {0, 0, 0, 4, 4, 4, 3, 1, 0};
constexpr int kDefVariantMass[9] = {0, 0, 0, 3, 3, 1, 3, 0, 4};
constexpr int kDefChainMass[9] = {2, 2, 2, 4, 2, 4, 4, 4, 2};
// Device basis block (elements): B [Q][P], B^T [P][Q], D [Q][Q], D^T [Q][Q],
// then the folded (even-odd) forms of the same four matrices: for a matrix M
// with NO rows and NI columns, row o < ceil(NO/2) holds
//   [ (M[o][i] + M[o][NI-1-i])/2 for i < NI/2 | (M[o][i] - M[o][NI-1-i])/2 for i < NI/2 | M[o][NI/2] if NI odd ].
constexpr int half_up(int n) { return (n + 1) / 2; }
constexpr int basis_b(int, int) { return 0; }
constexpr int basis_bt(int P, int Q) { return Q * P; }
constexpr int basis_d(int P, int Q) { return 2 * Q * P; }
constexpr int basis_dt(int P, int Q) { return 2 * Q * P + Q * Q; }
constexpr int basis_bf(int P, int Q) { return 2 * Q * P + 2 * Q * Q; }
constexpr int basis_btf(int P, int Q) { return basis_bf(P, Q) + half_up(Q) * P; }
constexpr int basis_df(int P, int Q) { return basis_btf(P, Q) + half_up(P) * Q; }
constexpr int basis_dtf(int P, int Q) { return basis_df(P, Q) + half_up(Q) * Q; }
constexpr int basis_xq(int P, int Q) { return basis_dtf(P, Q) + half_up(Q) * Q; }  // quadrature points [Q]
constexpr int basis_wq(int P, int Q) { return basis_xq(P, Q) + Q; }                  // quadrature weights [Q]
// folded G [Q][P] (G[a][i] = l_i'(x_a), the basis derivative at the points) and folded G^T [P][Q]
constexpr int basis_gf(int P, int Q) { return basis_wq(P, Q) + Q; }
constexpr int basis_gtf(int P, int Q) { return basis_gf(P, Q) + half_up(Q) * P; }
constexpr int basis_len(int P, int Q) { return basis_gtf(P, Q) + half_up(P) * Q; }

// Per-order dispatch (one translation unit per order, apply_p<N>.hip).
hipError_t launch_apply(const ApplyLaunch &a);
hipError_t launch_kgrad(const KgradLaunch &a);
hipError_t launch_diag(const DiagLaunch &a);

#define MFHEX_DECLARE_ORDER(N)                                  \
    hipError_t launch_apply_p##N(const ApplyLaunch &a);         \
    hipError_t launch_kgrad_p##N(const KgradLaunch &a);         \
    hipError_t launch_diag_p##N(const DiagLaunch &a);
MFHEX_DECLARE_ORDER(1)
MFHEX_DECLARE_ORDER(2)
MFHEX_DECLARE_ORDER(3)
MFHEX_DECLARE_ORDER(4)
MFHEX_DECLARE_ORDER(5)
MFHEX_DECLARE_ORDER(6)
MFHEX_DECLARE_ORDER(7)
MFHEX_DECLARE_ORDER(8)

// Setup kernels (setup.hip).
struct GeomLaunch {
    int32_t nex, ney, nez, p, q;
    const double *vert;      // device copy of the vertices
    const Basis1D *basis;
    hipStream_t stream;
};
// Quadrature data: diffusion -> 6 factors w adj(J) adj(J)^T / detJ per point,
// mass -> w detJ.  q32 (optional) gets the FP32 rounding, wdet (optional) w detJ.
// bad gets a nonzero value if some detJ <= 0 (caller zeroes it first).
hipError_t launch_qdata(const GeomLaunch &g, int kind, double *q64, float *q32, double *wdet, int32_t *bad);
// Deterministic transposed restriction: y[n][v] (+)= sum of the element values ebuf[e][local][v] of
// the (up to 8) elements holding node n, in increasing element order; masked nodes keep y (add) or
// get 0.  prec: MFHEX_F64 / MFHEX_F32.
hipError_t launch_det_assemble(const GeomLaunch &g, int dirichlet, int nvec, int prec, const void *ebuf, void *y,
                               bool add);
hipError_t launch_offsets(const GeomLaunch &g, int dirichlet, int32_t *off);
hipError_t launch_qpoint_coords(const GeomLaunch &g, double *xyz);
hipError_t launch_node_coords(const GeomLaunch &g, double *xyz);

}  // namespace mfhex
