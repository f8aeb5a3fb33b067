// Fused matrix-free operator kernels for gfx950, templated on the 1D sizes.
//
// One thread group (one wavefront, or two for the largest orders) owns G
// elements and carries them through every stage of the operator without
// leaving the chip: restriction (gather), the 1D basis contractions along x,
// y and z, the pointwise geometric factors, the transposed contractions and
// the scatter-add with hardware atomics.  This is the operator-level fused
// form of Sec. 2 (w_L = A_L u_L with A^e = D^T G^e D: tensor derivatives
// D_r, D_s, D_t and six symmetric factors per point), evaluated by the sum
// factorization of Sec. 1; fusing restriction, basis and pointwise stages
// into one kernel follows the generated fused operator kernels of Sec. 3.
//
// Groups are independent: stages are separated by a wavefront-level sync
// (no workgroup barrier) when a group is one wavefront, so memory latency in
// one group is hidden by the others on the CU.
//
// Contractions ("pencils"): a 1D contraction along one axis is done by lanes
// that each own whole lines (pencils) along that axis, R of them per lane:
// the lane reads its lines from LDS into registers, then walks the output
// index o in a rolled loop; row o of the small 1D matrix is uniform across
// the group, so it is a short scalar load from a device copy of the matrix
// and feeds R x NI fused multiply-adds from scalar registers.  LDS traffic is
// one read per input and one write per output.  An element's LDS array is
// [c][b][a] with an odd row pitch, so lines along x (lane stride = pitch), y
// and z (lane stride 1) are conflict free, and contractions run in place.
//
// Diffusion with Gauss points (q = p+2): interpolate to the points along x,
// y, z (B), take the reference gradient with the collocated derivative on the
// points (D, q x q), apply the 3x3 symmetric factors, and run the transposes
// in reverse order.  With Gauss-Lobatto points collocated at the nodes
// (q = p+1) B is the identity.  Mass: interpolate, scale by w detJ,
// interpolate back.
#pragma once

#include <type_traits>

#include "diag_kernels.hpp"
#include "geom.hpp"
#include "mfhex_internal.h"

namespace mfhex {

template <int Q>
struct Lds {
    static constexpr int PITCH = lds_pitch(Q);
    static constexpr int PLANE = PITCH * Q;
    static constexpr int BUF = lds_buf(Q);
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

// Stage separator.  A one-wavefront group needs no barrier: LDS operations
// of a wavefront complete in order, so only compiler reordering is fenced.
template <int NT>
__device__ __forceinline__ void group_sync()
{
    if constexpr (NT <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        asm volatile("" ::: "memory");
    } else {
        __syncthreads();
    }
}

// Contract axis AX of the G element arrays (extents E0 x E1 x E2 before the
// contraction) from NI = E_AX to NO entries: dst[..o..] = sum_i M[o][i]
// src[..i..] (+ a1[..o..] + a2[..o..] with ADD2).  Every lane handles the same
// lines for a given (AX, extents), so a second contraction along the same axis
// may follow without a sync.
//
// The 1D matrices are centro-symmetric (B, B^T: M[NO-1-o][NI-1-i] = M[o][i],
// SYM = +1) or anti-centro-symmetric (D, D^T: = -M[o][i], SYM = -1), because
// nodes and points are symmetric about 0.  The contraction is evaluated in
// even-odd form: with e_i = v_i + v_{NI-1-i} and d_i = v_i - v_{NI-1-i},
//   E_o = sum_i Me[o][i] e_i (+ M[o][mid] v_mid),  O_o = sum_i Mo[o][i] d_i,
//   out_o = E_o + O_o,   out_{NO-1-o} = SYM (E_o - O_o),   o < ceil(NO/2),
// which halves the multiply-adds; MF points at the folded rows
// [Me[o][0..NI/2) | Mo[o][0..NI/2) | M[o][mid]].  Only the output pairs
// OB <= o < OE (default: all) are formed, so that two halves of a group can
// share one contraction.
template <int AX, int E0, int E1, int E2, int NO, int G, int NT, int Q, int SYM, typename T, bool ADD2 = false,
          int OB = 0, int OE = -1>
__device__ __forceinline__ void contract(const T *src, T *dst, const T *__restrict__ MF, int tid, const T *a1 = nullptr,
                                         const T *a2 = nullptr)
{
    using L = Lds<Q>;
    constexpr int NI = AX == 0 ? E0 : AX == 1 ? E1 : E2;
    constexpr int NA = AX == 0 ? E1 : E0;  // fastest-varying line index
    constexpr int NB = AX == 2 ? E1 : E2;
    constexpr int SA = AX == 0 ? L::PITCH : 1;
    constexpr int SB = AX == 2 ? L::PITCH : L::PLANE;
    constexpr int ST = AX == 0 ? 1 : AX == 1 ? L::PITCH : L::PLANE;  // stride along the line
    constexpr int NPEN = G * NA * NB;
    constexpr int R = (NPEN + NT - 1) / NT;
    constexpr int H = NI / 2, MID = NI & 1, NOH = (NO + 1) / 2;
    T ev[R][H + MID], dv[R][H > 0 ? H : 1];
    int base[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int id = tid + r * NT;
        base[r] = -1;
        if (id < NPEN) {
            const int a = id % NA, t = id / NA, b = t % NB, g = t / NB;
            base[r] = g * L::BUF + a * SA + b * SB;
            T v[NI];
#pragma unroll
            for (int i = 0; i < NI; ++i) v[i] = src[base[r] + i * ST];
#pragma unroll
            for (int i = 0; i < H; ++i) {
                ev[r][i] = v[i] + v[NI - 1 - i];
                dv[r][i] = v[i] - v[NI - 1 - i];
            }
            if constexpr (MID) ev[r][H] = v[H];
        }
    }
    constexpr int OEND = OE < 0 ? NOH : OE;
    // coefficient half-rows in flight per scalar-load wait: about 24 coefficients
    constexpr int UR = NI >= 12 ? 2 : 24 / NI;
#pragma unroll UR
    for (int o = OB; o < OEND; ++o) {
        const T *row = MF + o * NI;
        const int om = NO - 1 - o;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (base[r] >= 0) {
                T E = T(0), O = T(0);
#pragma unroll
                for (int i = 0; i < H; ++i) {
                    E += row[i] * ev[r][i];
                    O += row[H + i] * dv[r][i];
                }
                if constexpr (MID) E += row[2 * H] * ev[r][H];
                T lo = E + O;
                T hi = SYM > 0 ? E - O : O - E;
                if constexpr (ADD2) {
                    lo += a1[base[r] + o * ST] + a2[base[r] + o * ST];
                    hi += a1[base[r] + om * ST] + a2[base[r] + om * ST];
                }
                dst[base[r] + o * ST] = lo;
                if (om != o) dst[base[r] + om * ST] = hi;
            }
        }
    }
}

// Two independent contractions of G cubes Q^3 -> Q^3 with the same folded
// matrix, along x (src0 -> dst0) and along y (src1 -> dst1), taken as one
// list of 2 G Q^2 lines: lanes that one contraction would leave idle take
// lines of the other, and each coefficient row is loaded once for both.  Same
// lane-to-line order within each contraction as contract(); every line is
// read whole before any is written, so either pair may be in place.
template <int Q, int G, int NT, int SYM, typename T>
__device__ __forceinline__ void contract_xy(const T *src0, T *dst0, const T *src1, T *dst1, const T *__restrict__ MF,
                                            int tid)
{
    using L = Lds<Q>;
    constexpr int N1 = G * Q * Q, NPEN = 2 * N1, R = (NPEN + NT - 1) / NT;
    constexpr int H = Q / 2, MID = Q & 1, NOH = (Q + 1) / 2;
    T ev[R][H + MID], dv[R][H > 0 ? H : 1];
    int base[R];
    bool ax1[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int id = tid + r * NT;
        base[r] = -1;
        ax1[r] = id >= N1;
        if (id < NPEN) {
            const int l = ax1[r] ? id - N1 : id;
            const int a = l % Q, t = l / Q, c = t % Q, g = t / Q;
            // x lines start at (0, a, c), y lines at (a, 0, c); the branches keep the strides constant
            // (with G Q^2 a multiple of 64 they are uniform across each wavefront)
            T v[Q];
            if (ax1[r]) {
                base[r] = g * L::BUF + a + c * L::PLANE;
#pragma unroll
                for (int i = 0; i < Q; ++i) v[i] = src1[base[r] + i * L::PITCH];
            } else {
                base[r] = g * L::BUF + a * L::PITCH + c * L::PLANE;
#pragma unroll
                for (int i = 0; i < Q; ++i) v[i] = src0[base[r] + i];
            }
#pragma unroll
            for (int i = 0; i < H; ++i) {
                ev[r][i] = v[i] + v[Q - 1 - i];
                dv[r][i] = v[i] - v[Q - 1 - i];
            }
            if constexpr (MID) ev[r][H] = v[H];
        }
    }
    constexpr int UR = Q >= 12 ? 2 : 24 / Q;
#pragma unroll UR
    for (int o = 0; o < NOH; ++o) {
        const T *row = MF + o * Q;
        const int om = Q - 1 - o;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (base[r] >= 0) {
                T E = T(0), O = T(0);
#pragma unroll
                for (int i = 0; i < H; ++i) {
                    E += row[i] * ev[r][i];
                    O += row[H + i] * dv[r][i];
                }
                if constexpr (MID) E += row[2 * H] * ev[r][H];
                const T lo = E + O, hi = SYM > 0 ? E - O : O - E;
                if (ax1[r]) {
                    dst1[base[r] + o * L::PITCH] = lo;
                    if (om != o) dst1[base[r] + om * L::PITCH] = hi;
                } else {
                    dst0[base[r] + o] = lo;
                    if (om != o) dst0[base[r] + om] = hi;
                }
            }
        }
    }
}

// The x and y contractions of the gradient (and of its transpose) share one
// pass over the lanes when both fit in the group together.
constexpr bool fuse_xy(int Q, int G, int NT) { return 2 * G * Q * Q <= NT; }

// Element groups.  The G elements of a group are consecutive in one x-row of
// elements (the last group of a row may hold fewer), so elements g and g+1
// share their face i = P-1 / i = 0.
struct GroupPos {
    int64_t e0;  // first element
    int nvalid;  // elements of the group inside the row
};

template <int G>
__device__ __forceinline__ GroupPos group_pos(int64_t grp, int nex)
{
    GroupPos gp;
    if constexpr (G == 1) {
        gp.e0 = grp;
        gp.nvalid = 1;
    } else {
        const int64_t gpr = (nex + G - 1) / G;  // groups per row
        const int64_t row = grp / gpr, ex0 = (grp - row * gpr) * G;
        gp.e0 = row * nex + ex0;
        gp.nvalid = (int)(nex - ex0 < G ? nex - ex0 : G);
    }
    return gp;
}

// Restriction and its transpose work on the distinct nodes of a group: P^2
// lines along x of W = G(P-1)+1 nodes, node u = (j + P k) W + X with X the
// position along the line, and with VC vectors the pair id = u VC + vc
// (vector fastest).  Consecutive lanes then touch consecutive doubles of one
// line of x and y, so a gather instruction reads whole cache lines and a
// scatter-add instruction updates them with few requests; a node on a face
// shared inside the group is read once and updated once (its two element
// values are summed on chip first), which saves atomic traffic.
template <int P, int G, int NT, int VC>
struct NodeIO {
    static constexpr int P3 = P * P * P;
    static constexpr int W = G * (P - 1) + 1;  // nodes per x-line of a full group
    static constexpr int NID = W * P * P * VC;
    static constexpr int NR = (NID + NT - 1) / NT;  // (node, vector) pairs per lane
};

// Element g and its local x index i of position X on a line of a group of nvalid elements.
template <int P, int G>
__device__ __forceinline__ void line_pos(int X, int nvalid, int &g, int &i)
{
    if constexpr (G == 1) {
        g = 0;
        i = X;
    } else {
        g = X / (P - 1);
        if (g > nvalid - 1) g = nvalid - 1;
        i = X - g * (P - 1);
    }
}

// Positions X <= nvalid (P-1) of a line belong to the group's elements.
template <int P, int G>
__device__ __forceinline__ bool line_valid(int X, int nvalid)
{
    if constexpr (G == 1) return true;
    else return X <= nvalid * (P - 1);
}

// off[r] = global node of pair tid + r NT, or -1 (masked node, or past the group).
template <int P, int G, int NT, int VC, int NR>
__device__ __forceinline__ void load_offsets(int32_t (&off)[NR], const int32_t *__restrict__ offsets, int64_t e0,
                                             int nvalid, int tid)
{
    static_assert(NR == NodeIO<P, G, NT, VC>::NR, "offset count");
    using IO = NodeIO<P, G, NT, VC>;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int id = tid + r * NT;
        const int u = id / VC, line = u / IO::W, X = u - line * IO::W;
        int g, i;
        line_pos<P, G>(X, nvalid, g, i);
        const int j = line % P, k = line / P;
        // read once per element: streamed past the caches that keep x and y lines
        off[r] = (id < IO::NID && line_valid<P, G>(X, nvalid))
                     ? __builtin_nontemporal_load(&offsets[(e0 + g) * IO::P3 + i + P * (j + P * k)])
                     : -1;
    }
}

// Element values of vectors v0 .. v0+VC-1, first into registers (all loads
// issued before any is used; masked nodes read node 0 and vectors past nvec
// read the last vector), then into s0 (virtual element g VC + vc; a shared
// face node into both elements), where the masked entries are zeroed.  The
// halves are separate so that a pipelined kernel can have the next group's
// loads in flight while it computes.  Elements past nvalid are left unset:
// they are computed on but never scattered.
template <int P, int G, int NT, int VC, typename T, int NR>
__device__ __forceinline__ void gather_load(T (&val)[NR], const int32_t (&off)[NR], const T *__restrict__ x, int nvec,
                                            int v0, int tid)
{
    static_assert(NR == NodeIO<P, G, NT, VC>::NR, "offset count");
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int vc = (tid + r * NT) % VC;
        const int64_t node = off[r] >= 0 ? off[r] : 0;
        val[r] = x[node * nvec + (v0 + vc < nvec ? v0 + vc : nvec - 1)];
    }
}

template <int P, int Q, int G, int NT, int VC, typename T, int NR>
__device__ __forceinline__ void gather_store(T *s0, const T (&val)[NR], const int32_t (&off)[NR], int nvec, int v0,
                                             int nvalid, int tid)
{
    using L = Lds<Q>;
    using IO = NodeIO<P, G, NT, VC>;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int id = tid + r * NT;
        const int vc = id % VC, u = id / VC, line = u / IO::W, X = u - line * IO::W;
        if (id < IO::NID && line_valid<P, G>(X, nvalid)) {
            int g, i;
            line_pos<P, G>(X, nvalid, g, i);
            const int jk = L::PITCH * (line % P) + L::PLANE * (line / P);
            const T v = (off[r] >= 0 && v0 + vc < nvec) ? val[r] : T(0);
            s0[(g * VC + vc) * L::BUF + i + jk] = v;
            if (G > 1 && i == 0 && g > 0) s0[((g - 1) * VC + vc) * L::BUF + (P - 1) + jk] = v;
        }
    }
}

template <int P, int Q, int G, int NT, int VC, typename T, int NR>
__device__ __forceinline__ void gather(T *s0, const int32_t (&off)[NR], const T *__restrict__ x, int nvec, int v0,
                                       int nvalid, int tid)
{
    T val[NR];
    gather_load<P, G, NT, VC>(val, off, x, nvec, v0, tid);
    gather_store<P, Q, G, NT, VC>(s0, val, off, nvec, v0, nvalid, tid);
}

// Transposed restriction: y[node][v0 + vc] += element values (both elements'
// values summed for a face shared inside the group) for unmasked nodes, with
// hardware atomics (nodes on the group boundary are shared with other groups).
//
// Deterministic form (DET, a separate instantiation so that the atomic form
// keeps its registers): no atomics; every element stores its own values at
// ebuf[(e P^3 + local node) nvec + vector] with plain stores (a face node
// shared inside the group is stored once for each of its two elements), and
// k_det_assemble later sums each node's element values in a fixed order.
template <int P, int Q, int G, int NT, int VC, bool DET, typename T, int NR>
__device__ __forceinline__ void scatter_add(const T *s0, const int32_t (&off)[NR], T *__restrict__ y, int nvec, int v0,
                                            int nvalid, int tid, T *__restrict__ ebuf, int64_t e0)
{
    static_assert(NR == NodeIO<P, G, NT, VC>::NR, "offset count");
    using L = Lds<Q>;
    using IO = NodeIO<P, G, NT, VC>;
    if constexpr (DET) {
        constexpr int P3 = P * P * P;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int id = tid + r * NT;
            const int vc = id % VC;
            if (off[r] >= 0 && v0 + vc < nvec) {
                const int u = id / VC, line = u / IO::W, X = u - line * IO::W;
                int g, i;
                line_pos<P, G>(X, nvalid, g, i);
                const int jk = L::PITCH * (line % P) + L::PLANE * (line / P);
                const int ljk = P * line;  // P (j + P k)
                ebuf[((e0 + g) * P3 + i + ljk) * nvec + v0 + vc] = s0[(g * VC + vc) * L::BUF + i + jk];
                if (G > 1 && i == 0 && g > 0)
                    ebuf[((e0 + g - 1) * P3 + (P - 1) + ljk) * nvec + v0 + vc] =
                        s0[((g - 1) * VC + vc) * L::BUF + (P - 1) + jk];
            }
        }
    } else {
        (void)ebuf;
        (void)e0;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int id = tid + r * NT;
            const int vc = id % VC;
            if (off[r] >= 0 && v0 + vc < nvec) {
                const int u = id / VC, line = u / IO::W, X = u - line * IO::W;
                int g, i;
                line_pos<P, G>(X, nvalid, g, i);
                const int jk = L::PITCH * (line % P) + L::PLANE * (line / P);
                T v = s0[(g * VC + vc) * L::BUF + i + jk];
                if (G > 1 && i == 0 && g > 0) v += s0[((g - 1) * VC + vc) * L::BUF + (P - 1) + jk];
                unsafeAtomicAdd(&y[(int64_t)off[r] * nvec + v0 + vc], v);
            }
        }
    }
}

// Nodes (s0) -> values at the points (s0).  Ends with a sync.
template <int P, int Q, bool COLLOC, int G, int NT, typename T>
__device__ __forceinline__ void interp(T *s0, const T *__restrict__ bas, int tid)
{
    if constexpr (!COLLOC) {
        contract<0, P, P, P, Q, G, NT, Q, 1>(s0, s0, bas + basis_bf(P, Q), tid);
        group_sync<NT>();
        contract<1, Q, P, P, Q, G, NT, Q, 1>(s0, s0, bas + basis_bf(P, Q), tid);
        group_sync<NT>();
        contract<2, Q, Q, P, Q, G, NT, Q, 1>(s0, s0, bas + basis_bf(P, Q), tid);
        group_sync<NT>();
    }
}

// Values at the points in s0 -> reference gradient: d/dr in s1, d/ds in s2,
// d/dt in s0.  Ends with a sync.
template <int P, int Q, int G, int NT, typename T>
__device__ __forceinline__ void grad(T *s0, T *s1, T *s2, const T *__restrict__ bas, int tid)
{
    if constexpr (fuse_xy(Q, G, NT)) {
        contract_xy<Q, G, NT, -1>(s0, s1, s0, s2, bas + basis_df(P, Q), tid);
    } else {
        contract<0, Q, Q, Q, Q, G, NT, Q, -1>(s0, s1, bas + basis_df(P, Q), tid);
        contract<1, Q, Q, Q, Q, G, NT, Q, -1>(s0, s2, bas + basis_df(P, Q), tid);
    }
    group_sync<NT>();
    contract<2, Q, Q, Q, Q, G, NT, Q, -1>(s0, s0, bas + basis_df(P, Q), tid);
    group_sync<NT>();
}

// Matrix-core form of the collocated gradient's contractions (Sec. 2.2 puts
// the tensor contractions of a batch of elements on batched small GEMMs).
// Each contraction is a product C = M S of the Q x Q matrix M (D or D^T) with
// S = [Q x lines], 16 lines at a time on the FP64 16x16x4 matrix instruction:
// A = M padded to 16 rows, K = Q in steps of 4 (zero-padded), B = the 4 x 16
// slice of the lines' values.  Lane l holds A[l % 16][4s + l / 16] and
// B[4s + l / 16][l % 16] for step s, and result register r holds
// C[4r + l / 16][l % 16].  The product runs on the unfolded matrix: the matrix
// cores cannot use the even-odd folding, so they issue 16/Q times (rows) and
// 4 ceil(Q/4)/Q times (depth) the products the folded VALU form needs.
constexpr int mx_steps(int Q) { return (Q + 3) / 4; }

// A-operand fragments of the unfolded matrix M, rebuilt from its folded rows
// (see contract): M[o][i] = Me[o][i] + Mo[o][i], M[o][Q-1-i] = Me[o][i] -
// Mo[o][i] (i < Q/2), M[o][mid] = the middle coefficient, for o < ceil(Q/2);
// M[Q-1-o][Q-1-i] = SYM M[o][i].
template <int Q, int SYM>
__device__ __forceinline__ void mx_fragments(const double *__restrict__ MF, double (&a)[mx_steps(Q)], int lane)
{
    constexpr int H = Q / 2, NOH = (Q + 1) / 2;
    const int o = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int s = 0; s < mx_steps(Q); ++s) {
        const int i = 4 * s + kq;
        double m = 0.0;
        if (o < Q && i < Q) {
            const bool top = o < NOH;
            const int oo = top ? o : Q - 1 - o, ii = top ? i : Q - 1 - i;
            const double *row = MF + oo * Q;
            double v;
            if ((Q & 1) && ii == H) v = row[2 * H];
            else if (ii < H) v = row[ii] + row[H + ii];
            else v = row[Q - 1 - ii] - row[H + Q - 1 - ii];
            m = top ? v : SYM * v;
        }
        a[s] = m;
    }
}

// Contract axis AX of the GV cubes Q^3 (same lines and LDS layout as
// contract): dst = M src (+ a1 + a2 with ADD2), in place allowed.  The tiles
// of 16 lines are dealt to the wavefronts of the group; a wavefront reads all
// values of its tile before it writes any, and no two tiles share a line.
template <int AX, int Q, int GV, int NT, bool ADD2 = false>
__device__ __forceinline__ void contract_mx(const double *src, double *dst, const double (&a)[mx_steps(Q)], int tid,
                                            const double *a1 = nullptr, const double *a2 = nullptr)
{
    typedef double d4 __attribute__((ext_vector_type(4)));
    using L = Lds<Q>;
    constexpr int SA = AX == 0 ? L::PITCH : 1;
    constexpr int SB = AX == 2 ? L::PITCH : L::PLANE;
    constexpr int ST = AX == 0 ? 1 : AX == 1 ? L::PITCH : L::PLANE;
    constexpr int NPEN = GV * Q * Q, NTILE = (NPEN + 15) / 16, NW = NT / 64;
    static_assert(NT % 64 == 0 && Q <= 16, "whole wavefronts, at most 16 rows");
    const int lane = tid & 63, w = tid >> 6;
    const int col = lane & 15, kq = lane >> 4;
    for (int t = w; t < NTILE; t += NW) {
        const int id = t * 16 + col;
        const bool ok = id < NPEN;
        const int idc = ok ? id : 0;
        const int la = idc % Q, tt = idc / Q, lb = tt % Q, g = tt / Q;
        const int base = g * L::BUF + la * SA + lb * SB;
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < mx_steps(Q); ++s) {
            const int i = 4 * s + kq;
            const double b = i < Q ? src[base + (i < Q ? i : 0) * ST] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 4 * r + kq;
            if (ok && o < Q) {
                double v = acc[r];
                if constexpr (ADD2) v += a1[base + o * ST] + a2[base + o * ST];
                dst[base + o * ST] = v;
            }
        }
    }
}

// One contraction shared by the two halves of a split group (G elements,
// NT2 threads per half, every line owned by one lane of each half): half 0
// forms output pairs o < OM, half 1 the rest.
template <int AX, int E0, int E1, int E2, int NO, int G, int NT2, int Q, int SYM, typename T, bool ADD2 = false,
          int OM = ((NO + 1) / 2 + 1) / 2>
__device__ __forceinline__ void contract_halves(const T *src, T *dst, const T *__restrict__ MF, int half, int lane,
                                                const T *a1 = nullptr, const T *a2 = nullptr)
{
    constexpr int NOH = (NO + 1) / 2;
    static_assert(G * (E0 * E1 * E2 / (AX == 0 ? E0 : AX == 1 ? E1 : E2)) <= NT2, "one line per lane");
    if (half == 0) contract<AX, E0, E1, E2, NO, G, NT2, Q, SYM, T, ADD2, 0, OM>(src, dst, MF, lane, a1, a2);
    else contract<AX, E0, E1, E2, NO, G, NT2, Q, SYM, T, ADD2, OM, NOH>(src, dst, MF, lane, a1, a2);
}

// ---------------------------------------------------------------------------
// y += A x  (diffusion), or y += B^T (w detJ f) for the load vector.
// VC vectors of the multi-vector travel together (virtual elements g*VC + vc).
// ---------------------------------------------------------------------------
//
// OTF (diffusion, FP64, constant coefficient): no stored factors.  Along a
// trilinear map dx/dr depends on (s, t) only, dx/ds on (r, t) and dx/dt on
// (r, s), so each element's Jacobian is fully described by three tables of
// Q^2 columns, built once per element group in LDS from its 8 vertices; each
// point then reads its three columns and forms w adj(J) adj(J)^T / detJ in
// registers (the same expressions as the set-up kernel), instead of reading
// six factors per point from HBM.
template <int P, int Q, bool COLLOC, int MODE, bool VARK, typename T, int G, int NT, int VC, bool OTF, bool DET,
          bool STAGE = false, int LATE = 0, bool MX = false, int PRE = 0>
__global__ void __launch_bounds__(NT)
k_apply(const T *__restrict__ bas, const int nex, const int ney, const int nvec, const int32_t *__restrict__ offsets,
        const T *__restrict__ qdata, const double *__restrict__ kappa, const double *__restrict__ wdet,
        const double *__restrict__ vert, const T *__restrict__ x, T *__restrict__ y, T *__restrict__ ebuf)
{
    constexpr int Q2 = Q * Q, Q3 = Q2 * Q;
    constexpr int NPT = G * Q3, RQ = (NPT + NT - 1) / NT;
    constexpr int GV = G * VC;
    constexpr bool SPLIT = split_stages(Q, MODE, G, NT, VC);
    constexpr int NT2 = NT / 2;
    static_assert(MODE != kMass, "the mass operator runs in k_mass");
    static_assert(!OTF || (MODE == kDiff && !VARK && VC == 1 && sizeof(T) == 8), "in-kernel factors: FP64 diffusion");
    using L = Lds<Q>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *const s0 = reinterpret_cast<T *>(smem_raw);
    T *const s1 = s0 + GV * L::BUF;
    T *const s2 = s1 + GV * L::BUF;
    T *const s3 = s2 + GV * L::BUF;  // split stages only
    // OTF: element vertices [G][8][3], 1D rule x [Q], w [Q] (one contiguous run), Jacobian columns [G][3][Q^2][3]
    double *const sV = reinterpret_cast<double *>(SPLIT ? s3 + GV * L::BUF : s2 + GV * L::BUF);
    double *const sR = sV + G * 24;
    double *const sJ = sR + 2 * Q;
    // staged scatter of multi-vector chunks: element values [P^3][SC - VC], then offsets [P^3]
    constexpr int P3 = P * P * P;
    static_assert(!STAGE || (staged_scatter(MODE, VC, sizeof(T)) && !DET), "staged scatter: multi-vector diffusion");
    constexpr int SC = scatter_run(VC, sizeof(T));
    T *const sst = s2 + GV * L::BUF;
    int32_t *const soff = reinterpret_cast<int32_t *>(sst + P3 * (SC - VC));
    const int tid = threadIdx.x;
    const int half = tid / NT2, lane = tid - half * NT2;  // split stages: wave-uniform halves
    const GroupPos gpos = group_pos<G>(xcd_block(blockIdx.x, gridDim.x), nex);
    const int64_t e0 = gpos.e0;
    const int nvalid = gpos.nvalid;
    // MX: the collocated gradient and its transpose on the matrix cores (fragments of D and D^T)
    static_assert(!MX || (COLLOC && MODE == kDiff && !SPLIT && !OTF && sizeof(T) == 8), "matrix-core stages");
    double mxd[MX ? mx_steps(Q) : 1], mxt[MX ? mx_steps(Q) : 1];
    if constexpr (MX) {
        mx_fragments<Q, -1>(reinterpret_cast<const double *>(bas) + basis_df(P, Q), mxd, tid & 63);
        mx_fragments<Q, -1>(reinterpret_cast<const double *>(bas) + basis_dtf(P, Q), mxt, tid & 63);
    }
    if constexpr (STAGE) {
        static_assert(G == 1 && !SPLIT && !OTF, "staged scatter: one element, plain stages");
        for (int t = tid; t < P3; t += NT) soff[t] = __builtin_nontemporal_load(&offsets[e0 * P3 + t]);
    }

    int32_t off[NodeIO<P, G, NT, VC>::NR];
    load_offsets<P, G, NT, VC>(off, offsets, e0, nvalid, tid);

    // OTF: the group's vertex coordinates, issued now, stored to LDS after the gather is issued
    constexpr int VR = OTF ? (24 * G + 2 * Q + NT - 1) / NT : 1;
    double vtx[VR];
    if constexpr (OTF) {
#pragma unroll
        for (int r = 0; r < VR; ++r) {
            const int t = tid + r * NT;
            if (t < 24 * G) {
                const int g = t / 24, v = (t % 24) / 3, d = t % 3;
                const int64_t e = g < nvalid ? e0 + g : e0;
                vtx[r] = vert[3 * elem_vertex(e, nex, ney, v) + d];
            } else if (t < 24 * G + 2 * Q) {
                vtx[r] = bas[basis_xq(P, Q) + (t - 24 * G)];  // x [Q] then w [Q], contiguous
            }
        }
    }

    // This lane's geometric factors, loaded once per element group and issued
    // first, so their HBM latency overlaps the gather and the forward
    // contractions, and every chunk of vectors reuses them (LATE > 0: loaded in
    // the pointwise stage instead, LATE points at a time, which keeps their
    // registers free through the contractions; with PRE > 0 the lane's first PRE points are still
    // prefetched and only the rest load late).
    static_assert(LATE == 0 || (VC == 1 && !OTF && MODE == kDiff), "late factor loads: one-vector diffusion");
    static_assert(PRE == 0 || (LATE > 0 && PRE < RQ), "partial prefetch: some points late");
    constexpr int NQD = MODE == kDiff && !OTF && (LATE == 0 || PRE > 0) ? kQdDiff : 0;
    constexpr int KP = LATE == 0 ? RQ : PRE;  // points whose factors are prefetched
    T qv[KP > 0 ? KP : 1][NQD > 0 ? NQD : 1];
    if constexpr (NQD > 0) {
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int id = tid + k * NT < NPT ? tid + k * NT : NPT - 1;
            const int g = id / Q3, pt = id - g * Q3;
            // elements past the end of the row read the first element's data (and scatter nothing)
            const int64_t e = g < nvalid ? e0 + g : e0;
            const T *qd = qdata + e * (NQD * Q3) + pt;
#pragma unroll
            for (int m = 0; m < NQD; ++m) qv[k][m] = __builtin_nontemporal_load(&qd[m * Q3]);
            if constexpr (VARK) {
                const T kap = T(kappa[e * Q3 + pt]);
#pragma unroll
                for (int m = 0; m < NQD; ++m) qv[k][m] *= kap;
            }
        }
    }

    // Chunks of several vectors: the input values of the first chunk are loaded here and each later
    // chunk's right after the previous chunk is in LDS, so their memory latency overlaps that
    // chunk's contractions.  (One-vector groups keep no such registers: at q = 10 they would cost
    // a wavefront per SIMD.)
    constexpr bool PREFETCH = VC > 1 && MODE != kRhs && !OTF;
    T xn[PREFETCH ? NodeIO<P, G, NT, VC>::NR : 1];
    if constexpr (PREFETCH) gather_load<P, G, NT, VC>(xn, off, x, nvec, 0, tid);

    for (int v0 = 0; v0 < nvec; v0 += VC) {
        if constexpr (MODE == kRhs) {
            static_assert(VC == 1, "load vector: one vector");
            const double *f = reinterpret_cast<const double *>(x);
#pragma unroll 4
            for (int k = 0; k < RQ; ++k) {
                const int id = tid + k * NT;
                if (id < NPT) {
                    const int g = id / Q3, pt = id - g * Q3;
                    const int a = pt % Q, b = (pt / Q) % Q, c = pt / Q2;
                    const int64_t gp = (g < nvalid ? e0 + g : e0) * Q3 + pt;
                    s0[g * L::BUF + a + L::PITCH * b + L::PLANE * c] = T(wdet[gp] * f[gp]);
                }
            }
            group_sync<NT>();
        } else {
            if constexpr (OTF) {
                T xv[NodeIO<P, G, NT, VC>::NR];
                gather_load<P, G, NT, VC>(xv, off, x, nvec, v0, tid);
                if (v0 == 0) {
                    // vertices and rule into LDS, then the Jacobian-column tables (the x loads stay in flight)
#pragma unroll
                    for (int r = 0; r < VR; ++r)
                        if (tid + r * NT < 24 * G + 2 * Q) sV[tid + r * NT] = vtx[r];
                    group_sync<NT>();
                    for (int t = tid; t < G * 3 * Q2; t += NT) {
                        const int g = t / (3 * Q2), dir = (t / Q2) % 3, uw = t % Q2;
                        const double u = sR[uw % Q], w = sR[uw / Q];
                        const double *Xg = sV + g * 24;
                        auto X = [&](int v, int d) { return Xg[3 * v + d]; };
                        double j[3];
                        if (dir == 0) jacobian_col<0>(X, u, w, j);
                        else if (dir == 1) jacobian_col<1>(X, u, w, j);
                        else jacobian_col<2>(X, u, w, j);
#pragma unroll
                        for (int d = 0; d < 3; ++d) sJ[3 * t + d] = j[d];
                    }
                }
                gather_store<P, Q, G, NT, VC>(SPLIT && COLLOC ? s3 : s0, xv, off, nvec, v0, nvalid, tid);
            } else if constexpr (PREFETCH) {
                gather_store<P, Q, G, NT, VC>(s0, xn, off, nvec, v0, nvalid, tid);
                if (v0 + VC < nvec) gather_load<P, G, NT, VC>(xn, off, x, nvec, v0 + VC, tid);
            } else {
                gather<P, Q, G, NT, VC, T>(SPLIT && COLLOC ? s3 : s0, off, x, nvec, v0, nvalid, tid);
            }
            group_sync<NT>();
            if constexpr (SPLIT) {
                // nodes (s0) -> points (s3), ping-ponging between s0 and s3
                if constexpr (!COLLOC) {
                    contract_halves<0, P, P, P, Q, G, NT2, Q, 1>(s0, s3, bas + basis_bf(P, Q), half, lane);
                    group_sync<NT>();
                    contract_halves<1, Q, P, P, Q, G, NT2, Q, 1>(s3, s0, bas + basis_bf(P, Q), half, lane);
                    group_sync<NT>();
                    contract_halves<2, Q, Q, P, Q, G, NT2, Q, 1>(s0, s3, bas + basis_bf(P, Q), half, lane);
                    group_sync<NT>();
                }
                // gradient of s3: d/dr -> s1 and the first d/dt rows -> s0 (half 0), d/ds -> s2 and the
                // other d/dt rows (half 1)
                constexpr int NQH = (Q + 1) / 2;
                if (half == 0) {
                    contract<0, Q, Q, Q, Q, G, NT2, Q, -1>(s3, s1, bas + basis_df(P, Q), lane);
                    contract<2, Q, Q, Q, Q, G, NT2, Q, -1, T, false, 0, NQH / 2>(s3, s0, bas + basis_df(P, Q), lane);
                } else {
                    contract<1, Q, Q, Q, Q, G, NT2, Q, -1>(s3, s2, bas + basis_df(P, Q), lane);
                    contract<2, Q, Q, Q, Q, G, NT2, Q, -1, T, false, NQH / 2, NQH>(s3, s0, bas + basis_df(P, Q),
                                                                                     lane);
                }
                group_sync<NT>();
            } else if constexpr (MX) {
                double *const d0 = reinterpret_cast<double *>(s0);
                contract_mx<0, Q, GV, NT>(d0, reinterpret_cast<double *>(s1), mxd, tid);
                contract_mx<1, Q, GV, NT>(d0, reinterpret_cast<double *>(s2), mxd, tid);
                group_sync<NT>();
                contract_mx<2, Q, GV, NT>(d0, d0, mxd, tid);
                group_sync<NT>();
            } else {
                interp<P, Q, COLLOC, GV, NT, T>(s0, bas, tid);
                grad<P, Q, GV, NT, T>(s0, s1, s2, bas, tid);
            }
            {
                // split stages write d/dt's factor product to s3 (s0 is the transposed gradient's output)
                T *const st = SPLIT ? s3 : s0;
                // one point: prefetched factors (LT = false) or factors loaded here (LT = true)
                auto point = [&](int k, auto late_tag) {
                    constexpr bool LT = decltype(late_tag)::value;
                    const int id = tid + k * NT;
                    if (id < NPT) {
                        const int g = id / Q3, pt = id - g * Q3;
                        const int a = pt % Q, b = (pt / Q) % Q, c = pt / Q2;
                        const int loc = a + L::PITCH * b + L::PLANE * c;
                        const T *gm = qv[0];
                        if constexpr (!LT && NQD > 0) gm = qv[k];
                        T gl[kQdDiff];
                        if constexpr (LT) {
                            const int64_t e = g < nvalid ? e0 + g : e0;
                            const T *qd = qdata + e * (kQdDiff * Q3) + pt;
#pragma unroll
                            for (int m = 0; m < kQdDiff; ++m) gl[m] = __builtin_nontemporal_load(&qd[m * Q3]);
                            if constexpr (VARK) {
                                const T kap = T(kappa[e * Q3 + pt]);
#pragma unroll
                                for (int m = 0; m < kQdDiff; ++m) gl[m] *= kap;
                            }
                            gm = gl;
                        }
                        double gotf[kQdDiff];
                        if constexpr (OTF) {
                            // columns dx/dr at (b, c), dx/ds at (a, c), dx/dt at (a, b) of element g
                            const double *Jg = sJ + g * 9 * Q2;
                            const double *jr = Jg + 3 * (b + Q * c), *js = Jg + 3 * (Q2 + a + Q * c),
                                         *jt = Jg + 3 * (2 * Q2 + a + Q * b);
                            const double wq = sR[Q + a] * sR[Q + b] * sR[Q + c];
                            diffusion_factors(jr, js, jt, wq, gotf);
                            gm = gotf;
                        }
#pragma unroll
                        for (int vc = 0; vc < VC; ++vc) {
                            const int ls = (g * VC + vc) * L::BUF + loc;
                            const T ur = s1[ls], us = s2[ls], ut = s0[ls];
                            s1[ls] = gm[0] * ur + gm[5] * us + gm[4] * ut;
                            s2[ls] = gm[5] * ur + gm[1] * us + gm[3] * ut;
                            st[ls] = gm[4] * ur + gm[3] * us + gm[2] * ut;
                        }
                    }
                };
                if constexpr (LATE == 0) {
#pragma unroll
                    for (int k = 0; k < RQ; ++k) point(k, std::false_type{});
                } else {
#pragma unroll
                    for (int k = 0; k < PRE; ++k) point(k, std::false_type{});
#pragma unroll(LATE > 0 ? LATE : 1)
                    for (int k = PRE; k < RQ; ++k) point(k, std::true_type{});
                }
                group_sync<NT>();
                if constexpr (SPLIT) {
                    // transposed gradient: x lines of s1 (half 0) and y lines of s2 (half 1) in place,
                    // then the z lines of s3 with both added, into s0, shared by the halves
                    if (half == 0) contract<0, Q, Q, Q, Q, G, NT2, Q, -1>(s1, s1, bas + basis_dtf(P, Q), lane);
                    else contract<1, Q, Q, Q, Q, G, NT2, Q, -1>(s2, s2, bas + basis_dtf(P, Q), lane);
                    group_sync<NT>();
                    contract_halves<2, Q, Q, Q, Q, G, NT2, Q, -1, T, true>(s3, s0, bas + basis_dtf(P, Q), half, lane,
                                                                          s1, s2);
                    if constexpr (!COLLOC) group_sync<NT>();
                } else {
                    // transposed gradient: x and y lines in place, then the z lines
                    // of s0 with the x and y parts added
                    if constexpr (MX) {
                        double *const d1 = reinterpret_cast<double *>(s1), *const d2 = reinterpret_cast<double *>(s2);
                        contract_mx<0, Q, GV, NT>(d1, d1, mxt, tid);
                        contract_mx<1, Q, GV, NT>(d2, d2, mxt, tid);
                    } else if constexpr (fuse_xy(Q, GV, NT)) {
                        contract_xy<Q, GV, NT, -1>(s1, s1, s2, s2, bas + basis_dtf(P, Q), tid);
                    } else {
                        contract<0, Q, Q, Q, Q, GV, NT, Q, -1>(s1, s1, bas + basis_dtf(P, Q), tid);
                        contract<1, Q, Q, Q, Q, GV, NT, Q, -1>(s2, s2, bas + basis_dtf(P, Q), tid);
                    }
                    group_sync<NT>();
                    if constexpr (MX)
                        contract_mx<2, Q, GV, NT, true>(reinterpret_cast<double *>(s0), reinterpret_cast<double *>(s0),
                                                        mxt, tid, reinterpret_cast<const double *>(s1),
                                                        reinterpret_cast<const double *>(s2));
                    else
                        contract<2, Q, Q, Q, Q, GV, NT, Q, -1, T, true>(s0, s0, bas + basis_dtf(P, Q), tid, s1, s2);
                    // same lines, same lanes: B^T along z follows without a sync
                }
            }
        }
        // transposed interpolation back to the nodes
        T *sout = s0;
        if constexpr (!COLLOC) {
            if constexpr (SPLIT) {
                contract_halves<2, Q, Q, Q, P, G, NT2, Q, 1>(s0, s3, bas + basis_btf(P, Q), half, lane);
                group_sync<NT>();
                contract_halves<1, Q, Q, P, P, G, NT2, Q, 1>(s3, s0, bas + basis_btf(P, Q), half, lane);
                group_sync<NT>();
                contract_halves<0, Q, P, P, P, G, NT2, Q, 1>(s0, s3, bas + basis_btf(P, Q), half, lane);
                sout = s3;
            } else {
                contract<2, Q, Q, Q, P, GV, NT, Q, 1>(s0, s0, bas + basis_btf(P, Q), tid);
                group_sync<NT>();
                contract<1, Q, Q, P, P, GV, NT, Q, 1>(s0, s0, bas + basis_btf(P, Q), tid);
                group_sync<NT>();
                contract<0, Q, P, P, P, GV, NT, Q, 1>(s0, s0, bas + basis_btf(P, Q), tid);
            }
        }
        group_sync<NT>();
        if constexpr (STAGE) {
            // the run of vectors this chunk belongs to: [r0, r0 + SC); nst of them are staged already
            const int r0 = v0 - v0 % SC, nst = v0 - r0;
            if ((v0 + VC) % SC != 0 && v0 + VC < nvec) {
                // not the run's last chunk: keep its element values
                for (int t = tid; t < P3 * VC; t += NT) {
                    const int vc = t % VC, u = t / VC;
                    const int i = u % P, j = (u / P) % P, k = u / (P * P);
                    sst[u * (SC - VC) + nst + vc] = sout[vc * L::BUF + i + L::PITCH * j + L::PLANE * k];
                }
            } else {
                // the run's last chunk: add all its vectors, consecutive lanes on consecutive vectors of a node
                const int run = nst + VC;
                for (int t = tid; t < P3 * run; t += NT) {
                    const int w = t % run, u = t / run;
                    const int32_t o = soff[u];
                    if (o >= 0 && r0 + w < nvec) {
                        const int i = u % P, j = (u / P) % P, k = u / (P * P);
                        const T v = w < nst ? sst[u * (SC - VC) + w]
                                            : sout[(w - nst) * L::BUF + i + L::PITCH * j + L::PLANE * k];
                        unsafeAtomicAdd(&y[(int64_t)o * nvec + r0 + w], v);
                    }
                }
            }
        } else {
            scatter_add<P, Q, G, NT, VC, DET, T>(sout, off, y, nvec, v0, nvalid, tid, ebuf, e0);
        }
        group_sync<NT>();
    }
}

// ---------------------------------------------------------------------------
// y += M x  (mass).  A thread group works through `chain` consecutive element
// groups (and, per group, the chunks of VC vectors) as a software pipeline:
// the offsets of the next group are loaded when the current one starts, and
// its point weights (into the registers the current group has just used) and
// its input values right after the current pointwise scaling, so that their
// memory latency is hidden by the transposed interpolation and the
// scatter-add.  With one basis pass each way the mass operator has too little
// arithmetic per byte to hide that latency otherwise.
// ---------------------------------------------------------------------------
template <int Q, int G, int NT, typename T, int RQ>
__device__ __forceinline__ void load_mass_weights(T (&w)[RQ], const T *__restrict__ qdata, int64_t e0, int nvalid,
                                                  int tid)
{
    constexpr int Q3 = Q * Q * Q, NPT = G * Q3;
#pragma unroll
    for (int k = 0; k < RQ; ++k) {
        const int id = tid + k * NT < NPT ? tid + k * NT : NPT - 1;
        const int g = id / Q3, pt = id - g * Q3;
        const int64_t e = g < nvalid ? e0 + g : e0;  // past the end of the row: the first element's (scatters nothing)
        w[k] = __builtin_nontemporal_load(&qdata[e * Q3 + pt]);
    }
}

template <int P, int Q, bool COLLOC, typename T, int G, int NT, int VC, bool DET>
__global__ void __launch_bounds__(NT)
k_mass(const T *__restrict__ bas, const int nex, const int64_t ngroups, const int nvec, const int chain,
       const int32_t *__restrict__ offsets, const T *__restrict__ qdata, const T *__restrict__ x, T *__restrict__ y,
       T *__restrict__ ebuf)
{
    constexpr int Q2 = Q * Q, Q3 = Q2 * Q;
    constexpr int NPT = G * Q3, RQ = (NPT + NT - 1) / NT;
    constexpr int GV = G * VC;
    constexpr int NR = NodeIO<P, G, NT, VC>::NR;
    using L = Lds<Q>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *const s0 = reinterpret_cast<T *>(smem_raw);
    const int tid = threadIdx.x;
    int64_t grp = xcd_block(blockIdx.x, gridDim.x) * chain;
    const int64_t gend = grp + chain < ngroups ? grp + chain : ngroups;

    GroupPos gpos = group_pos<G>(grp, nex), npos = gpos;
    int32_t off[NR], offn[NR];
    load_offsets<P, G, NT, VC>(off, offsets, gpos.e0, gpos.nvalid, tid);
    T w[RQ], xv[NR];
    load_mass_weights<Q, G, NT>(w, qdata, gpos.e0, gpos.nvalid, tid);
    gather_load<P, G, NT, VC>(xv, off, x, nvec, 0, tid);

    for (int v0 = 0;;) {
        // the next work item: the next chunk of vectors, else the next group
        int nv0 = v0 + VC;
        int64_t ngrp = grp;
        if (nv0 >= nvec) {
            nv0 = 0;
            ngrp = grp + 1;
        }
        const bool more = ngrp < gend, newgrp = more && ngrp != grp;
        if (newgrp) {
            npos = group_pos<G>(ngrp, nex);
            load_offsets<P, G, NT, VC>(offn, offsets, npos.e0, npos.nvalid, tid);
        }
        gather_store<P, Q, G, NT, VC>(s0, xv, off, nvec, v0, gpos.nvalid, tid);
        group_sync<NT>();
        // the next chunk of the same group needs no new offsets: load it now
        if (more && !newgrp) gather_load<P, G, NT, VC>(xv, off, x, nvec, nv0, tid);
        interp<P, Q, COLLOC, GV, NT, T>(s0, bas, tid);
#pragma unroll
        for (int k = 0; k < RQ; ++k) {
            const int id = tid + k * NT;
            if (id < NPT) {
                const int g = id / Q3, pt = id - g * Q3;
                const int a = pt % Q, b = (pt / Q) % Q, c = pt / Q2;
                const int loc = a + L::PITCH * b + L::PLANE * c;
#pragma unroll
                for (int vc = 0; vc < VC; ++vc) s0[(g * VC + vc) * L::BUF + loc] *= w[k];
            }
        }
        group_sync<NT>();
        if (newgrp) {
            load_mass_weights<Q, G, NT>(w, qdata, npos.e0, npos.nvalid, tid);
            gather_load<P, G, NT, VC>(xv, offn, x, nvec, 0, tid);
        }
        if constexpr (!COLLOC) {
            contract<2, Q, Q, Q, P, GV, NT, Q, 1>(s0, s0, bas + basis_btf(P, Q), tid);
            group_sync<NT>();
            contract<1, Q, Q, P, P, GV, NT, Q, 1>(s0, s0, bas + basis_btf(P, Q), tid);
            group_sync<NT>();
            contract<0, Q, P, P, P, GV, NT, Q, 1>(s0, s0, bas + basis_btf(P, Q), tid);
        }
        group_sync<NT>();
        scatter_add<P, Q, G, NT, VC, DET, T>(s0, off, y, nvec, v0, gpos.nvalid, tid, ebuf, gpos.e0);
        group_sync<NT>();
        if (!more) break;
        if (newgrp) {
#pragma unroll
            for (int r = 0; r < NR; ++r) off[r] = offn[r];
            gpos = npos;
        }
        grp = ngrp;
        v0 = nv0;
    }
}

// ---------------------------------------------------------------------------
// Coefficient gradient g[e][pt] = (Dhat r)^T G0 (Dhat u) at every point.
// ---------------------------------------------------------------------------
template <int P, int Q, bool COLLOC, int G, int NT>
__global__ void __launch_bounds__(NT)
k_kgrad(const double *__restrict__ bas, const int64_t nelem, const int32_t *__restrict__ offsets,
        const double *__restrict__ qdata, const double *__restrict__ u, const double *__restrict__ r,
        double *__restrict__ gout)
{
    using T = double;
    constexpr int Q2 = Q * Q, Q3 = Q2 * Q;
    constexpr int NPT = G * Q3, RQ = (NPT + NT - 1) / NT;
    using L = Lds<Q>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *const s0 = reinterpret_cast<T *>(smem_raw);
    T *const s1 = s0 + G * L::BUF;
    T *const s2 = s1 + G * L::BUF;
    T *const t0 = s2 + G * L::BUF;
    T *const t1 = t0 + G * L::BUF;
    T *const t2 = t1 + G * L::BUF;
    const int tid = threadIdx.x;
    const int64_t e0 = xcd_block(blockIdx.x, gridDim.x) * G;
    int32_t off[NodeIO<P, G, NT, 1>::NR];
    static_assert(G == 1, "one element per group");
    load_offsets<P, G, NT, 1>(off, offsets, e0, 1, tid);
    gather<P, Q, G, NT, 1, T>(s0, off, u, 1, 0, 1, tid);
    gather<P, Q, G, NT, 1, T>(t0, off, r, 1, 0, 1, tid);
    group_sync<NT>();
    interp<P, Q, COLLOC, G, NT, T>(s0, bas, tid);
    interp<P, Q, COLLOC, G, NT, T>(t0, bas, tid);
    grad<P, Q, G, NT, T>(s0, s1, s2, bas, tid);
    grad<P, Q, G, NT, T>(t0, t1, t2, bas, tid);
#pragma unroll 4
    for (int k = 0; k < RQ; ++k) {
        const int id = tid + k * NT;
        if (id < NPT) {
            const int g = id / Q3, pt = id - g * Q3;
            if (e0 + g < nelem) {
                const int a = pt % Q, b = (pt / Q) % Q, c = pt / Q2;
                const int ls = g * L::BUF + a + L::PITCH * b + L::PLANE * c;
                const T *qd = qdata + (e0 + g) * (kQdDiff * Q3) + pt;
                T gm[kQdDiff];
#pragma unroll
                for (int m = 0; m < kQdDiff; ++m) gm[m] = __builtin_nontemporal_load(&qd[m * Q3]);
                const T ur = s1[ls], us = s2[ls], ut = s0[ls];
                const T vr = gm[0] * ur + gm[5] * us + gm[4] * ut;
                const T vs = gm[5] * ur + gm[1] * us + gm[3] * ut;
                const T vt = gm[4] * ur + gm[3] * us + gm[2] * ut;
                __builtin_nontemporal_store(t1[ls] * vr + t2[ls] * vs + t0[ls] * vt, &gout[(e0 + g) * Q3 + pt]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// y += A x (diffusion, Gauss points, q = p+2) with the gradient factored
// through the basis derivative at the points, G[a][i] = l_i'(x_a):
//   u_r = (G (x) B (x) B) u,  u_s = (B (x) G (x) B) u,  u_t = (B (x) B (x) G) u
// (x fastest in the Kronecker products), and back
//   y = (G^T B^T B^T) v_r + (B^T G^T B^T) v_s + (B^T B^T G^T) v_t.
// Sharing the partial products, the whole operator is six contraction
// stages instead of twelve: z (B u and G u), y (B and G of the first, B of
// the second), x (G, B, B), then the pointwise factors, and x (G^T, B^T,
// B^T), y (B^T + G^T, B^T), z (B^T + G^T).  Each stage reads every line it
// owns once from LDS and forms two or three contractions from it, so there
// are half as many stage barriers and about 40% less LDS traffic, at the
// cost of about 20% more multiply-adds (G is Q x P where the collocated
// derivative D is Q x Q, but it is applied to P-long lines).  Same element
// groups, restriction, even-odd folding and factor prefetch as k_apply.
// ---------------------------------------------------------------------------

// One line of NI values, folded: e_i = v_i + v_{NI-1-i}, d_i = v_i - v_{NI-1-i} (i < NI/2), e_{NI/2} = v_mid.
template <int NI, typename T>
struct FLine {
    static constexpr int H = NI / 2, MID = NI & 1;
    T e[H + MID];
    T d[H > 0 ? H : 1];
};

template <int NI, int ST, typename T>
__device__ __forceinline__ void fold_line(const T *src, int base, FLine<NI, T> &f)
{
    constexpr int H = NI / 2;
    T v[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) v[i] = src[base + i * ST];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        f.e[i] = v[i] + v[NI - 1 - i];
        f.d[i] = v[i] - v[NI - 1 - i];
    }
    if constexpr (NI & 1) f.e[H] = v[H];
}

// Even and odd half-sums of one folded row against a folded line: out_o = E + O and
// out_{NO-1-o} = SYM (E - O).
template <int NI, typename T>
__device__ __forceinline__ void fdot(const T *__restrict__ row, const FLine<NI, T> &f, T &E, T &O)
{
    constexpr int H = NI / 2;
    E = T(0);
    O = T(0);
#pragma unroll
    for (int i = 0; i < H; ++i) {
        E += row[i] * f.e[i];
        O += row[H + i] * f.d[i];
    }
    if constexpr (NI & 1) E += row[2 * H] * f.e[H];
}

// Lines along axis AX of G element arrays with extents (E0, E1, E2) (same lane-to-line order as contract()).
template <int AX, int E0, int E1, int E2, int G, int NT, int Q>
struct LineSet {
    using L = Lds<Q>;
    static constexpr int NI = AX == 0 ? E0 : AX == 1 ? E1 : E2;
    static constexpr int NA = AX == 0 ? E1 : E0;
    static constexpr int NB = AX == 2 ? E1 : E2;
    static constexpr int SA = AX == 0 ? L::PITCH : 1;
    static constexpr int SB = AX == 2 ? L::PITCH : L::PLANE;
    static constexpr int ST = AX == 0 ? 1 : AX == 1 ? L::PITCH : L::PLANE;
    static constexpr int NPEN = G * NA * NB;
    static constexpr int R = (NPEN + NT - 1) / NT;
    __device__ static __forceinline__ int base(int id)
    {
        const int a = id % NA, t = id / NA, b = t % NB, g = t / NB;
        return g * L::BUF + a * SA + b * SB;
    }
};

// Forward z: A (nodes) -> A = B_z u, Bb = G_z u.
template <int P, int Q, int G, int NT, typename T>
__device__ __forceinline__ void gf_z(T *A, T *Bb, const T *__restrict__ bas, int tid)
{
    using LS = LineSet<2, P, P, P, G, NT, Q>;
    constexpr int NOH = (Q + 1) / 2, UR = 2;
    FLine<P, T> f[LS::R];
    int base[LS::R];
#pragma unroll
    for (int r = 0; r < LS::R; ++r) {
        const int id = tid + r * NT;
        base[r] = id < LS::NPEN ? LS::base(id) : -1;
        if (base[r] >= 0) fold_line<P, LS::ST>(A, base[r], f[r]);
    }
    const T *bf = bas + basis_bf(P, Q), *gf = bas + basis_gf(P, Q);
#pragma unroll UR
    for (int o = 0; o < NOH; ++o) {
        const int om = Q - 1 - o;
#pragma unroll
        for (int r = 0; r < LS::R; ++r) {
            if (base[r] < 0) continue;
            T E, O;
            fdot<P>(bf + o * P, f[r], E, O);
            A[base[r] + o * LS::ST] = E + O;
            if (om != o) A[base[r] + om * LS::ST] = E - O;
            fdot<P>(gf + o * P, f[r], E, O);
            Bb[base[r] + o * LS::ST] = E + O;
            if (om != o) Bb[base[r] + om * LS::ST] = O - E;
        }
    }
}

// Forward y: A (B_z u), Bb (G_z u) -> A = B_y A, C = G_y A, Bb = B_y Bb.
template <int P, int Q, int G, int NT, typename T>
__device__ __forceinline__ void gf_y(T *A, T *Bb, T *C, const T *__restrict__ bas, int tid)
{
    using LS = LineSet<1, P, P, Q, G, NT, Q>;
    constexpr int NOH = (Q + 1) / 2, UR = 2;
    FLine<P, T> fa[LS::R], fb[LS::R];
    int base[LS::R];
#pragma unroll
    for (int r = 0; r < LS::R; ++r) {
        const int id = tid + r * NT;
        base[r] = id < LS::NPEN ? LS::base(id) : -1;
        if (base[r] >= 0) {
            fold_line<P, LS::ST>(A, base[r], fa[r]);
            fold_line<P, LS::ST>(Bb, base[r], fb[r]);
        }
    }
    const T *bf = bas + basis_bf(P, Q), *gf = bas + basis_gf(P, Q);
#pragma unroll UR
    for (int o = 0; o < NOH; ++o) {
        const int om = Q - 1 - o;
#pragma unroll
        for (int r = 0; r < LS::R; ++r) {
            if (base[r] < 0) continue;
            T E, O;
            fdot<P>(bf + o * P, fa[r], E, O);
            A[base[r] + o * LS::ST] = E + O;
            if (om != o) A[base[r] + om * LS::ST] = E - O;
            fdot<P>(gf + o * P, fa[r], E, O);
            C[base[r] + o * LS::ST] = E + O;
            if (om != o) C[base[r] + om * LS::ST] = O - E;
            fdot<P>(bf + o * P, fb[r], E, O);
            Bb[base[r] + o * LS::ST] = E + O;
            if (om != o) Bb[base[r] + om * LS::ST] = E - O;
        }
    }
}

// Forward x: A, C, Bb -> A = G_x A (d/dr), C = B_x C (d/ds), Bb = B_x Bb (d/dt), all at the points.
template <int P, int Q, int G, int NT, typename T>
__device__ __forceinline__ void gf_x(T *A, T *Bb, T *C, const T *__restrict__ bas, int tid)
{
    using LS = LineSet<0, P, Q, Q, G, NT, Q>;
    constexpr int NOH = (Q + 1) / 2, UR = 1;
    FLine<P, T> fa[LS::R], fb[LS::R], fc[LS::R];
    int base[LS::R];
#pragma unroll
    for (int r = 0; r < LS::R; ++r) {
        const int id = tid + r * NT;
        base[r] = id < LS::NPEN ? LS::base(id) : -1;
        if (base[r] >= 0) {
            fold_line<P, LS::ST>(A, base[r], fa[r]);
            fold_line<P, LS::ST>(Bb, base[r], fb[r]);
            fold_line<P, LS::ST>(C, base[r], fc[r]);
        }
    }
    const T *bf = bas + basis_bf(P, Q), *gf = bas + basis_gf(P, Q);
#pragma unroll UR
    for (int o = 0; o < NOH; ++o) {
        const int om = Q - 1 - o;
#pragma unroll
        for (int r = 0; r < LS::R; ++r) {
            if (base[r] < 0) continue;
            T E, O;
            fdot<P>(gf + o * P, fa[r], E, O);
            A[base[r] + o] = E + O;
            if (om != o) A[base[r] + om] = O - E;
            fdot<P>(bf + o * P, fc[r], E, O);
            C[base[r] + o] = E + O;
            if (om != o) C[base[r] + om] = E - O;
            fdot<P>(bf + o * P, fb[r], E, O);
            Bb[base[r] + o] = E + O;
            if (om != o) Bb[base[r] + om] = E - O;
        }
    }
}

// Transposed x: A (v_r), C (v_s), Bb (v_t) at the points -> A = G_x^T A, C = B_x^T C, Bb = B_x^T Bb.
template <int P, int Q, int G, int NT, typename T>
__device__ __forceinline__ void gf_xt(T *A, T *Bb, T *C, const T *__restrict__ bas, int tid)
{
    using LS = LineSet<0, Q, Q, Q, G, NT, Q>;
    constexpr int NOH = (P + 1) / 2, UR = 1;
    FLine<Q, T> fa[LS::R], fb[LS::R], fc[LS::R];
    int base[LS::R];
#pragma unroll
    for (int r = 0; r < LS::R; ++r) {
        const int id = tid + r * NT;
        base[r] = id < LS::NPEN ? LS::base(id) : -1;
        if (base[r] >= 0) {
            fold_line<Q, LS::ST>(A, base[r], fa[r]);
            fold_line<Q, LS::ST>(Bb, base[r], fb[r]);
            fold_line<Q, LS::ST>(C, base[r], fc[r]);
        }
    }
    const T *btf = bas + basis_btf(P, Q), *gtf = bas + basis_gtf(P, Q);
#pragma unroll UR
    for (int o = 0; o < NOH; ++o) {
        const int om = P - 1 - o;
#pragma unroll
        for (int r = 0; r < LS::R; ++r) {
            if (base[r] < 0) continue;
            T E, O;
            fdot<Q>(gtf + o * Q, fa[r], E, O);
            A[base[r] + o] = E + O;
            if (om != o) A[base[r] + om] = O - E;
            fdot<Q>(btf + o * Q, fc[r], E, O);
            C[base[r] + o] = E + O;
            if (om != o) C[base[r] + om] = E - O;
            fdot<Q>(btf + o * Q, fb[r], E, O);
            Bb[base[r] + o] = E + O;
            if (om != o) Bb[base[r] + om] = E - O;
        }
    }
}

// Transposed y: A, C, Bb (nodes along x, points along y and z) -> A = B_y^T A + G_y^T C, Bb = B_y^T Bb.
template <int P, int Q, int G, int NT, typename T>
__device__ __forceinline__ void gf_yt(T *A, T *Bb, const T *C, const T *__restrict__ bas, int tid)
{
    using LS = LineSet<1, P, Q, Q, G, NT, Q>;
    constexpr int NOH = (P + 1) / 2, UR = 1;
    FLine<Q, T> fa[LS::R], fb[LS::R], fc[LS::R];
    int base[LS::R];
#pragma unroll
    for (int r = 0; r < LS::R; ++r) {
        const int id = tid + r * NT;
        base[r] = id < LS::NPEN ? LS::base(id) : -1;
        if (base[r] >= 0) {
            fold_line<Q, LS::ST>(A, base[r], fa[r]);
            fold_line<Q, LS::ST>(Bb, base[r], fb[r]);
            fold_line<Q, LS::ST>(C, base[r], fc[r]);
        }
    }
    const T *btf = bas + basis_btf(P, Q), *gtf = bas + basis_gtf(P, Q);
#pragma unroll UR
    for (int o = 0; o < NOH; ++o) {
        const int om = P - 1 - o;
#pragma unroll
        for (int r = 0; r < LS::R; ++r) {
            if (base[r] < 0) continue;
            T E1, O1, E2, O2;
            fdot<Q>(btf + o * Q, fa[r], E1, O1);
            fdot<Q>(gtf + o * Q, fc[r], E2, O2);
            A[base[r] + o * LS::ST] = (E1 + O1) + (E2 + O2);
            if (om != o) A[base[r] + om * LS::ST] = (E1 - O1) + (O2 - E2);
            fdot<Q>(btf + o * Q, fb[r], E1, O1);
            Bb[base[r] + o * LS::ST] = E1 + O1;
            if (om != o) Bb[base[r] + om * LS::ST] = E1 - O1;
        }
    }
}

// Transposed z: A, Bb (nodes along x and y, points along z) -> A = B_z^T A + G_z^T Bb (element values).
template <int P, int Q, int G, int NT, typename T>
__device__ __forceinline__ void gf_zt(T *A, const T *Bb, const T *__restrict__ bas, int tid)
{
    using LS = LineSet<2, P, P, Q, G, NT, Q>;
    constexpr int NOH = (P + 1) / 2, UR = 2;
    FLine<Q, T> fa[LS::R], fb[LS::R];
    int base[LS::R];
#pragma unroll
    for (int r = 0; r < LS::R; ++r) {
        const int id = tid + r * NT;
        base[r] = id < LS::NPEN ? LS::base(id) : -1;
        if (base[r] >= 0) {
            fold_line<Q, LS::ST>(A, base[r], fa[r]);
            fold_line<Q, LS::ST>(Bb, base[r], fb[r]);
        }
    }
    const T *btf = bas + basis_btf(P, Q), *gtf = bas + basis_gtf(P, Q);
#pragma unroll UR
    for (int o = 0; o < NOH; ++o) {
        const int om = P - 1 - o;
#pragma unroll
        for (int r = 0; r < LS::R; ++r) {
            if (base[r] < 0) continue;
            T E1, O1, E2, O2;
            fdot<Q>(btf + o * Q, fa[r], E1, O1);
            fdot<Q>(gtf + o * Q, fb[r], E2, O2);
            A[base[r] + o * LS::ST] = (E1 + O1) + (E2 + O2);
            if (om != o) A[base[r] + om * LS::ST] = (E1 - O1) + (O2 - E2);
        }
    }
}

// PF: the lane's geometric factors are loaded at the start of the element group (as in k_apply);
// otherwise in the pointwise stage, keeping their registers free through the forward stages.
template <int P, int Q, bool VARK, typename T, int G, int NT, bool PF, bool DET>
__global__ void __launch_bounds__(NT)
k_apply_gf(const T *__restrict__ bas, const int nex, const int nvec, const int32_t *__restrict__ offsets,
           const T *__restrict__ qdata, const double *__restrict__ kappa, const T *__restrict__ x, T *__restrict__ y,
           T *__restrict__ ebuf)
{
    constexpr int Q2 = Q * Q, Q3 = Q2 * Q;
    constexpr int NPT = G * Q3, RQ = (NPT + NT - 1) / NT;
    using L = Lds<Q>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *const A = reinterpret_cast<T *>(smem_raw);
    T *const Bb = A + G * L::BUF;
    T *const C = Bb + G * L::BUF;
    const int tid = threadIdx.x;
    const GroupPos gpos = group_pos<G>(xcd_block(blockIdx.x, gridDim.x), nex);
    const int64_t e0 = gpos.e0;
    const int nvalid = gpos.nvalid;

    int32_t off[NodeIO<P, G, NT, 1>::NR];
    load_offsets<P, G, NT, 1>(off, offsets, e0, nvalid, tid);

    // factors of the points of this lane (elements past the end of the row read the first element's)
    auto load_factors = [&](T (&qv)[RQ][kQdDiff]) {
#pragma unroll
        for (int k = 0; k < RQ; ++k) {
            const int id = tid + k * NT < NPT ? tid + k * NT : NPT - 1;
            const int g = id / Q3, pt = id - g * Q3;
            const int64_t e = g < nvalid ? e0 + g : e0;
            const T *qd = qdata + e * (kQdDiff * Q3) + pt;
#pragma unroll
            for (int m = 0; m < kQdDiff; ++m) qv[k][m] = __builtin_nontemporal_load(&qd[m * Q3]);
            if constexpr (VARK) {
                const T kap = T(kappa[e * Q3 + pt]);
#pragma unroll
                for (int m = 0; m < kQdDiff; ++m) qv[k][m] *= kap;
            }
        }
    };
    T qv[RQ][kQdDiff];
    if constexpr (PF) load_factors(qv);

    for (int v0 = 0; v0 < nvec; ++v0) {
        gather<P, Q, G, NT, 1, T>(A, off, x, nvec, v0, nvalid, tid);
        group_sync<NT>();
        gf_z<P, Q, G, NT, T>(A, Bb, bas, tid);
        group_sync<NT>();
        gf_y<P, Q, G, NT, T>(A, Bb, C, bas, tid);
        if constexpr (!PF) {
            if (v0 == 0) load_factors(qv);
        }
        group_sync<NT>();
        gf_x<P, Q, G, NT, T>(A, Bb, C, bas, tid);
        group_sync<NT>();
#pragma unroll
        for (int k = 0; k < RQ; ++k) {
            const int id = tid + k * NT;
            if (id < NPT) {
                const int g = id / Q3, pt = id - g * Q3;
                const int a = pt % Q, b = (pt / Q) % Q, c = pt / Q2;
                const int ls = g * L::BUF + a + L::PITCH * b + L::PLANE * c;
                const T *gm = qv[k];
                const T ur = A[ls], us = C[ls], ut = Bb[ls];
                A[ls] = gm[0] * ur + gm[5] * us + gm[4] * ut;
                C[ls] = gm[5] * ur + gm[1] * us + gm[3] * ut;
                Bb[ls] = gm[4] * ur + gm[3] * us + gm[2] * ut;
            }
        }
        group_sync<NT>();
        gf_xt<P, Q, G, NT, T>(A, Bb, C, bas, tid);
        group_sync<NT>();
        gf_yt<P, Q, G, NT, T>(A, Bb, C, bas, tid);
        group_sync<NT>();
        gf_zt<P, Q, G, NT, T>(A, Bb, bas, tid);
        group_sync<NT>();
        scatter_add<P, Q, G, NT, 1, DET, T>(A, off, y, nvec, v0, nvalid, tid, ebuf, e0);
        group_sync<NT>();
    }
}

// ---------------------------------------------------------------------------
// Host launchers for one (P, Q) pair.
// ---------------------------------------------------------------------------
template <typename K>
static hipError_t prepare_lds(K kernel, size_t lds)
{
    if (lds > 65536) return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return hipSuccess;
}

template <int P, int Q, bool COLLOC, int MODE, bool VARK, typename T, int V, bool OTF, bool DET>
static hipError_t launch_apply_v(const ApplyLaunch &a)
{
    constexpr int G = variant_g(Q, V, MODE), NT = variant_nt(Q, V), VC = variant_vc(V);
    constexpr size_t lds = apply_lds(P, Q, MODE, sizeof(T), V, OTF);
    // matrix-core gradient: collocated FP64 diffusion with stored factors
    constexpr bool MX = variant_mx(V);
    constexpr bool mx_ok = COLLOC && MODE == kDiff && sizeof(T) == 8 && !OTF && !VARK;
    // chunked multi-vector variants exist for the plain mass / diffusion operators only
    if constexpr ((VC > 1 && (MODE == kRhs || VARK || OTF)) || lds > kMaxLds || (MX && !mx_ok)) {
        (void)a;
        return hipErrorInvalidValue;
    } else if constexpr (MODE == kMass) {
        const int chain = a.chain > 0 ? a.chain : 1;
        const int64_t ngroups = (int64_t)a.v.ney * a.v.nez * ((a.v.nex + G - 1) / G);
        const int64_t nblk = (ngroups + chain - 1) / chain;
        auto kern = k_mass<P, Q, COLLOC, T, G, NT, VC, DET>;
        const hipError_t e = prepare_lds(kern, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(NT), lds, a.stream, static_cast<const T *>(a.basis_dev),
                           a.v.nex, ngroups, a.nvec, chain, a.v.offsets, static_cast<const T *>(a.v.qdata),
                           static_cast<const T *>(a.x), static_cast<T *>(a.y), static_cast<T *>(a.ebuf));
        return hipGetLastError();
    } else {
        const int64_t nblk = (int64_t)a.v.ney * a.v.nez * ((a.v.nex + G - 1) / G);
        auto go = [&](auto kern, size_t lds_bytes) {
            const hipError_t e = prepare_lds(kern, lds_bytes);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(NT), lds_bytes, a.stream,
                               static_cast<const T *>(a.basis_dev), a.v.nex, a.v.ney, a.nvec, a.v.offsets,
                               static_cast<const T *>(a.v.qdata), a.v.kappa, a.wdet, a.vert,
                               static_cast<const T *>(a.x), static_cast<T *>(a.y), static_cast<T *>(a.ebuf));
            return hipGetLastError();
        };
        // several chunks per launch: staged scatter in runs of at least 64 bytes per node
        if constexpr (staged_scatter(MODE, VC, sizeof(T)) && !DET && !VARK && !OTF) {
            constexpr size_t lds_st = apply_lds(P, Q, MODE, sizeof(T), V, OTF, true);
            if constexpr (lds_st <= kMaxLds) {
                if (a.nvec > VC)
                    return go(k_apply<P, Q, COLLOC, MODE, VARK, T, G, NT, VC, OTF, DET, true, 0, MX>, lds_st);
            }
        }
        constexpr int LATE = MODE == kDiff && VC == 1 && !OTF ? variant_late(Q, V) : 0;
        constexpr int PRE = LATE > 0 ? variant_pre(Q, V) : 0;
        return go(k_apply<P, Q, COLLOC, MODE, VARK, T, G, NT, VC, OTF, DET, false, LATE, MX, PRE>, lds);
    }
}

template <int P, int Q, bool COLLOC, int MODE, bool VARK, typename T, int V, bool OTF, bool DET>
static hipError_t launch_apply_gfv(const ApplyLaunch &a)
{
    // the factored-gradient kernel: diffusion with Gauss points (not collocated), stored factors
    if constexpr (MODE != kDiff || COLLOC || OTF) {
        (void)a;
        return hipErrorInvalidValue;
    } else {
        constexpr int G = variant_g(Q, V, MODE), NT = variant_nt(Q, V);
        constexpr bool PF = gf_prefetch(V);
        constexpr size_t lds = apply_lds(P, Q, MODE, sizeof(T), V, OTF);
        if constexpr (lds > kMaxLds) {
            (void)a;
            return hipErrorInvalidValue;
        } else {
            const int64_t nblk = (int64_t)a.v.ney * a.v.nez * ((a.v.nex + G - 1) / G);
            auto kern = k_apply_gf<P, Q, VARK, T, G, NT, PF, DET>;
            const hipError_t e = prepare_lds(kern, lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(NT), lds, a.stream,
                               static_cast<const T *>(a.basis_dev), a.v.nex, a.nvec, a.v.offsets,
                               static_cast<const T *>(a.v.qdata), a.v.kappa, static_cast<const T *>(a.x),
                               static_cast<T *>(a.y), static_cast<T *>(a.ebuf));
            return hipGetLastError();
        }
    }
}

template <int P, int Q, bool COLLOC, int MODE, bool VARK, typename T, bool OTF, bool DET>
static hipError_t launch_apply_vd(const ApplyLaunch &a)
{
    switch (a.variant) {
    case 9: return launch_apply_gfv<P, Q, COLLOC, MODE, VARK, T, 9, OTF, DET>(a);
    case 10: return launch_apply_gfv<P, Q, COLLOC, MODE, VARK, T, 10, OTF, DET>(a);
    case 11: return launch_apply_gfv<P, Q, COLLOC, MODE, VARK, T, 11, OTF, DET>(a);
    case 12: return launch_apply_gfv<P, Q, COLLOC, MODE, VARK, T, 12, OTF, DET>(a);
    case 13: return launch_apply_gfv<P, Q, COLLOC, MODE, VARK, T, 13, OTF, DET>(a);
    case 14: return launch_apply_gfv<P, Q, COLLOC, MODE, VARK, T, 14, OTF, DET>(a);
    case 8: return launch_apply_v<P, Q, COLLOC, MODE, VARK, T, 8, OTF, DET>(a);
    case 0: return launch_apply_v<P, Q, COLLOC, MODE, VARK, T, 0, OTF, DET>(a);
    case 1: return launch_apply_v<P, Q, COLLOC, MODE, VARK, T, 1, OTF, DET>(a);
    case 2: return launch_apply_v<P, Q, COLLOC, MODE, VARK, T, 2, OTF, DET>(a);
    case 3: return launch_apply_v<P, Q, COLLOC, MODE, VARK, T, 3, OTF, DET>(a);
    case 4: return launch_apply_v<P, Q, COLLOC, MODE, VARK, T, 4, OTF, DET>(a);
    case 5: return launch_apply_v<P, Q, COLLOC, MODE, VARK, T, 5, OTF, DET>(a);
    case 6: return launch_apply_v<P, Q, COLLOC, MODE, VARK, T, 6, OTF, DET>(a);
    case 7: return launch_apply_v<P, Q, COLLOC, MODE, VARK, T, 7, OTF, DET>(a);
    case 15: return launch_apply_v<P, Q, COLLOC, MODE, VARK, T, 15, OTF, DET>(a);
    case 16: return launch_apply_v<P, Q, COLLOC, MODE, VARK, T, 16, OTF, DET>(a);
    default: return hipErrorInvalidValue;
    }
}

// The deterministic (element-buffer) form is a separate instantiation; the load vector keeps atomics.
template <int P, int Q, bool COLLOC, int MODE, bool VARK, typename T, bool OTF = false>
static hipError_t launch_apply_t(const ApplyLaunch &a)
{
    if constexpr (MODE != kRhs) {
        if (a.ebuf) return launch_apply_vd<P, Q, COLLOC, MODE, VARK, T, OTF, true>(a);
    }
    return launch_apply_vd<P, Q, COLLOC, MODE, VARK, T, OTF, false>(a);
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
    if (a.otf) return launch_apply_t<P, Q, COLLOC, kDiff, false, double, true>(a);
    return launch_apply_t<P, Q, COLLOC, kDiff, false, double>(a);
}

template <int P, int Q, bool COLLOC>
static hipError_t launch_kgrad_pq(const KgradLaunch &a)
{
    constexpr int G = 1, NT = Q <= 6 ? 64 : 128;
    const int64_t nblk = a.v.nelem;
    const size_t lds = (size_t)G * 6 * Lds<Q>::BUF * sizeof(double);
    auto kern = k_kgrad<P, Q, COLLOC, G, NT>;
    hipError_t err = prepare_lds(kern, lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(NT), lds, a.stream, a.basis_dev, a.v.nelem, a.v.offsets,
                       static_cast<const double *>(a.v.qdata), a.u, a.r, a.g);
    return hipGetLastError();
}

}  // namespace mfhex

// Instantiate the launchers of order N (P = N+1): Gauss q = N+2, Lobatto q = N+1.
#define MFHEX_DEFINE_ORDER(N)                                                                          \
    namespace mfhex {                                                                                  \
    hipError_t launch_apply_p##N(const ApplyLaunch &a)                                                 \
    {                                                                                                  \
        if (a.colloc) return launch_apply_pq<N + 1, N + 1, true>(a);                                   \
        return launch_apply_pq<N + 1, N + 2, false>(a);                                                \
    }                                                                                                  \
    hipError_t launch_kgrad_p##N(const KgradLaunch &a)                                                 \
    {                                                                                                  \
        if (a.colloc) return launch_kgrad_pq<N + 1, N + 1, true>(a);                                   \
        return launch_kgrad_pq<N + 1, N + 2, false>(a);                                                \
    }                                                                                                  \
    hipError_t launch_diag_p##N(const DiagLaunch &a)                                                   \
    {                                                                                                  \
        if (a.colloc) return launch_diag_pq<N + 1, N + 1>(a);                                          \
        return launch_diag_pq<N + 1, N + 2>(a);                                                        \
    }                                                                                                  \
    }
