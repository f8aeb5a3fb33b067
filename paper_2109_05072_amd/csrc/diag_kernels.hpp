// Diagonal of the assembled operator, evaluated matrix-free by sum factorization.
//
// With phi_ijk(abc) = B_ai B_bj B_ck and its reference derivatives
// d_r phi = G_ai B_bj B_ck, d_s phi = B_ai G_bj B_ck, d_t phi = B_ai B_bj G_ck
// (G = D B: the basis derivative at the points; G = D when collocated), the
// element matrix diagonal of A^e = Dhat^T G^e Dhat (Sec. 2) is
//
//   (A^e)_ijk,ijk = sum_abc [ g_rr (G.G)_ai (B.B)_bj (B.B)_ck + g_ss ... + g_tt ...
//                             + 2 g_st (B.B)_ai (B.G)_bj (B.G)_ck + 2 g_rt ... + 2 g_rs ... ]
//
// (. the elementwise product), i.e. six transposed interpolations of the
// point factors with squared or mixed 1D matrices, each evaluated as three 1D
// contractions (z, then y, then x); the mass diagonal is one such term with
// w detJ and (B.B) along every axis.  Element diagonals are added into the
// global diagonal with atomics, masked nodes skipped.  This is set-up work
// for Jacobi preconditioning (run once per solve), so it is written plainly:
// one element per thread group, unpadded LDS, matrices in LDS.
#pragma once

#include "mfhex_internal.h"

namespace mfhex {

template <int P, int Q, int MODE, bool VARK, int NT>
__global__ void __launch_bounds__(NT)
k_diag(const double *__restrict__ bas, const int32_t *__restrict__ offsets, const double *__restrict__ qdata,
       const double *__restrict__ kappa, double *__restrict__ d)
{
    constexpr int P3 = P * P * P, Q3 = Q * Q * Q;
    constexpr int R = (P3 + NT - 1) / NT;
    __shared__ double sB2[Q * P], sG2[Q * P], sBG[Q * P];
    __shared__ double sF[Q3], sT1[P * Q * Q], sT2[P * P * Q];
    const int tid = threadIdx.x;
    const int64_t e = blockIdx.x;

    // 1D matrices: B [Q][P] and the collocated derivative D [Q][Q] from the basis block
    const double *B = bas + basis_b(P, Q), *D = bas + basis_d(P, Q);
    for (int t = tid; t < Q * P; t += NT) {
        const int a = t / P, i = t - a * P;
        double g = 0.0;
        for (int c = 0; c < Q; ++c) g += D[a * Q + c] * B[c * P + i];
        const double b = B[t];
        sB2[t] = b * b;
        sG2[t] = g * g;
        sBG[t] = b * g;
    }

    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;

    constexpr int NTERM = MODE == kMass ? 1 : kQdDiff;
    const double *qd = qdata + e * (int64_t)(MODE == kMass ? 1 : kQdDiff) * Q3;
    for (int m = 0; m < NTERM; ++m) {
        // factor order rr, ss, tt, st, rt, rs; matrices along x, y, z
        const double *X = sB2, *Y = sB2, *Z = sB2;
        double w = 1.0;
        if constexpr (MODE != kMass) {
            if (m == 0) X = sG2;
            if (m == 1) Y = sG2;
            if (m == 2) Z = sG2;
            if (m == 3) Y = Z = sBG;
            if (m == 4) X = Z = sBG;
            if (m == 5) X = Y = sBG;
            if (m >= 3) w = 2.0;
        }
        __syncthreads();  // previous term done with sF / sT1 / sT2; matrices ready
        for (int t = tid; t < Q3; t += NT) {
            double f = w * qd[m * Q3 + t];
            if constexpr (VARK) f *= kappa[e * Q3 + t];
            sF[t] = f;
        }
        __syncthreads();
        // z: T1[k][b][a] = sum_c Z[c][k] F[c][b][a]
        for (int t = tid; t < P * Q * Q; t += NT) {
            const int a = t % Q, b = (t / Q) % Q, k = t / (Q * Q);
            double s = 0.0;
            for (int c = 0; c < Q; ++c) s += Z[c * P + k] * sF[a + Q * (b + Q * c)];
            sT1[t] = s;
        }
        __syncthreads();
        // y: T2[k][j][a] = sum_b Y[b][j] T1[k][b][a]
        for (int t = tid; t < P * P * Q; t += NT) {
            const int a = t % Q, j = (t / Q) % P, k = t / (Q * P);
            double s = 0.0;
            for (int b = 0; b < Q; ++b) s += Y[b * P + j] * sT1[a + Q * (b + Q * k)];
            sT2[t] = s;
        }
        __syncthreads();
        // x: acc[k][j][i] += sum_a X[a][i] T2[k][j][a]
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int t = tid + r * NT;
            if (t < P3) {
                const int i = t % P, jk = t / P;
                double s = 0.0;
                for (int a = 0; a < Q; ++a) s += X[a * P + i] * sT2[a + Q * jk];
                acc[r] += s;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int t = tid + r * NT;
        if (t < P3) {
            const int32_t o = offsets[e * P3 + t];
            if (o >= 0) unsafeAtomicAdd(&d[o], acc[r]);
        }
    }
}

template <int P, int Q>
static hipError_t launch_diag_pq(const DiagLaunch &a)
{
    constexpr int NT = Q <= 6 ? 64 : 128;
    const dim3 grid((unsigned)a.v.nelem), block(NT);
    const double *qd = static_cast<const double *>(a.v.qdata);
    if (a.mode == kMass)
        hipLaunchKernelGGL((k_diag<P, Q, kMass, false, NT>), grid, block, 0, a.stream, a.basis_dev, a.v.offsets, qd,
                           nullptr, a.d);
    else if (a.vark)
        hipLaunchKernelGGL((k_diag<P, Q, kDiff, true, NT>), grid, block, 0, a.stream, a.basis_dev, a.v.offsets, qd,
                           a.v.kappa, a.d);
    else
        hipLaunchKernelGGL((k_diag<P, Q, kDiff, false, NT>), grid, block, 0, a.stream, a.basis_dev, a.v.offsets, qd,
                           nullptr, a.d);
    return hipGetLastError();
}

}  // namespace mfhex
