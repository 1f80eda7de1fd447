// Forward sum-factorized sweeps of the hex kernels on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64), the alternative to the pencil sweeps of forward3.
// Same contractions (Sec. 3.2), same LDS buffers and layouts in and out:
//   axis 1:  R1[(v,q1)][(r,i3,i2)] = sum_i1 T_v[q1][i1] X[r][i3][i2][i1],
//            T_0 = B, T_1 = G                                 rows 2 n_q
//   axis 2:  rows (BB, BG, GB) x q2, columns (r, i3, q1), the two R1
//            planes stacked along k                            rows 3 n_q
//   axis 3:  rows (d = 0, 1, 2) x q3, columns (r, q2, q1), the three R2
//            planes stacked along k, d = 0 and 1 with B, d = 2 with G
// Each contraction is a matrix product whose k (the contracted 1D index, n_i
// values) runs in steps of 4; the rows of one 16 x 16 output tile hold every
// output variant of a column, and the columns run over the elements of the
// workgroup, so the four waves share the tiles of a stage.  Rows beyond
// 3 n_q and k beyond n_i multiply zeros; classes with n_q > 5 have no
// matrix-core form.
//
// Operand layout of the instruction (one double per lane for A and B, four
// for the accumulator): A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
// D[i][j] in lane j + 16 (i % 4), item i / 4.
#pragma once
#include "tmop_dev.hpp"

namespace tmop {

typedef double dvec4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dvec4 mfma_f64(double a, double b, dvec4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// The 1D tables B (n_q x n_i) then G, copied to LDS so that every lane can
// read the entry its operand needs (the kernel argument is indexed with
// compile-time constants only).  Called before a barrier that precedes the
// sweeps.
template <int NI, int NQ>
__device__ __forceinline__ void mfma_tables(const Tables &tb, double *sT)
{
#pragma unroll
    for (int k = 0; k < NQ * NI; ++k)
        if (threadIdx.x == k) {
            sT[k] = tb.B[k];
            sT[NQ * NI + k] = tb.G[k];
        }
}

template <int P, int NQ, int NR = 9>
__device__ __forceinline__ void forward3_mfma(const double *sT, const double *X, double *R1,
                                              double *R2, double *RY, int nel)
{
    constexpr int NI = P + 1, L1 = NI * NI * NQ, L2 = NI * NQ * NQ, NQ2 = NQ * NQ,
                  NQ3 = NQ * NQ * NQ;
    constexpr int KS = (NI + 3) / 4;  // k steps of 4 per contracted index
    constexpr int NW = BLOCK / 64;
    static_assert(3 * NQ <= 16, "the output variants of a column must fit in 16 rows");
    const double *TB = sT, *TG = sT + NQ * NI;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int l16 = lane & 15, l4 = lane >> 4;

    // axis 1
    {
        const int n = nel * 3 * NI * NI;
        double a[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = s * 4 + l4;
            a[s] = 0.0;
            if (k < NI && l16 < 2 * NQ) a[s] = l16 < NQ ? TB[l16 * NI + k] : TG[(l16 - NQ) * NI + k];
        }
        for (int t = wv; t * 16 < n; t += NW) {
            const int j = t * 16 + l16;
            dvec4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int k = s * 4 + l4;
                const double b = (j < n && k < NI) ? X[j * NI + k] : 0.0;
                acc = mfma_f64(a[s], b, acc);
            }
            if (j < n) {
                const int r = j / (NI * NI), i23 = j % (NI * NI);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int row = l4 + 4 * m;
                    if (row < 2 * NQ) {
                        const int v = row < NQ ? 0 : 1;
                        R1[r * 2 * L1 + v * L1 + i23 * NQ + row - v * NQ] = acc[m];
                    }
                }
            }
        }
    }
    __syncthreads();
    // axis 2: rows 0..n_q-1 B R1_B (BB), n_q..2n_q-1 G R1_B (BG), 2n_q.. B R1_G (GB)
    {
        const int n = nel * 3 * NI * NQ;
        double a0[KS], a1[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = s * 4 + l4;
            a0[s] = 0.0;
            a1[s] = 0.0;
            if (k < NI) {
                if (l16 < NQ)
                    a0[s] = TB[l16 * NI + k];
                else if (l16 < 2 * NQ)
                    a0[s] = TG[(l16 - NQ) * NI + k];
                else if (l16 < 3 * NQ)
                    a1[s] = TB[(l16 - 2 * NQ) * NI + k];
            }
        }
        for (int t = wv; t * 16 < n; t += NW) {
            const int j = t * 16 + l16;
            const int r = j / (NI * NQ), i3 = (j / NQ) % NI, q1 = j % NQ;
            dvec4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int k = s * 4 + l4;
                const bool ok = j < n && k < NI;
                const int at = r * 2 * L1 + (i3 * NI + k) * NQ + q1;
                const double b0 = ok ? R1[at] : 0.0;
                const double b1 = ok ? R1[at + L1] : 0.0;
                acc = mfma_f64(a0[s], b0, acc);
                acc = mfma_f64(a1[s], b1, acc);
            }
            if (j < n) {
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int row = l4 + 4 * m;
                    if (row < 3 * NQ) {
                        const int wr = row / NQ, q2 = row % NQ;
                        // R2 planes: 0 GB, 1 BG, 2 BB
                        R2[r * 3 * L2 + (2 - wr) * L2 + i3 * NQ2 + q2 * NQ + q1] = acc[m];
                    }
                }
            }
        }
    }
    __syncthreads();
    // axis 3: row block d takes R2 plane d (GB, BG with B; BB with G)
    {
        const int n = nel * 3 * NQ2;
        double a[3][KS];
#pragma unroll
        for (int src = 0; src < 3; ++src)
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int k = s * 4 + l4;
                a[src][s] = 0.0;
                if (k < NI && l16 < 3 * NQ && l16 / NQ == src) {
                    const int q3 = l16 % NQ;
                    a[src][s] = src < 2 ? TB[q3 * NI + k] : TG[q3 * NI + k];
                }
            }
        for (int t = wv; t * 16 < n; t += NW) {
            const int j = t * 16 + l16;
            const int r = j / NQ2, q12 = j % NQ2;
            dvec4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int src = 0; src < 3; ++src)
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    const int k = s * 4 + l4;
                    const double b = (j < n && k < NI) ? R2[r * 3 * L2 + src * L2 + k * NQ2 + q12] : 0.0;
                    acc = mfma_f64(a[src][s], b, acc);
                }
            if (j < n) {
                const int el = r / 3, c = r % 3;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int row = l4 + 4 * m;
                    if (row < 3 * NQ) {
                        const int d = row / NQ, q3 = row % NQ;
                        RY[(el * NR + c * 3 + d) * NQ3 + q3 * NQ2 + q12] = acc[m];
                    }
                }
            }
        }
    }
    __syncthreads();
}

}  // namespace tmop
