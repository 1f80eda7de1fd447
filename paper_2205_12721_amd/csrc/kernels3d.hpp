// 3D (hex) PA-TMOP kernels, templated on the order P and the points per
// direction NQ.  Sum factorization follows Sec. 3.2: the Jacobian entries at
// all quadrature points of an element come from three 1D contractions with
// B = l_i(chi_q) and G = l_i'(chi_q), one per axis, e.g.
//   A_a1(q) = sum_i1 G[q1][i1] sum_i2 B[q2][i2] sum_i3 B[q3][i3] x_a(i1,i2,i3)
// and the transposed contractions map quadrature values back to nodes.
//
// LDS layout per workgroup (CT = compute type, double or float):
//   sB, sG   [NQ][NI]                 1D tables
//   sX       [EPB][3][NI^3]           element nodes (or v_E)
//   R1       [EPB][3][2][NI][NI][NQ]  after the axis-1 contraction (B, G variants)
//   R2       [EPB][3][3][NI][NQ][NQ]  after the axis-2 contraction (GB, BG, BB)
//   RY       [EPB][9][NQ^3]           per-point 3x3 values (Y = H : grad v, or P)
// Forward:  sX -> R1 -> R2 -> (points) ; backward: RY -> R2 -> R1 -> E-vector.
#pragma once
#include "tmop_dev.hpp"

namespace tmop {

template <int P, int NQ>
struct S3 {
    static constexpr int NI = P + 1;
    static constexpr int NP = NI * NI * NI;
    static constexpr int NQ2 = NQ * NQ;
    static constexpr int NQ3 = NQ * NQ * NQ;
    static constexpr int EPB = NQ3 >= BLOCK ? 1 : BLOCK / NQ3;
    static constexpr int L1 = NI * NI * NQ;  // one R1 plane
    static constexpr int L2 = NI * NQ * NQ;  // one R2 plane
    static constexpr int NS = 45;            // packed tensor entries
};

template <int P, int NQ, typename CT>
struct Lds3 {
    using S = S3<P, NQ>;
    CT B[NQ * S::NI];
    CT G[NQ * S::NI];
    CT X[S::EPB * 3 * S::NP];
    CT R1[S::EPB * 6 * S::L1];
    CT R2[S::EPB * 9 * S::L2];
    CT RY[S::EPB * 9 * S::NQ3];
};

template <int P, int NQ, typename CT>
__device__ inline void load_tables3(const Tables &t, CT *sB, CT *sG)
{
    constexpr int NI = P + 1;
    for (int k = threadIdx.x; k < NQ * NI; k += BLOCK) {
        sB[k] = (CT)t.B[k];
        sG[k] = (CT)t.G[k];
    }
}

// Global node of local node (i1,i2,i3) of element e, and its grid coordinates.
template <int P>
__device__ inline int node3(const Geom &g, int e, int i1, int i2, int i3, int &gx, int &gy,
                            int &gz)
{
    constexpr int NI = P + 1;
    if (g.e2n) {
        gx = gy = gz = -1;
        return g.e2n[(size_t)e * (NI * NI * NI) + i1 + NI * (i2 + NI * i3)];
    }
    const int ex = e % g.nel[0];
    const int t = e / g.nel[0];
    const int ey = t % g.nel[1];
    const int ez = t / g.nel[1];
    gx = ex * P + i1;
    gy = ey * P + i2;
    gz = ez * P + i3;
    return gx + g.M[0] * (gy + g.M[1] * gz);
}

// Gather d components of a global vector into sX for the block's elements.
// masked: fixed DoFs read as zero (the P of H_c = P H P + (I - P)).
template <int P, int NQ, typename CT>
__device__ inline void gather3(const Geom &g, const double *__restrict__ vec, int e0, int nel,
                               CT *sX, bool masked)
{
    using S = S3<P, NQ>;
    constexpr int NI = S::NI, NP = S::NP;
    for (int idx = threadIdx.x; idx < nel * 3 * NP; idx += BLOCK) {
        const int i = idx % NP;
        const int r = idx / NP;  // el*3 + c
        const int c = r % 3, el = r / 3;
        const int i1 = i % NI, i2 = (i / NI) % NI, i3 = i / (NI * NI);
        int gx, gy, gz;
        const int node = node3<P>(g, e0 + el, i1, i2, i3, gx, gy, gz);
        double v = vec[(size_t)c * g.nx + node];
        if (masked && is_fixed(g, c, node, gx, gy, gz)) v = 0.0;
        sX[idx] = (CT)v;
    }
}

// Axis-1 and axis-2 contractions: sX -> R1 -> R2.
template <int P, int NQ, typename CT>
__device__ inline void forward12(const CT *sB, const CT *sG, const CT *sX, CT *R1, CT *R2, int nel)
{
    using S = S3<P, NQ>;
    constexpr int NI = S::NI, L1 = S::L1, L2 = S::L2;
    for (int idx = threadIdx.x; idx < nel * 3 * NI * NI * NQ; idx += BLOCK) {
        const int q1 = idx % NQ;
        int r = idx / NQ;
        const int i2 = r % NI;
        r /= NI;
        const int i3 = r % NI;
        r /= NI;  // el*3 + c
        const CT *x = sX + r * S::NP + (i3 * NI + i2) * NI;
        CT b = 0, gg = 0;
#pragma unroll
        for (int i1 = 0; i1 < NI; ++i1) {
            const CT xv = x[i1];
            b += sB[q1 * NI + i1] * xv;
            gg += sG[q1 * NI + i1] * xv;
        }
        CT *o = R1 + r * 2 * L1 + (i3 * NI + i2) * NQ + q1;
        o[0] = b;
        o[L1] = gg;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nel * 3 * NI * NQ * NQ; idx += BLOCK) {
        const int q1 = idx % NQ;
        int r = idx / NQ;
        const int q2 = r % NQ;
        r /= NQ;
        const int i3 = r % NI;
        r /= NI;
        const CT *tb = R1 + r * 2 * L1 + i3 * NI * NQ + q1;  // B variant, [i2] stride NQ
        const CT *tg = tb + L1;                             // G variant
        CT gb = 0, bg = 0, bb = 0;
#pragma unroll
        for (int i2 = 0; i2 < NI; ++i2) {
            const CT B2 = sB[q2 * NI + i2], G2 = sG[q2 * NI + i2];
            const CT xb = tb[i2 * NQ], xg = tg[i2 * NQ];
            gb += B2 * xg;
            bg += G2 * xb;
            bb += B2 * xb;
        }
        CT *o = R2 + r * 3 * L2 + (i3 * NQ + q2) * NQ + q1;
        o[0] = gb;
        o[L2] = bg;
        o[2 * L2] = bb;
    }
    __syncthreads();
}

// Axis-3 contraction at one point: J[c*3+b] = d x_c / d xbar_b.
template <int P, int NQ, typename CT>
__device__ inline void point_grad3(const CT *sB, const CT *sG, const CT *R2, int el, int q1,
                                   int q2, int q3, CT *J)
{
    using S = S3<P, NQ>;
    constexpr int NI = S::NI, L2 = S::L2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const CT *t = R2 + (el * 3 + c) * 3 * L2 + q2 * NQ + q1;  // [i3] stride NQ^2
        CT a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
        for (int i3 = 0; i3 < NI; ++i3) {
            const CT B3 = sB[q3 * NI + i3], G3 = sG[q3 * NI + i3];
            a0 += B3 * t[i3 * NQ * NQ];
            a1 += B3 * t[L2 + i3 * NQ * NQ];
            a2 += G3 * t[2 * L2 + i3 * NQ * NQ];
        }
        J[c * 3 + 0] = a0;
        J[c * 3 + 1] = a1;
        J[c * 3 + 2] = a2;
    }
}

// Transposed contractions RY -> R2 -> R1 -> out (E-vector, element-major
// [e][c][i]).  y_c(i) = sum_q sum_b RY[c][b](q) d w_i/d xbar_b (q).
template <int P, int NQ, typename CT, typename OT>
__device__ inline void backward3(const CT *sB, const CT *sG, const CT *RY, CT *R2, CT *R1, int nel,
                                 OT *__restrict__ out)
{
    using S = S3<P, NQ>;
    constexpr int NI = S::NI, L1 = S::L1, L2 = S::L2, NQ3 = S::NQ3;
    for (int idx = threadIdx.x; idx < nel * 3 * NI * NQ * NQ; idx += BLOCK) {
        const int q1 = idx % NQ;
        int r = idx / NQ;
        const int q2 = r % NQ;
        r /= NQ;
        const int i3 = r % NI;
        r /= NI;  // el*3 + c
        const CT *y = RY + r * 3 * NQ3 + q2 * NQ + q1;  // [b] stride NQ3, [q3] stride NQ^2
        CT t0 = 0, t1 = 0, t2 = 0;
#pragma unroll
        for (int q3 = 0; q3 < NQ; ++q3) {
            const CT B3 = sB[q3 * NI + i3], G3 = sG[q3 * NI + i3];
            t0 += B3 * y[q3 * NQ * NQ];
            t1 += B3 * y[NQ3 + q3 * NQ * NQ];
            t2 += G3 * y[2 * NQ3 + q3 * NQ * NQ];
        }
        CT *o = R2 + r * 3 * L2 + (i3 * NQ + q2) * NQ + q1;
        o[0] = t0;
        o[L2] = t1;
        o[2 * L2] = t2;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nel * 3 * NI * NI * NQ; idx += BLOCK) {
        const int q1 = idx % NQ;
        int r = idx / NQ;
        const int i2 = r % NI;
        r /= NI;
        const int i3 = r % NI;
        r /= NI;
        const CT *t = R2 + r * 3 * L2 + i3 * NQ * NQ + q1;  // [q2] stride NQ
        CT u0 = 0, u1 = 0;
#pragma unroll
        for (int q2 = 0; q2 < NQ; ++q2) {
            const CT B2 = sB[q2 * NI + i2], G2 = sG[q2 * NI + i2];
            u0 += B2 * t[q2 * NQ];
            u1 += G2 * t[L2 + q2 * NQ] + B2 * t[2 * L2 + q2 * NQ];
        }
        CT *o = R1 + r * 2 * L1 + (i3 * NI + i2) * NQ + q1;
        o[0] = u0;   // still needs G along axis 1
        o[L1] = u1;  // still needs B along axis 1
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nel * 3 * S::NP; idx += BLOCK) {
        const int i1 = idx % NI;
        int r = idx / NI;
        const int i2 = r % NI;
        r /= NI;
        const int i3 = r % NI;
        r /= NI;
        const CT *t = R1 + r * 2 * L1 + (i3 * NI + i2) * NQ;
        CT s = 0;
#pragma unroll
        for (int q1 = 0; q1 < NQ; ++q1) s += sG[q1 * NI + i1] * t[q1] + sB[q1 * NI + i1] * t[L1 + q1];
        out[idx] = (OT)s;
    }
}

// ------------------------------------------------------------------------
// Kernels
// ------------------------------------------------------------------------

// Energy and minimum det A: per-block partial sums of z mu and minima of det A,
// count of points with det T <= 0 (Sec. 3.3, eq. D0_expression; Sec. 2.3).
template <int P, int NQ>
__device__ inline void b3_energy(const Geom &g, const Tables &tb, const Target &tg, const double *__restrict__ x, double *__restrict__ part, int e0, int nel)
{
    using S = S3<P, NQ>;
    __shared__ Lds3<P, NQ, double> L;
    __shared__ double red[BLOCK / 64];
    load_tables3<P, NQ>(tb, L.B, L.G);
    gather3<P, NQ>(g, x, e0, nel, L.X, false);
    __syncthreads();
    forward12<P, NQ>(L.B, L.G, L.X, L.R1, L.R2, nel);
    double esum = 0.0, dmin = 1.0e300, bad = 0.0;
    for (int idx = threadIdx.x; idx < nel * S::NQ3; idx += BLOCK) {
        const int el = idx / S::NQ3, q = idx % S::NQ3;
        const int q1 = q % NQ, q2 = (q / NQ) % NQ, q3 = q / S::NQ2;
        double J[9];
        point_grad3<P, NQ>(L.B, L.G, L.R2, el, q1, q2, q3, J);
        const double dA = det_only<3>(J);
        dmin = fmin(dmin, dA);
        const double z = tb.w[q1] * tb.w[q2] * tb.w[q3] * tg.detW;
        double mu, Pm[9];
        if (metric_first<3>(tg, J, z, &mu, Pm))
            esum += z * mu;
        else
            bad += 1.0;
    }
    const double s = block_sum(esum, red);
    const double m = block_min(dmin, red);
    const double b = block_sum(bad, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s;
        part[gridDim.x + blockIdx.x] = m;
        part[2 * gridDim.x + blockIdx.x] = b;
    }
}

// Gradient E-vector (Sec. 3.3, eq. eq_vm_pa_grad): per point z P, then the
// transposed contractions.  bad[blockIdx] counts points with det T <= 0.
template <int P, int NQ>
__device__ inline void b3_gradient(const Geom &g, const Tables &tb, const Target &tg, const double *__restrict__ x, double *__restrict__ gE, double *__restrict__ bad, int e0, int nel)
{
    using S = S3<P, NQ>;
    __shared__ Lds3<P, NQ, double> L;
    __shared__ double red[BLOCK / 64];
    load_tables3<P, NQ>(tb, L.B, L.G);
    gather3<P, NQ>(g, x, e0, nel, L.X, false);
    __syncthreads();
    forward12<P, NQ>(L.B, L.G, L.X, L.R1, L.R2, nel);
    double nbad = 0.0;
    for (int idx = threadIdx.x; idx < nel * S::NQ3; idx += BLOCK) {
        const int el = idx / S::NQ3, q = idx % S::NQ3;
        const int q1 = q % NQ, q2 = (q / NQ) % NQ, q3 = q / S::NQ2;
        double J[9], Pm[9], mu;
        point_grad3<P, NQ>(L.B, L.G, L.R2, el, q1, q2, q3, J);
        const double z = tb.w[q1] * tb.w[q2] * tb.w[q3] * tg.detW;
        if (!metric_first<3>(tg, J, z, &mu, Pm)) {
            nbad += 1.0;
#pragma unroll
            for (int k = 0; k < 9; ++k) Pm[k] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) L.RY[(el * 9 + k) * S::NQ3 + q] = Pm[k];
    }
    __syncthreads();
    backward3<P, NQ>(L.B, L.G, L.RY, L.R2, L.R1, nel, gE + (size_t)e0 * 3 * S::NP);
    const double b = block_sum(nbad, red);
    if (threadIdx.x == 0) bad[blockIdx.x] = b;
}

// Hessian setup (Sec. 3.4): per point the packed z * H_A tensor, stored
// element-major [e][45][NQ^3] so that each entry is one coalesced plane.
template <int P, int NQ, typename TT>
__device__ inline void b3_setup(const Geom &g, const Tables &tb, const Target &tg, const double *__restrict__ x, TT *__restrict__ H, double *__restrict__ bad, int e0, int nel)
{
    using S = S3<P, NQ>;
    __shared__ Lds3<P, NQ, double> L;
    __shared__ double red[BLOCK / 64];
    load_tables3<P, NQ>(tb, L.B, L.G);
    gather3<P, NQ>(g, x, e0, nel, L.X, false);
    __syncthreads();
    forward12<P, NQ>(L.B, L.G, L.X, L.R1, L.R2, nel);
    double nbad = 0.0;
    for (int idx = threadIdx.x; idx < nel * S::NQ3; idx += BLOCK) {
        const int el = idx / S::NQ3, q = idx % S::NQ3;
        const int q1 = q % NQ, q2 = (q / NQ) % NQ, q3 = q / S::NQ2;
        double J[9], Hp[45];
        point_grad3<P, NQ>(L.B, L.G, L.R2, el, q1, q2, q3, J);
        const double z = tb.w[q1] * tb.w[q2] * tb.w[q3] * tg.detW;
        if (!metric_second<3>(tg, J, z, Hp)) {
            nbad += 1.0;
#pragma unroll
            for (int k = 0; k < 45; ++k) Hp[k] = 0.0;
        }
        TT *h = H + (size_t)(e0 + el) * 45 * S::NQ3 + q;
#pragma unroll
        for (int k = 0; k < 45; ++k) h[k * S::NQ3] = (TT)Hp[k];
    }
    const double b = block_sum(nbad, red);
    if (threadIdx.x == 0) bad[blockIdx.x] = b;
}

// Hessian action, element part (Sec. 3.4, eq. eq_vm_pa_hess):
//   grad v at the points (forward contractions of P v),
//   Y_an = sum_bp H[an,bp] (grad v)_bp  with the stored tensor,
//   transposed contractions -> E-vector yE[e][c][i].
// CT = double (FP64) or float (mixed: FP32 tensor, FP32 arithmetic and
// accumulation).
template <int P, int NQ, typename TT, typename CT>
__device__ inline void b3_apply(const Geom &g, const Tables &tb, const TT *__restrict__ H, const double *__restrict__ v, CT *__restrict__ yE, int e0, int nel)
{
    using S = S3<P, NQ>;
    __shared__ Lds3<P, NQ, CT> L;
    load_tables3<P, NQ>(tb, L.B, L.G);
    gather3<P, NQ>(g, v, e0, nel, L.X, true);
    __syncthreads();
    forward12<P, NQ>(L.B, L.G, L.X, L.R1, L.R2, nel);
    for (int idx = threadIdx.x; idx < nel * S::NQ3; idx += BLOCK) {
        const int el = idx / S::NQ3, q = idx % S::NQ3;
        const int q1 = q % NQ, q2 = (q / NQ) % NQ, q3 = q / S::NQ2;
        const TT *h = H + (size_t)(e0 + el) * 45 * S::NQ3 + q;
        CT hv[45];
#pragma unroll
        for (int k = 0; k < 45; ++k) hv[k] = (CT)h[k * S::NQ3];
        CT J[9];
        point_grad3<P, NQ>(L.B, L.G, L.R2, el, q1, q2, q3, J);
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            CT s = 0;
#pragma unroll
            for (int c = 0; c < 9; ++c) s += hv[sym_index<9>(r, c)] * J[c];
            L.RY[(el * 9 + r) * S::NQ3 + q] = s;
        }
    }
    __syncthreads();
    backward3<P, NQ>(L.B, L.G, L.RY, L.R2, L.R1, nel, yE + (size_t)e0 * 3 * S::NP);
}

// ------------------------------------------------------------------------
// Compact quadrature data: per point T = A W^{-1} (9 values) and the four
// weighted metric coefficients z c_id, z c_tc, z c_cc, z c_dc (layout
// [e][13][q]).  The fourth-order tensor is then applied in closed form:
//   d2mu : M = c_id M + c_tc (T (C:M) + C (T:M)) + c_cc C (C:M) + c_dc dC[M],
// with C = cof T and dC[M] the derivative of the cofactor at T in direction M
// (the bilinear part of cof(T + M)).  Same result as the stored tensor,
// 13 instead of 45 values per point.
// ------------------------------------------------------------------------
constexpr int NC3 = 13;

template <typename CT>
__device__ inline void cof3(const CT *T, CT *C)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            C[i * 3 + j] = T[i1 * 3 + j1] * T[i2 * 3 + j2] - T[i1 * 3 + j2] * T[i2 * 3 + j1];
        }
}

template <typename CT>
__device__ inline void compact_action3(const CT *T, CT ca, CT cb, CT cc, CT cd, const CT *M, CT *Y)
{
    CT C[9];
    cof3(T, C);
    CT tm = 0, cm = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        tm += T[k] * M[k];
        cm += C[k] * M[k];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            const CT dC = T[i1 * 3 + j1] * M[i2 * 3 + j2] + M[i1 * 3 + j1] * T[i2 * 3 + j2] -
                          T[i1 * 3 + j2] * M[i2 * 3 + j1] - M[i1 * 3 + j2] * T[i2 * 3 + j1];
            const int r = i * 3 + j;
            Y[r] = ca * M[r] + cb * (T[r] * cm + C[r] * tm) + cc * C[r] * cm + cd * dC;
        }
}

// out = in W^{-1} (tr = false) or in W^{-T} (tr = true), D x D row-major.
template <int D, typename CT>
__device__ inline void mul_winv(const Target &t, const CT *in, CT *out, bool tr)
{
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int k = 0; k < D; ++k) {
            CT s = 0;
#pragma unroll
            for (int n = 0; n < D; ++n)
                s += in[a * D + n] * (CT)(tr ? t.Winv[k * D + n] : t.Winv[n * D + k]);
            out[a * D + k] = s;
        }
}

template <int P, int NQ, typename TT>
__device__ inline void b3_setupc(const Geom &g, const Tables &tb, const Target &tg, const double *__restrict__ x, TT *__restrict__ Q, double *__restrict__ bad, int e0, int nel)
{
    using S = S3<P, NQ>;
    __shared__ Lds3<P, NQ, double> L;
    __shared__ double red[BLOCK / 64];
    load_tables3<P, NQ>(tb, L.B, L.G);
    gather3<P, NQ>(g, x, e0, nel, L.X, false);
    __syncthreads();
    forward12<P, NQ>(L.B, L.G, L.X, L.R1, L.R2, nel);
    double nbad = 0.0;
    for (int idx = threadIdx.x; idx < nel * S::NQ3; idx += BLOCK) {
        const int el = idx / S::NQ3, q = idx % S::NQ3;
        const int q1 = q % NQ, q2 = (q / NQ) % NQ, q3 = q / S::NQ2;
        double J[9], T[9], C[9], out[NC3];
        point_grad3<P, NQ>(L.B, L.G, L.R2, el, q1, q2, q3, J);
        apply_winv<3>(tg, J, T);
        const double tau = det_cof<3>(T, C);
        const double z = tb.w[q1] * tb.w[q2] * tb.w[q3] * tg.detW;
        if (tau > 0.0) {
            double I1 = 0.0;
#pragma unroll
            for (int k = 0; k < 9; ++k) I1 += T[k] * T[k];
            const MetricCoef m = metric_coef(tg.metric, I1, tau);
#pragma unroll
            for (int k = 0; k < 9; ++k) out[k] = T[k];
            out[9] = z * m.c_id;
            out[10] = z * m.c_tc;
            out[11] = z * m.c_cc;
            out[12] = z * m.c_dc;
        } else {
            nbad += 1.0;
#pragma unroll
            for (int k = 0; k < NC3; ++k) out[k] = 0.0;
        }
        TT *h = Q + (size_t)(e0 + el) * NC3 * S::NQ3 + q;
#pragma unroll
        for (int k = 0; k < NC3; ++k) h[k * S::NQ3] = (TT)out[k];
    }
    const double b = block_sum(nbad, red);
    if (threadIdx.x == 0) bad[blockIdx.x] = b;
}

template <int P, int NQ, typename TT, typename CT>
__device__ inline void b3_applyc(const Geom &g, const Tables &tb, const Target &tg, const TT *__restrict__ Q, const double *__restrict__ v, CT *__restrict__ yE, int e0, int nel)
{
    using S = S3<P, NQ>;
    __shared__ Lds3<P, NQ, CT> L;
    load_tables3<P, NQ>(tb, L.B, L.G);
    gather3<P, NQ>(g, v, e0, nel, L.X, true);
    __syncthreads();
    forward12<P, NQ>(L.B, L.G, L.X, L.R1, L.R2, nel);
    for (int idx = threadIdx.x; idx < nel * S::NQ3; idx += BLOCK) {
        const int el = idx / S::NQ3, q = idx % S::NQ3;
        const int q1 = q % NQ, q2 = (q / NQ) % NQ, q3 = q / S::NQ2;
        const TT *h = Q + (size_t)(e0 + el) * NC3 * S::NQ3 + q;
        CT d[NC3];
#pragma unroll
        for (int k = 0; k < NC3; ++k) d[k] = (CT)h[k * S::NQ3];
        CT J[9], Y[9];
        point_grad3<P, NQ>(L.B, L.G, L.R2, el, q1, q2, q3, J);
        if (tg.ideal) {
            compact_action3<CT>(d, d[9], d[10], d[11], d[12], J, Y);
        } else {
            CT M[9], Yt[9];
            mul_winv<3, CT>(tg, J, M, false);
            compact_action3<CT>(d, d[9], d[10], d[11], d[12], M, Yt);
            mul_winv<3, CT>(tg, Yt, Y, true);
        }
#pragma unroll
        for (int r = 0; r < 9; ++r) L.RY[(el * 9 + r) * S::NQ3 + q] = Y[r];
    }
    __syncthreads();
    backward3<P, NQ>(L.B, L.G, L.RY, L.R2, L.R1, nel, yE + (size_t)e0 * 3 * S::NP);
}

// Hessian diagonal, element part (Sec. 3.4, last paragraph):
//   d_a(i) = sum_q sum_{n,p} H[an,ap](q) dw_i/dxbar_n dw_i/dxbar_p,
// contracted per (n,p) pair with the squared 1D tables BB, BG, GG.  The 18
// needed entries H[an,ap] (3 components x 6 pairs n <= p, off-diagonal pairs
// doubled) are first placed in LDS planes sQ[el][pair][a][q].
template <int P, int NQ>
struct DiagLds3 {
    using S = S3<P, NQ>;
    double T[3][NQ * S::NI];  // BB, BG, GG
    double sQ[S::EPB * 18 * S::NQ3];
    double U2[S::EPB * 3 * S::NI * NQ * NQ];
    double U1[S::EPB * 3 * S::NI * S::NI * NQ];
    double sD[S::EPB * 3 * S::NP];
};

__device__ constexpr int diag_pn(int pr) { return pr < 3 ? 0 : (pr < 5 ? 1 : 2); }
__device__ constexpr int diag_pp(int pr) { return pr < 3 ? pr : (pr < 5 ? pr - 2 : 2); }

template <int P, int NQ>
__device__ inline void diag_contract3(const Tables &tb, DiagLds3<P, NQ> &L, int nel,
                                      double *__restrict__ dE)
{
    using S = S3<P, NQ>;
    constexpr int NI = S::NI, NQ3 = S::NQ3, NP = S::NP;
    for (int k = threadIdx.x; k < NQ * NI; k += BLOCK) {
        const double b = tb.B[k], gg = tb.G[k];
        L.T[0][k] = b * b;
        L.T[1][k] = b * gg;
        L.T[2][k] = gg * gg;
    }
    for (int k = threadIdx.x; k < nel * 3 * NP; k += BLOCK) L.sD[k] = 0.0;
    for (int pr = 0; pr < 6; ++pr) {
        const int n = diag_pn(pr), p = diag_pp(pr);
        // table index along axis k: number of derivative factors on that axis
        const int t1 = (n == 0) + (p == 0), t2 = (n == 1) + (p == 1), t3 = (n == 2) + (p == 2);
        __syncthreads();
        for (int idx = threadIdx.x; idx < nel * 3 * NI * NQ * NQ; idx += BLOCK) {
            const int q1 = idx % NQ;
            int r = idx / NQ;
            const int q2 = r % NQ;
            r /= NQ;
            const int i3 = r % NI;
            r /= NI;  // el*3 + a
            const int el = r / 3, a = r % 3;
            const double *y = L.sQ + ((el * 6 + pr) * 3 + a) * NQ3 + q2 * NQ + q1;
            double s = 0.0;
#pragma unroll
            for (int q3 = 0; q3 < NQ; ++q3) s += L.T[t3][q3 * NI + i3] * y[q3 * NQ * NQ];
            L.U2[((r * NI + i3) * NQ + q2) * NQ + q1] = s;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < nel * 3 * NI * NI * NQ; idx += BLOCK) {
            const int q1 = idx % NQ;
            int r = idx / NQ;
            const int i2 = r % NI;
            r /= NI;
            const int i3 = r % NI;
            r /= NI;
            const double *y = L.U2 + (r * NI + i3) * NQ * NQ + q1;
            double s = 0.0;
#pragma unroll
            for (int q2 = 0; q2 < NQ; ++q2) s += L.T[t2][q2 * NI + i2] * y[q2 * NQ];
            L.U1[((r * NI + i3) * NI + i2) * NQ + q1] = s;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < nel * 3 * NP; idx += BLOCK) {
            const int i1 = idx % NI;
            const int rest = idx / NI;  // (r*NI + i3)*NI + i2
            const double *y = L.U1 + rest * NQ;
            double s = 0.0;
#pragma unroll
            for (int q1 = 0; q1 < NQ; ++q1) s += L.T[t1][q1 * NI + i1] * y[q1];
            L.sD[idx] += s;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nel * 3 * NP; k += BLOCK) dE[k] = L.sD[k];
}

template <int P, int NQ, typename TT>
__device__ inline void b3_diag(const Geom &g, const Tables &tb, const TT *__restrict__ H, double *__restrict__ dE, int e0, int nel)
{
    using S = S3<P, NQ>;
    __shared__ DiagLds3<P, NQ> L;
    for (int idx = threadIdx.x; idx < nel * S::NQ3; idx += BLOCK) {
        const int el = idx / S::NQ3, q = idx % S::NQ3;
        const TT *h = H + (size_t)(e0 + el) * 45 * S::NQ3 + q;
#pragma unroll
        for (int pr = 0; pr < 6; ++pr) {
            const int n = diag_pn(pr), p = diag_pp(pr);
            const double f = (n == p) ? 1.0 : 2.0;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                L.sQ[((el * 6 + pr) * 3 + a) * S::NQ3 + q] =
                    f * (double)h[sym_index<9>(a * 3 + n, a * 3 + p) * S::NQ3];
        }
    }
    diag_contract3<P, NQ>(tb, L, nel, dE + (size_t)e0 * 3 * S::NP);
}

// Diagonal from compact data: within one component a the cofactor-derivative
// term vanishes, so H[an,ap] = c_id (W^-1 W^-T)_np + c_tc (Tw_an Cw_ap +
// Cw_an Tw_ap) + c_cc Cw_an Cw_ap with Tw = T W^{-T}, Cw = C W^{-T}.
template <int P, int NQ, typename TT>
__device__ inline void b3_diagc(const Geom &g, const Tables &tb, const Target &tg, const TT *__restrict__ Q, double *__restrict__ dE, int e0, int nel)
{
    using S = S3<P, NQ>;
    __shared__ DiagLds3<P, NQ> L;
    for (int idx = threadIdx.x; idx < nel * S::NQ3; idx += BLOCK) {
        const int el = idx / S::NQ3, q = idx % S::NQ3;
        const TT *h = Q + (size_t)(e0 + el) * NC3 * S::NQ3 + q;
        double T[9], C[9], Tw[9], Cw[9], WW[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) T[k] = (double)h[k * S::NQ3];
        const double cid = h[9 * S::NQ3], ctc = h[10 * S::NQ3], ccc = h[11 * S::NQ3];
        cof3(T, C);
        if (tg.ideal) {
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                Tw[k] = T[k];
                Cw[k] = C[k];
                WW[k] = (k % 4 == 0) ? 1.0 : 0.0;
            }
        } else {
            mul_winv<3, double>(tg, T, Tw, true);
            mul_winv<3, double>(tg, C, Cw, true);
#pragma unroll
            for (int n = 0; n < 3; ++n)
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    double s = 0.0;
#pragma unroll
                    for (int k = 0; k < 3; ++k) s += tg.Winv[n * 3 + k] * tg.Winv[p * 3 + k];
                    WW[n * 3 + p] = s;
                }
        }
#pragma unroll
        for (int pr = 0; pr < 6; ++pr) {
            const int n = diag_pn(pr), p = diag_pp(pr);
            const double f = (n == p) ? 1.0 : 2.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double hv = cid * WW[n * 3 + p] +
                                  ctc * (Tw[a * 3 + n] * Cw[a * 3 + p] + Cw[a * 3 + n] * Tw[a * 3 + p]) +
                                  ccc * Cw[a * 3 + n] * Cw[a * 3 + p];
                L.sQ[((el * 6 + pr) * 3 + a) * S::NQ3 + q] = f * hv;
            }
        }
    }
    diag_contract3<P, NQ>(tb, L, nel, dE + (size_t)e0 * 3 * S::NP);
}

// ------------------------------------------------------------------------
// Kernel entry points: single mesh (grid over element blocks) and batched
// (grid over a tile list of (slot, first element) with per-slot geometry,
// target and offsets into packed pools).
// ------------------------------------------------------------------------

template <int P, int NQ>
__global__ __launch_bounds__(BLOCK) void k3_energy(Geom g, Tables tb, Target tg, const double *__restrict__ x, double *__restrict__ part)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const int e0 = blockIdx.x * EPB;
    b3_energy<P, NQ>(g, tb, tg, x, part, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ>
__global__ __launch_bounds__(BLOCK) void k3_gradient(Geom g, Tables tb, Target tg, const double *__restrict__ x, double *__restrict__ gE, double *__restrict__ bad)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const int e0 = blockIdx.x * EPB;
    b3_gradient<P, NQ>(g, tb, tg, x, gE, bad, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT>
__global__ __launch_bounds__(BLOCK) void k3_setup(Geom g, Tables tb, Target tg, const double *__restrict__ x, TT *__restrict__ H, double *__restrict__ bad)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const int e0 = blockIdx.x * EPB;
    b3_setup<P, NQ, TT>(g, tb, tg, x, H, bad, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT, typename CT>
__global__ __launch_bounds__(BLOCK) void k3_apply(Geom g, Tables tb, const TT *__restrict__ H, const double *__restrict__ v, CT *__restrict__ yE)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const int e0 = blockIdx.x * EPB;
    b3_apply<P, NQ, TT, CT>(g, tb, H, v, yE, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT>
__global__ __launch_bounds__(BLOCK) void k3_setupc(Geom g, Tables tb, Target tg, const double *__restrict__ x, TT *__restrict__ Q, double *__restrict__ bad)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const int e0 = blockIdx.x * EPB;
    b3_setupc<P, NQ, TT>(g, tb, tg, x, Q, bad, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT, typename CT>
__global__ __launch_bounds__(BLOCK) void k3_applyc(Geom g, Tables tb, Target tg, const TT *__restrict__ Q, const double *__restrict__ v, CT *__restrict__ yE)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const int e0 = blockIdx.x * EPB;
    b3_applyc<P, NQ, TT, CT>(g, tb, tg, Q, v, yE, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT>
__global__ __launch_bounds__(BLOCK) void k3_diag(Geom g, Tables tb, const TT *__restrict__ H, double *__restrict__ dE)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const int e0 = blockIdx.x * EPB;
    b3_diag<P, NQ, TT>(g, tb, H, dE, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT>
__global__ __launch_bounds__(BLOCK) void k3_diagc(Geom g, Tables tb, Target tg, const TT *__restrict__ Q, double *__restrict__ dE)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const int e0 = blockIdx.x * EPB;
    b3_diagc<P, NQ, TT>(g, tb, tg, Q, dE, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ>
__global__ __launch_bounds__(BLOCK) void kb3_energy(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate, int vin, double *__restrict__ part)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b3_energy<P, NQ>(s.g, tb, s.tg, s.vec[vin], part, t.e0, min(EPB, s.g.ne - t.e0));
}

template <int P, int NQ>
__global__ __launch_bounds__(BLOCK) void kb3_gradient(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate, int vin, double *__restrict__ bad)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b3_gradient<P, NQ>(s.g, tb, s.tg, s.vec[vin], (double *)s.eV, bad, t.e0, min(EPB, s.g.ne - t.e0));
}

template <int P, int NQ, typename TT>
__global__ __launch_bounds__(BLOCK) void kb3_setup(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate, int vin, double *__restrict__ bad)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b3_setup<P, NQ, TT>(s.g, tb, s.tg, s.vec[vin], (TT *)s.H, bad, t.e0, min(EPB, s.g.ne - t.e0));
}

template <int P, int NQ, typename TT, typename CT>
__global__ __launch_bounds__(BLOCK) void kb3_apply(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate, int vin)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b3_apply<P, NQ, TT, CT>(s.g, tb, (const TT *)s.H, s.vec[vin], (CT *)s.eV, t.e0, min(EPB, s.g.ne - t.e0));
}

template <int P, int NQ, typename TT>
__global__ __launch_bounds__(BLOCK) void kb3_setupc(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate, int vin, double *__restrict__ bad)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b3_setupc<P, NQ, TT>(s.g, tb, s.tg, s.vec[vin], (TT *)s.H, bad, t.e0, min(EPB, s.g.ne - t.e0));
}

template <int P, int NQ, typename TT, typename CT>
__global__ __launch_bounds__(BLOCK) void kb3_applyc(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate, int vin)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b3_applyc<P, NQ, TT, CT>(s.g, tb, s.tg, (const TT *)s.H, s.vec[vin], (CT *)s.eV, t.e0, min(EPB, s.g.ne - t.e0));
}

template <int P, int NQ, typename TT>
__global__ __launch_bounds__(BLOCK) void kb3_diag(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b3_diag<P, NQ, TT>(s.g, tb, (const TT *)s.H, (double *)s.eV, t.e0, min(EPB, s.g.ne - t.e0));
}

template <int P, int NQ, typename TT>
__global__ __launch_bounds__(BLOCK) void kb3_diagc(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b3_diagc<P, NQ, TT>(s.g, tb, s.tg, (const TT *)s.H, (double *)s.eV, t.e0, min(EPB, s.g.ne - t.e0));
}

}  // namespace tmop
