// 2D (quad) PA-TMOP kernels, templated on the order P and the points per
// direction NQ.  Same structure as the hex kernels with two 1D contractions
// (Sec. 3.2):
//   A_a1(q) = sum_i1 G[q1][i1] sum_i2 B[q2][i2] x_a(i1,i2),
//   A_a2(q) = sum_i1 B[q1][i1] sum_i2 G[q2][i2] x_a(i1,i2).
// Pencil sweeps with the 1D tables read from the kernel arguments (scalar
// operands).  LDS per workgroup:
//   X   [EPB][2][NI^2]          element nodes (or v_E)
//   R1  [EPB][2][2][NI][NQ]     after the axis-1 contraction (B, G variants)
//   RY  [EPB][NR][NQ^2]         J (planes c*2+b), then Y or P; with the
//                               limiting term (NR = 6) the values of
//                               component c in plane 4+c
// with X and RY overlaid (X is dead once the axis-1 sweep has read it).
#pragma once
#include "tmop_dev.hpp"

namespace tmop {

template <int P, int NQ>
struct S2 {
    static constexpr int NI = P + 1;
    static constexpr int NP = NI * NI;
    static constexpr int NQ2 = NQ * NQ;
    static constexpr int EPB = NQ2 >= BLOCK ? 1 : BLOCK / NQ2;
    static constexpr int L1 = NI * NQ;
    static constexpr int NS = 10;
};

template <int P, int NQ, typename CT, int NR = 4>
struct Lds2 {
    using S = S2<P, NQ>;
    union {
        CT X[S::EPB * 2 * S::NP];
        CT RY[S::EPB * NR * S::NQ2];
    };
    CT R1[S::EPB * 4 * S::L1];
};

template <bool LIM>
struct Planes2 {
    static constexpr int NR = LIM ? 6 : 4;
};

template <int P>
__device__ __forceinline__ int node2(const Geom &g, int e, int i1, int i2, int &gx, int &gy)
{
    constexpr int NI = P + 1;
    if (g.e2n) {
        gx = gy = -1;
        return g.e2n[(size_t)e * (NI * NI) + i1 + NI * i2];
    }
    int ex, ey, ez;
    box_elem<2>(g, e, ex, ey, ez);
    gx = ex * P + i1;
    gy = ey * P + i2;
    return gx + g.M[0] * gy;
}

// E-vector index of (element e, component c, local node i1,i2): element-major
// [e][c][i] on general meshes, the exploded grid [c][ey*NI+i2][ex*NI+i1] on
// the structured box (the layout the node gather expects).
template <int P>
__device__ __forceinline__ long ev_index2(const Geom &g, int e, int c, int i1, int i2)
{
    constexpr int NI = P + 1, NP = NI * NI;
    if (g.e2n) return ((long)e * 2 + c) * NP + i1 + NI * i2;
    int ex, ey, ez;
    box_elem<2>(g, e, ex, ey, ez);
    const long EX = (long)g.nel[0] * NI;
    return (long)c * g.ne * NP + (long)(ey * NI + i2) * EX + ex * NI + i1;
}

// Gather 2 components of a global vector into X (masked: fixed DoFs as zero;
// sub: a vector subtracted entry by entry).
template <int P, int NQ, typename CT>
__device__ __forceinline__ void gather2(const Geom &g, const double *__restrict__ vec, int e0, int nel,
                               CT *sX, bool masked, const double *__restrict__ sub = nullptr)
{
    using S = S2<P, NQ>;
    constexpr int NI = S::NI, NP = S::NP;
    constexpr int NIT = (S::EPB * 2 * NP + BLOCK - 1) / BLOCK;
    const int n = nel * 2 * NP;
    double val[NIT];
    bool fix[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int idx = threadIdx.x + it * BLOCK;
        val[it] = 0.0;
        fix[it] = false;
        if (idx < n) {
            const int i = idx % NP;
            const int r = idx / NP;  // el*2 + c
            const int c = r % 2, el = r / 2;
            int gx, gy;
            const int node = node2<P>(g, e0 + el, i % NI, i / NI, gx, gy);
            val[it] = vec[(size_t)c * g.nx + node];
            if (sub) val[it] -= sub[(size_t)c * g.nx + node];
            fix[it] = masked && is_fixed(g, c, node, gx, gy, 0);
        }
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int idx = threadIdx.x + it * BLOCK;
        if (idx < n) sX[idx] = fix[it] ? (CT)0 : (CT)val[it];
    }
}

// Forward sweeps X -> R1 -> RY: J (plane el*NR + c*2 + b), with VAL also the
// value of component c (plane el*NR + 4 + c).
template <int P, int NQ, typename CT, int NR = 4, bool VAL = false>
__device__ __forceinline__ void forward2(const Tables &tb, const CT *X, CT *R1, CT *RY, int nel)
{
    using S = S2<P, NQ>;
    constexpr int NI = S::NI, NP = S::NP, L1 = S::L1, NQ2 = S::NQ2;
    // axis 1: pencils (r, i2), r = el*2 + c
    for (int pen = threadIdx.x; pen < nel * 2 * NI; pen += BLOCK) {
        const int i2 = pen % NI, r = pen / NI;
        const CT *x = X + r * NP + i2 * NI;
        CT xv[NI];
#pragma unroll
        for (int k = 0; k < NI; ++k) xv[k] = x[k];
        CT *o = R1 + r * 2 * L1 + i2 * NQ;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            CT b = 0, d = 0;
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                b += tabB<CT>(tb, q * NI + k) * xv[k];
                d += tabG<CT>(tb, q * NI + k) * xv[k];
            }
            o[q] = b;
            o[L1 + q] = d;
        }
    }
    __syncthreads();
    // axis 2: pencils (r, q1)
    for (int pen = threadIdx.x; pen < nel * 2 * NQ; pen += BLOCK) {
        const int q1 = pen % NQ, r = pen / NQ;
        const int el = r / 2, c = r % 2;
        const CT *t = R1 + r * 2 * L1 + q1;  // [i2] stride NQ
        CT xb[NI], xg[NI];
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            xb[k] = t[k * NQ];
            xg[k] = t[L1 + k * NQ];
        }
        CT *o = RY + (el * NR + c * 2) * NQ2 + q1;
        CT *ov = RY + (el * NR + 4 + c) * NQ2 + q1;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            CT a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                const CT b2 = tabB<CT>(tb, q * NI + k), g2 = tabG<CT>(tb, q * NI + k);
                a0 += b2 * xg[k];
                a1 += g2 * xb[k];
                if (VAL) a2 += b2 * xb[k];
            }
            o[q * NQ] = a0;
            o[NQ2 + q * NQ] = a1;
            if (VAL) ov[q * NQ] = a2;
        }
    }
    __syncthreads();
}

// Backward (transposed) sweeps RY -> R1 -> E-vector:
//   y_c(i) = sum_q sum_b RY[c][b](q) d w_i/d xbar_b (q)  (+ RY[4+c](q) w_i(q) with VAL).
template <int P, int NQ, typename CT, typename OT, int NR = 4, bool VAL = false>
__device__ __forceinline__ void backward2(const Tables &tb, const Geom &g, int e0, const CT *RY, CT *R1,
                                 int nel, OT *__restrict__ out)
{
    using S = S2<P, NQ>;
    constexpr int NI = S::NI, L1 = S::L1, NQ2 = S::NQ2;
    // axis 2: pencils (r, q1)
    for (int pen = threadIdx.x; pen < nel * 2 * NQ; pen += BLOCK) {
        const int q1 = pen % NQ, r = pen / NQ;
        const int el = r / 2, c = r % 2;
        const CT *y = RY + (el * NR + c * 2) * NQ2 + q1;  // [b] stride NQ^2, [q2] stride NQ
        const CT *yv = RY + (el * NR + 4 + c) * NQ2 + q1;
        CT y0[NQ], y1[NQ], ym[VAL ? NQ : 1];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            y0[q] = y[q * NQ];
            y1[q] = y[NQ2 + q * NQ];
            if (VAL) ym[q] = yv[q * NQ];
        }
        CT *o = R1 + r * 2 * L1 + q1;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            CT u0 = 0, u1 = 0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const CT b2 = tabB<CT>(tb, q * NI + k), g2 = tabG<CT>(tb, q * NI + k);
                u0 += b2 * y0[q];
                u1 += g2 * y1[q];
                if (VAL) u1 += b2 * ym[q];
            }
            o[k * NQ] = u0;       // G along axis 1 still to apply
            o[L1 + k * NQ] = u1;  // B along axis 1 still to apply
        }
    }
    __syncthreads();
    // axis 1: pencils (r, i2) -> NI consecutive outputs
    for (int pen = threadIdx.x; pen < nel * 2 * NI; pen += BLOCK) {
        const int i2 = pen % NI, r = pen / NI;
        const int c = r % 2, el = r / 2;
        const CT *t = R1 + r * 2 * L1 + i2 * NQ;
        CT u0[NQ], u1[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            u0[q] = t[q];
            u1[q] = t[L1 + q];
        }
        OT *o = out + ev_index2<P>(g, e0 + el, c, 0, i2);
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            CT s = 0;
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                s += tabG<CT>(tb, q * NI + k) * u0[q] + tabB<CT>(tb, q * NI + k) * u1[q];
            o[k] = (OT)s;
        }
    }
}

template <int P, int NQ, typename CT, int NR = 4>
__device__ __forceinline__ void point_J2(const CT *RY, int el, int q, CT *J)
{
    constexpr int NQ2 = NQ * NQ;
#pragma unroll
    for (int k = 0; k < 4; ++k) J[k] = RY[(el * NR + k) * NQ2 + q];
}

template <int NQ>
__device__ __forceinline__ double qweight2(const Tables &tb, int q)
{
    return tab_w<NQ>(tb, q % NQ) * tab_w<NQ>(tb, q / NQ);
}

// Values of x - x0 at the points into U[el][c][q] (limiting term).
template <int P, int NQ, typename L2>
__device__ __forceinline__ void lim_values2(const Geom &g, const Tables &tb, const double *__restrict__ x,
                                   int e0, int nel, L2 &L, double *U)
{
    using S = S2<P, NQ>;
    gather2<P, NQ>(g, x, e0, nel, L.X, false, g.x0);
    __syncthreads();
    forward2<P, NQ, double, 6, true>(tb, L.X, L.R1, L.RY, nel);
    for (int idx = threadIdx.x; idx < nel * 2 * S::NQ2; idx += BLOCK) {
        const int q = idx % S::NQ2, r = idx / S::NQ2;  // r = el*2 + c
        U[idx] = L.RY[((r / 2) * 6 + 4 + r % 2) * S::NQ2 + q];
    }
    __syncthreads();
}

// Limiting term in the Hessian action: value planes v_c(q) -> 2 w_q lim v_c(q).
template <int NQ, typename CT, int NR>
__device__ __forceinline__ void lim_point2(const Tables &tb, const Geom &g, int el, int q, CT *RY)
{
    constexpr int NQ2 = NQ * NQ;
    const CT f = (CT)(2.0 * g.lim * qweight2<NQ>(tb, q));
#pragma unroll
    for (int c = 0; c < 2; ++c) RY[(el * NR + 4 + c) * NQ2 + q] *= f;
}

// ------------------------------------------------------------------------
// Element bodies (see the hex kernels for the description of each)
// ------------------------------------------------------------------------

template <int P, int NQ, bool LIM = false>
__device__ __forceinline__ void b2_energy(const Geom &g, const Tables &tb, const Target &tg,
                                 const double *__restrict__ x, double *__restrict__ part, int e0,
                                 int nel)
{
    using S = S2<P, NQ>;
    constexpr int NR = Planes2<LIM>::NR;
    __shared__ Lds2<P, NQ, double, NR> L;
    __shared__ double U[LIM ? S::EPB * 2 * S::NQ2 : 1];
    __shared__ double red[3 * (BLOCK / 64)];
    if (LIM) lim_values2<P, NQ>(g, tb, x, e0, nel, L, U);
    gather2<P, NQ>(g, x, e0, nel, L.X, false);
    __syncthreads();
    forward2<P, NQ, double, NR>(tb, L.X, L.R1, L.RY, nel);
    double esum = 0.0, dmin = 1.0e300, bad = 0.0;
    for (int idx = threadIdx.x; idx < nel * S::NQ2; idx += BLOCK) {
        const int el = idx / S::NQ2, q = idx % S::NQ2;
        double J[4], Pm[4], mu;
        point_J2<P, NQ, double, NR>(L.RY, el, q, J);
        dmin = fmin(dmin, det_only<2>(J));
        const double z = qweight2<NQ>(tb, q) * tg.detW;
        if (metric_first<2>(tg, J, z, &mu, Pm))
            esum += z * mu;
        else
            bad += 1.0;
        if (LIM) {
            const double u0 = U[(el * 2) * S::NQ2 + q], u1 = U[(el * 2 + 1) * S::NQ2 + q];
            esum += qweight2<NQ>(tb, q) * g.lim * (u0 * u0 + u1 * u1);
        }
    }
    block_energy3(esum, dmin, bad, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = esum;
        part[gridDim.x + blockIdx.x] = dmin;
        part[2 * gridDim.x + blockIdx.x] = bad;
    }
}

// EN: also the energy partials of b2_energy, as in b3_gradient.
template <int P, int NQ, bool LIM = false, bool EN = false>
__device__ __forceinline__ void b2_gradient(const Geom &g, const Tables &tb, const Target &tg,
                                   const double *__restrict__ x, double *__restrict__ gE,
                                   double *__restrict__ bad, int e0, int nel)
{
    using S = S2<P, NQ>;
    constexpr int NR = Planes2<LIM>::NR;
    __shared__ Lds2<P, NQ, double, NR> L;
    __shared__ double U[LIM ? S::EPB * 2 * S::NQ2 : 1];
    __shared__ double red[3 * (BLOCK / 64)];
    if (LIM) lim_values2<P, NQ>(g, tb, x, e0, nel, L, U);
    gather2<P, NQ>(g, x, e0, nel, L.X, false);
    __syncthreads();
    forward2<P, NQ, double, NR>(tb, L.X, L.R1, L.RY, nel);
    double nbad = 0.0, esum = 0.0, dmin = 1.0e300;
    for (int idx = threadIdx.x; idx < nel * S::NQ2; idx += BLOCK) {
        const int el = idx / S::NQ2, q = idx % S::NQ2;
        double J[4], Pm[4], mu;
        point_J2<P, NQ, double, NR>(L.RY, el, q, J);
        if (EN) dmin = fmin(dmin, det_only<2>(J));
        const double z = qweight2<NQ>(tb, q) * tg.detW;
        if (!metric_first<2>(tg, J, z, &mu, Pm)) {
            nbad += 1.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) Pm[k] = 0.0;
        } else if (EN) {
            esum += z * mu;
        }
        if (EN && LIM) {
            const double u0 = U[(el * 2) * S::NQ2 + q], u1 = U[(el * 2 + 1) * S::NQ2 + q];
            esum += qweight2<NQ>(tb, q) * g.lim * (u0 * u0 + u1 * u1);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) L.RY[(el * NR + k) * S::NQ2 + q] = Pm[k];
        if (LIM) {
#pragma unroll
            for (int c = 0; c < 2; ++c)
                L.RY[(el * NR + 4 + c) * S::NQ2 + q] =
                    2.0 * qweight2<NQ>(tb, q) * g.lim * U[(el * 2 + c) * S::NQ2 + q];
        }
    }
    __syncthreads();
    backward2<P, NQ, double, double, NR, LIM>(tb, g, e0, L.RY, L.R1, nel, gE);
    if (EN) {
        block_energy3(esum, dmin, nbad, red);
        if (threadIdx.x == 0) {
            bad[blockIdx.x] = esum;
            bad[gridDim.x + blockIdx.x] = dmin;
            bad[2 * gridDim.x + blockIdx.x] = nbad;
        }
    } else {
        const double b = block_sum(nbad, red);
        if (threadIdx.x == 0) bad[blockIdx.x] = b;
    }
}

template <int P, int NQ, typename TT>
__device__ __forceinline__ void b2_setup(const Geom &g, const Tables &tb, const Target &tg,
                                const double *__restrict__ x, TT *__restrict__ H,
                                double *__restrict__ bad, int e0, int nel)
{
    using S = S2<P, NQ>;
    __shared__ Lds2<P, NQ, double> L;
    __shared__ double red[BLOCK / 64];
    gather2<P, NQ>(g, x, e0, nel, L.X, false);
    __syncthreads();
    forward2<P, NQ, double>(tb, L.X, L.R1, L.RY, nel);
    double nbad = 0.0;
    for (int idx = threadIdx.x; idx < nel * S::NQ2; idx += BLOCK) {
        const int el = idx / S::NQ2, q = idx % S::NQ2;
        double J[4], Hp[10];
        point_J2<P, NQ>(L.RY, el, q, J);
        const double z = qweight2<NQ>(tb, q) * tg.detW;
        if (!metric_second<2>(tg, J, z, Hp)) {
            nbad += 1.0;
#pragma unroll
            for (int k = 0; k < 10; ++k) Hp[k] = 0.0;
        }
        TT *h = H + (size_t)(e0 + el) * qdata_stride(10, S::NQ2, sizeof(TT)) + q;
#pragma unroll
        for (int k = 0; k < 10; ++k) h[k * S::NQ2] = (TT)Hp[k];
    }
    const double b = block_sum(nbad, red);
    if (threadIdx.x == 0) bad[blockIdx.x] = b;
}

template <int P, int NQ, typename TT, typename CT, bool LIM = false>
__device__ __forceinline__ void b2_apply(const Geom &g, const Tables &tb, const TT *__restrict__ H,
                                const double *__restrict__ v, CT *__restrict__ yE, int e0, int nel)
{
    using S = S2<P, NQ>;
    constexpr int NR = Planes2<LIM>::NR;
    __shared__ Lds2<P, NQ, CT, NR> L;
    gather2<P, NQ>(g, v, e0, nel, L.X, true);
    __syncthreads();
    forward2<P, NQ, CT, NR, LIM>(tb, L.X, L.R1, L.RY, nel);
    for (int idx = threadIdx.x; idx < nel * S::NQ2; idx += BLOCK) {
        const int el = idx / S::NQ2, q = idx % S::NQ2;
        const TT *h = H + (size_t)(e0 + el) * qdata_stride(10, S::NQ2, sizeof(TT)) + q;
        CT hv[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) hv[k] = (CT)h[k * S::NQ2];
        CT J[4];
        point_J2<P, NQ, CT, NR>(L.RY, el, q, J);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            CT s = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) s += hv[sym_index<4>(r, c)] * J[c];
            L.RY[(el * NR + r) * S::NQ2 + q] = s;
        }
        if (LIM) lim_point2<NQ, CT, NR>(tb, g, el, q, L.RY);
    }
    __syncthreads();
    backward2<P, NQ, CT, CT, NR, LIM>(tb, g, e0, L.RY, L.R1, nel, yE);
}

// ------------------------------------------------------------------------
// Compact quadrature data for quads: T (4) and z c_id, z c_tc, z c_cc, z c_dc,
// layout [e][8][q].  In 2D C = cof T = [[T11, -T10], [-T01, T00]] and the
// cofactor derivative is the constant map dC[M] = cof M.
// ------------------------------------------------------------------------
constexpr int NC2 = 8;

template <typename CT>
__device__ __forceinline__ void compact_action2(const CT *T, CT ca, CT cb, CT cc, CT cd, const CT *M, CT *Y)
{
    const CT C[4] = {T[3], -T[2], -T[1], T[0]};
    const CT dC[4] = {M[3], -M[2], -M[1], M[0]};
    CT tm = 0, cm = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        tm += T[k] * M[k];
        cm += C[k] * M[k];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        Y[r] = ca * M[r] + cb * (T[r] * cm + C[r] * tm) + cc * C[r] * cm + cd * dC[r];
}

template <typename CT>
__device__ __forceinline__ void mul_winv2(const Target &t, const CT *in, CT *out, bool tr)
{
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            CT s = 0;
#pragma unroll
            for (int n = 0; n < 2; ++n)
                s += in[a * 2 + n] * (CT)(tr ? t.Winv[k * 2 + n] : t.Winv[n * 2 + k]);
            out[a * 2 + k] = s;
        }
}


template <int P, int NQ, typename TT>
__device__ __forceinline__ void b2_setupc(const Geom &g, const Tables &tb, const Target &tg,
                                 const double *__restrict__ x, TT *__restrict__ Q,
                                 double *__restrict__ bad, int e0, int nel)
{
    using S = S2<P, NQ>;
    __shared__ Lds2<P, NQ, double> L;
    __shared__ double red[BLOCK / 64];
    gather2<P, NQ>(g, x, e0, nel, L.X, false);
    __syncthreads();
    forward2<P, NQ, double>(tb, L.X, L.R1, L.RY, nel);
    double nbad = 0.0;
    for (int idx = threadIdx.x; idx < nel * S::NQ2; idx += BLOCK) {
        const int el = idx / S::NQ2, q = idx % S::NQ2;
        double J[4], T[4], C[4], out[NC2];
        point_J2<P, NQ>(L.RY, el, q, J);
        apply_winv<2>(tg, J, T);
        const double tau = det_cof<2>(T, C);
        const double z = qweight2<NQ>(tb, q) * tg.detW;
        if (tau > 0.0) {
            double I1 = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) I1 += T[k] * T[k];
            const MetricCoef m = metric_coef(tg.metric, I1, tau);
#pragma unroll
            for (int k = 0; k < 4; ++k) out[k] = T[k];
            out[4] = z * m.c_id;
            out[5] = z * m.c_tc;
            out[6] = z * m.c_cc;
            out[7] = z * m.c_dc;
        } else {
            nbad += 1.0;
#pragma unroll
            for (int k = 0; k < NC2; ++k) out[k] = 0.0;
        }
        TT *h = Q + (size_t)(e0 + el) * qdata_stride(NC2, S::NQ2, sizeof(TT)) + q;
#pragma unroll
        for (int k = 0; k < NC2; ++k) h[k * S::NQ2] = (TT)out[k];
    }
    const double b = block_sum(nbad, red);
    if (threadIdx.x == 0) bad[blockIdx.x] = b;
}

template <int P, int NQ, typename TT, typename CT, bool LIM = false>
__device__ __forceinline__ void b2_applyc(const Geom &g, const Tables &tb, const Target &tg,
                                 const TT *__restrict__ Q, const double *__restrict__ v,
                                 CT *__restrict__ yE, int e0, int nel)
{
    using S = S2<P, NQ>;
    constexpr int NR = Planes2<LIM>::NR;
    __shared__ Lds2<P, NQ, CT, NR> L;
    gather2<P, NQ>(g, v, e0, nel, L.X, true);
    __syncthreads();
    forward2<P, NQ, CT, NR, LIM>(tb, L.X, L.R1, L.RY, nel);
    for (int idx = threadIdx.x; idx < nel * S::NQ2; idx += BLOCK) {
        const int el = idx / S::NQ2, q = idx % S::NQ2;
        const TT *h = Q + (size_t)(e0 + el) * qdata_stride(NC2, S::NQ2, sizeof(TT)) + q;
        CT d[NC2];
#pragma unroll
        for (int k = 0; k < NC2; ++k) d[k] = (CT)h[k * S::NQ2];
        CT J[4], Y[4];
        point_J2<P, NQ, CT, NR>(L.RY, el, q, J);
        if (tg.ideal) {
            compact_action2<CT>(d, d[4], d[5], d[6], d[7], J, Y);
        } else {
            CT M[4], Yt[4];
            mul_winv2<CT>(tg, J, M, false);
            compact_action2<CT>(d, d[4], d[5], d[6], d[7], M, Yt);
            mul_winv2<CT>(tg, Yt, Y, true);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) L.RY[(el * NR + r) * S::NQ2 + q] = Y[r];
        if (LIM) lim_point2<NQ, CT, NR>(tb, g, el, q, L.RY);
    }
    __syncthreads();
    backward2<P, NQ, CT, CT, NR, LIM>(tb, g, e0, L.RY, L.R1, nel, yE);
}

// Hessian diagonal (Sec. 3.4): 2 components x 3 pairs (n <= p) of planes
// sQ[el][pair][a][q], then one contraction pass per pair with BB, BG, GG; with
// the limiting term a fourth pair 2 w_q lim contracted with BB on both axes.
template <int P, int NQ, bool LIM = false>
struct DiagLds2 {
    using S = S2<P, NQ>;
    static constexpr int NPR = LIM ? 4 : 3;
    double T[3][NQ * S::NI];
    double sQ[S::EPB * NPR * 2 * S::NQ2];
    double U1[S::EPB * 2 * S::NI * NQ];
    double sD[S::EPB * 2 * S::NP];
};

template <int P, int NQ, bool LIM>
__device__ __forceinline__ void diag_contract2(const Tables &tb, const Geom &g, int e0,
                                      DiagLds2<P, NQ, LIM> &L, int nel, double *__restrict__ dE)
{
    using S = S2<P, NQ>;
    constexpr int NI = S::NI, NQ2 = S::NQ2, NP = S::NP, NPR = DiagLds2<P, NQ, LIM>::NPR;
    for (int k = threadIdx.x; k < NQ * NI; k += BLOCK) {
        const double b = tb.B[k], gg = tb.G[k];
        L.T[0][k] = b * b;
        L.T[1][k] = b * gg;
        L.T[2][k] = gg * gg;
    }
    for (int k = threadIdx.x; k < nel * 2 * NP; k += BLOCK) L.sD[k] = 0.0;
    for (int pr = 0; pr < NPR; ++pr) {
        const int n = pr == 2 ? 1 : 0, p = pr == 0 ? 0 : 1;
        const bool val = pr == 3;
        const int t1 = val ? 0 : (n == 0) + (p == 0), t2 = val ? 0 : (n == 1) + (p == 1);
        __syncthreads();
        for (int idx = threadIdx.x; idx < nel * 2 * NI * NQ; idx += BLOCK) {
            const int q1 = idx % NQ;
            int r = idx / NQ;
            const int i2 = r % NI;
            r /= NI;  // el*2 + a
            const int el = r / 2, a = r % 2;
            const double *y = L.sQ + ((el * NPR + pr) * 2 + a) * NQ2 + q1;
            double s = 0.0;
#pragma unroll
            for (int q2 = 0; q2 < NQ; ++q2) s += L.T[t2][q2 * NI + i2] * y[q2 * NQ];
            L.U1[(r * NI + i2) * NQ + q1] = s;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < nel * 2 * NP; idx += BLOCK) {
            const int i1 = idx % NI;
            const int rest = idx / NI;
            const double *y = L.U1 + rest * NQ;
            double s = 0.0;
#pragma unroll
            for (int q1 = 0; q1 < NQ; ++q1) s += L.T[t1][q1 * NI + i1] * y[q1];
            L.sD[idx] += s;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nel * 2 * NP; k += BLOCK) {
        const int i = k % NP, r = k / NP;
        dE[ev_index2<P>(g, e0 + r / 2, r % 2, i % NI, i / NI)] = L.sD[k];
    }
}

template <int P, int NQ, bool LIM>
__device__ __forceinline__ void diag_lim2(const Tables &tb, const Geom &g, DiagLds2<P, NQ, LIM> &L, int el,
                                 int q)
{
    if (!LIM) return;
    constexpr int NQ2 = NQ * NQ, NPR = DiagLds2<P, NQ, LIM>::NPR;
    const double f = 2.0 * g.lim * qweight2<NQ>(tb, q);
#pragma unroll
    for (int a = 0; a < 2; ++a) L.sQ[((el * NPR + 3) * 2 + a) * NQ2 + q] = f;
}

template <int P, int NQ, typename TT, bool LIM = false>
__device__ __forceinline__ void b2_diag(const Geom &g, const Tables &tb, const TT *__restrict__ H,
                               double *__restrict__ dE, int e0, int nel)
{
    using S = S2<P, NQ>;
    constexpr int NPR = DiagLds2<P, NQ, LIM>::NPR;
    __shared__ DiagLds2<P, NQ, LIM> L;
    for (int idx = threadIdx.x; idx < nel * S::NQ2; idx += BLOCK) {
        const int el = idx / S::NQ2, q = idx % S::NQ2;
        const TT *h = H + (size_t)(e0 + el) * qdata_stride(10, S::NQ2, sizeof(TT)) + q;
#pragma unroll
        for (int pr = 0; pr < 3; ++pr) {
            const int n = pr == 2 ? 1 : 0, p = pr == 0 ? 0 : 1;
            const double f = (n == p) ? 1.0 : 2.0;
#pragma unroll
            for (int a = 0; a < 2; ++a)
                L.sQ[((el * NPR + pr) * 2 + a) * S::NQ2 + q] =
                    f * (double)h[sym_index<4>(a * 2 + n, a * 2 + p) * S::NQ2];
        }
        diag_lim2<P, NQ, LIM>(tb, g, L, el, q);
    }
    diag_contract2<P, NQ, LIM>(tb, g, e0, L, nel, dE);
}

template <int P, int NQ, typename TT, bool LIM = false>
__device__ __forceinline__ void b2_diagc(const Geom &g, const Tables &tb, const Target &tg,
                                const TT *__restrict__ Q, double *__restrict__ dE, int e0, int nel)
{
    using S = S2<P, NQ>;
    constexpr int NPR = DiagLds2<P, NQ, LIM>::NPR;
    __shared__ DiagLds2<P, NQ, LIM> L;
    for (int idx = threadIdx.x; idx < nel * S::NQ2; idx += BLOCK) {
        const int el = idx / S::NQ2, q = idx % S::NQ2;
        const TT *h = Q + (size_t)(e0 + el) * qdata_stride(NC2, S::NQ2, sizeof(TT)) + q;
        double T[4], Tw[4], Cw[4], WW[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) T[k] = (double)h[k * S::NQ2];
        const double cid = h[4 * S::NQ2], ctc = h[5 * S::NQ2], ccc = h[6 * S::NQ2];
        const double C[4] = {T[3], -T[2], -T[1], T[0]};
        if (tg.ideal) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                Tw[k] = T[k];
                Cw[k] = C[k];
                WW[k] = (k % 3 == 0) ? 1.0 : 0.0;
            }
        } else {
            mul_winv2<double>(tg, T, Tw, true);
            mul_winv2<double>(tg, C, Cw, true);
#pragma unroll
            for (int n = 0; n < 2; ++n)
#pragma unroll
                for (int p = 0; p < 2; ++p)
                    WW[n * 2 + p] = tg.Winv[n * 2] * tg.Winv[p * 2] + tg.Winv[n * 2 + 1] * tg.Winv[p * 2 + 1];
        }
#pragma unroll
        for (int pr = 0; pr < 3; ++pr) {
            const int n = pr == 2 ? 1 : 0, p = pr == 0 ? 0 : 1;
            const double f = (n == p) ? 1.0 : 2.0;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const double hv = cid * WW[n * 2 + p] +
                                  ctc * (Tw[a * 2 + n] * Cw[a * 2 + p] + Cw[a * 2 + n] * Tw[a * 2 + p]) +
                                  ccc * Cw[a * 2 + n] * Cw[a * 2 + p];
                L.sQ[((el * NPR + pr) * 2 + a) * S::NQ2 + q] = f * hv;
            }
        }
        diag_lim2<P, NQ, LIM>(tb, g, L, el, q);
    }
    diag_contract2<P, NQ, LIM>(tb, g, e0, L, nel, dE);
}

// ------------------------------------------------------------------------
// Kernel entry points: single mesh (grid over element blocks; LIM selects the
// variant with the limiting term) and batched (grid over a tile list of
// (slot, first element) with per-slot geometry, target and offsets into
// packed pools; no limiting term).
// ------------------------------------------------------------------------

template <int P, int NQ, bool LIM>
__global__ __launch_bounds__(BLOCK) void k2_energy(Geom g, Tables tb, Target tg, const double *__restrict__ x, double *__restrict__ part)
{
    constexpr int EPB = S2<P, NQ>::EPB;
    const int e0 = blockIdx.x * EPB;
    b2_energy<P, NQ, LIM>(g, tb, tg, x, part, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, bool LIM, bool EN = false>
__global__ __launch_bounds__(BLOCK) void k2_gradient(Geom g, Tables tb, Target tg, const double *__restrict__ x, double *__restrict__ gE, double *__restrict__ bad)
{
    constexpr int EPB = S2<P, NQ>::EPB;
    const int e0 = blockIdx.x * EPB;
    b2_gradient<P, NQ, LIM, EN>(g, tb, tg, x, gE, bad, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT>
__global__ __launch_bounds__(BLOCK) void k2_setup(Geom g, Tables tb, Target tg, const double *__restrict__ x, TT *__restrict__ H, double *__restrict__ bad)
{
    constexpr int EPB = S2<P, NQ>::EPB;
    const int e0 = blockIdx.x * EPB;
    b2_setup<P, NQ, TT>(g, tb, tg, x, H, bad, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT, typename CT, bool LIM>
__global__ __launch_bounds__(BLOCK) void k2_apply(Geom g, Tables tb, const TT *__restrict__ H, const double *__restrict__ v, CT *__restrict__ yE)
{
    constexpr int EPB = S2<P, NQ>::EPB;
    const int e0 = blockIdx.x * EPB;
    b2_apply<P, NQ, TT, CT, LIM>(g, tb, H, v, yE, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT>
__global__ __launch_bounds__(BLOCK) void k2_setupc(Geom g, Tables tb, Target tg, const double *__restrict__ x, TT *__restrict__ Q, double *__restrict__ bad)
{
    constexpr int EPB = S2<P, NQ>::EPB;
    const int e0 = blockIdx.x * EPB;
    b2_setupc<P, NQ, TT>(g, tb, tg, x, Q, bad, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT, typename CT, bool LIM>
__global__ __launch_bounds__(BLOCK) void k2_applyc(Geom g, Tables tb, Target tg, const TT *__restrict__ Q, const double *__restrict__ v, CT *__restrict__ yE)
{
    constexpr int EPB = S2<P, NQ>::EPB;
    const int e0 = blockIdx.x * EPB;
    b2_applyc<P, NQ, TT, CT, LIM>(g, tb, tg, Q, v, yE, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT, bool LIM>
__global__ __launch_bounds__(BLOCK) void k2_diag(Geom g, Tables tb, const TT *__restrict__ H, double *__restrict__ dE)
{
    constexpr int EPB = S2<P, NQ>::EPB;
    const int e0 = blockIdx.x * EPB;
    b2_diag<P, NQ, TT, LIM>(g, tb, H, dE, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT, bool LIM>
__global__ __launch_bounds__(BLOCK) void k2_diagc(Geom g, Tables tb, Target tg, const TT *__restrict__ Q, double *__restrict__ dE)
{
    constexpr int EPB = S2<P, NQ>::EPB;
    const int e0 = blockIdx.x * EPB;
    b2_diagc<P, NQ, TT, LIM>(g, tb, tg, Q, dE, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, bool LIM = false>
__global__ __launch_bounds__(BLOCK) void kb2_energy(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate, int vin, double *__restrict__ part)
{
    constexpr int EPB = S2<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b2_energy<P, NQ, LIM>(s.g, tb, s.tg, s.vec[vin], part, t.e0, min(EPB, s.g.ne - t.e0));
}

template <int P, int NQ, bool LIM = false, bool EN = false>
__global__ __launch_bounds__(BLOCK) void kb2_gradient(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate, int vin, double *__restrict__ bad)
{
    constexpr int EPB = S2<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b2_gradient<P, NQ, LIM, EN>(s.g, tb, s.tg, s.vec[vin], (double *)s.eV, bad, t.e0, min(EPB, s.g.ne - t.e0));
}

template <int P, int NQ, typename TT>
__global__ __launch_bounds__(BLOCK) void kb2_setup(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate, int vin, double *__restrict__ bad)
{
    constexpr int EPB = S2<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b2_setup<P, NQ, TT>(s.g, tb, s.tg, s.vec[vin], (TT *)s.H, bad, t.e0, min(EPB, s.g.ne - t.e0));
}

template <int P, int NQ, typename TT, typename CT, bool LIM = false>
__global__ __launch_bounds__(BLOCK) void kb2_apply(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate, int vin)
{
    constexpr int EPB = S2<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b2_apply<P, NQ, TT, CT, LIM>(s.g, tb, (const TT *)s.H, s.vec[vin], (CT *)s.eV, t.e0, min(EPB, s.g.ne - t.e0));
}

template <int P, int NQ, typename TT>
__global__ __launch_bounds__(BLOCK) void kb2_setupc(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate, int vin, double *__restrict__ bad)
{
    constexpr int EPB = S2<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b2_setupc<P, NQ, TT>(s.g, tb, s.tg, s.vec[vin], (TT *)s.H, bad, t.e0, min(EPB, s.g.ne - t.e0));
}

template <int P, int NQ, typename TT, typename CT, bool LIM = false>
__global__ __launch_bounds__(BLOCK) void kb2_applyc(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate, int vin)
{
    constexpr int EPB = S2<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b2_applyc<P, NQ, TT, CT, LIM>(s.g, tb, s.tg, (const TT *)s.H, s.vec[vin], (CT *)s.eV, t.e0, min(EPB, s.g.ne - t.e0));
}

template <int P, int NQ, typename TT, bool LIM = false>
__global__ __launch_bounds__(BLOCK) void kb2_diag(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate)
{
    constexpr int EPB = S2<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b2_diag<P, NQ, TT, LIM>(s.g, tb, (const TT *)s.H, (double *)s.eV, t.e0, min(EPB, s.g.ne - t.e0));
}

template <int P, int NQ, typename TT, bool LIM = false>
__global__ __launch_bounds__(BLOCK) void kb2_diagc(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate)
{
    constexpr int EPB = S2<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b2_diagc<P, NQ, TT, LIM>(s.g, tb, s.tg, (const TT *)s.H, (double *)s.eV, t.e0, min(EPB, s.g.ne - t.e0));
}

}  // namespace tmop
