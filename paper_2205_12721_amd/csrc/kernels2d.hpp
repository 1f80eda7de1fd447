// 2D (quad) PA-TMOP kernels, templated on the order P and the points per
// direction NQ.  Same structure as the hex kernels with two 1D contractions
// (Sec. 3.2):
//   A_a1(q) = sum_i1 G[q1][i1] sum_i2 B[q2][i2] x_a(i1,i2),
//   A_a2(q) = sum_i1 B[q1][i1] sum_i2 G[q2][i2] x_a(i1,i2).
// LDS per workgroup: sB, sG [NQ][NI]; sX [EPB][2][NI^2];
// R1 [EPB][2][2][NI][NQ] (axis-1 B and G variants); RY [EPB][4][NQ^2].
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

template <int P, int NQ, typename CT>
struct Lds2 {
    using S = S2<P, NQ>;
    CT B[NQ * S::NI];
    CT G[NQ * S::NI];
    CT X[S::EPB * 2 * S::NP];
    CT R1[S::EPB * 4 * S::L1];
    CT RY[S::EPB * 4 * S::NQ2];
};

template <int P>
__device__ inline int node2(const Geom &g, int e, int i1, int i2, int &gx, int &gy)
{
    constexpr int NI = P + 1;
    if (g.e2n) {
        gx = gy = -1;
        return g.e2n[(size_t)e * (NI * NI) + i1 + NI * i2];
    }
    const int ex = e % g.nel[0];
    const int ey = e / g.nel[0];
    gx = ex * P + i1;
    gy = ey * P + i2;
    return gx + g.M[0] * gy;
}

template <int P, int NQ, typename CT>
__device__ inline void prologue2(const Geom &g, const Tables &t, const double *__restrict__ vec,
                                 int e0, int nel, Lds2<P, NQ, CT> &L, bool masked)
{
    using S = S2<P, NQ>;
    constexpr int NI = S::NI, NP = S::NP;
    for (int k = threadIdx.x; k < NQ * NI; k += BLOCK) {
        L.B[k] = (CT)t.B[k];
        L.G[k] = (CT)t.G[k];
    }
    for (int idx = threadIdx.x; idx < nel * 2 * NP; idx += BLOCK) {
        const int i = idx % NP;
        const int r = idx / NP;
        const int c = r % 2, el = r / 2;
        int gx, gy;
        const int node = node2<P>(g, e0 + el, i % NI, i / NI, gx, gy);
        double v = vec[(size_t)c * g.nx + node];
        if (masked && is_fixed(g, c, node, gx, gy, 0)) v = 0.0;
        L.X[idx] = (CT)v;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nel * 2 * NI * NQ; idx += BLOCK) {
        const int q1 = idx % NQ;
        int r = idx / NQ;
        const int i2 = r % NI;
        r /= NI;  // el*2 + c
        const CT *x = L.X + r * NP + i2 * NI;
        CT b = 0, gg = 0;
#pragma unroll
        for (int i1 = 0; i1 < NI; ++i1) {
            b += L.B[q1 * NI + i1] * x[i1];
            gg += L.G[q1 * NI + i1] * x[i1];
        }
        CT *o = L.R1 + r * 2 * S::L1 + i2 * NQ + q1;
        o[0] = b;
        o[S::L1] = gg;
    }
    __syncthreads();
}

template <int P, int NQ, typename CT>
__device__ inline void point_grad2(const Lds2<P, NQ, CT> &L, int el, int q1, int q2, CT *J)
{
    using S = S2<P, NQ>;
    constexpr int NI = S::NI;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const CT *tb = L.R1 + (el * 2 + c) * 2 * S::L1 + q1;  // [i2] stride NQ
        const CT *tg = tb + S::L1;
        CT a0 = 0, a1 = 0;
#pragma unroll
        for (int i2 = 0; i2 < NI; ++i2) {
            a0 += L.B[q2 * NI + i2] * tg[i2 * NQ];
            a1 += L.G[q2 * NI + i2] * tb[i2 * NQ];
        }
        J[c * 2 + 0] = a0;
        J[c * 2 + 1] = a1;
    }
}

template <int P, int NQ, typename CT, typename OT>
__device__ inline void backward2(Lds2<P, NQ, CT> &L, int nel, OT *__restrict__ out)
{
    using S = S2<P, NQ>;
    constexpr int NI = S::NI, NQ2 = S::NQ2;
    for (int idx = threadIdx.x; idx < nel * 2 * NI * NQ; idx += BLOCK) {
        const int q1 = idx % NQ;
        int r = idx / NQ;
        const int i2 = r % NI;
        r /= NI;  // el*2 + c
        const CT *y = L.RY + r * 2 * NQ2 + q1;  // [b] stride NQ2, [q2] stride NQ
        CT u0 = 0, u1 = 0;
#pragma unroll
        for (int q2 = 0; q2 < NQ; ++q2) {
            u0 += L.B[q2 * NI + i2] * y[q2 * NQ];
            u1 += L.G[q2 * NI + i2] * y[NQ2 + q2 * NQ];
        }
        CT *o = L.R1 + r * 2 * S::L1 + i2 * NQ + q1;
        o[0] = u0;
        o[S::L1] = u1;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nel * 2 * S::NP; idx += BLOCK) {
        const int i1 = idx % NI;
        const int r = idx / NI;  // (el*2+c)*NI + i2
        const int rc = r / NI, i2 = r % NI;
        const CT *t = L.R1 + rc * 2 * S::L1 + i2 * NQ;
        CT s = 0;
#pragma unroll
        for (int q1 = 0; q1 < NQ; ++q1)
            s += L.G[q1 * NI + i1] * t[q1] + L.B[q1 * NI + i1] * t[S::L1 + q1];
        out[idx] = (OT)s;
    }
}

template <int P, int NQ>
__global__ __launch_bounds__(BLOCK) void k2_energy(Geom g, Tables tb, Target tg,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ part)
{
    using S = S2<P, NQ>;
    __shared__ Lds2<P, NQ, double> L;
    __shared__ double red[BLOCK / 64];
    const int e0 = blockIdx.x * S::EPB;
    const int nel = min(S::EPB, g.ne - e0);
    prologue2<P, NQ>(g, tb, x, e0, nel, L, false);
    double esum = 0.0, dmin = 1.0e300, bad = 0.0;
    for (int idx = threadIdx.x; idx < nel * S::NQ2; idx += BLOCK) {
        const int el = idx / S::NQ2, q = idx % S::NQ2;
        const int q1 = q % NQ, q2 = q / NQ;
        double J[4], Pm[4], mu;
        point_grad2<P, NQ>(L, el, q1, q2, J);
        dmin = fmin(dmin, det_only<2>(J));
        const double z = tb.w[q1] * tb.w[q2] * tg.detW;
        if (metric_first<2>(tg, J, z, &mu, Pm))
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

template <int P, int NQ>
__global__ __launch_bounds__(BLOCK) void k2_gradient(Geom g, Tables tb, Target tg,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ gE,
                                                     double *__restrict__ bad)
{
    using S = S2<P, NQ>;
    __shared__ Lds2<P, NQ, double> L;
    __shared__ double red[BLOCK / 64];
    const int e0 = blockIdx.x * S::EPB;
    const int nel = min(S::EPB, g.ne - e0);
    prologue2<P, NQ>(g, tb, x, e0, nel, L, false);
    double nbad = 0.0;
    for (int idx = threadIdx.x; idx < nel * S::NQ2; idx += BLOCK) {
        const int el = idx / S::NQ2, q = idx % S::NQ2;
        const int q1 = q % NQ, q2 = q / NQ;
        double J[4], Pm[4], mu;
        point_grad2<P, NQ>(L, el, q1, q2, J);
        const double z = tb.w[q1] * tb.w[q2] * tg.detW;
        if (!metric_first<2>(tg, J, z, &mu, Pm)) {
            nbad += 1.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) Pm[k] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) L.RY[(el * 4 + k) * S::NQ2 + q] = Pm[k];
    }
    __syncthreads();
    backward2<P, NQ>(L, nel, gE + (size_t)e0 * 2 * S::NP);
    const double b = block_sum(nbad, red);
    if (threadIdx.x == 0) bad[blockIdx.x] = b;
}

template <int P, int NQ, typename TT>
__global__ __launch_bounds__(BLOCK) void k2_setup(Geom g, Tables tb, Target tg,
                                                  const double *__restrict__ x,
                                                  TT *__restrict__ H, double *__restrict__ bad)
{
    using S = S2<P, NQ>;
    __shared__ Lds2<P, NQ, double> L;
    __shared__ double red[BLOCK / 64];
    const int e0 = blockIdx.x * S::EPB;
    const int nel = min(S::EPB, g.ne - e0);
    prologue2<P, NQ>(g, tb, x, e0, nel, L, false);
    double nbad = 0.0;
    for (int idx = threadIdx.x; idx < nel * S::NQ2; idx += BLOCK) {
        const int el = idx / S::NQ2, q = idx % S::NQ2;
        const int q1 = q % NQ, q2 = q / NQ;
        double J[4], Hp[10];
        point_grad2<P, NQ>(L, el, q1, q2, J);
        const double z = tb.w[q1] * tb.w[q2] * tg.detW;
        if (!metric_second<2>(tg, J, z, Hp)) {
            nbad += 1.0;
#pragma unroll
            for (int k = 0; k < 10; ++k) Hp[k] = 0.0;
        }
        TT *h = H + (size_t)(e0 + el) * 10 * S::NQ2 + q;
#pragma unroll
        for (int k = 0; k < 10; ++k) h[k * S::NQ2] = (TT)Hp[k];
    }
    const double b = block_sum(nbad, red);
    if (threadIdx.x == 0) bad[blockIdx.x] = b;
}

template <int P, int NQ, typename TT, typename CT>
__global__ __launch_bounds__(BLOCK) void k2_apply(Geom g, Tables tb, const TT *__restrict__ H,
                                                  const double *__restrict__ v,
                                                  CT *__restrict__ yE)
{
    using S = S2<P, NQ>;
    __shared__ Lds2<P, NQ, CT> L;
    const int e0 = blockIdx.x * S::EPB;
    const int nel = min(S::EPB, g.ne - e0);
    prologue2<P, NQ>(g, tb, v, e0, nel, L, true);
    for (int idx = threadIdx.x; idx < nel * S::NQ2; idx += BLOCK) {
        const int el = idx / S::NQ2, q = idx % S::NQ2;
        const int q1 = q % NQ, q2 = q / NQ;
        const TT *h = H + (size_t)(e0 + el) * 10 * S::NQ2 + q;
        CT hv[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) hv[k] = (CT)h[k * S::NQ2];
        CT J[4];
        point_grad2<P, NQ>(L, el, q1, q2, J);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            CT s = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) s += hv[sym_index<4>(r, c)] * J[c];
            L.RY[(el * 4 + r) * S::NQ2 + q] = s;
        }
    }
    __syncthreads();
    backward2<P, NQ>(L, nel, yE + (size_t)e0 * 2 * S::NP);
}

template <int P, int NQ, typename TT>
__global__ __launch_bounds__(BLOCK) void k2_diag(Geom g, Tables tb, const TT *__restrict__ H,
                                                 double *__restrict__ dE)
{
    using S = S2<P, NQ>;
    constexpr int NI = S::NI, NQ2 = S::NQ2, NP = S::NP;
    __shared__ double T[3][NQ * NI];
    __shared__ double sQ[S::EPB * 2 * NQ2];
    __shared__ double U1[S::EPB * 2 * NI * NQ];
    __shared__ double sD[S::EPB * 2 * NP];
    const int e0 = blockIdx.x * S::EPB;
    const int nel = min(S::EPB, g.ne - e0);
    for (int k = threadIdx.x; k < NQ * NI; k += BLOCK) {
        const double b = tb.B[k], gg = tb.G[k];
        T[0][k] = b * b;
        T[1][k] = b * gg;
        T[2][k] = gg * gg;
    }
    for (int k = threadIdx.x; k < nel * 2 * NP; k += BLOCK) sD[k] = 0.0;
    const int pn[3] = {0, 0, 1};
    const int pp[3] = {0, 1, 1};
    for (int pr = 0; pr < 3; ++pr) {
        const int n = pn[pr], p = pp[pr];
        const double f = (n == p) ? 1.0 : 2.0;
        const int t1 = (n == 0) + (p == 0), t2 = (n == 1) + (p == 1);
        __syncthreads();
        for (int idx = threadIdx.x; idx < nel * 2 * NQ2; idx += BLOCK) {
            const int q = idx % NQ2;
            const int r = idx / NQ2;
            const int a = r % 2, el = r / 2;
            const int s = sym_index<4>(a * 2 + n, a * 2 + p);
            sQ[idx] = f * (double)H[((size_t)(e0 + el) * 10 + s) * NQ2 + q];
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < nel * 2 * NI * NQ; idx += BLOCK) {
            const int q1 = idx % NQ;
            int r = idx / NQ;
            const int i2 = r % NI;
            r /= NI;
            const double *y = sQ + r * NQ2 + q1;
            double s = 0.0;
#pragma unroll
            for (int q2 = 0; q2 < NQ; ++q2) s += T[t2][q2 * NI + i2] * y[q2 * NQ];
            U1[(r * NI + i2) * NQ + q1] = s;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < nel * 2 * NP; idx += BLOCK) {
            const int i1 = idx % NI;
            const int rest = idx / NI;
            const double *y = U1 + rest * NQ;
            double s = 0.0;
#pragma unroll
            for (int q1 = 0; q1 < NQ; ++q1) s += T[t1][q1 * NI + i1] * y[q1];
            sD[idx] += s;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nel * 2 * NP; k += BLOCK) dE[(size_t)e0 * 2 * NP + k] = sD[k];
}

}  // namespace tmop
