// 3D (hex) PA-TMOP kernels, templated on the order P and the points per
// direction NQ.  Sum factorization follows Sec. 3.2: the Jacobian entries at
// all quadrature points of an element come from three 1D contractions with
// B = l_i(chi_q) and G = l_i'(chi_q), one per axis, e.g.
//   A_a1(q) = sum_i1 G[q1][i1] sum_i2 B[q2][i2] sum_i3 B[q3][i3] x_a(i1,i2,i3)
// and the transposed contractions map quadrature values back to nodes.
//
// Each contraction stage is a loop over "pencils": one work item loads one 1D
// line of its input from LDS once and produces the whole 1D line of outputs.
// The 1D tables are indexed with compile-time constants in the kernel
// arguments, so they are read into scalar registers instead of from LDS.
//
// LDS per workgroup (CT = compute type, double or float):
//   X   [EPB][3][NI^3]            element nodes (or v_E)
//   R1  [EPB][3][2][NI][NI][NQ]   after the axis-1 contraction (B, G variants)
//   R2  [EPB][3][3][NI][NQ][NQ]   after the axis-2 contraction (GB, BG, BB)
//   RY  [EPB][NR][NQ^3]           per-point 3x3 values: J = dx/dxbar after
//                                 the forward sweeps, then Y (H : grad v, or P);
//                                 with the limiting term (NR = 12) also the
//                                 vector's values at the points, then the
//                                 limiting term's point values
// with X/R2 and R1/RY overlaid.
// Forward:  X -> R1 -> R2 -> RY(J);  point stage RY(J) -> RY(Y) in place;
// backward: RY(Y) -> R2 -> R1 -> E-vector.
#pragma once
#include "mfma3.hpp"
#include "tmop_dev.hpp"

namespace tmop {

// T2 = tile shape of the workgroup, in halves of the base number of
// elements per workgroup EPB0 = max(1, 256 / NQ^3): 1 half, 2 base (one point
// per lane), 4 double (two points per lane).  Only the Hessian action is
// instantiated with other than the base shape (its autotuned tile).
template <int P, int NQ, int T2 = 2>
struct S3 {
    static constexpr int NI = P + 1;
    static constexpr int NP = NI * NI * NI;
    static constexpr int NQ2 = NQ * NQ;
    static constexpr int NQ3 = NQ * NQ * NQ;
    static constexpr int EPB0 = NQ3 >= BLOCK ? 1 : BLOCK / NQ3;
    static constexpr int EPB = EPB0 * T2 / 2 >= 1 ? EPB0 * T2 / 2 : 1;
    static constexpr int L1 = NI * NI * NQ;  // one R1 plane
    static constexpr int L2 = NI * NQ * NQ;  // one R2 plane
    static constexpr int NS = 45;            // packed tensor entries
};

// X and R2 share storage, and so do R1 and RY: each stage reads one of the
// two buffers and writes the other, so a buffer is overwritten only after the
// barrier that ends the last read of its previous contents.
// NR = planes of RY per element: 9 (J or Y), or 12 when the three value
// planes of the limiting term (the vector itself at the points) follow.
template <int P, int NQ, typename CT, int NR = 9, int T2 = 2>
struct Lds3 {
    using S = S3<P, NQ, T2>;
    union {
        CT X[S::EPB * 3 * S::NP];
        CT R2[S::EPB * 9 * S::L2];
    };
    union {
        CT R1[S::EPB * 6 * S::L1];
        CT RY[S::EPB * NR * S::NQ3];
    };
};

// RY planes per element for a body with (LIM) or without the limiting term.
template <bool LIM>
struct Planes3 {
    static constexpr int NR = LIM ? 12 : 9;
};

// Global node of local node (i1,i2,i3) of element e, and its grid coordinates.
template <int P>
__device__ __forceinline__ int node3(const Geom &g, int e, int i1, int i2, int i3, int &gx, int &gy,
                            int &gz)
{
    constexpr int NI = P + 1;
    if (g.e2n) {
        gx = gy = gz = -1;
        return g.e2n[(size_t)e * (NI * NI * NI) + i1 + NI * (i2 + NI * i3)];
    }
    int ex, ey, ez;
    box_elem<3>(g, e, ex, ey, ez);
    gx = ex * P + i1;
    gy = ey * P + i2;
    gz = ez * P + i3;
    return gx + g.M[0] * (gy + g.M[1] * gz);
}

// Gather 3 components of a global vector into X for the block's elements.
// masked: fixed DoFs read as zero (the P of H_c = P H P + (I - P)); sub:
// a vector subtracted entry by entry (x - x0 of the limiting term).  Split in
// a load phase (registers) and a store phase (LDS) so that a caller can issue
// other loads in between; the loop has a compile-time trip count so that all
// of a lane's loads are issued before the first one is waited for.
template <int P, int NQ, int T2 = 2>
struct Gath3 {
    static constexpr int NIT = (S3<P, NQ, T2>::EPB * 3 * S3<P, NQ>::NP + BLOCK - 1) / BLOCK;
    double val[NIT];
    bool fix[NIT];
};

template <int P, int NQ, int T2, bool SUB>
__device__ __forceinline__ void gather3_box(const Geom &g, const double *__restrict__ vec,
                                            const double *__restrict__ sub, int e0, int n,
                                            bool bmask, Gath3<P, NQ, T2> &r)
{
    using S = S3<P, NQ>;
    constexpr int NI = S::NI, NP = S::NP, NIT = Gath3<P, NQ, T2>::NIT;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int idx = threadIdx.x + it * BLOCK;
        const bool in = idx < n;
        const int i = idx % NP;
        const int rr = idx / NP;  // el*3 + c
        const int c = rr % 3, el = rr / 3;
        const int i1 = i % NI, i2 = (i / NI) % NI, i3 = i / (NI * NI);
        int ex, ey, ez;
        box_elem<3>(g, e0 + el, ex, ey, ez);
        const int gx = ex * P + i1, gy = ey * P + i2, gz = ez * P + i3;
        // lanes past the end read node 0 and are dropped
        const size_t at = in ? (size_t)c * g.nx + gx + g.M[0] * (gy + g.M[1] * gz) : 0;
        double v = vec[at];
        if (SUB) v -= sub[at];
        r.val[it] = v;
        r.fix[it] = !in || (bmask && box_boundary(g, gx, gy, gz));
    }
}

template <int P, int NQ, int T2 = 2>
__device__ __forceinline__ void gather3_load(const Geom &g, const double *__restrict__ vec, int e0,
                                             int nel, bool masked, Gath3<P, NQ, T2> &r,
                                             const double *__restrict__ sub = nullptr)
{
    using S = S3<P, NQ>;
    constexpr int NI = S::NI, NP = S::NP, NIT = Gath3<P, NQ, T2>::NIT;
    const int n = nel * 3 * NP;
    if (!g.e2n && !(masked && g.ess_mode == 2)) {
        // box mesh without a mask array: branch-free, so that every load of
        // the lane is issued before any is waited for
        const bool bmask = masked && g.ess_mode == 0;
        if (sub)
            gather3_box<P, NQ, T2, true>(g, vec, sub, e0, n, bmask, r);
        else
            gather3_box<P, NQ, T2, false>(g, vec, sub, e0, n, bmask, r);
        return;
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int idx = threadIdx.x + it * BLOCK;
        r.val[it] = 0.0;
        r.fix[it] = false;
        if (idx < n) {
            const int i = idx % NP;
            const int rr = idx / NP;  // el*3 + c
            const int c = rr % 3, el = rr / 3;
            const int i1 = i % NI, i2 = (i / NI) % NI, i3 = i / (NI * NI);
            int gx, gy, gz;
            const int node = node3<P>(g, e0 + el, i1, i2, i3, gx, gy, gz);
            r.val[it] = vec[(size_t)c * g.nx + node];
            if (sub) r.val[it] -= sub[(size_t)c * g.nx + node];
            r.fix[it] = masked && is_fixed(g, c, node, gx, gy, gz);
        }
    }
}

template <int P, int NQ, typename CT, int T2 = 2>
__device__ __forceinline__ void gather3_store(const Gath3<P, NQ, T2> &r, int nel, CT *sX)
{
    constexpr int NIT = Gath3<P, NQ, T2>::NIT;
    const int n = nel * 3 * S3<P, NQ>::NP;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int idx = threadIdx.x + it * BLOCK;
        if (idx < n) sX[idx] = r.fix[it] ? (CT)0 : (CT)r.val[it];
    }
}

template <int P, int NQ, typename CT>
__device__ __forceinline__ void gather3(const Geom &g, const double *__restrict__ vec, int e0,
                                        int nel, CT *sX, bool masked,
                                        const double *__restrict__ sub = nullptr)
{
    Gath3<P, NQ> r;
    gather3_load<P, NQ>(g, vec, e0, nel, masked, r, sub);
    gather3_store<P, NQ, CT>(r, nel, sX);
}

// Forward sweeps X -> R1 -> R2 -> RY (J at every point, plane el*NR + c*3 + b;
// with VAL also the value of component c, plane el*NR + 9 + c).
// Forward sweeps of axes 1 and 2: X -> R1 -> R2, ending with a barrier.
template <int P, int NQ, typename CT>
__device__ __forceinline__ void forward3_head(const Tables &tb, const CT *X, CT *R1, CT *R2, int nel)
{
    using S = S3<P, NQ>;
    constexpr int NI = S::NI, NP = S::NP, L1 = S::L1, L2 = S::L2, NQ2 = S::NQ2;
    // axis 1: pencils (r, i3, i2), r = el*3 + c
    for (int pen = threadIdx.x; pen < nel * 3 * NI * NI; pen += BLOCK) {
        const int i23 = pen % (NI * NI), r = pen / (NI * NI);
        const CT *x = X + r * NP + i23 * NI;
        CT xv[NI];
#pragma unroll
        for (int k = 0; k < NI; ++k) xv[k] = x[k];
        CT *o = R1 + r * 2 * L1 + i23 * NQ;
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
    // axis 2: pencils (r, i3, q1)
    for (int pen = threadIdx.x; pen < nel * 3 * NI * NQ; pen += BLOCK) {
        const int q1 = pen % NQ, i3 = (pen / NQ) % NI, r = pen / (NQ * NI);
        const CT *t = R1 + r * 2 * L1 + i3 * NI * NQ + q1;  // [i2] stride NQ
        CT xb[NI], xg[NI];
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            xb[k] = t[k * NQ];
            xg[k] = t[L1 + k * NQ];
        }
        CT *o = R2 + r * 3 * L2 + i3 * NQ2 + q1;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            CT gb = 0, bg = 0, bb = 0;
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                const CT b2 = tabB<CT>(tb, q * NI + k), g2 = tabG<CT>(tb, q * NI + k);
                gb += b2 * xg[k];
                bg += g2 * xb[k];
                bb += b2 * xb[k];
            }
            o[q * NQ] = gb;
            o[L2 + q * NQ] = bg;
            o[2 * L2 + q * NQ] = bb;
        }
    }
    __syncthreads();
}

template <int P, int NQ, typename CT, int NR = 9, bool VAL = false>
__device__ __forceinline__ void forward3(const Tables &tb, const CT *X, CT *R1, CT *R2, CT *RY, int nel)
{
    using S = S3<P, NQ>;
    constexpr int NI = S::NI, L2 = S::L2, NQ2 = S::NQ2, NQ3 = S::NQ3;
    forward3_head<P, NQ, CT>(tb, X, R1, R2, nel);
    // axis 3: pencils (r, q2, q1) -> J at the NQ points of the pencil
    for (int pen = threadIdx.x; pen < nel * 3 * NQ2; pen += BLOCK) {
        const int q12 = pen % NQ2, r = pen / NQ2;
        const CT *t = R2 + r * 3 * L2 + q12;  // [i3] stride NQ^2
        CT t0[NI], t1[NI], t2[NI];
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            t0[k] = t[k * NQ2];
            t1[k] = t[L2 + k * NQ2];
            t2[k] = t[2 * L2 + k * NQ2];
        }
        const int el = r / 3, c = r % 3;
        CT *o = RY + (el * NR + c * 3) * NQ3 + q12;
        CT *ov = RY + (el * NR + 9 + c) * NQ3 + q12;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            CT a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                const CT b3 = tabB<CT>(tb, q * NI + k), g3 = tabG<CT>(tb, q * NI + k);
                a0 += b3 * t0[k];
                a1 += b3 * t1[k];
                a2 += g3 * t2[k];
                if (VAL) a3 += b3 * t2[k];
            }
            o[q * NQ2] = a0;
            o[NQ3 + q * NQ2] = a1;
            o[2 * NQ3 + q * NQ2] = a2;
            if (VAL) ov[q * NQ2] = a3;
        }
    }
    __syncthreads();
}

// E-vector index of (element e, component c, local node i1,i2,i3).  General
// meshes: element-major [e][c][i].  Structured box: the exploded grid
// [c][ez*NI+i3][ey*NI+i2][ex*NI+i1], in which the node gather reads runs of
// neighbouring addresses.
template <int P>
__device__ __forceinline__ long ev_index3(const Geom &g, int e, int c, int i1, int i2, int i3)
{
    constexpr int NI = P + 1, NP = NI * NI * NI;
    if (g.e2n) return ((long)e * 3 + c) * NP + i1 + NI * (i2 + NI * i3);
    int ex, ey, ez;
    box_elem<3>(g, e, ex, ey, ez);
    const long EX = (long)g.nel[0] * NI, EY = (long)g.nel[1] * NI;
    return (long)c * g.ne * NP + ((long)(ez * NI + i3) * EY + (ey * NI + i2)) * EX + ex * NI + i1;
}

// Backward sweeps of axes 2 and 1: R2 (the axis-3 contractions) -> R1 ->
// E-vector.  Called after a barrier that ends the writes of R2.
template <int P, int NQ, typename CT, typename OT, bool CW = false>
__device__ __forceinline__ void backward3_tail(const Tables &tb, const Geom &g, int e0, CT *R2,
                                               CT *R1, int nel, OT *__restrict__ out)
{
    using S = S3<P, NQ>;
    constexpr int NI = S::NI, L1 = S::L1, L2 = S::L2, NQ2 = S::NQ2;
    // axis 2: pencils (r, i3, q1)
    for (int pen = threadIdx.x; pen < nel * 3 * NI * NQ; pen += BLOCK) {
        const int q1 = pen % NQ, i3 = (pen / NQ) % NI, r = pen / (NQ * NI);
        const CT *t = R2 + r * 3 * L2 + i3 * NQ2 + q1;  // [q2] stride NQ
        CT t0[NQ], t1[NQ], t2[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            t0[q] = t[q * NQ];
            t1[q] = t[L2 + q * NQ];
            t2[q] = t[2 * L2 + q * NQ];
        }
        CT *o = R1 + r * 2 * L1 + i3 * NI * NQ + q1;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            CT u0 = 0, u1 = 0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const CT b2 = tabB<CT>(tb, q * NI + k), g2 = tabG<CT>(tb, q * NI + k);
                u0 += b2 * t0[q];
                u1 += g2 * t1[q] + b2 * t2[q];
            }
            o[k * NQ] = u0;       // G along axis 1 still to apply
            o[L1 + k * NQ] = u1;  // B along axis 1 still to apply
        }
    }
    __syncthreads();
    // axis 1: pencils (r, i3, i2) -> NI consecutive outputs
    if (!CW) {
        for (int pen = threadIdx.x; pen < nel * 3 * NI * NI; pen += BLOCK) {
            const int i2 = pen % NI, i3 = (pen / NI) % NI, r = pen / (NI * NI);
            const int c = r % 3, el = r / 3;
            const CT *t = R1 + r * 2 * L1 + (i3 * NI + i2) * NQ;
            CT u0[NQ], u1[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                u0[q] = t[q];
                u1[q] = t[L1 + q];
            }
            OT *o = out + ev_index3<P>(g, e0 + el, c, 0, i2, i3);
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                CT s = 0;
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    s += tabG<CT>(tb, q * NI + k) * u0[q] + tabB<CT>(tb, q * NI + k) * u1[q];
                o[k] = (OT)s;
            }
        }
        return;
    }
    // CW (coalesced writes): the outputs are staged in R2 (free again) as
    // [el][c][i3][i2][i1]
    static_assert(9 * L2 >= 3 * S::NP, "staging of the element outputs must fit in R2");
    CT *Y = R2;
    for (int pen = threadIdx.x; pen < nel * 3 * NI * NI; pen += BLOCK) {
        const int r = pen / (NI * NI), i32 = pen % (NI * NI);
        const CT *t = R1 + r * 2 * L1 + i32 * NQ;
        CT u0[NQ], u1[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            u0[q] = t[q];
            u1[q] = t[L1 + q];
        }
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            CT s = 0;
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                s += tabG<CT>(tb, q * NI + k) * u0[q] + tabB<CT>(tb, q * NI + k) * u1[q];
            Y[pen * NI + k] = s;
        }
    }
    __syncthreads();
    // E-vector writes with the lanes in (c, i3, i2, el, i1) order: on the box
    // the tile's elements are neighbours along x, so consecutive lanes write
    // consecutive addresses of the exploded grid (runs of nel*NI values)
    for (int idx = threadIdx.x; idx < nel * 3 * NI * NI * NI; idx += BLOCK) {
        const int k = idx % NI, el = (idx / NI) % nel, rest = idx / (NI * nel);
        const int i2 = rest % NI, i3 = (rest / NI) % NI, c = rest / (NI * NI);
        out[ev_index3<P>(g, e0 + el, c, k, i2, i3)] = (OT)Y[(((el * 3 + c) * NI + i3) * NI + i2) * NI + k];
    }
}


// Backward (transposed) sweeps RY -> R2 -> R1 -> E-vector:
//   y_c(i) = sum_q sum_b RY[c][b](q) d w_i/d xbar_b (q)  (+ RY[9+c](q) w_i(q) with VAL).
template <int P, int NQ, typename CT, typename OT, int NR = 9, bool VAL = false, bool CW = false>
__device__ __forceinline__ void backward3(const Tables &tb, const Geom &g, int e0, const CT *RY, CT *R2,
                                 CT *R1, int nel, OT *__restrict__ out)
{
    using S = S3<P, NQ>;
    constexpr int NI = S::NI, L1 = S::L1, L2 = S::L2, NQ2 = S::NQ2, NQ3 = S::NQ3;
    // axis 3: pencils (r, q2, q1)
    for (int pen = threadIdx.x; pen < nel * 3 * NQ2; pen += BLOCK) {
        const int q12 = pen % NQ2, r = pen / NQ2;
        const int el = r / 3, c = r % 3;
        const CT *y = RY + (el * NR + c * 3) * NQ3 + q12;  // [b] stride NQ^3, [q3] stride NQ^2
        const CT *yv = RY + (el * NR + 9 + c) * NQ3 + q12;
        CT y0[NQ], y1[NQ], y2[NQ], ym[VAL ? NQ : 1];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            y0[q] = y[q * NQ2];
            y1[q] = y[NQ3 + q * NQ2];
            y2[q] = y[2 * NQ3 + q * NQ2];
            if (VAL) ym[q] = yv[q * NQ2];
        }
        CT *o = R2 + r * 3 * L2 + q12;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            CT t0 = 0, t1 = 0, t2 = 0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const CT b3 = tabB<CT>(tb, q * NI + k), g3 = tabG<CT>(tb, q * NI + k);
                t0 += b3 * y0[q];
                t1 += b3 * y1[q];
                t2 += g3 * y2[q];
                // the value term follows the B B path of plane 2 on axes 1, 2
                if (VAL) t2 += b3 * ym[q];
            }
            o[k * NQ2] = t0;
            o[L2 + k * NQ2] = t1;
            o[2 * L2 + k * NQ2] = t2;
        }
    }
    __syncthreads();
    backward3_tail<P, NQ, CT, OT, CW>(tb, g, e0, R2, R1, nel, out);
}

// J[c*3+b] = d x_c / d xbar_b at point q of element el, left in RY by forward3.
template <int P, int NQ, typename CT, int NR = 9>
__device__ __forceinline__ void point_J3(const CT *RY, int el, int q, CT *J)
{
    constexpr int NQ3 = S3<P, NQ>::NQ3;
#pragma unroll
    for (int k = 0; k < 9; ++k) J[k] = RY[(el * NR + k) * NQ3 + q];
}

// Product of the 1D quadrature weights at point q.
template <int NQ>
__device__ __forceinline__ double qweight3(const Tables &tb, int q)
{
    const int q1 = q % NQ, q2 = (q / NQ) % NQ, q3 = q / (NQ * NQ);
    return tab_w<NQ>(tb, q1) * tab_w<NQ>(tb, q2) * tab_w<NQ>(tb, q3);
}

// z = w_q det W: the weight of point q in the integral over the target element.
template <int NQ>
__device__ __forceinline__ double point_weight3(const Tables &tb, const Target &tg, int q)
{
    return qweight3<NQ>(tb, q) * tg.detW;
}

// ------------------------------------------------------------------------
// Quadrature data layout per element (hex kernels): NS values per point in
// runs of VEC = 16 / sizeof(TT) consecutive values per point, [run][q][VEC],
// then the NS % VEC remaining values as plain planes [s][q]; runs and planes
// hold NQP = qdata_pts(NQT) points (the last NQP - NQT unused), so each
// starts on a 128-byte line; element blocks of qdata_stride(NS, NQT,
// sizeof(TT)) values.  A lane reads or writes VEC values of its point with
// one 16-byte access, and the lanes of a wave cover consecutive 16-byte words.
// ------------------------------------------------------------------------
template <typename TT>
struct alignas(16) Vec16 {
    TT v[16 / sizeof(TT)];
};

template <typename TT, int NS, int NQT>
struct QLay {
    static constexpr int VEC = 16 / sizeof(TT);
    static constexpr int NV = NS / VEC;    // full runs
    static constexpr int TAIL = NV * VEC;  // first value stored in a plain plane
    static constexpr long NQP = qdata_pts(NQT, sizeof(TT));  // points per run / plane
    static constexpr long STRIDE = qdata_stride(NS, NQT, sizeof(TT));
    static_assert(NQP * 16 % 128 == 0 && NQP * sizeof(TT) % 128 == 0, "line-aligned runs");
};

// NT: non-temporal loads, for a stream read once per call that should not
// displace reused data from the caches (the stored tensor of the Hessian action).
template <typename TT, int NS, int NQT, bool NT = false>
__device__ __forceinline__ void qdata_load(const TT *__restrict__ he, int q, TT *out)
{
    using L = QLay<TT, NS, NQT>;
    typedef TT V __attribute__((ext_vector_type(L::VEC)));
#pragma unroll
    for (int r = 0; r < L::NV; ++r) {
        const V *a = (const V *)(he + (r * L::NQP + q) * L::VEC);
        const V w = NT ? __builtin_nontemporal_load(a) : *a;
#pragma unroll
        for (int k = 0; k < L::VEC; ++k) out[r * L::VEC + k] = w[k];
    }
#pragma unroll
    for (int s = L::TAIL; s < NS; ++s) {
        const TT *a = he + L::TAIL * L::NQP + (s - L::TAIL) * L::NQP + q;
        out[s] = NT ? __builtin_nontemporal_load(a) : *a;
    }
}

// Where a run's (a plane's) data ends inside a 128-byte line, the lanes of
// its last PR (PP) points also write zeros into the padding points that fill
// that line, so that the wave writing the line's data writes all of it.
template <typename TT, int NS, int NQT>
__device__ __forceinline__ void qdata_store(TT *__restrict__ he, int q, const TT *in)
{
    using L = QLay<TT, NS, NQT>;
    constexpr int TB = (int)sizeof(TT);
    constexpr int PR = (NQT * 16) % 128 ? (128 - (NQT * 16) % 128) / 16 : 0;
    constexpr int PP = (NQT * TB) % 128 ? (128 - (NQT * TB) % 128) / TB : 0;
    static_assert(PR <= L::NQP - NQT && PP <= L::NQP - NQT, "padding within the block");
#pragma unroll
    for (int r = 0; r < L::NV; ++r) {
        Vec16<TT> w;
#pragma unroll
        for (int k = 0; k < L::VEC; ++k) w.v[k] = in[r * L::VEC + k];
        *(Vec16<TT> *)(he + (r * L::NQP + q) * L::VEC) = w;
        if (PR && q >= NQT - PR) {
            Vec16<TT> z;
#pragma unroll
            for (int k = 0; k < L::VEC; ++k) z.v[k] = (TT)0;
            *(Vec16<TT> *)(he + (r * L::NQP + q + PR) * L::VEC) = z;
        }
    }
#pragma unroll
    for (int s = L::TAIL; s < NS; ++s) {
        he[L::TAIL * L::NQP + (s - L::TAIL) * L::NQP + q] = in[s];
        if (PP && q >= NQT - PP) he[L::TAIL * L::NQP + (s - L::TAIL) * L::NQP + q + PP] = (TT)0;
    }
}

// one value s (diagonal kernels read a subset)
template <typename TT, int NS, int NQT>
__device__ __forceinline__ TT qdata_at(const TT *__restrict__ he, int q, int s)
{
    using L = QLay<TT, NS, NQT>;
    return s < L::TAIL ? he[((s / L::VEC) * L::NQP + q) * L::VEC + s % L::VEC]
                       : he[L::TAIL * L::NQP + (s - L::TAIL) * L::NQP + q];
}

// ------------------------------------------------------------------------
// Element bodies
// ------------------------------------------------------------------------

// Limiting term in the Hessian action (eq. eq_pa_limiting): the value planes
// v_c(q) become 2 w_q lim v_c(q), a mass-like operator with no stored data
// (lim = coef det W / delta^2 folds the target volume factor in).
template <int NQ, typename CT, int NR>
__device__ __forceinline__ void lim_point3(const Tables &tb, const Geom &g, int el, int q, CT *RY)
{
    constexpr int NQ3 = NQ * NQ * NQ;
    const CT f = (CT)(2.0 * g.lim * qweight3<NQ>(tb, q));
#pragma unroll
    for (int c = 0; c < 3; ++c) RY[(el * NR + 9 + c) * NQ3 + q] *= f;
}

// Values of x - x0 (limiting term) at the points of the block's elements,
// into U[el][c][q]: forward sweeps with value planes on the difference.
template <int P, int NQ, typename L3>
__device__ __forceinline__ void lim_values3(const Geom &g, const Tables &tb, const double *__restrict__ x,
                                   int e0, int nel, L3 &L, double *U)
{
    using S = S3<P, NQ>;
    gather3<P, NQ>(g, x, e0, nel, L.X, false, g.x0);
    __syncthreads();
    forward3<P, NQ, double, 12, true>(tb, L.X, L.R1, L.R2, L.RY, nel);
    for (int idx = threadIdx.x; idx < nel * 3 * S::NQ3; idx += BLOCK) {
        const int q = idx % S::NQ3, r = idx / S::NQ3;  // r = el*3 + c
        U[idx] = L.RY[((r / 3) * 12 + 9 + r % 3) * S::NQ3 + q];
    }
    __syncthreads();
}

// Energy and minimum det A: per-block partial sums of z mu and minima of det A,
// count of points with det T <= 0 (Sec. 3.3, eq. D0_expression; Sec. 2.3).
// LIM adds w_q lim |x - x0|^2 (the limiting integral of eq. eq_F_full with
// xi = |y|^2 / delta^2 over the target element, lim = coef det W / delta^2).
// MF: forward sweeps on the matrix cores (forward3_mfma) instead of the
// pencil sweeps (classes with n_q <= 5, without the limiting term).
template <int P, int NQ, bool LIM = false, bool MF = false>
__device__ __forceinline__ void b3_energy(const Geom &g, const Tables &tb, const Target &tg,
                                 const double *__restrict__ x, double *__restrict__ part, int e0,
                                 int nel)
{
    using S = S3<P, NQ>;
    constexpr int NR = Planes3<LIM>::NR;
    static_assert(!(MF && LIM), "no matrix-core sweeps with the limiting term");
    __shared__ Lds3<P, NQ, double, NR> L;
    __shared__ double U[LIM ? S::EPB * 3 * S::NQ3 : 1];
    // the matrix-core tables during the sweeps, the reduction at the end
    constexpr int NRED = 3 * (BLOCK / 64), NMF = MF ? 2 * NQ * S::NI : 0;
    __shared__ double red[NRED > NMF ? NRED : NMF];
    double *mft = red;
    if (LIM) lim_values3<P, NQ>(g, tb, x, e0, nel, L, U);
    if (MF) mfma_tables<S::NI, NQ>(tb, mft);
    gather3<P, NQ>(g, x, e0, nel, L.X, false);
    __syncthreads();
    if constexpr (MF)
        forward3_mfma<P, NQ, NR>(mft, L.X, L.R1, L.R2, L.RY, nel);
    else
        forward3<P, NQ, double, NR>(tb, L.X, L.R1, L.R2, L.RY, nel);
    double esum = 0.0, dmin = 1.0e300, bad = 0.0;
    for (int idx = threadIdx.x; idx < nel * S::NQ3; idx += BLOCK) {
        const int el = idx / S::NQ3, q = idx % S::NQ3;
        double J[9];
        point_J3<P, NQ, double, NR>(L.RY, el, q, J);
        dmin = fmin(dmin, det_only<3>(J));
        const double z = point_weight3<NQ>(tb, tg, q);
        double mu, Pm[9];
        if (metric_first<3>(tg, J, z, &mu, Pm))
            esum += z * mu;
        else
            bad += 1.0;
        if (LIM) {
            double y2 = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double u = U[(el * 3 + c) * S::NQ3 + q];
                y2 += u * u;
            }
            esum += qweight3<NQ>(tb, q) * g.lim * y2;
        }
    }
    block_energy3(esum, dmin, bad, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = esum;
        part[gridDim.x + blockIdx.x] = dmin;
        part[2 * gridDim.x + blockIdx.x] = bad;
    }
}

// Gradient E-vector (Sec. 3.3, eq. eq_vm_pa_grad): per point z P, then the
// transposed contractions.  bad[blockIdx] counts points with det T <= 0.
// LIM adds 2 w_q lim (x - x0)_c(q) wbar_i(q) through the value planes.
// EN: also the energy partials of b3_energy (the point stage evaluates mu
// anyway): the sums, the min det and the count of points with det T <= 0 go
// to the planes bad[blockIdx], bad[grid + blockIdx], bad[2 grid + blockIdx]
// (the same terms in the same order as b3_energy: bitwise its partials, and
// the gradient bitwise that of EN = false).
template <int P, int NQ, bool LIM = false, bool EN = false, bool MF = false>
__device__ __forceinline__ void b3_gradient(const Geom &g, const Tables &tb, const Target &tg,
                                   const double *__restrict__ x, double *__restrict__ gE,
                                   double *__restrict__ bad, int e0, int nel)
{
    using S = S3<P, NQ>;
    constexpr int NR = Planes3<LIM>::NR;
    static_assert(!(MF && LIM), "no matrix-core sweeps with the limiting term");
    __shared__ Lds3<P, NQ, double, NR> L;
    __shared__ double U[LIM ? S::EPB * 3 * S::NQ3 : 1];
    // the matrix-core tables during the sweeps, the reduction at the end
    constexpr int NRED = 3 * (BLOCK / 64), NMF = MF ? 2 * NQ * S::NI : 0;
    __shared__ double red[NRED > NMF ? NRED : NMF];
    double *mft = red;
    if (LIM) lim_values3<P, NQ>(g, tb, x, e0, nel, L, U);
    if (MF) mfma_tables<S::NI, NQ>(tb, mft);
    gather3<P, NQ>(g, x, e0, nel, L.X, false);
    __syncthreads();
    if constexpr (MF)
        forward3_mfma<P, NQ, NR>(mft, L.X, L.R1, L.R2, L.RY, nel);
    else
        forward3<P, NQ, double, NR>(tb, L.X, L.R1, L.R2, L.RY, nel);
    double nbad = 0.0, esum = 0.0, dmin = 1.0e300;
    for (int idx = threadIdx.x; idx < nel * S::NQ3; idx += BLOCK) {
        const int el = idx / S::NQ3, q = idx % S::NQ3;
        double J[9], Pm[9], mu;
        point_J3<P, NQ, double, NR>(L.RY, el, q, J);
        if (EN) dmin = fmin(dmin, det_only<3>(J));
        const double z = point_weight3<NQ>(tb, tg, q);
        if (!metric_first<3>(tg, J, z, &mu, Pm)) {
            nbad += 1.0;
#pragma unroll
            for (int k = 0; k < 9; ++k) Pm[k] = 0.0;
        } else if (EN) {
            esum += z * mu;
        }
        if (EN && LIM) {
            double y2 = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double u = U[(el * 3 + c) * S::NQ3 + q];
                y2 += u * u;
            }
            esum += qweight3<NQ>(tb, q) * g.lim * y2;
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) L.RY[(el * NR + k) * S::NQ3 + q] = Pm[k];
        if (LIM) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
                L.RY[(el * NR + 9 + c) * S::NQ3 + q] =
                    2.0 * qweight3<NQ>(tb, q) * g.lim * U[(el * 3 + c) * S::NQ3 + q];
        }
    }
    __syncthreads();
    backward3<P, NQ, double, double, NR, LIM>(tb, g, e0, L.RY, L.R2, L.R1, nel, gE);
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

// Hessian setup (Sec. 3.4): per point the packed z * H_A tensor, stored
// element-major in the 16-byte-run layout of qdata_store.
template <int P, int NQ, typename TT, bool MF = false>
__device__ __forceinline__ void b3_setup(const Geom &g, const Tables &tb, const Target &tg,
                                const double *__restrict__ x, TT *__restrict__ H,
                                double *__restrict__ bad, int e0, int nel)
{
    using S = S3<P, NQ>;
    __shared__ Lds3<P, NQ, double> L;
    __shared__ double red[BLOCK / 64];
    __shared__ double mft[MF ? 2 * NQ * S::NI : 1];
    if (MF) mfma_tables<S::NI, NQ>(tb, mft);
    gather3<P, NQ>(g, x, e0, nel, L.X, false);
    __syncthreads();
    if constexpr (MF)
        forward3_mfma<P, NQ>(mft, L.X, L.R1, L.R2, L.RY, nel);
    else
        forward3<P, NQ>(tb, L.X, L.R1, L.R2, L.RY, nel);
    double nbad = 0.0;
    for (int idx = threadIdx.x; idx < nel * S::NQ3; idx += BLOCK) {
        const int el = idx / S::NQ3, q = idx % S::NQ3;
        double J[9], Hp[45];
        point_J3<P, NQ>(L.RY, el, q, J);
        const double z = point_weight3<NQ>(tb, tg, q);
        if (!metric_second<3>(tg, J, z, Hp)) {
            nbad += 1.0;
#pragma unroll
            for (int k = 0; k < 45; ++k) Hp[k] = 0.0;
        }
        using QL = QLay<TT, 45, S::NQ3>;
        TT hs[45];
#pragma unroll
        for (int k = 0; k < 45; ++k) hs[k] = (TT)Hp[k];
        qdata_store<TT, 45, S::NQ3>(H + (size_t)(e0 + el) * QL::STRIDE, q, hs);
    }
    const double b = block_sum(nbad, red);
    if (threadIdx.x == 0) bad[blockIdx.x] = b;
}

// Point stage of the action at point q of element el: Y = H : (grad v) from
// the point's stored tensor hr, in place of the gradient planes of RY.
template <int P, int NQ, typename TT, typename CT, int NR, bool LIM>
__device__ __forceinline__ void apply_point3(const Tables &tb, const Geom &g, const TT *hr, int el,
                                             int q, CT *RY)
{
    constexpr int NQ3 = S3<P, NQ>::NQ3;
    CT hv[45];
#pragma unroll
    for (int k = 0; k < 45; ++k) hv[k] = (CT)hr[k];
    CT J[9];
    point_J3<P, NQ, CT, NR>(RY, el, q, J);
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        CT s = 0;
#pragma unroll
        for (int c = 0; c < 9; ++c) s += hv[sym_index<9>(r, c)] * J[c];
        RY[(el * NR + r) * NQ3 + q] = s;
    }
    if (LIM) lim_point3<NQ, CT, NR>(tb, g, el, q, RY);
}

// Hessian action, element part (Sec. 3.4, eq. eq_vm_pa_hess):
//   grad v at the points (forward contractions of P v),
//   Y_an = sum_bp H[an,bp] (grad v)_bp  with the stored tensor,
//   transposed contractions -> E-vector.
// CT = double (FP64) or float (mixed: FP32 tensor, FP32 arithmetic and
// accumulation).  This is the point-pass body; b3_apply chooses between it
// and the layer-chunked body (b3_apply_layers).
template <int P, int NQ, typename TT, typename CT, bool LIM = false, int T2 = 2>
__device__ __forceinline__ void b3_apply_points(const Geom &g, const Tables &tb,
                                                const TT *__restrict__ H,
                                                const double *__restrict__ v,
                                                CT *__restrict__ yE, int e0, int nel)
{
    using S = S3<P, NQ, T2>;
    using QL = QLay<TT, 45, S::NQ3>;
    constexpr int NR = Planes3<LIM>::NR;
    // The lanes take the workgroup's points in PASSES passes of BLOCK.  With
    // one pass (ONE) each lane's tensor is loaded before the sweeps and stays
    // in flight behind them (barriers wait on LDS only).  With PF (more than
    // one pass at the base tile shape, n_q^3 > 256) the first pass is loaded
    // so too and each later pass while the previous one computes, at the cost
    // of a second register set for the tensor: taken for FP32 data, and for
    // FP64 data only where the LDS already limits a CU to two workgroups (the
    // registers would otherwise cut the workgroups per CU).
    constexpr int PASSES = (S::EPB * S::NQ3 + BLOCK - 1) / BLOCK;
    constexpr bool ONE = PASSES == 1;
    constexpr bool PF = !ONE && T2 == 2 &&
                        (sizeof(TT) == 4 || 3 * sizeof(Lds3<P, NQ, CT, NR, T2>) > LDS_PER_CU);
    __shared__ Lds3<P, NQ, CT, NR, T2> L;
    // v loads first, then the tensor loads, then v to LDS: waiting for v
    // leaves the tensor loads in flight
    Gath3<P, NQ, T2> gv;
    gather3_load<P, NQ, T2>(g, v, e0, nel, true, gv);
    const int npts = nel * S::NQ3;
    if constexpr (PF) {
        // point data of pass k; lanes past the last point re-read the first
        // point, so that no branch sits around the loads
        TT hraw[2][45];
        auto load_pass = [&](int k, TT *dst) {
            const int i = threadIdx.x + k * BLOCK;
            const int t = i < npts ? i : 0;
            qdata_load<TT, 45, S::NQ3, true>(H + (size_t)(e0 + t / S::NQ3) * QL::STRIDE,
                                             t % S::NQ3, dst);
        };
        load_pass(0, hraw[0]);
        gather3_store<P, NQ, CT, T2>(gv, nel, L.X);
        __syncthreads();
        forward3<P, NQ, CT, NR, LIM>(tb, L.X, L.R1, L.R2, L.RY, nel);
#pragma unroll
        for (int k = 0; k < PASSES; ++k) {
            const int idx = threadIdx.x + k * BLOCK;
            if (k + 1 < PASSES) load_pass(k + 1, hraw[(k + 1) & 1]);
            if (idx < npts)
                apply_point3<P, NQ, TT, CT, NR, LIM>(tb, g, hraw[k & 1], idx / S::NQ3,
                                                     idx % S::NQ3, L.RY);
        }
    } else {
        TT hraw[45];
        if (ONE) {
            // every lane loads (lanes past the last point re-read the first
            // point): with no branch around these loads, the wait for the v
            // loads can leave all of them in flight
            const int t = threadIdx.x < npts ? threadIdx.x : 0;
            const int el = t / S::NQ3, q = t % S::NQ3;
            qdata_load<TT, 45, S::NQ3, true>(H + (size_t)(e0 + el) * QL::STRIDE, q, hraw);
        }
        gather3_store<P, NQ, CT, T2>(gv, nel, L.X);
        __syncthreads();
        forward3<P, NQ, CT, NR, LIM>(tb, L.X, L.R1, L.R2, L.RY, nel);
        for (int idx = threadIdx.x; idx < npts; idx += BLOCK) {
            const int el = idx / S::NQ3, q = idx % S::NQ3;
            if (!ONE) qdata_load<TT, 45, S::NQ3, true>(H + (size_t)(e0 + el) * QL::STRIDE, q, hraw);
            CT hv[45];
#pragma unroll
            for (int k = 0; k < 45; ++k) hv[k] = (CT)hraw[k];
            CT J[9];
            point_J3<P, NQ, CT, NR>(L.RY, el, q, J);
#pragma unroll
            for (int r = 0; r < 9; ++r) {
                CT s = 0;
#pragma unroll
                for (int c = 0; c < 9; ++c) s += hv[sym_index<9>(r, c)] * J[c];
                L.RY[(el * NR + r) * S::NQ3 + q] = s;
            }
            if (LIM) lim_point3<NQ, CT, NR>(tb, g, el, q, L.RY);
        }
    }
    __syncthreads();
    backward3<P, NQ, CT, CT, NR, LIM, true>(tb, g, e0, L.RY, L.R2, L.R1, nel, yE);
}

// ------------------------------------------------------------------------
// Compact quadrature data: per point T = A W^{-1} (9 values) and the four
// weighted metric coefficients z c_id, z c_tc, z c_cc, z c_dc (13 values per
// point, in the layout of qdata_store).  The fourth-order tensor is then applied in closed form:
//   d2mu : M = c_id M + c_tc (T (C:M) + C (T:M)) + c_cc C (C:M) + c_dc dC[M],
// with C = cof T and dC[M] the derivative of the cofactor at T in direction M
// (the bilinear part of cof(T + M)).  Same result as the stored tensor,
// 13 instead of 45 values per point.
// ------------------------------------------------------------------------
constexpr int NC3 = 13;

template <typename CT>
__device__ __forceinline__ void cof3(const CT *T, CT *C)
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
__device__ __forceinline__ void compact_action3(const CT *T, CT ca, CT cb, CT cc, CT cd, const CT *M, CT *Y)
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
__device__ __forceinline__ void mul_winv(const Target &t, const CT *in, CT *out, bool tr)
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

// Hessian action of the classes with more points than lanes (n_q^3 > 256:
// n_q = 7 and the 9-point classes; one element per workgroup), point layers
// along the third axis taken CH at a time, CH n_q^2 <= 256.  Per chunk: the
// axis-3 forward contraction for its layers only (J at its points), the
// point stage, and the axis-3 transposed contraction added into per-lane
// accumulators (one lane per (component, q1, q2) pencil, 3 n_q^2 <= 256).
// Only one chunk of point values is held in LDS (9 CH n_q^2 instead of
// 9 n_q^3 entries: 47 instead of 82 KB per workgroup at p = 4, n_q = 9 in
// FP64, three workgroups per CU instead of two).  The point data of the next
// chunk is loaded as soon as the point stage has used the current one, so it
// is in flight during the accumulation and the next forward contraction.
// Every sum runs in the order of the unchunked sweeps (q3 ascending), so the
// result is bitwise that of forward3 / point stage / backward3.
template <int P, int NQ, typename TT, typename CT, bool COMPACT>
__device__ __forceinline__ void b3_apply_layers(const Geom &g, const Tables &tb, const Target &tg,
                                                const TT *__restrict__ Hq,
                                                const double *__restrict__ v,
                                                CT *__restrict__ yE, int e0, int nel)
{
    using S = S3<P, NQ>;
    constexpr int NI = S::NI, L2 = S::L2, NQ2 = S::NQ2, NQ3 = S::NQ3;
    constexpr int NS = COMPACT ? NC3 : 45;
    using QL = QLay<TT, NS, NQ3>;
    constexpr int CH = BLOCK / NQ2;          // point layers per chunk
    constexpr int NCH = (NQ + CH - 1) / CH;  // chunks
    constexpr int CN = CH * NQ2;             // points per chunk (at most)
    static_assert(S::EPB == 1 && CH >= 1 && 3 * NQ2 <= BLOCK, "one element, one pencil per lane");
    // X / R2 and R1 / point values share storage as in Lds3
    __shared__ union {
        CT X[3 * S::NP];
        CT R2[9 * L2];
    } A;
    __shared__ union {
        CT R1[6 * S::L1];
        CT RY[9 * CN];
    } B;
    Gath3<P, NQ> gv;
    gather3_load<P, NQ>(g, v, e0, nel, true, gv);
    const TT *he = Hq + (size_t)e0 * QL::STRIDE;
    // the point data of chunk ch for this lane (lanes past the chunk's points
    // re-read point 0, so that no branch sits around the loads)
    TT hraw[NS];
    auto load_chunk = [&](int ch) {
        const int q3 = ch * CH + (int)threadIdx.x / NQ2;
        const bool in = (int)threadIdx.x < CN && q3 < NQ;
        const int q = in ? q3 * NQ2 + (int)threadIdx.x % NQ2 : 0;
        qdata_load<TT, NS, NQ3, !COMPACT>(he, q, hraw);
    };
    load_chunk(0);
    gather3_store<P, NQ, CT>(gv, nel, A.X);
    __syncthreads();
    forward3_head<P, NQ, CT>(tb, A.X, B.R1, A.R2, nel);
    // pencil of this lane for the axis-3 contractions
    const bool pen = (int)threadIdx.x < 3 * NQ2;
    const int c = (int)threadIdx.x / NQ2, q12 = (int)threadIdx.x % NQ2;
    CT acc0[NI], acc1[NI], acc2[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) acc0[k] = acc1[k] = acc2[k] = 0;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        const int nl = (ch + 1) * CH <= NQ ? CH : NQ - ch * CH;  // layers of this chunk
        // axis 3, forward: J[c][b] at this chunk's layers (plane c*3+b of RY)
        if (pen) {
            const CT *t = A.R2 + c * 3 * L2 + q12;
            CT t0[NI], t1[NI], t2[NI];
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                t0[k] = t[k * NQ2];
                t1[k] = t[L2 + k * NQ2];
                t2[k] = t[2 * L2 + k * NQ2];
            }
#pragma unroll
            for (int l = 0; l < CH; ++l) {
                if (l < nl) {
                    const int q = ch * CH + l;
                    CT a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
                    for (int k = 0; k < NI; ++k) {
                        const CT b3 = tabB<CT>(tb, q * NI + k), g3 = tabG<CT>(tb, q * NI + k);
                        a0 += b3 * t0[k];
                        a1 += b3 * t1[k];
                        a2 += g3 * t2[k];
                    }
                    CT *o = B.RY + (c * 3) * CN + l * NQ2 + q12;
                    o[0] = a0;
                    o[CN] = a1;
                    o[2 * CN] = a2;
                }
            }
        }
        __syncthreads();
        // point stage at this chunk's points
        const int tp = threadIdx.x;
        if (tp < nl * NQ2) {
            CT J[9], Y[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) J[k] = B.RY[k * CN + tp];
            if constexpr (COMPACT) {
                CT d[NC3];
#pragma unroll
                for (int m = 0; m < NC3; ++m) d[m] = (CT)hraw[m];
                if (tg.ideal) {
                    compact_action3<CT>(d, d[9], d[10], d[11], d[12], J, Y);
                } else {
                    CT M[9], Yt[9];
                    mul_winv<3, CT>(tg, J, M, false);
                    compact_action3<CT>(d, d[9], d[10], d[11], d[12], M, Yt);
                    mul_winv<3, CT>(tg, Yt, Y, true);
                }
            } else {
                CT hv[45];
#pragma unroll
                for (int m = 0; m < 45; ++m) hv[m] = (CT)hraw[m];
#pragma unroll
                for (int r = 0; r < 9; ++r) {
                    CT sr = 0;
#pragma unroll
                    for (int k = 0; k < 9; ++k) sr += hv[sym_index<9>(r, k)] * J[k];
                    Y[r] = sr;
                }
            }
#pragma unroll
            for (int k = 0; k < 9; ++k) B.RY[k * CN + tp] = Y[k];
        }
        if (ch + 1 < NCH) load_chunk(ch + 1);
        __syncthreads();
        // axis 3, transposed: this chunk's layers added into the accumulators
        if (pen) {
            const CT *y = B.RY + (c * 3) * CN + q12;
#pragma unroll
            for (int l = 0; l < CH; ++l) {
                if (l < nl) {
                    const int q = ch * CH + l;
                    const CT y0 = y[l * NQ2], y1 = y[CN + l * NQ2], y2 = y[2 * CN + l * NQ2];
#pragma unroll
                    for (int k = 0; k < NI; ++k) {
                        const CT b3 = tabB<CT>(tb, q * NI + k), g3 = tabG<CT>(tb, q * NI + k);
                        acc0[k] += b3 * y0;
                        acc1[k] += b3 * y1;
                        acc2[k] += g3 * y2;
                    }
                }
            }
        }
        if (ch + 1 < NCH) __syncthreads();
    }
    // R2 was last read before the point stage of the last chunk
    if (pen) {
        CT *o = A.R2 + c * 3 * L2 + q12;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            o[k * NQ2] = acc0[k];
            o[L2 + k * NQ2] = acc1[k];
            o[2 * L2 + k * NQ2] = acc2[k];
        }
    }
    __syncthreads();
    backward3_tail<P, NQ, CT, CT, !COMPACT>(tb, g, e0, A.R2, B.R1, nel, yE);
}

// The compact data of one point (T and z times the four metric
// coefficients), rounded to TT as stored; all zero and false when det T <= 0.
template <typename TT>
__device__ __forceinline__ bool compact_point3(const Target &tg, const double *J, double z, TT *hs)
{
    double T[9], C[9], out[NC3];
    apply_winv<3>(tg, J, T);
    const double tau = det_cof<3>(T, C);
    const bool ok = tau > 0.0;
    if (ok) {
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
#pragma unroll
        for (int k = 0; k < NC3; ++k) out[k] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < NC3; ++k) hs[k] = (TT)out[k];
    return ok;
}

template <int P, int NQ, typename TT, bool MF = false>
__device__ __forceinline__ void b3_setupc(const Geom &g, const Tables &tb, const Target &tg,
                                 const double *__restrict__ x, TT *__restrict__ Q,
                                 double *__restrict__ bad, int e0, int nel)
{
    using S = S3<P, NQ>;
    __shared__ Lds3<P, NQ, double> L;
    __shared__ double red[BLOCK / 64];
    __shared__ double mft[MF ? 2 * NQ * S::NI : 1];
    if (MF) mfma_tables<S::NI, NQ>(tb, mft);
    gather3<P, NQ>(g, x, e0, nel, L.X, false);
    __syncthreads();
    if constexpr (MF)
        forward3_mfma<P, NQ>(mft, L.X, L.R1, L.R2, L.RY, nel);
    else
        forward3<P, NQ>(tb, L.X, L.R1, L.R2, L.RY, nel);
    double nbad = 0.0;
    for (int idx = threadIdx.x; idx < nel * S::NQ3; idx += BLOCK) {
        const int el = idx / S::NQ3, q = idx % S::NQ3;
        double J[9];
        point_J3<P, NQ>(L.RY, el, q, J);
        TT hs[NC3];
        if (!compact_point3<TT>(tg, J, point_weight3<NQ>(tb, tg, q), hs)) nbad += 1.0;
        qdata_store<TT, NC3, S::NQ3>(Q + (size_t)(e0 + el) * QLay<TT, NC3, S::NQ3>::STRIDE, q, hs);
    }
    const double b = block_sum(nbad, red);
    if (threadIdx.x == 0) bad[blockIdx.x] = b;
}

template <int P, int NQ, typename TT, typename CT, bool LIM = false, int T2 = 2>
__device__ __forceinline__ void b3_applyc_points(const Geom &g, const Tables &tb,
                                                 const Target &tg, const TT *__restrict__ Q,
                                                 const double *__restrict__ v,
                                                 CT *__restrict__ yE, int e0, int nel)
{
    using S = S3<P, NQ, T2>;
    using QL = QLay<TT, NC3, S::NQ3>;
    constexpr int NR = Planes3<LIM>::NR;
    // passes of the points as in b3_apply_points; the 13 values of a point are
    // few enough that PF (the next pass loaded while the previous one
    // computes) costs no workgroups per CU at any tile shape (with two points
    // per lane: -6% at 24^3 Q3, -9% at 32^3 Q4, -3% for the 256-mesh batch),
    // and one pass runs unrolled (fewer registers than the loop form: 90
    // instead of 107 VGPRs at Q3, five workgroups per CU instead of four)
    constexpr int PASSES = (S::EPB * S::NQ3 + BLOCK - 1) / BLOCK;
    constexpr bool ONE = PASSES == 1;
    constexpr bool PF = !ONE;
    __shared__ Lds3<P, NQ, CT, NR, T2> L;
    Gath3<P, NQ, T2> gv;
    gather3_load<P, NQ, T2>(g, v, e0, nel, true, gv);
    const int npts = nel * S::NQ3;
    auto load_pass = [&](int k, TT *dst) {
        const int i = threadIdx.x + k * BLOCK;
        const int t = i < npts ? i : 0;
        qdata_load<TT, NC3, S::NQ3>(Q + (size_t)(e0 + t / S::NQ3) * QL::STRIDE, t % S::NQ3, dst);
    };
    TT draw[PF ? 2 : 1][NC3];
    if (ONE || PF) load_pass(0, draw[0]);
    gather3_store<P, NQ, CT, T2>(gv, nel, L.X);
    __syncthreads();
    forward3<P, NQ, CT, NR, LIM>(tb, L.X, L.R1, L.R2, L.RY, nel);
#pragma unroll
    for (int k = 0; k < PASSES; ++k) {
        const int idx = threadIdx.x + k * BLOCK;
        if (PF && k + 1 < PASSES) load_pass(k + 1, draw[(k + 1) & 1]);
        if (!ONE && !PF && idx < npts) load_pass(k, draw[0]);
        if (idx < npts) {
            const TT *dr = draw[PF ? (k & 1) : 0];
            const int el = idx / S::NQ3, q = idx % S::NQ3;
            CT d[NC3];
#pragma unroll
            for (int m = 0; m < NC3; ++m) d[m] = (CT)dr[m];
            CT J[9], Y[9];
            point_J3<P, NQ, CT, NR>(L.RY, el, q, J);
            if (tg.ideal) {
                compact_action3<CT>(d, d[9], d[10], d[11], d[12], J, Y);
            } else {
                CT M[9], Yt[9];
                mul_winv<3, CT>(tg, J, M, false);
                compact_action3<CT>(d, d[9], d[10], d[11], d[12], M, Yt);
                mul_winv<3, CT>(tg, Yt, Y, true);
            }
#pragma unroll
            for (int r = 0; r < 9; ++r) L.RY[(el * NR + r) * S::NQ3 + q] = Y[r];
            if (LIM) lim_point3<NQ, CT, NR>(tb, g, el, q, L.RY);
        }
    }
    __syncthreads();
    backward3<P, NQ, CT, CT, NR, LIM>(tb, g, e0, L.RY, L.R2, L.R1, nel, yE);
}

// Hessian action, element part: the layer-chunked body or the point-pass
// body.  Layer chunks apply to the classes with more points than lanes at the
// base tile shape, without the limiting term, where they measured faster
// (24^3 Kershaw meshes p = 1..4 with 9^3 points, and p = 4 with 7^3 points):
// FP64 compact data (-11% to -26%, from 3 to 5 workgroups per CU) and the
// FP64 tensor at p = 4 (-5%).  The FP64 tensor at p <= 3 (+3%: its 360 bytes
// per point gain more from the point-pass body's two passes of loads in
// flight) and the FP32 forms (+2% to +7%) keep the point-pass body.
template <int P, int NQ, int T2, bool LIM, typename CT, bool COMPACT>
constexpr bool apply_layers3()
{
    return S3<P, NQ>::NQ3 > BLOCK && T2 == 2 && !LIM && sizeof(CT) == 8 && (COMPACT || P >= 4);
}

template <int P, int NQ, typename TT, typename CT, bool LIM = false, int T2 = 2>
__device__ __forceinline__ void b3_apply(const Geom &g, const Tables &tb, const TT *__restrict__ H,
                                const double *__restrict__ v, CT *__restrict__ yE, int e0, int nel)
{
    if constexpr (apply_layers3<P, NQ, T2, LIM, CT, false>())
        b3_apply_layers<P, NQ, TT, CT, false>(g, tb, Target{}, H, v, yE, e0, nel);
    else
        b3_apply_points<P, NQ, TT, CT, LIM, T2>(g, tb, H, v, yE, e0, nel);
}

template <int P, int NQ, typename TT, typename CT, bool LIM = false, int T2 = 2>
__device__ __forceinline__ void b3_applyc(const Geom &g, const Tables &tb, const Target &tg,
                                 const TT *__restrict__ Q, const double *__restrict__ v,
                                 CT *__restrict__ yE, int e0, int nel)
{
    if constexpr (apply_layers3<P, NQ, T2, LIM, CT, true>())
        b3_apply_layers<P, NQ, TT, CT, true>(g, tb, tg, Q, v, yE, e0, nel);
    else
        b3_applyc_points<P, NQ, TT, CT, LIM, T2>(g, tb, tg, Q, v, yE, e0, nel);
}

// Hessian diagonal, element part (Sec. 3.4, last paragraph):
//   d_a(i) = sum_q sum_{n,p} H[an,ap](q) dw_i/dxbar_n dw_i/dxbar_p,
// contracted per (n,p) pair with the squared 1D tables BB, BG, GG.  The 18
// needed entries H[an,ap] (3 components x 6 pairs n <= p, off-diagonal pairs
// doubled) are first placed in LDS planes sQ[el][pair][a][q].  With the
// limiting term a seventh "pair" holds 2 w_q lim, contracted with BB on every
// axis (the diagonal of the mass-like term, eq. eq_pa_limiting).
template <int P, int NQ, bool LIM = false>
struct DiagLds3 {
    using S = S3<P, NQ>;
    static constexpr int NPR = LIM ? 7 : 6;
    double T[3][NQ * S::NI];  // B B, B G, G G at (chi_q, node i)
    double sQ[S::EPB * NPR * 3 * S::NQ3];
    double U2[S::EPB * 3 * S::NI * NQ * NQ];
    double U1[S::EPB * 3 * S::NI * S::NI * NQ];
    double sD[S::EPB * 3 * S::NP];
};

// pair pr < 6: (n, p) = (0,0) (0,1) (0,2) (1,1) (1,2) (2,2); pr = 6: value term
__device__ constexpr int diag_pn(int pr) { return pr < 3 ? 0 : (pr < 5 ? 1 : 2); }
__device__ constexpr int diag_pp(int pr) { return pr < 3 ? pr : (pr < 5 ? pr - 2 : 2); }

// One 1D line of the diagonal contraction: out[i] = sum_q Tt[q*NI + i] y[q],
// Tt the product table of the axis in LDS; every lane reads the same entry at
// once (a broadcast).
template <int NQ, int NI>
__device__ __forceinline__ void diag_line(const double *Tt, const double *yv, double *out)
{
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) s += Tt[q * NI + i] * yv[q];
        out[i] = s;
    }
}

template <int P, int NQ, bool LIM>
__device__ __forceinline__ void diag_contract3(const Tables &tb, const Geom &g, int e0,
                                      DiagLds3<P, NQ, LIM> &L, int nel, double *__restrict__ dE)
{
    using S = S3<P, NQ>;
    constexpr int NI = S::NI, NQ3 = S::NQ3, NP = S::NP, NPR = DiagLds3<P, NQ, LIM>::NPR;
    for (int k = threadIdx.x; k < NQ * NI; k += BLOCK) {
        const double b = tb.B[k], gg = tb.G[k];
        L.T[0][k] = b * b;
        L.T[1][k] = b * gg;
        L.T[2][k] = gg * gg;
    }
    for (int k = threadIdx.x; k < nel * 3 * NP; k += BLOCK) L.sD[k] = 0.0;
    // one pass per pair as three pencil sweeps: a lane loads one 1D line from
    // LDS and produces the n_i outputs of that line
    for (int pr = 0; pr < NPR; ++pr) {
        const int n = diag_pn(pr), p = diag_pp(pr);
        // number of derivative factors on each axis
        const bool val = pr == 6;
        const int t1 = val ? 0 : (n == 0) + (p == 0), t2 = val ? 0 : (n == 1) + (p == 1),
                  t3 = val ? 0 : (n == 2) + (p == 2);
        // sQ and sD ready; later pairs need no barrier here (their axis-3 pass
        // writes U2 only, which the previous pair's axis-1 pass does not read)
        if (pr == 0) __syncthreads();
        // axis 3: pencils (r = el*3 + a, q2, q1) -> U2[r][i3][q2][q1]
        for (int pen = threadIdx.x; pen < nel * 3 * NQ * NQ; pen += BLOCK) {
            const int q21 = pen % (NQ * NQ), r = pen / (NQ * NQ);
            const int el = r / 3, a = r % 3;
            const double *y = L.sQ + ((el * NPR + pr) * 3 + a) * NQ3 + q21;
            double yv[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) yv[q] = y[q * NQ * NQ];
            double o[NI];
            diag_line<NQ, NI>(L.T[t3], yv, o);
#pragma unroll
            for (int i = 0; i < NI; ++i) L.U2[(r * NI + i) * NQ * NQ + q21] = o[i];
        }
        __syncthreads();
        // axis 2: pencils (r, i3, q1) -> U1[r][i3][i2][q1]
        for (int pen = threadIdx.x; pen < nel * 3 * NI * NQ; pen += BLOCK) {
            const int q1 = pen % NQ, ri3 = pen / NQ;
            const double *y = L.U2 + ri3 * NQ * NQ + q1;
            double yv[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) yv[q] = y[q * NQ];
            double o[NI];
            diag_line<NQ, NI>(L.T[t2], yv, o);
#pragma unroll
            for (int i = 0; i < NI; ++i) L.U1[(ri3 * NI + i) * NQ + q1] = o[i];
        }
        __syncthreads();
        // axis 1: pencils (r, i3, i2) -> the n_i diagonal entries of the line,
        // each written by one lane
        for (int pen = threadIdx.x; pen < nel * 3 * NI * NI; pen += BLOCK) {
            const double *y = L.U1 + pen * NQ;
            double yv[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) yv[q] = y[q];
            double o[NI];
            diag_line<NQ, NI>(L.T[t1], yv, o);
#pragma unroll
            for (int i = 0; i < NI; ++i) L.sD[pen * NI + i] += o[i];
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nel * 3 * NP; k += BLOCK) {
        const int i = k % NP, r = k / NP;
        dE[ev_index3<P>(g, e0 + r / 3, r % 3, i % NI, (i / NI) % NI, i / (NI * NI))] = L.sD[k];
    }
}

// the limiting pair's planes: 2 w_q lim for each component
template <int P, int NQ, bool LIM>
__device__ __forceinline__ void diag_lim3(const Tables &tb, const Geom &g, DiagLds3<P, NQ, LIM> &L, int el,
                                 int q)
{
    if (!LIM) return;
    constexpr int NQ3 = S3<P, NQ>::NQ3, NPR = DiagLds3<P, NQ, LIM>::NPR;
    const double f = 2.0 * g.lim * qweight3<NQ>(tb, q);
#pragma unroll
    for (int a = 0; a < 3; ++a) L.sQ[((el * NPR + 6) * 3 + a) * NQ3 + q] = f;
}

template <int P, int NQ, typename TT, bool LIM = false>
__device__ __forceinline__ void b3_diag(const Geom &g, const Tables &tb, const TT *__restrict__ H,
                               double *__restrict__ dE, int e0, int nel)
{
    using S = S3<P, NQ>;
    constexpr int NPR = DiagLds3<P, NQ, LIM>::NPR;
    __shared__ DiagLds3<P, NQ, LIM> L;
    for (int idx = threadIdx.x; idx < nel * S::NQ3; idx += BLOCK) {
        const int el = idx / S::NQ3, q = idx % S::NQ3;
        const TT *h = H + (size_t)(e0 + el) * QLay<TT, 45, S::NQ3>::STRIDE;
#pragma unroll
        for (int pr = 0; pr < 6; ++pr) {
            const int n = diag_pn(pr), p = diag_pp(pr);
            const double f = (n == p) ? 1.0 : 2.0;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                L.sQ[((el * NPR + pr) * 3 + a) * S::NQ3 + q] =
                    f * (double)qdata_at<TT, 45, S::NQ3>(h, q, sym_index<9>(a * 3 + n, a * 3 + p));
        }
        diag_lim3<P, NQ, LIM>(tb, g, L, el, q);
    }
    diag_contract3<P, NQ, LIM>(tb, g, e0, L, nel, dE);
}

// The diagonal's LDS planes of one point from its compact data (b3_diagc).
template <int P, int NQ, typename TT, bool LIM>
__device__ __forceinline__ void diagc_point3(const Tables &tb, const Geom &g, const Target &tg,
                                    const TT *hr, DiagLds3<P, NQ, LIM> &L, int el, int q)
{
    using S = S3<P, NQ>;
    constexpr int NPR = DiagLds3<P, NQ, LIM>::NPR;
    {
        double T[9], C[9], Tw[9], Cw[9], WW[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) T[k] = (double)hr[k];
        const double cid = hr[9], ctc = hr[10], ccc = hr[11];
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
                L.sQ[((el * NPR + pr) * 3 + a) * S::NQ3 + q] = f * hv;
            }
        }
        diag_lim3<P, NQ, LIM>(tb, g, L, el, q);
    }
}

// Diagonal from compact data: within one component a the cofactor-derivative
// term vanishes, so H[an,ap] = c_id (W^-1 W^-T)_np + c_tc (Tw_an Cw_ap +
// Cw_an Tw_ap) + c_cc Cw_an Cw_ap with Tw = T W^{-T}, Cw = C W^{-T}.
template <int P, int NQ, typename TT, bool LIM = false>
__device__ __forceinline__ void b3_diagc(const Geom &g, const Tables &tb, const Target &tg,
                                const TT *__restrict__ Q, double *__restrict__ dE, int e0, int nel)
{
    using S = S3<P, NQ>;
    __shared__ DiagLds3<P, NQ, LIM> L;
    for (int idx = threadIdx.x; idx < nel * S::NQ3; idx += BLOCK) {
        const int el = idx / S::NQ3, q = idx % S::NQ3;
        TT hr[NC3];
        qdata_load<TT, NC3, S::NQ3>(Q + (size_t)(e0 + el) * QLay<TT, NC3, S::NQ3>::STRIDE, q, hr);
        diagc_point3<P, NQ, TT, LIM>(tb, g, tg, hr, L, el, q);
    }
    diag_contract3<P, NQ, LIM>(tb, g, e0, L, nel, dE);
}

// Hessian setup and the element part of the Hessian diagonal in one pass
// (Sec. 3.4, the diagonal in its last paragraph), for the Jacobi
// preconditioner of each Newton step: the setup's per-point tensor, rounded to
// TT as it is stored, fills the diagonal's LDS planes at once instead of being
// read back from HBM by b3_diag.  The diagonal's buffers overlay the sweeps'
// (every lane holds its J before the barrier that hands the memory over), so
// the workgroup needs no more LDS than b3_diag.  Classes whose points fit one
// pass of the workgroup.  H, bad and dE are bitwise those of b3_setup then
// b3_diag.
template <int P, int NQ, typename TT, bool LIM>
__device__ __forceinline__ void b3_setupd(const Geom &g, const Tables &tb, const Target &tg,
                                 const double *__restrict__ x, TT *__restrict__ H,
                                 double *__restrict__ dE, double *__restrict__ bad, int e0,
                                 int nel)
{
    using S = S3<P, NQ>;
    static_assert(S::EPB * S::NQ3 <= BLOCK, "one pass over the workgroup's points");
    constexpr int NPR = DiagLds3<P, NQ, LIM>::NPR;
    union Buf {
        Lds3<P, NQ, double> s;
        DiagLds3<P, NQ, LIM> d;
    };
    __shared__ Buf L;
    __shared__ double red[BLOCK / 64];
    gather3<P, NQ>(g, x, e0, nel, L.s.X, false);
    __syncthreads();
    forward3<P, NQ>(tb, L.s.X, L.s.R1, L.s.R2, L.s.RY, nel);
    const bool act = (int)threadIdx.x < nel * S::NQ3;
    const int el = act ? threadIdx.x / S::NQ3 : 0, q = act ? threadIdx.x % S::NQ3 : 0;
    double J[9];
    if (act) point_J3<P, NQ>(L.s.RY, el, q, J);
    __syncthreads();
    double nbad = 0.0;
    if (act) {
        double Hp[45];
        const double z = point_weight3<NQ>(tb, tg, q);
        if (!metric_second<3>(tg, J, z, Hp)) {
            nbad = 1.0;
#pragma unroll
            for (int k = 0; k < 45; ++k) Hp[k] = 0.0;
        }
        using QL = QLay<TT, 45, S::NQ3>;
        TT hs[45];
#pragma unroll
        for (int k = 0; k < 45; ++k) hs[k] = (TT)Hp[k];
        qdata_store<TT, 45, S::NQ3>(H + (size_t)(e0 + el) * QL::STRIDE, q, hs);
#pragma unroll
        for (int pr = 0; pr < 6; ++pr) {
            const int n = diag_pn(pr), p = diag_pp(pr);
            const double f = (n == p) ? 1.0 : 2.0;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                L.d.sQ[((el * NPR + pr) * 3 + a) * S::NQ3 + q] =
                    f * (double)hs[sym_index<9>(a * 3 + n, a * 3 + p)];
        }
        diag_lim3<P, NQ, LIM>(tb, g, L.d, el, q);
    }
    diag_contract3<P, NQ, LIM>(tb, g, e0, L.d, nel, dE);
    const double b = block_sum(nbad, red);
    if (threadIdx.x == 0) bad[blockIdx.x] = b;
}

// The same for compact storage: the setup's compact values, rounded to TT as
// stored, give the diagonal's planes as b3_diagc computes them from the
// stored data.  Q, bad and dE are bitwise those of b3_setupc then b3_diagc.
template <int P, int NQ, typename TT, bool LIM>
__device__ __forceinline__ void b3_setupcd(const Geom &g, const Tables &tb, const Target &tg,
                                  const double *__restrict__ x, TT *__restrict__ Q,
                                  double *__restrict__ dE, double *__restrict__ bad, int e0,
                                  int nel)
{
    using S = S3<P, NQ>;
    static_assert(S::EPB * S::NQ3 <= BLOCK, "one pass over the workgroup's points");
    union Buf {
        Lds3<P, NQ, double> s;
        DiagLds3<P, NQ, LIM> d;
    };
    __shared__ Buf L;
    __shared__ double red[BLOCK / 64];
    gather3<P, NQ>(g, x, e0, nel, L.s.X, false);
    __syncthreads();
    forward3<P, NQ>(tb, L.s.X, L.s.R1, L.s.R2, L.s.RY, nel);
    const bool act = (int)threadIdx.x < nel * S::NQ3;
    const int el = act ? threadIdx.x / S::NQ3 : 0, q = act ? threadIdx.x % S::NQ3 : 0;
    double J[9];
    if (act) point_J3<P, NQ>(L.s.RY, el, q, J);
    __syncthreads();
    double nbad = 0.0;
    if (act) {
        TT hs[NC3];
        if (!compact_point3<TT>(tg, J, point_weight3<NQ>(tb, tg, q), hs)) nbad = 1.0;
        qdata_store<TT, NC3, S::NQ3>(Q + (size_t)(e0 + el) * QLay<TT, NC3, S::NQ3>::STRIDE, q, hs);
        diagc_point3<P, NQ, TT, LIM>(tb, g, tg, hs, L.d, el, q);
    }
    diag_contract3<P, NQ, LIM>(tb, g, e0, L.d, nel, dE);
    const double b = block_sum(nbad, red);
    if (threadIdx.x == 0) bad[blockIdx.x] = b;
}

// ------------------------------------------------------------------------
// Kernel entry points: single mesh (grid over element blocks; LIM selects the
// variant with the limiting term) and batched (grid over a tile list of
// (slot, first element) with per-slot geometry, target and offsets into
// packed pools; no limiting term).
// ------------------------------------------------------------------------

template <int P, int NQ, bool LIM, bool MF = false>
__global__ __launch_bounds__(BLOCK) void k3_energy(Geom g, Tables tb, Target tg, const double *__restrict__ x, double *__restrict__ part)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const int e0 = xcd_block(blockIdx.x, gridDim.x) * EPB;
    b3_energy<P, NQ, LIM, MF>(g, tb, tg, x, part, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, bool LIM, bool EN = false, bool MF = false>
__global__ __launch_bounds__(BLOCK) void k3_gradient(Geom g, Tables tb, Target tg, const double *__restrict__ x, double *__restrict__ gE, double *__restrict__ bad)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const int e0 = xcd_block(blockIdx.x, gridDim.x) * EPB;
    b3_gradient<P, NQ, LIM, EN, MF>(g, tb, tg, x, gE, bad, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT, bool MF = false>
__global__ __launch_bounds__(BLOCK) void k3_setup(Geom g, Tables tb, Target tg, const double *__restrict__ x, TT *__restrict__ H, double *__restrict__ bad)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const int e0 = xcd_block(blockIdx.x, gridDim.x) * EPB;
    b3_setup<P, NQ, TT, MF>(g, tb, tg, x, H, bad, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT, typename CT, bool LIM, int T2 = 2>
__global__ __launch_bounds__(BLOCK) void k3_apply(Geom g, Tables tb, const TT *__restrict__ H, const double *__restrict__ v, CT *__restrict__ yE)
{
    constexpr int EPB = S3<P, NQ, T2>::EPB;
    const int e0 = xcd_block(blockIdx.x, gridDim.x) * EPB;
    b3_apply<P, NQ, TT, CT, LIM, T2>(g, tb, H, v, yE, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT, bool MF = false>
__global__ __launch_bounds__(BLOCK) void k3_setupc(Geom g, Tables tb, Target tg, const double *__restrict__ x, TT *__restrict__ Q, double *__restrict__ bad)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const int e0 = xcd_block(blockIdx.x, gridDim.x) * EPB;
    b3_setupc<P, NQ, TT, MF>(g, tb, tg, x, Q, bad, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT, typename CT, bool LIM, int T2 = 2>
__global__ __launch_bounds__(BLOCK) void k3_applyc(Geom g, Tables tb, Target tg, const TT *__restrict__ Q, const double *__restrict__ v, CT *__restrict__ yE)
{
    constexpr int EPB = S3<P, NQ, T2>::EPB;
    const int e0 = xcd_block(blockIdx.x, gridDim.x) * EPB;
    b3_applyc<P, NQ, TT, CT, LIM, T2>(g, tb, tg, Q, v, yE, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT, bool LIM>
__global__ __launch_bounds__(BLOCK) void k3_diag(Geom g, Tables tb, const TT *__restrict__ H, double *__restrict__ dE)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const int e0 = xcd_block(blockIdx.x, gridDim.x) * EPB;
    b3_diag<P, NQ, TT, LIM>(g, tb, H, dE, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT, bool LIM>
__global__ __launch_bounds__(BLOCK) void k3_setupd(Geom g, Tables tb, Target tg, const double *__restrict__ x, TT *__restrict__ H, double *__restrict__ dE, double *__restrict__ bad)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const int e0 = xcd_block(blockIdx.x, gridDim.x) * EPB;
    b3_setupd<P, NQ, TT, LIM>(g, tb, tg, x, H, dE, bad, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT, bool LIM>
__global__ __launch_bounds__(BLOCK) void k3_setupcd(Geom g, Tables tb, Target tg, const double *__restrict__ x, TT *__restrict__ Q, double *__restrict__ dE, double *__restrict__ bad)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const int e0 = xcd_block(blockIdx.x, gridDim.x) * EPB;
    b3_setupcd<P, NQ, TT, LIM>(g, tb, tg, x, Q, dE, bad, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, typename TT, bool LIM>
__global__ __launch_bounds__(BLOCK) void k3_diagc(Geom g, Tables tb, Target tg, const TT *__restrict__ Q, double *__restrict__ dE)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const int e0 = xcd_block(blockIdx.x, gridDim.x) * EPB;
    b3_diagc<P, NQ, TT, LIM>(g, tb, tg, Q, dE, e0, min(EPB, g.ne - e0));
}

template <int P, int NQ, bool LIM = false>
__global__ __launch_bounds__(BLOCK) void kb3_energy(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate, int vin, double *__restrict__ part)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b3_energy<P, NQ, LIM>(s.g, tb, s.tg, s.vec[vin], part, t.e0, min(EPB, s.g.ne - t.e0));
}

template <int P, int NQ, bool LIM = false, bool EN = false>
__global__ __launch_bounds__(BLOCK) void kb3_gradient(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate, int vin, double *__restrict__ bad)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b3_gradient<P, NQ, LIM, EN>(s.g, tb, s.tg, s.vec[vin], (double *)s.eV, bad, t.e0, min(EPB, s.g.ne - t.e0));
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

template <int P, int NQ, typename TT, typename CT, bool LIM = false, int T2 = 2>
__global__ __launch_bounds__(BLOCK) void kb3_apply(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate, int vin)
{
    constexpr int EPB = S3<P, NQ, T2>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b3_apply<P, NQ, TT, CT, LIM, T2>(s.g, tb, (const TT *)s.H, s.vec[vin], (CT *)s.eV, t.e0, min(EPB, s.g.ne - t.e0));
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

template <int P, int NQ, typename TT, typename CT, bool LIM = false, int T2 = 2>
__global__ __launch_bounds__(BLOCK) void kb3_applyc(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate, int vin)
{
    constexpr int EPB = S3<P, NQ, T2>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b3_applyc<P, NQ, TT, CT, LIM, T2>(s.g, tb, s.tg, (const TT *)s.H, s.vec[vin], (CT *)s.eV, t.e0, min(EPB, s.g.ne - t.e0));
}

// Does the Hessian action of this class have a tile shape T2 distinct from
// the base one that fits the LDS?  (FP64 data, the larger of the two types.)
template <int P, int NQ, int T2>
constexpr bool tile_ok3()
{
    return T2 == 2 || (S3<P, NQ, T2>::EPB != S3<P, NQ>::EPB &&
                       sizeof(Lds3<P, NQ, double, 9, T2>) <= 96 * 1024);
}

template <int P, int NQ, typename TT, bool LIM = false>
__global__ __launch_bounds__(BLOCK) void kb3_diag(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b3_diag<P, NQ, TT, LIM>(s.g, tb, (const TT *)s.H, (double *)s.eV, t.e0, min(EPB, s.g.ne - t.e0));
}

template <int P, int NQ, typename TT, bool LIM = false>
__global__ __launch_bounds__(BLOCK) void kb3_diagc(Tables tb, const Tile *__restrict__ tiles, const SlotDev *__restrict__ slots, const int *__restrict__ gate)
{
    constexpr int EPB = S3<P, NQ>::EPB;
    const Tile t = tiles[blockIdx.x];
    if (gate && !gate[t.slot]) return;
    const SlotDev &s = slots[t.slot];
    b3_diagc<P, NQ, TT, LIM>(s.g, tb, s.tg, (const TT *)s.H, (double *)s.eV, t.e0, min(EPB, s.g.ne - t.e0));
}

}  // namespace tmop
