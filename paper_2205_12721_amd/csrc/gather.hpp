// Node-centric G^T (transpose of the element restriction, Sec. 3 operator
// decomposition): the value of a global DoF is the sum of its element-local
// copies in the E-vector, visited in a fixed order (deterministic, no atomics).
#pragma once
#include "tmop_dev.hpp"

namespace tmop {

// ------------------------------------------------------------------------
// G^T on the structured box: sum of the (up to 2^dim) element-local copies of
// global node `node`, component c, in a fixed order (deterministic, no
// atomics).  The box E-vector is the exploded grid: along axis k, element e
// owns positions e*(p+1) .. e*(p+1)+p, so grid coordinate gk = e*p + j lands
// at position gk + e (owner e < nel) and, for a vertex shared with element
// e-1 (j = 0, e > 0), also at gk + e - 1.  The copies of one node are thus
// neighbours in x, and the lanes of a wave read runs of consecutive words.
// ------------------------------------------------------------------------
// Where the copies of box node gc lie in one component's exploded grid.
// Rows (y, z copies) that do not exist are skipped; the test is uniform along
// a row of nodes, so it rarely diverges within a wave.  Within a row both x
// copies are loaded (a missing one reads the row's first entry and is dropped
// afterwards).
template <int DIM>
struct BoxCopies {
    static constexpr int NR = DIM == 3 ? 4 : 2;
    int lo[NR], hi[NR];  // offsets of the lower / upper x copy in each row
    bool rok[NR];        // the row exists
    bool xlo, xhi;       // the lower / upper x copy exists
};

template <int DIM>
__device__ __forceinline__ BoxCopies<DIM> box_copies(const Geom &g, const int *gc)
{
    const int ni = g.p + 1;
    // per axis: position of the copy owned by the lower element (slot 0) and
    // by the upper element (slot 1), and whether each exists
    int pos[3][2];
    bool has[3][2];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const int gk = gc[k];
        const int e = fdiv(gk, g.dP), j = gk - e * g.p;
        has[k][0] = j == 0 && e > 0;
        has[k][1] = e < g.nel[k];
        pos[k][0] = gk + e - 1;
        pos[k][1] = gk + e;
    }
    const int EX = g.nel[0] * ni;
    BoxCopies<DIM> b;
    b.xlo = has[0][0];
    b.xhi = has[0][1];
#pragma unroll
    for (int t = 0; t < BoxCopies<DIM>::NR; ++t) {
        const int y = t & 1, z = t >> 1;
        b.rok[t] = has[1][y] && (DIM == 2 || has[2][z]);
        const int off = pos[1][y] * EX + (DIM == 3 ? pos[2][z] * (g.nel[1] * ni) * EX : 0);
        b.lo[t] = off + (has[0][0] ? pos[0][0] : 0);
        b.hi[t] = off + (has[0][1] ? pos[0][1] : 0);
    }
    return b;
}

// Sum of the copies of one node in one component's exploded grid `base`.
// No loaded value is used before the last load is issued, so all are in
// flight together; the sum runs in a fixed order.
template <int DIM, typename ET>
__device__ __forceinline__ ET box_sum(const BoxCopies<DIM> &b, const ET *__restrict__ base)
{
    constexpr int NR = BoxCopies<DIM>::NR;
    ET lo[NR], hi[NR];
#pragma unroll
    for (int t = 0; t < NR; ++t) {
        lo[t] = hi[t] = 0;
        if (b.rok[t]) {
            lo[t] = base[b.lo[t]];
            hi[t] = base[b.hi[t]];
        }
    }
    ET s = 0;
#pragma unroll
    for (int t = 0; t < NR; ++t) {
        s += (b.rok[t] && b.xlo) ? lo[t] : (ET)0;
        s += (b.rok[t] && b.xhi) ? hi[t] : (ET)0;
    }
    return s;
}

// ------------------------------------------------------------------------
// G^T on the structured box: sum of the (up to 2^dim) element-local copies of
// global node `node`, component c, in a fixed order (deterministic, no
// atomics).  The box E-vector is the exploded grid: along axis k, element e
// owns positions e*(p+1) .. e*(p+1)+p, so grid coordinate gk = e*p + j lands
// at position gk + e (owner e < nel) and, for a vertex shared with element
// e-1 (j = 0, e > 0), also at gk + e - 1.  The copies of one node are thus
// neighbours in x, and the lanes of a wave read runs of consecutive words.
// ------------------------------------------------------------------------
template <int DIM, typename ET>
__device__ inline ET gather_box_node(const Geom &g, const ET *__restrict__ eV, int c, int node,
                                     const int *gc)
{
    const int ni = g.p + 1;
    const int np = DIM == 3 ? ni * ni * ni : ni * ni;
    const BoxCopies<DIM> b = box_copies<DIM>(g, gc);
    return box_sum<DIM, ET>(b, eV + (size_t)c * g.ne * np);
}

// All components of box node `node` at once: the copy positions are worked
// out once and the loads of every component are in flight together.
template <int DIM, typename ET>
__device__ inline void gather_box_all(const Geom &g, const ET *__restrict__ eV, const int *gc,
                                      ET s[DIM])
{
    const int ni = g.p + 1;
    const int np = DIM == 3 ? ni * ni * ni : ni * ni;
    const BoxCopies<DIM> b = box_copies<DIM>(g, gc);
#pragma unroll
    for (int c = 0; c < DIM; ++c) s[c] = box_sum<DIM, ET>(b, eV + (size_t)c * g.ne * np);
}

template <int DIM, typename ET>
__device__ inline ET gather_csr_node(const Geom &g, const int32_t *__restrict__ ptr,
                                     const int32_t *__restrict__ ent, const ET *__restrict__ eV,
                                     int c, int node)
{
    const int ni = g.p + 1;
    const int np = DIM == 3 ? ni * ni * ni : ni * ni;
    ET s = 0;
    for (int k = ptr[node]; k < ptr[node + 1]; ++k) {
        const long en = ent[k];
        const long e = en / np;
        const int i = (int)(en % np);
        s += eV[(e * DIM + c) * np + i];
    }
    return s;
}

// All components of a general-mesh node: one walk over its element copies.
template <int DIM, typename ET>
__device__ inline void gather_csr_all(const Geom &g, const int32_t *__restrict__ ptr,
                                      const int32_t *__restrict__ ent, const ET *__restrict__ eV,
                                      int node, ET s[DIM])
{
    const int ni = g.p + 1;
    const int np = DIM == 3 ? ni * ni * ni : ni * ni;
#pragma unroll
    for (int c = 0; c < DIM; ++c) s[c] = 0;
    for (int k = ptr[node]; k < ptr[node + 1]; ++k) {
        const long en = ent[k];
        const long e = en / np;
        const int i = (int)(en % np);
#pragma unroll
        for (int c = 0; c < DIM; ++c) s[c] += eV[(e * DIM + c) * np + i];
    }
}

// Assembled values of every component of node `node`; fixed[c] tells whether
// component c is a fixed DoF (then its value is meaningless).
template <int DIM, typename ET>
__device__ inline void gather_node(const Geom &g, const int32_t *__restrict__ ptr,
                                   const int32_t *__restrict__ ent, const ET *__restrict__ eV,
                                   int node, double a[DIM], bool fixed[DIM])
{
    ET s[DIM];
    if (ptr) {
        gather_csr_all<DIM, ET>(g, ptr, ent, eV, node, s);
#pragma unroll
        for (int c = 0; c < DIM; ++c) fixed[c] = is_fixed(g, c, node, -1, -1, -1);
    } else {
        int gc[3];
        box_coords<DIM>(g, node, gc);
        gather_box_all<DIM, ET>(g, eV, gc, s);
#pragma unroll
        for (int c = 0; c < DIM; ++c) fixed[c] = is_fixed(g, c, node, gc[0], gc[1], gc[2]);
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) a[c] = fixed[c] ? 0.0 : (double)s[c];
}

}  // namespace tmop
