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
template <int DIM, typename ET>
__device__ inline ET gather_box_node(const Geom &g, const ET *__restrict__ eV, int c, int node,
                                     const int *gc)
{
    const int p = g.p, ni = p + 1;
    const int np = DIM == 3 ? ni * ni * ni : ni * ni;
    // per axis: position of the copy owned by the lower element (slot 0) and
    // by the upper element (slot 1), and whether each exists
    int pos[3][2];
    bool has[3][2];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const int gk = gc[k];
        const int e = gk / p, j = gk - e * p;
        has[k][0] = j == 0 && e > 0;
        has[k][1] = e < g.nel[k];
        pos[k][0] = gk + e - 1;
        pos[k][1] = gk + e;
    }
    const int EX = g.nel[0] * ni;
    const ET *base = eV + (size_t)c * g.ne * np;
    // Rows (y, z copies) that do not exist are skipped; the test is uniform
    // along a row of nodes, so it rarely diverges within a wave.  Within a
    // row both x copies are loaded (a missing one reads the row's first entry
    // and is dropped afterwards).  No loaded value is used before the last
    // load is issued, so all are in flight together; the sum runs in a fixed
    // order.
    constexpr int NR = DIM == 3 ? 4 : 2;
    ET lo[NR], hi[NR];
    bool rok[NR];
#pragma unroll
    for (int t = 0; t < NR; ++t) {
        const int b = t & 1, a = t >> 1;
        rok[t] = has[1][b] && (DIM == 2 || has[2][a]);
        const int off = pos[1][b] * EX + (DIM == 3 ? pos[2][a] * (g.nel[1] * ni) * EX : 0);
        lo[t] = hi[t] = 0;
        if (rok[t]) {
            lo[t] = base[off + (has[0][0] ? pos[0][0] : 0)];
            hi[t] = base[off + (has[0][1] ? pos[0][1] : 0)];
        }
    }
    ET s = 0;
#pragma unroll
    for (int t = 0; t < NR; ++t) {
        s += (rok[t] && has[0][0]) ? lo[t] : (ET)0;
        s += (rok[t] && has[0][1]) ? hi[t] : (ET)0;
    }
    return s;
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

// Assembled value of entry idx = c*nx + node; *fixed tells whether the DoF is
// fixed (then the value is meaningless).
template <int DIM, typename ET>
__device__ inline double gather_entry(const Geom &g, const int32_t *__restrict__ ptr,
                                      const int32_t *__restrict__ ent, const ET *__restrict__ eV,
                                      int idx, bool *fixed)
{
    const int c = idx / g.nx;
    const int node = idx - c * g.nx;
    if (ptr) {
        *fixed = is_fixed(g, c, node, -1, -1, -1);
        return *fixed ? 0.0 : (double)gather_csr_node<DIM, ET>(g, ptr, ent, eV, c, node);
    }
    int gc[3];
    const int t = node / g.M[0];
    gc[0] = node - t * g.M[0];
    gc[1] = DIM == 3 ? t % g.M[1] : t;
    gc[2] = DIM == 3 ? t / g.M[1] : 0;
    *fixed = is_fixed(g, c, node, gc[0], gc[1], gc[2]);
    return *fixed ? 0.0 : (double)gather_box_node<DIM, ET>(g, eV, c, node, gc);
}

}  // namespace tmop
