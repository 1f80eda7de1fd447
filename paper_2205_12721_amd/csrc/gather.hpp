// Node-centric G^T (transpose of the element restriction, Sec. 3 operator
// decomposition): the value of a global DoF is the sum of its element-local
// copies in the E-vector, visited in a fixed order (deterministic, no atomics).
#pragma once
#include "tmop_dev.hpp"

namespace tmop {

// ------------------------------------------------------------------------
// G^T: sum of the (up to 2^dim) element-local copies of global node `node`,
// component c, in a fixed order (deterministic, no atomics).
// ------------------------------------------------------------------------
template <int DIM, typename ET>
__device__ inline ET gather_box_node(const Geom &g, const ET *__restrict__ eV, int c, int node,
                                     const int *gc)
{
    const int p = g.p, ni = p + 1;
    const int np = DIM == 3 ? ni * ni * ni : ni * ni;
    int ce[3][2], cj[3][2], nc[3];
    for (int k = 0; k < DIM; ++k) {
        const int gk = gc[k];
        if (gk == g.M[k] - 1) {
            ce[k][0] = g.nel[k] - 1;
            cj[k][0] = p;
            nc[k] = 1;
        } else {
            const int e = gk / p, j = gk - e * p;
            if (j == 0 && e > 0) {
                ce[k][0] = e - 1;
                cj[k][0] = p;
                ce[k][1] = e;
                cj[k][1] = 0;
                nc[k] = 2;
            } else {
                ce[k][0] = e;
                cj[k][0] = j;
                nc[k] = 1;
            }
        }
    }
    ET s = 0;
    if constexpr (DIM == 3) {
        for (int a = 0; a < nc[2]; ++a)
            for (int b = 0; b < nc[1]; ++b)
                for (int d = 0; d < nc[0]; ++d) {
                    const long e = ce[0][d] + (long)g.nel[0] * (ce[1][b] + (long)g.nel[1] * ce[2][a]);
                    const int i = cj[0][d] + ni * (cj[1][b] + ni * cj[2][a]);
                    s += eV[(e * DIM + c) * np + i];
                }
    } else {
        for (int b = 0; b < nc[1]; ++b)
            for (int d = 0; d < nc[0]; ++d) {
                const long e = ce[0][d] + (long)g.nel[0] * ce[1][b];
                const int i = cj[0][d] + ni * cj[1][b];
                s += eV[(e * DIM + c) * np + i];
            }
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
                                      long idx, bool *fixed)
{
    const int c = (int)(idx / g.nx);
    const int node = (int)(idx % g.nx);
    if (ptr) {
        *fixed = is_fixed(g, c, node, -1, -1, -1);
        return *fixed ? 0.0 : (double)gather_csr_node<DIM, ET>(g, ptr, ent, eV, c, node);
    }
    int gc[3];
    gc[0] = node % g.M[0];
    const int t = node / g.M[0];
    gc[1] = DIM == 3 ? t % g.M[1] : t;
    gc[2] = DIM == 3 ? t / g.M[1] : 0;
    *fixed = is_fixed(g, c, node, gc[0], gc[1], gc[2]);
    return *fixed ? 0.0 : (double)gather_box_node<DIM, ET>(g, eV, c, node, gc);
}

}  // namespace tmop
