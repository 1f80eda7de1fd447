// Launch table: one entry per (dim, p, nq) with host launchers for every
// element kernel.  The element kernels are instantiated in k2.hip and
// k3_p*.hip; the table is filled by find_ops().
#pragma once
#include <hip/hip_runtime.h>

#include "tmop_dev.hpp"

namespace tmop {

struct Ops {
    int epb;  // elements per workgroup
    void (*energy)(int grid, hipStream_t, const Geom &, const Tables &, const Target &,
                   const double *x, double *part);
    void (*gradient)(int grid, hipStream_t, const Geom &, const Tables &, const Target &,
                     const double *x, double *gE, double *bad);
    void (*setup64)(int grid, hipStream_t, const Geom &, const Tables &, const Target &,
                    const double *x, double *H, double *bad);
    void (*setup32)(int grid, hipStream_t, const Geom &, const Tables &, const Target &,
                    const double *x, float *H, double *bad);
    void (*apply64)(int grid, hipStream_t, const Geom &, const Tables &, const double *H,
                    const double *v, double *yE);
    void (*apply32)(int grid, hipStream_t, const Geom &, const Tables &, const float *H,
                    const double *v, float *yE);
    void (*diag64)(int grid, hipStream_t, const Geom &, const Tables &, const double *H,
                   double *dE);
    void (*diag32)(int grid, hipStream_t, const Geom &, const Tables &, const float *H,
                   double *dE);
};

// Returns false if no kernel was built for this combination.
bool find_ops(int dim, int p, int nq, Ops *out);
bool ops2(int p, int nq, Ops *out);
bool ops3_p1(int nq, Ops *out);
bool ops3_p2(int nq, Ops *out);
bool ops3_p3(int nq, Ops *out);
bool ops3_p4(int nq, Ops *out);

#define TMOP_OPS_BODY(K, SZ, P, NQ)                                                              \
    {                                                                                            \
        Ops o;                                                                                   \
        o.epb = SZ<P, NQ>::EPB;                                                                  \
        o.energy = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const Target &w, \
                      const double *x, double *part) {                                          \
            hipLaunchKernelGGL((K##_energy<P, NQ>), dim3(grid), dim3(BLOCK), 0, s, g, t, w, x,  \
                               part);                                                           \
        };                                                                                       \
        o.gradient = [](int grid, hipStream_t s, const Geom &g, const Tables &t,                \
                        const Target &w, const double *x, double *gE, double *bad) {            \
            hipLaunchKernelGGL((K##_gradient<P, NQ>), dim3(grid), dim3(BLOCK), 0, s, g, t, w,   \
                               x, gE, bad);                                                     \
        };                                                                                       \
        o.setup64 = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const Target &w, \
                       const double *x, double *H, double *bad) {                                \
            hipLaunchKernelGGL((K##_setup<P, NQ, double>), dim3(grid), dim3(BLOCK), 0, s, g, t, \
                               w, x, H, bad);                                                   \
        };                                                                                       \
        o.setup32 = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const Target &w, \
                       const double *x, float *H, double *bad) {                                 \
            hipLaunchKernelGGL((K##_setup<P, NQ, float>), dim3(grid), dim3(BLOCK), 0, s, g, t,  \
                               w, x, H, bad);                                                   \
        };                                                                                       \
        o.apply64 = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const double *H, \
                       const double *v, double *yE) {                                            \
            hipLaunchKernelGGL((K##_apply<P, NQ, double, double>), dim3(grid), dim3(BLOCK), 0,  \
                               s, g, t, H, v, yE);                                              \
        };                                                                                       \
        o.apply32 = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const float *H,  \
                       const double *v, float *yE) {                                             \
            hipLaunchKernelGGL((K##_apply<P, NQ, float, float>), dim3(grid), dim3(BLOCK), 0, s, \
                               g, t, H, v, yE);                                                 \
        };                                                                                       \
        o.diag64 = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const double *H,  \
                      double *dE) {                                                              \
            hipLaunchKernelGGL((K##_diag<P, NQ, double>), dim3(grid), dim3(BLOCK), 0, s, g, t,  \
                               H, dE);                                                          \
        };                                                                                       \
        o.diag32 = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const float *H,   \
                      double *dE) {                                                              \
            hipLaunchKernelGGL((K##_diag<P, NQ, float>), dim3(grid), dim3(BLOCK), 0, s, g, t,   \
                               H, dE);                                                          \
        };                                                                                       \
        *out = o;                                                                                \
        return true;                                                                             \
    }

}  // namespace tmop
