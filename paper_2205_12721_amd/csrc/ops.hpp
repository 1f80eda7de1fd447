// Launch table: one entry per (dim, p, nq) with host launchers for every
// element kernel.  The element kernels are instantiated in k2.hip and
// k3_p*.hip; the table is filled by find_ops().
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/tmop.h"
#include "tmop_dev.hpp"

namespace tmop {

struct Ops {
    int epb;  // elements per workgroup
    void (*energy)(int grid, hipStream_t, const Geom &, const Tables &, const Target &,
                   const double *x, double *part);
    void (*gradient)(int grid, hipStream_t, const Geom &, const Tables &, const Target &,
                     const double *x, double *gE, double *bad);
    // gradient E-vector plus the energy partials (three planes of grid
    // entries in part, as energy writes them)
    decltype(gradient) gradientE;
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
    // compact quadrature data (T and four weighted metric coefficients)
    void (*setupc64)(int grid, hipStream_t, const Geom &, const Tables &, const Target &,
                     const double *x, double *Q, double *bad);
    void (*setupc32)(int grid, hipStream_t, const Geom &, const Tables &, const Target &,
                     const double *x, float *Q, double *bad);
    void (*applyc64)(int grid, hipStream_t, const Geom &, const Tables &, const Target &,
                     const double *Q, const double *v, double *yE);
    void (*applyc32)(int grid, hipStream_t, const Geom &, const Tables &, const Target &,
                     const float *Q, const double *v, float *yE);
    void (*diagc64)(int grid, hipStream_t, const Geom &, const Tables &, const Target &,
                    const double *Q, double *dE);
    void (*diagc32)(int grid, hipStream_t, const Geom &, const Tables &, const Target &,
                    const float *Q, double *dE);
    // Hessian action (without the limiting term) per tile shape t: 0 half, 1
    // base, 2 double the elements per workgroup; epb_t[t] = 0 where the shape
    // does not exist for this class.  Index 1 is the launcher set above.
    int epb_t[3];
    decltype(apply64) apply64_t[3];
    decltype(apply32) apply32_t[3];
    decltype(applyc64) applyc64_t[3];
    decltype(applyc32) applyc32_t[3];
    // forward sweeps on the matrix cores (tmop_set_sweeps): energy, gradient
    // and the FP64 setups without the limiting term; null where the class
    // has no such form (quads, n_q > 5)
    decltype(energy) energyM;
    decltype(gradient) gradientM, gradientEM;
    decltype(setup64) setupM64;
    decltype(setupc64) setupcM64;
    // tensor setup plus the element part of the Hessian diagonal (into dE) in
    // one pass; null where the class has no such kernel (quads, more than one
    // pass of points per workgroup)
    void (*setupd64)(int grid, hipStream_t, const Geom &, const Tables &, const Target &,
                     const double *x, double *H, double *dE, double *bad);
    void (*setupd32)(int grid, hipStream_t, const Geom &, const Tables &, const Target &,
                     const double *x, float *H, double *dE, double *bad);
    decltype(setupd64) setupcd64;  // the same for compact storage
    decltype(setupd32) setupcd32;
};

// Batched launchers (grid = number of tiles); every batched element kernel
// takes the same arguments: 1D tables of its class, tile list, slot table,
// per-slot gate, input vector id, partial-sum output.
typedef void (*BLaunch)(int grid, hipStream_t, const Tables &, const Tile *, const SlotDev *,
                        const int *gate, int vin, double *part);

struct BOps {
    int epb;
    BLaunch energy, gradient;
    // gradient plus the energy partials of energy (same three planes)
    BLaunch gradientE, gradientEL;
    BLaunch setup[2][2];  // [storage tensor/compact][fp64/fp32]
    BLaunch apply[2][2];
    BLaunch diag[2][2];
    // with the limiting term (slots that carry reference nodes x0; the
    // quadrature data and its setup are the same)
    BLaunch energyL, gradientL;
    BLaunch applyL[2][2];
    BLaunch diagL[2][2];
    // Hessian action per tile shape (as in Ops); apply_t[..][..][1] == apply
    int epb_t[3];
    BLaunch apply_t[2][2][3];
};

// Base tile shape only (quads).
template <int P, int NQ>
inline void fill_tiles_k2(Ops &o)
{
    for (int t = 0; t < 3; ++t) {
        o.epb_t[t] = t == 1 ? o.epb : 0;
        o.apply64_t[t] = t == 1 ? o.apply64 : nullptr;
        o.apply32_t[t] = t == 1 ? o.apply32 : nullptr;
        o.applyc64_t[t] = t == 1 ? o.applyc64 : nullptr;
        o.applyc32_t[t] = t == 1 ? o.applyc32 : nullptr;
    }
    o.energyM = nullptr;
    o.gradientM = nullptr;
    o.gradientEM = nullptr;
    o.setupM64 = nullptr;
    o.setupcM64 = nullptr;
    o.setupd64 = nullptr;
    o.setupd32 = nullptr;
    o.setupcd64 = nullptr;
    o.setupcd32 = nullptr;
}

template <int P, int NQ>
inline void fill_tiles_kb2(BOps &o)
{
    for (int t = 0; t < 3; ++t) {
        o.epb_t[t] = t == 1 ? o.epb : 0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) o.apply_t[a][b][t] = t == 1 ? o.apply[a][b] : nullptr;
    }
}

// Host-side 1D tables (GLL basis at Gauss-Legendre points) and constant
// target of a (p, n_q) / params pair; defined in capi.hip.
int internal_tables(int p, int nq, Tables *tb, int rule = 0);
int internal_target(const tmop_params *prm, int dim, Target *tg);

// Tile shapes of the Hessian action chosen by the autotuner, per class
// (process-wide; tmop_autotune / tmop_pool_autotune record them): the shape
// index, or -1 when the class was not tuned.  Defined in capi.hip.
int tuned_tile(int dim, int p, int nq, int storage, int precision);
void record_tile(int dim, int p, int nq, int storage, int precision, int t);

// Returns false if no kernel was built for this combination.
bool find_ops(int dim, int p, int nq, Ops *out);
bool find_bops(int dim, int p, int nq, BOps *out);
bool bops2(int p, int nq, BOps *out);
bool bops3_p1(int nq, BOps *out);
bool bops3_p2(int nq, BOps *out);
bool bops3_p3(int nq, BOps *out);
bool bops3_p4(int nq, BOps *out);

#define TMOP_BOPS_BODY(K, SZ, P, NQ)                                                           \
    {                                                                                          \
        BOps o;                                                                                \
        o.epb = SZ<P, NQ>::EPB;                                                                \
        o.energy = [](int grid, hipStream_t s, const Tables &t, const Tile *tl, const SlotDev *sl, \
                      const int *gt, int vin, double *part) {                                  \
            hipLaunchKernelGGL((K##_energy<P, NQ>), dim3(grid), dim3(BLOCK), 0, s, t, tl, sl, gt, \
                               vin, part);                                                     \
        };                                                                                     \
        o.gradient = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,               \
                        const SlotDev *sl, const int *gt, int vin, double *part) {             \
            hipLaunchKernelGGL((K##_gradient<P, NQ>), dim3(grid), dim3(BLOCK), 0, s, t, tl, sl, \
                               gt, vin, part);                                                 \
        };                                                                                     \
        o.gradientE = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,              \
                         const SlotDev *sl, const int *gt, int vin, double *part) {            \
            hipLaunchKernelGGL((K##_gradient<P, NQ, false, true>), dim3(grid), dim3(BLOCK), 0, s, t, tl, \
                               sl, gt, vin, part);                                             \
        };                                                                                     \
        o.gradientEL = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,             \
                          const SlotDev *sl, const int *gt, int vin, double *part) {           \
            hipLaunchKernelGGL((K##_gradient<P, NQ, true, true>), dim3(grid), dim3(BLOCK), 0, s, t, tl, \
                               sl, gt, vin, part);                                             \
        };                                                                                     \
        o.energyL = [](int grid, hipStream_t s, const Tables &t, const Tile *tl, const SlotDev *sl, \
                       const int *gt, int vin, double *part) {                                 \
            hipLaunchKernelGGL((K##_energy<P, NQ, true>), dim3(grid), dim3(BLOCK), 0, s, t, tl, sl, \
                               gt, vin, part);                                                 \
        };                                                                                     \
        o.gradientL = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,              \
                         const SlotDev *sl, const int *gt, int vin, double *part) {            \
            hipLaunchKernelGGL((K##_gradient<P, NQ, true>), dim3(grid), dim3(BLOCK), 0, s, t, tl, \
                               sl, gt, vin, part);                                             \
        };                                                                                     \
        TMOP_BOPS_PREC(K, P, NQ, 0, double, double)                                            \
        TMOP_BOPS_PREC(K, P, NQ, 1, float, float)                                              \
        fill_tiles_##K<P, NQ>(o);                                                              \
        *out = o;                                                                              \
        return true;                                                                           \
    }

#define TMOP_BOPS_PREC(K, P, NQ, IDX, TT, CT)                                                  \
    o.setup[0][IDX] = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,             \
                         const SlotDev *sl, const int *gt, int vin, double *part) {            \
        hipLaunchKernelGGL((K##_setup<P, NQ, TT>), dim3(grid), dim3(BLOCK), 0, s, t, tl, sl, gt, \
                           vin, part);                                                         \
    };                                                                                         \
    o.setup[1][IDX] = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,             \
                         const SlotDev *sl, const int *gt, int vin, double *part) {            \
        hipLaunchKernelGGL((K##_setupc<P, NQ, TT>), dim3(grid), dim3(BLOCK), 0, s, t, tl, sl,   \
                           gt, vin, part);                                                     \
    };                                                                                         \
    o.apply[0][IDX] = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,             \
                         const SlotDev *sl, const int *gt, int vin, double *) {                \
        hipLaunchKernelGGL((K##_apply<P, NQ, TT, CT>), dim3(grid), dim3(BLOCK), 0, s, t, tl, sl, \
                           gt, vin);                                                           \
    };                                                                                         \
    o.apply[1][IDX] = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,             \
                         const SlotDev *sl, const int *gt, int vin, double *) {                \
        hipLaunchKernelGGL((K##_applyc<P, NQ, TT, CT>), dim3(grid), dim3(BLOCK), 0, s, t, tl,   \
                           sl, gt, vin);                                                       \
    };                                                                                         \
    o.diag[0][IDX] = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,              \
                        const SlotDev *sl, const int *gt, int, double *) {                     \
        hipLaunchKernelGGL((K##_diag<P, NQ, TT>), dim3(grid), dim3(BLOCK), 0, s, t, tl, sl, gt); \
    };                                                                                         \
    o.diag[1][IDX] = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,              \
                        const SlotDev *sl, const int *gt, int, double *) {                     \
        hipLaunchKernelGGL((K##_diagc<P, NQ, TT>), dim3(grid), dim3(BLOCK), 0, s, t, tl, sl, gt); \
    };                                                                                         \
    o.applyL[0][IDX] = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,            \
                          const SlotDev *sl, const int *gt, int vin, double *) {               \
        hipLaunchKernelGGL((K##_apply<P, NQ, TT, CT, true>), dim3(grid), dim3(BLOCK), 0, s, t, tl, \
                           sl, gt, vin);                                                       \
    };                                                                                         \
    o.applyL[1][IDX] = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,            \
                          const SlotDev *sl, const int *gt, int vin, double *) {               \
        hipLaunchKernelGGL((K##_applyc<P, NQ, TT, CT, true>), dim3(grid), dim3(BLOCK), 0, s, t, \
                           tl, sl, gt, vin);                                                   \
    };                                                                                         \
    o.diagL[0][IDX] = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,             \
                         const SlotDev *sl, const int *gt, int, double *) {                    \
        hipLaunchKernelGGL((K##_diag<P, NQ, TT, true>), dim3(grid), dim3(BLOCK), 0, s, t, tl, sl, \
                           gt);                                                                \
    };                                                                                         \
    o.diagL[1][IDX] = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,             \
                         const SlotDev *sl, const int *gt, int, double *) {                    \
        hipLaunchKernelGGL((K##_diagc<P, NQ, TT, true>), dim3(grid), dim3(BLOCK), 0, s, t, tl,  \
                           sl, gt);                                                            \
    };
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
            if (g.lim != 0.0) {                                                                   \
                hipLaunchKernelGGL((K##_energy<P, NQ, true>), dim3(grid), dim3(BLOCK), 0, s, g, t, w, x, part); \
            } else {                                                                         \
                hipLaunchKernelGGL((K##_energy<P, NQ, false>), dim3(grid), dim3(BLOCK), 0, s, g, t, w, x, part); \
            }                                                                      \
        };                                                                                       \
        o.gradient = [](int grid, hipStream_t s, const Geom &g, const Tables &t,                \
                        const Target &w, const double *x, double *gE, double *bad) {            \
            if (g.lim != 0.0) {                                                                   \
                hipLaunchKernelGGL((K##_gradient<P, NQ, true>), dim3(grid), dim3(BLOCK), 0, s, g, t, w, x, gE, bad); \
            } else {                                                                         \
                hipLaunchKernelGGL((K##_gradient<P, NQ, false>), dim3(grid), dim3(BLOCK), 0, s, g, t, w, x, gE, bad); \
            }                                                                      \
        };                                                                                       \
        o.gradientE = [](int grid, hipStream_t s, const Geom &g, const Tables &t,               \
                         const Target &w, const double *x, double *gE, double *part) {          \
            if (g.lim != 0.0) {                                                                   \
                hipLaunchKernelGGL((K##_gradient<P, NQ, true, true>), dim3(grid), dim3(BLOCK), 0, s, g, t, w, x, gE, part); \
            } else {                                                                         \
                hipLaunchKernelGGL((K##_gradient<P, NQ, false, true>), dim3(grid), dim3(BLOCK), 0, s, g, t, w, x, gE, part); \
            }                                                                      \
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
            if (g.lim != 0.0) {                                                                   \
                hipLaunchKernelGGL((K##_apply<P, NQ, double, double, true>), dim3(grid), dim3(BLOCK), 0, s, g, t, H, v, yE); \
            } else {                                                                         \
                hipLaunchKernelGGL((K##_apply<P, NQ, double, double, false>), dim3(grid), dim3(BLOCK), 0, s, g, t, H, v, yE); \
            }                                                                      \
        };                                                                                       \
        o.apply32 = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const float *H,  \
                       const double *v, float *yE) {                                             \
            if (g.lim != 0.0) {                                                                   \
                hipLaunchKernelGGL((K##_apply<P, NQ, float, float, true>), dim3(grid), dim3(BLOCK), 0, s, g, t, H, v, yE); \
            } else {                                                                         \
                hipLaunchKernelGGL((K##_apply<P, NQ, float, float, false>), dim3(grid), dim3(BLOCK), 0, s, g, t, H, v, yE); \
            }                                                                      \
        };                                                                                       \
        o.diag64 = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const double *H,  \
                      double *dE) {                                                              \
            if (g.lim != 0.0) {                                                                   \
                hipLaunchKernelGGL((K##_diag<P, NQ, double, true>), dim3(grid), dim3(BLOCK), 0, s, g, t, H, dE); \
            } else {                                                                         \
                hipLaunchKernelGGL((K##_diag<P, NQ, double, false>), dim3(grid), dim3(BLOCK), 0, s, g, t, H, dE); \
            }                                                                      \
        };                                                                                       \
        o.diag32 = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const float *H,   \
                      double *dE) {                                                              \
            if (g.lim != 0.0) {                                                                   \
                hipLaunchKernelGGL((K##_diag<P, NQ, float, true>), dim3(grid), dim3(BLOCK), 0, s, g, t, H, dE); \
            } else {                                                                         \
                hipLaunchKernelGGL((K##_diag<P, NQ, float, false>), dim3(grid), dim3(BLOCK), 0, s, g, t, H, dE); \
            }                                                                      \
        };                                                                                       \
        o.setupc64 = [](int grid, hipStream_t s, const Geom &g, const Tables &t,                \
                        const Target &w, const double *x, double *Q, double *bad) {             \
            hipLaunchKernelGGL((K##_setupc<P, NQ, double>), dim3(grid), dim3(BLOCK), 0, s, g, t,\
                               w, x, Q, bad);                                                   \
        };                                                                                       \
        o.setupc32 = [](int grid, hipStream_t s, const Geom &g, const Tables &t,                \
                        const Target &w, const double *x, float *Q, double *bad) {              \
            hipLaunchKernelGGL((K##_setupc<P, NQ, float>), dim3(grid), dim3(BLOCK), 0, s, g, t, \
                               w, x, Q, bad);                                                   \
        };                                                                                       \
        o.applyc64 = [](int grid, hipStream_t s, const Geom &g, const Tables &t,                \
                        const Target &w, const double *Q, const double *v, double *yE) {        \
            if (g.lim != 0.0) {                                                                   \
                hipLaunchKernelGGL((K##_applyc<P, NQ, double, double, true>), dim3(grid), dim3(BLOCK), 0, s, g, t, w, Q, v, yE); \
            } else {                                                                         \
                hipLaunchKernelGGL((K##_applyc<P, NQ, double, double, false>), dim3(grid), dim3(BLOCK), 0, s, g, t, w, Q, v, yE); \
            }                                                                      \
        };                                                                                       \
        o.applyc32 = [](int grid, hipStream_t s, const Geom &g, const Tables &t,                \
                        const Target &w, const float *Q, const double *v, float *yE) {          \
            if (g.lim != 0.0) {                                                                   \
                hipLaunchKernelGGL((K##_applyc<P, NQ, float, float, true>), dim3(grid), dim3(BLOCK), 0, s, g, t, w, Q, v, yE); \
            } else {                                                                         \
                hipLaunchKernelGGL((K##_applyc<P, NQ, float, float, false>), dim3(grid), dim3(BLOCK), 0, s, g, t, w, Q, v, yE); \
            }                                                                      \
        };                                                                                       \
        o.diagc64 = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const Target &w,\
                       const double *Q, double *dE) {                                            \
            if (g.lim != 0.0) {                                                                   \
                hipLaunchKernelGGL((K##_diagc<P, NQ, double, true>), dim3(grid), dim3(BLOCK), 0, s, g, t, w, Q, dE); \
            } else {                                                                         \
                hipLaunchKernelGGL((K##_diagc<P, NQ, double, false>), dim3(grid), dim3(BLOCK), 0, s, g, t, w, Q, dE); \
            }                                                                      \
        };                                                                                       \
        o.diagc32 = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const Target &w,\
                       const float *Q, double *dE) {                                             \
            if (g.lim != 0.0) {                                                                   \
                hipLaunchKernelGGL((K##_diagc<P, NQ, float, true>), dim3(grid), dim3(BLOCK), 0, s, g, t, w, Q, dE); \
            } else {                                                                         \
                hipLaunchKernelGGL((K##_diagc<P, NQ, float, false>), dim3(grid), dim3(BLOCK), 0, s, g, t, w, Q, dE); \
            }                                                                      \
        };                                                                                       \
        fill_tiles_##K<P, NQ>(o);                                                                \
        *out = o;                                                                                \
        return true;                                                                             \
    }

}  // namespace tmop
