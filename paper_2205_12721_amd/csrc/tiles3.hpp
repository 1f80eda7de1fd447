// Hessian-action launchers of the hex kernels for every tile shape of a
// class (elements per workgroup: half, base, double), filled into the launch
// tables; shapes that do not exist for a class (tile_ok3) are never
// instantiated.
#pragma once
#include "kernels3d.hpp"
#include "ops.hpp"

namespace tmop {

template <int P, int NQ, int T2, int IDX>
inline void fill_tile3(Ops &o)
{
    if constexpr (tile_ok3<P, NQ, T2>()) {
        o.epb_t[IDX] = S3<P, NQ, T2>::EPB;
        o.apply64_t[IDX] = [](int grid, hipStream_t s, const Geom &g, const Tables &t,
                              const double *H, const double *v, double *yE) {
            hipLaunchKernelGGL((k3_apply<P, NQ, double, double, false, T2>), dim3(grid),
                               dim3(BLOCK), 0, s, g, t, H, v, yE);
        };
        o.apply32_t[IDX] = [](int grid, hipStream_t s, const Geom &g, const Tables &t,
                              const float *H, const double *v, float *yE) {
            hipLaunchKernelGGL((k3_apply<P, NQ, float, float, false, T2>), dim3(grid),
                               dim3(BLOCK), 0, s, g, t, H, v, yE);
        };
        o.applyc64_t[IDX] = [](int grid, hipStream_t s, const Geom &g, const Tables &t,
                               const Target &w, const double *Q, const double *v, double *yE) {
            hipLaunchKernelGGL((k3_applyc<P, NQ, double, double, false, T2>), dim3(grid),
                               dim3(BLOCK), 0, s, g, t, w, Q, v, yE);
        };
        o.applyc32_t[IDX] = [](int grid, hipStream_t s, const Geom &g, const Tables &t,
                               const Target &w, const float *Q, const double *v, float *yE) {
            hipLaunchKernelGGL((k3_applyc<P, NQ, float, float, false, T2>), dim3(grid),
                               dim3(BLOCK), 0, s, g, t, w, Q, v, yE);
        };
    } else {
        o.epb_t[IDX] = 0;
        o.apply64_t[IDX] = nullptr;
        o.apply32_t[IDX] = nullptr;
        o.applyc64_t[IDX] = nullptr;
        o.applyc32_t[IDX] = nullptr;
    }
}

// Matrix-core forward sweeps (forward3_mfma) where the class has them.
template <int P, int NQ>
inline void fill_mfma3(Ops &o)
{
    if constexpr (3 * NQ <= 16) {
        o.energyM = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const Target &w,
                       const double *x, double *part) {
            hipLaunchKernelGGL((k3_energy<P, NQ, false, true>), dim3(grid), dim3(BLOCK), 0, s, g,
                               t, w, x, part);
        };
        o.gradientM = [](int grid, hipStream_t s, const Geom &g, const Tables &t,
                         const Target &w, const double *x, double *gE, double *bad) {
            hipLaunchKernelGGL((k3_gradient<P, NQ, false, false, true>), dim3(grid), dim3(BLOCK),
                               0, s, g, t, w, x, gE, bad);
        };
        o.gradientEM = [](int grid, hipStream_t s, const Geom &g, const Tables &t,
                          const Target &w, const double *x, double *gE, double *part) {
            hipLaunchKernelGGL((k3_gradient<P, NQ, false, true, true>), dim3(grid), dim3(BLOCK),
                               0, s, g, t, w, x, gE, part);
        };
        o.setupM64 = [](int grid, hipStream_t s, const Geom &g, const Tables &t,
                        const Target &w, const double *x, double *H, double *bad) {
            hipLaunchKernelGGL((k3_setup<P, NQ, double, true>), dim3(grid), dim3(BLOCK), 0, s, g,
                               t, w, x, H, bad);
        };
        o.setupcM64 = [](int grid, hipStream_t s, const Geom &g, const Tables &t,
                         const Target &w, const double *x, double *Q, double *bad) {
            hipLaunchKernelGGL((k3_setupc<P, NQ, double, true>), dim3(grid), dim3(BLOCK), 0, s,
                               g, t, w, x, Q, bad);
        };
    } else {
        o.energyM = nullptr;
        o.gradientM = nullptr;
        o.gradientEM = nullptr;
        o.setupM64 = nullptr;
        o.setupcM64 = nullptr;
    }
}

// Setup with the element diagonal (b3_setupd, b3_setupcd) where the class's
// points fit one pass of the workgroup.
template <int P, int NQ>
inline void fill_setupd3(Ops &o)
{
    if constexpr (S3<P, NQ>::EPB * S3<P, NQ>::NQ3 <= BLOCK) {
        o.setupd64 = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const Target &w,
                        const double *x, double *H, double *dE, double *bad) {
            if (g.lim != 0.0)
                hipLaunchKernelGGL((k3_setupd<P, NQ, double, true>), dim3(grid), dim3(BLOCK), 0, s,
                                   g, t, w, x, H, dE, bad);
            else
                hipLaunchKernelGGL((k3_setupd<P, NQ, double, false>), dim3(grid), dim3(BLOCK), 0, s,
                                   g, t, w, x, H, dE, bad);
        };
        o.setupd32 = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const Target &w,
                        const double *x, float *H, double *dE, double *bad) {
            if (g.lim != 0.0)
                hipLaunchKernelGGL((k3_setupd<P, NQ, float, true>), dim3(grid), dim3(BLOCK), 0, s,
                                   g, t, w, x, H, dE, bad);
            else
                hipLaunchKernelGGL((k3_setupd<P, NQ, float, false>), dim3(grid), dim3(BLOCK), 0, s,
                                   g, t, w, x, H, dE, bad);
        };
        o.setupcd64 = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const Target &w,
                         const double *x, double *Q, double *dE, double *bad) {
            if (g.lim != 0.0)
                hipLaunchKernelGGL((k3_setupcd<P, NQ, double, true>), dim3(grid), dim3(BLOCK), 0, s,
                                   g, t, w, x, Q, dE, bad);
            else
                hipLaunchKernelGGL((k3_setupcd<P, NQ, double, false>), dim3(grid), dim3(BLOCK), 0,
                                   s, g, t, w, x, Q, dE, bad);
        };
        o.setupcd32 = [](int grid, hipStream_t s, const Geom &g, const Tables &t, const Target &w,
                         const double *x, float *Q, double *dE, double *bad) {
            if (g.lim != 0.0)
                hipLaunchKernelGGL((k3_setupcd<P, NQ, float, true>), dim3(grid), dim3(BLOCK), 0, s,
                                   g, t, w, x, Q, dE, bad);
            else
                hipLaunchKernelGGL((k3_setupcd<P, NQ, float, false>), dim3(grid), dim3(BLOCK), 0, s,
                                   g, t, w, x, Q, dE, bad);
        };
    } else {
        o.setupd64 = nullptr;
        o.setupd32 = nullptr;
        o.setupcd64 = nullptr;
        o.setupcd32 = nullptr;
    }
}

template <int P, int NQ>
inline void fill_tiles_k3(Ops &o)
{
    fill_tile3<P, NQ, 1, 0>(o);
    fill_tile3<P, NQ, 2, 1>(o);
    fill_tile3<P, NQ, 4, 2>(o);
    fill_mfma3<P, NQ>(o);
    fill_setupd3<P, NQ>(o);
}

template <int P, int NQ, int T2, int IDX>
inline void fill_btile3(BOps &o)
{
    if constexpr (tile_ok3<P, NQ, T2>()) {
        o.epb_t[IDX] = S3<P, NQ, T2>::EPB;
        o.apply_t[0][0][IDX] = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,
                                  const SlotDev *sl, const int *gt, int vin, double *) {
            hipLaunchKernelGGL((kb3_apply<P, NQ, double, double, false, T2>), dim3(grid), dim3(BLOCK),
                               0, s, t, tl, sl, gt, vin);
        };
        o.apply_t[0][1][IDX] = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,
                                  const SlotDev *sl, const int *gt, int vin, double *) {
            hipLaunchKernelGGL((kb3_apply<P, NQ, float, float, false, T2>), dim3(grid), dim3(BLOCK), 0,
                               s, t, tl, sl, gt, vin);
        };
        o.apply_t[1][0][IDX] = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,
                                  const SlotDev *sl, const int *gt, int vin, double *) {
            hipLaunchKernelGGL((kb3_applyc<P, NQ, double, double, false, T2>), dim3(grid), dim3(BLOCK),
                               0, s, t, tl, sl, gt, vin);
        };
        o.apply_t[1][1][IDX] = [](int grid, hipStream_t s, const Tables &t, const Tile *tl,
                                  const SlotDev *sl, const int *gt, int vin, double *) {
            hipLaunchKernelGGL((kb3_applyc<P, NQ, float, float, false, T2>), dim3(grid), dim3(BLOCK), 0,
                               s, t, tl, sl, gt, vin);
        };
    } else {
        o.epb_t[IDX] = 0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) o.apply_t[a][b][IDX] = nullptr;
    }
}

template <int P, int NQ>
inline void fill_tiles_kb3(BOps &o)
{
    fill_btile3<P, NQ, 1, 0>(o);
    fill_btile3<P, NQ, 2, 1>(o);
    fill_btile3<P, NQ, 4, 2>(o);
}

}  // namespace tmop
