// Host launchers of the node-level kernels (vec.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tmop_dev.hpp"

namespace tmop {

// Device-resident scalar state of one MINRES solve.
struct MinresState {
    double tmp;
    double beta1, beta, oldb, alpha, dbar, eps, oldeps, phibar, phi, cs, sn, gamma, delta, rtol;
    int its;
    int stop;  // last iteration index that runs; INT_MAX while running
    int indefinite_precond;
    int pad;
};

// Scalars of one MINRES update, kept when the Lanczos vectors stay resident
// and the solution is formed once after the loop: the update m takes
// w_m = (v_m - oldeps w_{m-2} - delta w_{m-1}) ig and x += phi w_m, with
// v_m = sv z_m (z_m the unscaled preconditioned Lanczos vector).
struct MrHist {
    double ig, oldeps, delta, phi, sv;
    double pad[3];
};
// Most updates one combination can take (one lane per coefficient).
constexpr int MR_MAX_BASIS = 256;

void launch_gather(const Geom &g, const int32_t *csr_ptr, const int32_t *csr_ent, const void *eV,
                   bool fp32, double *out, int fix_mode, const double *src, hipStream_t s);
void launch_reduce3(const double *part, int nb, double *out, hipStream_t s);
void launch_reduce_sum(const double *part, int nb, double *out, hipStream_t s);
int reduce_blocks(long n);
void launch_dot(long n, const double *a, const double *b, double *part, double *out,
                hipStream_t s);
void launch_absmax(long n, const double *a, double *part, double *out, hipStream_t s);
void launch_step(long n, const double *x, const double *dx, double alpha, double *xt,
                 hipStream_t s);
void launch_jacobi(long n, const double *d, const double *dmax, double *minv, hipStream_t s);

void mr_init(long n, const double *b, const double *minv, double *r1, double *r2, double *y,
             double *v, double *x, double *w, double *w1, double *w2, double *part,
             MinresState *st, double rtol, hipStream_t s);
void mr_gather_upd(const Geom &g, const int32_t *csr_ptr, const int32_t *csr_ent, const void *eV,
                   bool fp32, int j, const MinresState *sin, MinresState *sout,
                   const double *p1prev, const double *p2prev, const double *zp, const double *zc,
                   const double *w1, const double *w2, double *wout, double *x, double *r1hv,
                   double *part, MrHist *hist, hipStream_t s);
// Workgroups of mr_gather_upd, i.e. the count of its partials (nb1 below);
// at most MR_MAX_PARTIALS.
int mr_gather_grid(const Geom &g);
constexpr int MR_MAX_PARTIALS = 2048;
void mr_lanczos2(long n, int nb1, int j, const MinresState *st, const double *part1, double *hv,
                 const double *r2, const double *minv, double *z, double *part2, hipStream_t s);
void mr_finish(long n, int nb1, int jm, const MinresState *sin, MinresState *sout,
               const double *p1, const double *p2, const double *zp, const double *w1,
               const double *w2, double *wout, double *x, hipStream_t s);
void mr_combine(long n, int nb1, int jm, const MinresState *sin, MinresState *sout,
                const double *p1, const double *p2, MrHist *hist, const double *bank, long stride,
                double *x, hipStream_t s);

}  // namespace tmop
