// Node-level kernels: the transpose of the element restriction (E-vector ->
// global vector, Sec. 3 operator decomposition, G^T), deterministic
// reductions, and the vector work of Newton and of preconditioned MINRES.
#include <hip/hip_runtime.h>

#include "tmop_dev.hpp"
#include "gather.hpp"
#include "vec.hpp"

namespace tmop {

constexpr int VBLOCK = 256;

// out = G^T eV; fixed DoFs get 0 (fix_mode 0), 1 (fix_mode 1) or src (fix_mode 2).
template <int DIM, typename ET>
__global__ __launch_bounds__(VBLOCK) void k_gather(Geom g, const int32_t *__restrict__ ptr,
                                                   const int32_t *__restrict__ ent,
                                                   const ET *__restrict__ eV,
                                                   double *__restrict__ out, int fix_mode,
                                                   const double *__restrict__ src)
{
    // one lane per node, all components
    for (int node = xcd_block(blockIdx.x, gridDim.x) * VBLOCK + threadIdx.x; node < g.nx;
         node += gridDim.x * VBLOCK) {
        double a[DIM];
        bool fixed[DIM];
        gather_node<DIM, ET>(g, ptr, ent, eV, node, a, fixed);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const size_t idx = (size_t)c * g.nx + node;
            out[idx] = fixed[c] ? (fix_mode == 0 ? 0.0 : (fix_mode == 1 ? 1.0 : src[idx])) : a[c];
        }
    }
}

static int vgrid(long n, int cap = 2048)
{
    long b = (n + VBLOCK - 1) / VBLOCK;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

void launch_gather(const Geom &g, const int32_t *csr_ptr, const int32_t *csr_ent, const void *eV,
                   bool fp32, double *out, int fix_mode, const double *src, hipStream_t s)
{
    const int grid = vgrid((long)g.nx, 8192);
#define TMOP_G(D, T)                                                                          \
    hipLaunchKernelGGL((k_gather<D, T>), dim3(grid), dim3(VBLOCK), 0, s, g, csr_ptr, csr_ent, \
                       (const T *)eV, out, fix_mode, src);
    if (g.dim == 3) {
        if (fp32) {
            TMOP_G(3, float)
        } else {
            TMOP_G(3, double)
        }
    } else {
        if (fp32) {
            TMOP_G(2, float)
        } else {
            TMOP_G(2, double)
        }
    }
#undef TMOP_G
}

// ------------------------------------------------------------------------
// Reductions
// ------------------------------------------------------------------------

// Final reduce of the element kernels' partials: out[0] = sum part[0:nb],
// out[1] = min part[nb:2nb], out[2] = sum part[2nb:3nb].
__global__ __launch_bounds__(VBLOCK) void k_reduce3(const double *__restrict__ part, int nb,
                                                    double *__restrict__ out)
{
    __shared__ double red[VBLOCK / 64];
    double s = 0.0, m = 1.0e300, b = 0.0;
    // loads in batches of RU strides, each lane's sums in the order of k
    constexpr int RU = 8;
    int k = threadIdx.x;
    for (; k + (RU - 1) * VBLOCK < nb; k += RU * VBLOCK) {
        double a[RU], c[RU], d[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            a[u] = part[k + u * VBLOCK];
            c[u] = part[nb + k + u * VBLOCK];
            d[u] = part[2 * nb + k + u * VBLOCK];
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            s += a[u];
            m = fmin(m, c[u]);
            b += d[u];
        }
    }
    for (; k < nb; k += VBLOCK) {
        s += part[k];
        m = fmin(m, part[nb + k]);
        b += part[2 * nb + k];
    }
    s = block_sum(s, red);
    m = block_min(m, red);
    b = block_sum(b, red);
    if (threadIdx.x == 0) {
        out[0] = s;
        out[1] = m;
        out[2] = b;
    }
}

__global__ __launch_bounds__(VBLOCK) void k_reduce_sum(const double *__restrict__ part, int nb,
                                                       double *__restrict__ out)
{
    __shared__ double red[VBLOCK / 64];
    double s = 0.0;
    constexpr int RU = 8;  // batched loads, sums in the order of k
    int k = threadIdx.x;
    for (; k + (RU - 1) * VBLOCK < nb; k += RU * VBLOCK) {
        double a[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) a[u] = part[k + u * VBLOCK];
#pragma unroll
        for (int u = 0; u < RU; ++u) s += a[u];
    }
    for (; k < nb; k += VBLOCK) s += part[k];
    s = block_sum(s, red);
    if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(VBLOCK) void k_reduce_max(const double *__restrict__ part, int nb,
                                                       double *__restrict__ out)
{
    __shared__ double red[VBLOCK / 64];
    double s = 0.0;
    for (int k = threadIdx.x; k < nb; k += VBLOCK) s = fmax(s, part[k]);
    // max via -min(-x)
    s = -block_min(-s, red);
    if (threadIdx.x == 0) *out = s;
}

void launch_reduce3(const double *part, int nb, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce3, dim3(1), dim3(VBLOCK), 0, s, part, nb, out);
}

void launch_reduce_sum(const double *part, int nb, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(VBLOCK), 0, s, part, nb, out);
}

// partial dot products, fixed grid of nb blocks
__global__ __launch_bounds__(VBLOCK) void k_dot_part(long n, const double *__restrict__ a,
                                                     const double *__restrict__ b,
                                                     double *__restrict__ part)
{
    __shared__ double red[VBLOCK / 64];
    double s = 0.0;
    for (long i = blockIdx.x * (long)VBLOCK + threadIdx.x; i < n; i += (long)gridDim.x * VBLOCK)
        s += a[i] * b[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(VBLOCK) void k_absmax_part(long n, const double *__restrict__ a,
                                                        double *__restrict__ part)
{
    __shared__ double red[VBLOCK / 64];
    double s = 0.0;
    for (long i = blockIdx.x * (long)VBLOCK + threadIdx.x; i < n; i += (long)gridDim.x * VBLOCK)
        s = fmax(s, fabs(a[i]));
    s = -block_min(-s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

int reduce_blocks(long n) { return vgrid(n, 1024); }

void launch_dot(long n, const double *a, const double *b, double *part, double *out,
                hipStream_t s)
{
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(VBLOCK), 0, s, n, a, b, part);
    hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(VBLOCK), 0, s, part, nb, out);
}

void launch_absmax(long n, const double *a, double *part, double *out, hipStream_t s)
{
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_absmax_part, dim3(nb), dim3(VBLOCK), 0, s, n, a, part);
    hipLaunchKernelGGL(k_reduce_max, dim3(1), dim3(VBLOCK), 0, s, part, nb, out);
}

// ------------------------------------------------------------------------
// Newton / line-search vector work
// ------------------------------------------------------------------------

// xt = x - alpha dx
__global__ __launch_bounds__(VBLOCK) void k_step(long n, const double *__restrict__ x,
                                                 const double *__restrict__ dx, double alpha,
                                                 double *__restrict__ xt)
{
    for (long i = blockIdx.x * (long)VBLOCK + threadIdx.x; i < n; i += (long)gridDim.x * VBLOCK)
        xt[i] = x[i] - alpha * dx[i];
}

void launch_step(long n, const double *x, const double *dx, double alpha, double *xt,
                 hipStream_t s)
{
    hipLaunchKernelGGL(k_step, dim3(vgrid(n, 8192)), dim3(VBLOCK), 0, s, n, x, dx, alpha, xt);
}

// Jacobi inverse: minv = 1 / max(|d|, floor), floor = 1e-14 max|d| (read on
// device), entries equal to exactly 1 on fixed DoFs stay 1.
__global__ __launch_bounds__(VBLOCK) void k_jacobi(long n, const double *__restrict__ d,
                                                   const double *__restrict__ dmax,
                                                   double *__restrict__ minv)
{
    const double floor = 1e-14 * (*dmax);
    for (long i = blockIdx.x * (long)VBLOCK + threadIdx.x; i < n; i += (long)gridDim.x * VBLOCK) {
        double a = fabs(d[i]);
        a = fmax(a, floor);
        minv[i] = a > 0.0 ? 1.0 / a : 1.0;
    }
}

void launch_jacobi(long n, const double *d, const double *dmax, double *minv, hipStream_t s)
{
    hipLaunchKernelGGL(k_jacobi, dim3(vgrid(n, 8192)), dim3(VBLOCK), 0, s, n, d, dmax, minv);
}

// ------------------------------------------------------------------------
// Preconditioned MINRES (Paige-Saunders), device-resident scalars.
//
// Lanczos on M^{-1} H with the three-term recurrence, Givens QR of the
// tridiagonal matrix, short-recurrence update of the solution.  Per
// iteration j, after the element kernel has produced the E-vector of H v:
//   gather_l1:  hv = G^T eV (fixed DoFs: v);  hv -= (beta/oldb) r1;  part1 = <v, hv>
//   l2:         alpha = sum part1;  hv -= (alpha/beta) r2;  z = M^{-1} hv;  part2 = <hv, z>
//   update:     beta' = sqrt(sum part2), Givens rotation, phi;
//               w' = (v - oldeps w1 - delta w2)/gamma;  x += phi w';  v = z/beta'
// The scalar recurrences run redundantly in every workgroup (same partials,
// same order, same result) so no single-lane kernels sit between the vector
// passes; the state is double-buffered (iteration j reads st[j&1], the update
// writes st[(j+1)&1], also when it skips, so the stop flag propagates).
// Kernels of iteration j return at once when j > stop (set when the residual
// estimate drops below rtol*beta1 or the Lanczos vector vanishes).
// ------------------------------------------------------------------------

// Sum of part[0..nb) in a fixed order, identical in every workgroup.
__device__ inline double sum_partials(const double *__restrict__ part, int nb, double *red)
{
    double s = 0.0;
    for (int k = threadIdx.x; k < nb; k += VBLOCK) s += part[k];
    s = block_sum(s, red);
    __shared__ double bcast;
    if (threadIdx.x == 0) bcast = s;
    __syncthreads();
    return bcast;
}

__global__ __launch_bounds__(VBLOCK) void k_mr_init(long n, const double *__restrict__ b,
                                                    const double *__restrict__ minv,
                                                    double *__restrict__ r1,
                                                    double *__restrict__ r2,
                                                    double *__restrict__ y,
                                                    double *__restrict__ part)
{
    __shared__ double red[VBLOCK / 64];
    double s = 0.0;
    for (long i = blockIdx.x * (long)VBLOCK + threadIdx.x; i < n; i += (long)gridDim.x * VBLOCK) {
        const double bi = b[i];
        const double yi = minv ? minv[i] * bi : bi;
        r1[i] = bi;
        r2[i] = bi;
        y[i] = yi;
        s += bi * yi;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// beta1 from the partials; st[0] initial state; v = y / beta1; x = w = w1 = w2 = 0.
__global__ __launch_bounds__(VBLOCK) void k_mr_start(long n, MinresState *st, double rtol,
                                                     const double *__restrict__ part, int nb,
                                                     const double *__restrict__ y,
                                                     double *__restrict__ v,
                                                     double *__restrict__ x,
                                                     double *__restrict__ w,
                                                     double *__restrict__ w1,
                                                     double *__restrict__ w2)
{
    __shared__ double red[VBLOCK / 64];
    const double bb = sum_partials(part, nb, red);
    const double b1 = sqrt(fmax(bb, 0.0));
    const double s = b1 > 0.0 ? 1.0 / b1 : 0.0;
    for (long i = blockIdx.x * (long)VBLOCK + threadIdx.x; i < n; i += (long)gridDim.x * VBLOCK) {
        v[i] = s * y[i];
        x[i] = 0.0;
        w[i] = 0.0;
        w1[i] = 0.0;
        w2[i] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        MinresState &o = st[0];
        o.tmp = bb;
        o.beta1 = b1;
        o.beta = b1;
        o.oldb = 0.0;
        o.alpha = 0.0;
        o.dbar = 0.0;
        o.eps = 0.0;
        o.oldeps = 0.0;
        o.phibar = b1;
        o.phi = 0.0;
        o.cs = -1.0;
        o.sn = 0.0;
        o.gamma = 1.0;
        o.delta = 0.0;
        o.rtol = rtol;
        o.its = 0;
        o.stop = (b1 > 0.0 && bb >= 0.0) ? 0x7fffffff : -1;
        o.indefinite_precond = bb < 0.0 ? 1 : 0;
        st[1] = o;
    }
}

template <int DIM, typename ET>
__global__ __launch_bounds__(VBLOCK) void k_mr_gather_l1(Geom g, const int32_t *__restrict__ ptr,
                                                         const int32_t *__restrict__ ent,
                                                         const ET *__restrict__ eV, int j,
                                                         const MinresState *__restrict__ st,
                                                         const double *__restrict__ v,
                                                         const double *__restrict__ r1,
                                                         double *__restrict__ hv,
                                                         double *__restrict__ part)
{
    if (j > st->stop) return;
    __shared__ double red[VBLOCK / 64];
    const double cr = j >= 1 ? st->beta / st->oldb : 0.0;
    double s = 0.0;
    // one lane per node, all components
    for (int node = xcd_block(blockIdx.x, gridDim.x) * VBLOCK + threadIdx.x; node < g.nx;
         node += gridDim.x * VBLOCK) {
        double a[DIM];
        bool fixed[DIM];
        gather_node<DIM, ET>(g, ptr, ent, eV, node, a, fixed);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const size_t idx = (size_t)c * g.nx + node;
            const double vi = v[idx];
            double h = fixed[c] ? vi : a[c];
            if (j >= 1) h -= cr * r1[idx];
            hv[idx] = h;
            s += vi * h;
        }
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(VBLOCK) void k_mr_l2(long n, int j, const MinresState *__restrict__ st,
                                                  const double *__restrict__ part1, int nb,
                                                  double *__restrict__ hv,
                                                  const double *__restrict__ r2,
                                                  const double *__restrict__ minv,
                                                  double *__restrict__ z,
                                                  double *__restrict__ part2)
{
    if (j > st->stop) return;
    __shared__ double red[VBLOCK / 64];
    const double alpha = sum_partials(part1, nb, red);
    const double c = alpha / st->beta;
    double s = 0.0;
    for (long i = blockIdx.x * (long)VBLOCK + threadIdx.x; i < n; i += (long)gridDim.x * VBLOCK) {
        const double h = hv[i] - c * r2[i];
        hv[i] = h;
        const double zi = minv ? minv[i] * h : h;
        z[i] = zi;
        s += h * zi;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part2[blockIdx.x] = s;
}

__global__ __launch_bounds__(VBLOCK) void k_mr_update(long n, int j,
                                                      const MinresState *__restrict__ sin,
                                                      MinresState *__restrict__ sout,
                                                      const double *__restrict__ part1,
                                                      const double *__restrict__ part2, int nb,
                                                      double *__restrict__ v,
                                                      const double *__restrict__ w1,
                                                      const double *__restrict__ w2,
                                                      double *__restrict__ wout,
                                                      double *__restrict__ x,
                                                      const double *__restrict__ z)
{
    if (j > sin->stop) {
        // carry the stopped state forward so later iterations see it
        if (blockIdx.x == 0 && threadIdx.x == 0) *sout = *sin;
        return;
    }
    __shared__ double red[VBLOCK / 64];
    const double alpha = sum_partials(part1, nb, red);
    const double bb = sum_partials(part2, nb, red);
    const double beta = sqrt(fmax(bb, 0.0));
    const double oldeps = sin->eps;
    const double delta = sin->cs * sin->dbar + sin->sn * alpha;
    const double gbar = sin->sn * sin->dbar - sin->cs * alpha;
    const double eps = sin->sn * beta;
    const double dbar = -sin->cs * beta;
    const double gamma = fmax(hypot(gbar, beta), 2.2250738585072014e-308);
    const double cs = gbar / gamma, sn = beta / gamma;
    const double phi = cs * sin->phibar;
    const double phibar = sn * sin->phibar;
    const double ig = 1.0 / gamma;
    const double sv = beta > 0.0 ? 1.0 / beta : 0.0;
    for (long i = blockIdx.x * (long)VBLOCK + threadIdx.x; i < n; i += (long)gridDim.x * VBLOCK) {
        const double wn = (v[i] - oldeps * w1[i] - delta * w2[i]) * ig;
        wout[i] = wn;
        x[i] += phi * wn;
        v[i] = sv * z[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        MinresState o = *sin;
        o.tmp = bb;
        o.alpha = alpha;
        o.oldb = sin->beta;
        o.beta = beta;
        o.oldeps = oldeps;
        o.eps = eps;
        o.dbar = dbar;
        o.delta = delta;
        o.gamma = gamma;
        o.cs = cs;
        o.sn = sn;
        o.phi = phi;
        o.phibar = phibar;
        o.its = j + 1;
        if (bb < 0.0) o.indefinite_precond = 1;
        if (phibar <= sin->rtol * sin->beta1 || beta == 0.0) o.stop = j;
        *sout = o;
    }
}

void mr_init(long n, const double *b, const double *minv, double *r1, double *r2, double *y,
             double *v, double *x, double *w, double *w1, double *w2, double *part,
             MinresState *st, double rtol, hipStream_t s)
{
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_mr_init, dim3(nb), dim3(VBLOCK), 0, s, n, b, minv, r1, r2, y, part);
    hipLaunchKernelGGL(k_mr_start, dim3(nb), dim3(VBLOCK), 0, s, n, st, rtol, part, nb, y, v, x,
                       w, w1, w2);
}

void mr_gather_l1(const Geom &g, const int32_t *csr_ptr, const int32_t *csr_ent, const void *eV,
                  bool fp32, int j, const MinresState *st, const double *v, const double *r1,
                  double *hv, double *part, hipStream_t s)
{
    const int nb = reduce_blocks((long)g.dim * g.nx);
#define TMOP_G(D, T)                                                                            \
    hipLaunchKernelGGL((k_mr_gather_l1<D, T>), dim3(nb), dim3(VBLOCK), 0, s, g, csr_ptr, csr_ent, \
                       (const T *)eV, j, st, v, r1, hv, part);
    if (g.dim == 3) {
        if (fp32) {
            TMOP_G(3, float)
        } else {
            TMOP_G(3, double)
        }
    } else {
        if (fp32) {
            TMOP_G(2, float)
        } else {
            TMOP_G(2, double)
        }
    }
#undef TMOP_G
}

void mr_lanczos2(long n, int j, const MinresState *st, const double *part1, double *hv,
                 const double *r2, const double *minv, double *z, double *part2, hipStream_t s)
{
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_mr_l2, dim3(nb), dim3(VBLOCK), 0, s, n, j, st, part1, nb, hv, r2, minv, z,
                       part2);
}

void mr_update(long n, int j, const MinresState *sin, MinresState *sout, const double *part1,
               const double *part2, double *v, const double *w1, const double *w2, double *wout,
               double *x, const double *z, hipStream_t s)
{
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_mr_update, dim3(nb), dim3(VBLOCK), 0, s, n, j, sin, sout, part1, part2, nb,
                       v, w1, w2, wout, x, z);
}

}  // namespace tmop
