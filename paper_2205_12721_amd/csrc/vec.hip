// Node-level kernels: the transpose of the element restriction (E-vector ->
// global vector, Sec. 3 operator decomposition, G^T), deterministic
// reductions, and the vector work of Newton and of preconditioned MINRES.
#include <hip/hip_runtime.h>

#include "tmop_dev.hpp"
#include "vec.hpp"

namespace tmop {

constexpr int VBLOCK = 256;

// ------------------------------------------------------------------------
// G^T for the structured box: out[c][node] = sum over the (up to 2^dim)
// element-local copies of the node, in a fixed order (deterministic).
// Fixed DoFs get: 0 (fix_mode 0), 1 (fix_mode 1) or src[c][node] (fix_mode 2).
// ------------------------------------------------------------------------
template <int DIM, typename ET>
__global__ __launch_bounds__(VBLOCK) void k_gather_box(Geom g, const ET *__restrict__ eV,
                                                       double *__restrict__ out, int fix_mode,
                                                       const double *__restrict__ src)
{
    const int p = g.p, ni = p + 1;
    const int np = DIM == 3 ? ni * ni * ni : ni * ni;
    const long total = (long)DIM * g.nx;
    for (long idx = blockIdx.x * (long)VBLOCK + threadIdx.x; idx < total;
         idx += (long)gridDim.x * VBLOCK) {
        const int c = (int)(idx / g.nx);
        const int node = (int)(idx % g.nx);
        int gc[3];
        gc[0] = node % g.M[0];
        const int t = node / g.M[0];
        gc[1] = DIM == 3 ? t % g.M[1] : t;
        gc[2] = DIM == 3 ? t / g.M[1] : 0;
        const bool fixed = is_fixed(g, c, node, gc[0], gc[1], gc[2]);
        if (fixed) {
            out[idx] = fix_mode == 0 ? 0.0 : (fix_mode == 1 ? 1.0 : src[idx]);
            continue;
        }
        // per axis: up to two (element, local index) candidates
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
        out[idx] = (double)s;
    }
}

// G^T for a general mesh through the node -> (element*np + local) CSR map.
template <int DIM, typename ET>
__global__ __launch_bounds__(VBLOCK) void k_gather_csr(Geom g, const int32_t *__restrict__ ptr,
                                                       const int32_t *__restrict__ ent,
                                                       const ET *__restrict__ eV,
                                                       double *__restrict__ out, int fix_mode,
                                                       const double *__restrict__ src)
{
    const int ni = g.p + 1;
    const int np = DIM == 3 ? ni * ni * ni : ni * ni;
    const long total = (long)DIM * g.nx;
    for (long idx = blockIdx.x * (long)VBLOCK + threadIdx.x; idx < total;
         idx += (long)gridDim.x * VBLOCK) {
        const int c = (int)(idx / g.nx);
        const int node = (int)(idx % g.nx);
        if (is_fixed(g, c, node, -1, -1, -1)) {
            out[idx] = fix_mode == 0 ? 0.0 : (fix_mode == 1 ? 1.0 : src[idx]);
            continue;
        }
        ET s = 0;
        for (int k = ptr[node]; k < ptr[node + 1]; ++k) {
            const long en = ent[k];
            const long e = en / np;
            const int i = (int)(en % np);
            s += eV[(e * DIM + c) * np + i];
        }
        out[idx] = (double)s;
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
    const int grid = vgrid((long)g.dim * g.nx, 8192);
#define TMOP_G(D, T)                                                                              \
    if (csr_ptr)                                                                                  \
        hipLaunchKernelGGL((k_gather_csr<D, T>), dim3(grid), dim3(VBLOCK), 0, s, g, csr_ptr,     \
                           csr_ent, (const T *)eV, out, fix_mode, src);                           \
    else                                                                                          \
        hipLaunchKernelGGL((k_gather_box<D, T>), dim3(grid), dim3(VBLOCK), 0, s, g,              \
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
    for (int k = threadIdx.x; k < nb; k += VBLOCK) {
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
    for (int k = threadIdx.x; k < nb; k += VBLOCK) s += part[k];
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
// tridiagonal matrix, short-recurrence update of the solution; see the
// documentation of tmop_minres.  Iteration j's kernels skip once
// j > st->stop (set by the QR kernel when the residual estimate drops below
// rtol * beta1 or the Lanczos vector vanishes).
// ------------------------------------------------------------------------

__global__ __launch_bounds__(VBLOCK) void k_mr_init(long n, const double *__restrict__ b,
                                                    const double *__restrict__ minv,
                                                    double *__restrict__ r1,
                                                    double *__restrict__ r2,
                                                    double *__restrict__ y,
                                                    double *__restrict__ x,
                                                    double *__restrict__ w,
                                                    double *__restrict__ w1,
                                                    double *__restrict__ w2,
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
        x[i] = 0.0;
        w[i] = 0.0;
        w1[i] = 0.0;
        w2[i] = 0.0;
        s += bi * yi;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_mr_start(MinresState *st, double rtol)
{
    const double b1 = sqrt(fmax(st->tmp, 0.0));
    st->beta1 = b1;
    st->beta = b1;
    st->oldb = 0.0;
    st->dbar = 0.0;
    st->eps = 0.0;
    st->phibar = b1;
    st->cs = -1.0;
    st->sn = 0.0;
    st->rtol = rtol;
    st->its = 0;
    st->stop = (b1 > 0.0 && st->tmp >= 0.0) ? 0x7fffffff : -1;
    st->indefinite_precond = st->tmp < 0.0 ? 1 : 0;
}

// v = y / beta
__global__ __launch_bounds__(VBLOCK) void k_mr_v(long n, int j, const MinresState *__restrict__ st,
                                                 const double *__restrict__ y,
                                                 double *__restrict__ v)
{
    if (j > st->stop) return;
    const double s = 1.0 / st->beta;
    for (long i = blockIdx.x * (long)VBLOCK + threadIdx.x; i < n; i += (long)gridDim.x * VBLOCK)
        v[i] = s * y[i];
}

// hv -= (beta/oldb) r1 (j >= 1); partial <v, hv>
__global__ __launch_bounds__(VBLOCK) void k_mr_l1(long n, int j,
                                                  const MinresState *__restrict__ st,
                                                  double *__restrict__ hv,
                                                  const double *__restrict__ r1,
                                                  const double *__restrict__ v,
                                                  double *__restrict__ part)
{
    if (j > st->stop) return;
    __shared__ double red[VBLOCK / 64];
    const double c = j >= 1 ? st->beta / st->oldb : 0.0;
    double s = 0.0;
    for (long i = blockIdx.x * (long)VBLOCK + threadIdx.x; i < n; i += (long)gridDim.x * VBLOCK) {
        double h = hv[i];
        if (j >= 1) h -= c * r1[i];
        hv[i] = h;
        s += v[i] * h;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_mr_alpha(MinresState *st, int j, const double *__restrict__ part, int nb)
{
    if (j > st->stop) return;
    // single wave64: fixed-order sum
    double s = 0.0;
    for (int k = threadIdx.x; k < nb; k += 64) s += part[k];
    s = wave_sum(s);
    if (threadIdx.x == 0) st->alpha = s;
}

// hv -= (alpha/beta) r2; z = M^{-1} hv; partial <hv, z>
__global__ __launch_bounds__(VBLOCK) void k_mr_l2(long n, int j,
                                                  const MinresState *__restrict__ st,
                                                  double *__restrict__ hv,
                                                  const double *__restrict__ r2,
                                                  const double *__restrict__ minv,
                                                  double *__restrict__ z,
                                                  double *__restrict__ part)
{
    if (j > st->stop) return;
    __shared__ double red[VBLOCK / 64];
    const double c = st->alpha / st->beta;
    double s = 0.0;
    for (long i = blockIdx.x * (long)VBLOCK + threadIdx.x; i < n; i += (long)gridDim.x * VBLOCK) {
        const double h = hv[i] - c * r2[i];
        hv[i] = h;
        const double zi = minv ? minv[i] * h : h;
        z[i] = zi;
        s += h * zi;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// New beta, Givens rotation, step length phi and residual estimate phibar.
__global__ void k_mr_qr(MinresState *st, int j, const double *__restrict__ part, int nb)
{
    if (j > st->stop) return;
    double s = 0.0;
    for (int k = threadIdx.x; k < nb; k += 64) s += part[k];
    s = wave_sum(s);
    if (threadIdx.x != 0) return;
    if (s < 0.0) st->indefinite_precond = 1;
    st->oldb = st->beta;
    st->beta = sqrt(fmax(s, 0.0));
    st->oldeps = st->eps;
    const double delta = st->cs * st->dbar + st->sn * st->alpha;
    const double gbar = st->sn * st->dbar - st->cs * st->alpha;
    st->eps = st->sn * st->beta;
    st->dbar = -st->cs * st->beta;
    double gamma = hypot(gbar, st->beta);
    gamma = fmax(gamma, 2.2250738585072014e-308);
    st->cs = gbar / gamma;
    st->sn = st->beta / gamma;
    st->phi = st->cs * st->phibar;
    st->phibar = st->sn * st->phibar;
    st->delta = delta;
    st->gamma = gamma;
    st->its = j + 1;
    if (st->phibar <= st->rtol * st->beta1 || st->beta == 0.0) st->stop = j;
}

// wout = (v - oldeps w1 - delta w2) / gamma; x += phi wout
__global__ __launch_bounds__(VBLOCK) void k_mr_x(long n, int j, const MinresState *__restrict__ st,
                                                 const double *__restrict__ v,
                                                 const double *__restrict__ w1,
                                                 const double *__restrict__ w2,
                                                 double *__restrict__ wout,
                                                 double *__restrict__ x)
{
    if (j > st->stop) return;
    const double oe = st->oldeps, de = st->delta, ig = 1.0 / st->gamma, ph = st->phi;
    for (long i = blockIdx.x * (long)VBLOCK + threadIdx.x; i < n; i += (long)gridDim.x * VBLOCK) {
        const double wn = (v[i] - oe * w1[i] - de * w2[i]) * ig;
        wout[i] = wn;
        x[i] += ph * wn;
    }
}

void mr_init(long n, const double *b, const double *minv, double *r1, double *r2, double *y,
             double *x, double *w, double *w1, double *w2, double *part, MinresState *st,
             double rtol, hipStream_t s)
{
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_mr_init, dim3(nb), dim3(VBLOCK), 0, s, n, b, minv, r1, r2, y, x, w, w1,
                       w2, part);
    hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(VBLOCK), 0, s, part, nb, &st->tmp);
    hipLaunchKernelGGL(k_mr_start, dim3(1), dim3(1), 0, s, st, rtol);
}

void mr_v(long n, int j, const MinresState *st, const double *y, double *v, hipStream_t s)
{
    hipLaunchKernelGGL(k_mr_v, dim3(vgrid(n, 8192)), dim3(VBLOCK), 0, s, n, j, st, y, v);
}

void mr_lanczos1(long n, int j, MinresState *st, double *hv, const double *r1, const double *v,
                 double *part, hipStream_t s)
{
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_mr_l1, dim3(nb), dim3(VBLOCK), 0, s, n, j, st, hv, r1, v, part);
    hipLaunchKernelGGL(k_mr_alpha, dim3(1), dim3(64), 0, s, st, j, part, nb);
}

void mr_lanczos2(long n, int j, MinresState *st, double *hv, const double *r2, const double *minv,
                 double *z, double *part, hipStream_t s)
{
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_mr_l2, dim3(nb), dim3(VBLOCK), 0, s, n, j, st, hv, r2, minv, z, part);
    hipLaunchKernelGGL(k_mr_qr, dim3(1), dim3(64), 0, s, st, j, part, nb);
}

void mr_update(long n, int j, const MinresState *st, const double *v, const double *w1,
               const double *w2, double *wout, double *x, hipStream_t s)
{
    hipLaunchKernelGGL(k_mr_x, dim3(vgrid(n, 8192)), dim3(VBLOCK), 0, s, n, j, st, v, w1, w2, wout,
                       x);
}

}  // namespace tmop
