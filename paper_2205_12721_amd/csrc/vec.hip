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
// tridiagonal matrix, short-recurrence update of the solution.  The Lanczos
// vector v_j = z_{j-1} / beta_j is never written: the element kernel runs on
// z_{j-1} and the gather scales its result by 1/beta_j (H is linear).  Per
// iteration j, after the element kernel has produced the E-vector of H z_{j-1}:
//   gather_upd: the update of iteration j-1, deferred to here (its scalars
//               need beta_j, known only after the previous l2):
//                 Givens rotation, phi;  w' = (v_{j-1} - oldeps w1 - delta w2)/gamma;
//                 x += phi w'
//               then hv = G^T eV / beta_j (fixed DoFs: v_j) - (beta_j/beta_{j-1}) r1
//               (in place of r1);  part1 = <v_j, hv>
//   l2:         alpha = sum part1;  hv -= (alpha/beta) r2;  z_j = M^{-1} hv;  part2 = <hv, z_j>
// and after the last iteration a finishing pass applies its deferred update.
// The scalar recurrences run redundantly in every workgroup (same partials,
// same order, same result) so no single-lane kernels sit between the vector
// passes; the state is double-buffered (the state after the update of
// iteration j - 1 goes to st[j&1], also when nothing runs, so the stop flag
// propagates).  Work of iteration j is skipped when j > stop (set when the
// residual estimate drops below rtol*beta1 or the Lanczos vector vanishes).
// ------------------------------------------------------------------------

// Sum of part[0..nb) by one wave (lane l adds l, l+64, ... in that order,
// 16 loads in flight, then a butterfly): the same bits in every workgroup.
__device__ inline double wave_sum_partials(const double *__restrict__ part, int nb)
{
    constexpr int RU = 16;
    const int l = threadIdx.x & 63;
    double s = 0.0;
    for (int k0 = 0; k0 < nb; k0 += 64 * RU) {
        double t[RU];
#pragma unroll
        for (int r = 0; r < RU; ++r) {
            const int k = k0 + r * 64 + l;
            t[r] = k < nb ? part[k] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < RU; ++r) s += t[r];
    }
    return wave_sum(s);
}

// Sums of pa[0..na) (wave 0) and, when pb is given, pb[0..nb) (wave 1), to
// every thread of the workgroup after one barrier.  Called at most once per
// kernel, by every thread.
__device__ inline void sum_partials(const double *__restrict__ pa, int na,
                                    const double *__restrict__ pb, int nb, double &a, double &b)
{
    __shared__ double sh[2];
    const int w = threadIdx.x >> 6;
    if (w == 0) {
        const double t = wave_sum_partials(pa, na);
        if (threadIdx.x == 0) sh[0] = t;
    } else if (w == 1 && pb) {
        const double t = wave_sum_partials(pb, nb);
        if (threadIdx.x == 64) sh[1] = t;
    }
    __syncthreads();
    a = sh[0];
    b = pb ? sh[1] : 0.0;
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

// beta1 from the partials; st[0] and st[1] the initial state; x = 0, and
// w = w1 = w2 = 0 when w is given (the three-term update); v = y / beta1 when
// v is given (the solver here keeps y unscaled instead).
__global__ __launch_bounds__(VBLOCK) void k_mr_start(long n, MinresState *st, double rtol,
                                                     const double *__restrict__ part, int nb,
                                                     const double *__restrict__ y,
                                                     double *__restrict__ v,
                                                     double *__restrict__ x,
                                                     double *__restrict__ w,
                                                     double *__restrict__ w1,
                                                     double *__restrict__ w2)
{
    double bb, unused;
    sum_partials(part, nb, nullptr, 0, bb, unused);
    const double b1 = sqrt(fmax(bb, 0.0));
    const double s = b1 > 0.0 ? 1.0 / b1 : 0.0;
    for (long i = blockIdx.x * (long)VBLOCK + threadIdx.x; i < n; i += (long)gridDim.x * VBLOCK) {
        if (v) v[i] = s * y[i];
        x[i] = 0.0;
        if (w) {
            w[i] = 0.0;
            w1[i] = 0.0;
            w2[i] = 0.0;
        }
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

// Scalars of the update of iteration jm (Givens rotation of the Lanczos
// tridiagonal matrix) from the state before it, alpha_jm and beta_{jm+1}^2.
struct MrUpd {
    MinresState o;  // state after the update
    double ig, oldeps, delta, phi;
};

__device__ inline MrUpd mr_scalars(const MinresState &sin, int jm, double alpha, double bb)
{
    MrUpd u;
    const double beta = sqrt(fmax(bb, 0.0));
    u.oldeps = sin.eps;
    u.delta = sin.cs * sin.dbar + sin.sn * alpha;
    const double gbar = sin.sn * sin.dbar - sin.cs * alpha;
    const double eps = sin.sn * beta;
    const double dbar = -sin.cs * beta;
    const double gamma = fmax(hypot(gbar, beta), 2.2250738585072014e-308);
    const double cs = gbar / gamma, sn = beta / gamma;
    u.phi = cs * sin.phibar;
    const double phibar = sn * sin.phibar;
    u.ig = 1.0 / gamma;
    MinresState o = sin;
    o.tmp = bb;
    o.alpha = alpha;
    o.oldb = sin.beta;
    o.beta = beta;
    o.oldeps = u.oldeps;
    o.eps = eps;
    o.dbar = dbar;
    o.delta = u.delta;
    o.gamma = gamma;
    o.cs = cs;
    o.sn = sn;
    o.phi = u.phi;
    o.phibar = phibar;
    o.its = jm + 1;
    if (bb < 0.0) o.indefinite_precond = 1;
    if (phibar <= sin.rtol * sin.beta1 || beta == 0.0) o.stop = jm;
    u.o = o;
    return u;
}

// Iteration j after the element kernel ran on z_{j-1} (the Lanczos vector
// v_j = z_{j-1} / beta_j, left unscaled so that nothing writes v):
//   the deferred update of iteration j-1 (state S_{j-1} -> S_j, from the
//   partials of alpha_{j-1} and beta_j^2):
//     w' = (z_{j-2}/beta_{j-1} - oldeps w1 - delta w2) / gamma;  x += phi w'
//   then hv = G^T eV / beta_j (fixed DoFs: v_j) - (beta_j/beta_{j-1}) r1, in
//   place of r1;  part1 = <v_j, hv>.
// With hist given (the Lanczos vectors kept resident) the update's scalars go
// to hist[j-1] instead and w, x are not touched: the solution is formed once
// after the loop (k_mr_combine).
template <int DIM, typename ET>
__global__ __launch_bounds__(VBLOCK) void k_mr_gather_upd(
    Geom g, const int32_t *__restrict__ ptr, const int32_t *__restrict__ ent,
    const ET *__restrict__ eV, int j, const MinresState *__restrict__ sin,
    MinresState *__restrict__ sout, const double *__restrict__ p1prev, int nb1,
    const double *__restrict__ p2prev, int nb2, const double *__restrict__ zp,
    const double *__restrict__ zc, const double *__restrict__ w1, const double *__restrict__ w2,
    double *__restrict__ wout, double *__restrict__ x, double *__restrict__ r1hv,
    double *__restrict__ part, MrHist *__restrict__ hist)
{
    __shared__ double red[VBLOCK / 64];
    const int nstride = gridDim.x * VBLOCK;
    const int node0 = xcd_block(blockIdx.x, gridDim.x) * VBLOCK + threadIdx.x;
    // The first node's loads go out before the state and the partial sums
    // are read (they are in bounds whether or not the gather runs).
    const bool pre = node0 < g.nx;
    double a0[DIM], z0[DIM], q0[DIM];
    bool f0[DIM];
    if (pre) {
        gather_node<DIM, ET>(g, ptr, ent, eV, node0, a0, f0);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const size_t idx = (size_t)c * g.nx + node0;
            z0[c] = zc[idx];
            q0[c] = j >= 1 ? r1hv[idx] : 0.0;
        }
    }
    const MinresState S = *sin;
    const bool upd = j >= 1 && j - 1 <= S.stop;
    MrUpd u{};
    u.o = S;
    if (upd) {
        double alpha, bb;
        sum_partials(p1prev, nb1, p2prev, nb2, alpha, bb);
        u = mr_scalars(S, j - 1, alpha, bb);
    }
    const double sp = S.beta > 0.0 ? 1.0 / S.beta : 0.0;      // v_{j-1} = sp z_{j-2}
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *sout = u.o;
        if (hist && upd) hist[j - 1] = MrHist{u.ig, u.oldeps, u.delta, u.phi, sp, {}};
    }
    const bool gat = j <= u.o.stop;
    const bool vupd = upd && !hist;
    if (!vupd && !gat) return;
    const double sc = u.o.beta > 0.0 ? 1.0 / u.o.beta : 0.0;  // v_j = sc z_{j-1}
    const double cr = j >= 1 ? u.o.beta / u.o.oldb : 0.0;
    double s = 0.0;
    // one lane per node, all components
    for (int node = node0; node < g.nx; node += nstride) {
        double a[DIM], zv[DIM], qv[DIM];
        bool fixed[DIM];
        if (node == node0 && pre) {
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                a[c] = a0[c];
                fixed[c] = f0[c];
                zv[c] = z0[c];
                qv[c] = q0[c];
            }
        } else if (gat) {
            gather_node<DIM, ET>(g, ptr, ent, eV, node, a, fixed);
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const size_t idx = (size_t)c * g.nx + node;
                zv[c] = zc[idx];
                qv[c] = j >= 1 ? r1hv[idx] : 0.0;
            }
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const size_t idx = (size_t)c * g.nx + node;
            if (vupd) {
                const double wn = (sp * zp[idx] - u.oldeps * w1[idx] - u.delta * w2[idx]) * u.ig;
                wout[idx] = wn;
                x[idx] += u.phi * wn;
            }
            if (gat) {
                const double vi = sc * zv[c];
                double h = fixed[c] ? vi : sc * a[c];
                if (j >= 1) h -= cr * qv[c];
                r1hv[idx] = h;
                s += vi * h;
            }
        }
    }
    if (!gat) return;
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// The update of the last iteration jm run (deferred past the loop).
__global__ __launch_bounds__(VBLOCK) void k_mr_finish(long n, int jm,
                                                      const MinresState *__restrict__ sin,
                                                      MinresState *__restrict__ sout,
                                                      const double *__restrict__ p1, int nb1,
                                                      const double *__restrict__ p2, int nb2,
                                                      const double *__restrict__ zp,
                                                      const double *__restrict__ w1,
                                                      const double *__restrict__ w2,
                                                      double *__restrict__ wout,
                                                      double *__restrict__ x)
{
    const MinresState S = *sin;
    if (jm < 0 || jm > S.stop) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *sout = S;
        return;
    }
    double alpha, bb;
    sum_partials(p1, nb1, p2, nb2, alpha, bb);
    const MrUpd u = mr_scalars(S, jm, alpha, bb);
    if (blockIdx.x == 0 && threadIdx.x == 0) *sout = u.o;
    const double sp = S.beta > 0.0 ? 1.0 / S.beta : 0.0;
    for (long i = blockIdx.x * (long)VBLOCK + threadIdx.x; i < n; i += (long)gridDim.x * VBLOCK) {
        const double wn = (sp * zp[i] - u.oldeps * w1[i] - u.delta * w2[i]) * u.ig;
        wout[i] = wn;
        x[i] += u.phi * wn;
    }
}

// The solution from the resident Lanczos vectors, once after the loop.  The
// last update (jm) is taken here from its partials as in k_mr_finish; then
// x = sum_m phi_m w_m with every w_m a combination of v_0..v_m, so
// x = sum_i c_i v_i where lane i runs the three-term recurrence of the w's
// on their i-th coefficients:  W_m[i] = (delta_{mi} - oldeps_m W_{m-2}[i]
// - delta_m W_{m-1}[i]) ig_m,  c_i = sum_{m>=i} phi_m W_m[i].  Every block
// forms the same coefficients in the same order.  bank holds z_0..z_{K-1}
// with the given stride (v_i = sv_i z_i).
__global__ __launch_bounds__(VBLOCK) void k_mr_combine(long n, int jm,
                                                       const MinresState *__restrict__ sin,
                                                       MinresState *__restrict__ sout,
                                                       const double *__restrict__ p1, int nb1,
                                                       const double *__restrict__ p2, int nb2,
                                                       MrHist *__restrict__ hist,
                                                       const double *__restrict__ bank,
                                                       long stride, double *__restrict__ x)
{
    static_assert(MR_MAX_BASIS <= VBLOCK, "one lane per coefficient");
    __shared__ double hig[MR_MAX_BASIS], hoe[MR_MAX_BASIS], hde[MR_MAX_BASIS],
        hph[MR_MAX_BASIS], coef[MR_MAX_BASIS];
    const MinresState S = *sin;
    const bool last = jm >= 0 && jm <= S.stop;
    // updates taken: 0..K-1 (the earlier ones by the gathers)
    const int K = last ? jm + 1 : (S.stop < jm ? S.stop + 1 : (jm > 0 ? jm : 0));
    MrUpd u{};
    u.o = S;
    if (last) {
        double alpha, bb;
        sum_partials(p1, nb1, p2, nb2, alpha, bb);
        u = mr_scalars(S, jm, alpha, bb);
    }
    const double sp = S.beta > 0.0 ? 1.0 / S.beta : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *sout = u.o;
        if (last) hist[jm] = MrHist{u.ig, u.oldeps, u.delta, u.phi, sp, {}};
    }
    const int t = threadIdx.x;
    double svt = 0.0;
    if (t < K) {
        MrHist h;
        if (last && t == jm)
            h = MrHist{u.ig, u.oldeps, u.delta, u.phi, sp, {}};
        else
            h = hist[t];
        hig[t] = h.ig;
        hoe[t] = h.oldeps;
        hde[t] = h.delta;
        hph[t] = h.phi;
        svt = h.sv;
    }
    __syncthreads();
    if (t < K) {
        double a2 = 0.0, a1 = 0.0, c = 0.0;
        for (int m = t; m < K; ++m) {
            const double wn = ((m == t ? 1.0 : 0.0) - hoe[m] * a2 - hde[m] * a1) * hig[m];
            c += hph[m] * wn;
            a2 = a1;
            a1 = wn;
        }
        coef[t] = c * svt;
    }
    __syncthreads();
    for (long i = blockIdx.x * (long)VBLOCK + threadIdx.x; i < n; i += (long)gridDim.x * VBLOCK) {
        double acc = 0.0;
        int m = 0;
        for (; m + 4 <= K; m += 4) {
            const double z0 = bank[(long)m * stride + i], z1 = bank[(long)(m + 1) * stride + i];
            const double z2 = bank[(long)(m + 2) * stride + i];
            const double z3 = bank[(long)(m + 3) * stride + i];
            acc += coef[m] * z0;
            acc += coef[m + 1] * z1;
            acc += coef[m + 2] * z2;
            acc += coef[m + 3] * z3;
        }
        for (; m < K; ++m) acc += coef[m] * bank[(long)m * stride + i];
        x[i] = acc;
    }
}

__global__ __launch_bounds__(VBLOCK) void k_mr_l2(long n, int j, const MinresState *__restrict__ st,
                                                  const double *__restrict__ part1, int nb1,
                                                  double *__restrict__ hv,
                                                  const double *__restrict__ r2,
                                                  const double *__restrict__ minv,
                                                  double *__restrict__ z,
                                                  double *__restrict__ part2)
{
    __shared__ double red[VBLOCK / 64];
    // this lane's first RU entries are loaded before the state is read and
    // alpha summed
    constexpr int RU = 8;
    const long stride = (long)gridDim.x * VBLOCK;
    const long i0 = blockIdx.x * (long)VBLOCK + threadIdx.x;
    double hr[RU], rr[RU], mr[RU];
#pragma unroll
    for (int k = 0; k < RU; ++k) {
        const long i = i0 + k * stride;
        hr[k] = i < n ? hv[i] : 0.0;
        rr[k] = i < n ? r2[i] : 0.0;
        mr[k] = i < n && minv ? minv[i] : 1.0;
    }
    if (j > st->stop) return;
    double alpha, unused;
    sum_partials(part1, nb1, nullptr, 0, alpha, unused);
    const double c = alpha / st->beta;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < RU; ++k) {
        const long i = i0 + k * stride;
        if (i < n) {
            const double h = hr[k] - c * rr[k];
            hv[i] = h;
            const double zi = minv ? mr[k] * h : h;
            z[i] = zi;
            s += h * zi;
        }
    }
    for (long i = i0 + RU * stride; i < n; i += stride) {
        const double h = hv[i] - c * r2[i];
        hv[i] = h;
        const double zi = minv ? minv[i] * h : h;
        z[i] = zi;
        s += h * zi;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part2[blockIdx.x] = s;
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

void mr_gather_upd(const Geom &g, const int32_t *csr_ptr, const int32_t *csr_ent, const void *eV,
                   bool fp32, int j, const MinresState *sin, MinresState *sout,
                   const double *p1prev, const double *p2prev, const double *zp, const double *zc,
                   const double *w1, const double *w2, double *wout, double *x, double *r1hv,
                   double *part, MrHist *hist, hipStream_t s)
{
    // one node per lane up to 1024 workgroups; its partials (alpha) number
    // nb1, those of the vector kernels (beta^2) nb2
    const int nb1 = mr_gather_grid(g), nb2 = reduce_blocks((long)g.dim * g.nx);
#define TMOP_G(D, T)                                                                          \
    hipLaunchKernelGGL((k_mr_gather_upd<D, T>), dim3(nb1), dim3(VBLOCK), 0, s, g, csr_ptr,    \
                       csr_ent, (const T *)eV, j, sin, sout, p1prev, nb1, p2prev, nb2, zp, zc, \
                       w1, w2, wout, x, r1hv, part, hist);
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

// At most 1024 workgroups (a lane takes several nodes on large meshes): every
// workgroup of the next kernel sums all of these partials, and with 2048 the
// Newton step measured 0.4-1.9% slower (24^3 Q3, 64^3 Q2, Kershaw p = 4).
int mr_gather_grid(const Geom &g) { return vgrid((long)g.nx, 1024); }

void mr_lanczos2(long n, int nb1, int j, const MinresState *st, const double *part1, double *hv,
                 const double *r2, const double *minv, double *z, double *part2, hipStream_t s)
{
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_mr_l2, dim3(nb), dim3(VBLOCK), 0, s, n, j, st, part1, nb1, hv, r2, minv,
                       z, part2);
}

void mr_finish(long n, int nb1, int jm, const MinresState *sin, MinresState *sout,
               const double *p1, const double *p2, const double *zp, const double *w1,
               const double *w2, double *wout, double *x, hipStream_t s)
{
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_mr_finish, dim3(nb), dim3(VBLOCK), 0, s, n, jm, sin, sout, p1, nb1, p2,
                       nb, zp, w1, w2, wout, x);
}

void mr_combine(long n, int nb1, int jm, const MinresState *sin, MinresState *sout,
                const double *p1, const double *p2, MrHist *hist, const double *bank, long stride,
                double *x, hipStream_t s)
{
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_mr_combine, dim3(nb), dim3(VBLOCK), 0, s, n, jm, sin, sout, p1, nb1, p2,
                       nb, hist, bank, stride, x);
}

}  // namespace tmop
