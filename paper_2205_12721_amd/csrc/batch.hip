// Batched and served TMOP solves: many meshes of different orders advance
// together through the Newton-MINRES loop (Sec. 2.3), each phase issued as
// one launch per kernel class (dim, p, n_q) over a tile list that spans every
// participating mesh, plus chunked vector launches over all meshes' DoFs.
//
// Memory: one device arena sized by an HBM budget; each admitted mesh (slot)
// takes one contiguous region holding its DoF vectors, quadrature data and
// E-vector scratch (first-fit allocation).  Per-mesh reductions are segmented:
// a vector tile never straddles two meshes, and a mesh's sums run over its
// own tiles in a fixed order, so a mesh's arithmetic does not depend on the
// other meshes in the batch.
//
// MINRES runs in lockstep for all meshes with a device-resident,
// double-buffered state per mesh (iteration counter included), so a block of
// six iterations is position independent and is captured once as a hipGraph
// and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/tmop.h"
#include "ops.hpp"
#include "tmop_dev.hpp"
#include <rocprofiler-sdk-roctx/roctx.h>

#include "gather.hpp"
#include "vec.hpp"

namespace tmop {

// vector ids inside SlotDev::vec
enum {
    BX, BXT, BG, BGT, BDX, BR1, BR2, BZ1, BZ0, BW, BW1, BW2, BMINV, BDIAG, BY, BNV
};
// not allocated: the MINRES input of the element kernels (the current
// preconditioned Lanczos vector, in the bank or in BZ0/BZ1), set on the
// device by kv_mr_start and kv_mr_l2
constexpr int BZIN = BNV;
static_assert(BNV < NVEC, "too many vectors per slot");

constexpr int VB = 256;      // threads per vector block
constexpr int VCH = 8 * VB;  // DoFs per vector tile

struct VTile {
    int slot;
    int start;
    int count;
};

// per-slot tile ranges for segmented reductions
struct SlotRange {
    int ebase;    // first element-tile partial (absolute index in the partial array)
    int ecount;   // element tiles of the slot
    int estride;  // tiles of the slot's class launch (stride between partial planes)
    int vbegin;   // first vector tile
    int vcount;   // vector tiles of the slot
};

// per-slot device scalars
enum { SC_F, SC_MD, SC_BAD, SC_DOT, SC_DMAX, SC_ALPHA, NSC = 8 };

// Per-slot MINRES state (double-buffered): like MinresState plus the
// iteration counter and cap.
struct BState {
    double beta1, beta, oldb, dbar, eps, phibar, cs, sn, rtol;
    int j, maxit, stop, indefinite;
    int first;  // no iteration has run yet (no update pending)
    int pad;
};

__device__ inline bool bs_skip(const BState &s) { return s.j > s.stop || s.j >= s.maxit; }

// sum of part[b .. b+n) in a fixed order, identical in every block
__device__ inline double seg_sum(const double *__restrict__ part, int b, int n, double *red)
{
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += VB) s += part[b + k];
    s = block_sum(s, red);
    __shared__ double bc;
    if (threadIdx.x == 0) bc = s;
    __syncthreads();
    return bc;
}

// ---------------------------------------------------------------------------
// Segmented reductions: one block per slot
// ---------------------------------------------------------------------------

// energy partials of element tiles -> F, min det, bad count
__global__ __launch_bounds__(VB) void kr_energy(const SlotRange *__restrict__ rg,
                                                const int *__restrict__ gate,
                                                const double *__restrict__ part,
                                                double *__restrict__ sc)
{
    const int s = blockIdx.x;
    if (!gate[s]) return;
    __shared__ double red[VB / 64];
    const SlotRange r = rg[s];
    double a = 0.0, m = 1.0e300, b = 0.0;
    for (int k = threadIdx.x; k < r.ecount; k += VB) {
        a += part[r.ebase + k];
        m = fmin(m, part[r.ebase + r.estride + k]);
        b += part[r.ebase + 2 * r.estride + k];
    }
    a = block_sum(a, red);
    m = block_min(m, red);
    b = block_sum(b, red);
    if (threadIdx.x == 0) {
        sc[s * NSC + SC_F] = a;
        sc[s * NSC + SC_MD] = m;
        sc[s * NSC + SC_BAD] = b;
    }
}

// vector-tile partials -> per-slot sum (op 0) or max (op 1) into sc[slot*NSC + which]
__global__ __launch_bounds__(VB) void kr_vec(const SlotRange *__restrict__ rg,
                                             const int *__restrict__ gate,
                                             const double *__restrict__ part, int op, int which,
                                             double *__restrict__ sc)
{
    const int s = blockIdx.x;
    if (!gate[s]) return;
    __shared__ double red[VB / 64];
    const SlotRange r = rg[s];
    double a = 0.0;
    for (int k = threadIdx.x; k < r.vcount; k += VB)
        a = op == 0 ? a + part[r.vbegin + k] : fmax(a, part[r.vbegin + k]);
    a = op == 0 ? block_sum(a, red) : -block_min(-a, red);
    if (threadIdx.x == 0) sc[s * NSC + which] = a;
}

// ---------------------------------------------------------------------------
// Vector kernels over vector tiles
// ---------------------------------------------------------------------------

#define VT_PROLOGUE                                     \
    const VTile t = vt[blockIdx.x];                     \
    if (gate && !gate[t.slot]) return;                  \
    const SlotDev &S = slots[t.slot];                   \
    const int i0 = t.start + threadIdx.x, i1 = t.start + t.count;

__global__ __launch_bounds__(VB) void kv_step(const VTile *__restrict__ vt,
                                              const SlotDev *__restrict__ slots,
                                              const int *__restrict__ gate,
                                              const double *__restrict__ sc)
{
    VT_PROLOGUE
    const double a = sc[t.slot * NSC + SC_ALPHA];
    const double *__restrict__ x = S.vec[BX], *__restrict__ dx = S.vec[BDX];
    double *__restrict__ xt = S.vec[BXT];
    for (int i = i0; i < i1; i += VB) xt[i] = x[i] - a * dx[i];
}

__global__ __launch_bounds__(VB) void kv_copy(const VTile *__restrict__ vt,
                                              const SlotDev *__restrict__ slots,
                                              const int *__restrict__ gate, int vs, int vd)
{
    VT_PROLOGUE
    const double *__restrict__ a = S.vec[vs];
    double *__restrict__ b = S.vec[vd];
    for (int i = i0; i < i1; i += VB) b[i] = a[i];
}

__global__ __launch_bounds__(VB) void kv_dot(const VTile *__restrict__ vt,
                                             const SlotDev *__restrict__ slots,
                                             const int *__restrict__ gate, int va, int vb,
                                             double *__restrict__ part)
{
    VT_PROLOGUE
    __shared__ double red[VB / 64];
    const double *__restrict__ a = S.vec[va], *__restrict__ b = S.vec[vb];
    double s = 0.0;
    for (int i = i0; i < i1; i += VB) s += a[i] * b[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(VB) void kv_absmax(const VTile *__restrict__ vt,
                                                const SlotDev *__restrict__ slots,
                                                const int *__restrict__ gate, int va,
                                                double *__restrict__ part)
{
    VT_PROLOGUE
    __shared__ double red[VB / 64];
    const double *__restrict__ a = S.vec[va];
    double s = 0.0;
    for (int i = i0; i < i1; i += VB) s = fmax(s, fabs(a[i]));
    s = -block_min(-s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(VB) void kv_jacobi(const VTile *__restrict__ vt,
                                                const SlotDev *__restrict__ slots,
                                                const int *__restrict__ gate,
                                                const double *__restrict__ sc)
{
    VT_PROLOGUE
    const double floor = 1e-14 * sc[t.slot * NSC + SC_DMAX];
    const double *__restrict__ d = S.vec[BDIAG];
    double *__restrict__ m = S.vec[BMINV];
    for (int i = i0; i < i1; i += VB) {
        const double a = fmax(fabs(d[i]), floor);
        m[i] = a > 0.0 ? 1.0 / a : 1.0;
    }
}

// out = G^T eV of the slot; fixed DoFs get 0 / 1 / vec[vsrc]
template <int DIM, typename ET>
__global__ __launch_bounds__(VB) void kv_gather(const VTile *__restrict__ vt,
                                                const SlotDev *__restrict__ slots,
                                                const int *__restrict__ gate, int vout,
                                                int fix_mode, int vsrc)
{
    VT_PROLOGUE
    const Geom &g = S.g;
    const ET *__restrict__ eV = (const ET *)S.eV;
    double *__restrict__ out = S.vec[vout];
    const double *__restrict__ src = S.vec[vsrc];
    for (int i = i0; i < i1; i += VB) {
        const int c = i >= g.nx ? (DIM == 3 && i >= 2 * g.nx ? 2 : 1) : 0;
        const int node = i - c * g.nx;
        int gc[3];
        box_coords<DIM>(g, node, gc);
        const bool fixed = is_fixed(g, c, node, gc[0], gc[1], gc[2]);
        double v;
        if (fixed)
            v = fix_mode == 0 ? 0.0 : (fix_mode == 1 ? 1.0 : src[i]);
        else
            v = (double)gather_box_node<DIM, ET>(g, eV, c, node, gc);
        out[i] = v;
    }
}

// ---------------------------------------------------------------------------
// MINRES (see vec.hip for the recurrences); per-slot state st[2*slot + parity]
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(VB) void kv_mr_init(const VTile *__restrict__ vt,
                                                 const SlotDev *__restrict__ slots,
                                                 const int *__restrict__ gate,
                                                 const int *__restrict__ jac,
                                                 double *__restrict__ part)
{
    VT_PROLOGUE
    __shared__ double red[VB / 64];
    const bool useM = jac[t.slot] != 0;
    const double *__restrict__ b = S.vec[BG], *__restrict__ m = S.vec[BMINV];
    double *__restrict__ r1 = S.vec[BR1], *__restrict__ r2 = S.vec[BR2];
    double *__restrict__ y = S.vec[BY];
    double s = 0.0;
    for (int i = i0; i < i1; i += VB) {
        const double bi = b[i];
        const double yi = useM ? m[i] * bi : bi;
        r1[i] = bi;
        r2[i] = bi;
        y[i] = yi;
        s += bi * yi;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(VB) void kv_mr_start(const VTile *__restrict__ vt,
                                                  const SlotDev *__restrict__ slots,
                                                  const int *__restrict__ gate,
                                                  const SlotRange *__restrict__ rg,
                                                  const double *__restrict__ part,
                                                  const int *__restrict__ maxit,
                                                  const double *__restrict__ rtol,
                                                  BState *__restrict__ st,
                                                  int *__restrict__ run, SlotDev *wslots)
{
    VT_PROLOGUE
    __shared__ double red[VB / 64];
    const SlotRange r = rg[t.slot];
    const double bb = seg_sum(part, r.vbegin, r.vcount, red);
    const double b1 = sqrt(fmax(bb, 0.0));
    const double *__restrict__ y = S.vec[BY];
    // z_{-1} = M^{-1} b, unscaled (the first Lanczos vector is z_{-1} / beta1)
    double *__restrict__ v = S.vec[BZ0], *__restrict__ x = S.vec[BDX];
    double *__restrict__ w = S.vec[BW];
    double *__restrict__ w1 = S.vec[BW1], *__restrict__ w2 = S.vec[BW2];
    double *__restrict__ zb = S.bank;  // bank vector 0 = z_{-1}, else BZ0
    for (int i = i0; i < i1; i += VB) {
        x[i] = 0.0;
        if (zb) {
            zb[i] = y[i];
        } else {
            v[i] = y[i];
            w[i] = 0.0;
            w1[i] = 0.0;
            w2[i] = 0.0;
        }
    }
    if (t.start == 0 && threadIdx.x == 0) {
        BState o;
        o.beta1 = b1;
        o.beta = b1;
        o.oldb = 0.0;
        o.dbar = 0.0;
        o.eps = 0.0;
        o.phibar = b1;
        o.cs = -1.0;
        o.sn = 0.0;
        o.rtol = rtol[t.slot];
        o.j = 0;
        o.maxit = maxit[t.slot];
        o.stop = (b1 > 0.0 && bb >= 0.0) ? 0x7fffffff : -1;
        o.indefinite = bb < 0.0 ? 1 : 0;
        o.first = 1;
        o.pad = 0;
        st[2 * t.slot] = o;
        st[2 * t.slot + 1] = o;
        run[t.slot] = bs_skip(o) ? 0 : 1;
        wslots[t.slot].vec[BZIN] = zb ? zb : v;
    }
}

// Update of iteration si.j (Givens rotation) from the state before it and
// the slot's partials of alpha_j and beta_{j+1}^2.
struct BUpd {
    BState o;
    double ig, oldeps, delta, phi;
};

__device__ inline BUpd bs_update(const BState &si, double alpha, double bb)
{
    BUpd u;
    const double beta = sqrt(fmax(bb, 0.0));
    u.oldeps = si.eps;
    u.delta = si.cs * si.dbar + si.sn * alpha;
    const double gbar = si.sn * si.dbar - si.cs * alpha;
    const double gamma = fmax(hypot(gbar, beta), 2.2250738585072014e-308);
    const double cs = gbar / gamma, sn = beta / gamma;
    u.phi = cs * si.phibar;
    u.ig = 1.0 / gamma;
    BState o = si;
    o.oldb = si.beta;
    o.beta = beta;
    o.eps = si.sn * beta;
    o.dbar = -si.cs * beta;
    o.cs = cs;
    o.sn = sn;
    o.phibar = sn * si.phibar;
    if (bb < 0.0) o.indefinite = 1;
    if (o.phibar <= si.rtol * si.beta1 || beta == 0.0) o.stop = si.j;
    o.j = si.j + 1;
    u.o = o;
    return u;
}

// One lockstep position, after the element kernel ran on z_{j-1} (the
// Lanczos vector v_j = z_{j-1} / beta_j is never written).  Per slot: the
// deferred update of the iteration before (state st[par^1] -> st[par]):
//   w' = (z_{j-2}/beta_{j-1} - oldeps w1 - delta w2)/gamma;  x += phi w'
// then, while the slot runs, hv = G^T eV / beta_j (fixed DoFs: v_j)
// - (beta_j/beta_{j-1}) r1 in place of r1 and the partials of <v_j, hv>.
// Every iterating slot writes its state (carried forward when nothing runs)
// and its run flag.  A slot with resident Lanczos vectors records the
// update's scalars instead of applying it (kv_mr_finish forms dx).
template <int DIM, typename ET>
__global__ __launch_bounds__(VB) void kv_mr_gather_upd(
    const VTile *__restrict__ vt, const SlotDev *__restrict__ slots, const int *__restrict__ gate,
    const SlotRange *__restrict__ rg, BState *__restrict__ st, int par,
    const double *__restrict__ p1prev, const double *__restrict__ p2, int vr1, int vzc, int vzp,
    int vw1, int vw2, int vwout, double *__restrict__ part, int pbase, int *__restrict__ run)
{
    VT_PROLOGUE
    __shared__ double red[VB / 64];
    const BState sp = st[2 * t.slot + (par ^ 1)];
    const bool upd = !sp.first && !bs_skip(sp);
    BUpd u{};
    u.o = sp;
    if (upd) {
        const SlotRange r = rg[t.slot];
        const double alpha = seg_sum(p1prev, r.vbegin, r.vcount, red);
        const double bb = seg_sum(p2, r.vbegin, r.vcount, red);
        u = bs_update(sp, alpha, bb);
    }
    u.o.first = 0;
    const bool gat = !bs_skip(u.o);
    const bool res = S.bank != nullptr;
    const double sprev = sp.beta > 0.0 ? 1.0 / sp.beta : 0.0;
    if (t.start == 0 && threadIdx.x == 0) {
        st[2 * t.slot + par] = u.o;
        run[t.slot] = gat ? 1 : 0;
        if (upd && res) {
            double *h = S.hist + 8 * sp.j;
            h[0] = u.ig;
            h[1] = u.oldeps;
            h[2] = u.delta;
            h[3] = u.phi;
            h[4] = sprev;
        }
    }
    const bool vupd = upd && !res;
    if (!vupd && !gat) return;
    const Geom &g = S.g;
    const ET *__restrict__ eV = (const ET *)S.eV;
    const double sc = u.o.beta > 0.0 ? 1.0 / u.o.beta : 0.0;
    const double cr = u.o.j >= 1 ? u.o.beta / u.o.oldb : 0.0;
    // the element kernel's input, z_{j-1} (vzc names its buffer when the
    // slot has no bank)
    const double *__restrict__ zc = S.vec[BZIN], *__restrict__ zp = S.vec[vzp];
    const double *__restrict__ w1 = S.vec[vw1], *__restrict__ w2 = S.vec[vw2];
    double *__restrict__ r1 = S.vec[vr1], *__restrict__ x = S.vec[BDX];
    double *__restrict__ wo = S.vec[vwout];
    if (vupd)
        for (int i = i0; i < i1; i += VB) {
            const double wn = (sprev * zp[i] - u.oldeps * w1[i] - u.delta * w2[i]) * u.ig;
            wo[i] = wn;
            x[i] += u.phi * wn;
        }
    if (!gat) return;
    // G^T with one lane per node for all components (the copy positions are
    // worked out once per node and the loads of every component are in
    // flight together): the slot's nodes are split evenly over its vector
    // tiles (the tiles of a slot are consecutive VCH-DoF chunks from 0)
    double acc = 0.0;
    const int ntile = (DIM * g.nx + VCH - 1) / VCH, jt = t.start / VCH;
    const int npt = (g.nx + ntile - 1) / ntile;
    const int nb = jt * npt, ne = nb + npt < g.nx ? nb + npt : g.nx;
    for (int node = nb + (int)threadIdx.x; node < ne; node += VB) {
        int gc[3];
        box_coords<DIM>(g, node, gc);
        ET sv[DIM];
        gather_box_all<DIM, ET>(g, eV, gc, sv);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const size_t i = (size_t)c * g.nx + node;
            const double vi = sc * zc[i];
            double h = is_fixed(g, c, node, gc[0], gc[1], gc[2]) ? vi : sc * (double)sv[c];
            if (u.o.j >= 1) h -= cr * r1[i];
            r1[i] = h;
            acc += vi * h;
        }
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[pbase + blockIdx.x] = acc;
}

__global__ __launch_bounds__(VB) void kv_mr_l2(const VTile *__restrict__ vt,
                                               const SlotDev *__restrict__ slots,
                                               const int *__restrict__ gate,
                                               const SlotRange *__restrict__ rg,
                                               const int *__restrict__ jac,
                                               const BState *__restrict__ st, int par,
                                               const double *__restrict__ part1, int vhv, int vr2,
                                               int vz, double *__restrict__ part2,
                                               SlotDev *wslots)
{
    VT_PROLOGUE
    const BState &s = st[2 * t.slot + par];
    if (bs_skip(s)) return;
    __shared__ double red[VB / 64];
    const SlotRange r = rg[t.slot];
    const double alpha = seg_sum(part1, r.vbegin, r.vcount, red);
    const double c = alpha / s.beta;
    const bool useM = jac[t.slot] != 0;
    const double *__restrict__ m = S.vec[BMINV], *__restrict__ r2 = S.vec[vr2];
    // z_j to bank vector j + 1 (j < maxit here, and the bank holds maxit + 1),
    // else to the buffer vz; it is the next element kernel's input
    double *__restrict__ z = S.bank ? S.bank + (long)(s.j + 1) * S.bstride : S.vec[vz];
    double *__restrict__ hv = S.vec[vhv];
    if (t.start == 0 && threadIdx.x == 0) wslots[t.slot].vec[BZIN] = z;
    double acc = 0.0;
    for (int i = i0; i < i1; i += VB) {
        const double h = hv[i] - c * r2[i];
        hv[i] = h;
        const double zi = useM ? m[i] * h : h;
        z[i] = zi;
        acc += h * zi;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part2[blockIdx.x] = acc;
}

// The deferred update of the last iteration of every slot still running
// after the lockstep loop (state st[par] -> st[par^1]); every slot's run flag
// is cleared (the element kernels of later MINRES calls are gated by it).
// A slot with resident Lanczos vectors then forms dx = sum_m c_m z_m from
// the recorded scalars: lane m runs the three-term w recurrence on the m-th
// coefficients (as k_mr_combine), every tile of the slot alike.
__global__ __launch_bounds__(VB) void kv_mr_finish(const VTile *__restrict__ vt,
                                                   const SlotDev *__restrict__ slots,
                                                   const int *__restrict__ gate,
                                                   const SlotRange *__restrict__ rg,
                                                   BState *__restrict__ st, int par,
                                                   const double *__restrict__ p1,
                                                   const double *__restrict__ p2, int vzp,
                                                   int vw1, int vw2, int vwout,
                                                   int *__restrict__ run)
{
    VT_PROLOGUE
    __shared__ double red[VB / 64];
    static_assert(MR_MAX_BASIS <= VB, "one lane per coefficient");
    __shared__ double hig[MR_MAX_BASIS], hoe[MR_MAX_BASIS], hde[MR_MAX_BASIS],
        hph[MR_MAX_BASIS], coef[MR_MAX_BASIS];
    const BState sp = st[2 * t.slot + par];
    if (t.start == 0 && threadIdx.x == 0) run[t.slot] = 0;
    const bool res = S.bank != nullptr;
    const bool last = !sp.first && !bs_skip(sp);
    if (!last) {
        if (t.start == 0 && threadIdx.x == 0) st[2 * t.slot + (par ^ 1)] = sp;
        if (!res || sp.first) return;
    }
    const double sprev = sp.beta > 0.0 ? 1.0 / sp.beta : 0.0;
    BUpd u{};
    u.o = sp;
    if (last) {
        const SlotRange r = rg[t.slot];
        const double alpha = seg_sum(p1, r.vbegin, r.vcount, red);
        const double bb = seg_sum(p2, r.vbegin, r.vcount, red);
        u = bs_update(sp, alpha, bb);
        if (t.start == 0 && threadIdx.x == 0) st[2 * t.slot + (par ^ 1)] = u.o;
    }
    if (res) {
        // updates 0..K-1 taken (the last one here when `last`)
        const int K = last ? sp.j + 1 : sp.j;
        const int tm = threadIdx.x;
        double svt = 0.0;
        if (tm < K) {
            if (last && tm == sp.j) {
                hig[tm] = u.ig;
                hoe[tm] = u.oldeps;
                hde[tm] = u.delta;
                hph[tm] = u.phi;
                svt = sprev;
            } else {
                const double *h = S.hist + 8 * tm;
                hig[tm] = h[0];
                hoe[tm] = h[1];
                hde[tm] = h[2];
                hph[tm] = h[3];
                svt = h[4];
            }
        }
        __syncthreads();
        if (tm < K) {
            double a2 = 0.0, a1 = 0.0, cf = 0.0;
            for (int m = tm; m < K; ++m) {
                const double wn = ((m == tm ? 1.0 : 0.0) - hoe[m] * a2 - hde[m] * a1) * hig[m];
                cf += hph[m] * wn;
                a2 = a1;
                a1 = wn;
            }
            coef[tm] = cf * svt;
        }
        __syncthreads();
        const double *__restrict__ zb = S.bank;
        double *__restrict__ x = S.vec[BDX];
        const long bs = S.bstride;
        for (int i = i0; i < i1; i += VB) {
            // four vectors' loads in flight per step, summed in the order of m
            double acc = 0.0;
            int m = 0;
            for (; m + 4 <= K; m += 4) {
                const double z0 = zb[(long)m * bs + i], z1 = zb[(long)(m + 1) * bs + i];
                const double z2 = zb[(long)(m + 2) * bs + i], z3 = zb[(long)(m + 3) * bs + i];
                acc += coef[m] * z0;
                acc += coef[m + 1] * z1;
                acc += coef[m + 2] * z2;
                acc += coef[m + 3] * z3;
            }
            for (; m < K; ++m) acc += coef[m] * zb[(long)m * bs + i];
            x[i] = acc;
        }
        return;
    }
    const double *__restrict__ zp = S.vec[vzp];
    const double *__restrict__ w1 = S.vec[vw1], *__restrict__ w2 = S.vec[vw2];
    double *__restrict__ x = S.vec[BDX], *__restrict__ wo = S.vec[vwout];
    for (int i = i0; i < i1; i += VB) {
        const double wn = (sprev * zp[i] - u.oldeps * w1[i] - u.delta * w2[i]) * u.ig;
        wo[i] = wn;
        x[i] += u.phi * wn;
    }
}

// ---------------------------------------------------------------------------
// Newton step decisions on the device (Sec. 2.3), for the whole-step graph:
// one thread per slot.  The host mirror of NState is uploaded before a step
// and read back after it; in between the line search (accept a trial when
// det A > 0 at every point, F_t < 1.2 F and |g_t| < 1.2 |g|, else halve
// alpha) and the stop test run here, with the same comparisons the host
// makes in the eager step.
// ---------------------------------------------------------------------------
struct NState {
    double F, gn, g0, tol, alpha, Ft;
    int newton_its, max_newton, minres_its, halvings, max_halvings, status, phase, searching;
};
enum { NS_ITER = 1, NS_DONE = 2 };

// after MINRES: iteration count, breakdown check, alpha = 1 and the search gate
__global__ __launch_bounds__(VB) void kn_after_minres(int M, const int *__restrict__ gate,
                                                      const BState *__restrict__ st,
                                                      NState *__restrict__ ns,
                                                      int *__restrict__ search,
                                                      double *__restrict__ sc)
{
    const int s = blockIdx.x * VB + threadIdx.x;
    if (s >= M) return;
    search[s] = 0;
    if (!gate[s]) return;
    const BState &a = st[2 * s], &b = st[2 * s + 1];
    const BState &f = a.j >= b.j ? a : b;
    NState &n = ns[s];
    n.minres_its += f.j;
    n.alpha = 1.0;
    sc[s * NSC + SC_ALPHA] = 1.0;
    if (f.indefinite) {
        n.status = TMOP_ERR_NONFINITE;
        n.phase = NS_DONE;
        return;
    }
    n.searching = 1;
    search[s] = 1;
}

// trial energy test: det A > 0 at every point and F_t < 1.2 F
__global__ __launch_bounds__(VB) void kn_ls_trial(int M, const int *__restrict__ search,
                                                  const double *__restrict__ sc,
                                                  NState *__restrict__ ns, int *__restrict__ ftest)
{
    const int s = blockIdx.x * VB + threadIdx.x;
    if (s >= M) return;
    ftest[s] = 0;
    if (!search[s]) return;
    const double *c = sc + s * NSC;
    NState &n = ns[s];
    n.Ft = c[SC_F];
    ftest[s] = (c[SC_BAD] == 0.0 && c[SC_MD] > 0.0 && c[SC_F] < 1.2 * n.F) ? 1 : 0;
}

// gradient test |g_t| < 1.2 |g| and the decision of round h: accept (the
// copies x_t -> x, g_t -> g follow, gated by acc) or halve alpha; a slot out
// of halvings ends with TMOP_ERR_LINESEARCH
__global__ __launch_bounds__(VB) void kn_ls_decide(int M, int h, int *__restrict__ search,
                                                   const int *__restrict__ ftest,
                                                   double *__restrict__ sc, NState *__restrict__ ns,
                                                   int *__restrict__ acc)
{
    const int s = blockIdx.x * VB + threadIdx.x;
    if (s >= M) return;
    acc[s] = 0;
    if (!search[s]) return;
    NState &n = ns[s];
    if (ftest[s]) {
        const double gtn = sqrt(sc[s * NSC + SC_DOT]);
        if (gtn < 1.2 * n.gn) {
            n.F = n.Ft;
            n.gn = gtn;
            n.newton_its++;
            n.searching = 0;
            search[s] = 0;
            acc[s] = 1;
            return;
        }
    }
    n.halvings++;
    n.alpha *= 0.5;
    sc[s * NSC + SC_ALPHA] = n.alpha;
    if (h >= n.max_halvings) {
        n.searching = 0;
        search[s] = 0;
        n.status = TMOP_ERR_LINESEARCH;
        n.phase = NS_DONE;
    }
}

// stop test of the slots that finished their line search this step
__global__ __launch_bounds__(VB) void kn_end(int M, const int *__restrict__ gate, NState *__restrict__ ns)
{
    const int s = blockIdx.x * VB + threadIdx.x;
    if (s >= M || !gate[s]) return;
    NState &n = ns[s];
    if (n.phase != NS_ITER || n.searching) return;
    if (n.F == 0.0 || n.gn <= n.tol * n.g0) {
        n.status = TMOP_OK;
        n.phase = NS_DONE;
    } else if (n.newton_its >= n.max_newton) {
        n.status = TMOP_ERR_NOT_CONVERGED;
        n.phase = NS_DONE;
    }
}

}  // namespace tmop

// ===========================================================================
// Host engine
// ===========================================================================

using namespace tmop;

namespace {

thread_local std::string g_perr;

int pfail(int code, const std::string &m)
{
    g_perr = m;
    return code;
}

#define PHIP(call)                                                                           \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return pfail(e_ == hipErrorOutOfMemory ? TMOP_ERR_OOM : TMOP_ERR_HIP,            \
                         std::string(#call) + ": " + hipGetErrorString(e_));                 \
    } while (0)

#define PCHK(call)                    \
    do {                              \
        int r_ = (call);              \
        if (r_ != TMOP_OK) return r_; \
    } while (0)

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// a kernel class: slots with the limiting term (lim = 1) launch their own
// kernel variants
struct ClassKey {
    int dim, p, nq, storage, prec, lim;
    bool operator<(const ClassKey &o) const
    {
        return std::tie(dim, p, nq, storage, prec, lim) <
               std::tie(o.dim, o.p, o.nq, o.storage, o.prec, o.lim);
    }
};

struct ClassH {
    ClassKey key{};
    BOps bops{};
    Tables tb{};
    std::vector<Tile> tiles;
    Tile *d_tiles = nullptr;
    int cap = 0;
    int pbase = 0;
    // Hessian action tile shape (index into BOps::epb_t) and, when it is not
    // the base shape, its own tile list
    int tile = 1;
    std::vector<Tile> atiles;
    Tile *d_atiles = nullptr;
    int acap = 0;
};

enum { PH_NEW = 0, PH_ITER = 1, PH_DONE = 2 };

struct SlotH {
    bool used = false;
    int dim = 0, p = 0, nq = 0, storage = 0, prec = 0;
    int lim = 0;  // the slot carries the limiting term
    int ne = 0, nx = 0, ndof = 0, nqe = 0, np = 0, S = 0;
    size_t off = 0, bytes = 0;
    SlotDev dev{};
    tmop_solve_params sp{};
    int phase = PH_NEW;
    int status = TMOP_OK;
    double F = 0, F0 = 0, gn = 0, g0 = 0, alpha = 1.0;
    int newton_its = 0, minres_its = 0, halvings = 0;
    bool h_ready = false;  // the slot's quadrature data holds a Hessian setup
    double t_start = 0, t_done = 0;
    int first_vt = 0, nvt = 0;
};

}  // namespace

// sizes of one request (mesh + params); returns false if invalid
static int request_sizes(const tmop_mesh_desc *m, const tmop_params *prm, SlotH &s, std::string &why)
{
    if (!m || !prm) {
        why = "null mesh or params";
        return TMOP_ERR_INVALID_ARG;
    }
    if (m->elem_to_node) {
        why = "pooled solves take structured boxes (elem_to_node must be NULL)";
        return TMOP_ERR_UNSUPPORTED;
    }
    if (m->dim != 2 && m->dim != 3) {
        why = "dim must be 2 or 3";
        return TMOP_ERR_INVALID_ARG;
    }
    if (!metric_supported(m->dim, prm->metric)) {
        why = "metric must be 2, 7, 9 or 55 (dim 2) or 303 or 55 (dim 3)";
        return TMOP_ERR_UNSUPPORTED;
    }
    if (m->ess_mode == TMOP_ESS_MASK && !m->ess_mask) {
        why = "TMOP_ESS_MASK needs ess_mask";
        return TMOP_ERR_INVALID_ARG;
    }
    const int d = m->dim, p = m->order_p;
    if (p < 1 || p > 4 || m->nx <= 0 || m->ny <= 0 || (d == 3 && m->nz <= 0)) {
        why = "order 1..4 and positive element counts required";
        return TMOP_ERR_INVALID_ARG;
    }
    s.dim = d;
    s.p = p;
    s.nq = prm->nq1d;
    if (prm->quad_rule != TMOP_QUAD_GL) {
        why = "pooled solves use Gauss-Legendre quadrature (quad_rule = TMOP_QUAD_GL)";
        return TMOP_ERR_UNSUPPORTED;
    }
    s.storage = prm->hess_storage == TMOP_HESS_COMPACT ? 1 : 0;
    s.prec = prm->precision == TMOP_MIXED ? 1 : 0;
    const long ne = (long)m->nx * m->ny * (d == 3 ? m->nz : 1);
    const long nx = (long)(m->nx * p + 1) * (m->ny * p + 1) * (d == 3 ? (m->nz * p + 1) : 1);
    if (ne * (long)(p + 1) * (p + 1) * (p + 1) * 3 > 0x7fffffffL || nx * 3 > 0x7fffffffL) {
        why = "mesh too large";
        return TMOP_ERR_INVALID_ARG;
    }
    s.ne = (int)ne;
    s.nx = (int)nx;
    s.ndof = (int)(d * nx);
    s.nqe = d == 3 ? s.nq * s.nq * s.nq : s.nq * s.nq;
    s.np = d == 3 ? (p + 1) * (p + 1) * (p + 1) : (p + 1) * (p + 1);
    s.S = s.storage ? (d == 3 ? 13 : 8) : d * d * (d * d + 1) / 2;
    const size_t tb = s.prec ? 4 : 8;
    s.bytes = BNV * up256((size_t)s.ndof * 8) + up256((size_t)s.ne * qdata_stride(s.S, s.nqe, (int)tb) * tb) +
              up256((size_t)s.ne * d * s.np * 8);
    // the pool keeps its own copy of a caller's mask of fixed DoFs
    if (m->ess_mode == TMOP_ESS_MASK) s.bytes += up256((size_t)s.ndof);
    return TMOP_OK;
}


// Bytes of a slot's resident Lanczos vectors (max_minres + 1 of them) and
// per-update scalars; 0 when MINRES may run more updates than one
// combination takes.
static size_t bank_bytes_of(int ndof, int max_minres)
{
    const int kb = max_minres + 1;
    if (kb < 1 || kb > MR_MAX_BASIS) return 0;
    return (size_t)kb * up256((size_t)ndof * 8) + up256((size_t)MR_MAX_BASIS * 64);
}

struct tmop_pool {
    hipStream_t s = nullptr;
    bool own_stream = false;  // the pool created s (else it is the caller's)
    size_t budget = 0, used = 0;
    int max_slots = 0;
    char *arena = nullptr;
    std::map<size_t, size_t> free_;  // offset -> size
    std::vector<SlotH> slots;
    std::map<ClassKey, ClassH> classes;
    // device tables
    SlotDev *d_slots = nullptr;
    SlotRange *d_rg = nullptr;
    VTile *d_vt = nullptr;
    int vt_cap = 0;
    double *d_part = nullptr;
    size_t part_cap = 0;
    double *d_sc = nullptr;
    BState *d_st = nullptr;
    int *d_run = nullptr, *d_jac = nullptr, *d_maxit = nullptr;
    double *d_rtol = nullptr, *h_rtol = nullptr;  // per-slot MINRES tolerance
    // gates: 0 new slots, 1 iterating, 2 searching, 3 trial accepted so far,
    // 4 host staging of the iteration caps, 5 tmop_pool_evaluate's one slot
    int *d_gate[6] = {};
    int *h_gate[6] = {};
    double *h_sc = nullptr;
    BState *h_st = nullptr;
    int *h_int = nullptr;
    // layout
    std::vector<VTile> vts;
    std::vector<SlotRange> rg;
    int vt_range[4][2] = {};  // [dim3 fp64, dim3 mixed, dim2 fp64, dim2 mixed] -> [begin, count]
    int epart = 0;            // element partials (3 planes per class)
    bool dirty = true;
    // resident MINRES Lanczos vectors for slots whose region fits the budget
    // (opt-in: such a slot takes more of the budget)
    bool use_bank = false;
    // HIP graphs: 0 none, 1 a block of six MINRES iterations replayed,
    // 2 the whole Newton step (setup, diagonal, every MINRES iteration, the
    // first LS_ROUNDS line-search rounds and the stop test) replayed once
    // per step
    int graph_mode = 1;
    bool graph_ok = false;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    bool sgraph_ok = false;
    int sg_maxj = -1;
    hipGraphExec_t sgexec = nullptr;
    hipGraph_t sgraph = nullptr;
    // per-slot Newton state on the device (graph mode 2) and its host mirror;
    // gates of the device line search
    NState *d_ns = nullptr, *h_ns = nullptr;
    int *d_search = nullptr, *d_ftest = nullptr, *d_acc = nullptr;
};

// line-search rounds inside the whole-step graph; a slot still searching
// after them continues in rounds launched one by one
constexpr int LS_ROUNDS = 2;

static void pool_free_region(tmop_pool *P, size_t off, size_t bytes)
{
    // insert and merge
    auto it = P->free_.emplace(off, bytes).first;
    if (it != P->free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            P->free_.erase(it);
            it = pv;
        }
    }
    auto nx = std::next(it);
    if (nx != P->free_.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        P->free_.erase(nx);
    }
}

static bool pool_alloc_region(tmop_pool *P, size_t bytes, size_t *off)
{
    for (auto it = P->free_.begin(); it != P->free_.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes, noff = it->first + bytes;
            P->free_.erase(it);
            if (rest) P->free_.emplace(noff, rest);
            return true;
        }
    }
    return false;
}

static int upload_gate(tmop_pool *P, int k)
{
    PHIP(hipMemcpyAsync(P->d_gate[k], P->h_gate[k], sizeof(int) * P->max_slots,
                        hipMemcpyHostToDevice, P->s));
    return TMOP_OK;
}

static void invalidate_graph(tmop_pool *P)
{
    if (P->gexec) hipGraphExecDestroy(P->gexec);
    if (P->graph) hipGraphDestroy(P->graph);
    P->gexec = nullptr;
    P->graph = nullptr;
    P->graph_ok = false;
    if (P->sgexec) hipGraphExecDestroy(P->sgexec);
    if (P->sgraph) hipGraphDestroy(P->sgraph);
    P->sgexec = nullptr;
    P->sgraph = nullptr;
    P->sgraph_ok = false;
    P->sg_maxj = -1;
}

// Rebuild tile lists, vector tiles, ranges and partial layout for the used slots.
static int pool_rebuild(tmop_pool *P)
{
    invalidate_graph(P);
    for (auto &kv : P->classes) {
        kv.second.tiles.clear();
        kv.second.atiles.clear();
    }
    // element tiles per class
    for (int si = 0; si < P->max_slots; ++si) {
        SlotH &s = P->slots[si];
        if (!s.used) continue;
        ClassKey k{s.dim, s.p, s.nq, s.storage, s.prec, s.lim};
        auto it = P->classes.find(k);
        if (it == P->classes.end()) {
            ClassH c;
            c.key = k;
            if (!find_bops(s.dim, s.p, s.nq, &c.bops))
                return pfail(TMOP_ERR_UNSUPPORTED, "no kernel for this (dim, p, nq1d)");
            if (internal_tables(s.p, s.nq, &c.tb) != TMOP_OK)
                return pfail(TMOP_ERR_INVALID_ARG, "bad order / quadrature");
            // start from the tile shape recorded for the class by the autotuner
            // (classes with the limiting term keep the base shape)
            const int tt = tuned_tile(s.dim, s.p, s.nq, s.storage ? TMOP_HESS_COMPACT : TMOP_HESS_TENSOR,
                                      s.prec ? TMOP_MIXED : TMOP_FP64);
            if (!s.lim && tt >= 0 && c.bops.epb_t[tt] > 0) c.tile = tt;
            it = P->classes.emplace(k, c).first;
        }
        ClassH &c = it->second;
        for (int e = 0; e < s.ne; e += c.bops.epb) c.tiles.push_back(Tile{si, e});
        if (c.tile != 1)
            for (int e = 0; e < s.ne; e += c.bops.epb_t[c.tile]) c.atiles.push_back(Tile{si, e});
    }
    int pb = 0;
    P->rg.assign(P->max_slots, SlotRange{0, 0, 1, 0, 0});
    for (auto &kv : P->classes) {
        ClassH &c = kv.second;
        c.pbase = pb;
        const int nt = (int)c.tiles.size();
        if (nt > c.cap) {
            hipFree(c.d_tiles);
            c.d_tiles = nullptr;
            c.cap = std::max(nt, 2 * c.cap);
            PHIP(hipMalloc((void **)&c.d_tiles, sizeof(Tile) * c.cap));
        }
        if (nt) PHIP(hipMemcpyAsync(c.d_tiles, c.tiles.data(), sizeof(Tile) * nt, hipMemcpyHostToDevice, P->s));
        const int na = (int)c.atiles.size();
        if (na > c.acap) {
            hipFree(c.d_atiles);
            c.d_atiles = nullptr;
            c.acap = std::max(na, 2 * c.acap);
            PHIP(hipMalloc((void **)&c.d_atiles, sizeof(Tile) * c.acap));
        }
        if (na) PHIP(hipMemcpyAsync(c.d_atiles, c.atiles.data(), sizeof(Tile) * na, hipMemcpyHostToDevice, P->s));
        for (int t = 0; t < nt; ++t) {
            SlotRange &r = P->rg[c.tiles[t].slot];
            if (r.ecount == 0) {
                r.ebase = pb + t;
                r.estride = nt;
            }
            r.ecount++;
        }
        pb += 3 * nt;
    }
    P->epart = pb;
    // vector tiles grouped as (3D fp64, 3D mixed, 2D fp64, 2D mixed)
    P->vts.clear();
    for (int grp = 0; grp < 4; ++grp) {
        const int gd = grp < 2 ? 3 : 2, gp = grp & 1;
        P->vt_range[grp][0] = (int)P->vts.size();
        for (int si = 0; si < P->max_slots; ++si) {
            SlotH &s = P->slots[si];
            if (!s.used || s.dim != gd || s.prec != gp) continue;
            s.first_vt = (int)P->vts.size();
            for (int st = 0; st < s.ndof; st += VCH)
                P->vts.push_back(VTile{si, st, std::min(VCH, s.ndof - st)});
            s.nvt = (int)P->vts.size() - s.first_vt;
            P->rg[si].vbegin = s.first_vt;
            P->rg[si].vcount = s.nvt;
        }
        P->vt_range[grp][1] = (int)P->vts.size() - P->vt_range[grp][0];
    }
    const int nvt = (int)P->vts.size();
    if (nvt > P->vt_cap) {
        hipFree(P->d_vt);
        P->d_vt = nullptr;
        P->vt_cap = std::max(nvt, 2 * P->vt_cap);
        PHIP(hipMalloc((void **)&P->d_vt, sizeof(VTile) * P->vt_cap));
    }
    if (nvt) PHIP(hipMemcpyAsync(P->d_vt, P->vts.data(), sizeof(VTile) * nvt, hipMemcpyHostToDevice, P->s));
    const size_t need = (size_t)P->epart + 3 * (size_t)nvt + 64;
    if (need > P->part_cap) {
        hipFree(P->d_part);
        P->d_part = nullptr;
        P->part_cap = std::max(need, 2 * P->part_cap);
        PHIP(hipMalloc((void **)&P->d_part, sizeof(double) * P->part_cap));
    }
    PHIP(hipMemcpyAsync(P->d_rg, P->rg.data(), sizeof(SlotRange) * P->max_slots, hipMemcpyHostToDevice, P->s));
    PHIP(hipStreamSynchronize(P->s));
    P->dirty = false;
    return TMOP_OK;
}

// --- batched phase launchers ------------------------------------------------

static double *vpart1(tmop_pool *P) { return P->d_part + P->epart; }
static double *vpart2(tmop_pool *P) { return P->d_part + P->epart + P->vts.size(); }
// the first-Lanczos partials alternate between lockstep positions (a position
// reads the previous one's while writing its own)
static double *vpart1_at(tmop_pool *P, int par)
{
    return par ? P->d_part + P->epart + 2 * P->vts.size() : vpart1(P);
}

// One element kernel over every class's tiles: which = 0 energy, 1 gradient,
// 2 setup, 3 Hessian action, 4 diagonal, 5 gradient with the energy partials.
static void launch_elem(tmop_pool *P, int which, const int *gate, int vin)
{
    for (auto &kv : P->classes) {
        ClassH &c = kv.second;
        const int nt = (int)c.tiles.size();
        if (!nt) continue;
        const int st = c.key.storage, pr = c.key.prec;
        if (c.key.lim) {
            BLaunch f = which == 0   ? c.bops.energyL
                        : which == 1 ? c.bops.gradientL
                        : which == 2 ? c.bops.setup[st][pr]
                        : which == 3 ? c.bops.applyL[st][pr]
                        : which == 4 ? c.bops.diagL[st][pr]
                                     : c.bops.gradientEL;
            f(nt, P->s, c.tb, c.d_tiles, P->d_slots, gate, vin, P->d_part + c.pbase);
            continue;
        }
        if (which == 3 && c.tile != 1) {
            c.bops.apply_t[st][pr][c.tile]((int)c.atiles.size(), P->s, c.tb, c.d_atiles, P->d_slots,
                                          gate, vin, nullptr);
            continue;
        }
        BLaunch f = which == 0   ? c.bops.energy
                    : which == 1 ? c.bops.gradient
                    : which == 2 ? c.bops.setup[st][pr]
                    : which == 3 ? c.bops.apply[st][pr]
                    : which == 4 ? c.bops.diag[st][pr]
                                 : c.bops.gradientE;
        f(nt, P->s, c.tb, c.d_tiles, P->d_slots, gate, vin, P->d_part + c.pbase);
    }
}

static void launch_gather(tmop_pool *P, const int *gate, int vout, int fix_mode, int vsrc, bool ev32)
{
    for (int grp = 0; grp < 4; ++grp) {
        const int b = P->vt_range[grp][0], n = P->vt_range[grp][1];
        if (!n) continue;
        const bool f32 = ev32 && (grp & 1);
        const VTile *vt = P->d_vt + b;
        if (grp < 2) {
            if (f32)
                hipLaunchKernelGGL((kv_gather<3, float>), dim3(n), dim3(VB), 0, P->s, vt, P->d_slots, gate, vout, fix_mode, vsrc);
            else
                hipLaunchKernelGGL((kv_gather<3, double>), dim3(n), dim3(VB), 0, P->s, vt, P->d_slots, gate, vout, fix_mode, vsrc);
        } else {
            if (f32)
                hipLaunchKernelGGL((kv_gather<2, float>), dim3(n), dim3(VB), 0, P->s, vt, P->d_slots, gate, vout, fix_mode, vsrc);
            else
                hipLaunchKernelGGL((kv_gather<2, double>), dim3(n), dim3(VB), 0, P->s, vt, P->d_slots, gate, vout, fix_mode, vsrc);
        }
    }
}

static int nvt_all(tmop_pool *P) { return (int)P->vts.size(); }

static void dot_to_sc(tmop_pool *P, const int *gate, int va, int vb, int which)
{
    const int n = nvt_all(P);
    if (!n) return;
    hipLaunchKernelGGL(kv_dot, dim3(n), dim3(VB), 0, P->s, P->d_vt, P->d_slots, gate, va, vb, vpart1(P));
    hipLaunchKernelGGL(kr_vec, dim3(P->max_slots), dim3(VB), 0, P->s, P->d_rg, gate, vpart1(P), 0, which, P->d_sc);
}

static void energy_to_sc(tmop_pool *P, const int *gate, int vin)
{
    launch_elem(P, 0, gate, vin);
    hipLaunchKernelGGL(kr_energy, dim3(P->max_slots), dim3(VB), 0, P->s, P->d_rg, gate, P->d_part, P->d_sc);
}

static void gradient_to(tmop_pool *P, const int *gate, int vin, int vout)
{
    launch_elem(P, 1, gate, vin);
    launch_gather(P, gate, vout, 0, vout, false);
}

// One element pass for both (the gradient kernel also sums the energy):
// F, min det and the bad count of the slots of gate ge into sc, their
// gradient E-vectors into the slots' eV; the gather of g into vout follows
// separately, for the slots that need it.
static void energy_grad_elem(tmop_pool *P, const int *ge, int vin)
{
    launch_elem(P, 5, ge, vin);
    hipLaunchKernelGGL(kr_energy, dim3(P->max_slots), dim3(VB), 0, P->s, P->d_rg, ge, P->d_part, P->d_sc);
}

static int read_sc(tmop_pool *P)
{
    PHIP(hipMemcpyAsync(P->h_sc, P->d_sc, sizeof(double) * NSC * P->max_slots, hipMemcpyDeviceToHost, P->s));
    PHIP(hipStreamSynchronize(P->s));
    return TMOP_OK;
}

// vector ids of lockstep position k: r1 (overwritten in place by hv) and r2
// swap every position, as do z_{j-1} (the element kernel's input) and
// z_{j-2} (overwritten by z_j); (w, w1, w2) of the update of iteration m
// rotate with period 3: W[m % 3]
static const int MR_W[3][3] = {{BW, BW1, BW2}, {BW1, BW2, BW}, {BW2, BW, BW1}};
static int mr_r1(int k) { return (k & 1) ? BR2 : BR1; }
static int mr_r2(int k) { return (k & 1) ? BR1 : BR2; }
static int mr_zc(int k) { return (k & 1) ? BZ1 : BZ0; }
static int mr_zp(int k) { return (k & 1) ? BZ0 : BZ1; }

// one lockstep MINRES iteration for all running slots (see vec.hip for the
// recurrences; here the update of iteration j - 1 runs in position j's gather)
static void minres_iter(tmop_pool *P, int k)
{
    const int r1 = mr_r1(k), r2 = mr_r2(k), zc = mr_zc(k), zp = mr_zp(k);
    const int *W = MR_W[(k + 2) % 3];  // update of iteration k - 1
    const int par = k & 1;
    double *p1 = vpart1_at(P, par);
    const double *p1prev = vpart1_at(P, par ^ 1);
    launch_elem(P, 3, P->d_run, BZIN);
    for (int grp = 0; grp < 4; ++grp) {
        const int b = P->vt_range[grp][0], n = P->vt_range[grp][1];
        if (!n) continue;
        const VTile *vt = P->d_vt + b;
        // formula (w1, w2) = (ids w2, w), new w into id w1
#define TMOP_KG(D, T)                                                                           \
    hipLaunchKernelGGL((kv_mr_gather_upd<D, T>), dim3(n), dim3(VB), 0, P->s, vt, P->d_slots,   \
                       P->d_gate[1], P->d_rg, P->d_st, par, p1prev, vpart2(P), r1, zc, zp,     \
                       W[2], W[0], W[1], p1, b, P->d_run);
        if (grp == 0)
            TMOP_KG(3, double)
        else if (grp == 1)
            TMOP_KG(3, float)
        else if (grp == 2)
            TMOP_KG(2, double)
        else
            TMOP_KG(2, float)
#undef TMOP_KG
    }
    const int n = nvt_all(P);
    // hv -> r2 of the next position (in place in r1); z_j into zp
    hipLaunchKernelGGL(kv_mr_l2, dim3(n), dim3(VB), 0, P->s, P->d_vt, P->d_slots, P->d_gate[1], P->d_rg, P->d_jac, P->d_st, par, p1, r1, r2, zp, vpart2(P), P->d_slots);
}

static int run_minres(tmop_pool *P, int maxj)
{
    const int nv = nvt_all(P);
    hipLaunchKernelGGL(kv_mr_init, dim3(nv), dim3(VB), 0, P->s, P->d_vt, P->d_slots, P->d_gate[1], P->d_jac, vpart1(P));
    // each slot's own iteration cap and tolerance (uploaded with the gates)
    hipLaunchKernelGGL(kv_mr_start, dim3(nv), dim3(VB), 0, P->s, P->d_vt, P->d_slots, P->d_gate[1], P->d_rg, vpart1(P), P->d_maxit, P->d_rtol, P->d_st, P->d_run, P->d_slots);
    int j = 0;
    while (j < maxj) {
        if (P->graph_mode == 1 && maxj - j >= 6) {
            if (!P->graph_ok) {
                PHIP(hipStreamBeginCapture(P->s, hipStreamCaptureModeThreadLocal));
                for (int k = 0; k < 6; ++k) minres_iter(P, k);
                PHIP(hipStreamEndCapture(P->s, &P->graph));
                PHIP(hipGraphInstantiate(&P->gexec, P->graph, nullptr, nullptr, 0));
                P->graph_ok = true;
            }
            PHIP(hipGraphLaunch(P->gexec, P->s));
            j += 6;
        } else {
            // the ids/parity of a partial block continue from position j % 6 == 0
            for (int k = 0; j < maxj && k < 6; ++k, ++j) minres_iter(P, k);
        }
        if (j < maxj && j % 12 == 0) {
            PHIP(hipMemcpyAsync(P->h_int, P->d_run, sizeof(int) * P->max_slots, hipMemcpyDeviceToHost, P->s));
            PHIP(hipStreamSynchronize(P->s));
            bool any = false;
            for (int si = 0; si < P->max_slots; ++si) any = any || (P->slots[si].used && P->h_int[si]);
            if (!any) break;
        }
    }
    if (j > 0) {
        // the deferred update of the last iteration run (position k = (j - 1) % 6,
        // whose element-kernel input z_{j-2} gives v_{j-1})
        const int k = (j - 1) % 6, par = k & 1;
        const int *W = MR_W[(j - 1) % 3];
        hipLaunchKernelGGL(kv_mr_finish, dim3(nv), dim3(VB), 0, P->s, P->d_vt, P->d_slots, P->d_gate[1], P->d_rg, P->d_st, par, vpart1_at(P, par), vpart2(P), mr_zc(k), W[2], W[0], W[1], P->d_run);
    }
    PHIP(hipMemcpyAsync(P->h_st, P->d_st, sizeof(BState) * 2 * P->max_slots, hipMemcpyDeviceToHost, P->s));
    PHIP(hipStreamSynchronize(P->s));
    PHIP(hipGetLastError());
    return TMOP_OK;
}

static void finish_slot(SlotH &s, int status)
{
    s.phase = PH_DONE;
    s.status = status;
    s.t_done = now_ms();
}

static int nblk(int n) { return (n + VB - 1) / VB; }

// one line-search round h of every searching slot, decided on the device
static void ls_round_device(tmop_pool *P, int h)
{
    const int M = P->max_slots, nv = nvt_all(P);
    hipLaunchKernelGGL(kv_step, dim3(nv), dim3(VB), 0, P->s, P->d_vt, P->d_slots, P->d_search, P->d_sc);
    energy_grad_elem(P, P->d_search, BXT);
    hipLaunchKernelGGL(kn_ls_trial, dim3(nblk(M)), dim3(VB), 0, P->s, M, P->d_search, P->d_sc, P->d_ns, P->d_ftest);
    launch_gather(P, P->d_ftest, BGT, 0, BGT, false);
    dot_to_sc(P, P->d_ftest, BGT, BGT, SC_DOT);
    hipLaunchKernelGGL(kn_ls_decide, dim3(nblk(M)), dim3(VB), 0, P->s, M, h, P->d_search, P->d_ftest, P->d_sc, P->d_ns, P->d_acc);
    hipLaunchKernelGGL(kv_copy, dim3(nv), dim3(VB), 0, P->s, P->d_vt, P->d_slots, P->d_acc, BXT, BX);
    hipLaunchKernelGGL(kv_copy, dim3(nv), dim3(VB), 0, P->s, P->d_vt, P->d_slots, P->d_acc, BGT, BG);
}

// The Newton step of every iterating slot (gate 1) as one stream of launches
// with no host decision: setup, Jacobi diagonal, maxj lockstep MINRES
// iterations (slots stop on the device), LS_ROUNDS line-search rounds and the
// stop test.  Captured once per layout and replayed.
static void record_step(tmop_pool *P, int maxj)
{
    const int M = P->max_slots, nv = nvt_all(P);
    const int *g1 = P->d_gate[1];
    launch_elem(P, 2, g1, BX);  // setup
    launch_elem(P, 4, g1, BX);  // diagonal
    launch_gather(P, g1, BDIAG, 1, BDIAG, false);
    hipLaunchKernelGGL(kv_absmax, dim3(nv), dim3(VB), 0, P->s, P->d_vt, P->d_slots, g1, BDIAG, vpart1(P));
    hipLaunchKernelGGL(kr_vec, dim3(M), dim3(VB), 0, P->s, P->d_rg, g1, vpart1(P), 1, SC_DMAX, P->d_sc);
    hipLaunchKernelGGL(kv_jacobi, dim3(nv), dim3(VB), 0, P->s, P->d_vt, P->d_slots, g1, P->d_sc);
    hipLaunchKernelGGL(kv_mr_init, dim3(nv), dim3(VB), 0, P->s, P->d_vt, P->d_slots, g1, P->d_jac, vpart1(P));
    hipLaunchKernelGGL(kv_mr_start, dim3(nv), dim3(VB), 0, P->s, P->d_vt, P->d_slots, g1, P->d_rg, vpart1(P), P->d_maxit, P->d_rtol, P->d_st, P->d_run, P->d_slots);
    for (int j = 0; j < maxj; ++j) minres_iter(P, j % 6);
    if (maxj > 0) {
        const int k = (maxj - 1) % 6, par = k & 1;
        const int *W = MR_W[(maxj - 1) % 3];
        hipLaunchKernelGGL(kv_mr_finish, dim3(nv), dim3(VB), 0, P->s, P->d_vt, P->d_slots, g1, P->d_rg, P->d_st, par, vpart1_at(P, par), vpart2(P), mr_zc(k), W[2], W[0], W[1], P->d_run);
    }
    hipLaunchKernelGGL(kn_after_minres, dim3(nblk(M)), dim3(VB), 0, P->s, M, g1, P->d_st, P->d_ns, P->d_search, P->d_sc);
    for (int h = 0; h < LS_ROUNDS; ++h) ls_round_device(P, h);
    hipLaunchKernelGGL(kn_end, dim3(nblk(M)), dim3(VB), 0, P->s, M, g1, P->d_ns);
}

// Newton step with the decisions on the device (graph mode 2): upload the
// Newton state, replay the step graph, read the state back once; rounds
// beyond LS_ROUNDS (rare) follow one by one, each with a read-back.
static int step_device(tmop_pool *P, int maxj, int maxh)
{
    const int M = P->max_slots;
    for (int si = 0; si < M; ++si) {
        const SlotH &s = P->slots[si];
        NState &n = P->h_ns[si];
        n.F = s.F;
        n.gn = s.gn;
        n.g0 = s.g0;
        n.tol = s.sp.rel_grad_tol;
        n.alpha = 1.0;
        n.Ft = 0.0;
        n.newton_its = s.newton_its;
        n.max_newton = s.sp.max_newton;
        n.minres_its = s.minres_its;
        n.halvings = s.halvings;
        n.max_halvings = s.sp.max_halvings;
        n.status = s.status;
        n.phase = s.used ? s.phase : PH_DONE;
        n.searching = 0;
    }
    PHIP(hipMemcpyAsync(P->d_ns, P->h_ns, sizeof(NState) * M, hipMemcpyHostToDevice, P->s));
    if (!P->sgraph_ok || P->sg_maxj != maxj) {
        if (P->sgexec) hipGraphExecDestroy(P->sgexec);
        if (P->sgraph) hipGraphDestroy(P->sgraph);
        P->sgexec = nullptr;
        P->sgraph = nullptr;
        PHIP(hipStreamBeginCapture(P->s, hipStreamCaptureModeThreadLocal));
        record_step(P, maxj);
        PHIP(hipStreamEndCapture(P->s, &P->sgraph));
        PHIP(hipGraphInstantiate(&P->sgexec, P->sgraph, nullptr, nullptr, 0));
        P->sgraph_ok = true;
        P->sg_maxj = maxj;
    }
    PHIP(hipGraphLaunch(P->sgexec, P->s));
    for (int h = LS_ROUNDS;; ++h) {
        PHIP(hipMemcpyAsync(P->h_ns, P->d_ns, sizeof(NState) * M, hipMemcpyDeviceToHost, P->s));
        PHIP(hipStreamSynchronize(P->s));
        bool searching = false;
        for (int si = 0; si < M; ++si) searching = searching || (P->h_gate[1][si] && P->h_ns[si].searching);
        if (!searching || h > maxh) break;
        ls_round_device(P, h);
        hipLaunchKernelGGL(kn_end, dim3(nblk(M)), dim3(VB), 0, P->s, M, P->d_gate[1], P->d_ns);
    }
    PHIP(hipGetLastError());
    for (int si = 0; si < M; ++si) {
        if (!P->h_gate[1][si]) continue;
        SlotH &s = P->slots[si];
        const NState &n = P->h_ns[si];
        s.F = n.F;
        s.gn = n.gn;
        s.newton_its = n.newton_its;
        s.minres_its = n.minres_its;
        s.halvings = n.halvings;
        if (n.phase == NS_DONE) finish_slot(s, n.status);
    }
    return TMOP_OK;
}

// One Newton iteration for every active slot (initial evaluation first for new slots).
static int pool_step_impl(tmop_pool *P, int *n_active)
{
    // roctx range (rocprofv3 --marker-trace); a no-op without a profiler
    struct Range {
        Range() { roctxRangePush("tmop pool step"); }
        ~Range() { roctxRangePop(); }
    } range;
    if (P->dirty) PCHK(pool_rebuild(P));
    const int M = P->max_slots;
    // ---- initial evaluation of new slots -------------------------------
    bool any_new = false;
    for (int si = 0; si < M; ++si) {
        SlotH &s = P->slots[si];
        P->h_gate[0][si] = (s.used && s.phase == PH_NEW) ? 1 : 0;
        any_new = any_new || P->h_gate[0][si];
    }
    if (any_new) {
        PCHK(upload_gate(P, 0));
        const int *g0 = P->d_gate[0];
        dot_to_sc(P, g0, BX, BX, SC_DOT);
        energy_grad_elem(P, g0, BX);
        launch_gather(P, g0, BG, 0, BG, false);
        PCHK(read_sc(P));
        std::vector<double> xx(M);
        for (int si = 0; si < M; ++si) xx[si] = P->h_sc[si * NSC + SC_DOT];
        dot_to_sc(P, g0, BG, BG, SC_DOT);
        PCHK(read_sc(P));
        for (int si = 0; si < M; ++si) {
            SlotH &s = P->slots[si];
            if (!P->h_gate[0][si]) continue;
            const double *sc = P->h_sc + si * NSC;
            if (!std::isfinite(xx[si])) {
                finish_slot(s, TMOP_ERR_NONFINITE);
                continue;
            }
            if (sc[SC_BAD] > 0.0 || !(sc[SC_MD] > 0.0)) {
                s.F = INFINITY;
                finish_slot(s, TMOP_ERR_INVERTED);
                continue;
            }
            s.F = s.F0 = sc[SC_F];
            s.gn = std::sqrt(sc[SC_DOT]);
            s.g0 = s.sp.g0_norm > 0.0 ? s.sp.g0_norm : s.gn;
            s.phase = PH_ITER;
            if (s.g0 == 0.0 || s.F == 0.0 || s.gn <= s.sp.rel_grad_tol * s.g0) finish_slot(s, TMOP_OK);
        }
    }
    // ---- Newton iteration ---------------------------------------------
    int maxj = 0, maxh = 0, nit = 0;
    for (int si = 0; si < M; ++si) {
        SlotH &s = P->slots[si];
        if (s.used && s.phase == PH_ITER && s.newton_its >= s.sp.max_newton)
            finish_slot(s, TMOP_ERR_NOT_CONVERGED);
        const bool it = s.used && s.phase == PH_ITER;
        P->h_gate[1][si] = it ? 1 : 0;
        P->h_int[si] = it && s.sp.jacobi ? 1 : 0;
        if (it) {
            nit++;
            maxj = std::max(maxj, s.sp.max_minres);
            maxh = std::max(maxh, s.sp.max_halvings);
        }
    }
    if (nit) {
        PCHK(upload_gate(P, 1));
        PHIP(hipMemcpyAsync(P->d_jac, P->h_int, sizeof(int) * M, hipMemcpyHostToDevice, P->s));
        for (int si = 0; si < M; ++si) {
            P->h_gate[4][si] = P->slots[si].sp.max_minres;
            P->h_rtol[si] = P->slots[si].sp.minres_rtol;
        }
        PHIP(hipMemcpyAsync(P->d_maxit, P->h_gate[4], sizeof(int) * M, hipMemcpyHostToDevice, P->s));
        PHIP(hipMemcpyAsync(P->d_rtol, P->h_rtol, sizeof(double) * M, hipMemcpyHostToDevice, P->s));
        if (P->graph_mode == 2) {
            for (int si = 0; si < M; ++si)
                if (P->h_gate[1][si]) P->slots[si].h_ready = true;
            PCHK(step_device(P, maxj, maxh));
            int na = 0;
            for (auto &s : P->slots) na += (s.used && s.phase != PH_DONE) ? 1 : 0;
            if (n_active) *n_active = na;
            return TMOP_OK;
        }
        const int *g1 = P->d_gate[1];
        launch_elem(P, 2, g1, BX);   // setup
        for (int si = 0; si < M; ++si)
            if (P->h_gate[1][si]) P->slots[si].h_ready = true;
        launch_elem(P, 4, g1, BX);   // diagonal
        launch_gather(P, g1, BDIAG, 1, BDIAG, false);
        const int nv = nvt_all(P);
        hipLaunchKernelGGL(kv_absmax, dim3(nv), dim3(VB), 0, P->s, P->d_vt, P->d_slots, g1, BDIAG, vpart1(P));
        hipLaunchKernelGGL(kr_vec, dim3(M), dim3(VB), 0, P->s, P->d_rg, g1, vpart1(P), 1, SC_DMAX, P->d_sc);
        hipLaunchKernelGGL(kv_jacobi, dim3(nv), dim3(VB), 0, P->s, P->d_vt, P->d_slots, g1, P->d_sc);
        PCHK(run_minres(P, maxj));
        for (int si = 0; si < M; ++si) {
            SlotH &s = P->slots[si];
            if (!P->h_gate[1][si]) continue;
            const BState &a = P->h_st[2 * si], &b = P->h_st[2 * si + 1];
            const BState &f = a.j >= b.j ? a : b;
            s.minres_its += f.j;
            if (f.indefinite) {
                finish_slot(s, TMOP_ERR_NONFINITE);
                P->h_gate[1][si] = 0;
            }
            s.alpha = 1.0;
        }
        // ---- line search rounds -------------------------------------------
        for (int si = 0; si < M; ++si) P->h_gate[2][si] = P->h_gate[1][si];
        for (int h = 0; h <= maxh; ++h) {
            bool any = false;
            for (int si = 0; si < M; ++si) {
                any = any || P->h_gate[2][si];
                P->h_sc[si * NSC + SC_ALPHA] = P->slots[si].alpha;
            }
            if (!any) break;
            PCHK(upload_gate(P, 2));
            PHIP(hipMemcpyAsync(P->d_sc, P->h_sc, sizeof(double) * NSC * M, hipMemcpyHostToDevice, P->s));
            const int *g2 = P->d_gate[2];
            hipLaunchKernelGGL(kv_step, dim3(nv), dim3(VB), 0, P->s, P->d_vt, P->d_slots, g2, P->d_sc);
            energy_grad_elem(P, g2, BXT);
            PCHK(read_sc(P));
            bool any3 = false;
            std::vector<double> Ft(M);
            for (int si = 0; si < M; ++si) {
                const double *sc = P->h_sc + si * NSC;
                const bool ok = P->h_gate[2][si] && sc[SC_BAD] == 0.0 && sc[SC_MD] > 0.0 &&
                                sc[SC_F] < 1.2 * P->slots[si].F;
                P->h_gate[3][si] = ok ? 1 : 0;
                Ft[si] = sc[SC_F];
                any3 = any3 || ok;
            }
            if (any3) {
                PCHK(upload_gate(P, 3));
                const int *g3 = P->d_gate[3];
                launch_gather(P, g3, BGT, 0, BGT, false);
                dot_to_sc(P, g3, BGT, BGT, SC_DOT);
                PCHK(read_sc(P));
                bool anyacc = false;
                for (int si = 0; si < M; ++si) {
                    int acc = 0;
                    if (P->h_gate[3][si]) {
                        const double gtn = std::sqrt(P->h_sc[si * NSC + SC_DOT]);
                        SlotH &s = P->slots[si];
                        if (gtn < 1.2 * s.gn) {
                            acc = 1;
                            s.F = Ft[si];
                            s.gn = gtn;
                            s.newton_its++;
                        }
                    }
                    P->h_gate[3][si] = acc;
                    anyacc = anyacc || acc;
                }
                if (anyacc) {
                    PCHK(upload_gate(P, 3));
                    hipLaunchKernelGGL(kv_copy, dim3(nv), dim3(VB), 0, P->s, P->d_vt, P->d_slots, P->d_gate[3], BXT, BX);
                    hipLaunchKernelGGL(kv_copy, dim3(nv), dim3(VB), 0, P->s, P->d_vt, P->d_slots, P->d_gate[3], BGT, BG);
                    PHIP(hipStreamSynchronize(P->s));
                }
            }
            for (int si = 0; si < M; ++si) {
                if (!P->h_gate[2][si]) continue;
                SlotH &s = P->slots[si];
                if (any3 && P->h_gate[3][si]) {
                    P->h_gate[2][si] = 0;  // accepted
                    continue;
                }
                s.halvings++;
                s.alpha *= 0.5;
                if (h >= s.sp.max_halvings) {
                    P->h_gate[2][si] = 0;
                    finish_slot(s, TMOP_ERR_LINESEARCH);
                }
            }
        }
        // ---- convergence test ---------------------------------------------
        for (int si = 0; si < M; ++si) {
            SlotH &s = P->slots[si];
            if (!s.used || s.phase != PH_ITER) continue;
            if (s.F == 0.0 || s.gn <= s.sp.rel_grad_tol * s.g0) finish_slot(s, TMOP_OK);
            else if (s.newton_its >= s.sp.max_newton) finish_slot(s, TMOP_ERR_NOT_CONVERGED);
        }
    }
    int na = 0;
    for (auto &s : P->slots) na += (s.used && s.phase != PH_DONE) ? 1 : 0;
    if (n_active) *n_active = na;
    return TMOP_OK;
}

extern "C" int tmop_pool_create(tmop_pool **out, size_t budget, int max_slots, void *stream)
{
    if (!out || budget == 0 || max_slots <= 0 || max_slots > 65536)
        return pfail(TMOP_ERR_INVALID_ARG, "bad pool arguments");
    *out = nullptr;
    tmop_pool *P = new tmop_pool();
    P->budget = budget;
    P->max_slots = max_slots;
    P->slots.resize(max_slots);
    hipError_t e = hipSuccess;
    if (stream) {
        P->s = (hipStream_t)stream;
    } else {
        e = hipStreamCreateWithFlags(&P->s, hipStreamNonBlocking);
        P->own_stream = e == hipSuccess;
    }
    if (e == hipSuccess) e = hipMalloc((void **)&P->arena, budget);
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_slots, sizeof(SlotDev) * max_slots);
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_rg, sizeof(SlotRange) * max_slots);
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_sc, sizeof(double) * NSC * max_slots);
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_st, sizeof(BState) * 2 * max_slots);
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_run, sizeof(int) * max_slots);
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_jac, sizeof(int) * max_slots);
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_maxit, sizeof(int) * max_slots);
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_rtol, sizeof(double) * max_slots);
    if (e == hipSuccess) e = hipHostMalloc((void **)&P->h_rtol, sizeof(double) * max_slots, 0);
    for (int k = 0; k < 6 && e == hipSuccess; ++k) {
        e = hipMalloc((void **)&P->d_gate[k], sizeof(int) * max_slots);
        if (e == hipSuccess) e = hipHostMalloc((void **)&P->h_gate[k], sizeof(int) * max_slots, 0);
    }
    if (e == hipSuccess) e = hipHostMalloc((void **)&P->h_sc, sizeof(double) * NSC * max_slots, 0);
    if (e == hipSuccess) e = hipHostMalloc((void **)&P->h_st, sizeof(BState) * 2 * max_slots, 0);
    if (e == hipSuccess) e = hipHostMalloc((void **)&P->h_int, sizeof(int) * max_slots, 0);
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_ns, sizeof(NState) * max_slots);
    if (e == hipSuccess) e = hipHostMalloc((void **)&P->h_ns, sizeof(NState) * max_slots, 0);
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_search, sizeof(int) * max_slots);
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_ftest, sizeof(int) * max_slots);
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_acc, sizeof(int) * max_slots);
    if (e != hipSuccess) {
        tmop_pool_destroy(P);
        return pfail(e == hipErrorOutOfMemory ? TMOP_ERR_OOM : TMOP_ERR_HIP,
                     std::string("pool allocation: ") + hipGetErrorString(e));
    }
    P->free_.emplace(0, budget);
    std::vector<int> z(max_slots, 0);
    hipMemcpy(P->d_run, z.data(), sizeof(int) * max_slots, hipMemcpyHostToDevice);
    *out = P;
    return TMOP_OK;
}

extern "C" int tmop_pool_destroy(tmop_pool *P)
{
    if (!P) return TMOP_OK;
    if (P->s) hipStreamSynchronize(P->s);
    invalidate_graph(P);
    for (auto &kv : P->classes) {
        hipFree(kv.second.d_tiles);
        hipFree(kv.second.d_atiles);
    }
    hipFree(P->arena);
    hipFree(P->d_slots);
    hipFree(P->d_rg);
    hipFree(P->d_vt);
    hipFree(P->d_part);
    hipFree(P->d_sc);
    hipFree(P->d_st);
    hipFree(P->d_run);
    hipFree(P->d_jac);
    hipFree(P->d_maxit);
    hipFree(P->d_rtol);
    if (P->h_rtol) hipHostFree(P->h_rtol);
    for (int k = 0; k < 6; ++k) {
        hipFree(P->d_gate[k]);
        if (P->h_gate[k]) hipHostFree(P->h_gate[k]);
    }
    if (P->h_sc) hipHostFree(P->h_sc);
    if (P->h_st) hipHostFree(P->h_st);
    if (P->h_int) hipHostFree(P->h_int);
    hipFree(P->d_ns);
    if (P->h_ns) hipHostFree(P->h_ns);
    hipFree(P->d_search);
    hipFree(P->d_ftest);
    hipFree(P->d_acc);
    if (P->s && P->own_stream) hipStreamDestroy(P->s);
    delete P;
    return TMOP_OK;
}

extern "C" int tmop_pool_request_bytes(const tmop_mesh_desc *m, const tmop_params *prm, size_t *bytes)
{
    SlotH s;
    std::string why;
    const int r = request_sizes(m, prm, s, why);
    if (r != TMOP_OK) return pfail(r, why);
    if (bytes) *bytes = s.bytes;
    return TMOP_OK;
}

// Admission of one solve; x0_dev != NULL adds the limiting term
// coef |x - x0|^2 / delta^2 with the reference nodes copied into the region.
static int pool_admit_impl(tmop_pool *P, const tmop_mesh_desc *m, const tmop_params *prm,
                           const tmop_solve_params *sp, const double *x_dev, const double *x0_dev,
                           double coef, double delta, void *src_stream, int *slot)
{
    if (!P || !sp || !x_dev || !slot) return pfail(TMOP_ERR_INVALID_ARG, "null argument");
    if (x0_dev && (!(delta > 0.0) || !(coef >= 0.0) || !std::isfinite(coef) || !std::isfinite(delta)))
        return pfail(TMOP_ERR_INVALID_ARG, "limiting term needs coef >= 0 and delta > 0");
    SlotH s;
    std::string why;
    int r = request_sizes(m, prm, s, why);
    if (r != TMOP_OK) return pfail(r, why);
    const bool with_x0 = x0_dev != nullptr && coef > 0.0;
    if (with_x0) s.bytes += up256((size_t)s.ndof * 8);
    BOps probe;
    if (!find_bops(s.dim, s.p, s.nq, &probe))
        return pfail(TMOP_ERR_UNSUPPORTED, "no kernel for this (dim, p, nq1d)");
    if (s.bytes > P->budget) return pfail(TMOP_ERR_BUDGET, "request larger than the pool budget");
    int si = -1;
    for (int k = 0; k < P->max_slots; ++k)
        if (!P->slots[k].used) {
            si = k;
            break;
        }
    size_t off = 0;
    // with room, the slot also keeps its max_minres + 1 Lanczos vectors and
    // the per-update scalars (else the three-term update)
    const size_t base_bytes = s.bytes;
    const int kb = sp->max_minres + 1;
    size_t bank_bytes = P->use_bank ? bank_bytes_of(s.ndof, sp->max_minres) : 0;
    if (si >= 0 && bank_bytes && base_bytes + bank_bytes <= P->budget &&
        pool_alloc_region(P, base_bytes + bank_bytes, &off)) {
        s.bytes = base_bytes + bank_bytes;
    } else {
        bank_bytes = 0;
        if (si < 0 || !pool_alloc_region(P, s.bytes, &off))
            return pfail(TMOP_ERR_BUSY, "pool full (slots or HBM budget); retry after a release");
    }
    Tables tb;
    Target tg;
    if (internal_tables(s.p, s.nq, &tb) != TMOP_OK ||
        internal_target(prm, s.dim, &tg) != TMOP_OK) {
        pool_free_region(P, off, s.bytes);
        return pfail(TMOP_ERR_INVALID_ARG, "bad quadrature or target");
    }
    s.off = off;
    s.sp = *sp;
    s.used = true;
    s.phase = PH_NEW;
    s.t_start = now_ms();
    Geom &g = s.dev.g;
    g.dim = s.dim;
    g.p = s.p;
    g.ne = s.ne;
    g.nx = s.nx;
    g.nel[0] = m->nx;
    g.nel[1] = m->ny;
    g.nel[2] = s.dim == 3 ? m->nz : 1;
    for (int k = 0; k < 3; ++k) g.M[k] = g.nel[k] * s.p + 1;
    if (s.dim == 2) g.M[2] = 1;
    set_divisors(g);
    g.e2n = nullptr;
    g.ess_mode = m->ess_mode;
    g.ess = nullptr;  // a mask is copied into the slot's region below
    g.x0 = nullptr;  // the limiting term, when asked for, is set below
    g.lim = 0.0;
    s.dev.tg = tg;
    char *base = P->arena + off;
    size_t o = 0;
    for (int k = 0; k < NVEC; ++k) s.dev.vec[k] = nullptr;
    for (int k = 0; k < BNV; ++k) {
        s.dev.vec[k] = (double *)(base + o);
        o += up256((size_t)s.ndof * 8);
    }
    s.dev.H = base + o;
    o += up256((size_t)s.ne * qdata_stride(s.S, s.nqe, s.prec ? 4 : 8) * (s.prec ? 4 : 8));
    s.dev.eV = base + o;
    o += up256((size_t)s.ne * s.dim * s.np * 8);
    uint8_t *mask = nullptr;
    if (m->ess_mode == TMOP_ESS_MASK) {
        mask = (uint8_t *)(base + o);
        g.ess = mask;
        o += up256((size_t)s.ndof);
    }
    double *x0 = nullptr;
    if (with_x0) {
        // limiting term: reference nodes in the region, lim = coef det W / delta^2
        x0 = (double *)(base + o);
        o += up256((size_t)s.ndof * 8);
        g.x0 = x0;
        g.lim = coef * tg.detW / (delta * delta);
        s.lim = 1;
    }
    s.dev.bank = nullptr;
    s.dev.hist = nullptr;
    s.dev.bstride = 0;
    if (bank_bytes) {
        s.dev.bstride = (long)(up256((size_t)s.ndof * 8) / 8);
        s.dev.bank = (double *)(base + o);
        o += (size_t)kb * up256((size_t)s.ndof * 8);
        s.dev.hist = (double *)(base + o);
    }
    // copy the caller's nodes (and mask) after the caller's stream has produced them
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, (hipStream_t)src_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(P->s, ev, 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s.dev.vec[BX], x_dev, sizeof(double) * s.ndof, hipMemcpyDeviceToDevice, P->s);
    if (e == hipSuccess && mask)
        e = hipMemcpyAsync(mask, m->ess_mask, (size_t)s.ndof, hipMemcpyDeviceToDevice, P->s);
    if (e == hipSuccess && x0)
        e = hipMemcpyAsync(x0, x0_dev, sizeof(double) * s.ndof, hipMemcpyDeviceToDevice, P->s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(P->d_slots + si, &s.dev, sizeof(SlotDev), hipMemcpyHostToDevice, P->s);
    if (e == hipSuccess) e = hipStreamSynchronize(P->s);
    if (ev) hipEventDestroy(ev);
    if (e != hipSuccess) {
        pool_free_region(P, off, s.bytes);
        return pfail(TMOP_ERR_HIP, std::string("pool admission: ") + hipGetErrorString(e));
    }
    P->slots[si] = s;
    P->used += s.bytes;
    P->dirty = true;
    *slot = si;
    return TMOP_OK;
}

extern "C" int tmop_pool_admit(tmop_pool *P, const tmop_mesh_desc *m, const tmop_params *prm,
                               const tmop_solve_params *sp, const double *x_dev, void *src_stream,
                               int *slot)
{
    return pool_admit_impl(P, m, prm, sp, x_dev, nullptr, 0.0, 1.0, src_stream, slot);
}

extern "C" int tmop_pool_admit_limited(tmop_pool *P, const tmop_mesh_desc *m, const tmop_params *prm,
                                       const tmop_solve_params *sp, const double *x_dev,
                                       const double *x0_dev, double coef, double delta,
                                       void *src_stream, int *slot)
{
    if (!x0_dev) return pfail(TMOP_ERR_INVALID_ARG, "null reference nodes");
    return pool_admit_impl(P, m, prm, sp, x_dev, x0_dev, coef, delta, src_stream, slot);
}

extern "C" int tmop_pool_step(tmop_pool *P, int *n_active)
{
    if (!P) return pfail(TMOP_ERR_INVALID_ARG, "null pool");
    return pool_step_impl(P, n_active);
}

extern "C" int tmop_pool_poll(tmop_pool *P, int slot, int *done, tmop_solve_report *rep)
{
    if (!P || slot < 0 || slot >= P->max_slots || !P->slots[slot].used)
        return pfail(TMOP_ERR_INVALID_ARG, "bad slot");
    const SlotH &s = P->slots[slot];
    if (done) *done = s.phase == PH_DONE ? 1 : 0;
    if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        rep->newton_its = s.newton_its;
        rep->minres_its_total = s.minres_its;
        rep->halvings_total = s.halvings;
        rep->status = s.status;
        rep->F0 = s.F0;
        rep->F = s.F;
        rep->g0_norm = s.g0;
        rep->g_norm = s.gn;
        rep->t_total_ms = (s.phase == PH_DONE ? s.t_done : now_ms()) - s.t_start;
    }
    return TMOP_OK;
}

extern "C" int tmop_pool_result(tmop_pool *P, int slot, double *x_dev, void *dst_stream)
{
    if (!P || !x_dev || slot < 0 || slot >= P->max_slots || !P->slots[slot].used)
        return pfail(TMOP_ERR_INVALID_ARG, "bad slot");
    const SlotH &s = P->slots[slot];
    PHIP(hipMemcpyAsync(x_dev, s.dev.vec[BX], sizeof(double) * s.ndof, hipMemcpyDeviceToDevice, P->s));
    PHIP(hipStreamSynchronize(P->s));
    (void)dst_stream;
    return TMOP_OK;
}

extern "C" int tmop_pool_evaluate(tmop_pool *P, int slot, int what, const double *in_dev,
                                  double *out_dev, double *out_host, void *stream)
{
    if (!P || slot < 0 || slot >= P->max_slots || !P->slots[slot].used)
        return pfail(TMOP_ERR_INVALID_ARG, "bad slot");
    if (what < TMOP_EVAL_ENERGY || what > TMOP_EVAL_DIAG)
        return pfail(TMOP_ERR_INVALID_ARG, "unknown evaluation");
    SlotH &s = P->slots[slot];
    const bool need_in = what != TMOP_EVAL_DIAG;
    const bool need_out = what == TMOP_EVAL_GRADIENT || what == TMOP_EVAL_APPLY || what == TMOP_EVAL_DIAG;
    if ((need_in && !in_dev) || (need_out && !out_dev) || (what == TMOP_EVAL_ENERGY && !out_host))
        return pfail(TMOP_ERR_INVALID_ARG, "null argument");
    if ((what == TMOP_EVAL_APPLY || what == TMOP_EVAL_DIAG) && !s.h_ready)
        return pfail(TMOP_ERR_STATE, "no Hessian setup for this slot yet");
    if (P->dirty) PCHK(pool_rebuild(P));
    for (int k = 0; k < P->max_slots; ++k) P->h_gate[5][k] = k == slot ? 1 : 0;
    PCHK(upload_gate(P, 5));
    const int *ge = P->d_gate[5];
    const size_t nb = sizeof(double) * (size_t)s.ndof;
    // read the caller's input after the caller's stream has produced it
    hipEvent_t ev;
    PHIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    PHIP(hipEventRecord(ev, (hipStream_t)stream));
    PHIP(hipStreamWaitEvent(P->s, ev, 0));
    hipEventDestroy(ev);
    int status = TMOP_OK;
    switch (what) {
    case TMOP_EVAL_ENERGY: {
        PHIP(hipMemcpyAsync(s.dev.vec[BXT], in_dev, nb, hipMemcpyDeviceToDevice, P->s));
        energy_to_sc(P, ge, BXT);
        PCHK(read_sc(P));
        const double *sc = P->h_sc + slot * NSC;
        const bool bad = sc[SC_BAD] > 0.0 || !(sc[SC_MD] > 0.0);
        out_host[0] = bad ? INFINITY : sc[SC_F];
        out_host[1] = sc[SC_MD];
        if (bad) status = TMOP_ERR_INVERTED;
        break;
    }
    case TMOP_EVAL_GRADIENT:
        PHIP(hipMemcpyAsync(s.dev.vec[BXT], in_dev, nb, hipMemcpyDeviceToDevice, P->s));
        gradient_to(P, ge, BXT, BGT);
        PHIP(hipMemcpyAsync(out_dev, s.dev.vec[BGT], nb, hipMemcpyDeviceToDevice, P->s));
        break;
    case TMOP_EVAL_SETUP:
        PHIP(hipMemcpyAsync(s.dev.vec[BXT], in_dev, nb, hipMemcpyDeviceToDevice, P->s));
        launch_elem(P, 2, ge, BXT);
        s.h_ready = true;
        break;
    case TMOP_EVAL_APPLY: {
        // the element kernels read the action's input through the slot's
        // BZIN pointer (set by MINRES on the device); point it at BZ0
        PHIP(hipMemcpyAsync(s.dev.vec[BZ0], in_dev, nb, hipMemcpyDeviceToDevice, P->s));
        double *const zin = s.dev.vec[BZ0];
        PHIP(hipMemcpyAsync(&P->d_slots[slot].vec[BZIN], &zin, sizeof(double *), hipMemcpyHostToDevice, P->s));
        PHIP(hipStreamSynchronize(P->s));
        launch_elem(P, 3, ge, BZIN);
        // fixed DoFs: y = v (H_c = P H P + I - P); mixed slots' E-vectors are FP32
        launch_gather(P, ge, BY, 2, BZ0, true);
        PHIP(hipMemcpyAsync(out_dev, s.dev.vec[BY], nb, hipMemcpyDeviceToDevice, P->s));
        break;
    }
    case TMOP_EVAL_DIAG:
        launch_elem(P, 4, ge, BX);
        launch_gather(P, ge, BDIAG, 1, BDIAG, false);
        PHIP(hipMemcpyAsync(out_dev, s.dev.vec[BDIAG], nb, hipMemcpyDeviceToDevice, P->s));
        break;
    }
    PHIP(hipStreamSynchronize(P->s));
    PHIP(hipGetLastError());
    if (status != TMOP_OK) return pfail(status, "det A <= 0 at a quadrature point");
    return TMOP_OK;
}

extern "C" int tmop_pool_release(tmop_pool *P, int slot)
{
    if (!P || slot < 0 || slot >= P->max_slots || !P->slots[slot].used)
        return pfail(TMOP_ERR_INVALID_ARG, "bad slot");
    PHIP(hipStreamSynchronize(P->s));
    SlotH &s = P->slots[slot];
    pool_free_region(P, s.off, s.bytes);
    P->used -= s.bytes;
    s = SlotH();
    P->dirty = true;
    return TMOP_OK;
}

extern "C" int tmop_pool_info(tmop_pool *P, size_t *used_bytes, size_t *budget_bytes, int *slots_used)
{
    if (!P) return pfail(TMOP_ERR_INVALID_ARG, "null pool");
    if (used_bytes) *used_bytes = P->used;
    if (budget_bytes) *budget_bytes = P->budget;
    if (slots_used) {
        int n = 0;
        for (auto &s : P->slots) n += s.used ? 1 : 0;
        *slots_used = n;
    }
    return TMOP_OK;
}

extern "C" int tmop_pool_autotune(tmop_pool *P, int reps)
{
    if (!P || reps <= 0) return pfail(TMOP_ERR_INVALID_ARG, "bad argument");
    if (P->dirty) PCHK(pool_rebuild(P));
    hipEvent_t e0, e1;
    PHIP(hipEventCreate(&e0));
    PHIP(hipEventCreate(&e1));
    for (auto &kv : P->classes) {
        ClassH &c = kv.second;
        if (c.tiles.empty() || c.key.lim) continue;
        const int st = c.key.storage, pr = c.key.prec;
        int best = -1;
        float tbest = 0.f;
        float tmin[3] = {0.f, 0.f, 0.f};
        // three rounds over the shapes, each shape's best round counts
        for (int round = 0; round < 3; ++round) {
            for (int t = 0; t < 3; ++t) {
                if (c.bops.epb_t[t] == 0) continue;
                const Tile *dl = c.d_tiles;
                int n = (int)c.tiles.size();
                if (t != 1) {
                    // tile list of this shape for the class's resident meshes
                    std::vector<Tile> tl;
                    for (const Tile &b : c.tiles)
                        if (b.e0 == 0)  // first tile of each resident mesh of the class
                            for (int e = 0; e < P->slots[b.slot].ne; e += c.bops.epb_t[t])
                                tl.push_back(Tile{b.slot, e});
                    n = (int)tl.size();
                    if (n > c.acap) {
                        hipFree(c.d_atiles);
                        c.d_atiles = nullptr;
                        c.acap = std::max(n, 2 * c.acap);
                        PHIP(hipMalloc((void **)&c.d_atiles, sizeof(Tile) * c.acap));
                    }
                    PHIP(hipMemcpyAsync(c.d_atiles, tl.data(), sizeof(Tile) * n, hipMemcpyHostToDevice, P->s));
                    dl = c.d_atiles;
                }
                BLaunch f = c.bops.apply_t[st][pr][t];
                for (int k = 0; k < 2; ++k) f(n, P->s, c.tb, dl, P->d_slots, nullptr, 0, nullptr);
                PHIP(hipEventRecord(e0, P->s));
                for (int k = 0; k < reps; ++k) f(n, P->s, c.tb, dl, P->d_slots, nullptr, 0, nullptr);
                PHIP(hipEventRecord(e1, P->s));
                PHIP(hipEventSynchronize(e1));
                float ms = 0.f;
                PHIP(hipEventElapsedTime(&ms, e0, e1));
                if (round == 0 || ms < tmin[t]) tmin[t] = ms;
            }
        }
        for (int t = 0; t < 3; ++t)
            if (c.bops.epb_t[t] != 0 && (best < 0 || tmin[t] < tbest)) {
                best = t;
                tbest = tmin[t];
            }
        c.tile = best;
        record_tile(c.key.dim, c.key.p, c.key.nq, st ? TMOP_HESS_COMPACT : TMOP_HESS_TENSOR,
                    pr ? TMOP_MIXED : TMOP_FP64, best);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    P->dirty = true;
    return TMOP_OK;
}

extern "C" int tmop_pool_set_lanczos_bank(tmop_pool *P, int enable)
{
    if (!P) return pfail(TMOP_ERR_INVALID_ARG, "null pool");
    P->use_bank = enable != 0;
    return TMOP_OK;
}

extern "C" int tmop_pool_set_graph(tmop_pool *P, int enable)
{
    if (!P) return pfail(TMOP_ERR_INVALID_ARG, "null pool");
    if (enable < 0 || enable > 2) return pfail(TMOP_ERR_INVALID_ARG, "graph mode must be 0, 1 or 2");
    P->graph_mode = enable;
    invalidate_graph(P);
    return TMOP_OK;
}

extern "C" const char *tmop_pool_last_error(void) { return g_perr.c_str(); }

extern "C" int tmop_batch_solve(int count, const tmop_mesh_desc *meshes, const tmop_params *prms,
                                double *const *x_devs, const tmop_solve_params *sps,
                                tmop_solve_report *reps, void *stream)
{
    if (count <= 0 || !meshes || !prms || !x_devs || !sps || !reps)
        return pfail(TMOP_ERR_INVALID_ARG, "bad batch arguments");
    // every mesh's region with its resident Lanczos vectors
    size_t total = 0;
    for (int k = 0; k < count; ++k) {
        SlotH s;
        std::string why;
        const int r = request_sizes(meshes + k, prms + k, s, why);
        if (r != TMOP_OK) return pfail(r, why);
        total += s.bytes + bank_bytes_of(s.ndof, sps[k].max_minres);
    }
    tmop_pool *P = nullptr;
    PCHK(tmop_pool_create(&P, total, count, stream));
    P->use_bank = true;
    // one graph launch per Newton step: the batch's layout never changes
    P->graph_mode = 2;
    std::vector<int> slot(count, -1);
    int r = TMOP_OK;
    for (int k = 0; k < count && r == TMOP_OK; ++k)
        r = tmop_pool_admit(P, meshes + k, prms + k, sps + k, x_devs[k], stream, &slot[k]);
    // tile shapes of the Hessian action, per class, for this batch
    if (r == TMOP_OK) r = tmop_pool_autotune(P, 3);
    int active = count;
    while (r == TMOP_OK && active > 0) r = tmop_pool_step(P, &active);
    for (int k = 0; k < count && r == TMOP_OK; ++k) {
        int done = 0;
        r = tmop_pool_poll(P, slot[k], &done, reps + k);
        if (r == TMOP_OK) r = tmop_pool_result(P, slot[k], x_devs[k], stream);
    }
    tmop_pool_destroy(P);
    return r;
}
