// C ABI of the PA-TMOP library: context, evaluations, Newton-MINRES driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/tmop.h"
#include "ops.hpp"
#include "tmop_dev.hpp"
#include "vec.hpp"

using namespace tmop;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

// roctx range over a host scope (phases of the Newton-MINRES solve, visible
// in rocprofv3 --marker-trace; a no-op when no profiler is attached)
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePush(name); }
    ~TraceRange() { roctxRangePop(); }
};

#define HIPCHK(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(e_ == hipErrorOutOfMemory ? TMOP_ERR_OOM : TMOP_ERR_HIP,             \
                        std::string(#call) + ": " + hipGetErrorString(e_));                  \
    } while (0)

#define CHK(call)                   \
    do {                            \
        int r_ = (call);            \
        if (r_ != TMOP_OK) return r_; \
    } while (0)

// ---------------------------------------------------------------------------
// 1D bases on [0,1] (Sec. 3.1): Gauss-Lobatto-Legendre nodes for the Lagrange
// basis, Gauss-Legendre points and weights for quadrature.
// ---------------------------------------------------------------------------

// P_n(t) and P_n'(t) by the three-term recurrence.
void legendre(int n, double t, double &P, double &dP)
{
    double p0 = 1.0, p1 = t;
    if (n == 0) {
        P = 1.0;
        dP = 0.0;
        return;
    }
    for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    P = p1;
    // derivative from (1 - t^2) P_n' = n (P_{n-1} - t P_n)
    dP = (std::fabs(1.0 - t * t) > 0.0) ? n * (p0 - t * p1) / (1.0 - t * t)
                                         : 0.5 * n * (n + 1.0) * std::pow(t, n + 1);
}

void gauss_legendre01(int n, double *x, double *w)
{
    for (int k = 0; k < n; ++k) {
        double t = std::cos(M_PI * (k + 0.75) / (n + 0.5));
        double P, dP;
        for (int it = 0; it < 100; ++it) {
            legendre(n, t, P, dP);
            const double dt = P / dP;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        legendre(n, t, P, dP);
        // t descends with k: store ascending on [0,1]
        x[n - 1 - k] = 0.5 * (1.0 + t);
        w[n - 1 - k] = 1.0 / ((1.0 - t * t) * dP * dP);  // (2/((1-t^2)P'^2)) / 2
    }
}

// n-point Gauss-Lobatto-Legendre rule on [0,1]: the GLL nodes of order n-1
// and weights 2 / (n (n-1) P_{n-1}(t)^2) on [-1,1], halved.
void gll_nodes01(int p, double *x);
void gauss_lobatto01(int n, double *x, double *w)
{
    gll_nodes01(n - 1, x);
    for (int k = 0; k < n; ++k) {
        double P, dP;
        legendre(n - 1, 2.0 * x[k] - 1.0, P, dP);
        w[k] = 1.0 / (n * (n - 1.0) * P * P);
    }
}

void gll_nodes01(int p, double *x)
{
    x[0] = 0.0;
    x[p] = 1.0;
    for (int j = 1; j < p; ++j) {
        // interior nodes: roots of P_p'; Newton with P_p'' from Legendre's equation
        double t = -std::cos(M_PI * j / p);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(p, t, P, dP);
            const double d2P = (2.0 * t * dP - p * (p + 1.0) * P) / (1.0 - t * t);
            const double dt = dP / d2P;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        x[j] = 0.5 * (1.0 + t);
    }
    // exact symmetry about 1/2
    for (int j = 0; j <= p / 2; ++j) {
        const double a = 0.5 * (x[j] + (1.0 - x[p - j]));
        x[j] = a;
        x[p - j] = 1.0 - a;
    }
}

// B[q][i] = l_i(chi_q), G[q][i] = l_i'(chi_q) with barycentric weights.
void lagrange_tables(int p, int nq, const double *xi, const double *chi, double *B, double *G)
{
    const int ni = p + 1;
    double lam[MAXNI];  // no heap allocation: the no-allocation entry point builds tables too
    for (int i = 0; i < ni; ++i) {
        double d = 1.0;
        for (int m = 0; m < ni; ++m)
            if (m != i) d *= xi[i] - xi[m];
        lam[i] = 1.0 / d;
    }
    for (int q = 0; q < nq; ++q) {
        const double t = chi[q];
        for (int i = 0; i < ni; ++i) {
            double v = lam[i];
            for (int m = 0; m < ni; ++m)
                if (m != i) v *= t - xi[m];
            double dv = 0.0;
            for (int r = 0; r < ni; ++r) {
                if (r == i) continue;
                double prod = lam[i];
                for (int m = 0; m < ni; ++m)
                    if (m != i && m != r) prod *= t - xi[m];
                dv += prod;
            }
            B[q * ni + i] = v;
            G[q * ni + i] = dv;
        }
    }
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

namespace tmop {

int tuned_tile(int dim, int p, int nq, int storage, int precision);
void record_tile(int dim, int p, int nq, int storage, int precision, int t);

int internal_tables(int p, int nq, Tables *tb, int rule)
{
    if (p < 1 || p >= MAXNI || nq < 1 || nq > MAXNQ) return TMOP_ERR_INVALID_ARG;
    if (rule != TMOP_QUAD_GL && !(rule == TMOP_QUAD_GLL && nq >= 2)) return TMOP_ERR_INVALID_ARG;
    double xi[MAXNI], chi[MAXNQ], w[MAXNQ];
    gll_nodes01(p, xi);
    if (rule == TMOP_QUAD_GLL)
        gauss_lobatto01(nq, chi, w);
    else
        gauss_legendre01(nq, chi, w);
    std::memset(tb, 0, sizeof(*tb));
    lagrange_tables(p, nq, xi, chi, tb->B, tb->G);
    for (int q = 0; q < nq; ++q) tb->w[q] = w[q];
    for (int k = 0; k < MAXNQ * MAXNI; ++k) {
        tb->Bf[k] = (float)tb->B[k];
        tb->Gf[k] = (float)tb->G[k];
    }
    return TMOP_OK;
}

int internal_target(const tmop_params *prm, int d, Target *tp)
{
    Target &t = *tp;
    t.metric = prm->metric;
    t.ideal = prm->has_W ? 0 : 1;
    t.detW = 1.0;
    for (int k = 0; k < 9; ++k) t.Winv[k] = 0.0;
    if (prm->has_W) {
        const double *W = prm->W;
        double det, inv[9];
        if (d == 2) {
            det = W[0] * W[3] - W[1] * W[2];
            inv[0] = W[3] / det;
            inv[1] = -W[1] / det;
            inv[2] = -W[2] / det;
            inv[3] = W[0] / det;
        } else {
            const double c00 = W[4] * W[8] - W[5] * W[7], c01 = W[5] * W[6] - W[3] * W[8],
                         c02 = W[3] * W[7] - W[4] * W[6];
            det = W[0] * c00 + W[1] * c01 + W[2] * c02;
            // inverse = adj / det, adj = cof^T
            inv[0] = c00 / det;
            inv[3] = c01 / det;
            inv[6] = c02 / det;
            inv[1] = (W[2] * W[7] - W[1] * W[8]) / det;
            inv[4] = (W[0] * W[8] - W[2] * W[6]) / det;
            inv[7] = (W[1] * W[6] - W[0] * W[7]) / det;
            inv[2] = (W[1] * W[5] - W[2] * W[4]) / det;
            inv[5] = (W[2] * W[3] - W[0] * W[5]) / det;
            inv[8] = (W[0] * W[4] - W[1] * W[3]) / det;
        }
        if (!(det > 0.0) || !std::isfinite(det)) return TMOP_ERR_INVALID_ARG;
        t.detW = det;
        for (int k = 0; k < d * d; ++k) t.Winv[k] = inv[k];
    }
    return TMOP_OK;
}

}  // namespace tmop

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------

enum { SV_DX, SV_XT, SV_G, SV_GT, SV_R1, SV_R2, SV_Y, SV_V, SV_W, SV_W1, SV_W2, SV_COUNT };

struct tmop_ctx {
    double *x0buf = nullptr;  // reference nodes of the limiting term (library copy)
    int tile = 1;             // Hessian-action tile shape (index into Ops::epb_t)
    int sweeps = TMOP_SWEEPS_PENCIL;  // forward sweeps of energy, gradient, setup
    Geom g{};
    Tables tb{};
    Target tg{};
    Ops ops{};
    int dim = 0, p = 0, nq = 0, ni = 0, np = 0, nqe = 0, ne = 0, nx = 0, ndof = 0;
    int precision = TMOP_FP64;
    int storage = TMOP_HESS_TENSOR;
    int grid = 0;
    hipStream_t s = nullptr;
    void *H = nullptr;
    size_t H_bytes = 0;
    bool have_setup = false;
    void *eV = nullptr;
    size_t eV_bytes = 0;
    double *part = nullptr;
    int part_len = 0;
    double *scal = nullptr;   // device scalars
    double *hscal = nullptr;  // pinned host mirror
    int32_t *csr_ptr = nullptr, *csr_ent = nullptr;
    double *diag = nullptr, *minv = nullptr;
    bool have_diag = false;
    double *sv[SV_COUNT] = {};
    MinresState *mst = nullptr;
    MinresState *hmst = nullptr;
    // resident Lanczos vectors (bank_cap of them, bank_stride doubles apart)
    // and the per-update scalars; bank_limit caps the bank's bytes
    double *bank = nullptr;
    int bank_cap = 0;
    long bank_stride = 0;
    size_t bank_limit = SIZE_MAX;
    MrHist *mhist = nullptr;
    // HIP-event timing of the Hessian actions inside MINRES
    bool timing = false;
    std::vector<hipEvent_t> tev;
    std::vector<tmop_iter_record> hist;  // per-iteration record of the last tmop_solve
    int tev_used = 0;
    double acc_apply_ms = 0.0, acc_elem_ms = 0.0;
    int acc_napply = 0;
};

static int ctx_sizes(const tmop_mesh_desc *m, const tmop_params *prm, long &ne, long &nx,
                     int &nqe, int &np)
{
    if (!m || !prm) return fail(TMOP_ERR_INVALID_ARG, "null mesh or params");
    if (m->dim != 2 && m->dim != 3) return fail(TMOP_ERR_INVALID_ARG, "dim must be 2 or 3");
    if (m->order_p < 1 || m->order_p > 4)
        return fail(TMOP_ERR_UNSUPPORTED, "order_p must be in 1..4");
    const int p = m->order_p, d = m->dim;
    np = d == 3 ? (p + 1) * (p + 1) * (p + 1) : (p + 1) * (p + 1);
    if (prm->nq1d < 2 || prm->nq1d > MAXNQ) return fail(TMOP_ERR_INVALID_ARG, "nq1d out of range");
    nqe = d == 3 ? prm->nq1d * prm->nq1d * prm->nq1d : prm->nq1d * prm->nq1d;
    if (m->elem_to_node) {
        if (m->num_elems <= 0 || m->num_nodes <= 0)
            return fail(TMOP_ERR_INVALID_ARG, "general mesh needs num_elems and num_nodes");
        ne = m->num_elems;
        nx = m->num_nodes;
    } else {
        if (m->nx <= 0 || m->ny <= 0 || (d == 3 && m->nz <= 0))
            return fail(TMOP_ERR_INVALID_ARG, "structured box needs nx, ny (, nz) > 0");
        ne = (long)m->nx * m->ny * (d == 3 ? m->nz : 1);
        nx = (long)(m->nx * p + 1) * (m->ny * p + 1) * (d == 3 ? (m->nz * p + 1) : 1);
    }
    if (ne * (long)np * d > INT_MAX || nx * (long)d > INT_MAX)
        return fail(TMOP_ERR_INVALID_ARG, "mesh too large for 32-bit indexing");
    return TMOP_OK;
}

extern "C" int tmop_workspace_bytes(const tmop_mesh_desc *m, const tmop_params *prm,
                                    int with_solver, size_t *bytes)
{
    long ne, nx;
    int nqe, np;
    CHK(ctx_sizes(m, prm, ne, nx, nqe, np));
    const int d = m->dim;
    const int S = prm->hess_storage == TMOP_HESS_COMPACT ? (d == 3 ? 13 : 8) : d * d * (d * d + 1) / 2;
    const size_t tb = prm->precision == TMOP_MIXED ? 4 : 8;
    size_t b = align256((size_t)ne * qdata_stride(S, nqe, (int)tb) * tb);
    b += align256((size_t)ne * d * np * 8);
    b += align256(sizeof(double) * (3 * ((ne + 0) + 1024) + 64));
    b += 2 * align256((size_t)d * nx * 8);  // diag, minv
    if (m->elem_to_node) b += align256((nx + 1) * 4) + align256((size_t)ne * np * 4);
    if (with_solver) b += SV_COUNT * align256((size_t)d * nx * 8);
    *bytes = b;
    return TMOP_OK;
}

extern "C" int tmop_sizes(const tmop_ctx *c, int *num_nodes, int *num_dofs)
{
    if (!c) return fail(TMOP_ERR_INVALID_ARG, "null context");
    if (num_nodes) *num_nodes = c->nx;
    if (num_dofs) *num_dofs = c->ndof;
    return TMOP_OK;
}

extern "C" int tmop_basis_nodes(int p, double *nodes)
{
    if (p < 1 || p >= MAXNI || !nodes) return fail(TMOP_ERR_INVALID_ARG, "bad order or pointer");
    gll_nodes01(p, nodes);
    return TMOP_OK;
}

static void free_ctx(tmop_ctx *c)
{
    if (!c) return;
    for (auto &e : c->tev) hipEventDestroy(e);
    hipFree(c->H);
    hipFree(c->eV);
    hipFree(c->part);
    hipFree(c->scal);
    if (c->hscal) hipHostFree(c->hscal);
    hipFree(c->csr_ptr);
    hipFree(c->csr_ent);
    hipFree(c->diag);
    hipFree(c->minv);
    hipFree(c->x0buf);
    for (auto &v : c->sv) hipFree(v);
    hipFree(c->mst);
    hipFree(c->bank);
    hipFree(c->mhist);
    if (c->hmst) hipHostFree(c->hmst);
    delete c;
}

extern "C" int tmop_create(tmop_ctx **out, const tmop_mesh_desc *m, const tmop_params *prm,
                           void *stream)
{
    if (!out) return fail(TMOP_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    long ne, nx;
    int nqe, np;
    CHK(ctx_sizes(m, prm, ne, nx, nqe, np));
    const int d = m->dim, p = m->order_p, nq = prm->nq1d;
    if (!metric_supported(d, prm->metric))
        return fail(TMOP_ERR_UNSUPPORTED, "metric must be 2, 7, 9 or 55 (dim 2) or 303 or 55 (dim 3)");
    if (prm->precision != TMOP_FP64 && prm->precision != TMOP_MIXED)
        return fail(TMOP_ERR_INVALID_ARG, "precision must be TMOP_FP64 or TMOP_MIXED");
    if (prm->hess_storage != TMOP_HESS_TENSOR && prm->hess_storage != TMOP_HESS_COMPACT)
        return fail(TMOP_ERR_INVALID_ARG, "hess_storage must be TMOP_HESS_TENSOR or _COMPACT");
    if (m->ess_mode == TMOP_ESS_BOUNDARY && m->elem_to_node)
        return fail(TMOP_ERR_INVALID_ARG, "TMOP_ESS_BOUNDARY needs the structured box");
    if (m->ess_mode == TMOP_ESS_MASK && !m->ess_mask)
        return fail(TMOP_ERR_INVALID_ARG, "TMOP_ESS_MASK needs ess_mask");
    if (m->ess_mode < 0 || m->ess_mode > 2) return fail(TMOP_ERR_INVALID_ARG, "bad ess_mode");
    Ops ops;
    if (!find_ops(d, p, nq, &ops))
        return fail(TMOP_ERR_UNSUPPORTED, "no kernel for this (dim, p, nq1d); nq1d must be p+1..p+3");

    tmop_ctx *c = new tmop_ctx();
    c->ops = ops;
    c->dim = d;
    c->p = p;
    c->nq = nq;
    c->ni = p + 1;
    c->np = np;
    c->nqe = nqe;
    c->ne = (int)ne;
    c->nx = (int)nx;
    c->ndof = (int)(d * nx);
    c->precision = prm->precision;
    c->storage = prm->hess_storage;
    c->s = (hipStream_t)stream;
    c->grid = (int)((ne + ops.epb - 1) / ops.epb);
    const int tt = tuned_tile(d, p, nq, c->storage, c->precision);
    if (tt >= 0 && ops.epb_t[tt] > 0) c->tile = tt;

    Geom &g = c->g;
    g.dim = d;
    g.p = p;
    g.ne = (int)ne;
    g.nx = (int)nx;
    if (!m->elem_to_node) {
        g.nel[0] = m->nx;
        g.nel[1] = m->ny;
        g.nel[2] = d == 3 ? m->nz : 1;
        for (int k = 0; k < 3; ++k) g.M[k] = g.nel[k] * p + 1;
        if (d == 2) g.M[2] = 1;
    }
    set_divisors(g);
    g.e2n = m->elem_to_node;
    g.ess_mode = m->ess_mode;
    g.ess = m->ess_mask;

    if (internal_tables(p, nq, &c->tb, prm->quad_rule) != TMOP_OK) {
        delete c;
        return fail(TMOP_ERR_INVALID_ARG, "quad_rule must be TMOP_QUAD_GL or TMOP_QUAD_GLL");
    }
    if (internal_target(prm, d, &c->tg) != TMOP_OK) {
        delete c;
        return fail(TMOP_ERR_INVALID_ARG, "target W must have det > 0");
    }

    // workspace
    const int S = c->storage == TMOP_HESS_COMPACT ? (d == 3 ? 13 : 8) : d * d * (d * d + 1) / 2;
    const size_t tbytes = c->precision == TMOP_MIXED ? 4 : 8;
    c->H_bytes = (size_t)ne * qdata_stride(S, nqe, (int)tbytes) * tbytes;
    c->eV_bytes = (size_t)ne * d * np * 8;
    c->part_len = std::max(3 * std::max(c->grid, 1024), 2 * MR_MAX_PARTIALS + 1024) + 64;
    hipError_t e = hipSuccess;
#define ALLOC(ptr, bytes)                                       \
    if (e == hipSuccess) e = hipMalloc((void **)&(ptr), (bytes));
    ALLOC(c->H, c->H_bytes);
    ALLOC(c->eV, c->eV_bytes);
    ALLOC(c->part, sizeof(double) * c->part_len);
    ALLOC(c->scal, sizeof(double) * 64);
    ALLOC(c->diag, sizeof(double) * c->ndof);
    ALLOC(c->minv, sizeof(double) * c->ndof);
    ALLOC(c->mst, 2 * sizeof(MinresState));
    ALLOC(c->mhist, MR_MAX_BASIS * sizeof(MrHist));
#undef ALLOC
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->hscal, sizeof(double) * 64, 0);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->hmst, 2 * sizeof(MinresState), 0);
    if (e != hipSuccess) {
        free_ctx(c);
        return fail(e == hipErrorOutOfMemory ? TMOP_ERR_OOM : TMOP_ERR_HIP,
                    std::string("workspace allocation: ") + hipGetErrorString(e));
    }

    // general mesh: node -> (element, local) CSR for the deterministic G^T
    if (m->elem_to_node) {
        std::vector<int32_t> e2n((size_t)ne * np);
        e = hipMemcpy(e2n.data(), m->elem_to_node, e2n.size() * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            free_ctx(c);
            return fail(TMOP_ERR_HIP, "copying elem_to_node");
        }
        std::vector<int32_t> ptr(nx + 1, 0), ent(e2n.size());
        for (size_t k = 0; k < e2n.size(); ++k) {
            if (e2n[k] < 0 || e2n[k] >= nx) {
                free_ctx(c);
                return fail(TMOP_ERR_INVALID_ARG, "elem_to_node entry out of range");
            }
            ptr[e2n[k] + 1]++;
        }
        for (long k = 0; k < nx; ++k) ptr[k + 1] += ptr[k];
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
        for (size_t k = 0; k < e2n.size(); ++k) ent[fill[e2n[k]]++] = (int32_t)k;
        e = hipMalloc((void **)&c->csr_ptr, ptr.size() * 4);
        if (e == hipSuccess) e = hipMalloc((void **)&c->csr_ent, ent.size() * 4);
        if (e == hipSuccess) e = hipMemcpy(c->csr_ptr, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c->csr_ent, ent.data(), ent.size() * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            free_ctx(c);
            return fail(TMOP_ERR_HIP, "uploading node map");
        }
    }
    *out = c;
    return TMOP_OK;
}

extern "C" int tmop_destroy(tmop_ctx *c)
{
    if (!c) return TMOP_OK;
    hipStreamSynchronize(c->s);
    free_ctx(c);
    return TMOP_OK;
}

// ---------------------------------------------------------------------------
// Evaluations
// ---------------------------------------------------------------------------

// The matrix-core forward sweeps apply when chosen and the objective has no
// limiting term.
static bool use_mfma(const tmop_ctx *c)
{
    return c->sweeps == TMOP_SWEEPS_MFMA && c->g.lim == 0.0;
}

static int energy_mindet_impl(tmop_ctx *c, const double *x, double *F, double *mindet)
{
    (use_mfma(c) ? c->ops.energyM : c->ops.energy)(c->grid, c->s, c->g, c->tb, c->tg, x, c->part);
    launch_reduce3(c->part, c->grid, c->scal, c->s);
    HIPCHK(hipMemcpyAsync(c->hscal, c->scal, 3 * sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    const double bad = c->hscal[2];
    if (mindet) *mindet = c->hscal[1];
    if (F) *F = bad > 0.0 ? INFINITY : c->hscal[0];
    if (bad > 0.0) return fail(TMOP_ERR_INVERTED, "det T <= 0 at a quadrature point");
    return TMOP_OK;
}

extern "C" int tmop_energy(tmop_ctx *c, const double *x, double *F)
{
    if (!c || !x || !F) return fail(TMOP_ERR_INVALID_ARG, "null argument");
    return energy_mindet_impl(c, x, F, nullptr);
}

extern "C" int tmop_min_det(tmop_ctx *c, const double *x, double *md)
{
    if (!c || !x || !md) return fail(TMOP_ERR_INVALID_ARG, "null argument");
    const int r = energy_mindet_impl(c, x, nullptr, md);
    return r == TMOP_ERR_INVERTED ? TMOP_OK : r;
}

extern "C" int tmop_energy_mindet(tmop_ctx *c, const double *x, double *F, double *md)
{
    if (!c || !x) return fail(TMOP_ERR_INVALID_ARG, "null argument");
    return energy_mindet_impl(c, x, F, md);
}

static void gradient_impl(tmop_ctx *c, const double *x, double *g)
{
    (use_mfma(c) ? c->ops.gradientM : c->ops.gradient)(c->grid, c->s, c->g, c->tb, c->tg, x,
                                                       (double *)c->eV, c->part);
    launch_gather(c->g, c->csr_ptr, c->csr_ent, c->eV, false, g, 0, nullptr, c->s);
}

// Energy, min det A, gradient and |g|^2 of one point in one element pass
// (the gradient kernel also sums the energy) and one host synchronisation.
// F, md and g are bitwise those of energy_mindet_impl and gradient_impl, g2
// a dot of g with itself.  F = inf and TMOP_ERR_INVERTED when det T <= 0
// somewhere (g is then of no use).
static int energy_gradient_impl(tmop_ctx *c, const double *x, double *F, double *md, double *g,
                                double *g2)
{
    (use_mfma(c) ? c->ops.gradientEM : c->ops.gradientE)(c->grid, c->s, c->g, c->tb, c->tg, x,
                                                         (double *)c->eV, c->part);
    launch_reduce3(c->part, c->grid, c->scal, c->s);
    launch_gather(c->g, c->csr_ptr, c->csr_ent, c->eV, false, g, 0, nullptr, c->s);
    launch_dot(c->ndof, g, g, c->part, c->scal + 8, c->s);
    HIPCHK(hipMemcpyAsync(c->hscal, c->scal, 9 * sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    const double bad = c->hscal[2];
    *md = c->hscal[1];
    *F = bad > 0.0 ? INFINITY : c->hscal[0];
    *g2 = c->hscal[8];
    if (bad > 0.0) return fail(TMOP_ERR_INVERTED, "det T <= 0 at a quadrature point");
    return TMOP_OK;
}

extern "C" int tmop_energy_gradient(tmop_ctx *c, const double *x, double *F, double *md,
                                    double *g, double *g2)
{
    if (!c || !x || !g) return fail(TMOP_ERR_INVALID_ARG, "null argument");
    double f, m, gg;
    const int r = energy_gradient_impl(c, x, &f, &m, g, &gg);
    if (F) *F = f;
    if (md) *md = m;
    if (g2) *g2 = gg;
    return r;
}

extern "C" int tmop_gradient(tmop_ctx *c, const double *x, double *g)
{
    if (!c || !x || !g) return fail(TMOP_ERR_INVALID_ARG, "null argument");
    gradient_impl(c, x, g);
    HIPCHK(hipGetLastError());
    return TMOP_OK;
}

static void setup_impl(tmop_ctx *c, const double *x)
{
    const bool mixed = c->precision == TMOP_MIXED;
    if (c->storage == TMOP_HESS_COMPACT) {
        if (mixed)
            c->ops.setupc32(c->grid, c->s, c->g, c->tb, c->tg, x, (float *)c->H, c->part);
        else
            (use_mfma(c) ? c->ops.setupcM64 : c->ops.setupc64)(c->grid, c->s, c->g, c->tb, c->tg,
                                                               x, (double *)c->H, c->part);
    } else if (mixed)
        c->ops.setup32(c->grid, c->s, c->g, c->tb, c->tg, x, (float *)c->H, c->part);
    else
        (use_mfma(c) ? c->ops.setupM64 : c->ops.setup64)(c->grid, c->s, c->g, c->tb, c->tg, x,
                                                         (double *)c->H, c->part);
    c->have_setup = true;
    c->have_diag = false;
}

extern "C" int tmop_hessian_setup(tmop_ctx *c, const double *x)
{
    if (!c || !x) return fail(TMOP_ERR_INVALID_ARG, "null argument");
    setup_impl(c, x);
    HIPCHK(hipGetLastError());
    return TMOP_OK;
}

static void apply_elem(tmop_ctx *c, const double *v)
{
    // the autotuned tile shape; the variant with the limiting term has the base one
    const int t = c->g.lim != 0.0 ? 1 : c->tile;
    const int grid = (int)((c->g.ne + c->ops.epb_t[t] - 1) / c->ops.epb_t[t]);
    if (c->storage == TMOP_HESS_COMPACT) {
        if (c->precision == TMOP_MIXED)
            (t == 1 ? c->ops.applyc32 : c->ops.applyc32_t[t])(grid, c->s, c->g, c->tb, c->tg,
                                                              (const float *)c->H, v, (float *)c->eV);
        else
            (t == 1 ? c->ops.applyc64 : c->ops.applyc64_t[t])(grid, c->s, c->g, c->tb, c->tg,
                                                              (const double *)c->H, v, (double *)c->eV);
        return;
    }
    if (c->precision == TMOP_MIXED)
        (t == 1 ? c->ops.apply32 : c->ops.apply32_t[t])(grid, c->s, c->g, c->tb, (const float *)c->H, v,
                                                        (float *)c->eV);
    else
        (t == 1 ? c->ops.apply64 : c->ops.apply64_t[t])(grid, c->s, c->g, c->tb, (const double *)c->H, v,
                                                        (double *)c->eV);
}

static void apply_gather(tmop_ctx *c, const double *v, double *y)
{
    launch_gather(c->g, c->csr_ptr, c->csr_ent, c->eV, c->precision == TMOP_MIXED, y, 2, v, c->s);
}

extern "C" int tmop_hessian_apply(tmop_ctx *c, const double *v, double *y)
{
    if (!c || !v || !y) return fail(TMOP_ERR_INVALID_ARG, "null argument");
    if (v == y) return fail(TMOP_ERR_INVALID_ARG, "v and y must not alias");
    if (!c->have_setup) return fail(TMOP_ERR_STATE, "tmop_hessian_setup was not called");
    apply_elem(c, v);
    apply_gather(c, v, y);
    HIPCHK(hipGetLastError());
    return TMOP_OK;
}

// Setup and the element diagonal (into eV) in one kernel, where the class
// has it (hexes with one pass of points per workgroup, pencil sweeps);
// false, with nothing launched, elsewhere.
static bool setup_diag_impl(tmop_ctx *c, const double *x)
{
    if (use_mfma(c)) return false;
    const bool cp = c->storage == TMOP_HESS_COMPACT;
    if (c->precision == TMOP_MIXED) {
        const auto f = cp ? c->ops.setupcd32 : c->ops.setupd32;
        if (!f) return false;
        f(c->grid, c->s, c->g, c->tb, c->tg, x, (float *)c->H, (double *)c->eV, c->part);
    } else {
        const auto f = cp ? c->ops.setupcd64 : c->ops.setupd64;
        if (!f) return false;
        f(c->grid, c->s, c->g, c->tb, c->tg, x, (double *)c->H, (double *)c->eV, c->part);
    }
    c->have_setup = true;
    c->have_diag = false;
    return true;
}

static void diag_impl(tmop_ctx *c, double *d)
{
    if (c->storage == TMOP_HESS_COMPACT) {
        if (c->precision == TMOP_MIXED)
            c->ops.diagc32(c->grid, c->s, c->g, c->tb, c->tg, (const float *)c->H, (double *)c->eV);
        else
            c->ops.diagc64(c->grid, c->s, c->g, c->tb, c->tg, (const double *)c->H, (double *)c->eV);
    } else if (c->precision == TMOP_MIXED)
        c->ops.diag32(c->grid, c->s, c->g, c->tb, (const float *)c->H, (double *)c->eV);
    else
        c->ops.diag64(c->grid, c->s, c->g, c->tb, (const double *)c->H, (double *)c->eV);
    launch_gather(c->g, c->csr_ptr, c->csr_ent, c->eV, false, d, 1, nullptr, c->s);
}

extern "C" int tmop_hessian_diag(tmop_ctx *c, double *d)
{
    if (!c || !d) return fail(TMOP_ERR_INVALID_ARG, "null argument");
    if (!c->have_setup) return fail(TMOP_ERR_STATE, "tmop_hessian_setup was not called");
    diag_impl(c, d);
    HIPCHK(hipGetLastError());
    return TMOP_OK;
}

// Setup and diagonal: one kernel where the class has it, else the two.
static void setup_diag_to(tmop_ctx *c, const double *x, double *d)
{
    if (setup_diag_impl(c, x)) {
        launch_gather(c->g, c->csr_ptr, c->csr_ent, c->eV, false, d, 1, nullptr, c->s);
    } else {
        setup_impl(c, x);
        diag_impl(c, d);
    }
}

extern "C" int tmop_hessian_setup_diag(tmop_ctx *c, const double *x, double *d)
{
    if (!c || !x || !d) return fail(TMOP_ERR_INVALID_ARG, "null argument");
    setup_diag_to(c, x, d);
    HIPCHK(hipGetLastError());
    return TMOP_OK;
}

extern "C" int tmop_time_apply(tmop_ctx *c, const double *v, double *y, int n, double *elem_ms,
                               double *total_ms)
{
    if (!c || !v || !y || n <= 0) return fail(TMOP_ERR_INVALID_ARG, "bad argument");
    if (!c->have_setup) return fail(TMOP_ERR_STATE, "tmop_hessian_setup was not called");
    std::vector<hipEvent_t> ev(3 * n);
    for (auto &e : ev) HIPCHK(hipEventCreate(&e));
    for (int k = 0; k < n; ++k) {
        HIPCHK(hipEventRecord(ev[3 * k], c->s));
        apply_elem(c, v);
        HIPCHK(hipEventRecord(ev[3 * k + 1], c->s));
        apply_gather(c, v, y);
        HIPCHK(hipEventRecord(ev[3 * k + 2], c->s));
    }
    HIPCHK(hipStreamSynchronize(c->s));
    double se = 0.0, st = 0.0;
    for (int k = 0; k < n; ++k) {
        float a = 0.f, b = 0.f;
        HIPCHK(hipEventElapsedTime(&a, ev[3 * k], ev[3 * k + 1]));
        HIPCHK(hipEventElapsedTime(&b, ev[3 * k], ev[3 * k + 2]));
        se += a;
        st += b;
    }
    (void)st;
    // whole actions back to back, events only around the run: the action
    // rate without the event records between its two kernels
    HIPCHK(hipEventRecord(ev[0], c->s));
    for (int k = 0; k < n; ++k) {
        apply_elem(c, v);
        apply_gather(c, v, y);
    }
    HIPCHK(hipEventRecord(ev[1], c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    float tt = 0.f;
    HIPCHK(hipEventElapsedTime(&tt, ev[0], ev[1]));
    for (auto &e : ev) hipEventDestroy(e);
    if (elem_ms) *elem_ms = se / n;
    if (total_ms) *total_ms = (double)tt / n;
    return TMOP_OK;
}

// ---------------------------------------------------------------------------
// Solver
// ---------------------------------------------------------------------------

static int ensure_solver(tmop_ctx *c)
{
    if (c->sv[0]) return TMOP_OK;
    for (int k = 0; k < SV_COUNT; ++k) HIPCHK(hipMalloc((void **)&c->sv[k], sizeof(double) * c->ndof));
    return TMOP_OK;
}

// |a|^2 to host (synchronises).
static int dot_host(tmop_ctx *c, const double *a, const double *b, double *out)
{
    launch_dot(c->ndof, a, b, c->part, c->scal + 8, c->s);
    HIPCHK(hipMemcpyAsync(c->hscal + 8, c->scal + 8, sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    *out = c->hscal[8];
    return TMOP_OK;
}

// The Jacobi preconditioner from the diagonal in c->diag.
static void jacobi_from_diag(tmop_ctx *c)
{
    launch_absmax(c->ndof, c->diag, c->part, c->scal + 9, c->s);
    launch_jacobi(c->ndof, c->diag, c->scal + 9, c->minv, c->s);
    c->have_diag = true;
}

static void make_jacobi(tmop_ctx *c)
{
    diag_impl(c, c->diag);
    jacobi_from_diag(c);
}

// Room for nvec resident Lanczos vectors, within bank_limit.  False (and
// nothing allocated) when they do not fit; the solve then takes the
// three-term update on every iteration.
static bool ensure_bank(tmop_ctx *c, int nvec)
{
    if (nvec > MR_MAX_BASIS) return false;
    const long stride = ((long)c->ndof + 31) / 32 * 32;  // 256-byte aligned vectors
    const size_t need = (size_t)nvec * stride * sizeof(double);
    if (need > c->bank_limit) return false;
    if (c->bank && c->bank_cap >= nvec) return true;
    if (c->bank) {
        // the previous solve's kernels may still read the old bank
        if (hipStreamSynchronize(c->s) != hipSuccess) return false;
        hipFree(c->bank);
        c->bank = nullptr;
        c->bank_cap = 0;
    }
    if (hipMalloc((void **)&c->bank, need) != hipSuccess) {
        (void)hipGetLastError();  // out of memory is not an error here
        c->bank = nullptr;
        return false;
    }
    c->bank_cap = nvec;
    c->bank_stride = stride;
    return true;
}

// Iterations with the preconditioned Lanczos vectors resident in the bank:
// z_j in bank vector j, the update scalars to mhist, dx formed once at the
// end.  Returns the iterations run.
static int minres_resident(tmop_ctx *c, const double *minv, double *R1, double *R2,
                           double *const P1[2], double *P2, double *dx, int max_its,
                           int check_every)
{
    const long n = c->ndof;
    const bool fp32 = c->precision == TMOP_MIXED;
    const int nbg = mr_gather_grid(c->g);
    int J = 0;
    for (int j = 0; j < max_its; ++j) {
        // S_{j-1} in mst[(j-1)&1], S_j to mst[j&1]
        MinresState *sin = c->mst + ((j + 1) & 1), *sout = c->mst + (j & 1);
        const double *zc = c->bank + (long)j * c->bank_stride;
        double *znext = c->bank + (long)(j + 1) * c->bank_stride;
        const bool rec = c->timing && c->tev_used + 3 <= (int)c->tev.size();
        if (rec) (void)hipEventRecord(c->tev[c->tev_used], c->s);
        apply_elem(c, zc);
        if (rec) (void)hipEventRecord(c->tev[c->tev_used + 1], c->s);
        // scalars of update j-1 to mhist, then G^T with the first Lanczos
        // update into R1
        mr_gather_upd(c->g, c->csr_ptr, c->csr_ent, c->eV, fp32, j, sin, sout, P1[(j + 1) & 1],
                      P2, nullptr, zc, nullptr, nullptr, nullptr, nullptr, R1, P1[j & 1],
                      c->mhist, c->s);
        if (rec) {
            (void)hipEventRecord(c->tev[c->tev_used + 2], c->s);
            c->tev_used += 3;
        }
        mr_lanczos2(n, nbg, j, sout, P1[j & 1], R1, R2, minv, znext, P2, c->s);
        std::swap(R1, R2);  // r1 <- r2, r2 <- hv
        J = j + 1;
        if (check_every > 0 && (j + 1) % check_every == 0 && j + 1 < max_its) {
            (void)hipMemcpyAsync(c->hmst, sout, sizeof(MinresState), hipMemcpyDeviceToHost, c->s);
            (void)hipStreamSynchronize(c->s);
            if (c->hmst->stop != 0x7fffffff) break;
        }
    }
    // the last update, then dx from the resident vectors (dx = 0 from the
    // start when nothing ran)
    if (J > 0)
        mr_combine(n, nbg, J - 1, c->mst + ((J - 1) & 1), c->mst + (J & 1), P1[(J - 1) & 1], P2,
                   c->mhist, c->bank, c->bank_stride, dx, c->s);
    // R1/R2 are scratch between calls; keep the pool's pointers as they were
    return J;
}

// Iterations with the three-term solution update in every gather (the
// Lanczos vectors ping-pong between two buffers).  Returns the iterations run.
static int minres_three_term(tmop_ctx *c, const double *minv, double *const P1[2], double *P2,
                             double *dx, int max_its, int check_every)
{
    const long n = c->ndof;
    const bool fp32 = c->precision == TMOP_MIXED;
    const int nbg = mr_gather_grid(c->g);
    // R1: r1, overwritten in place by hv; R2: r2; ZC: z_{j-1} (the element
    // kernel's input, v_j = z_{j-1} / beta_j); ZP: z_{j-2}, then z_j
    double *R1 = c->sv[SV_R1], *R2 = c->sv[SV_R2], *ZC = c->sv[SV_Y], *ZP = c->sv[SV_V];
    double *W = c->sv[SV_W], *W1 = c->sv[SV_W1], *W2 = c->sv[SV_W2];
    int J = 0;
    for (int j = 0; j < max_its; ++j) {
        MinresState *sin = c->mst + ((j + 1) & 1), *sout = c->mst + (j & 1);
        const bool rec = c->timing && c->tev_used + 3 <= (int)c->tev.size();
        if (rec) (void)hipEventRecord(c->tev[c->tev_used], c->s);
        apply_elem(c, ZC);
        if (rec) (void)hipEventRecord(c->tev[c->tev_used + 1], c->s);
        // deferred update of iteration j-1 (formula's w1, w2 = buffers W2, W;
        // new w into W1), then G^T with the first Lanczos update into R1
        mr_gather_upd(c->g, c->csr_ptr, c->csr_ent, c->eV, fp32, j, sin, sout, P1[(j + 1) & 1],
                      P2, ZP, ZC, W2, W, W1, dx, R1, P1[j & 1], nullptr, c->s);
        if (rec) {
            (void)hipEventRecord(c->tev[c->tev_used + 2], c->s);
            c->tev_used += 3;
        }
        // z_j into ZP (z_{j-2} is dead after the update above)
        mr_lanczos2(n, nbg, j, sout, P1[j & 1], R1, R2, minv, ZP, P2, c->s);
        std::swap(R1, R2);  // r1 <- r2, r2 <- hv
        std::swap(ZP, ZC);  // z_{j-1}, z_j
        if (j >= 1) {
            double *oW = W, *oW1 = W1, *oW2 = W2;
            W1 = oW2;
            W2 = oW;
            W = oW1;
        }
        J = j + 1;
        if (check_every > 0 && (j + 1) % check_every == 0 && j + 1 < max_its) {
            (void)hipMemcpyAsync(c->hmst, sout, sizeof(MinresState), hipMemcpyDeviceToHost, c->s);
            (void)hipStreamSynchronize(c->s);
            if (c->hmst->stop != 0x7fffffff) break;
        }
    }
    // the update of the last iteration run
    if (J > 0) {
        mr_finish(n, nbg, J - 1, c->mst + ((J - 1) & 1), c->mst + (J & 1), P1[(J - 1) & 1], P2,
                  ZP, W2, W, W1, dx, c->s);
        double *oW = W, *oW1 = W1, *oW2 = W2;
        W1 = oW2;
        W2 = oW;
        W = oW1;
    }
    // keep the rotated pointers consistent for the next call
    c->sv[SV_Y] = ZC;
    c->sv[SV_V] = ZP;
    c->sv[SV_R1] = R1;
    c->sv[SV_R2] = R2;
    c->sv[SV_W] = W;
    c->sv[SV_W1] = W1;
    c->sv[SV_W2] = W2;
    return J;
}

// MINRES on H_c dx = b, x_0 = 0.  Device state double-buffered in
// c->mst[0..1] (see vec.hip for the recurrences).  When the max_its + 1
// preconditioned Lanczos vectors fit in the bank they stay resident and dx
// is formed once after the loop; otherwise every iteration takes the
// three-term solution update.
static int minres_impl(tmop_ctx *c, const double *b, double *dx, int max_its, double rtol,
                       bool jacobi, int check_every, int *its_out)
{
    CHK(ensure_solver(c));
    const long n = c->ndof;
    // part1 alternates between iterations (iteration j reads j-1's while writing its own)
    // alpha partials (one per gather workgroup), double-buffered, then beta^2
    double *const P1[2] = {c->part, c->part + MR_MAX_PARTIALS};
    double *P2 = c->part + 2 * MR_MAX_PARTIALS;
    const double *minv = jacobi ? c->minv : nullptr;
    const bool resident = ensure_bank(c, max_its + 1);
    c->tev_used = 0;
    if (resident) {
        // z_{-1} = M^{-1} b is bank vector 0; no w vectors
        mr_init(n, b, minv, c->sv[SV_R1], c->sv[SV_R2], c->bank, nullptr, dx, nullptr, nullptr,
                nullptr, P1[0], c->mst, rtol, c->s);
        minres_resident(c, minv, c->sv[SV_R1], c->sv[SV_R2], P1, P2, dx, max_its, check_every);
    } else {
        mr_init(n, b, minv, c->sv[SV_R1], c->sv[SV_R2], c->sv[SV_Y], nullptr, dx, c->sv[SV_W],
                c->sv[SV_W1], c->sv[SV_W2], P1[0], c->mst, rtol, c->s);
        minres_three_term(c, minv, P1, P2, dx, max_its, check_every);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c->hmst, c->mst, 2 * sizeof(MinresState), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    const MinresState &fin = c->hmst[0].its >= c->hmst[1].its ? c->hmst[0] : c->hmst[1];
    if (its_out) *its_out = fin.its;
    // every recorded action is counted (the element kernel runs even after
    // convergence; only the vector kernels skip)
    for (int k = 0; k + 2 < c->tev_used; k += 3) {
        float a = 0.f, bt = 0.f;
        HIPCHK(hipEventElapsedTime(&a, c->tev[k], c->tev[k + 1]));
        HIPCHK(hipEventElapsedTime(&bt, c->tev[k], c->tev[k + 2]));
        c->acc_elem_ms += a;
        c->acc_apply_ms += bt;
        c->acc_napply += 1;
    }
    c->tev_used = 0;
    if (fin.indefinite_precond) return fail(TMOP_ERR_NONFINITE, "preconditioner not SPD");
    return TMOP_OK;
}

extern "C" int tmop_minres(tmop_ctx *c, const double *b, double *dx, int max_its, double rtol,
                           int jacobi, int *its)
{
    if (!c || !b || !dx || max_its < 0) return fail(TMOP_ERR_INVALID_ARG, "bad argument");
    if (!c->have_setup) return fail(TMOP_ERR_STATE, "tmop_hessian_setup was not called");
    if (jacobi && !c->have_diag) make_jacobi(c);
    return minres_impl(c, b, dx, max_its, rtol, jacobi != 0, 8, its);
}

static double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// One Newton update of x (in place): setup, Jacobi, MINRES, line search.
// F, gn, g (in c->sv[SV_G]) describe x on entry and are updated on accept.
static int newton_update(tmop_ctx *c, double *x, double &F, double &gn, int max_minres,
                         double rtol, int max_halvings, bool jacobi, int check_every,
                         tmop_solve_report *rep)
{
    TraceRange step_range("tmop newton step");
    double t0 = now_ms();
    {
        TraceRange r("tmop setup+diagonal");
        if (jacobi) {
            setup_diag_to(c, x, c->diag);
            jacobi_from_diag(c);
        } else {
            setup_impl(c, x);
        }
        HIPCHK(hipStreamSynchronize(c->s));
    }
    double t1 = now_ms();
    int its = 0;
    {
        TraceRange r("tmop minres");
        CHK(minres_impl(c, c->sv[SV_G], c->sv[SV_DX], max_minres, rtol, jacobi, check_every, &its));
    }
    double t2 = now_ms();
    TraceRange ls_range("tmop line search");
    rep->minres_its_total += its;
    rep->t_apply_ms += c->acc_apply_ms;
    rep->t_apply_elem_ms += c->acc_elem_ms;
    rep->n_apply += c->acc_napply;
    c->acc_apply_ms = c->acc_elem_ms = 0.0;
    c->acc_napply = 0;
    double alpha = 1.0;
    bool ok = false;
    double Ft = 0.0, gtn = 0.0;
    for (int h = 0; h <= max_halvings; ++h) {
        launch_step(c->ndof, x, c->sv[SV_DX], alpha, c->sv[SV_XT], c->s);
        double md = 0.0, g2 = 0.0;
        const int r = energy_gradient_impl(c, c->sv[SV_XT], &Ft, &md, c->sv[SV_GT], &g2);
        if (r != TMOP_OK && r != TMOP_ERR_INVERTED) return r;
        if (r == TMOP_OK && md > 0.0 && Ft < 1.2 * F) {
            gtn = std::sqrt(g2);
            if (gtn < 1.2 * gn) {
                ok = true;
                break;
            }
        }
        alpha *= 0.5;
        rep->halvings_total++;
    }
    double t3 = now_ms();
    rep->t_setup_ms += t1 - t0;
    rep->t_minres_ms += t2 - t1;
    rep->t_linesearch_ms += t3 - t2;
    if (!ok) return fail(TMOP_ERR_LINESEARCH, "line search found no admissible step");
    HIPCHK(hipMemcpyAsync(x, c->sv[SV_XT], sizeof(double) * c->ndof, hipMemcpyDeviceToDevice, c->s));
    std::swap(c->sv[SV_G], c->sv[SV_GT]);
    F = Ft;
    gn = gtn;
    rep->newton_its++;
    return TMOP_OK;
}

static int solve_start(tmop_ctx *c, double *x, double &F, double &gn, tmop_solve_report *rep)
{
    CHK(ensure_solver(c));
    double xx;
    CHK(dot_host(c, x, x, &xx));
    if (!std::isfinite(xx)) return fail(TMOP_ERR_NONFINITE, "non-finite node coordinates");
    double md, g2;
    const int r = energy_gradient_impl(c, x, &F, &md, c->sv[SV_G], &g2);
    if (r != TMOP_OK) return r;
    if (!(md > 0.0)) return fail(TMOP_ERR_INVERTED, "det A <= 0 at a quadrature point");
    gn = std::sqrt(g2);
    rep->F0 = F;
    return TMOP_OK;
}

extern "C" int tmop_solve(tmop_ctx *c, double *x, const tmop_solve_params *sp,
                          tmop_solve_report *rep)
{
    if (!c || !x || !sp || !rep) return fail(TMOP_ERR_INVALID_ARG, "null argument");
    std::memset(rep, 0, sizeof(*rep));
    c->hist.clear();
    const double t0 = now_ms();
    double F = 0.0, gn = 0.0;
    int r = solve_start(c, x, F, gn, rep);
    if (r != TMOP_OK) {
        rep->status = r;
        return r;
    }
    const double n0 = sp->g0_norm > 0.0 ? sp->g0_norm : gn;
    rep->g0_norm = n0;
    c->hist.push_back(tmop_iter_record{F, gn, 0, 0});
    int status = TMOP_ERR_NOT_CONVERGED;
    for (int it = 0; it <= sp->max_newton; ++it) {
        if (n0 == 0.0 || F == 0.0 || gn <= sp->rel_grad_tol * n0) {
            status = TMOP_OK;
            break;
        }
        if (it == sp->max_newton) break;
        const int its0 = rep->minres_its_total, h0 = rep->halvings_total;
        r = newton_update(c, x, F, gn, sp->max_minres, sp->minres_rtol, sp->max_halvings,
                          sp->jacobi != 0, 8, rep);
        if (r != TMOP_OK) {
            status = r;
            break;
        }
        c->hist.push_back(
            tmop_iter_record{F, gn, rep->minres_its_total - its0, rep->halvings_total - h0});
    }
    rep->F = F;
    rep->g_norm = gn;
    rep->status = status;
    rep->t_total_ms = now_ms() - t0;
    if (status != TMOP_OK && status != TMOP_ERR_NOT_CONVERGED && status != TMOP_ERR_LINESEARCH)
        return status;
    if (status == TMOP_ERR_NOT_CONVERGED) g_err = "max_newton reached";
    return status;
}

extern "C" int tmop_newton_step(tmop_ctx *c, double *x, int n_minres, int jacobi,
                                tmop_solve_report *rep)
{
    if (!c || !x || !rep || n_minres < 0) return fail(TMOP_ERR_INVALID_ARG, "bad argument");
    std::memset(rep, 0, sizeof(*rep));
    const double t0 = now_ms();
    double F = 0.0, gn = 0.0;
    int r = solve_start(c, x, F, gn, rep);
    if (r == TMOP_OK) {
        rep->g0_norm = gn;
        // fixed amount of linear work: rtol 0, no early exit checks
        r = newton_update(c, x, F, gn, n_minres, 0.0, 30, jacobi != 0, 0, rep);
    }
    rep->F = F;
    rep->g_norm = gn;
    rep->status = r;
    rep->t_total_ms = now_ms() - t0;
    return r;
}

// Process-wide table of autotuned tile shapes per kernel class.
namespace {
struct TileKey {
    int dim, p, nq, storage, precision;
    bool operator<(const TileKey &o) const
    {
        return std::tie(dim, p, nq, storage, precision) <
               std::tie(o.dim, o.p, o.nq, o.storage, o.precision);
    }
};
std::mutex g_tile_mu;
std::map<TileKey, int> g_tile;

}  // namespace

namespace tmop {
// tile shape index recorded for a class by an earlier autotuning, or -1
int tuned_tile(int dim, int p, int nq, int storage, int precision)
{
    std::lock_guard<std::mutex> lk(g_tile_mu);
    auto it = g_tile.find(TileKey{dim, p, nq, storage, precision});
    return it == g_tile.end() ? -1 : it->second;
}
void record_tile(int dim, int p, int nq, int storage, int precision, int t)
{
    std::lock_guard<std::mutex> lk(g_tile_mu);
    g_tile[TileKey{dim, p, nq, storage, precision}] = t;
}
}  // namespace tmop

extern "C" int tmop_autotune(tmop_ctx *c, const double *v, double *y, int reps, int *epb)
{
    if (!c || !v || !y || reps <= 0) return fail(TMOP_ERR_INVALID_ARG, "bad argument");
    if (!c->have_setup) return fail(TMOP_ERR_STATE, "tmop_hessian_setup was not called");
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const int keep = c->tile;
    // three rounds over the shapes, each shape's best round counts: a shape
    // timed first is not penalised by clocks or caches still settling
    float tmin[3] = {0.f, 0.f, 0.f};
    for (int round = 0; round < 3; ++round)
        for (int t = 0; t < 3; ++t) {
            if (c->ops.epb_t[t] == 0) continue;
            c->tile = t;
            for (int k = 0; k < 2; ++k) apply_elem(c, v);
            HIPCHK(hipEventRecord(e0, c->s));
            for (int k = 0; k < reps; ++k) apply_elem(c, v);
            HIPCHK(hipEventRecord(e1, c->s));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (round == 0 || ms < tmin[t]) tmin[t] = ms;
        }
    int best = -1;
    for (int t = 0; t < 3; ++t)
        if (c->ops.epb_t[t] != 0 && (best < 0 || tmin[t] < tmin[best])) best = t;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    c->tile = best < 0 ? keep : best;
    record_tile(c->dim, c->p, c->nq, c->storage, c->precision, c->tile);
    // leave y = H v with the chosen shape
    apply_elem(c, v);
    apply_gather(c, v, y);
    if (epb) *epb = c->ops.epb_t[c->tile];
    return TMOP_OK;
}

extern "C" int tmop_set_tile(tmop_ctx *c, int epb)
{
    if (!c) return fail(TMOP_ERR_INVALID_ARG, "null context");
    for (int t = 0; t < 3; ++t)
        if (c->ops.epb_t[t] > 0 && c->ops.epb_t[t] == epb) {
            c->tile = t;
            return TMOP_OK;
        }
    return fail(TMOP_ERR_UNSUPPORTED, "no Hessian-action tile with this many elements per workgroup");
}

extern "C" int tmop_tile_epb(tmop_ctx *c, int *epb)
{
    if (!c || !epb) return fail(TMOP_ERR_INVALID_ARG, "null argument");
    *epb = c->ops.epb_t[c->tile];
    return TMOP_OK;
}

extern "C" int tmop_set_limiting(tmop_ctx *c, const double *x0, double coef, double delta)
{
    if (!c) return fail(TMOP_ERR_INVALID_ARG, "null context");
    c->have_diag = false;
    if (!x0) {
        c->g.x0 = nullptr;
        c->g.lim = 0.0;
        return TMOP_OK;
    }
    if (!(delta > 0.0) || !(coef >= 0.0) || !std::isfinite(coef) || !std::isfinite(delta))
        return fail(TMOP_ERR_INVALID_ARG, "limiting term needs coef >= 0 and delta > 0");
    if (!c->x0buf) {
        const hipError_t e = hipMalloc((void **)&c->x0buf, sizeof(double) * c->ndof);
        if (e != hipSuccess) {
            c->x0buf = nullptr;
            return fail(e == hipErrorOutOfMemory ? TMOP_ERR_OOM : TMOP_ERR_HIP,
                        "limiting term reference nodes");
        }
    }
    HIPCHK(hipMemcpyAsync(c->x0buf, x0, sizeof(double) * c->ndof, hipMemcpyDeviceToDevice, c->s));
    c->g.x0 = c->x0buf;
    c->g.lim = coef * c->tg.detW / (delta * delta);
    return TMOP_OK;
}

extern "C" int tmop_solve_history(tmop_ctx *c, tmop_iter_record *out, int cap, int *n)
{
    if (!c || !n || cap < 0 || (cap > 0 && !out)) return fail(TMOP_ERR_INVALID_ARG, "bad argument");
    const int m = (int)c->hist.size();
    for (int k = 0; k < m && k < cap; ++k) out[k] = c->hist[k];
    *n = m;
    return TMOP_OK;
}

extern "C" int tmop_set_sweeps(tmop_ctx *c, int mode)
{
    if (!c || (mode != TMOP_SWEEPS_PENCIL && mode != TMOP_SWEEPS_MFMA))
        return fail(TMOP_ERR_INVALID_ARG, "bad argument");
    if (mode == TMOP_SWEEPS_MFMA && !c->ops.energyM)
        return fail(TMOP_ERR_UNSUPPORTED, "no matrix-core sweeps for this class");
    c->sweeps = mode;
    return TMOP_OK;
}

extern "C" int tmop_set_timing(tmop_ctx *c, int enable)
{
    if (!c) return fail(TMOP_ERR_INVALID_ARG, "null context");
    c->timing = enable != 0;
    if (c->timing && c->tev.empty()) {
        c->tev.resize(3 * 256);
        for (auto &e : c->tev) HIPCHK(hipEventCreate(&e));
    }
    return TMOP_OK;
}

extern "C" int tmop_set_lanczos_bank_limit(tmop_ctx *c, size_t max_bytes)
{
    if (!c) return fail(TMOP_ERR_INVALID_ARG, "null context");
    c->bank_limit = max_bytes;
    if (c->bank && (size_t)c->bank_cap * c->bank_stride * sizeof(double) > max_bytes) {
        HIPCHK(hipStreamSynchronize(c->s));
        HIPCHK(hipFree(c->bank));
        c->bank = nullptr;
        c->bank_cap = 0;
    }
    return TMOP_OK;
}

// ---------------------------------------------------------------------------
// Energy and min det with no allocation, for callers that cannot allocate
// device memory.  The energy kernel's per-workgroup partials (3 planes of
// grid doubles, each fully written by the kernel before the final reduction
// reads it) live in this file-scope array instead of a context's workspace.
// Each GPU holds its own copy; host code reaches it only through the address
// hipGetSymbolAddress returns on that device.
// ---------------------------------------------------------------------------

static __device__ __align__(256) double scratch[3 * TMOP_NOALLOC_MAX_TILES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
int scratch_on_current_device(double **out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(TMOP_ERR_HIP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(TMOP_ERR_HIP, "no device address for the scratch array");
        g_scratch_dev[dev] = (double *)p;
    }
    *out = g_scratch_dev[dev];
    return TMOP_OK;
}

}  // namespace

extern "C" int tmop_energy_mindet_noalloc(const tmop_mesh_desc *m, const tmop_params *prm,
                                          const double *x, double *out, void *stream)
{
    if (!m || !prm || !x || !out) return fail(TMOP_ERR_INVALID_ARG, "null argument");
    long ne, nx;
    int nqe, np;
    CHK(ctx_sizes(m, prm, ne, nx, nqe, np));
    if (m->elem_to_node)
        return fail(TMOP_ERR_UNSUPPORTED, "the no-allocation energy takes structured boxes only");
    const int d = m->dim, p = m->order_p, nq = prm->nq1d;
    if (!metric_supported(d, prm->metric))
        return fail(TMOP_ERR_UNSUPPORTED, "metric must be 2, 7, 9 or 55 (dim 2) or 303 or 55 (dim 3)");
    Ops ops;
    if (!find_ops(d, p, nq, &ops))
        return fail(TMOP_ERR_UNSUPPORTED, "no kernel for this (dim, p, nq1d); nq1d must be p+1..p+3");
    const long grid = (ne + ops.epb - 1) / ops.epb;
    if (grid > TMOP_NOALLOC_MAX_TILES)
        return fail(TMOP_ERR_INVALID_ARG,
                    "mesh too large for the no-allocation energy: " + std::to_string(grid) +
                        " element tiles of " + std::to_string(ops.epb) + " elements, at most " +
                        std::to_string(TMOP_NOALLOC_MAX_TILES));
    Tables tb;
    Target tg;
    if (internal_tables(p, nq, &tb, prm->quad_rule) != TMOP_OK)
        return fail(TMOP_ERR_INVALID_ARG, "quad_rule must be TMOP_QUAD_GL or TMOP_QUAD_GLL");
    if (internal_target(prm, d, &tg) != TMOP_OK)
        return fail(TMOP_ERR_INVALID_ARG, "target W must have det > 0");
    Geom g{};
    g.dim = d;
    g.p = p;
    g.ne = (int)ne;
    g.nx = (int)nx;
    g.nel[0] = m->nx;
    g.nel[1] = m->ny;
    g.nel[2] = d == 3 ? m->nz : 1;
    for (int k = 0; k < 3; ++k) g.M[k] = g.nel[k] * p + 1;
    if (d == 2) g.M[2] = 1;
    set_divisors(g);
    g.ess_mode = TMOP_ESS_NONE;
    double *part = nullptr;
    CHK(scratch_on_current_device(&part));
    const hipStream_t s = (hipStream_t)stream;
    ops.energy((int)grid, s, g, tb, tg, x, part);
    launch_reduce3(part, (int)grid, out, s);
    HIPCHK(hipGetLastError());
    return TMOP_OK;
}

extern "C" const char *tmop_last_error(void) { return g_err.c_str(); }

extern "C" const char *tmop_version(void) { return "tmop-mi355x 0.1 (gfx950)"; }
