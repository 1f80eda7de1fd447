// Device-side building blocks of the PA-TMOP kernels for gfx950.
//
// One workgroup of BLOCK = 256 lanes (four wave64s) processes EPB elements;
// every stage is a flattened loop over (element, index) pairs with the
// innermost index fastest, so the lanes of a wave touch consecutive LDS
// words and consecutive HBM addresses.  Element data (nodes, sum-factorized
// partial contractions, quadrature values) live in LDS; the quadrature
// tensor streams from HBM once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmop {

constexpr int BLOCK = 256;
constexpr int MAXNI = 9;   // p <= 8
constexpr int MAXNQ = 10;  // up to 10 points per direction
constexpr int LDS_PER_CU = 160 * 1024;  // bytes of LDS per compute unit (gfx950)

// Division by a divisor d >= 1 fixed at set-up, exact for 0 <= n < 2^31:
// floor(n / d) = (n m) >> s with l = ceil(log2 d), m = ceil(2^(31+l) / d),
// s = 31 + l (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994, Thm. 4.2; m < 2^32).  Two multiplies and a shift
// in place of the long sequence of a run-time integer division.
struct FastDiv {
    uint32_t m;
    uint32_t s;
};

inline FastDiv make_fastdiv(int d)
{
    int l = 0;
    while ((1ll << l) < (long long)d) ++l;
    const unsigned long long num = 1ull << (31 + l);
    FastDiv f;
    f.m = (uint32_t)((num + (unsigned long long)d - 1) / (unsigned long long)d);
    f.s = (uint32_t)(31 + l);
    return f;
}

__host__ __device__ __forceinline__ int fdiv(int n, FastDiv f)
{
    return (int)(((uint64_t)(uint32_t)n * f.m) >> f.s);
}

// Mesh geometry passed by value to every kernel.
struct Geom {
    int dim;
    int p;
    int ne;                // number of elements
    int nel[3];            // elements per axis (structured box)
    int M[3];              // grid nodes per axis, nel*p + 1
    int nx;                // global nodes N_x
    const int32_t *e2n;    // general mesh connectivity or nullptr
    int ess_mode;          // 0 box boundary, 1 none, 2 mask
    const uint8_t *ess;    // [dim * nx] for mode 2
    // limiting term (eq. eq_F_full, xi = |x - x0|^2 / delta^2): reference
    // nodes x0 [dim * nx] and lim = coef det W / delta^2; lim = 0 means off
    const double *x0;
    double lim;
    // box meshes: divisions by M[0], M[1], p, nel[0] and nel[1] (set by
    // set_divisors)
    FastDiv dM0, dM1, dP, dE0, dE1;
};

inline void set_divisors(Geom &g)
{
    g.dM0 = make_fastdiv(g.M[0] > 0 ? g.M[0] : 1);
    g.dM1 = make_fastdiv(g.M[1] > 0 ? g.M[1] : 1);
    g.dP = make_fastdiv(g.p > 0 ? g.p : 1);
    g.dE0 = make_fastdiv(g.nel[0] > 0 ? g.nel[0] : 1);
    g.dE1 = make_fastdiv(g.nel[1] > 0 ? g.nel[1] : 1);
}

// Element coordinates (ex, ey[, ez]) of element e of a box mesh.
template <int DIM>
__device__ __forceinline__ void box_elem(const Geom &g, int e, int &ex, int &ey, int &ez)
{
    const int t = fdiv(e, g.dE0);
    ex = e - t * g.nel[0];
    if (DIM == 3) {
        ez = fdiv(t, g.dE1);
        ey = t - ez * g.nel[1];
    } else {
        ey = t;
        ez = 0;
    }
}

// Grid coordinates of global node `node` of a box mesh.
template <int DIM>
__device__ __forceinline__ void box_coords(const Geom &g, int node, int gc[3])
{
    const int t = fdiv(node, g.dM0);
    gc[0] = node - t * g.M[0];
    if (DIM == 3) {
        gc[2] = fdiv(t, g.dM1);
        gc[1] = t - gc[2] * g.M[1];
    } else {
        gc[1] = t;
        gc[2] = 0;
    }
}

// 1D tables: B[q][i] = l_i(chi_q), G[q][i] = l_i'(chi_q), w[q] (Sec. 3.1, eq. eq_B_G_1D).
// Bf, Gf: the same tables rounded to FP32 for the mixed-precision action.
// Kernels take Tables by value, so the entries they index with compile-time
// constants are read from the kernel arguments into scalar registers.
struct Tables {
    double B[MAXNQ * MAXNI];
    double G[MAXNQ * MAXNI];
    double w[MAXNQ];
    float Bf[MAXNQ * MAXNI];
    float Gf[MAXNQ * MAXNI];
};

template <typename CT>
__device__ inline CT tabB(const Tables &t, int k);
template <>
__device__ inline double tabB<double>(const Tables &t, int k) { return t.B[k]; }
template <>
__device__ inline float tabB<float>(const Tables &t, int k) { return t.Bf[k]; }
// 1D weight w[i] for a run-time i, selected with compile-time indices only:
// indexing the by-value Tables argument with a run-time index would make the
// compiler copy the whole structure to scratch memory.
template <int NQ>
__device__ __forceinline__ double tab_w(const Tables &t, int i)
{
    double w = 0.0;
#pragma unroll
    for (int k = 0; k < NQ; ++k)
        if (i == k) w = t.w[k];
    return w;
}

template <typename CT>
__device__ inline CT tabG(const Tables &t, int k);
template <>
__device__ inline double tabG<double>(const Tables &t, int k) { return t.G[k]; }
template <>
__device__ inline float tabG<float>(const Tables &t, int k) { return t.Gf[k]; }

// Constant target: W^{-1} (row-major) and det W; ideal != 0 means W = I.
struct Target {
    double Winv[9];
    double detW;
    int ideal;
    int metric;
};

// Batched launches: one tile = up to EPB consecutive elements of one slot
// (mesh); a slot carries its geometry, target and device pointers to its DoF
// vectors (by vector id), quadrature data and E-vector scratch.
struct Tile {
    int slot;
    int e0;
};

constexpr int NVEC = 16;

struct SlotDev {
    Geom g;
    Target tg;
    double *vec[NVEC];
    void *H;
    void *eV;
    // resident MINRES Lanczos vectors (bank vector m at bank + m * bstride)
    // and the scalars of each update (8 doubles per update); null when the
    // slot takes the three-term update
    double *bank;
    double *hist;
    long bstride;
};

// Symmetric packing of a d^2 x d^2 tensor: entry (r, s), r <= s, row-major
// upper triangle.
template <int D2>
__host__ __device__ constexpr int sym_index(int r, int s)
{
    return r <= s ? r * D2 - (r * (r - 1)) / 2 + (s - r) : s * D2 - (s * (s - 1)) / 2 + (r - s);
}

// ------------------------------------------------------------------------
// Fixed-DoF predicate
// ------------------------------------------------------------------------

__device__ inline bool box_boundary(const Geom &g, int gx, int gy, int gz)
{
    bool b = gx == 0 || gx == g.M[0] - 1 || gy == 0 || gy == g.M[1] - 1;
    if (g.dim == 3) b = b || gz == 0 || gz == g.M[2] - 1;
    return b;
}

// Is component c of global node `node` (grid coordinates gx,gy,gz when the
// mesh is a box) fixed?
__device__ inline bool is_fixed(const Geom &g, int c, int node, int gx, int gy, int gz)
{
    if (g.ess_mode == 1) return false;
    if (g.ess_mode == 2) return g.ess[(size_t)c * g.nx + node] != 0;
    return box_boundary(g, gx, gy, gz);
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup i runs on
// XCD i % 8), each with its own L2.  Renumbering them so that every XCD works
// on one contiguous range of logical blocks keeps neighbouring elements, which
// share nodes, in one L2.  A bijection of [0, n).
__device__ __forceinline__ int xcd_block(int i, int n)
{
    constexpr int NXCD = 8;
    const int q = n / NXCD, r = n % NXCD;
    const int x = i % NXCD, k = i / NXCD;
    return x * q + (x < r ? x : r) + k;
}

// ------------------------------------------------------------------------
// Block reductions (deterministic order)
// ------------------------------------------------------------------------

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double wave_min(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

// Sum over the workgroup; result valid in thread 0.
__device__ inline double block_sum(double v, double *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < BLOCK / 64; ++k) s += red[k];
    return s;
}

__device__ inline double block_min(double v, double *red)
{
    v = wave_min(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
    if (threadIdx.x == 0)
        for (int k = 1; k < BLOCK / 64; ++k) s = fmin(s, red[k]);
    return s;
}

// The energy partials of a workgroup: sum of s, min of m, sum of b, with the
// shuffles and the order of block_sum / block_min but one exchange through
// LDS (red holds 3 BLOCK/64 doubles).  Results valid in thread 0.
__device__ inline void block_energy3(double &s, double &m, double &b, double *red)
{
    constexpr int NW = BLOCK / 64;
    s = wave_sum(s);
    m = wave_min(m);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        red[w] = s;
        red[NW + w] = m;
        red[2 * NW + w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, c = red[NW], e = 0.0;
        for (int k = 0; k < NW; ++k) a += red[k];
        for (int k = 1; k < NW; ++k) c = fmin(c, red[NW + k]);
        for (int k = 0; k < NW; ++k) e += red[2 * NW + k];
        s = a;
        m = c;
        b = e;
    }
}

// ------------------------------------------------------------------------
// Quality metrics at one point (T = A W^{-1}); closed-form derivatives of
// mu_2 = |T|^2/(2 tau) - 1 and mu_303 = |T|^2/(3 tau^{2/3}) - 1.
//
// With I1 = |T|^2, tau = det T and C = cof T = d tau / dT:
//   dmu   = cT T + cC C
//   d2mu  = c_id Id + c_tc (T (x) C + C (x) T) + c_cc C (x) C + c_dc dC/dT
// ------------------------------------------------------------------------

// Quadrature data of one element: ns values per point, stored for nqt
// points rounded up to qdata_pts(nqt, tbytes) so that every plane of one
// value per point (tbytes each) and every run of 16 bytes per point starts
// on a 128-byte cache line (element blocks included).  Without the padding
// a line that straddles two runs was fetched from HBM once for each run the
// streaming loads read it for.  No lane reads or writes the padding.
inline __host__ __device__ constexpr int qdata_pts(int nqt, int tbytes)
{
    return (nqt + 128 / tbytes - 1) / (128 / tbytes) * (128 / tbytes);
}

inline __host__ __device__ constexpr long qdata_stride(int ns, int nqt, int tbytes)
{
    return (long)ns * qdata_pts(nqt, tbytes);
}

// Metrics with kernels: 2, 7, 9, 55 in 2D; 303, 55 in 3D.
inline __host__ __device__ bool metric_supported(int dim, int metric)
{
    if (dim == 2) return metric == 2 || metric == 7 || metric == 9 || metric == 55;
    return dim == 3 && (metric == 303 || metric == 55);
}

struct MetricCoef {
    double mu, cT, cC, c_id, c_tc, c_cc, c_dc;
};

// Quality metrics of Sec. 2.2 / 4.1, each a function f(I1, tau) of I1 = |T|^2 and
// tau = det T that is linear in I1, so that
//   dmu/dT   = cT T + cC C                       (cT = 2 f_1, cC = f_tau)
//   d2mu/dT2 = c_id Id + c_tc (T x C + C x T) + c_cc C x C + c_dc dC/dT
// with c_id = 2 f_1, c_tc = 2 f_1tau, c_cc = f_tautau, c_dc = f_tau.
//   2   mu_2   = I1 / (2 tau) - 1                 (2D shape)
//   303 mu_303 = I1 / (3 tau^{2/3}) - 1           (3D shape)
//   55  mu_55  = (tau - 1)^2                      (size, 2D and 3D)
//   7   mu_7   = |T - T^{-t}|^2 = I1 (1 + tau^-2) - 4          (2D shape+size)
//   9   mu_9   = tau |T - T^{-t}|^2 = I1 (tau + 1/tau) - 4 tau (2D shape+size)
// (the 2D forms of mu_7, mu_9 use |C| = |T| and T : C = 2 tau; metric_value
// evaluates them from their definition instead, which is exact at T = I).
// The metric code below fuses multiply-adds per source expression only
// (fp contract(on)), not wherever the code generator finds them after
// inlining, so every kernel that evaluates a metric at a point rounds the
// same way (the one-pass kernels give bitwise the results of the separate
// ones).
__device__ inline MetricCoef metric_coef(int metric, double I1, double tau)
{
#pragma clang fp contract(on)
    MetricCoef m;
    if (metric == 2) {
        const double it = 1.0 / tau;
        m.mu = 0.5 * I1 * it - 1.0;
        m.cT = it;
        m.cC = -0.5 * I1 * it * it;
        m.c_id = it;
        m.c_tc = -it * it;
        m.c_cc = I1 * it * it * it;
        m.c_dc = -0.5 * I1 * it * it;
    } else if (metric == 303) {
        const double r = 1.0 / cbrt(tau);  // tau^{-1/3}
        const double r2 = r * r;           // tau^{-2/3}
        const double r5 = r2 * r2 * r;     // tau^{-5/3}
        const double r8 = r5 * r2 * r;     // tau^{-8/3}
        m.mu = I1 * r2 / 3.0 - 1.0;
        m.cT = 2.0 * r2 / 3.0;
        m.cC = -2.0 * I1 * r5 / 9.0;
        m.c_id = 2.0 * r2 / 3.0;
        m.c_tc = -4.0 * r5 / 9.0;
        m.c_cc = 10.0 * I1 * r8 / 27.0;
        m.c_dc = -2.0 * I1 * r5 / 9.0;
    } else if (metric == 55) {
        const double dm = tau - 1.0;
        m.mu = dm * dm;
        m.cT = 0.0;
        m.cC = 2.0 * dm;
        m.c_id = 0.0;
        m.c_tc = 0.0;
        m.c_cc = 2.0;
        m.c_dc = 2.0 * dm;
    } else if (metric == 7) {
        const double it = 1.0 / tau, it2 = it * it, it3 = it2 * it;
        m.mu = I1 * (1.0 + it2) - 4.0;
        m.cT = 2.0 * (1.0 + it2);
        m.cC = -2.0 * I1 * it3;
        m.c_id = m.cT;
        m.c_tc = -4.0 * it3;
        m.c_cc = 6.0 * I1 * it2 * it2;
        m.c_dc = m.cC;
    } else {  // 9
        const double it = 1.0 / tau, it2 = it * it;
        m.mu = I1 * (tau + it) - 4.0 * tau;
        m.cT = 2.0 * (tau + it);
        m.cC = I1 * (1.0 - it2) - 4.0;
        m.c_id = m.cT;
        m.c_tc = 2.0 * (1.0 - it2);
        m.c_cc = 2.0 * I1 * it2 * it;
        m.c_dc = m.cC;
    }
    return m;
}

// mu at T (C = cof T, tau = det T > 0) for the energy: mu_7 and mu_9 from their
// definition |T - C / tau|^2 (no cancellation near T = I), the others from
// metric_coef.
template <int D>
__device__ inline double metric_value(int metric, const double *T, const double *C, double I1,
                                      double tau, const MetricCoef &m)
{
#pragma clang fp contract(on)
    if (metric != 7 && metric != 9) return m.mu;
    const double it = 1.0 / tau;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < D * D; ++k) {
        const double e = T[k] - C[k] * it;
        s += e * e;
    }
    return metric == 7 ? s : tau * s;
}

template <int D>
__device__ inline void apply_winv(const Target &t, const double *A, double *T)
{
#pragma clang fp contract(on)
    if (t.ideal) {
#pragma unroll
        for (int k = 0; k < D * D; ++k) T[k] = A[k];
        return;
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double s = 0.0;
#pragma unroll
            for (int n = 0; n < D; ++n) s += A[a * D + n] * t.Winv[n * D + k];
            T[a * D + k] = s;
        }
}

template <int D>
__device__ inline double det_cof(const double *T, double *C)
{
#pragma clang fp contract(on)
    if constexpr (D == 2) {
        C[0] = T[3];
        C[1] = -T[2];
        C[2] = -T[1];
        C[3] = T[0];
        return T[0] * T[3] - T[1] * T[2];
    } else {
        C[0] = T[4] * T[8] - T[5] * T[7];
        C[1] = T[5] * T[6] - T[3] * T[8];
        C[2] = T[3] * T[7] - T[4] * T[6];
        C[3] = T[2] * T[7] - T[1] * T[8];
        C[4] = T[0] * T[8] - T[2] * T[6];
        C[5] = T[1] * T[6] - T[0] * T[7];
        C[6] = T[1] * T[5] - T[2] * T[4];
        C[7] = T[2] * T[3] - T[0] * T[5];
        C[8] = T[0] * T[4] - T[1] * T[3];
        return T[0] * C[0] + T[1] * C[1] + T[2] * C[2];
    }
}

template <int D>
__device__ inline double det_only(const double *A)
{
#pragma clang fp contract(on)
    if constexpr (D == 2) return A[0] * A[3] - A[1] * A[2];
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// dC_{(ij)} / dT_{(kl)}.  3D: eps_ikm eps_jln T_mn, i.e. nonzero only for
// i != k and j != l, with m, n the remaining indices.  2D: constant.
template <int D>
__device__ inline double dcof(const double *T, int r, int s)
{
#pragma clang fp contract(on)
    const int i = r / D, j = r % D, k = s / D, l = s % D;
    if constexpr (D == 2) {
        if (i != k && j != l) return (i == j) ? 1.0 : -1.0;
        return 0.0;
    } else {
        if (i == k || j == l) return 0.0;
        const int m = 3 - i - k, n = 3 - j - l;
        const double sik = (k == (i + 1) % 3) ? 1.0 : -1.0;
        const double sjl = (l == (j + 1) % 3) ? 1.0 : -1.0;
        return sik * sjl * T[m * 3 + n];
    }
}

// mu and z * P with P = dmu/dT W^{-T}.  Returns false if tau <= 0.
template <int D>
__device__ inline bool metric_first(const Target &t, const double *A, double z, double *mu,
                                    double *P)
{
#pragma clang fp contract(on)
    double T[D * D], C[D * D];
    apply_winv<D>(t, A, T);
    const double tau = det_cof<D>(T, C);
    if (!(tau > 0.0)) return false;
    double I1 = 0.0;
#pragma unroll
    for (int k = 0; k < D * D; ++k) I1 += T[k] * T[k];
    const MetricCoef m = metric_coef(t.metric, I1, tau);
    *mu = metric_value<D>(t.metric, T, C, I1, tau, m);
    double dmu[D * D];
#pragma unroll
    for (int k = 0; k < D * D; ++k) dmu[k] = m.cT * T[k] + m.cC * C[k];
    if (t.ideal) {
#pragma unroll
        for (int k = 0; k < D * D; ++k) P[k] = z * dmu[k];
    } else {
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int n = 0; n < D; ++n) {
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k) s += dmu[a * D + k] * t.Winv[n * D + k];
                P[a * D + n] = z * s;
            }
    }
    return true;
}

// z * H_A, packed symmetric (D^2 (D^2+1)/2 entries), where
// H_A[an][bp] = sum_kl d2mu[ak][bl] Winv_nk Winv_pl.  Returns false if tau <= 0.
template <int D>
__device__ inline bool metric_second(const Target &t, const double *A, double z, double *Hp)
{
#pragma clang fp contract(on)
    constexpr int D2 = D * D;
    double T[D2], C[D2];
    apply_winv<D>(t, A, T);
    const double tau = det_cof<D>(T, C);
    if (!(tau > 0.0)) return false;
    double I1 = 0.0;
#pragma unroll
    for (int k = 0; k < D2; ++k) I1 += T[k] * T[k];
    const MetricCoef m = metric_coef(t.metric, I1, tau);
    if (t.ideal) {
#pragma unroll
        for (int r = 0; r < D2; ++r)
#pragma unroll
            for (int s = r; s < D2; ++s) {
                double v = m.c_tc * (T[r] * C[s] + C[r] * T[s]) + m.c_cc * C[r] * C[s] +
                           m.c_dc * dcof<D>(T, r, s);
                if (r == s) v += m.c_id;
                Hp[sym_index<D2>(r, s)] = z * v;
            }
        return true;
    }
    // general constant W: each entry H_A[an][bp] = sum_kl d2mu[ak][bl] Winv_nk Winv_pl,
    // with d2mu evaluated entry by entry (keeps register use low).  The loops
    // index at run time, so they work on copies (Tg, Cg, Hg): the arrays of
    // the ideal-target path above then stay in registers.
    {
        constexpr int NS = D2 * (D2 + 1) / 2;
        double Tg[D2], Cg[D2], Hg[NS];
#pragma unroll
        for (int k = 0; k < D2; ++k) {
            Tg[k] = T[k];
            Cg[k] = C[k];
        }
        for (int r = 0; r < D2; ++r)
            for (int s = r; s < D2; ++s) {
                const int a = r / D, n = r % D, b = s / D, p = s % D;
                double acc = 0.0;
                for (int k = 0; k < D; ++k)
                    for (int l = 0; l < D; ++l) {
                        const int rr = a * D + k, ss = b * D + l;
                        double v = m.c_tc * (Tg[rr] * Cg[ss] + Cg[rr] * Tg[ss]) +
                                   m.c_cc * Cg[rr] * Cg[ss] + m.c_dc * dcof<D>(Tg, rr, ss);
                        if (rr == ss) v += m.c_id;
                        acc += v * t.Winv[n * D + k] * t.Winv[p * D + l];
                    }
                Hg[sym_index<D2>(r, s)] = z * acc;
            }
#pragma unroll
        for (int k = 0; k < NS; ++k) Hp[k] = Hg[k];
    }
    return true;
}

}  // namespace tmop
