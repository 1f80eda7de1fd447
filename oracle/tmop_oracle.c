/*
 * Plain FP64 CPU oracle for the partially assembled TMOP operators.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so and is
 * called by the test-suite, by the smoke check and by the CPU-baseline leg of
 * the benchmark.  The product library never links, loads or calls it, and the
 * two share no source, header, table or helper.
 *
 * Everything here is the direct (not sum-factorized) form of the paper's
 * definitions, element by element and quadrature point by quadrature point:
 *
 *   - Jacobian A_ab = sum_i x_{a,i} d w_i / d xbar_b               (Sec. 2.2, eq. eq_A;
 *                                                                    Sec. 3.2, first display)
 *   - T = A W^{-1}, tau = det T                                     (Sec. 2.2, eq. eq_T)
 *   - mu_2 = |T|^2/(2 tau) - 1 (2D), mu_303 = |T|^2/(3 tau^{2/3}) - 1 (3D)
 *                                                                   (Sec. 2.2 metric list;
 *                                                                    Sec. 4.1, Kershaw setup)
 *   - F = sum_E sum_q w_q det(W) mu(T)                              (Sec. 2.2 eq. eq_F_full,
 *                                                                    Sec. 3.3 eq. D0_expression)
 *   - dF/dx_{a,i} = sum_q z_q sum_n P_an dw_i/dxbar_n               (Sec. 3.3 eq. eq_vm_pa_grad)
 *   - d2F/dx_{b,j}dx_{a,i} = sum_q z_q sum H_A[an,bp] dw_j/dxbar_p dw_i/dxbar_n
 *                                                                   (Sec. 3.4 eq. eq_vm_pa_hess)
 *   - the Hessian diagonal used by the Jacobi preconditioner         (Sec. 3.4, last paragraph)
 *
 * The paper writes the derivatives for W = I.  For a constant W the chain
 * rule through T = A W^{-1} gives P = (dmu/dT) W^{-T} and
 * H_A[an,bp] = sum_{k,l} d2mu/dT_ak dT_bl Winv_nk Winv_pl; the weight is
 * z_q = w_q det W (spatial weight omega = 1).
 *
 * Metric derivatives are the closed forms obtained with standard matrix
 * calculus (Sec. 3.2, second bullet):  with I1 = |T|^2, C = cof(T) = dtau/dT,
 *   mu_2  : dmu = T/tau - I1/(2 tau^2) C
 *           d2mu = Id/tau - (T(x)C + C(x)T)/tau^2 + I1/tau^3 C(x)C - I1/(2 tau^2) dC/dT
 *   mu_303: dmu = 2/(3 tau^{2/3}) T - 2 I1/(9 tau^{5/3}) C
 *           d2mu = 2/(3 tau^{2/3}) Id - 4/(9 tau^{5/3}) (T(x)C + C(x)T)
 *                  + 10 I1/(27 tau^{8/3}) C(x)C - 2 I1/(9 tau^{5/3}) dC/dT
 * where dC_ij/dT_kl = eps_ikm eps_jln T_mn in 3D and the constant
 * permutation pattern in 2D.
 *
 * Parallelism: OpenMP over elements into an element vector (E-vector), then a
 * serial scatter-add in element order, so results do not depend on the
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int dim;            /* 2 or 3 */
    int metric;         /* 2 (mu_2, 2D) or 303 (mu_303, 3D) */
    int ne;             /* number of elements */
    int np;             /* nodes per element, (p+1)^dim */
    int nq;             /* quadrature points per element, nq1d^dim */
    int nx;             /* global nodes N_x; vectors are dim*N_x, SoA x[c*nx+i] */
    const int32_t *e2n; /* ne*np global node index of local node i of element e */
    const double *wq;   /* nq quadrature weights (products of 1D weights) */
    const double *dphi; /* dim*nq*np: d wbar_i/d xbar_b at chi_q, index [b][q][i] */
    double Winv[9];     /* constant target inverse W^{-1}, row-major dim x dim */
    double detW;        /* det W */
    /* Limiting term of eq. eq_F_full, xi(y, delta) = |y|^2 / delta^2 with
     * y = x - x0 at the point, weighted by lim_coef; off when x0 is NULL. */
    const double *phi;  /* nq*np: wbar_i(chi_q), index [q][i] */
    const double *x0;   /* dim*nx reference node positions, or NULL */
    double lim_coef;    /* weight of the limiting integral */
    double lim_delta;   /* limiting distance delta (> 0) */
} oracle_problem;

/* ------------------------------------------------------------------------ */
/* Small dense helpers                                                      */
/* ------------------------------------------------------------------------ */

static double det_mat(int d, const double *M)
{
    if (d == 2) return M[0] * M[3] - M[1] * M[2];
    return M[0] * (M[4] * M[8] - M[5] * M[7])
         - M[1] * (M[3] * M[8] - M[5] * M[6])
         + M[2] * (M[3] * M[7] - M[4] * M[6]);
}

/* Levi-Civita symbol for indices in {0,1,2}. */
static int levi(int i, int j, int k)
{
    if (i == j || j == k || i == k) return 0;
    /* even permutations of (0,1,2) */
    if ((i == 0 && j == 1 && k == 2) || (i == 1 && j == 2 && k == 0) ||
        (i == 2 && j == 0 && k == 1))
        return 1;
    return -1;
}

/* Cofactor matrix C = d(det T)/dT (equals det(T) T^{-T} for invertible T). */
static void cofactor(int d, const double *T, double *C)
{
    if (d == 2) {
        C[0] = T[3];
        C[1] = -T[2];
        C[2] = -T[1];
        C[3] = T[0];
        return;
    }
    /* C_ij = 1/2 eps_ikm eps_jln T_kl T_mn */
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++)
                for (int m = 0; m < 3; m++) {
                    int eikm = levi(i, k, m);
                    if (!eikm) continue;
                    for (int l = 0; l < 3; l++)
                        for (int n = 0; n < 3; n++) {
                            int ejln = levi(j, l, n);
                            if (!ejln) continue;
                            s += 0.5 * eikm * ejln * T[k * 3 + l] * T[m * 3 + n];
                        }
                }
            C[i * 3 + j] = s;
        }
}

/* dC_ij/dT_kl, stored [i][j][k][l]. */
static void dcofactor(int d, const double *T, double *dC)
{
    int d2 = d * d;
    memset(dC, 0, sizeof(double) * d2 * d2);
    if (d == 2) {
        /* C = [[T11, -T10], [-T01, T00]] */
        dC[(0 * 2 + 0) * 4 + (1 * 2 + 1)] = 1.0;
        dC[(0 * 2 + 1) * 4 + (1 * 2 + 0)] = -1.0;
        dC[(1 * 2 + 0) * 4 + (0 * 2 + 1)] = -1.0;
        dC[(1 * 2 + 1) * 4 + (0 * 2 + 0)] = 1.0;
        return;
    }
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            for (int k = 0; k < 3; k++)
                for (int l = 0; l < 3; l++) {
                    double s = 0.0;
                    for (int m = 0; m < 3; m++)
                        for (int n = 0; n < 3; n++)
                            s += levi(i, k, m) * levi(j, l, n) * T[m * 3 + n];
                    dC[((i * 3 + j) * 3 + k) * 3 + l] = s;
                }
}

/* ------------------------------------------------------------------------ */
/* Quality metrics and their derivatives                                     */
/* ------------------------------------------------------------------------ */

/*
 * Evaluate mu(T) and, if requested, dmu/dT (dim*dim, row-major) and
 * d2mu/dT_ij dT_kl (dim^4, index [i][j][k][l]).  Returns 0 and leaves the
 * outputs untouched when det T <= 0 (the metrics are undefined there).
 * Returns -1 for an unknown metric/dimension pair.
 */
int oracle_metric(int dim, int metric, const double *T, double *mu, double *dmu,
                  double *d2mu)
{
    int d = dim, d2 = dim * dim;
    int known = (dim == 2 && (metric == 2 || metric == 7 || metric == 9 || metric == 55)) ||
                (dim == 3 && (metric == 303 || metric == 55));
    if (!known) return -1;
    double tau = det_mat(d, T);
    if (!(tau > 0.0)) return 0;
    double I1 = 0.0;
    for (int k = 0; k < d2; k++) I1 += T[k] * T[k];
    double C[9];
    cofactor(d, T, C);

    /* Every metric here is f(I1, tau), linear in I1, so that
     *   dmu    = 2 f_1 T + f_tau C,
     *   d2mu   = 2 f_1 Id + 2 f_1tau (T x C + C x T) + f_tautau C x C + f_tau dC/dT
     * (no T x T term since f_11 = 0). */
    double c_id, c_tc, c_cc, c_dc; /* coefficients of Id, (TxC+CxT), CxC, dC/dT */
    double c_T, c_C;               /* coefficients of T and C in dmu */
    if (metric == 2) {
        *mu = I1 / (2.0 * tau) - 1.0;
        c_T = 1.0 / tau;
        c_C = -I1 / (2.0 * tau * tau);
        c_id = 1.0 / tau;
        c_tc = -1.0 / (tau * tau);
        c_cc = I1 / (tau * tau * tau);
        c_dc = -I1 / (2.0 * tau * tau);
    } else if (metric == 303) {
        double t13 = cbrt(tau);     /* tau^{1/3} */
        double t23 = t13 * t13;     /* tau^{2/3} */
        double t53 = tau * t23;     /* tau^{5/3} */
        double t83 = tau * t53;     /* tau^{8/3} */
        *mu = I1 / (3.0 * t23) - 1.0;
        c_T = 2.0 / (3.0 * t23);
        c_C = -2.0 * I1 / (9.0 * t53);
        c_id = 2.0 / (3.0 * t23);
        c_tc = -4.0 / (9.0 * t53);
        c_cc = 10.0 * I1 / (27.0 * t83);
        c_dc = -2.0 * I1 / (9.0 * t53);
    } else if (metric == 55) {
        /* mu_55 = (tau - 1)^2: f_1 = 0, f_tau = 2 (tau - 1), f_tautau = 2 */
        *mu = (tau - 1.0) * (tau - 1.0);
        c_T = 0.0;
        c_C = 2.0 * (tau - 1.0);
        c_id = 0.0;
        c_tc = 0.0;
        c_cc = 2.0;
        c_dc = 2.0 * (tau - 1.0);
    } else {
        /* mu_7 = |T - T^{-t}|^2 and mu_9 = tau |T - T^{-t}|^2 (2D), evaluated from
         * the definition with T^{-t} = C / tau.  In 2D |C| = |T| and T : C = 2 tau,
         * so mu_7 = I1 (1 + tau^-2) - 4 and mu_9 = I1 (tau + 1/tau) - 4 tau give the
         * derivative coefficients. */
        double m7 = 0.0;
        for (int k = 0; k < d2; k++) {
            double e = T[k] - C[k] / tau;
            m7 += e * e;
        }
        double it = 1.0 / tau, it2 = it * it, it3 = it2 * it;
        if (metric == 7) {
            *mu = m7;
            c_T = 2.0 * (1.0 + it2);       /* 2 f_1 */
            c_C = -2.0 * I1 * it3;         /* f_tau */
            c_id = 2.0 * (1.0 + it2);
            c_tc = -4.0 * it3;             /* 2 f_1tau */
            c_cc = 6.0 * I1 * it2 * it2;   /* f_tautau */
            c_dc = -2.0 * I1 * it3;
        } else {
            *mu = tau * m7;
            c_T = 2.0 * (tau + it);
            c_C = I1 * (1.0 - it2) - 4.0;
            c_id = 2.0 * (tau + it);
            c_tc = 2.0 * (1.0 - it2);
            c_cc = 2.0 * I1 * it3;
            c_dc = I1 * (1.0 - it2) - 4.0;
        }
    }
    if (dmu)
        for (int k = 0; k < d2; k++) dmu[k] = c_T * T[k] + c_C * C[k];
    if (d2mu) {
        double dC[81];
        dcofactor(d, T, dC);
        for (int r = 0; r < d2; r++)
            for (int s = 0; s < d2; s++) {
                double v = (r == s ? c_id : 0.0)
                         + c_tc * (T[r] * C[s] + C[r] * T[s])
                         + c_cc * C[r] * C[s]
                         + c_dc * dC[r * d2 + s];
                d2mu[r * d2 + s] = v;
            }
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Quadrature-point kinematics                                               */
/* ------------------------------------------------------------------------ */

/* A_ab(q) = sum_i xE[a][i] dphi[b][q][i]  (direct O(Np) sum per entry). */
static void jacobian_at(const oracle_problem *pb, const double *xE, int q, double *A)
{
    int d = pb->dim, np = pb->np, nq = pb->nq;
    for (int a = 0; a < d; a++)
        for (int b = 0; b < d; b++) {
            const double *dp = pb->dphi + ((size_t)b * nq + q) * np;
            double s = 0.0;
            for (int i = 0; i < np; i++) s += xE[a * np + i] * dp[i];
            A[a * d + b] = s;
        }
}

static void gather_elem(const oracle_problem *pb, const double *x, int e, double *xE)
{
    int d = pb->dim, np = pb->np;
    const int32_t *map = pb->e2n + (size_t)e * np;
    for (int a = 0; a < d; a++)
        for (int i = 0; i < np; i++) xE[a * np + i] = x[(size_t)a * pb->nx + map[i]];
}

/* u_a = sum_i uE[a][i] wbar_i(chi_q): the FE function of element values uE at q. */
static void value_at(const oracle_problem *pb, const double *uE, int q, double *u)
{
    int d = pb->dim, np = pb->np;
    const double *ph = pb->phi + (size_t)q * np;
    for (int a = 0; a < d; a++) {
        double s = 0.0;
        for (int i = 0; i < np; i++) s += uE[a * np + i] * ph[i];
        u[a] = s;
    }
}

/* lim_coef / delta^2: the limiting integrand is this times |x - x0|^2; its
 * gradient with respect to x(q) is twice this times (x - x0), and its second
 * derivative twice this times the identity. */
static double lim_scale(const oracle_problem *pb)
{
    return pb->x0 ? pb->lim_coef / (pb->lim_delta * pb->lim_delta) : 0.0;
}

static void t_from_a(const oracle_problem *pb, const double *A, double *T)
{
    int d = pb->dim;
    for (int a = 0; a < d; a++)
        for (int k = 0; k < d; k++) {
            double s = 0.0;
            for (int n = 0; n < d; n++) s += A[a * d + n] * pb->Winv[n * d + k];
            T[a * d + k] = s;
        }
}

/* Serial scatter-add of an E-vector (ne x dim x np) into a global vector. */
static void scatter_add(const oracle_problem *pb, const double *ev, double *out)
{
    int d = pb->dim, np = pb->np;
    memset(out, 0, sizeof(double) * (size_t)d * pb->nx);
    for (int e = 0; e < pb->ne; e++) {
        const int32_t *map = pb->e2n + (size_t)e * np;
        const double *ee = ev + (size_t)e * d * np;
        for (int a = 0; a < d; a++)
            for (int i = 0; i < np; i++) out[(size_t)a * pb->nx + map[i]] += ee[a * np + i];
    }
}

/* ------------------------------------------------------------------------ */
/* Public oracle entry points                                                */
/* ------------------------------------------------------------------------ */

/* All Jacobians A (ne x nq x dim x dim). */
void oracle_jacobians(const oracle_problem *pb, const double *x, double *A_out)
{
    int d = pb->dim, d2 = d * d;
#pragma omp parallel for schedule(static)
    for (int e = 0; e < pb->ne; e++) {
        double xE[3 * 729];
        gather_elem(pb, x, e, xE);
        for (int q = 0; q < pb->nq; q++)
            jacobian_at(pb, xE, q, A_out + ((size_t)e * pb->nq + q) * d2);
    }
}

/* min over all quadrature points of det A (Sec. 2.3 line-search condition). */
double oracle_min_det(const oracle_problem *pb, const double *x)
{
    double m = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : m)
    for (int e = 0; e < pb->ne; e++) {
        double xE[3 * 729], A[9];
        gather_elem(pb, x, e, xE);
        for (int q = 0; q < pb->nq; q++) {
            jacobian_at(pb, xE, q, A);
            double dA = det_mat(pb->dim, A);
            if (dA < m) m = dA;
        }
    }
    return m;
}

/* Per-element energies (ne).  Sets *inverted = 1 if det T <= 0 anywhere. */
static void elem_energies(const oracle_problem *pb, const double *x, double *eE, int *inverted)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int e = 0; e < pb->ne; e++) {
        double xE[3 * 729], x0E[3 * 729], A[9], T[9], mu, u[3], u0[3];
        double ls = lim_scale(pb);
        gather_elem(pb, x, e, xE);
        if (ls != 0.0) gather_elem(pb, pb->x0, e, x0E);
        double s = 0.0;
        for (int q = 0; q < pb->nq; q++) {
            jacobian_at(pb, xE, q, A);
            t_from_a(pb, A, T);
            if (oracle_metric(pb->dim, pb->metric, T, &mu, NULL, NULL) != 1) {
                bad = 1;
                continue;
            }
            s += pb->wq[q] * pb->detW * mu;
            if (ls != 0.0) {
                value_at(pb, xE, q, u);
                value_at(pb, x0E, q, u0);
                double y2 = 0.0;
                for (int a = 0; a < pb->dim; a++) y2 += (u[a] - u0[a]) * (u[a] - u0[a]);
                s += pb->wq[q] * pb->detW * ls * y2;
            }
        }
        eE[e] = s;
    }
    *inverted = bad;
}

/* F(x) = sum_E sum_q w_q det W mu(T).  Returns +inf if any det T <= 0. */
double oracle_energy(const oracle_problem *pb, const double *x, int *inverted)
{
    double *eE = (double *)malloc(sizeof(double) * (size_t)pb->ne);
    int bad = 0;
    elem_energies(pb, x, eE, &bad);
    double F = 0.0;
    for (int e = 0; e < pb->ne; e++) F += eE[e];
    free(eE);
    if (inverted) *inverted = bad;
    return bad ? INFINITY : F;
}

/* Gradient dF/dx (dim*nx).  Returns 0 if det T <= 0 anywhere, else 1. */
int oracle_gradient(const oracle_problem *pb, const double *x, double *g)
{
    int d = pb->dim, d2 = d * d, np = pb->np, nq = pb->nq;
    double *ev = (double *)calloc((size_t)pb->ne * d * np, sizeof(double));
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int e = 0; e < pb->ne; e++) {
        double xE[3 * 729], x0E[3 * 729], A[9], T[9], mu, dmu[9], PA[9], u[3], u0[3];
        double *ee = ev + (size_t)e * d * np;
        double ls = lim_scale(pb);
        gather_elem(pb, x, e, xE);
        if (ls != 0.0) gather_elem(pb, pb->x0, e, x0E);
        for (int q = 0; q < nq; q++) {
            jacobian_at(pb, xE, q, A);
            t_from_a(pb, A, T);
            if (oracle_metric(d, pb->metric, T, &mu, dmu, NULL) != 1) {
                bad = 1;
                continue;
            }
            /* P_an = sum_k dmu_ak Winv_nk  (P = dmu/dT W^{-T}) */
            for (int a = 0; a < d; a++)
                for (int n = 0; n < d; n++) {
                    double s = 0.0;
                    for (int k = 0; k < d; k++) s += dmu[a * d + k] * pb->Winv[n * d + k];
                    PA[a * d + n] = s;
                }
            double z = pb->wq[q] * pb->detW;
            for (int a = 0; a < d; a++)
                for (int i = 0; i < np; i++) {
                    double s = 0.0;
                    for (int n = 0; n < d; n++)
                        s += PA[a * d + n] * pb->dphi[((size_t)n * nq + q) * np + i];
                    ee[a * np + i] += z * s;
                }
            if (ls != 0.0) {
                /* d/dx_{a,i} of z ls |x(q) - x0(q)|^2 = 2 z ls (x - x0)_a(q) wbar_i(q) */
                value_at(pb, xE, q, u);
                value_at(pb, x0E, q, u0);
                for (int a = 0; a < d; a++)
                    for (int i = 0; i < np; i++)
                        ee[a * np + i] += 2.0 * z * ls * (u[a] - u0[a]) * pb->phi[(size_t)q * np + i];
            }
        }
        (void)d2;
    }
    scatter_add(pb, ev, g);
    free(ev);
    return bad ? 0 : 1;
}

/* Hessian in A-space at one point: HA[an][bp] = sum_kl d2mu[ak][bl] Winv_nk Winv_pl. */
static int hessian_a_at(const oracle_problem *pb, const double *A, double *HA)
{
    int d = pb->dim, d2 = d * d;
    double T[9], mu, d2mu[81];
    t_from_a(pb, A, T);
    if (oracle_metric(d, pb->metric, T, &mu, NULL, d2mu) != 1) return 0;
    for (int a = 0; a < d; a++)
        for (int n = 0; n < d; n++)
            for (int b = 0; b < d; b++)
                for (int p = 0; p < d; p++) {
                    double s = 0.0;
                    for (int k = 0; k < d; k++)
                        for (int l = 0; l < d; l++)
                            s += d2mu[(a * d + k) * d2 + (b * d + l)] * pb->Winv[n * d + k] *
                                 pb->Winv[p * d + l];
                    HA[(a * d + n) * d2 + (b * d + p)] = s;
                }
    return 1;
}

/* y = d2F(x) v (dim*nx).  Returns 0 if det T <= 0 anywhere, else 1. */
int oracle_hessian_apply(const oracle_problem *pb, const double *x, const double *v, double *y)
{
    int d = pb->dim, d2 = d * d, np = pb->np, nq = pb->nq;
    double *ev = (double *)calloc((size_t)pb->ne * d * np, sizeof(double));
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int e = 0; e < pb->ne; e++) {
        double xE[3 * 729], vE[3 * 729], A[9], GV[9], HA[81], Y[9];
        double *ee = ev + (size_t)e * d * np;
        double ls = lim_scale(pb);
        gather_elem(pb, x, e, xE);
        gather_elem(pb, v, e, vE);
        for (int q = 0; q < nq; q++) {
            jacobian_at(pb, xE, q, A);
            if (!hessian_a_at(pb, A, HA)) {
                bad = 1;
                continue;
            }
            jacobian_at(pb, vE, q, GV); /* GV[b][p] = d v_b / d xbar_p */
            for (int r = 0; r < d2; r++) {
                double s = 0.0;
                for (int c = 0; c < d2; c++) s += HA[r * d2 + c] * GV[c];
                Y[r] = s;
            }
            double z = pb->wq[q] * pb->detW;
            for (int a = 0; a < d; a++)
                for (int i = 0; i < np; i++) {
                    double s = 0.0;
                    for (int n = 0; n < d; n++)
                        s += Y[a * d + n] * pb->dphi[((size_t)n * nq + q) * np + i];
                    ee[a * np + i] += z * s;
                }
            if (ls != 0.0) {
                /* limiting: the mass-like term 2 z ls v_a(q) wbar_i(q) (eq. eq_pa_limiting) */
                double vq[3];
                value_at(pb, vE, q, vq);
                for (int a = 0; a < d; a++)
                    for (int i = 0; i < np; i++)
                        ee[a * np + i] += 2.0 * z * ls * vq[a] * pb->phi[(size_t)q * np + i];
            }
        }
    }
    scatter_add(pb, ev, y);
    free(ev);
    return bad ? 0 : 1;
}

/* Diagonal of d2F(x) (dim*nx).  Returns 0 if det T <= 0 anywhere, else 1. */
int oracle_hessian_diag(const oracle_problem *pb, const double *x, double *dg)
{
    int d = pb->dim, d2 = d * d, np = pb->np, nq = pb->nq;
    double *ev = (double *)calloc((size_t)pb->ne * d * np, sizeof(double));
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int e = 0; e < pb->ne; e++) {
        double xE[3 * 729], A[9], HA[81];
        double *ee = ev + (size_t)e * d * np;
        gather_elem(pb, x, e, xE);
        for (int q = 0; q < nq; q++) {
            jacobian_at(pb, xE, q, A);
            if (!hessian_a_at(pb, A, HA)) {
                bad = 1;
                continue;
            }
            double z = pb->wq[q] * pb->detW;
            for (int a = 0; a < d; a++)
                for (int i = 0; i < np; i++) {
                    double s = 0.0;
                    for (int n = 0; n < d; n++)
                        for (int p = 0; p < d; p++)
                            s += HA[(a * d + n) * d2 + (a * d + p)] *
                                 pb->dphi[((size_t)n * nq + q) * np + i] *
                                 pb->dphi[((size_t)p * nq + q) * np + i];
                    double ph = pb->phi[(size_t)q * np + i];
                    ee[a * np + i] += z * (s + 2.0 * lim_scale(pb) * ph * ph);
                }
        }
    }
    scatter_add(pb, ev, dg);
    free(ev);
    return bad ? 0 : 1;
}

/*
 * Dense element Hessian of element e, (dim*np)^2, row index a*np+i and column
 * index b*np+j (local numbering).  This is the full-assembly element matrix of
 * eq. eq_vm_pa_hess, used only on tiny meshes to pin the matrix-free forms.
 * Returns 0 if det T <= 0 at a point of the element.
 */
int oracle_element_hessian(const oracle_problem *pb, const double *x, int e, double *H)
{
    int d = pb->dim, d2 = d * d, np = pb->np, nq = pb->nq, n = d * np;
    double xE[3 * 729], A[9], HA[81];
    memset(H, 0, sizeof(double) * (size_t)n * n);
    gather_elem(pb, x, e, xE);
    for (int q = 0; q < nq; q++) {
        jacobian_at(pb, xE, q, A);
        if (!hessian_a_at(pb, A, HA)) return 0;
        double z = pb->wq[q] * pb->detW;
        for (int a = 0; a < d; a++)
            for (int i = 0; i < np; i++)
                for (int b = 0; b < d; b++)
                    for (int j = 0; j < np; j++) {
                        double s = 0.0;
                        for (int nn = 0; nn < d; nn++)
                            for (int p = 0; p < d; p++)
                                s += HA[(a * d + nn) * d2 + (b * d + p)] *
                                     pb->dphi[((size_t)nn * nq + q) * np + i] *
                                     pb->dphi[((size_t)p * nq + q) * np + j];
                        if (a == b) /* limiting: mass-like block (eq. eq_pa_limiting) */
                            s += 2.0 * lim_scale(pb) * pb->phi[(size_t)q * np + i] *
                                 pb->phi[(size_t)q * np + j];
                        H[(size_t)(a * np + i) * n + (b * np + j)] += z * s;
                    }
    }
    return 1;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
