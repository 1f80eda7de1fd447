"""Oracle: preconditioned MINRES and the Newton / line-search loop.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``minres``       -- Paige-Saunders MINRES for a symmetric (possibly
  indefinite) operator with a symmetric positive definite preconditioner,
  started from x = 0 (Sec. 2.3: the Hessian is inverted with MINRES and
  Jacobi preconditioning; Sec. 3.4: the Hessian is symmetric but not
  necessarily positive definite).  Lanczos on the preconditioned operator,
  Givens QR of the tridiagonal matrix, and the short-recurrence update of
  the solution.  Stops when the preconditioned residual norm estimate drops
  below rtol times its initial value, or after maxit iterations.
* ``newton_solve`` -- Newton's method x <- x - alpha dx, dx = H^{-1} g
  (Sec. 2.3, eqs. eq_nodal_solve / eq_nodal_dx), alpha from backtracking by
  halving starting at 1 until det A > 0 at every quadrature point,
  F_new < 1.2 F and |g_new| < 1.2 |g| (Sec. 2.3), stopping when
  |g(x)| / |g(x0)| <= eps (Sec. 2.3, relative l2 norm of the gradient).

Readings where the paper is silent: the det test is taken first (F is
undefined for det <= 0); the inequalities are strict; norms are the l2 norm
of the constrained gradient over all d*N_x entries; fixed DoFs enter as
H_c = P H P + (I - P); the Jacobi diagonal is max(|d|, 1e-14 max|d|) so the
preconditioner is SPD even where mu is not convex.
"""
import math

import numpy as np

OK = 0
ERR_INVERTED = 3
ERR_LINESEARCH = 4
ERR_NOT_CONVERGED = 5
ERR_NONFINITE = 6


def minres(apply_A, b, apply_Minv=None, rtol=1e-12, maxit=50):
    """Solve A x = b.  Returns (x, iterations, estimated residual norms list)."""
    if apply_Minv is None:
        apply_Minv = lambda r: r.copy()  # noqa: E731
    n = b.size
    x = np.zeros(n)
    r1 = b.copy()
    y = apply_Minv(r1)
    beta1 = float(r1 @ y)
    if beta1 < 0:
        raise ValueError("preconditioner is not positive definite")
    beta1 = math.sqrt(beta1)
    res = [beta1]
    if beta1 == 0.0:
        return x, 0, res
    oldb = 0.0
    beta = beta1
    dbar = 0.0
    eps = 0.0
    phibar = beta1
    cs = -1.0
    sn = 0.0
    w = np.zeros(n)
    w2 = np.zeros(n)
    r2 = r1.copy()
    its = 0
    for k in range(1, maxit + 1):
        its = k
        # Lanczos step on the preconditioned operator
        v = y / beta
        y = apply_A(v)
        if k >= 2:
            y = y - (beta / oldb) * r1
        alpha = float(v @ y)
        y = y - (alpha / beta) * r2
        r1 = r2
        r2 = y
        y = apply_Minv(r2)
        oldb = beta
        bb = float(r2 @ y)
        if bb < 0:
            raise ValueError("preconditioner is not positive definite")
        beta = math.sqrt(bb)
        # apply the previous rotation, then build the new one
        oldeps = eps
        delta = cs * dbar + sn * alpha
        gbar = sn * dbar - cs * alpha
        eps = sn * beta
        dbar = -cs * beta
        gamma = math.hypot(gbar, beta)
        gamma = max(gamma, np.finfo(float).tiny)
        cs = gbar / gamma
        sn = beta / gamma
        phi = cs * phibar
        phibar = sn * phibar
        # solution update through the direction vectors w
        w1 = w2
        w2 = w
        w = (v - oldeps * w1 - delta * w2) / gamma
        x = x + phi * w
        res.append(phibar)
        if phibar <= rtol * beta1 or beta == 0.0:
            break
    return x, its, res


def jacobi_inverse(d, ess=None):
    """Inverse Jacobi preconditioner from the Hessian diagonal d (fixed DoFs -> 1)."""
    a = np.abs(d)
    floor = 1e-14 * float(a.max()) if a.size else 0.0
    a = np.maximum(a, floor)
    if ess is not None:
        a[ess] = 1.0
    a[a == 0.0] = 1.0
    return 1.0 / a


class Report(dict):
    pass


def newton_solve(pb, x0, rel_grad_tol=1e-8, max_newton=200, max_minres=50,
                 minres_rtol=1e-12, max_halvings=30, jacobi=True, g0_norm=None):
    """Minimise F over the free DoFs of ``pb`` starting from x0.

    Returns (x, report).  ``report`` holds newton_its, minres_its_total,
    halvings_total, F0, F, g0_norm, g_norm, status and per-iteration history.
    """
    x = np.array(x0, dtype=np.float64, copy=True)
    rep = Report(newton_its=0, minres_its_total=0, halvings_total=0, status=OK,
                 history=[])
    if not np.all(np.isfinite(x)):
        rep["status"] = ERR_NONFINITE
        return x, rep
    if not pb.min_det(x) > 0.0:
        rep["status"] = ERR_INVERTED
        return x, rep
    F = pb.energy(x)
    g = pb.gradient(x)
    gn = float(np.linalg.norm(g))
    n0 = gn if (g0_norm is None or g0_norm <= 0) else float(g0_norm)
    rep.update(F0=F, g0_norm=n0)
    status = ERR_NOT_CONVERGED
    for it in range(max_newton + 1):
        rep["history"].append((F, gn))
        if n0 == 0.0 or F == 0.0 or gn <= rel_grad_tol * n0:
            status = OK
            break
        if it == max_newton:
            break
        Minv = None
        if jacobi:
            minv = jacobi_inverse(pb.diag(x), pb.ess)
            Minv = lambda r, m=minv: m * r  # noqa: E731
        dx, its, _ = minres(lambda v: pb.hvp(x, v), g, Minv, rtol=minres_rtol, maxit=max_minres)
        rep["minres_its_total"] += its
        alpha = 1.0
        accepted = False
        for h in range(max_halvings + 1):
            xt = x - alpha * dx
            if pb.min_det(xt) > 0.0:
                Ft = pb.energy(xt)
                if Ft < 1.2 * F:
                    gt = pb.gradient(xt)
                    gtn = float(np.linalg.norm(gt))
                    if gtn < 1.2 * gn:
                        accepted = True
                        break
            alpha *= 0.5
            rep["halvings_total"] += 1
        if not accepted:
            status = ERR_LINESEARCH
            break
        x, F, g, gn = xt, Ft, gt, gtn
        rep["newton_its"] += 1
    rep.update(F=F, g_norm=gn, status=status)
    return x, rep
