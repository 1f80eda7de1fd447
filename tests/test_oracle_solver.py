"""Pins of the oracle's MINRES and Newton loops.

* MINRES on small SPD and symmetric indefinite systems, with and without an
  SPD diagonal preconditioner, reaches the LAPACK solution after n steps; its
  residual estimate is non-increasing and equals the true M^{-1}-norm of the
  residual.
* Newton on the pin workload (boundary fixed, interior-only jitter) reaches
  the uniform grid, which is the closed-form global minimiser with F = 0
  (shape metrics vanish exactly on similarities); the constrained Hessian at
  the optimum is positive definite on tiny meshes; the final steps converge
  quadratically.
* Error classification: inverted input, non-finite input, iteration cap and
  line-search failure.
"""
import numpy as np
import pytest

import oracle
from oracle import basis, solver
from paper_2205_12721_amd import inputs


def _sym(rng, n, indefinite):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = rng.uniform(0.5, 5.0, n)
    if indefinite:
        ev[::3] *= -1
    return Q @ np.diag(ev) @ Q.T


@pytest.mark.parametrize("indefinite", [False, True])
@pytest.mark.parametrize("precond", [False, True])
def test_minres_small_systems(indefinite, precond):
    rng = np.random.default_rng(11)
    n = 12
    A = _sym(rng, n, indefinite)
    b = rng.standard_normal(n)
    m = rng.uniform(0.5, 2.0, n) if precond else np.ones(n)
    x, its, res = solver.minres(lambda v: A @ v, b, (lambda r: r / m), rtol=1e-14, maxit=n)
    assert np.allclose(x, np.linalg.solve(A, b), atol=1e-9 * np.linalg.norm(x))
    assert all(res[k + 1] <= res[k] * (1 + 1e-12) for k in range(len(res) - 1))
    # the estimate is the M^{-1}-norm of the true residual
    x3, _, res3 = solver.minres(lambda v: A @ v, b, (lambda r: r / m), rtol=0.0, maxit=3)
    r = b - A @ x3
    assert abs(np.sqrt(r @ (r / m)) - res3[-1]) < 1e-10 * res3[0]


def test_minres_zero_rhs():
    x, its, _ = solver.minres(lambda v: v, np.zeros(5))
    assert its == 0 and not x.any()


def test_jacobi_inverse_floor():
    d = np.array([4.0, -2.0, 0.0, 1e-30])
    mi = solver.jacobi_inverse(d, ess=np.array([False, False, False, True]))
    assert mi[0] == 0.25 and mi[1] == 0.5
    assert mi[2] == 1.0 / (4e-14)
    assert mi[3] == 1.0


@pytest.mark.parametrize("dim,n,p,nq", [(2, 3, 2, 4), (3, 2, 2, 4), (3, 2, 1, 3)])
def test_newton_reaches_uniform_grid(dim, n, p, nq):
    pb = oracle.Problem.box(dim, n, p, nq, constrain="boundary")
    x0, _ = inputs.perturbed_box(dim, n, p, basis.gll_nodes(p), 21, recipe="pin", amp=0.1,
                                 is_valid=lambda x: pb.min_det(x) > 0)
    xu = inputs.uniform_nodes((n,) * dim, p, basis.gll_nodes(p))
    x, rep = oracle.newton_solve(pb, x0, rel_grad_tol=1e-8, max_newton=50)
    assert rep["status"] == solver.OK
    assert rep["F"] < 1e-12 * rep["F0"]
    assert np.abs(x - xu).max() < 1e-7
    # quadratic convergence: some step with r_k = |g_k|/|g_0| < 1e-2 has r_{k+1} < 100 r_k^2
    r = [h[1] / rep["g0_norm"] for h in rep["history"]]
    assert any(r[k] < 1e-2 and r[k + 1] < 100 * r[k] ** 2 for k in range(len(r) - 1))


def test_hessian_positive_definite_at_optimum():
    dim, n, p, nq = 2, 2, 2, 4
    pb = oracle.Problem.box(dim, n, p, nq, constrain="boundary")
    xu = inputs.uniform_nodes((n,) * dim, p, basis.gll_nodes(p))
    H = pb.dense_hessian(xu)
    free = ~pb.ess
    ev = np.linalg.eigvalsh(H[np.ix_(free, free)])
    assert ev.min() > 1e-8


def test_newton_error_codes():
    pb = oracle.Problem.box(2, 2, 1, 2, constrain="boundary")
    xu = inputs.uniform_nodes((2, 2), 1, basis.gll_nodes(1))
    bad = xu.copy()
    bad[4] = 1.3
    assert oracle.newton_solve(pb, bad)[1]["status"] == solver.ERR_INVERTED
    nan = xu.copy()
    nan[4] = np.nan
    assert oracle.newton_solve(pb, nan)[1]["status"] == solver.ERR_NONFINITE
    pb3 = oracle.Problem.box(2, 3, 2, 4, constrain="boundary")
    x0, _ = inputs.perturbed_box(2, 3, 2, basis.gll_nodes(2), 3, recipe="interior_jitter",
                                 amp=0.15, is_valid=lambda x: pb3.min_det(x) > 0)
    _, rep = oracle.newton_solve(pb3, x0, max_newton=1, rel_grad_tol=1e-14)
    assert rep["status"] == solver.ERR_NOT_CONVERGED and rep["newton_its"] == 1

    class Stiff:
        """Hessian scaled down by 1e6: the Newton step is 1e6 times too long."""

        def __init__(self, pb):
            self.pb, self.ess = pb, pb.ess

        def __getattr__(self, k):
            return getattr(self.pb, k)

        def hvp(self, x, v):
            return 1e-6 * self.pb.hvp(x, v)

        def diag(self, x):
            return 1e-6 * self.pb.diag(x)

    _, rep = oracle.newton_solve(Stiff(pb3), x0, max_halvings=0)
    assert rep["status"] == solver.ERR_LINESEARCH
