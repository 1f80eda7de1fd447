"""GPU parity of the limiting term (eq. eq_F_full, second integral, with
xi = |x - x0|^2 / delta^2; its Hessian is the mass-like operator of eq.
eq_pa_limiting): energy, gradient, Hessian action and diagonal within 1e-11
of the oracle, quads and hexes, both storages, ideal and constant target;
a full solve with the term ends at the oracle's nodes within 1e-9; removing
the term restores the plain values; bad arguments are rejected.
"""
import numpy as np
import pytest

import oracle
from paper_2205_12721_amd import inputs
from tests.gpu_common import TOL64, TOLX, log, make_case, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [(2, (5, 4), 2, 4), (2, (3, 3), 3, 5), (3, (2, 3, 2), 1, 3), (3, (3, 2, 2), 2, 4),
         (3, (3, 3, 3), 3, 5), (3, (2, 2, 2), 4, 6)]


@pytest.mark.parametrize("storage", ["tensor", "compact"])
@pytest.mark.parametrize("dim,ns,p,nq", CASES)
def test_limiting_matches_oracle(dim, ns, p, nq, storage):
    from paper_2205_12721_amd.tmop import Context
    log("case", dim, ns, p, nq, storage)
    W = None if p != 2 else 1.3 * np.eye(dim)
    pb, x = make_case(dim, ns, p, nq, seed=3, W=W)
    rng = np.random.default_rng(17)
    x0 = x + 0.01 * rng.standard_normal(x.size)
    coef, delta = 0.8, 0.05
    pb.set_limiting(x0, coef, delta)
    v = inputs.gaussian_vector(pb.ndof, 11, pb.ess)
    ctx = Context(dim, ns, p, nq, storage=storage, W=W)
    ctx.set_limiting(to_dev(x0), coef, delta)
    xd = to_dev(x)
    F = ctx.energy(xd)
    assert abs(F - pb.energy(x)) <= TOL64 * abs(pb.energy(x))
    assert rel(to_host(ctx.gradient(xd)), pb.gradient(x)) <= TOL64
    ctx.hessian_setup(xd)
    assert rel(to_host(ctx.hessian_apply(to_dev(v))), pb.hvp(x, v)) <= TOL64
    assert rel(to_host(ctx.hessian_diag()), pb.diag(x)) <= TOL64
    # removing the term restores the plain operators
    ctx.set_limiting(None)
    pb.set_limiting(None)
    assert abs(ctx.energy(xd) - pb.energy(x)) <= TOL64 * abs(pb.energy(x))
    assert rel(to_host(ctx.hessian_apply(to_dev(v))), pb.hvp(x, v)) <= TOL64
    assert rel(to_host(ctx.hessian_diag()), pb.diag(x)) <= TOL64
    ctx.close()


def test_limiting_mixed_action():
    from paper_2205_12721_amd.tmop import Context
    dim, ns, p, nq = 3, (3, 3, 2), 2, 4
    pb, x = make_case(dim, ns, p, nq, seed=4)
    x0 = x + 0.02
    pb.set_limiting(x0, 2.0, 0.1)
    v = inputs.gaussian_vector(pb.ndof, 12, pb.ess)
    for storage in ("tensor", "compact"):
        ctx = Context(dim, ns, p, nq, storage=storage, precision="mixed")
        ctx.set_limiting(to_dev(x0), 2.0, 0.1)
        xd = to_dev(x)
        ctx.hessian_setup(xd)
        assert rel(to_host(ctx.hessian_apply(to_dev(v))), pb.hvp(x, v)) <= 1e-5
        assert abs(ctx.energy(xd) - pb.energy(x)) <= TOL64 * pb.energy(x)
        ctx.close()


@pytest.mark.parametrize("dim,ns,p,nq", [(2, (4, 4), 2, 4), (3, (2, 2, 2), 2, 4)])
def test_limiting_solve_matches_oracle(dim, ns, p, nq):
    from paper_2205_12721_amd.tmop import Context
    pb, x = make_case(dim, ns, p, nq, seed=5)
    x0 = x.copy()
    pb.set_limiting(x0, 1.0, 0.02)
    xo, ro = oracle.newton_solve(pb, x, rel_grad_tol=1e-10, max_newton=100)
    assert ro["status"] == 0
    ctx = Context(dim, ns, p, nq)
    ctx.set_limiting(to_dev(x0), 1.0, 0.02)
    xd = to_dev(x)
    rep = ctx.solve(xd, rel_grad_tol=1e-10, max_newton=100)
    ctx.close()
    assert rep["status"] == 0
    assert rel(to_host(xd), xo) <= TOLX
    # the limited solve moves the nodes less than the free one
    pb.set_limiting(None)
    xf, _ = oracle.newton_solve(pb, x, rel_grad_tol=1e-10, max_newton=100)
    assert np.linalg.norm(xo - x0) < np.linalg.norm(xf - x0)


def test_limiting_bad_arguments():
    from paper_2205_12721_amd.tmop import Context, TmopError
    ctx = Context(2, (2, 2), 1, 2)
    x0 = to_dev(np.zeros(ctx.ndof))
    with pytest.raises(TmopError) as e:
        ctx.set_limiting(x0, 1.0, 0.0)
    assert e.value.code == 1
    with pytest.raises(TmopError):
        ctx.set_limiting(x0, -1.0, 1.0)
    ctx.close()
