"""Forward sweeps on the FP64 matrix cores (``tmop_set_sweeps(ctx, MFMA)``)
against the FP64 oracle.

Every hex class with n_q <= 5 (the classes that have the form), at the
sizes of the pencil-sweep parity tests: energy, min det, gradient, and the
Hessian action and diagonal of the quadrature data the MFMA setup stored
(tensor and compact storage), each at 1e-11 relative (l2 and entrywise,
``gpu_common.rel``), and within 1e-13 of the pencil sweeps' results (the two
differ only in rounding order).  A Newton solve with the MFMA sweeps ends on
the oracle's nodes (1e-9).  Classes without the form refuse it; with a
limiting term the context keeps the pencil sweeps, so results are bitwise
those of the pencil form.
"""
import numpy as np
import pytest

import oracle
from paper_2205_12721_amd import inputs
from tests.gpu_common import TOL64, TOLX, log, make_case, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [
    (3, (3, 4, 3), 1, 2),
    (3, (2, 3, 4), 1, 3),
    (3, (3, 2, 3), 1, 4),
    (3, (3, 2, 2), 2, 3),
    (3, (3, 3, 3), 2, 4),
    (3, (3, 3, 3), 2, 5),
    (3, (3, 3, 2), 3, 4),
    (3, (3, 3, 3), 3, 5),
    (3, (3, 3, 3), 4, 5),
]


def _ctx(dim, ns, p, nq, **kw):
    from paper_2205_12721_amd.tmop import Context
    return Context(dim, ns, p, nq, **kw)


def _evaluate(ctx, xd, v):
    F, md = ctx.energy_mindet(xd)
    g = to_host(ctx.gradient(xd))
    ctx.hessian_setup(xd)
    y = to_host(ctx.hessian_apply(to_dev(v)))
    d = to_host(ctx.hessian_diag())
    return F, md, g, y, d


@pytest.mark.parametrize("storage", ["tensor", "compact"])
@pytest.mark.parametrize("dim,ns,p,nq", CASES)
def test_mfma_sweeps_match_oracle(dim, ns, p, nq, storage):
    log("case", dim, ns, p, nq, storage)
    pb, x = make_case(dim, ns, p, nq, seed=3)
    v = inputs.gaussian_vector(pb.ndof, 11, pb.ess)
    xd = to_dev(x)
    ctx = _ctx(dim, ns, p, nq, storage=storage)
    ref = _evaluate(ctx, xd, v)
    ctx.set_sweeps("mfma")
    F, md, g, y, d = _evaluate(ctx, xd, v)
    ctx.close()
    assert abs(F - pb.energy(x)) <= TOL64 * abs(pb.energy(x))
    assert abs(md - pb.min_det(x)) <= 1e-12 * abs(pb.min_det(x))
    assert rel(g, pb.gradient(x)) <= TOL64
    assert rel(y, pb.hvp(x, v)) <= TOL64
    assert rel(d, pb.diag(x)) <= TOL64
    # the pencil form, same mesh: equal up to rounding order
    assert abs(F - ref[0]) <= 1e-13 * abs(ref[0])
    for a, b in zip((g, y, d), ref[2:]):
        assert rel(a, b) <= 1e-13


def test_mfma_constant_target_and_mask():
    """A sheared constant target and a random mask of fixed DoFs."""
    import torch
    rng = np.random.default_rng(7)
    W = np.eye(3) + 0.2 * rng.standard_normal((3, 3))
    if np.linalg.det(W) < 0:
        W[:, 0] *= -1
    pb, x = make_case(3, (2, 3, 2), 3, 5, seed=5, W=W)
    mask = pb.ess | (np.random.default_rng(5).uniform(size=pb.ndof) < 0.3)
    pb = oracle.Problem(3, 3, 5, pb.e2n, pb.nx, W=W, ess=mask)
    mdev = torch.as_tensor(mask.astype(np.uint8)).cuda()
    v = inputs.gaussian_vector(pb.ndof, 14)
    ctx = _ctx(3, (2, 3, 2), 3, 5, W=W, ess=mdev)
    ctx.set_sweeps("mfma")
    F, md, g, y, d = _evaluate(ctx, to_dev(x), v)
    ctx.close()
    assert abs(F - pb.energy(x)) <= TOL64 * pb.energy(x)
    assert rel(g, pb.gradient(x)) <= TOL64
    assert rel(y, pb.hvp(x, v)) <= TOL64
    assert rel(d, pb.diag(x)) <= TOL64


def test_mfma_solve_matches_oracle():
    pb, x0 = make_case(3, (3, 3, 3), 3, 5, seed=21)
    ctx = _ctx(3, (3, 3, 3), 3, 5)
    ctx.set_sweeps("mfma")
    xd = to_dev(x0)
    rep = ctx.solve(xd, rel_grad_tol=1e-10, max_newton=100)
    ctx.close()
    xo, ro = oracle.newton_solve(pb, x0, rel_grad_tol=1e-10, max_newton=100)
    e = rel(to_host(xd), xo)
    log("mfma solve", rep["newton_its"], ro["newton_its"], "x rel %.2e" % e)
    assert rep["status"] == 0 and ro["status"] == 0
    assert e <= TOLX


def test_mfma_refused_and_limiting_keeps_pencil():
    from paper_2205_12721_amd.tmop import TmopError
    for dim, ns, p, nq in [(3, (2, 2, 2), 3, 6), (2, (4, 4), 2, 4)]:
        ctx = _ctx(dim, ns, p, nq)
        with pytest.raises(TmopError):
            ctx.set_sweeps("mfma")
        ctx.close()
    pb, x = make_case(3, (2, 3, 2), 2, 4, seed=4)
    x0 = x + 0.01 * np.random.default_rng(4).standard_normal(x.shape) * (~pb.ess)
    xd = to_dev(x)
    out = []
    for mode in ("pencil", "mfma"):
        ctx = _ctx(3, (2, 3, 2), 2, 4)
        ctx.set_limiting(to_dev(x0), 0.5, 0.2)
        ctx.set_sweeps(mode)
        out.append((ctx.energy(xd), to_host(ctx.gradient(xd))))
        ctx.close()
    assert out[0][0] == out[1][0] and np.array_equal(out[0][1], out[1][1])
