"""GPU parity at the benchmark's full sizes, in the launch configuration bench.py
times (one context per mesh, FP64 and mixed).

* 24^3 Q3 hex (n_q = 5): every FP64 output compared in full with the oracle.
* 64^3 Q2 and 32^3 Q4 (6.4M DoFs): sampled outputs -- the oracle evaluates the
  sub-mesh of elements around 400 sampled nodes, whose entries equal the full
  operator's at those nodes -- plus, in mixed precision, the FP32 action's
  error against the FP64 oracle at the same input.
"""
import numpy as np
import pytest

import oracle
from oracle import basis
from paper_2205_12721_amd import inputs
from tests.gpu_common import TOL64, log, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


def _config(name):
    c = inputs.CONFIGS[name]
    pb = oracle.Problem.box(c["dim"], c["n"], c["p"], c["nq"])
    x, info = inputs.config_mesh(name, basis.gll_nodes(c["p"]), is_valid=lambda x: pb.min_det(x) > 0)
    v = inputs.gaussian_vector(pb.ndof, c["vec_seed"], pb.ess)
    return c, pb, x, v


@pytest.mark.parametrize("storage", ["tensor", "compact"])
def test_config2_full_parity(storage):
    from paper_2205_12721_amd.tmop import Context
    c, pb, x, v = _config("c2")
    log("c2 ndof", pb.ndof, storage)
    ctx = Context(3, c["n"], c["p"], c["nq"], storage=storage)
    xd = to_dev(x)
    F, md = ctx.energy_mindet(xd)
    assert abs(F - pb.energy(x)) <= TOL64 * pb.energy(x)
    assert abs(md - pb.min_det(x)) <= 1e-12 * abs(md)
    assert rel(to_host(ctx.gradient(xd)), pb.gradient(x)) <= TOL64
    ctx.hessian_setup(xd)
    yo = pb.hvp(x, v)
    assert rel(to_host(ctx.hessian_apply(to_dev(v))), yo) <= TOL64
    assert rel(to_host(ctx.hessian_diag()), pb.diag(x)) <= TOL64
    ctx.close()
    ctx = Context(3, c["n"], c["p"], c["nq"], precision="mixed", storage=storage)
    ctx.hessian_setup(xd)
    err = rel(to_host(ctx.hessian_apply(to_dev(v))), yo)
    log("c2 mixed hvp rel err %.3e" % err, storage)
    assert err <= 2e-6
    ctx.close()


@pytest.mark.parametrize("storage", ["tensor", "compact"])
@pytest.mark.parametrize("name", ["c3a", "c3b"])
def test_config3_sampled_parity(name, storage):
    from paper_2205_12721_amd.tmop import Context
    c = inputs.CONFIGS[name]
    ctx = Context(3, c["n"], c["p"], c["nq"], storage=storage)
    pb_full = oracle.Problem.box(3, c["n"], c["p"], c["nq"])
    # det check on the GPU path is not used to build oracle inputs: sample the
    # mesh with the oracle's own det test restricted to all elements is too slow
    # here, so accept the draw with the oracle's min det over the full mesh
    x, info = inputs.config_mesh(name, basis.gll_nodes(c["p"]), is_valid=lambda x: pb_full.min_det(x) > 0)
    v = inputs.gaussian_vector(pb_full.ndof, c["vec_seed"], pb_full.ess)
    log(name, "ndof", pb_full.ndof, "tries", info["tries"])
    rng = np.random.default_rng(77)
    nodes = rng.choice(pb_full.nx, size=400, replace=False)
    sub = oracle.restrict_to_nodes(pb_full, nodes)
    idx = np.concatenate([a * pb_full.nx + nodes for a in range(3)])
    xd = to_dev(x)
    g = to_host(ctx.gradient(xd))
    assert rel(g[idx], sub.gradient(x)[idx]) <= TOL64
    ctx.hessian_setup(xd)
    yo = sub.hvp(x, v)[idx]
    assert rel(to_host(ctx.hessian_apply(to_dev(v)))[idx], yo) <= TOL64
    assert rel(to_host(ctx.hessian_diag())[idx], sub.diag(x)[idx]) <= TOL64
    ctx.close()
    ctx = Context(3, c["n"], c["p"], c["nq"], precision="mixed", storage=storage)
    ctx.hessian_setup(xd)
    err = rel(to_host(ctx.hessian_apply(to_dev(v)))[idx], yo)
    log(name, "mixed hvp rel err (sampled) %.3e" % err)
    assert err <= 2e-6
    ctx.close()


def test_config2_minres_full():
    """24^3 Q3, FP64 tensor storage: 20 Jacobi-MINRES iterations on H_c dx = g (the
    bench's Newton step; the Lanczos vectors resident) against the oracle's MINRES on
    the same operator, in full."""
    from oracle import solver
    from paper_2205_12721_amd.tmop import Context
    c, pb, x, _ = _config("c2")
    g = pb.gradient(x)
    minv = solver.jacobi_inverse(pb.diag(x), pb.ess)
    xo, ito, _ = solver.minres(lambda w: pb.hvp(x, w), g, lambda r: minv * r, rtol=1e-12,
                               maxit=20)
    ctx = Context(3, c["n"], c["p"], c["nq"])
    ctx.hessian_setup(to_dev(x))
    dx, itg = ctx.minres(to_dev(g), max_its=20, rtol=1e-12, jacobi=True)
    e = rel(to_host(dx), xo)
    log("c2 minres its oracle", ito, "gpu", itg, "rel %.3e" % e)
    assert itg == ito == 20
    assert e <= 1e-9
    ctx.close()


@pytest.mark.parametrize("name", ["c3a", "c3b"])
def test_config3_mixed_solve_final_energy(name):
    """64^3 Q2 and 32^3 Q4: solves to |g|/|g0| <= 1e-8 with the FP32 action inside
    MINRES (tensor and compact storage) end at the FP64 tensor solve's energy within
    1e-10 relative."""
    from paper_2205_12721_amd.tmop import Context
    c = inputs.CONFIGS[name]
    pb_full = oracle.Problem.box(3, c["n"], c["p"], c["nq"])
    x, _ = inputs.config_mesh(name, basis.gll_nodes(c["p"]), is_valid=lambda x: pb_full.min_det(x) > 0)
    res = {}
    for storage, prec in (("tensor", "fp64"), ("tensor", "mixed"), ("compact", "mixed")):
        ctx = Context(3, c["n"], c["p"], c["nq"], precision=prec, storage=storage)
        xd = to_dev(x)
        rep = ctx.solve(xd, rel_grad_tol=1e-8, max_newton=100)
        ctx.close()
        assert rep["status"] == 0, rep
        res[(storage, prec)] = (rep["F"], to_host(xd), rep["newton_its"])
    F64, x64, _ = res[("tensor", "fp64")]
    for k, (F, xs, its) in res.items():
        eF = abs(F - F64) / abs(F64)
        log(name, k, "newton", its, "F rel diff %.2e" % eF, "x rel %.2e" % rel(xs, x64))
        assert eF <= 1e-10
