"""The one-pass energy + gradient (``tmop_energy_gradient``) against the
separate calls and the oracle.

F, min det A and g are bitwise those of ``tmop_energy_mindet`` and
``tmop_gradient`` (the fused kernel adds the same terms in the same order over
the same workgroups, and the metric code fuses its multiply-adds per source
expression, so it rounds the same way in both kernels); |g|^2 is the
library's sum of squares, within 1e-14 of numpy's.  Quads and hexes, with
and without the limiting term, pencil and matrix-core sweeps; an inverted
mesh gives F = inf and the INVERTED code, as ``tmop_energy_mindet`` does.
"""
import numpy as np
import pytest

from oracle import basis
from paper_2205_12721_amd import inputs
from tests.gpu_common import TOL64, log, make_case, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [(2, (5, 4), 1, 3), (2, (3, 3), 3, 5), (2, (4, 3), 4, 6), (3, (3, 4, 3), 1, 2),
         (3, (3, 2, 2), 2, 4), (3, (3, 3, 3), 3, 5), (3, (2, 2, 2), 4, 7)]


def _check(ctx, pb, x, xd):
    F0, md0 = ctx.energy_mindet(xd)
    g0 = to_host(ctx.gradient(xd))
    F, md, gd, g2 = ctx.energy_gradient(xd)
    g = to_host(gd)
    assert F == F0 and md == md0
    assert np.array_equal(g, g0)
    assert abs(g2 - float(g @ g)) <= 1e-14 * float(g @ g)
    assert abs(F - pb.energy(x)) <= TOL64 * abs(pb.energy(x))
    assert rel(g, pb.gradient(x)) <= TOL64


@pytest.mark.parametrize("lim", [False, True])
@pytest.mark.parametrize("dim,ns,p,nq", CASES)
def test_energy_gradient_matches_separate_calls(dim, ns, p, nq, lim):
    from paper_2205_12721_amd.tmop import Context
    log("case", dim, ns, p, nq, "lim" if lim else "plain")
    pb, x = make_case(dim, ns, p, nq, seed=6)
    ctx = Context(dim, ns, p, nq)
    if lim:
        x0 = x + 0.01 * np.random.default_rng(23).standard_normal(x.size)
        pb.set_limiting(x0, 0.7, 0.05)
        ctx.set_limiting(to_dev(x0), 0.7, 0.05)
    _check(ctx, pb, x, to_dev(x))
    if dim == 3 and nq <= 5 and not lim:
        ctx.set_sweeps("mfma")
        _check(ctx, pb, x, to_dev(x))
    ctx.close()


def test_energy_gradient_inverted():
    from paper_2205_12721_amd.tmop import Context
    ctx = Context(2, (2, 2), 1, 2, ess="none")
    xu = inputs.uniform_nodes((2, 2), 1, basis.gll_nodes(1))
    xu[4] = 1.3
    xd = to_dev(xu)
    F0, md0 = ctx.energy_mindet(xd)
    F, md, _, _ = ctx.energy_gradient(xd)
    assert F == float("inf") and F0 == F and md < 0 and md == md0
    ctx.close()
