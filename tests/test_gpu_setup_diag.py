"""Setup and diagonal in one element pass (``tmop_hessian_setup_diag``)
against ``tmop_hessian_setup`` followed by ``tmop_hessian_diag``.

The fused kernel rounds the per-point tensor to the storage precision before
it feeds the diagonal, as the separate diagonal kernel reads it back, so the
diagonal and every later Hessian action are bitwise equal; the diagonal is
also checked against the oracle (1e-11 FP64, 1e-6 mixed).  Every hex class
(one-pass classes take the fused kernel, the others the two kernels), quads,
tensor and compact storage, FP64 and mixed, the limiting term, a sheared
constant target and the matrix-core sweeps (which keep the two kernels).
"""
import numpy as np
import pytest

from paper_2205_12721_amd import inputs
from tests.gpu_common import TOL64, log, make_case, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [(3, (3, 4, 3), 1, 2), (3, (2, 3, 4), 1, 4), (3, (3, 2, 2), 2, 3), (3, (3, 3, 2), 2, 5),
         (3, (3, 3, 3), 3, 4), (3, (3, 3, 3), 3, 5), (3, (2, 3, 2), 3, 6), (3, (2, 2, 2), 4, 5),
         (3, (2, 2, 2), 4, 7), (3, (2, 2, 2), 1, 9), (2, (4, 3), 2, 4)]


def _pair(ctx, xd, v):
    ctx.hessian_setup(xd)
    d0 = to_host(ctx.hessian_diag())
    y0 = to_host(ctx.hessian_apply(to_dev(v)))
    d1 = to_host(ctx.hessian_setup_diag(xd))
    y1 = to_host(ctx.hessian_apply(to_dev(v)))
    return d0, y0, d1, y1


@pytest.mark.parametrize("storage", ["tensor", "compact"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("dim,ns,p,nq", CASES)
def test_setup_diag_bitwise(dim, ns, p, nq, precision, storage):
    from paper_2205_12721_amd.tmop import Context
    log("case", dim, ns, p, nq, precision, storage)
    pb, x = make_case(dim, ns, p, nq, seed=8)
    v = inputs.gaussian_vector(pb.ndof, 13, pb.ess)
    ctx = Context(dim, ns, p, nq, precision=precision, storage=storage)
    d0, y0, d1, y1 = _pair(ctx, to_dev(x), v)
    ctx.close()
    assert np.array_equal(d0, d1) and np.array_equal(y0, y1)
    assert rel(d1, pb.diag(x)) <= (TOL64 if precision == "fp64" else 1e-6)


@pytest.mark.parametrize("variant", ["compact_limiting", "limiting", "mfma", "target",
                                     "compact_target"])
def test_setup_diag_other_paths(variant):
    from paper_2205_12721_amd.tmop import Context
    log("variant", variant)
    dim, ns, p, nq = 3, (3, 3, 2), 3, 5
    W = None
    if variant.endswith("target"):  # a sheared constant target (general-W paths)
        rng = np.random.default_rng(41)
        W = np.eye(3) + 0.2 * rng.standard_normal((3, 3))
        if np.linalg.det(W) < 0:
            W[:, 0] *= -1
    pb, x = make_case(dim, ns, p, nq, seed=9, W=W)
    v = inputs.gaussian_vector(pb.ndof, 14, pb.ess)
    ctx = Context(dim, ns, p, nq, storage="compact" if variant.startswith("compact") else "tensor",
                  W=W)
    if variant in ("limiting", "compact_limiting"):
        x0 = x + 0.01 * np.random.default_rng(31).standard_normal(x.size)
        pb.set_limiting(x0, 0.6, 0.05)
        ctx.set_limiting(to_dev(x0), 0.6, 0.05)
    if variant == "mfma":
        ctx.set_sweeps("mfma")
    d0, y0, d1, y1 = _pair(ctx, to_dev(x), v)
    ctx.close()
    assert np.array_equal(d0, d1) and np.array_equal(y0, y1)
    assert rel(d1, pb.diag(x)) <= TOL64


def test_setup_diag_null_arguments():
    from paper_2205_12721_amd.tmop import lib
    assert lib().tmop_hessian_setup_diag(None, None, None) == 1
