"""Pin of ``oracle.restrict_to_nodes``, the helper that samples large meshes.

The gradient, Hessian action and Hessian diagonal at a global node are sums
over the elements that hold the node (Sec. 3.3, eq. eq_vm_pa_grad; Sec. 3.4,
eq. eq_vm_pa_hess: G^T gathers the element contributions), so a problem made
of only the elements touching a node set gives the full problem's entries at
those nodes.  Checked on small 2D and 3D meshes, with the boundary fixed, with
a random mask of fixed DoFs, and with the limiting term; the sub-problem must
also really be smaller and zero away from its elements.
"""
import numpy as np
import pytest

import oracle
from oracle import basis
from paper_2205_12721_amd import inputs


def _case(dim, ns, p, nq, seed, ess="boundary"):
    pb = oracle.Problem.box(dim, ns, p, nq)
    if ess == "mask":
        mask = np.random.default_rng(seed + 100).uniform(size=pb.ndof) < 0.3
        pb = oracle.Problem(dim, p, nq, pb.e2n, pb.nx, ess=mask)
    x, _ = inputs.perturbed_box(dim, ns, p, basis.gll_nodes(p), seed, recipe="smooth", amp=0.05,
                                is_valid=lambda x: pb.min_det(x) > 0)
    return pb, x


@pytest.mark.parametrize("ess", ["boundary", "mask", "limiting"])
@pytest.mark.parametrize("dim,ns,p,nq", [(2, (5, 4), 2, 4), (2, (4, 3), 3, 5), (3, (3, 3, 2), 2, 4),
                                         (3, (3, 2, 3), 1, 3)])
def test_restricted_entries_equal_full(dim, ns, p, nq, ess):
    pb, x = _case(dim, ns, p, nq, seed=31, ess="mask" if ess == "mask" else "boundary")
    if ess == "limiting":
        x0 = inputs.uniform_nodes(ns, p, basis.gll_nodes(p))
        pb.set_limiting(x0, 0.7, 0.3)
    rng = np.random.default_rng(32)
    nodes = rng.choice(pb.nx, size=max(2, pb.nx // 40), replace=False)
    sub = oracle.restrict_to_nodes(pb, nodes)
    assert sub.e2n.shape[0] < pb.e2n.shape[0]  # a real restriction
    idx = (np.arange(dim)[:, None] * pb.nx + nodes[None, :]).ravel()
    v = inputs.gaussian_vector(pb.ndof, 33)
    g, gs = pb.gradient(x), sub.gradient(x)
    y, ys = pb.hvp(x, v), sub.hvp(x, v)
    d, ds = pb.diag(x), sub.diag(x)
    for full, part in ((g, gs), (y, ys), (d, ds)):
        scale = np.abs(full).max()
        assert np.abs(part[idx] - full[idx]).max() <= 1e-14 * scale
    # away from the kept elements the sub-problem's gradient is zero
    touched = np.unique(sub.e2n)
    far = np.setdiff1d(np.arange(pb.nx), touched)
    assert far.size > 0
    far_idx = (np.arange(dim)[:, None] * pb.nx + far[None, :]).ravel()
    assert np.all(gs[far_idx] == 0.0)


def test_restriction_must_keep_every_touching_element():
    """Dropping one element that holds a sampled node changes that node's entries,
    so the equality above would catch a restriction that keeps too few."""
    pb, x = _case(3, (3, 3, 3), 2, 4, seed=34)
    centre = int(pb.e2n[13, 13])  # the centre node of the middle element (interior)
    sub = oracle.restrict_to_nodes(pb, [centre])
    assert sub.e2n.shape[0] == 1
    corner = int(pb.e2n[13, 0])  # a vertex of the middle element: eight elements hold it
    sub8 = oracle.restrict_to_nodes(pb, [corner])
    assert sub8.e2n.shape[0] == 8
    short = oracle.Problem(3, 2, 4, sub8.e2n[1:], pb.nx, ess=pb.ess)
    idx = np.arange(3) * pb.nx + corner
    assert np.abs(short.gradient(x)[idx] - pb.gradient(x)[idx]).max() > 1e-6 * np.abs(pb.gradient(x)).max()
    assert np.abs(sub8.gradient(x)[idx] - pb.gradient(x)[idx]).max() <= 1e-14 * np.abs(pb.gradient(x)).max()
