"""Pins of the oracle's FE operators with the size and shape+size metrics of
Sec. 2.2: mu_55 = (tau - 1)^2 (2D and 3D), mu_7 = |T - T^{-t}|^2 and
mu_9 = tau |T - T^{-t}|^2 (2D).

* with the target W = h I (h = 1/n, the uniform element size), F = 0 and
  g = 0 on the uniform grid and on its rigid motions (these metrics are not
  scale invariant, so a scaled grid has F > 0)
* gradient = central differences of F, Hessian action = central differences
  of the gradient (Richardson-extrapolated)
* symmetry of the action; the dense Hessian equals the action and its diagonal
  the Jacobi diagonal
* translation and rotation identities: g . t_a = 0, H t_a = 0,
  (Omega x) . g = 0, H (Omega x) = Omega g
"""
import numpy as np
import pytest

import oracle
from oracle import basis
from paper_2205_12721_amd import inputs

CASES = [(2, 7, 2, 2, 4), (2, 9, 2, 2, 4), (2, 55, 2, 2, 4), (2, 7, 3, 1, 3),
         (3, 55, 1, 2, 4), (3, 55, 2, 1, 3)]


def _problem(dim, metric, n, p, nq):
    return oracle.Problem.box(dim, n, p, nq, metric_id=metric, W=np.eye(dim) / n, constrain=None)


def _uniform(dim, n, p):
    return inputs.uniform_nodes((n,) * dim, p, basis.gll_nodes(p))


def _mesh(dim, metric, n, p, nq, seed=7):
    pb = _problem(dim, metric, n, p, nq)
    x, _ = inputs.perturbed_box(dim, n, p, basis.gll_nodes(p), seed, recipe="interior_jitter",
                                amp=0.12, is_valid=lambda x: pb.min_det(x) > 0)
    return pb, x


def _rotation(dim, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((dim, dim)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    return Q


@pytest.mark.parametrize("dim,metric,n,p,nq", CASES)
def test_zero_on_uniform_and_rigid_motions(dim, metric, n, p, nq):
    pb = _problem(dim, metric, n, p, nq)
    x = _uniform(dim, n, p)
    X = x.reshape(dim, -1)
    for M, c in [(np.eye(dim), np.zeros(dim)), (_rotation(dim, 1), np.arange(dim) + 0.3)]:
        xm = (M @ X + c[:, None]).ravel()
        assert abs(pb.energy(xm)) < 1e-13
        assert np.abs(pb.gradient_full(xm)).max() < 1e-12
    assert pb.energy(1.2 * x) > 1e-3


@pytest.mark.parametrize("dim,metric,n,p,nq", CASES)
def test_derivatives_match_finite_differences(dim, metric, n, p, nq):
    pb, x = _mesh(dim, metric, n, p, nq)
    g = pb.gradient_full(x)
    rng = np.random.default_rng(5)
    d = rng.standard_normal(x.size)
    fds = [(pb.energy(x + h * d) - pb.energy(x - h * d)) / (2 * h) for h in (2e-5, 1e-5)]
    rich = (4 * fds[1] - fds[0]) / 3
    assert abs(rich - g @ d) < 1e-8 * max(abs(g @ d), 1e-8)
    v = rng.standard_normal(x.size)
    y = pb.hvp_full(x, v)
    fdh = [(pb.gradient_full(x + h * v) - pb.gradient_full(x - h * v)) / (2 * h)
           for h in (2e-5, 1e-5)]
    assert np.linalg.norm((4 * fdh[1] - fdh[0]) / 3 - y) < 1e-7 * np.linalg.norm(y)


@pytest.mark.parametrize("dim,metric,n,p,nq", CASES)
def test_symmetry_dense_and_diagonal(dim, metric, n, p, nq):
    pb, x = _mesh(dim, metric, n, p, nq)
    rng = np.random.default_rng(8)
    v, w = rng.standard_normal(x.size), rng.standard_normal(x.size)
    Hv, Hw = pb.hvp_full(x, v), pb.hvp_full(x, w)
    assert abs(w @ Hv - v @ Hw) < 1e-12 * np.linalg.norm(Hv) * np.linalg.norm(w)
    H = pb.dense_hessian(x)
    assert np.allclose(H, H.T, atol=1e-12 * np.abs(H).max())
    assert np.allclose(H @ v, Hv, atol=1e-12 * np.abs(Hv).max())
    assert np.allclose(np.diag(H), pb.diag_full(x), atol=1e-12 * np.abs(H).max())


@pytest.mark.parametrize("dim,metric,n,p,nq", CASES)
def test_translation_rotation_identities(dim, metric, n, p, nq):
    pb, x = _mesh(dim, metric, n, p, nq)
    g = pb.gradient_full(x)
    gs = np.linalg.norm(g)
    X = x.reshape(dim, -1)
    nx = X.shape[1]
    for a in range(dim):
        t = np.zeros((dim, nx))
        t[a] = 1.0
        t = t.ravel()
        assert abs(g @ t) < 1e-12 * gs * np.sqrt(nx)
        assert np.linalg.norm(pb.hvp_full(x, t)) < 1e-11 * gs * np.sqrt(nx) * n
    for (i, j) in [(0, 1)] + ([(0, 2), (1, 2)] if dim == 3 else []):
        Om = np.zeros((dim, dim))
        Om[i, j], Om[j, i] = 1.0, -1.0
        ox = (Om @ X).ravel()
        og = (Om @ g.reshape(dim, -1)).ravel()
        assert abs(g @ ox) < 1e-12 * gs * np.linalg.norm(x)
        assert np.allclose(pb.hvp_full(x, ox), og, atol=1e-11 * np.abs(g).max())
