"""Pins of the oracle's limiting term (eq. eq_F_full, second integral, with
xi(y, delta) = |y|^2 / delta^2, and its mass-like Hessian, eq. eq_pa_limiting).

* at x = x0 the limiting term adds nothing to F and g
* for x = x0 + s (a constant shift) the basis is a partition of unity, so the
  term equals coef |s|^2 / delta^2 times the total target volume
  sum_E sum_q w_q det W = N_e det W, and its gradient pairs with a constant
  vector t_a as 2 coef s_a / delta^2 N_e det W
* the limiting Hessian is the FE mass matrix times 2 coef / delta^2 (det W):
  v^T M v for v = 1 in one component is 2 coef / delta^2 N_e det W; it does not
  depend on x
* total gradient and Hessian action = central differences; symmetry; dense
  element Hessians and the diagonal agree with the matrix-free forms
"""
import numpy as np
import pytest

import oracle
from oracle import basis
from paper_2205_12721_amd import inputs

CASES = [(2, 3, 2, 4), (2, 2, 3, 5), (3, 2, 1, 3), (3, 1, 2, 4)]


def _mesh(dim, n, p, nq, seed=7):
    pb = oracle.Problem.box(dim, n, p, nq, constrain=None)
    x, _ = inputs.perturbed_box(dim, n, p, basis.gll_nodes(p), seed, recipe="interior_jitter",
                                amp=0.12, is_valid=lambda x: pb.min_det(x) > 0)
    return pb, x


def _uniform(dim, n, p):
    return inputs.uniform_nodes((n,) * dim, p, basis.gll_nodes(p))


@pytest.mark.parametrize("dim,n,p,nq", CASES)
def test_limiting_closed_forms(dim, n, p, nq):
    pb, x = _mesh(dim, n, p, nq)
    F, g = pb.energy(x), pb.gradient_full(x)
    coef, delta = 0.7, 0.2
    pb.set_limiting(x, coef, delta)
    assert abs(pb.energy(x) - F) <= 1e-14 * F
    assert np.allclose(pb.gradient_full(x), g, atol=1e-13 * np.abs(g).max())
    s = np.array([0.03, -0.02, 0.05][:dim])
    nx = x.size // dim
    xs = (x.reshape(dim, -1) + s[:, None]).ravel()
    ne = n ** dim
    lim = coef * (s @ s) / delta ** 2 * ne * 1.0
    assert abs(pb.energy(xs) - (F + lim)) <= 1e-12 * (F + lim)
    gs = pb.gradient_full(xs)
    for a in range(dim):
        t = np.zeros((dim, nx))
        t[a] = 1.0
        # the TMOP part is translation invariant, so only the limiting part remains
        assert abs(gs @ t.ravel() - 2 * coef * s[a] / delta ** 2 * ne) <= 1e-11 * max(1.0, abs(gs).max())
        v = t.ravel()
        Hv = pb.hvp_full(xs, v)
        assert abs(v @ Hv - 2 * coef / delta ** 2 * ne) <= 1e-10 * (2 * coef / delta ** 2 * ne)


@pytest.mark.parametrize("dim,n,p,nq", CASES)
def test_limiting_hessian_is_constant_mass(dim, n, p, nq):
    pb, x = _mesh(dim, n, p, nq)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(x.size)
    H0 = pb.hvp_full(x, v)
    x0 = x + 0.01 * rng.standard_normal(x.size)
    pb.set_limiting(x0, 1.3, 0.5)
    Hl = pb.hvp_full(x, v)
    # the difference does not depend on x or x0
    pb.set_limiting(x0 + 0.02, 1.3, 0.5)
    assert np.allclose(pb.hvp_full(x, v) - H0, Hl - H0, atol=1e-12 * np.abs(Hl).max())
    # and is linear in coef / delta^2
    pb.set_limiting(x0, 2.6, 0.5)
    assert np.allclose(pb.hvp_full(x, v) - H0, 2 * (Hl - H0), atol=1e-12 * np.abs(Hl).max())


@pytest.mark.parametrize("dim,n,p,nq", CASES)
def test_limiting_derivatives(dim, n, p, nq):
    pb, x = _mesh(dim, n, p, nq)
    rng = np.random.default_rng(5)
    pb.set_limiting(x + 0.02 * rng.standard_normal(x.size), 0.9, 0.3)
    g = pb.gradient_full(x)
    d = rng.standard_normal(x.size)
    fds = [(pb.energy(x + h * d) - pb.energy(x - h * d)) / (2 * h) for h in (2e-5, 1e-5)]
    assert abs((4 * fds[1] - fds[0]) / 3 - g @ d) < 1e-8 * max(abs(g @ d), 1e-8)
    v = rng.standard_normal(x.size)
    y = pb.hvp_full(x, v)
    fdh = [(pb.gradient_full(x + h * v) - pb.gradient_full(x - h * v)) / (2 * h)
           for h in (2e-5, 1e-5)]
    assert np.linalg.norm((4 * fdh[1] - fdh[0]) / 3 - y) < 1e-7 * np.linalg.norm(y)
    w = rng.standard_normal(x.size)
    assert abs(w @ y - v @ pb.hvp_full(x, w)) < 1e-12 * np.linalg.norm(y) * np.linalg.norm(w)
    H = pb.dense_hessian(x)
    assert np.allclose(H, H.T, atol=1e-12 * np.abs(H).max())
    assert np.allclose(H @ v, y, atol=1e-12 * np.abs(y).max())
    assert np.allclose(np.diag(H), pb.diag_full(x), atol=1e-12 * np.abs(H).max())
