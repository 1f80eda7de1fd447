"""Pins of the oracle's FE-level operators (energy, gradient, Hessian, diagonal).

* affine meshes give A = M exactly (Sec. 3.2 Jacobian)
* F = 0 and g = 0 on uniform, rotated, translated and scaled meshes
  (ideal target, shape metrics)
* gradient = central differences of F; Hessian action = central differences
  of the gradient (second-order accurate, checked at two step sizes)
* symmetry of the Hessian action and of the dense (fully assembled) Hessian;
  the dense Hessian times v equals the matrix-free action (the paper's
  statement that partial assembly does not change the result, Sec. 1)
* exact identities of shape metrics: H t_a = 0, g . t_a = 0 (translation);
  x . g = 0, H x = -g (scale); (Omega x) . g = 0, H (Omega x) = Omega g
  (rotation)
* the Jacobi diagonal equals the diagonal of the dense Hessian
* a constant target W scales F by det W for W = cI and leaves it unchanged for
  a rotation W
"""
import numpy as np
import pytest

import oracle
from oracle import basis
from paper_2205_12721_amd import inputs

CASES = [(2, 3, 2, 4), (2, 2, 3, 5), (3, 2, 1, 3), (3, 1, 2, 4), (3, 1, 3, 5)]


def _mesh(dim, n, p, nq, recipe="interior_jitter", amp=0.12, seed=7, constrain=None):
    pb = oracle.Problem.box(dim, n, p, nq, constrain=constrain)
    x, _ = inputs.perturbed_box(dim, n, p, basis.gll_nodes(p), seed, recipe=recipe, amp=amp,
                                is_valid=lambda x: pb.min_det(x) > 0)
    return pb, x


def _uniform(dim, n, p):
    return inputs.uniform_nodes((n,) * dim, p, basis.gll_nodes(p))


def _rotation(dim, seed=0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((dim, dim)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    return Q


def _map_nodes(x, dim, M, c):
    X = x.reshape(dim, -1)
    return (M @ X + np.asarray(c)[:, None]).ravel()


@pytest.mark.parametrize("dim,n,p,nq", CASES)
def test_affine_jacobian(dim, n, p, nq):
    pb = oracle.Problem.box(dim, n, p, nq, constrain=None)
    rng = np.random.default_rng(4)
    M = np.eye(dim) + 0.3 * rng.standard_normal((dim, dim))
    x = _map_nodes(_uniform(dim, n, p), dim, M, rng.standard_normal(dim))
    A = pb.jacobians(x)
    assert np.allclose(A, M / n, atol=1e-13)


@pytest.mark.parametrize("dim,n,p,nq", CASES)
def test_zero_energy_gradient_on_similarity(dim, n, p, nq):
    pb = oracle.Problem.box(dim, n, p, nq, constrain=None)
    x = _uniform(dim, n, p)
    for M, c in [(np.eye(dim), np.zeros(dim)),
                 (2.5 * _rotation(dim, 1), np.arange(dim) + 0.3),
                 (0.2 * _rotation(dim, 2), -np.ones(dim))]:
        xm = _map_nodes(x, dim, M, c)
        assert abs(pb.energy(xm)) < 1e-13
        assert np.abs(pb.gradient_full(xm)).max() < 1e-12 * max(1.0, 1.0 / np.linalg.norm(M))


@pytest.mark.parametrize("dim,n,p,nq", CASES)
def test_energy_positive_on_perturbed(dim, n, p, nq):
    pb, x = _mesh(dim, n, p, nq)
    assert pb.energy(x) > 0


@pytest.mark.parametrize("dim,n,p,nq", CASES)
def test_gradient_matches_finite_differences(dim, n, p, nq):
    pb, x = _mesh(dim, n, p, nq)
    g = pb.gradient_full(x)
    rng = np.random.default_rng(5)
    for _ in range(3):
        d = rng.standard_normal(x.size)
        fds, errs = [], []
        for h in (2e-5, 1e-5):
            fd = (pb.energy(x + h * d) - pb.energy(x - h * d)) / (2 * h)
            fds.append(fd)
            errs.append(abs(fd - g @ d))
        scale = max(abs(g @ d), 1e-8)
        # second order: halving h divides the error by about 4
        assert errs[1] < 0.3 * errs[0] or errs[1] < 1e-9 * scale
        # Richardson extrapolation removes the h^2 term
        rich = (4 * fds[1] - fds[0]) / 3
        assert abs(rich - g @ d) < 1e-8 * scale


@pytest.mark.parametrize("dim,n,p,nq", CASES)
def test_hvp_matches_finite_differences(dim, n, p, nq):
    pb, x = _mesh(dim, n, p, nq)
    rng = np.random.default_rng(6)
    v = rng.standard_normal(x.size)
    y = pb.hvp_full(x, v)
    fds, errs = [], []
    for h in (2e-5, 1e-5):
        fd = (pb.gradient_full(x + h * v) - pb.gradient_full(x - h * v)) / (2 * h)
        fds.append(fd)
        errs.append(np.linalg.norm(fd - y))
    assert errs[1] < 0.3 * errs[0] or errs[1] < 1e-9 * np.linalg.norm(y)
    rich = (4 * fds[1] - fds[0]) / 3
    assert np.linalg.norm(rich - y) < 1e-7 * np.linalg.norm(y)


@pytest.mark.parametrize("dim,n,p,nq", CASES)
def test_hvp_symmetry_and_dense(dim, n, p, nq):
    pb, x = _mesh(dim, n, p, nq)
    rng = np.random.default_rng(8)
    v = rng.standard_normal(x.size)
    w = rng.standard_normal(x.size)
    Hv = pb.hvp_full(x, v)
    Hw = pb.hvp_full(x, w)
    assert abs(w @ Hv - v @ Hw) < 1e-12 * np.linalg.norm(Hv) * np.linalg.norm(w)
    H = pb.dense_hessian(x)
    assert np.allclose(H, H.T, atol=1e-12 * np.abs(H).max())
    assert np.allclose(H @ v, Hv, atol=1e-12 * np.abs(Hv).max())
    assert np.allclose(np.diag(H), pb.diag_full(x), atol=1e-12 * np.abs(H).max())


@pytest.mark.parametrize("dim,n,p,nq", CASES)
def test_shape_metric_identities(dim, n, p, nq):
    pb, x = _mesh(dim, n, p, nq)
    g = pb.gradient_full(x)
    gs = np.linalg.norm(g)
    X = x.reshape(dim, -1)
    nx = X.shape[1]
    # translation
    for a in range(dim):
        t = np.zeros((dim, nx))
        t[a] = 1.0
        t = t.ravel()
        assert abs(g @ t) < 1e-12 * gs * np.sqrt(nx)
        assert np.linalg.norm(pb.hvp_full(x, t)) < 1e-11 * gs * np.sqrt(nx) * n
    # scale
    assert abs(g @ x) < 1e-12 * gs * np.linalg.norm(x)
    assert np.allclose(pb.hvp_full(x, x), -g, atol=1e-11 * np.abs(g).max())
    # rotation generators
    for (i, j) in [(0, 1)] + ([(0, 2), (1, 2)] if dim == 3 else []):
        Om = np.zeros((dim, dim))
        Om[i, j], Om[j, i] = 1.0, -1.0
        ox = (Om @ X).ravel()
        og = (Om @ g.reshape(dim, -1)).ravel()
        assert abs(g @ ox) < 1e-12 * gs * np.linalg.norm(x)
        assert np.allclose(pb.hvp_full(x, ox), og, atol=1e-11 * np.abs(g).max())


@pytest.mark.parametrize("dim,n,p,nq", [(2, 2, 2, 4), (3, 1, 2, 4)])
def test_constant_target(dim, n, p, nq):
    pb, x = _mesh(dim, n, p, nq)
    F = pb.energy(x)
    g = pb.gradient_full(x)
    c = 1.7
    pbc = oracle.Problem.box(dim, n, p, nq, W=c * np.eye(dim), constrain=None)
    assert abs(pbc.energy(x) - c ** dim * F) < 1e-13 * F
    assert np.allclose(pbc.gradient_full(x), c ** dim * g, atol=1e-13 * np.abs(g).max())
    Q = _rotation(dim, 3)
    pbr = oracle.Problem.box(dim, n, p, nq, W=Q, constrain=None)
    assert abs(pbr.energy(x) - F) < 1e-13 * F
    v = np.random.default_rng(9).standard_normal(x.size)
    assert np.allclose(pbr.hvp_full(x, v), pb.hvp_full(x, v), atol=1e-12 * np.abs(pb.hvp_full(x, v)).max())


def test_constrained_forms():
    pb, x = _mesh(3, 2, 2, 4, constrain="boundary")
    ess = pb.ess
    v = np.random.default_rng(10).standard_normal(x.size)
    y = pb.hvp(x, v)
    assert np.array_equal(y[ess], v[ess])
    vf = v.copy()
    vf[ess] = 0
    assert np.allclose(y[~ess], pb.hvp_full(x, vf)[~ess], rtol=0, atol=0)
    assert np.all(pb.gradient(x)[ess] == 0)
    assert np.all(pb.diag(x)[ess] == 1)


def test_inverted_element_detected():
    pb = oracle.Problem.box(2, 2, 1, 2, constrain=None)
    x = _uniform(2, 2, 1)
    X = x.reshape(2, -1)
    X[0, 4] = 1.3  # drag the centre node past the right boundary
    assert pb.min_det(X.ravel()) < 0
    assert pb.energy(X.ravel()) == np.inf
    with pytest.raises(FloatingPointError):
        pb.gradient_full(X.ravel())
