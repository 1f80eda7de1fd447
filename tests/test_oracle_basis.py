"""Pins of the oracle's 1D bases, quadrature, tables and numbering.

Everything here is checked against closed forms, exactness properties and the
problem sizes printed in the paper (Sec. 4.1, Table tab_kershaw_baseline (a)).
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import basis, mesh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_gll_closed_forms():
    assert np.allclose(basis.gll_nodes(1), [0.0, 1.0], atol=0, rtol=0)
    assert np.allclose(basis.gll_nodes(2), [0.0, 0.5, 1.0], atol=1e-16)
    a = 1.0 / math.sqrt(5.0)
    assert np.allclose(basis.gll_nodes(3), [0, (1 - a) / 2, (1 + a) / 2, 1], atol=1e-15)
    b = math.sqrt(3.0 / 7.0)
    assert np.allclose(basis.gll_nodes(4), [0, (1 - b) / 2, 0.5, (1 + b) / 2, 1], atol=1e-15)


@pytest.mark.parametrize("n", range(1, 10))
def test_gauss_legendre_exactness(n):
    x, w = basis.gl_rule(n)
    assert abs(w.sum() - 1.0) < 1e-15
    for k in range(2 * n):
        assert abs((w * x ** k).sum() - 1.0 / (k + 1)) < 1e-14
    # not exact one degree higher
    assert abs((w * x ** (2 * n)).sum() - 1.0 / (2 * n + 1)) > 1e-13


def test_gauss_legendre_two_points():
    x, w = basis.gl_rule(2)
    r = 1.0 / (2.0 * math.sqrt(3.0))
    assert np.allclose(x, [0.5 - r, 0.5 + r], atol=1e-16)
    assert np.allclose(w, [0.5, 0.5], atol=1e-16)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
def test_lagrange_properties(p):
    nodes = basis.gll_nodes(p)
    L, dL = basis.lagrange(nodes, nodes)
    assert np.allclose(L, np.eye(p + 1), atol=1e-14)
    pts = np.linspace(-0.1, 1.1, 23)
    L, dL = basis.lagrange(nodes, pts)
    assert np.allclose(L.sum(axis=1), 1.0, atol=1e-13)
    assert np.allclose(dL.sum(axis=1), 0.0, atol=1e-11)
    # exact reproduction of x^k and its derivative for k <= p
    for k in range(p + 1):
        assert np.allclose(L @ nodes ** k, pts ** k, atol=1e-12)
        dk = k * pts ** (k - 1) if k > 0 else np.zeros_like(pts)
        assert np.allclose(dL @ nodes ** k, dk, atol=1e-10)


@pytest.mark.parametrize("p,nq", [(1, 3), (2, 4), (3, 5), (4, 6)])
def test_1d_tables(p, nq):
    B, G = basis.tables_1d(p, nq)
    assert B.shape == (nq, p + 1) and G.shape == (nq, p + 1)
    assert np.allclose(B.sum(axis=1), 1.0, atol=1e-14)
    assert np.allclose(G.sum(axis=1), 0.0, atol=1e-12)


@pytest.mark.parametrize("dim,p,nq", [(2, 2, 4), (3, 1, 3), (3, 3, 5)])
def test_dense_tables_reproduce_linears(dim, p, nq):
    """sum_i xbar_k(node i) dwbar_i/dxbar_b = delta_kb at every point (affine exactness)."""
    wq, dphi = basis.dense_tables(dim, p, nq)
    assert abs(wq.sum() - 1.0) < 1e-14
    nodes = basis.gll_nodes(p)
    ni = p + 1
    for k in range(dim):
        coord = np.array([nodes[(i // ni ** k) % ni] for i in range(ni ** dim)])
        for b in range(dim):
            assert np.allclose(dphi[b] @ coord, 1.0 if k == b else 0.0, atol=1e-13)


def _golden_counts():
    rows = []
    with open(os.path.join(GOLDEN, "kershaw_counts.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p, n = line.split()
            rows.append((int(p), int(n)))
    return rows


@pytest.mark.parametrize("p,dofs", _golden_counts())
def test_dof_counts_match_paper(p, dofs):
    """Unique DoFs of the 24^3 mesh printed in Sec. 4.1, Table (a)."""
    assert mesh.dof_count(3, 24, p) == dofs
    if p <= 2:
        e2n, nx = mesh.box_topology(3, (24, 24, 24), p)
        assert 3 * nx == dofs
        assert len(np.unique(e2n)) == nx


def test_qp_per_core_match_paper():
    """N_e N_q / #cores with N_q = 9^3 (Sec. 4.1, Table (a))."""
    ne, nq = 24 ** 3, 9 ** 3
    assert ne * nq // 36 == 279936
    assert ne * nq // 4 == 2519424


def test_box_topology_small():
    e2n, nx = mesh.box_topology(2, (2, 1), 1)
    # 3 x 2 grid of nodes, first axis fastest
    assert nx == 6
    assert e2n.tolist() == [[0, 1, 3, 4], [1, 2, 4, 5]]
    e2n, nx = mesh.box_topology(3, (1, 1, 2), 2)
    assert nx == 3 * 3 * 5
    # element 1 starts at grid z = 2
    assert e2n[1, 0] == 2 * 9
    assert e2n[1, -1] == nx - 1


def test_boundary_mask():
    m = mesh.box_boundary_mask(2, (2, 2), 1)
    # 3x3 grid: only the centre node is interior
    one = m[:9]
    assert one.sum() == 8 and not one[4]
    assert np.array_equal(m[9:], one)


# Gauss-Lobatto-Legendre rule on [0,1]: textbook closed forms for n = 2, 3, 4
# (trapezoid, Simpson, and the four-point Lobatto rule with interior nodes at
# (1 -+ 1/sqrt(5))/2 and weights 1/12, 5/12), end points included, exact for
# polynomials of degree <= 2n-3 and not for x^(2n-2).
def test_gauss_lobatto_closed_forms():
    x, w = basis.gll_rule(2)
    assert np.allclose(x, [0.0, 1.0], atol=1e-16) and np.allclose(w, [0.5, 0.5], atol=1e-16)
    x, w = basis.gll_rule(3)
    assert np.allclose(x, [0.0, 0.5, 1.0], atol=1e-16)
    assert np.allclose(w, [1 / 6, 2 / 3, 1 / 6], atol=1e-15)
    x, w = basis.gll_rule(4)
    r = 1.0 / np.sqrt(5.0)
    assert np.allclose(x, [0.0, (1 - r) / 2, (1 + r) / 2, 1.0], atol=1e-15)
    assert np.allclose(w, [1 / 12, 5 / 12, 5 / 12, 1 / 12], atol=1e-15)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 7, 9, 10])
def test_gauss_lobatto_exactness(n):
    x, w = basis.gll_rule(n)
    assert x[0] == 0.0 and x[-1] == 1.0
    assert abs(w.sum() - 1.0) < 1e-14 and (w > 0).all()
    for k in range(2 * n - 2):
        assert abs((w * x ** k).sum() - 1.0 / (k + 1)) < 1e-13
    k = 2 * n - 2
    assert abs((w * x ** k).sum() - 1.0 / (k + 1)) > 1e-12


def test_quad_rule_names():
    assert np.array_equal(basis.quad_rule(5, "gl")[0], basis.gl_rule(5)[0])
    assert np.array_equal(basis.quad_rule(5, "gll")[1], basis.gll_rule(5)[1])
    with pytest.raises(ValueError):
        basis.quad_rule(5, "uniform")
    with pytest.raises(ValueError):
        basis.gll_rule(1)
