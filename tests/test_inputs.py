"""CPU checks of the seeded input recipes (no method arithmetic involved)."""
import os

import numpy as np
import pytest

from oracle import basis
from paper_2205_12721_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kershaw_rows():
    rows = []
    with open(os.path.join(GOLDEN, "kershaw_points.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            x, t, e, expr = line.split()
            assert set(expr) <= set("0123456789.+-*/() ")
            rows.append((float(x), float(t), float(e), eval(expr)))
    return rows


@pytest.mark.parametrize("x,t,eps,expected", _kershaw_rows())
def test_kershaw_hand_values(x, t, eps, expected):
    v = inputs.kershaw_map(np.array([x]), np.array([t]), eps)[0]
    assert abs(v - expected) < 1e-14


def test_kershaw_blend_weight():
    """The right-end weight s(x): 0 on the first layer, 1 on the last, 1 at x = 1/3
    and 0 at x = 2/3 (the third and fourth layers fall from 1 to 0 together),
    continuous, and a quintic smoothstep across the second layer."""
    s = inputs.kershaw_blend
    assert np.all(s(np.linspace(0.0, 1.0 / 6.0, 11)) == 0.0)
    assert np.allclose(s(np.linspace(5.0 / 6.0, 1.0, 11)), 1.0, atol=1e-15)
    assert abs(s(1.0 / 3.0) - 1.0) < 1e-15 and abs(s(2.0 / 3.0)) < 1e-15
    assert abs(s(0.5) - 0.5) < 1e-15          # middle of the falling double layer
    u = 0.3
    assert abs(s((1.0 + u) / 6.0) - (10 * u ** 3 - 15 * u ** 4 + 6 * u ** 5)) < 1e-15
    xs = np.linspace(0.0, 1.0, 6001)
    assert np.abs(np.diff(s(xs))).max() < 3e-3  # continuous (step 1/6000)


def test_kershaw_properties():
    x = np.linspace(0, 1, 61)
    t = np.linspace(0, 1, 41)
    X, T = np.meshgrid(x, t, indexing="ij")
    assert np.allclose(inputs.kershaw_map(X, T, 1.0), T, atol=1e-15)
    K = inputs.kershaw_map(X, T, 0.3)
    assert np.allclose(K[:, 0], 0) and np.allclose(K[:, -1], 1)
    assert np.all(np.diff(K, axis=1) > 0)  # monotone in t: no folding
    xk = inputs.kershaw_nodes((6, 2, 2), 2, basis.gll_nodes(2))
    xu = inputs.uniform_nodes((6, 2, 2), 2, basis.gll_nodes(2))
    nx = xu.size // 3
    assert np.array_equal(xk[:nx], xu[:nx])
    m = inputs.sliding_mask((6, 2, 2), 2).astype(bool)
    # boundary nodes move only tangentially: fixed components keep their value
    assert np.allclose(xk[m], xu[m], atol=1e-15)


def test_perturbed_box_recipes():
    nodes = basis.gll_nodes(3)
    x, info = inputs.perturbed_box(3, (3, 2, 2), 3, nodes, 5, recipe="smooth", amp=0.05)
    xu = inputs.uniform_nodes((3, 2, 2), 3, nodes)
    bm = inputs.boundary_component_mask((3, 2, 2), 3).ravel()
    assert np.allclose(x[bm], xu[bm], atol=1e-15)  # no normal motion on faces
    assert np.abs(x - xu).max() > 0
    x2, _ = inputs.perturbed_box(3, (3, 2, 2), 3, nodes, 5, recipe="smooth", amp=0.05)
    assert np.array_equal(x, x2)  # seeded
    xp, _ = inputs.perturbed_box(2, (4, 4), 2, basis.gll_nodes(2), 1, recipe="pin", amp=0.1)
    xu2 = inputs.uniform_nodes((4, 4), 2, basis.gll_nodes(2))
    anyb = np.any(inputs.boundary_component_mask((4, 4), 2), axis=0)
    assert np.allclose(xp.reshape(2, -1)[:, anyb], xu2.reshape(2, -1)[:, anyb])


def test_batch_and_serving_specs():
    sp = inputs.batch_specs(256, seed=5)
    assert len(sp) == 256
    assert all(2 <= s["n"] <= 16 and 1 <= s["p"] <= 4 and s["nq"] == s["p"] + 2 for s in sp)
    assert sp == inputs.batch_specs(256, seed=5)
    st = inputs.serving_stream(100.0, count=300, seed=6)
    t = np.array([r["t_arrive"] for r in st])
    assert np.all(np.diff(t) > 0)
    assert 0.5 < len(st) / t[-1] / 100.0 < 2.0
    assert {r["dim"] for r in st} == {2, 3}
