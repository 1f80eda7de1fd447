"""Pins of the oracle's quality metrics and their derivatives.

Shape metrics mu_2 = |T|^2/(2 tau) - 1 (Sec. 2.2) and
mu_303 = |T|^2/(3 tau^(2/3)) - 1 (Sec. 4.1); size metric mu_55 = (tau - 1)^2 and
shape+size metrics mu_7 = |T - T^{-t}|^2, mu_9 = tau |T - T^{-t}|^2 (Sec. 2.2).
Values are pinned to hand-derived closed forms (golden file), to the metric
properties (non-negativity; zero exactly at similarities for shape metrics,
at rotations for shape+size metrics, at unit determinant for the size metric;
rotation invariance; scale invariance of shape metrics), and the closed-form
derivatives to complex-step differentiation of the metric *definition*
written below (only mu itself is written here, not its derivatives).
"""
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALL = [(2, 2), (3, 303), (2, 7), (2, 9), (2, 55), (3, 55)]


def mu_def(dim, metric, T):
    """The metric definition (works for complex T, used for complex-step)."""
    I1 = (T * T).sum()
    tau = T[0, 0] * T[1, 1] - T[0, 1] * T[1, 0] if dim == 2 else (
        T[0, 0] * (T[1, 1] * T[2, 2] - T[1, 2] * T[2, 1])
        - T[0, 1] * (T[1, 0] * T[2, 2] - T[1, 2] * T[2, 0])
        + T[0, 2] * (T[1, 0] * T[2, 1] - T[1, 1] * T[2, 0]))
    if metric == 2:
        return I1 / (2 * tau) - 1
    if metric == 303:
        return I1 / (3 * tau ** (2.0 / 3.0)) - 1
    if metric == 55:
        return (tau - 1) ** 2
    # 2D inverse transpose written out: [[a, b], [c, d]]^{-t} = [[d, -c], [-b, a]] / tau
    Tit = np.array([[T[1, 1], -T[1, 0]], [-T[0, 1], T[0, 0]]]) / tau
    m7 = ((T - Tit) * (T - Tit)).sum()
    return m7 if metric == 7 else tau * m7


def _rand_T(rng, dim):
    while True:
        T = np.eye(dim) + 0.4 * rng.standard_normal((dim, dim))
        if np.linalg.det(T) > 0.2:
            return T


def _golden():
    rows = []
    with open(os.path.join(GOLDEN, "metric_values.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            dim, metric = int(parts[0]), int(parts[1])
            T = np.array([float(v) for v in parts[2:2 + dim * dim]]).reshape(dim, dim)
            expr = parts[2 + dim * dim]
            assert set(expr) <= set("0123456789.+-*/() ")
            rows.append((dim, metric, T, eval(expr)))
    return rows


@pytest.mark.parametrize("dim,metric,T,expected", _golden())
def test_metric_closed_forms(dim, metric, T, expected):
    mu, _, _ = oracle.metric(dim, metric, T)
    assert abs(mu - expected) < 1e-14


SHAPE = {2, 303}


def _rotation(rng, dim):
    Q, _ = np.linalg.qr(rng.standard_normal((dim, dim)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    return Q


@pytest.mark.parametrize("dim,metric", ALL)
def test_metric_nonnegative_and_zero_at_optimum(dim, metric):
    rng = np.random.default_rng(0)
    for _ in range(50):
        T = _rand_T(rng, dim)
        mu, _, _ = oracle.metric(dim, metric, T)
        assert mu >= -1e-15
    for _ in range(10):
        Q = _rotation(rng, dim)
        # shape metrics vanish at every similarity, the others at rotations
        c = rng.uniform(0.1, 5.0) if metric in SHAPE else 1.0
        mu, dmu, _ = oracle.metric(dim, metric, c * Q)
        assert abs(mu) < 1e-14
        assert np.abs(dmu).max() < 1e-13 * max(1.0, 1.0 / c)
        if metric in SHAPE:
            continue
        # away from the optimum they are positive (scaled rotation)
        mu, _, _ = oracle.metric(dim, metric, 1.3 * Q)
        assert mu > 1e-3
    if metric == 55:
        # the size metric vanishes at any unit-determinant matrix
        S = np.eye(dim)
        S[0, 1] = 0.7
        assert abs(oracle.metric(dim, metric, S)[0]) < 1e-14


@pytest.mark.parametrize("dim,metric", ALL)
def test_metric_invariances(dim, metric):
    rng = np.random.default_rng(1)
    for _ in range(10):
        T = _rand_T(rng, dim)
        Q = _rotation(rng, dim)
        mu0 = oracle.metric(dim, metric, T)[0]
        assert abs(oracle.metric(dim, metric, Q @ T)[0] - mu0) < 1e-13 * max(1.0, mu0)
        assert abs(oracle.metric(dim, metric, T @ Q)[0] - mu0) < 1e-13 * max(1.0, mu0)
        if metric in SHAPE:
            assert abs(oracle.metric(dim, metric, 3.7 * T)[0] - mu0) < 1e-13


@pytest.mark.parametrize("dim,metric", ALL)
def test_first_derivative_complex_step(dim, metric):
    rng = np.random.default_rng(2)
    h = 1e-30
    for _ in range(10):
        T = _rand_T(rng, dim)
        mu, dmu, _ = oracle.metric(dim, metric, T)
        assert abs(mu - mu_def(dim, metric, T)) < 1e-14 * max(1.0, abs(mu))
        for r in range(dim * dim):
            E = np.zeros(dim * dim, dtype=complex)
            E[r] = 1j * h
            val = mu_def(dim, metric, T.astype(complex) + E.reshape(dim, dim))
            assert abs(val.imag / h - dmu.ravel()[r]) < 1e-13 * max(1.0, abs(dmu.ravel()[r]))


@pytest.mark.parametrize("dim,metric", ALL)
def test_second_derivative_complex_step(dim, metric):
    """d2mu/dT_r dT_s = Im[mu(T + ih e_r + d e_s) - mu(T + ih e_r - d e_s)]/(2 h d) + O(d^2)."""
    rng = np.random.default_rng(3)
    h, dd = 1e-30, 1e-5
    for _ in range(4):
        T = _rand_T(rng, dim)
        _, _, d2 = oracle.metric(dim, metric, T)
        d2 = d2.reshape(dim * dim, dim * dim)
        assert np.allclose(d2, d2.T, atol=1e-14 * max(1.0, np.abs(d2).max()), rtol=0)
        for r in range(dim * dim):
            for s in range(dim * dim):
                Er = np.zeros(dim * dim, dtype=complex)
                Er[r] = 1j * h
                Es = np.zeros(dim * dim)
                Es[s] = dd
                Tc = T.astype(complex)
                vp = mu_def(dim, metric, Tc + (Er + Es).reshape(dim, dim))
                vm = mu_def(dim, metric, Tc + (Er - Es).reshape(dim, dim))
                est = (vp.imag - vm.imag) / (2 * h * dd)
                assert abs(est - d2[r, s]) < 1e-8 * max(1.0, abs(d2[r, s]))


def test_metric_invalid_and_unknown():
    assert oracle.metric(2, 2, np.array([[1.0, 0], [0, -1.0]])) is None
    assert oracle.metric(3, 303, np.zeros((3, 3))) is None
    with pytest.raises(ValueError):
        oracle.metric(2, 303, np.eye(2))
    with pytest.raises(ValueError):
        oracle.metric(3, 7, np.eye(3))
