"""Pins of the oracle's quality metrics and their derivatives.

mu_2 = |T|^2/(2 tau) - 1 (Sec. 2.2) and mu_303 = |T|^2/(3 tau^(2/3)) - 1
(Sec. 4.1).  Values are pinned to hand-derived closed forms (golden file),
to the metric properties (non-negativity, zero exactly at similarities,
rotation and scale invariance), and the closed-form derivatives to
complex-step differentiation of the metric *definition* written below
(only mu itself is written here, not its derivatives).
"""
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def mu_def(dim, metric, T):
    """The metric definition (works for complex T, used for complex-step)."""
    I1 = (T * T).sum()
    tau = T[0, 0] * T[1, 1] - T[0, 1] * T[1, 0] if dim == 2 else (
        T[0, 0] * (T[1, 1] * T[2, 2] - T[1, 2] * T[2, 1])
        - T[0, 1] * (T[1, 0] * T[2, 2] - T[1, 2] * T[2, 0])
        + T[0, 2] * (T[1, 0] * T[2, 1] - T[1, 1] * T[2, 0]))
    if metric == 2:
        return I1 / (2 * tau) - 1
    return I1 / (3 * tau ** (2.0 / 3.0)) - 1


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


@pytest.mark.parametrize("dim,metric", [(2, 2), (3, 303)])
def test_metric_nonnegative_and_zero_at_similarity(dim, metric):
    rng = np.random.default_rng(0)
    for _ in range(50):
        T = _rand_T(rng, dim)
        mu, _, _ = oracle.metric(dim, metric, T)
        assert mu >= -1e-15
    for _ in range(10):
        Q, _ = np.linalg.qr(rng.standard_normal((dim, dim)))
        if np.linalg.det(Q) < 0:
            Q[:, 0] *= -1
        c = rng.uniform(0.1, 5.0)
        mu, dmu, _ = oracle.metric(dim, metric, c * Q)
        assert abs(mu) < 1e-14
        assert np.abs(dmu).max() < 1e-13 * max(1.0, 1.0 / c)


@pytest.mark.parametrize("dim,metric", [(2, 2), (3, 303)])
def test_metric_invariances(dim, metric):
    rng = np.random.default_rng(1)
    for _ in range(10):
        T = _rand_T(rng, dim)
        Q, _ = np.linalg.qr(rng.standard_normal((dim, dim)))
        if np.linalg.det(Q) < 0:
            Q[:, 0] *= -1
        mu0 = oracle.metric(dim, metric, T)[0]
        assert abs(oracle.metric(dim, metric, Q @ T)[0] - mu0) < 1e-13
        assert abs(oracle.metric(dim, metric, T @ Q)[0] - mu0) < 1e-13
        assert abs(oracle.metric(dim, metric, 3.7 * T)[0] - mu0) < 1e-13


@pytest.mark.parametrize("dim,metric", [(2, 2), (3, 303)])
def test_first_derivative_complex_step(dim, metric):
    rng = np.random.default_rng(2)
    h = 1e-30
    for _ in range(10):
        T = _rand_T(rng, dim)
        mu, dmu, _ = oracle.metric(dim, metric, T)
        assert abs(mu - mu_def(dim, metric, T)) < 1e-14
        for r in range(dim * dim):
            E = np.zeros(dim * dim, dtype=complex)
            E[r] = 1j * h
            val = mu_def(dim, metric, T.astype(complex) + E.reshape(dim, dim))
            assert abs(val.imag / h - dmu.ravel()[r]) < 1e-13 * max(1.0, abs(dmu.ravel()[r]))


@pytest.mark.parametrize("dim,metric", [(2, 2), (3, 303)])
def test_second_derivative_complex_step(dim, metric):
    """d2mu/dT_r dT_s = Im[mu(T + ih e_r + d e_s) - mu(T + ih e_r - d e_s)]/(2 h d) + O(d^2)."""
    rng = np.random.default_rng(3)
    h, dd = 1e-30, 1e-5
    for _ in range(4):
        T = _rand_T(rng, dim)
        _, _, d2 = oracle.metric(dim, metric, T)
        d2 = d2.reshape(dim * dim, dim * dim)
        assert np.allclose(d2, d2.T, atol=1e-14, rtol=0)
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
