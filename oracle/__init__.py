"""Plain FP64 CPU oracle of the PA-TMOP hot path.

TEST INFRASTRUCTURE.  Only ``tests/``, the smoke check in ``__graft_entry__``
and the CPU-baseline leg of ``bench.py`` may import this package.  The
product library (``paper_2205_12721_amd``) never imports it, and the two share
no code: the oracle's per-element arithmetic lives in ``tmop_oracle.c``
(direct O(N_q N_p) sums, no sum factorization), its bases and quadrature in
``basis.py``, its structured-box numbering in ``mesh.py`` and its MINRES and
Newton loops in ``solver.py``.

Parity pins: see ``tests/test_oracle_*.py``.  Every function here is pinned
by at least one of closed forms, invariants, finite differences, brute force
or values printed in the paper.
"""
import ctypes
import os
import subprocess
import functools

import numpy as np

from . import basis
from . import mesh

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tmop_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force=False):
    """Compile liboracle.so with gcc (-O2, OpenMP).  A library named by the
    environment variable TMOP_ORACLE_LIB (the sanitizer test's build of the
    same source) is used as it is."""
    alt = os.environ.get("TMOP_ORACLE_LIB")
    if alt:
        return alt
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("metric", ctypes.c_int),
        ("ne", ctypes.c_int),
        ("np", ctypes.c_int),
        ("nq", ctypes.c_int),
        ("nx", ctypes.c_int),
        ("e2n", ctypes.POINTER(ctypes.c_int32)),
        ("wq", ctypes.POINTER(ctypes.c_double)),
        ("dphi", ctypes.POINTER(ctypes.c_double)),
        ("Winv", ctypes.c_double * 9),
        ("detW", ctypes.c_double),
        ("phi", ctypes.POINTER(ctypes.c_double)),
        ("x0", ctypes.POINTER(ctypes.c_double)),
        ("lim_coef", ctypes.c_double),
        ("lim_delta", ctypes.c_double),
    ]


_D = ctypes.POINTER(ctypes.c_double)


@functools.lru_cache(maxsize=1)
def _lib():
    lib = ctypes.CDLL(build())
    P = ctypes.POINTER(_Problem)
    lib.oracle_metric.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D]
    lib.oracle_metric.restype = ctypes.c_int
    lib.oracle_jacobians.argtypes = [P, _D, _D]
    lib.oracle_min_det.argtypes = [P, _D]
    lib.oracle_min_det.restype = ctypes.c_double
    lib.oracle_energy.argtypes = [P, _D, ctypes.POINTER(ctypes.c_int)]
    lib.oracle_energy.restype = ctypes.c_double
    for name in ("oracle_gradient", "oracle_hessian_diag"):
        getattr(lib, name).argtypes = [P, _D, _D]
        getattr(lib, name).restype = ctypes.c_int
    lib.oracle_hessian_apply.argtypes = [P, _D, _D, _D]
    lib.oracle_hessian_apply.restype = ctypes.c_int
    lib.oracle_element_hessian.argtypes = [P, _D, ctypes.c_int, _D]
    lib.oracle_element_hessian.restype = ctypes.c_int
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    return lib


def _dp(a):
    return a.ctypes.data_as(_D)


def set_num_threads(n):
    _lib().oracle_set_num_threads(int(n))


def num_threads():
    return int(_lib().oracle_num_threads())


def metric(dim, metric_id, T):
    """(mu, dmu/dT, d2mu/dT2) at one matrix T; None if det T <= 0."""
    T = np.ascontiguousarray(T, dtype=np.float64).reshape(dim, dim)
    mu = np.zeros(1)
    dmu = np.zeros(dim * dim)
    d2mu = np.zeros(dim ** 4)
    rc = _lib().oracle_metric(dim, metric_id, _dp(T), _dp(mu), _dp(dmu), _dp(d2mu))
    if rc < 0:
        raise ValueError("unknown metric %d for dim %d" % (metric_id, dim))
    if rc == 0:
        return None
    return mu[0], dmu.reshape(dim, dim), d2mu.reshape(dim, dim, dim, dim)


class Problem:
    """One TMOP problem: mesh topology, discretisation and target.

    ``e2n``   int32 (E, N_p) global node index per local lexicographic node
    ``nx``    number of global nodes; vectors are float64 SoA of length dim*nx
    ``W``     constant target matrix (dim x dim); identity is the ideal element
    ``ess``   bool/uint8 mask of length dim*nx (True = fixed DoF) or None
    """

    def __init__(self, dim, p, nq1d, e2n, nx, metric_id=None, W=None, ess=None, quad="gl"):
        self.dim = dim
        self.p = p
        self.nq1d = nq1d
        self.quad = quad
        self.metric = metric_id if metric_id is not None else (2 if dim == 2 else 303)
        self.e2n = np.ascontiguousarray(e2n, dtype=np.int32)
        self.ne, self.npe = self.e2n.shape
        self.nx = int(nx)
        self.ndof = dim * self.nx
        self.wq, dphi, phi = _dense_tables(dim, p, nq1d, quad)
        self.dphi = np.ascontiguousarray(dphi)
        self.phi = np.ascontiguousarray(phi)
        self.nqe = len(self.wq)
        self.W = np.eye(dim) if W is None else np.asarray(W, dtype=np.float64).reshape(dim, dim)
        Winv = np.linalg.inv(self.W)
        self._pb = _Problem()
        self._pb.dim = dim
        self._pb.metric = self.metric
        self._pb.ne = self.ne
        self._pb.np = self.npe
        self._pb.nq = self.nqe
        self._pb.nx = self.nx
        self._pb.e2n = self.e2n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        self._pb.wq = _dp(self.wq)
        self._pb.dphi = _dp(self.dphi)
        wi = np.zeros(9)
        wi[: dim * dim] = Winv.ravel()
        for k in range(9):
            self._pb.Winv[k] = wi[k]
        self._pb.detW = float(np.linalg.det(self.W))
        self._pb.phi = _dp(self.phi)
        self.lim_x0 = None
        self._pb.x0 = None
        self._pb.lim_coef = 0.0
        self._pb.lim_delta = 1.0
        self.ess = None if ess is None else np.asarray(ess, dtype=bool).ravel()
        if self.npe != (p + 1) ** dim:
            raise ValueError("e2n width does not match (p+1)^dim")

    def set_limiting(self, x0, coef=1.0, delta=1.0):
        """Add the limiting term coef * sum_E int |x - x0|^2 / delta^2 of eq.
        eq_F_full (xi(y, delta) = |y|^2 / delta^2); x0=None removes it."""
        if x0 is None:
            self.lim_x0 = None
            self._pb.x0 = None
            self._pb.lim_coef = 0.0
            return
        if not delta > 0:
            raise ValueError("delta must be positive")
        self.lim_x0 = np.array(self._x(x0), dtype=np.float64, copy=True)
        self._pb.x0 = _dp(self.lim_x0)
        self._pb.lim_coef = float(coef)
        self._pb.lim_delta = float(delta)

    @classmethod
    def box(cls, dim, n, p, nq1d, metric_id=None, W=None, constrain="boundary", quad="gl"):
        """Structured box [0,1]^dim with n (int or tuple) elements per side."""
        ns = (n,) * dim if np.isscalar(n) else tuple(n)
        e2n, nx = mesh.box_topology(dim, ns, p)
        ess = None
        if constrain == "boundary":
            ess = mesh.box_boundary_mask(dim, ns, p)
        elif constrain not in (None, "none"):
            raise ValueError(constrain)
        pb = cls(dim, p, nq1d, e2n, nx, metric_id=metric_id, W=W, ess=ess, quad=quad)
        pb.shape = ns
        return pb

    # -- evaluations (unconstrained) -----------------------------------------
    def _x(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64).ravel()
        if x.size != self.ndof:
            raise ValueError("vector has %d entries, expected %d" % (x.size, self.ndof))
        return x

    def jacobians(self, x):
        x = self._x(x)
        A = np.zeros((self.ne, self.nqe, self.dim, self.dim))
        _lib().oracle_jacobians(ctypes.byref(self._pb), _dp(x), _dp(A))
        return A

    def min_det(self, x):
        return float(_lib().oracle_min_det(ctypes.byref(self._pb), _dp(self._x(x))))

    def energy(self, x):
        bad = ctypes.c_int(0)
        F = _lib().oracle_energy(ctypes.byref(self._pb), _dp(self._x(x)), ctypes.byref(bad))
        return float(F)

    def gradient_full(self, x):
        g = np.zeros(self.ndof)
        ok = _lib().oracle_gradient(ctypes.byref(self._pb), _dp(self._x(x)), _dp(g))
        if not ok:
            raise FloatingPointError("det T <= 0 at a quadrature point")
        return g

    def hvp_full(self, x, v):
        y = np.zeros(self.ndof)
        ok = _lib().oracle_hessian_apply(ctypes.byref(self._pb), _dp(self._x(x)),
                                         _dp(self._x(v)), _dp(y))
        if not ok:
            raise FloatingPointError("det T <= 0 at a quadrature point")
        return y

    def diag_full(self, x):
        d = np.zeros(self.ndof)
        ok = _lib().oracle_hessian_diag(ctypes.byref(self._pb), _dp(self._x(x)), _dp(d))
        if not ok:
            raise FloatingPointError("det T <= 0 at a quadrature point")
        return d

    def element_hessian(self, x, e):
        n = self.dim * self.npe
        H = np.zeros((n, n))
        ok = _lib().oracle_element_hessian(ctypes.byref(self._pb), _dp(self._x(x)), int(e), _dp(H))
        if not ok:
            raise FloatingPointError("det T <= 0 at a quadrature point")
        return H

    def dense_hessian(self, x):
        """Fully assembled global Hessian (tiny meshes only), unconstrained."""
        H = np.zeros((self.ndof, self.ndof))
        d, npe = self.dim, self.npe
        for e in range(self.ne):
            He = self.element_hessian(x, e)
            idx = np.concatenate([a * self.nx + self.e2n[e] for a in range(d)])
            H[np.ix_(idx, idx)] += He
        return H

    # -- constrained forms (fixed DoFs) --------------------------------------
    def gradient(self, x):
        """g_c = P g: gradient with fixed DoFs zeroed."""
        g = self.gradient_full(x)
        if self.ess is not None:
            g[self.ess] = 0.0
        return g

    def hvp(self, x, v):
        """H_c v = P H P v + (I - P) v."""
        v = self._x(v)
        if self.ess is None:
            return self.hvp_full(x, v)
        vf = v.copy()
        vf[self.ess] = 0.0
        y = self.hvp_full(x, vf)
        y[self.ess] = v[self.ess]
        return y

    def diag(self, x):
        """Diagonal of H_c: fixed entries are 1."""
        d = self.diag_full(x)
        if self.ess is not None:
            d[self.ess] = 1.0
        return d


@functools.lru_cache(maxsize=32)
def _dense_tables(dim, p, nq1d, quad="gl"):
    wq, dphi = basis.dense_tables(dim, p, nq1d, quad)
    phi = basis.dense_values(dim, p, nq1d, quad)
    for a in (wq, dphi, phi):
        a.setflags(write=False)
    return wq, dphi, phi


from .solver import minres, newton_solve  # noqa: E402,F401


def restrict_to_nodes(pb, nodes):
    """Sub-problem holding only the elements that touch ``nodes`` (global node ids).

    Energy-derivative entries at those nodes depend only on these elements, so
    the sub-problem's gradient, Hessian action and diagonal equal the full
    problem's there; used to sample large meshes entry by entry.
    """
    nodes = np.asarray(nodes)
    keep = np.isin(pb.e2n, nodes).any(axis=1)
    sub = Problem(pb.dim, pb.p, pb.nq1d, pb.e2n[keep], pb.nx, metric_id=pb.metric, W=pb.W,
                  ess=pb.ess, quad=pb.quad)
    if pb.lim_x0 is not None:
        sub.set_limiting(pb.lim_x0, pb._pb.lim_coef, pb._pb.lim_delta)
    return sub
