"""Python binding of libtmop_hip.so (argument marshalling only).

Every computation runs in the HIP library; this module converts torch
tensors (device memory owned by the caller) to pointers, passes the current
torch stream, and turns status codes into exceptions.  There is no fallback:
if the library is missing or no GPU is present, the calls raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtmop_hip.so")

TMOP_FP64, TMOP_MIXED = 0, 1
HESS_TENSOR, HESS_COMPACT = 0, 1
ESS_BOUNDARY, ESS_NONE, ESS_MASK = 0, 1, 2
EVAL_ENERGY, EVAL_GRADIENT, EVAL_SETUP, EVAL_APPLY, EVAL_DIAG = 0, 1, 2, 3, 4

STATUS = {
    0: "OK", 1: "ERR_INVALID_ARG", 2: "ERR_UNSUPPORTED", 3: "ERR_INVERTED",
    4: "ERR_LINESEARCH", 5: "ERR_NOT_CONVERGED", 6: "ERR_NONFINITE", 7: "ERR_OOM",
    8: "ERR_BUDGET", 9: "ERR_BUSY", 10: "ERR_HIP", 11: "ERR_STATE",
}
OK, ERR_INVERTED, ERR_LINESEARCH, ERR_NOT_CONVERGED, ERR_NONFINITE = 0, 3, 4, 5, 6
ERR_BUDGET, ERR_BUSY = 8, 9


class TmopError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class MeshDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("order_p", ctypes.c_int), ("nx", ctypes.c_int),
                ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("num_elems", ctypes.c_int),
                ("num_nodes", ctypes.c_int), ("elem_to_node", ctypes.c_void_p),
                ("ess_mode", ctypes.c_int), ("ess_mask", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("metric", ctypes.c_int), ("nq1d", ctypes.c_int), ("has_W", ctypes.c_int),
                ("W", ctypes.c_double * 9), ("precision", ctypes.c_int),
                ("hess_storage", ctypes.c_int), ("quad_rule", ctypes.c_int)]


QUAD_RULES = {"gl": 0, "gll": 1}   # TMOP_QUAD_GL, TMOP_QUAD_GLL
SWEEPS = {"pencil": 0, "mfma": 1}  # TMOP_SWEEPS_PENCIL, TMOP_SWEEPS_MFMA


class SolveParams(ctypes.Structure):
    _fields_ = [("rel_grad_tol", ctypes.c_double), ("max_newton", ctypes.c_int),
                ("max_minres", ctypes.c_int), ("minres_rtol", ctypes.c_double),
                ("max_halvings", ctypes.c_int), ("jacobi", ctypes.c_int),
                ("g0_norm", ctypes.c_double)]


class SolveReport(ctypes.Structure):
    _fields_ = [("newton_its", ctypes.c_int), ("minres_its_total", ctypes.c_int),
                ("halvings_total", ctypes.c_int), ("status", ctypes.c_int),
                ("F0", ctypes.c_double), ("F", ctypes.c_double), ("g0_norm", ctypes.c_double),
                ("g_norm", ctypes.c_double), ("t_setup_ms", ctypes.c_double),
                ("t_minres_ms", ctypes.c_double), ("t_linesearch_ms", ctypes.c_double),
                ("t_total_ms", ctypes.c_double), ("t_apply_ms", ctypes.c_double),
                ("t_apply_elem_ms", ctypes.c_double), ("n_apply", ctypes.c_int),
                ("reserved", ctypes.c_int)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["status_name"] = STATUS.get(self.status, "?")
        return d


class IterRecord(ctypes.Structure):
    _fields_ = [("F", ctypes.c_double), ("g_norm", ctypes.c_double),
                ("minres_its", ctypes.c_int), ("halvings", ctypes.c_int)]


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_lib_handle = None

# (name, argtypes) of every exported entry point declared in include/tmop.h
SIGNATURES = {
    "tmop_create": [ctypes.POINTER(_P), ctypes.POINTER(MeshDesc), ctypes.POINTER(Params), _P],
    "tmop_destroy": [_P],
    "tmop_workspace_bytes": [ctypes.POINTER(MeshDesc), ctypes.POINTER(Params), ctypes.c_int,
                             ctypes.POINTER(ctypes.c_size_t)],
    "tmop_sizes": [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
    "tmop_basis_nodes": [ctypes.c_int, _D],
    "tmop_energy": [_P, _P, _D],
    "tmop_min_det": [_P, _P, _D],
    "tmop_energy_mindet": [_P, _P, _D, _D],
    "tmop_gradient": [_P, _P, _P],
    "tmop_energy_gradient": [_P, _P, _D, _D, _P, _D],
    "tmop_hessian_setup": [_P, _P],
    "tmop_hessian_apply": [_P, _P, _P],
    "tmop_hessian_diag": [_P, _P],
    "tmop_hessian_setup_diag": [_P, _P, _P],
    "tmop_solve": [_P, _P, ctypes.POINTER(SolveParams), ctypes.POINTER(SolveReport)],
    "tmop_newton_step": [_P, _P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(SolveReport)],
    "tmop_minres": [_P, _P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                    ctypes.POINTER(ctypes.c_int)],
    "tmop_time_apply": [_P, _P, _P, ctypes.c_int, _D, _D],
    "tmop_set_timing": [_P, ctypes.c_int],
    "tmop_set_sweeps": [_P, ctypes.c_int],
    "tmop_solve_history": [_P, ctypes.POINTER(IterRecord), ctypes.c_int,
                           ctypes.POINTER(ctypes.c_int)],
    "tmop_set_lanczos_bank_limit": [_P, ctypes.c_size_t],
    "tmop_pool_set_lanczos_bank": [_P, ctypes.c_int],
    "tmop_set_limiting": [_P, _P, ctypes.c_double, ctypes.c_double],
    "tmop_autotune": [_P, _P, _P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
    "tmop_tile_epb": [_P, ctypes.POINTER(ctypes.c_int)],
    "tmop_set_tile": [_P, ctypes.c_int],
    "tmop_pool_create": [ctypes.POINTER(_P), ctypes.c_size_t, ctypes.c_int, _P],
    "tmop_pool_destroy": [_P],
    "tmop_pool_request_bytes": [ctypes.POINTER(MeshDesc), ctypes.POINTER(Params),
                                ctypes.POINTER(ctypes.c_size_t)],
    "tmop_pool_admit": [_P, ctypes.POINTER(MeshDesc), ctypes.POINTER(Params),
                        ctypes.POINTER(SolveParams), _P, _P, ctypes.POINTER(ctypes.c_int)],
    "tmop_pool_admit_limited": [_P, ctypes.POINTER(MeshDesc), ctypes.POINTER(Params),
                                ctypes.POINTER(SolveParams), _P, _P, ctypes.c_double,
                                ctypes.c_double, _P, ctypes.POINTER(ctypes.c_int)],
    "tmop_pool_step": [_P, ctypes.POINTER(ctypes.c_int)],
    "tmop_pool_poll": [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(SolveReport)],
    "tmop_pool_result": [_P, ctypes.c_int, _P, _P],
    "tmop_pool_evaluate": [_P, ctypes.c_int, ctypes.c_int, _P, _P, _D, _P],
    "tmop_pool_release": [_P, ctypes.c_int],
    "tmop_pool_info": [_P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                       ctypes.POINTER(ctypes.c_int)],
    "tmop_pool_set_graph": [_P, ctypes.c_int],
    "tmop_pool_autotune": [_P, ctypes.c_int],
    "tmop_pool_last_error": [],
    "tmop_batch_solve": [ctypes.c_int, ctypes.POINTER(MeshDesc), ctypes.POINTER(Params),
                         ctypes.POINTER(_P), ctypes.POINTER(SolveParams),
                         ctypes.POINTER(SolveReport), _P],
    "tmop_energy_mindet_noalloc": [ctypes.POINTER(MeshDesc), ctypes.POINTER(Params), _P, _P, _P],
    "tmop_last_error": [],
    "tmop_version": [],
}


def lib():
    """Load libtmop_hip.so (raises if it was not built)."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libtmop_hip.so is not built; run python -m paper_2205_12721_amd.build")
        # torch's GPU runtime comes up before the library's first HIP call:
        # the binding hands torch tensors and streams to the library, and
        # torch initialised after the library has failed to find the device
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
        h = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(h, name)
            f.argtypes = args
            f.restype = (ctypes.c_char_p if name in ("tmop_last_error", "tmop_version",
                                                     "tmop_pool_last_error") else ctypes.c_int)
        _lib_handle = h
    return _lib_handle


def _check(code):
    if code != 0:
        raise TmopError(code, lib().tmop_last_error().decode())


def basis_nodes(p):
    """The p+1 node positions on [0,1] at which the library places element nodes."""
    out = np.zeros(p + 1)
    _check(lib().tmop_basis_nodes(int(p), out.ctypes.data_as(_D)))
    return out


def _ptr(t, n=None, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError("expected dtype %s, got %s" % (dtype, t.dtype))
    if n is not None and t.numel() != n:
        raise ValueError("tensor has %d entries, expected %d" % (t.numel(), n))
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A PA-TMOP problem on one GPU.

    Structured box: ``Context(dim, n, p, nq1d)`` with ``n`` an int or a tuple of
    elements per axis.  General mesh: pass ``elem_to_node`` (int32 CUDA tensor,
    (E, (p+1)^dim)) and ``num_nodes``.
    ``ess``: "boundary" (box only), "none", or a uint8 CUDA mask of d*N_x.
    ``precision``: "fp64" or "mixed".
    ``storage``: "tensor" (packed second-derivative tensor per point) or
    "compact" (T and four metric coefficients per point).
    """

    def __init__(self, dim, n=None, p=1, nq1d=None, metric=None, precision="fp64", W=None,
                 ess="boundary", elem_to_node=None, num_nodes=None, stream=None,
                 storage="tensor", quad="gl"):
        import torch
        self._torch = torch
        self.dim, self.p = dim, p
        self.nq1d = nq1d if nq1d is not None else p + 2
        self.metric = metric if metric is not None else (2 if dim == 2 else 303)
        self.precision = precision
        md = MeshDesc()
        md.dim, md.order_p = dim, p
        self._keep = []
        if elem_to_node is None:
            ns = (n,) * dim if np.isscalar(n) else tuple(n)
            if len(ns) != dim:
                raise ValueError("need one element count per axis")
            md.nx, md.ny = ns[0], ns[1]
            md.nz = ns[2] if dim == 3 else 0
            self.shape = ns
        else:
            md.elem_to_node = _ptr(elem_to_node, dtype=torch.int32).value
            md.num_elems = elem_to_node.shape[0]
            md.num_nodes = int(num_nodes)
            self._keep.append(elem_to_node)
            self.shape = None
        if isinstance(ess, str):
            md.ess_mode = {"boundary": ESS_BOUNDARY, "none": ESS_NONE}[ess]
        else:
            md.ess_mode = ESS_MASK
            md.ess_mask = _ptr(ess, dtype=torch.uint8).value
            self._keep.append(ess)
        prm = Params()
        prm.metric = self.metric
        prm.nq1d = self.nq1d
        if W is not None:
            Wa = np.asarray(W, dtype=np.float64).reshape(dim, dim)
            prm.has_W = 1
            for k, v in enumerate(Wa.ravel()):
                prm.W[k] = v
        prm.precision = {"fp64": TMOP_FP64, "mixed": TMOP_MIXED}[precision]
        prm.hess_storage = {"tensor": HESS_TENSOR, "compact": HESS_COMPACT}[storage]
        prm.quad_rule = QUAD_RULES[quad]
        self.storage = storage
        self._md, self._prm = md, prm
        s = stream if stream is not None else torch.cuda.current_stream()
        self._stream = s
        h = ctypes.c_void_p()
        _check(lib().tmop_create(ctypes.byref(h), ctypes.byref(md), ctypes.byref(prm),
                                 ctypes.c_void_p(s.cuda_stream)))
        self._h = h
        nn, nd = ctypes.c_int(), ctypes.c_int()
        _check(lib().tmop_sizes(h, ctypes.byref(nn), ctypes.byref(nd)))
        self.num_nodes, self.ndof = nn.value, nd.value

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().tmop_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- helpers ----------------------------------------------------------
    def _vec(self, t):
        return _ptr(t, self.ndof, self._torch.float64)

    def new_vector(self):
        return self._torch.zeros(self.ndof, dtype=self._torch.float64, device="cuda")

    def workspace_bytes(self, with_solver=True):
        b = ctypes.c_size_t()
        _check(lib().tmop_workspace_bytes(ctypes.byref(self._md), ctypes.byref(self._prm),
                                          int(with_solver), ctypes.byref(b)))
        return b.value

    # -- evaluations --------------------------------------------------------
    def energy(self, x):
        F = ctypes.c_double()
        _check(lib().tmop_energy(self._h, self._vec(x), ctypes.byref(F)))
        return F.value

    def min_det(self, x):
        m = ctypes.c_double()
        _check(lib().tmop_min_det(self._h, self._vec(x), ctypes.byref(m)))
        return m.value

    def energy_mindet(self, x):
        F, m = ctypes.c_double(), ctypes.c_double()
        code = lib().tmop_energy_mindet(self._h, self._vec(x), ctypes.byref(F), ctypes.byref(m))
        if code not in (0, ERR_INVERTED):
            _check(code)
        return F.value, m.value

    def gradient(self, x, out=None):
        out = self.new_vector() if out is None else out
        _check(lib().tmop_gradient(self._h, self._vec(x), self._vec(out)))
        return out

    def energy_gradient(self, x, out=None):
        """(F, min det A, g, |g|^2) in one element pass; F = inf when inverted."""
        out = self.new_vector() if out is None else out
        F, m, g2 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        code = lib().tmop_energy_gradient(self._h, self._vec(x), ctypes.byref(F),
                                          ctypes.byref(m), self._vec(out), ctypes.byref(g2))
        if code not in (0, ERR_INVERTED):
            _check(code)
        return F.value, m.value, out, g2.value

    def hessian_setup(self, x):
        _check(lib().tmop_hessian_setup(self._h, self._vec(x)))

    def hessian_apply(self, v, out=None):
        out = self.new_vector() if out is None else out
        _check(lib().tmop_hessian_apply(self._h, self._vec(v), self._vec(out)))
        return out

    def hessian_diag(self, out=None):
        out = self.new_vector() if out is None else out
        _check(lib().tmop_hessian_diag(self._h, self._vec(out)))
        return out

    def hessian_setup_diag(self, x, out=None):
        """hessian_setup(x) then hessian_diag(), in one element pass where the class allows."""
        out = self.new_vector() if out is None else out
        _check(lib().tmop_hessian_setup_diag(self._h, self._vec(x), self._vec(out)))
        return out

    def minres(self, b, max_its=50, rtol=1e-12, jacobi=True, out=None):
        out = self.new_vector() if out is None else out
        its = ctypes.c_int()
        _check(lib().tmop_minres(self._h, self._vec(b), self._vec(out), int(max_its),
                                 float(rtol), int(bool(jacobi)), ctypes.byref(its)))
        return out, its.value

    def autotune(self, v, y, reps=10):
        """Pick the fastest Hessian-action tile shape (needs hessian_setup); returns the
        chosen elements per workgroup."""
        e = ctypes.c_int()
        _check(lib().tmop_autotune(self._h, self._vec(v), self._vec(y), int(reps), ctypes.byref(e)))
        return e.value

    def set_tile(self, epb):
        _check(lib().tmop_set_tile(self._h, int(epb)))

    def tile_epb(self):
        e = ctypes.c_int()
        _check(lib().tmop_tile_epb(self._h, ctypes.byref(e)))
        return e.value

    def set_limiting(self, x0=None, coef=1.0, delta=1.0):
        """Add (or, with x0=None, remove) the limiting term coef*|x - x0|^2/delta^2."""
        ptr = None if x0 is None else self._vec(x0)
        _check(lib().tmop_set_limiting(self._h, ptr, float(coef), float(delta)))

    def set_timing(self, enable=True):
        _check(lib().tmop_set_timing(self._h, int(bool(enable))))

    def set_sweeps(self, mode):
        """Forward contractions of energy, gradient and FP64 setup: "pencil"
        (default) or "mfma" (FP64 matrix cores; hex classes with nq1d <= 5)."""
        _check(lib().tmop_set_sweeps(self._h, SWEEPS[mode]))

    def set_lanczos_bank_limit(self, max_bytes):
        """Bytes the resident MINRES Lanczos vectors may take (0: three-term
        solution update every iteration)."""
        _check(lib().tmop_set_lanczos_bank_limit(self._h, int(max_bytes)))

    def time_apply(self, v, y, n):
        e, t = ctypes.c_double(), ctypes.c_double()
        _check(lib().tmop_time_apply(self._h, self._vec(v), self._vec(y), int(n),
                                     ctypes.byref(e), ctypes.byref(t)))
        return e.value, t.value

    # -- solve ----------------------------------------------------------------
    def solve(self, x, rel_grad_tol=1e-8, max_newton=200, max_minres=50, minres_rtol=1e-12,
              max_halvings=30, jacobi=True, g0_norm=0.0, raise_on_error=False):
        """Optimise x in place; returns the report as a dict (status in 'status')."""
        sp = SolveParams(rel_grad_tol, max_newton, max_minres, minres_rtol, max_halvings,
                         int(bool(jacobi)), g0_norm)
        rep = SolveReport()
        code = lib().tmop_solve(self._h, self._vec(x), ctypes.byref(sp), ctypes.byref(rep))
        if raise_on_error and code != 0:
            _check(code)
        d = rep.as_dict()
        d["message"] = lib().tmop_last_error().decode() if code else ""
        d["history"] = self.solve_history()
        return d

    def solve_history(self):
        """Per-iteration record of the last solve: (F, |g|, MINRES iterations,
        halvings) for the initial mesh and after each accepted Newton update."""
        n = ctypes.c_int()
        _check(lib().tmop_solve_history(self._h, None, 0, ctypes.byref(n)))
        buf = (IterRecord * max(n.value, 1))()
        _check(lib().tmop_solve_history(self._h, buf, n.value, ctypes.byref(n)))
        return [(r.F, r.g_norm, r.minres_its, r.halvings) for r in buf[:n.value]]

    def newton_step(self, x, n_minres=20, jacobi=True):
        rep = SolveReport()
        code = lib().tmop_newton_step(self._h, self._vec(x), int(n_minres), int(bool(jacobi)),
                                      ctypes.byref(rep))
        _check(code)
        return rep.as_dict()


# ---------------------------------------------------------------------------
# Batched and served solves
# ---------------------------------------------------------------------------

def _pcheck(code):
    if code != 0:
        raise TmopError(code, lib().tmop_pool_last_error().decode())


def request(dim, n, p, nq1d=None, metric=None, precision="fp64", storage="tensor", W=None,
            ess="boundary"):
    """(MeshDesc, Params) of a structured-box request."""
    ns = (n,) * dim if np.isscalar(n) else tuple(n)
    md = MeshDesc()
    md.dim, md.order_p = dim, p
    md.nx, md.ny = ns[0], ns[1]
    md.nz = ns[2] if dim == 3 else 0
    if isinstance(ess, str):
        md.ess_mode = {"boundary": ESS_BOUNDARY, "none": ESS_NONE}[ess]
    else:
        # a device uint8 mask of fixed DoFs; tmop_pool_admit copies it, so it
        # needs to live only until the request is admitted
        import torch
        md.ess_mode = ESS_MASK
        md.ess_mask = _ptr(ess, dtype=torch.uint8).value
    prm = Params()
    prm.metric = metric if metric is not None else (2 if dim == 2 else 303)
    prm.nq1d = nq1d if nq1d is not None else p + 2
    if W is not None:
        prm.has_W = 1
        for k, v in enumerate(np.asarray(W, dtype=np.float64).ravel()):
            prm.W[k] = v
    prm.precision = {"fp64": TMOP_FP64, "mixed": TMOP_MIXED}[precision]
    prm.hess_storage = {"tensor": HESS_TENSOR, "compact": HESS_COMPACT}[storage]
    return md, prm


def energy_mindet_noalloc(md, prm, x, out, stream=None):
    """tmop_energy_mindet_noalloc: F, min det A and the count of points with
    det A <= 0 written to the device tensor ``out`` (3 doubles) on ``stream``
    (default: torch's current stream), with no allocation by the library."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().tmop_energy_mindet_noalloc(ctypes.byref(md), ctypes.byref(prm),
                                            _ptr(x, dtype=torch.float64),
                                            _ptr(out, 3, torch.float64),
                                            ctypes.c_void_p(s.cuda_stream)))
    return out


def solve_params(rel_grad_tol=1e-8, max_newton=200, max_minres=50, minres_rtol=1e-12,
                 max_halvings=30, jacobi=True, g0_norm=0.0):
    return SolveParams(rel_grad_tol, max_newton, max_minres, minres_rtol, max_halvings,
                       int(bool(jacobi)), g0_norm)


def request_bytes(md, prm, limited=False):
    """Arena bytes of one pooled solve (with ``limited`` also its reference nodes)."""
    b = ctypes.c_size_t()
    _pcheck(lib().tmop_pool_request_bytes(ctypes.byref(md), ctypes.byref(prm), ctypes.byref(b)))
    if limited:
        nx = (md.nx * md.order_p + 1) * (md.ny * md.order_p + 1) * \
            ((md.nz * md.order_p + 1) if md.dim == 3 else 1)
        return b.value + (8 * md.dim * nx + 255) // 256 * 256
    return b.value


class Pool:
    """Many solves advanced together (see tmop_pool_* in include/tmop.h)."""

    def __init__(self, hbm_budget, max_slots, graph=True, lanczos_bank=False):
        """``graph``: 0 (or False) no HIP graphs, 1 (or True) a replayed block of
        six MINRES iterations, 2 the whole Newton step replayed once per step."""
        import torch
        self._torch = torch
        h = ctypes.c_void_p()
        _pcheck(lib().tmop_pool_create(ctypes.byref(h), int(hbm_budget), int(max_slots), None))
        self._h = h
        self._keep = {}
        mode = (1 if graph else 0) if isinstance(graph, bool) else int(graph)
        if mode != 1:
            _pcheck(lib().tmop_pool_set_graph(h, mode))
        if lanczos_bank:
            _pcheck(lib().tmop_pool_set_lanczos_bank(h, 1))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().tmop_pool_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, md, prm, sp, x, x0=None, coef=1.0, delta=1.0):
        """Returns the slot index; raises TmopError (code ERR_BUSY / ERR_BUDGET ...).
        With reference nodes x0 the solve carries the limiting term
        coef |x - x0|^2 / delta^2 (tmop_pool_admit_limited)."""
        slot = ctypes.c_int(-1)
        s = self._torch.cuda.current_stream().cuda_stream
        if x0 is None:
            _pcheck(lib().tmop_pool_admit(self._h, ctypes.byref(md), ctypes.byref(prm),
                                          ctypes.byref(sp), _ptr(x, dtype=self._torch.float64),
                                          ctypes.c_void_p(s), ctypes.byref(slot)))
        else:
            _pcheck(lib().tmop_pool_admit_limited(
                self._h, ctypes.byref(md), ctypes.byref(prm), ctypes.byref(sp),
                _ptr(x, dtype=self._torch.float64), _ptr(x0, dtype=self._torch.float64),
                float(coef), float(delta), ctypes.c_void_p(s), ctypes.byref(slot)))
        self._keep[slot.value] = (md, prm, sp)
        return slot.value

    def step(self):
        n = ctypes.c_int()
        _pcheck(lib().tmop_pool_step(self._h, ctypes.byref(n)))
        return n.value

    def poll(self, slot):
        done = ctypes.c_int()
        rep = SolveReport()
        _pcheck(lib().tmop_pool_poll(self._h, int(slot), ctypes.byref(done), ctypes.byref(rep)))
        return bool(done.value), rep.as_dict()

    def result(self, slot, out):
        _pcheck(lib().tmop_pool_result(self._h, int(slot), _ptr(out, dtype=self._torch.float64), None))
        return out

    def release(self, slot):
        _pcheck(lib().tmop_pool_release(self._h, int(slot)))
        self._keep.pop(slot, None)

    # -- one slot's operators with the pool's batched kernels (between steps) --
    def _eval(self, slot, what, x=None, out=None, host=None):
        s = self._torch.cuda.current_stream().cuda_stream
        xin = None if x is None else _ptr(x, dtype=self._torch.float64)
        o = None if out is None else _ptr(out, dtype=self._torch.float64)
        hp = None if host is None else host.ctypes.data_as(_D)
        _pcheck(lib().tmop_pool_evaluate(self._h, int(slot), what, xin, o, hp, ctypes.c_void_p(s)))

    def energy_mindet(self, slot, x):
        """(F, min det A) of the slot's mesh at nodes x; F = inf if det <= 0."""
        h = np.zeros(2)
        try:
            self._eval(slot, EVAL_ENERGY, x, host=h)
        except TmopError as e:
            if e.code != ERR_INVERTED:
                raise
        return float(h[0]), float(h[1])

    def gradient(self, slot, x):
        out = self._torch.empty_like(x)
        self._eval(slot, EVAL_GRADIENT, x, out)
        return out

    def hessian_setup(self, slot, x):
        self._eval(slot, EVAL_SETUP, x)

    def hessian_apply(self, slot, v):
        out = self._torch.empty_like(v)
        self._eval(slot, EVAL_APPLY, v, out)
        return out

    def hessian_diag(self, slot, like):
        out = self._torch.empty_like(like)
        self._eval(slot, EVAL_DIAG, None, out)
        return out

    def autotune(self, reps=5):
        """Pick the Hessian-action tile shape of every resident kernel class."""
        _pcheck(lib().tmop_pool_autotune(self._h, int(reps)))

    def info(self):
        u, b, n = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int()
        _pcheck(lib().tmop_pool_info(self._h, ctypes.byref(u), ctypes.byref(b), ctypes.byref(n)))
        return dict(used=u.value, budget=b.value, slots=n.value)


def batch_solve(requests, xs, sps):
    """Solve meshes together; xs (CUDA float64 tensors) are overwritten.  Returns reports."""
    import torch
    n = len(requests)
    mds = (MeshDesc * n)(*[r[0] for r in requests])
    prms = (Params * n)(*[r[1] for r in requests])
    spa = (SolveParams * n)(*sps)
    reps = (SolveReport * n)()
    ptrs = (ctypes.c_void_p * n)(*[_ptr(x, dtype=torch.float64).value for x in xs])
    code = lib().tmop_batch_solve(n, mds, prms, ptrs, spa, reps,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _pcheck(code)
    return [r.as_dict() for r in reps]
