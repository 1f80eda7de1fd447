"""CPU checks of the C ABI: the library loads and exports every declared entry point.

No compute call is made here (there is no GPU on the build machine).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tmop.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tmop_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_core_calls():
    names = declared_functions()
    for n in ["tmop_create", "tmop_destroy", "tmop_energy", "tmop_gradient", "tmop_min_det",
              "tmop_hessian_setup", "tmop_hessian_apply", "tmop_hessian_diag", "tmop_solve",
              "tmop_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2205_12721_amd import tmop
    if not os.path.exists(tmop.LIB_PATH):
        pytest.fail("libtmop_hip.so is not built (run __graft_entry__.build())")
    h = ctypes.CDLL(tmop.LIB_PATH)
    for name in declared_functions():
        assert hasattr(h, name), name
    # every declared function has a binding signature, and vice versa
    assert set(declared_functions()) == set(tmop.SIGNATURES)


def test_binding_struct_layouts():
    from paper_2205_12721_amd import tmop
    # layouts follow the C declarations (LP64): see include/tmop.h
    assert ctypes.sizeof(tmop.MeshDesc) == 56
    assert tmop.MeshDesc.elem_to_node.offset == 32
    assert tmop.MeshDesc.ess_mask.offset == 48
    assert tmop.Params.W.offset == 16
    assert ctypes.sizeof(tmop.Params) == 16 + 72 + 16
    assert tmop.Params.hess_storage.offset == 92
    assert tmop.Params.quad_rule.offset == 96
    assert ctypes.sizeof(tmop.SolveParams) == 40
    assert ctypes.sizeof(tmop.SolveReport) == 16 + 10 * 8 + 8


def test_cpu_only_calls_without_gpu():
    """Host-only entry points work and report errors through the status path."""
    from paper_2205_12721_amd import tmop
    lib = tmop.lib()
    assert lib.tmop_version().decode().startswith("tmop")
    import numpy as np
    nodes = np.zeros(5)
    assert lib.tmop_basis_nodes(4, nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
    assert nodes[0] == 0.0 and nodes[-1] == 1.0 and abs(nodes[2] - 0.5) < 1e-15
    md = tmop.MeshDesc(dim=3, order_p=3, nx=4, ny=4, nz=4)
    prm = tmop.Params(metric=303, nq1d=5)
    b = ctypes.c_size_t()
    assert lib.tmop_workspace_bytes(ctypes.byref(md), ctypes.byref(prm), 1, ctypes.byref(b)) == 0
    assert b.value > 64 * 125 * 45 * 8
    bad = tmop.MeshDesc(dim=4, order_p=3, nx=4, ny=4, nz=4)
    assert lib.tmop_workspace_bytes(ctypes.byref(bad), ctypes.byref(prm), 1, ctypes.byref(b)) == 1
    assert "dim" in lib.tmop_last_error().decode()


def test_basis_nodes_match_oracle():
    """The library's host-side GLL nodes equal the oracle's (independent codes)."""
    import numpy as np
    from oracle import basis
    from paper_2205_12721_amd.tmop import basis_nodes
    for p in range(1, 5):
        assert np.allclose(basis_nodes(p), basis.gll_nodes(p), atol=1e-15, rtol=0)


def test_pool_rejects_gauss_lobatto_on_host():
    """Pooled solves take the Gauss-Legendre rule only (host-side request check)."""
    from paper_2205_12721_amd import tmop
    lib = tmop.lib()
    md = tmop.MeshDesc(dim=3, order_p=2, nx=4, ny=4, nz=4)
    prm = tmop.Params(metric=303, nq1d=4, quad_rule=1)
    b = ctypes.c_size_t()
    assert lib.tmop_pool_request_bytes(ctypes.byref(md), ctypes.byref(prm), ctypes.byref(b)) != 0
    assert "Gauss-Legendre" in lib.tmop_pool_last_error().decode()
    prm.quad_rule = 0
    assert lib.tmop_pool_request_bytes(ctypes.byref(md), ctypes.byref(prm), ctypes.byref(b)) == 0


def test_fused_entry_points_reject_null_arguments():
    """The one-pass calls check their arguments on the host before any device work."""
    from paper_2205_12721_amd import tmop
    lib = tmop.lib()
    assert lib.tmop_energy_gradient(None, None, None, None, None, None) == 1
    assert "null" in lib.tmop_last_error().decode()
    assert lib.tmop_hessian_setup_diag(None, None, None) == 1
    assert "null" in lib.tmop_last_error().decode()
