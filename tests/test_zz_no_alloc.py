"""The no-allocation energy entry point against the context's energy.

tmop_energy_mindet_noalloc (partials in the library's fixed device array)
must give, through the C ABI, what tmop_energy_mindet gives with a context's
workspace: bitwise the same F and min det, the same inverted flag, on two
calls in a row (the second with a smaller mesh, so stale partials of the
first would show), and it must reject a mesh with more element tiles than
the array holds and a general-connectivity mesh before launching anything.
"""
import ctypes

import numpy as np
import pytest

from tests.gpu_common import make_case, to_dev, to_host

pytestmark = pytest.mark.gpu


def _context_energy(c, x):
    from paper_2205_12721_amd.tmop import Context
    ctx = Context(c["dim"], c["ns"], c["p"], c["nq"])
    F, md = ctx.energy_mindet(to_dev(x))
    ctx.close()
    return F, md


def _noalloc(c, x):
    import torch
    from paper_2205_12721_amd import tmop
    md, prm = tmop.request(c["dim"], c["ns"], c["p"], c["nq"])
    out = torch.full((3,), np.nan, dtype=torch.float64, device="cuda")
    tmop.energy_mindet_noalloc(md, prm, to_dev(x), out)
    return to_host(out)


CASES = [
    dict(dim=3, ns=(12, 11, 10), p=3, nq=5, seed=5),  # 660 tiles of 2 elements
    dict(dim=3, ns=(3, 4, 2), p=2, nq=4, seed=6),     # smaller: 6 tiles
    dict(dim=2, ns=(9, 7), p=4, nq=6, seed=7),
]


def test_noalloc_energy_matches_context_twice_shrinking():
    import oracle
    for c in CASES:
        pb, x = make_case(c["dim"], c["ns"], c["p"], c["nq"], seed=c["seed"],
                          recipe="smooth" if c["dim"] == 3 else "interior_jitter")
        out = _noalloc(c, x)
        F, md = _context_energy(c, x)
        print("noalloc", c, out, F, md, flush=True)
        assert out[2] == 0.0
        assert out[0] == F and out[1] == md
        Fo = pb.energy(x)
        assert abs(out[0] - Fo) <= 1e-11 * abs(Fo)
        assert abs(out[1] - pb.min_det(x)) <= 1e-12 * abs(pb.min_det(x))


def test_noalloc_inverted_mesh_flagged():
    c = dict(dim=2, ns=(4, 3), p=2, nq=4, seed=8)
    pb, x = make_case(c["dim"], c["ns"], c["p"], c["nq"], seed=c["seed"], recipe="interior_jitter")
    x = x.copy()
    # move the interior grid node (4, 3) of the 9 x 7 node grid by 0.6 in x,
    # past several neighbours (node spacing 0.125): det A < 0 next to it
    x[4 + 9 * 3] += 0.6
    out = _noalloc(c, x)
    assert out[2] > 0 and out[1] <= 0.0
    assert abs(out[1] - pb.min_det(x)) <= 1e-12 * abs(pb.min_det(x))


def test_noalloc_rejects_before_launch():
    import torch
    from paper_2205_12721_amd import tmop
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    # 64^3 Q2 with 4^3 points fills exactly 65536 tiles; one more layer exceeds it
    md, prm = tmop.request(3, (64, 64, 65), 2, 4)
    x = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(tmop.TmopError) as ei:
        tmop.energy_mindet_noalloc(md, prm, x, out)
    assert ei.value.code == 1 and "at most 65536" in str(ei.value)
    md, prm = tmop.request(3, 2, 1, 3)
    e2n = torch.zeros(8 * 8, dtype=torch.int32, device="cuda")
    md.elem_to_node = e2n.data_ptr()
    md.num_elems, md.num_nodes = 8, 27
    with pytest.raises(tmop.TmopError) as ei:
        tmop.energy_mindet_noalloc(md, prm, x, out)
    assert ei.value.code == 2
