"""Serving loop (continuous batching over a pool): a small Poisson stream with a
budget below the stream's total footprint, so requests wait for memory.  The
stream's sizes reach 16^3 elements (this draw holds 12^3 Q4, 14^3 Q3, 10^3 and
9^3 hexes and 38^2 and 23^2 quads beside smaller meshes).

* every request is solved, and its nodes are bitwise identical to the same
  request solved alone in its own pool (same arithmetic alone and in the mix);
* the pool never holds more bytes than its budget.
"""
import numpy as np
import pytest

from tests.gpu_common import log, to_host

pytestmark = pytest.mark.gpu


def test_stream_alone_equals_mix():
    from paper_2205_12721_amd import inputs, serve
    reqs = inputs.serving_stream(400.0, count=14, seed=17, max_n3=16)
    assert sum(1 for r in reqs if r["n"] ** r["dim"] > 8 ** 3) >= 5
    xs = serve.make_inputs(reqs)
    total = serve.budget_for(reqs)
    budget = serve.budget_for(reqs, factor=0.4)
    summary, rec = serve.serve(reqs, xs, budget, max_slots=8)
    log("serve", summary)
    assert summary["solved"] == len(reqs)
    assert summary["peak_bytes"] <= budget < total
    for k, r in enumerate(reqs):
        alone, rec1 = serve.serve([dict(r, t_arrive=0.0)], [xs[k]], serve.budget_for([r]), max_slots=1)
        assert rec1[0]["status"] == 0
        assert np.array_equal(to_host(rec[k]["x"]), to_host(rec1[0]["x"]))
        assert rec[k]["newton_its"] == rec1[0]["newton_its"]
