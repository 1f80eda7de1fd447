"""Continuous-batching server for mesh-optimisation requests on one GPU.

A request is a perturbed structured quad/hex mesh (its node vector already on
the device when it arrives) with its solve parameters.  The server admits
arrived requests in FIFO order into a ``Pool`` while its HBM budget and slot
count allow (``ERR_BUSY`` is back-pressure: the request waits), advances every
resident solve by one Newton iteration per tick (one batched launch per kernel
class and phase), and retires finished solves as soon as their tick ends, which
frees their slot and memory for waiting requests.  Latency runs from the
request's arrival time to the end of the tick in which it finished (host
monotonic clock).  Percentiles count every request: one that fails (line
search, iteration cap) or is rejected enters with the time at which its
result was known, so failures cannot make the latency look better; the
summaries also give the solved count and the percentiles over solved
requests alone.

``sequential`` runs the same stream one request at a time through a plain FP64
context (``Context.solve``), the reference the served form is compared with.
"""
import time

import numpy as np

from . import inputs
from .tmop import (ERR_BUSY, Context, Pool, TmopError, basis_nodes, request, request_bytes,
                   solve_params)


def make_inputs(reqs, amp=0.05, validate=True):
    """Host node vectors of a request stream (seeded, smooth + jitter recipe).

    With ``validate`` a draw with det A <= 0 at a quadrature point is redrawn
    from the continuing stream of its seed, the library deciding on the GPU
    (one context per mesh size, compact mixed storage to keep it small);
    ``redraws`` of each request are recorded in ``r["redraws"]``.
    """
    import torch
    out = [None] * len(reqs)
    groups = {}
    for k, r in enumerate(reqs):
        groups.setdefault((r["dim"], r["n"], r["p"], r["nq"]), []).append(k)
    for (dim, n, p, nq), ks in groups.items():
        ctx = Context(dim, n, p, nq, precision="mixed", storage="compact") if validate else None
        ok = (lambda x: ctx.min_det(torch.as_tensor(x).cuda()) > 0.0) if validate else None
        for k in ks:
            r = reqs[k]
            x, info = inputs.perturbed_box(dim, n, p, basis_nodes(p), r["seed"], recipe="smooth",
                                           amp=amp, is_valid=ok)
            r["redraws"] = info["tries"] - 1 if validate else 0
            out[k] = x
        if ctx is not None:
            ctx.close()
    return out


def _percentiles(lat, prefix=""):
    a = np.asarray(lat)
    if a.size == 0:
        return {prefix + "p50_ms": None, prefix + "p99_ms": None, prefix + "mean_ms": None}
    return {prefix + "p50_ms": float(np.percentile(a, 50)),
            prefix + "p99_ms": float(np.percentile(a, 99)), prefix + "mean_ms": float(a.mean())}


def _summary(rec, wall):
    """Latency over every request (failed and rejected ones at the time their
    result was known) and over solved requests alone."""
    n = len(rec)
    lat_all = [r["latency_ms"] for r in rec if r and r.get("latency_ms") is not None]
    lat_ok = [r["latency_ms"] for r in rec if r and r.get("latency_ms") is not None and r["status"] == 0]
    ok = sum(1 for r in rec if r and r["status"] == 0)
    out = dict(requests=n, solved=ok, failed=n - ok, wall_s=wall,
               solves_per_s=ok / wall if wall > 0 else None)
    out.update(_percentiles(lat_all))
    out.update(_percentiles(lat_ok, "solved_"))
    return out


def serve(reqs, xs_host, hbm_budget, max_slots=256, precision="mixed", storage="compact",
          rel_grad_tol=1e-8, max_newton=200, max_minres=50, graph=True, lanczos_bank=False):
    """Run the stream through a pool; returns a summary dict and per-request records."""
    import torch
    pool = Pool(hbm_budget, max_slots, graph=graph, lanczos_bank=lanczos_bank)
    sp = solve_params(rel_grad_tol=rel_grad_tol, max_newton=max_newton, max_minres=max_minres)
    # every request's nodes are on the device when it arrives
    xds = [torch.as_tensor(x).cuda() for x in xs_host]
    torch.cuda.synchronize()

    def describe(r):
        return request(r["dim"], r["n"], r["p"], r["nq"], precision=precision, storage=storage)

    try:
        return serve_loop(reqs, xds, pool, sp, describe)
    finally:
        pool.close()


def serve_loop(reqs, xs, pool, sp, describe):
    """The scheduling loop of ``serve`` over any pool object.

    ``pool`` provides ``admit(md, prm, sp, x) -> slot`` (raising ``TmopError``:
    ``ERR_BUSY`` is back-pressure, any other code rejects the request),
    ``step()``, ``poll(slot) -> (done, report)``, ``result(slot, x)``,
    ``release(slot)`` and ``info() -> {"used": bytes}``; ``xs[k]`` is request
    k's node vector (written with the result); ``describe(r)`` gives the
    ``(mesh, params)`` pair the pool admits.  Arrivals follow
    ``r["t_arrive"]`` (seconds from the start) on the host monotonic clock.
    Returns (summary, per-request records)."""
    n = len(reqs)
    pending = []            # arrived, not admitted (FIFO)
    resident = {}           # slot -> (request index, node vector)
    rec = [None] * n
    nxt = 0
    t0 = time.monotonic()
    ticks = 0
    peak_used = 0
    while nxt < n or pending or resident:
        now = (time.monotonic() - t0) * 1e3
        while nxt < n and reqs[nxt]["t_arrive"] * 1e3 <= now:
            pending.append(nxt)
            nxt += 1
        while pending:
            k = pending[0]
            r = reqs[k]
            md, prm = describe(r)
            xd = xs[k]
            try:
                slot = pool.admit(md, prm, sp, xd)
            except TmopError as e:
                if e.code == ERR_BUSY:
                    break
                rec[k] = dict(status=e.code, rejected=True,
                              latency_ms=(time.monotonic() - t0) * 1e3 - r["t_arrive"] * 1e3)
                pending.pop(0)
                continue
            pending.pop(0)
            resident[slot] = (k, xd)
        peak_used = max(peak_used, pool.info()["used"])
        if resident:
            pool.step()
            ticks += 1
            tend = (time.monotonic() - t0) * 1e3
            for slot in list(resident):
                done, rep = pool.poll(slot)
                if done:
                    k, xd = resident.pop(slot)
                    pool.result(slot, xd)
                    pool.release(slot)
                    rec[k] = dict(status=rep["status"], latency_ms=tend - reqs[k]["t_arrive"] * 1e3,
                                  newton_its=rep["newton_its"], minres_its=rep["minres_its_total"],
                                  F=rep["F"], x=xd)
        elif nxt < n:
            # idle until the next arrival
            wait = reqs[nxt]["t_arrive"] - (time.monotonic() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.01))
    wall = time.monotonic() - t0
    out = _summary(rec, wall)
    out.update(ticks=ticks, peak_bytes=peak_used)
    return out, rec


def sequential(reqs, xs_host, rel_grad_tol=1e-8, max_newton=200, max_minres=50):
    """The same stream one request at a time through FP64 contexts (arrival-time aware)."""
    import torch
    n = len(reqs)
    rec = [None] * n
    xds = [torch.as_tensor(x).cuda() for x in xs_host]
    torch.cuda.synchronize()
    t0 = time.monotonic()
    for k, r in enumerate(reqs):
        now = time.monotonic() - t0
        if r["t_arrive"] > now:
            time.sleep(r["t_arrive"] - now)
        ctx = Context(r["dim"], r["n"], r["p"], r["nq"])
        xd = xds[k]
        rep = ctx.solve(xd, rel_grad_tol=rel_grad_tol, max_newton=max_newton, max_minres=max_minres)
        torch.cuda.synchronize()
        ctx.close()
        tend = (time.monotonic() - t0) * 1e3
        rec[k] = dict(status=rep["status"], latency_ms=tend - r["t_arrive"] * 1e3,
                      newton_its=rep["newton_its"], F=rep["F"], x=xd)
    wall = time.monotonic() - t0
    return _summary(rec, wall), rec


def budget_for(reqs, precision="mixed", storage="compact", factor=1.0, cap=None):
    """Sum of the requests' arena bytes (times factor, optionally capped)."""
    tot = 0
    big = 0
    for r in reqs:
        b = request_bytes(*request(r["dim"], r["n"], r["p"], r["nq"], precision=precision,
                                   storage=storage))
        tot += b
        big = max(big, b)
    b = int(tot * factor)
    if cap is not None:
        b = min(b, cap)
    return max(b, big)
