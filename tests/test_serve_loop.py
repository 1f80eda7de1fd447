"""The serving loop's scheduling logic (``serve.serve_loop``) on the CPU.

The pool is a test double whose step is one Newton iteration of the FP64
oracle per resident solve (test infrastructure only; the product path is the
HIP pool).  Its admission follows the pool's contract: ``ERR_BUDGET`` for a
request larger than the whole budget, ``ERR_BUSY`` while the free budget or
the free slots do not fit it, a tangled mesh admitted and failing at its
first step with ``ERR_INVERTED``.  Checked:

* every request is answered; each solved request's nodes and Newton count are
  bitwise those of the same request solved alone by the oracle (one Newton
  iteration per tick changes nothing in the arithmetic);
* admission is FIFO in arrival order, the resident bytes never exceed the
  budget, and a budget below the stream's total makes requests wait;
* a tangled request fails alone (``ERR_INVERTED``) and a request larger than
  the budget is rejected (``ERR_BUDGET``), both counted in the latency
  percentiles, without changing any other request's result.
"""
import numpy as np

import oracle
from oracle import basis
from paper_2205_12721_amd import inputs, serve
from paper_2205_12721_amd.tmop import (ERR_BUDGET, ERR_BUSY, ERR_INVERTED, TmopError, request,
                                       solve_params)

OK = 0


def _dims(md):
    ns = (md.nx, md.ny, md.nz)[: md.dim]
    return md.dim, ns, md.order_p


class OraclePool:
    """Pool double: a slot holds an oracle problem and its current nodes."""

    def __init__(self, budget, max_slots):
        self.budget, self.max_slots = budget, max_slots
        self.used = 0
        self.slots = {}
        self.admitted = []   # the admitted node vectors, in admission order
        self.peak = 0
        self.busy = 0        # admissions answered with ERR_BUSY

    @staticmethod
    def nbytes(md):
        dim, ns, p = _dims(md)
        return 8 * 24 * dim * int(np.prod([n * p + 1 for n in ns]))

    def admit(self, md, prm, sp, x):
        b = self.nbytes(md)
        if b > self.budget:
            raise TmopError(ERR_BUDGET, "request alone exceeds the budget")
        if len(self.slots) >= self.max_slots or self.used + b > self.budget:
            self.busy += 1
            raise TmopError(ERR_BUSY, "no room now")
        dim, ns, p = _dims(md)
        slot = min(set(range(self.max_slots)) - set(self.slots))
        self.slots[slot] = dict(pb=oracle.Problem.box(dim, ns, p, prm.nq1d), x=np.array(x),
                                sp=sp, bytes=b, g0=None, its=0, minres=0, done=False,
                                status=None, F=None)
        self.used += b
        self.peak = max(self.peak, self.used)
        self.admitted.append(np.array(x))  # the nodes as admitted
        return slot

    def step(self):
        for s in self.slots.values():
            if s["done"]:
                continue
            sp = s["sp"]
            x, rep = oracle.newton_solve(s["pb"], s["x"], rel_grad_tol=sp.rel_grad_tol,
                                         max_newton=1, max_minres=sp.max_minres,
                                         minres_rtol=sp.minres_rtol, g0_norm=s["g0"])
            s["x"], s["F"] = x, rep.get("F")
            if s["g0"] is None:
                s["g0"] = rep.get("g0_norm")
            s["its"] += rep["newton_its"]
            s["minres"] += rep["minres_its_total"]
            st = rep["status"]
            if st == OK or st != 5 or s["its"] >= sp.max_newton:
                s["done"], s["status"] = True, st

    def poll(self, slot):
        s = self.slots[slot]
        return s["done"], dict(status=s["status"], newton_its=s["its"],
                               minres_its_total=s["minres"], F=s["F"])

    def result(self, slot, x):
        x[:] = self.slots[slot]["x"]

    def release(self, slot):
        self.used -= self.slots.pop(slot)["bytes"]

    def info(self):
        return {"used": self.used}


def _stream():
    specs = [(2, 3, 1), (3, 2, 1), (2, 4, 2), (2, 3, 2), (3, 2, 1), (2, 5, 1), (2, 3, 1)]
    reqs, xs = [], []
    for k, (dim, n, p) in enumerate(specs):
        r = dict(dim=dim, n=n, p=p, nq=p + 2, seed=100 + k, t_arrive=0.002 * k)
        pb = oracle.Problem.box(dim, n, p, p + 2)
        x, _ = inputs.perturbed_box(dim, n, p, basis.gll_nodes(p), r["seed"],
                                    recipe="smooth", amp=0.05,
                                    is_valid=lambda x, pb=pb: pb.min_det(x) > 0)
        reqs.append(r)
        xs.append(x)
    return reqs, xs


def _describe(r):
    return request(r["dim"], r["n"], r["p"], r["nq"])


def _alone(r, x0, sp):
    pb = oracle.Problem.box(r["dim"], r["n"], r["p"], r["nq"])
    return oracle.newton_solve(pb, x0, rel_grad_tol=sp.rel_grad_tol, max_newton=sp.max_newton,
                               max_minres=sp.max_minres, minres_rtol=sp.minres_rtol)


def test_loop_matches_alone_and_respects_budget():
    reqs, xs = _stream()
    sp = solve_params(rel_grad_tol=1e-8, max_newton=50)
    total = sum(OraclePool.nbytes(_describe(r)[0]) for r in reqs)
    big = max(OraclePool.nbytes(_describe(r)[0]) for r in reqs)
    pool = OraclePool(max(big, total // 3), max_slots=3)
    work = [x.copy() for x in xs]
    summary, rec = serve.serve_loop(reqs, work, pool, sp, _describe)
    assert summary["solved"] == len(reqs) and summary["failed"] == 0
    assert summary["peak_bytes"] <= pool.budget < total and pool.peak <= pool.budget
    assert pool.busy > 0  # requests waited for room
    # FIFO: admitted in arrival order
    order = [next(k for k, x in enumerate(xs) if np.array_equal(a, x)) for a in pool.admitted]
    assert order == sorted(order) == list(range(len(reqs)))
    for k, (r, x0) in enumerate(zip(reqs, xs)):
        xo, ro = _alone(r, x0, sp)
        assert ro["status"] == OK and rec[k]["status"] == OK
        assert np.array_equal(work[k], xo)
        assert rec[k]["newton_its"] == ro["newton_its"]
        assert rec[k]["latency_ms"] >= 0


def test_failing_and_rejected_requests_stand_alone():
    reqs, xs = _stream()
    sp = solve_params(rel_grad_tol=1e-8, max_newton=50)
    ref, _ = serve.serve_loop(reqs, [x.copy() for x in xs], OraclePool(10 ** 9, 8), sp, _describe)
    # request 2 tangled: one interior node moved far outside its element
    bad = [x.copy() for x in xs]
    pb = oracle.Problem.box(2, 4, 2, 4)
    free = np.flatnonzero(~pb.ess)
    bad[2][free[len(free) // 2]] += 3.0
    assert not pb.min_det(bad[2]) > 0
    # and a request far larger than the budget
    reqs2 = list(reqs) + [dict(dim=3, n=8, p=4, nq=6, seed=1, t_arrive=0.001)]
    reqs2.sort(key=lambda r: r["t_arrive"])
    kbig = next(k for k, r in enumerate(reqs2) if r["n"] == 8)
    bad.insert(kbig, np.zeros(3 * 33 ** 3))
    budget = max(OraclePool.nbytes(_describe(r)[0]) for r in reqs)
    summary, rec = serve.serve_loop(reqs2, bad, OraclePool(budget, 8), sp, _describe)
    assert rec[kbig]["status"] == ERR_BUDGET and rec[kbig]["rejected"]
    ktan = [k for k, r in enumerate(reqs2) if r is reqs[2]][0]
    assert rec[ktan]["status"] == ERR_INVERTED
    assert summary["solved"] == len(reqs) - 1 and summary["failed"] == 2
    # every request counted in the percentiles, failures included
    assert summary["p99_ms"] is not None
    for k, r in enumerate(reqs2):
        if k in (kbig, ktan):
            continue
        j = reqs.index(r)
        xo, ro = _alone(r, xs[j], sp)
        assert rec[k]["status"] == OK and np.array_equal(bad[k], xo)
