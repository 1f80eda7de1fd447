"""The pooled (batched) path against the FP64 oracle.

A heterogeneous pool (2D and 3D, p = 1..4, FP64 and mixed precision, tensor
and compact storage, one slot with a random mask of fixed DoFs) is checked
slot by slot with the pool's own batched kernels (``tmop_pool_evaluate``):

* energy and min det, gradient, Hessian action (on a vector zero on the fixed
  DoFs and on one that is not) and diagonal at the initial mesh: 1e-11
  relative for FP64 slots and for the FP64 parts of mixed slots (energy,
  gradient), the FP32 bound for the mixed action and diagonal;
* the Hessian action and diagonal of pooled classes with more quadrature
  points than lanes (p = 4 with 7^3 points, p = 2 with 9^3), whose element
  kernels take the layer-chunked body: 1e-11 (FP64), the FP32 bound (mixed);
* the first Newton step (the pool's lockstep MINRES, line search and update)
  against the oracle's first Newton step, with MINRES allowed 200 iterations
  so that it stops at its tolerance: the same line-search decisions; for
  FP64 slots MINRES counts within one (near the stop threshold rounding can
  move the count), the step x0 - x1 within 1e-9 relative (the
  single-context MINRES parity bound) and the new energy within 1e-10 of the
  initial one.  A Krylov solve cut off by the iteration cap before it
  converges is no parity case: on the 3x4 Q4 quad mesh, 50 iterations leave
  the residual at 6e-5 and the oracle's own direction moves by 1e-5 when its
  action is perturbed at 1e-16, so two correct FP64 runs need not agree;
  for mixed slots, whose MINRES runs on an FP32 action, the step within
  1e-4 (about sqrt of FP32 epsilon, the accuracy of a Krylov solve with an
  operator perturbed at FP32 rounding) and the energy within 1e-6;
* the solves to |g|/|g0| <= 1e-10 (the paper's eps) against the oracle's
  Newton solves: final nodes within 1e-9 relative, final energy within
  1e-10 of the initial one;
* a served stream (``serve.serve``) of requests solved to 1e-10, each against
  the oracle's solve;
* each slot keeps its own MINRES tolerance: two slots of one mesh with
  different tolerances give, in one pool, what each gives alone.
"""
import numpy as np
import pytest

import oracle
from oracle import basis
from paper_2205_12721_amd import inputs
from tests.gpu_common import TOL64, TOLX, log, make_case, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL32 = 2e-6  # mixed precision: FP32 quadrature data and FP32 action

MIX = [
    dict(dim=3, ns=(3, 3, 2), p=1, nq=3, precision="fp64", storage="tensor", seed=81),
    dict(dim=3, ns=(2, 3, 3), p=2, nq=4, precision="mixed", storage="compact", seed=82),
    dict(dim=3, ns=(3, 2, 3), p=3, nq=5, precision="fp64", storage="compact", seed=83),
    dict(dim=3, ns=(2, 2, 2), p=4, nq=6, precision="mixed", storage="tensor", seed=84),
    dict(dim=2, ns=(5, 4), p=1, nq=3, precision="mixed", storage="tensor", seed=85),
    dict(dim=2, ns=(6, 5), p=2, nq=4, precision="fp64", storage="compact", seed=86),
    dict(dim=2, ns=(4, 5), p=3, nq=5, precision="mixed", storage="compact", seed=87),
    dict(dim=2, ns=(3, 4), p=4, nq=6, precision="fp64", storage="tensor", seed=88),
    dict(dim=3, ns=(3, 3, 3), p=2, nq=4, precision="fp64", storage="tensor", seed=89, mask=True),
]


def _case(c):
    pb, x = make_case(c["dim"], c["ns"], c["p"], c["nq"], seed=c["seed"],
                      recipe="smooth" if c["dim"] == 3 else "interior_jitter")
    mdev = None
    if c.get("mask"):
        import torch
        # boundary fixed plus a random third of the interior DoFs
        mask = pb.ess | (np.random.default_rng(c["seed"]).uniform(size=pb.ndof) < 0.3)
        pb = oracle.Problem(c["dim"], c["p"], c["nq"], pb.e2n, pb.nx, ess=mask)
        mdev = torch.as_tensor(mask.astype(np.uint8)).cuda()
    return pb, x, mdev


def _admit_all(cases, rel_grad_tol=1e-10, max_newton=200, minres_rtol=1e-12, bank=False,
               max_minres=50):
    from paper_2205_12721_amd.tmop import Pool, request, request_bytes, solve_params
    probs, reqs = [], []
    for c in cases:
        pb, x, mdev = _case(c)
        md, prm = request(c["dim"], c["ns"], c["p"], c["nq"], precision=c["precision"],
                          storage=c["storage"], ess=mdev if mdev is not None else "boundary")
        probs.append((pb, x))
        reqs.append((md, prm, mdev))
    total = sum(request_bytes(md, prm) for md, prm, _ in reqs)
    pool = Pool(8 * total if bank else total, len(cases), lanczos_bank=bank)
    slots, xs = [], []
    for (md, prm, mdev), (pb, x) in zip(reqs, probs):
        xd = to_dev(x)
        sp = solve_params(rel_grad_tol=rel_grad_tol, max_newton=max_newton, minres_rtol=minres_rtol,
                          max_minres=max_minres)
        slots.append(pool.admit(md, prm, sp, xd))
        xs.append(xd)
    return pool, probs, slots, xs


def test_pool_operators_match_oracle():
    pool, probs, slots, _ = _admit_all(MIX)
    for c, (pb, x), sl in zip(MIX, probs, slots):
        t = TOL32 if c["precision"] == "mixed" else TOL64
        xd = to_dev(x)
        F, md = pool.energy_mindet(sl, xd)
        eF = abs(F - pb.energy(x)) / pb.energy(x)
        emd = abs(md - pb.min_det(x)) / abs(pb.min_det(x))
        eg = rel(to_host(pool.gradient(sl, xd)), pb.gradient(x))
        pool.hessian_setup(sl, xd)
        v = inputs.gaussian_vector(pb.ndof, c["seed"] + 1, pb.ess)
        v_raw = inputs.gaussian_vector(pb.ndof, c["seed"] + 2)
        ey = rel(to_host(pool.hessian_apply(sl, to_dev(v))), pb.hvp(x, v))
        ey2 = rel(to_host(pool.hessian_apply(sl, to_dev(v_raw))), pb.hvp(x, v_raw))
        ed = rel(to_host(pool.hessian_diag(sl, xd)), pb.diag(x))
        log("pool slot", sl, c, "F %.1e mindet %.1e g %.1e Hv %.1e %.1e diag %.1e"
            % (eF, emd, eg, ey, ey2, ed))
        assert eF <= TOL64 and emd <= 1e-12 and eg <= TOL64
        assert ey <= t and ey2 <= t and ed <= t
    pool.close()


# classes with more points than lanes: the pool's element kernels run the
# layer-chunked body for FP64 compact data and the FP64 tensor at p = 4, the
# point-pass body otherwise
LAYERED = [
    dict(dim=3, ns=(2, 2, 2), p=4, nq=7, precision="fp64", storage="compact", seed=91),
    dict(dim=3, ns=(2, 2, 2), p=4, nq=7, precision="fp64", storage="tensor", seed=92),
    dict(dim=3, ns=(2, 3, 2), p=2, nq=9, precision="fp64", storage="compact", seed=93),
    dict(dim=3, ns=(2, 2, 2), p=4, nq=7, precision="mixed", storage="compact", seed=94),
]


def test_pool_layered_classes_match_oracle():
    pool, probs, slots, _ = _admit_all(LAYERED)
    for c, (pb, x), sl in zip(LAYERED, probs, slots):
        t = TOL32 if c["precision"] == "mixed" else TOL64
        xd = to_dev(x)
        pool.hessian_setup(sl, xd)
        v = inputs.gaussian_vector(pb.ndof, c["seed"] + 1, pb.ess)
        ey = rel(to_host(pool.hessian_apply(sl, to_dev(v))), pb.hvp(x, v))
        ed = rel(to_host(pool.hessian_diag(sl, xd)), pb.diag(x))
        log("pool slot", sl, c, "Hv %.1e diag %.1e" % (ey, ed))
        assert ey <= t and ed <= t
    pool.close()


def test_pool_first_newton_step_matches_oracle():
    pool, probs, slots, xs = _admit_all(MIX, max_newton=1, max_minres=200)
    while pool.step() > 0:
        pass
    res = []
    for c, (pb, x0), sl, xd in zip(MIX, probs, slots, xs):
        done, rep = pool.poll(sl)
        assert done and rep["newton_its"] == 1
        pool.result(sl, xd)
        x1 = to_host(xd)
        xo, ro = oracle.newton_solve(pb, x0, rel_grad_tol=1e-10, max_newton=1, max_minres=200)
        assert ro["newton_its"] == 1
        e = rel(x0 - x1, x0 - xo)
        log("first step", c, "its", rep["minres_its_total"], ro["minres_its_total"],
            "halvings", rep["halvings_total"], ro["halvings_total"], "step rel %.2e" % e,
            "F rel %.2e" % (abs(rep["F"] - ro["F"]) / ro["F0"]))
        eF = abs(rep["F"] - ro["F"]) / ro["F0"]
        res.append((c, rep, ro, e, eF))
    pool.close()
    for c, rep, ro, e, eF in res:
        assert rep["halvings_total"] == ro["halvings_total"]
        if c["precision"] == "fp64":
            assert abs(rep["minres_its_total"] - ro["minres_its_total"]) <= 1
            assert e <= 1e-9 and eF <= 1e-10
        else:
            assert e <= 1e-4 and eF <= 1e-6


@pytest.mark.parametrize("bank", [False, True])
def test_pool_solves_match_oracle(bank):
    pool, probs, slots, xs = _admit_all(MIX, bank=bank)
    while pool.step() > 0:
        pass
    for c, (pb, x0), sl, xd in zip(MIX, probs, slots, xs):
        done, rep = pool.poll(sl)
        assert done
        pool.result(sl, xd)
        xo, ro = oracle.newton_solve(pb, x0, rel_grad_tol=1e-10, max_newton=200)
        e = rel(to_host(xd), xo)
        log("pool solve", c, "bank", bank, "status", rep["status"], "newton", rep["newton_its"],
            ro["newton_its"], "x rel %.2e" % e)
        assert rep["status"] == 0 and ro["status"] == 0
        assert e <= TOLX
        assert abs(rep["F"] - ro["F"]) <= 1e-10 * ro["F0"]
    pool.close()


def test_served_requests_match_oracle():
    from paper_2205_12721_amd import serve
    reqs = inputs.serving_stream(500.0, count=6, seed=21, max_n3=6)
    xs = serve.make_inputs(reqs)
    summary, rec = serve.serve(reqs, xs, serve.budget_for(reqs, factor=0.5), max_slots=4,
                               rel_grad_tol=1e-10, max_newton=200)
    log("served", summary)
    for r, x0, out in zip(reqs, xs, rec):
        pb = oracle.Problem.box(r["dim"], r["n"], r["p"], r["nq"])
        xo, ro = oracle.newton_solve(pb, x0, rel_grad_tol=1e-10, max_newton=200)
        e = rel(to_host(out["x"]), xo)
        log("request", r["dim"], r["n"], r["p"], "newton", out["newton_its"], ro["newton_its"],
            "x rel %.2e" % e)
        assert out["status"] == 0 and ro["status"] == 0
        assert e <= TOLX


def test_per_slot_minres_tolerance():
    """A slot's MINRES stops at its own tolerance, whatever the other slots ask for."""
    from paper_2205_12721_amd.tmop import Pool, request, request_bytes, solve_params
    c = MIX[2]
    pb, x, _ = _case(c)
    md, prm = request(c["dim"], c["ns"], c["p"], c["nq"], precision=c["precision"], storage=c["storage"])
    b = request_bytes(md, prm)

    def run(rtols):
        pool = Pool(len(rtols) * b, len(rtols))
        xs = [to_dev(x) for _ in rtols]
        sl = [pool.admit(md, prm, solve_params(rel_grad_tol=1e-10, minres_rtol=t), xd)
              for t, xd in zip(rtols, xs)]
        while pool.step() > 0:
            pass
        out = []
        for s, xd in zip(sl, xs):
            pool.result(s, xd)
            out.append((to_host(xd), pool.poll(s)[1]))
        pool.close()
        return out

    tight, loose = run([1e-12])[0], run([1e-3])[0]
    both = run([1e-3, 1e-12])
    assert tight[1]["minres_its_total"] > loose[1]["minres_its_total"]
    assert np.array_equal(both[0][0], loose[0]) and np.array_equal(both[1][0], tight[0])
    assert both[0][1]["minres_its_total"] == loose[1]["minres_its_total"]
    assert both[1][1]["minres_its_total"] == tight[1]["minres_its_total"]
