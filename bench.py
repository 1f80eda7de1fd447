"""Benchmark of the PA-TMOP hot path on one MI355X.

A step is one Newton iteration of the TMOP solve on the initial perturbed mesh
with a fixed number of MINRES iterations (20, as in the paper's throughput
runs of Sec. 4.1): energy and det check, gradient, Hessian setup, Jacobi
diagonal, 20 Hessian actions inside Jacobi-preconditioned MINRES, line search
and node update.  Every step restarts from the same initial mesh, so each
does the same work.

Reported metric (``value``): Hessian-action throughput in GDoF/s, the unique
DoFs d*N_x over the median time of one standalone ``tmop_hessian_apply`` call
(FP64, the paper's packed-tensor storage; 30 calls after one setup and 3
warm-up actions, each call bracketed by HIP events recorded on the library's
stream; the setup is not timed).  ``roofline`` is the same action's
algorithmic HBM bytes over its mean time back to back; the mixed-precision and
compact-storage variants, the 64^3 Q2 and 32^3 Q4 workloads, the 2D 8x8 Q2
ten-iteration solve, the batched and served forms and the Kershaw benchmark
are reported beside it, and the plain FP64 oracle is timed on the host cores
as a reference baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --apply-only [--workload c2|c3a|c3b|kershaw1..4] [--reps 10]
           [--storage tensor|compact|both] [--precision fp64|mixed|both] [--copy-ref]
           [--all-kernels [--mfma]]
       python bench.py --batch-only [--batch-meshes 256]

``--apply-only`` runs only the Hessian action, for profilers: one setup per
variant on the workload's mesh, then 2 x reps actions back to back on the
library's stream (``tmop_time_apply``), printing the mean device time per
action; ``--copy-ref`` adds a plain 1 GiB device-to-device copy, a kernel of
known traffic to scale hardware byte counters by; ``--all-kernels`` also runs
the energy, gradient, setup and diagonal kernels reps times per variant, and
``--mfma`` the FP64 energy, gradient and setup again with their forward sweeps
on the matrix cores (``tmop_set_sweeps``).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s

# HBM bytes per Hessian action (element kernel + gather), from two rocprofv3
# --pmc runs of the standalone action (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch), each scaled by the same counter's reading for a device copy of
# known size.  Valid only for the kernel sources they were taken on: the
# entry names the SHA-256 of the kernel sources (csrc_sha256()) and is
# reported as null once they differ.  Summary and commands:
# profiles/hessian_apply_traffic_24cube_q3.md.
_SHA_C2 = "a40a481d36b6bc943531a4a21cf3d3373af65a4006afbdadefbf6a753cfb6637"
TRAFFIC = {
    ("c2", "tensor_fp64"): {"bytes": 714546511, "elements_per_workgroup": 2,
                        "csrc_sha256": _SHA_C2},
    ("c2", "tensor_mixed"): {"bytes": 371956710, "elements_per_workgroup": 2,
                        "csrc_sha256": _SHA_C2},
    ("c2", "compact_fp64"): {"bytes": 249300935, "elements_per_workgroup": 2,
                        "csrc_sha256": _SHA_C2},
    ("c2", "compact_mixed"): {"bytes": 137360473, "elements_per_workgroup": 2,
                        "csrc_sha256": _SHA_C2},
}


# Sources of the device code a single-context Hessian action runs (its element
# kernels, the node gather and what they include); host-only files (capi.hip,
# batch.hip) and other element classes' units do not change the measured kernels.
ACTION_SOURCES = ("gather.hpp", "kernels3d.hpp", "kernels2d.hpp", "k2.hip", "k3_p1.hip", "mfma3.hpp",
                  "k3_p2.hip", "k3_p3.hip", "k3_p4.hip", "ops.hpp", "tiles3.hpp",
                  "tmop_dev.hpp", "vec.hip", "vec.hpp")


def csrc_sha256():
    import hashlib
    d = os.path.join(ROOT, "paper_2205_12721_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(ACTION_SOURCES):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def traffic_for(variant, workload, epb):
    t = TRAFFIC.get((workload, variant))
    if not t or t["csrc_sha256"] != csrc_sha256() or t["elements_per_workgroup"] != epb:
        return None
    return t["bytes"]

WORKLOADS = {
    # name: (inputs config, dim, n, p, nq)
    "c2": ("c2", 3, 24, 3, 5),
    "c3a": ("c3a", 3, 64, 2, 4),
    "c3b": ("c3b", 3, 32, 4, 6),
    "c1": ("c1", 2, 8, 2, 4),
}
# --apply-only also takes the Kershaw meshes (24^3, 9^3 points, sliding boundary)
KERSHAW_WORKLOADS = {"kershaw%d" % p: p for p in (1, 2, 3, 4)}


_T0 = time.monotonic()


def log(*a):
    print("[%7.1f s]" % (time.monotonic() - _T0), *a, file=sys.stderr, flush=True)


def copy_bandwidth(torch, nbytes=4 << 30, reps=5):
    """Device-to-device copy bandwidth (read + write bytes / time), GB/s."""
    n = nbytes // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    t = s.elapsed_time(e) / 1e3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / t / 1e9


def run_steps(ctx, x, x0, steps, n_minres):
    import torch
    acc = dict(t_apply_ms=0.0, t_apply_elem_ms=0.0, n_apply=0, t_setup_ms=0.0,
               t_minres_ms=0.0, t_linesearch_ms=0.0, halvings=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x.copy_(x0)
        rep = ctx.newton_step(x, n_minres=n_minres, jacobi=True)
        for k in ("t_apply_ms", "t_apply_elem_ms", "n_apply", "t_setup_ms", "t_minres_ms",
                  "t_linesearch_ms"):
            acc[k] += rep[k]
        acc["halvings"] += rep["halvings_total"]
    torch.cuda.synchronize()
    acc["wall_s"] = time.perf_counter() - t0
    acc["last"] = rep
    return acc


def instrumented_steps(ctx, x, x0, n_minres, steps=2):
    """Steps with HIP events around every Hessian action inside MINRES (their
    per-action time); kept out of the timed steps, which record no events."""
    ctx.set_timing(True)
    acc = run_steps(ctx, x, x0, steps, n_minres)
    ctx.set_timing(False)
    return acc


def time_actions(ctx, x, v, reps):
    """Standalone Hessian actions after one setup at x, with the autotuned tile
    shape: 3 warm-up actions, then (element kernel mean, whole-action mean) in ms
    over `reps` actions each, the elements per workgroup used, and the median in
    ms of `reps` single calls of tmop_hessian_apply, each bracketed by HIP events
    recorded on the context's stream."""
    import numpy as np
    import torch
    y = torch.empty_like(v)
    ctx.hessian_setup(x)
    epb = ctx.autotune(v, y, 5)
    ctx.time_apply(v, y, 3)
    e, t = ctx.time_apply(v, y, reps)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record(ctx._stream)
        ctx.hessian_apply(v, y)
        b.record(ctx._stream)
    torch.cuda.synchronize()
    med = float(np.median([a.elapsed_time(b) for a, b in evs]))
    return e, t, epb, med


def sweep_fma(dim, p, nq):
    """Multiply-adds of the sum-factorized forward (or backward) sweeps of one
    element, all components (Sec. 3.2): per component
    2 n_i^3 n_q + 3 n_i^2 n_q^2 + 3 n_i n_q^3 in 3D, 2 n_i^2 n_q + 2 n_i n_q^2 in 2D."""
    ni = p + 1
    if dim == 3:
        return 3 * (2 * ni ** 3 * nq + 3 * ni ** 2 * nq ** 2 + 3 * ni * nq ** 3)
    return 2 * (2 * ni ** 2 * nq + 2 * ni * nq ** 2)


def kernel_leg(ctx, x, ne, nqe, S, dim, p, nq, reps=20):
    """The other steps of the path on the headline context, each call timed alone
    (median of `reps`, HIP events on the context's stream): setup (a8), gradient
    (a7), energy (a6), diagonal (a10), and the two fused passes the Newton step
    runs, each beside the pair of calls it replaces: setup + diagonal
    (tmop_hessian_setup_diag, the Jacobi preconditioner's) and energy +
    gradient (tmop_energy_gradient, the line search's).  Sweep GFLOP/s counts
    only the sum-factorized sweeps (2 FLOP per multiply-add), not the point
    stage."""
    import numpy as np
    import torch
    g = torch.empty_like(x)
    d = torch.empty_like(x)

    def med(f):
        for _ in range(3):
            f()
        t = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(ctx._stream)
            f()
            b.record(ctx._stream)
            b.synchronize()
            t.append(a.elapsed_time(b) * 1e3)
        return float(np.median(t))

    fw = sweep_fma(dim, p, nq) * ne * 2.0   # FLOP of one set of sweeps over the mesh
    t_setup = med(lambda: ctx.hessian_setup(x))
    t_grad = med(lambda: ctx.gradient(x, g))
    t_en = med(lambda: ctx.energy(x))
    ctx.hessian_setup(x)
    t_diag = med(lambda: ctx.hessian_diag(d))
    t_sd_pair = med(lambda: (ctx.hessian_setup(x), ctx.hessian_diag(d)))
    t_sd = med(lambda: ctx.hessian_setup_diag(x, d))
    t_eg_pair = med(lambda: (ctx.energy(x), ctx.gradient(x, g)))
    t_eg = med(lambda: ctx.energy_gradient(x, g))
    tens = ne * nqe * S * 8
    r2 = lambda v: round(v, 2)  # noqa: E731
    return {
        "setup": {"us": r2(t_setup), "tensor_GB_s_written": r2(tens / t_setup / 1e3),
                  "sweep_GFLOP_s": r2(fw / t_setup / 1e3)},
        "gradient": {"us": r2(t_grad), "GDoF_s": r2(ctx.ndof / t_grad / 1e3),
                     "sweep_GFLOP_s": r2(2 * fw / t_grad / 1e3)},
        "energy": {"us": r2(t_en), "sweep_GFLOP_s": r2(fw / t_en / 1e3),
                   "note": "includes the copy of the result to the host"},
        "diagonal": {"us": r2(t_diag), "tensor_GB_s_read": r2(tens / t_diag / 1e3)},
        "setup_diag": {"us": r2(t_sd), "separate_calls_us": r2(t_sd_pair)},
        "energy_gradient": {"us": r2(t_eg), "separate_calls_us": r2(t_eg_pair),
                            "note": "both include the copy of the scalars to the host"},
        "action_GFLOP_s": None,
    }


def roofline(ne, nqe, S, ndof, tbytes, elem_ms, total_ms, traffic=None):
    t_app = total_ms / 1e3
    t_elem = elem_ms / 1e3
    b_alg = ne * nqe * S * tbytes + 2 * ndof * 8          # tensor + v in + y out
    b_elem = ne * nqe * S * tbytes + ndof * 8             # tensor + v in
    achieved = b_alg / t_app / 1e9
    return {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": "Hessian action = element kernel k3_apply + node gather k_gather",
        "alg_bytes_per_launch": int(b_alg),
        "avg_us": round(t_app * 1e6, 2),
        "elem_avg_us": round(t_elem * 1e6, 2),
        "elem_achieved_GBs": round(b_elem / t_elem / 1e9, 1),
    }


def cpu_baseline(cfg, x, v, seconds):
    import numpy as np  # noqa: F401
    import oracle
    _, dim, n, p, nq = cfg
    pb = oracle.Problem.box(dim, n, p, nq)
    y = pb.hvp(x, v)  # warm up; the action is kept for the precision leg
    reps, t0 = 0, time.perf_counter()
    while True:
        pb.hvp(x, v)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    cores = oracle.num_threads()
    # the oracle's energy (with the det check) and gradient on the same mesh
    t2 = time.perf_counter()
    pb.energy(x)
    t_en = time.perf_counter() - t2
    t2 = time.perf_counter()
    pb.gradient(x)
    t_gr = time.perf_counter() - t2
    # the same oracle on one thread, two actions
    oracle.set_num_threads(1)
    t1 = time.perf_counter()
    for _ in range(2):
        pb.hvp(x, v)
    t1 = time.perf_counter() - t1
    oracle.set_num_threads(cores)
    return {
        "value": round(pb.ndof * reps / el / 1e9, 6),
        "unit": "GDoF/s",
        "cores": cores,
        "kind": "oracle",
        "sample": "%d Hessian actions of the FP64 oracle (direct, not sum-factorized) on the "
                  "same mesh and vector, %.1f s" % (reps, el),
        "one_thread_value": round(pb.ndof * 2 / t1 / 1e9, 6),
        "energy_ms": round(t_en * 1e3, 2),
        "gradient_GDoF_s": round(pb.ndof / t_gr / 1e9, 6),
        "cpu_model": cpu_model(),
    }, y


def config1_leg(with_oracle):
    """The 2D 8x8 Q2 mu_2 configuration: 10 Newton-MINRES iterations (no early
    stop) on the GPU, wall time of the solve; with the oracle the same solve on
    the host, its time and the relative difference of the final nodes."""
    import numpy as np
    import torch

    from paper_2205_12721_amd import inputs
    from paper_2205_12721_amd.tmop import Context, basis_nodes
    c = inputs.CONFIGS["c1"]
    ctx = Context(c["dim"], c["n"], c["p"], c["nq"])
    buf = torch.empty(ctx.ndof, dtype=torch.float64, device="cuda")

    def valid(xh):
        buf.copy_(torch.as_tensor(xh))
        return ctx.min_det(buf) > 0

    xh, _ = inputs.config_mesh("c1", basis_nodes(c["p"]), is_valid=valid)
    x = torch.as_tensor(xh).cuda()
    for _ in range(2):  # warm-up solves
        buf.copy_(x)
        ctx.solve(buf, rel_grad_tol=0.0, max_newton=10)
    torch.cuda.synchronize()
    buf.copy_(x)
    t0 = time.perf_counter()
    rep = ctx.solve(buf, rel_grad_tol=0.0, max_newton=10)
    torch.cuda.synchronize()
    out = {"mesh": "2D 8x8 Q2, 4x4 Gauss-Legendre points, mu_2", "dofs": ctx.ndof,
           "gpu_ms": round((time.perf_counter() - t0) * 1e3, 3),
           "newton_its": rep["newton_its"], "minres_its": rep["minres_its_total"]}
    if with_oracle:
        import oracle
        pb = oracle.Problem.box(c["dim"], c["n"], c["p"], c["nq"])
        t0 = time.perf_counter()
        xo, ro = oracle.newton_solve(pb, xh, rel_grad_tol=0.0, max_newton=10)
        out["oracle_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
        out["oracle_newton_its"] = ro["newton_its"]
        xg = buf.cpu().numpy()
        out["x_rel_diff_vs_oracle"] = float("%.3g" % (np.linalg.norm(xg - xo) / np.linalg.norm(xo)))
    ctx.close()
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def precision_leg(cfg, x0, v_host, y_oracle, max_newton=100):
    """Error of each Hessian-action variant against the FP64 oracle's action (same mesh
    and vector), and FP64 vs mixed full solves to |g|/|g0| <= 1e-8 on the same mesh:
    time, Newton/MINRES counts and the relative final-energy difference."""
    import numpy as np
    import torch
    from paper_2205_12721_amd.tmop import Context
    _, dim, n, p, nq = cfg
    v = torch.as_tensor(v_host).cuda()
    yo = np.asarray(y_oracle)
    out = {"hvp_rel_err_vs_oracle": {}}
    for storage in ("tensor", "compact"):
        for prec in ("fp64", "mixed"):
            c = Context(dim, n, p, nq, precision=prec, storage=storage)
            c.hessian_setup(x0)
            y = c.hessian_apply(v).cpu().numpy()
            c.close()
            out["hvp_rel_err_vs_oracle"]["%s_%s" % (storage, prec)] = float(
                np.linalg.norm(y - yo) / np.linalg.norm(yo))
    sol = {}
    for storage, prec in (("tensor", "fp64"), ("tensor", "mixed"), ("compact", "fp64"),
                          ("compact", "mixed")):
        c = Context(dim, n, p, nq, precision=prec, storage=storage)
        x = x0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = c.solve(x, rel_grad_tol=1e-8, max_newton=max_newton)
        torch.cuda.synchronize()
        sol["%s_%s" % (storage, prec)] = {
            "seconds": round(time.perf_counter() - t0, 4), "status": rep["status_name"],
            "newton_its": rep["newton_its"], "minres_its": rep["minres_its_total"],
            "F0": rep["F0"], "F": rep["F"], "x": x}
        c.close()
    ref = sol["tensor_fp64"]
    for k, r in sol.items():
        r["rel_final_energy_diff_vs_tensor_fp64"] = abs(r["F"] - ref["F"]) / abs(ref["F"])
        r["rel_node_diff_vs_tensor_fp64"] = float((r["x"] - ref["x"]).norm() / ref["x"].norm())
    for r in sol.values():
        del r["x"]
    out["solve_to_1e-8"] = sol
    return out


def config3_leg(name, apply_reps, steps, n_minres, n_sample=400):
    """The 6.44 M-DoF workloads (64^3 Q2 with 4^3 points, 32^3 Q4 with 6^3): every
    action variant (tensor / compact storage x FP64 / mixed) timed as the headline
    (autotuned tile, median single call, back-to-back mean and its HBM roofline), a
    Newton step with n_minres MINRES iterations in FP64 and in mixed precision, and
    solves to |g|/|g0| <= 1e-8 with each variant, whose final energy is compared with
    the FP64 tensor solve's (bar: 1e-10 relative).  Returns the results, the host mesh
    and vector, the sampled node ids and each variant's action at those DoFs (for the
    oracle comparison in the CPU-baseline leg)."""
    import numpy as np
    import torch
    from paper_2205_12721_amd import inputs
    from paper_2205_12721_amd.tmop import Context, basis_nodes
    c = inputs.CONFIGS[name]
    dim, n, p, nq = c["dim"], c["n"], c["p"], c["nq"]
    ne, nqe, S = n ** dim, nq ** dim, dim * dim * (dim * dim + 1) // 2
    probe = Context(dim, n, p, nq, precision="mixed", storage="compact")
    buf = torch.empty(probe.ndof, dtype=torch.float64, device="cuda")

    def valid(xh):
        buf.copy_(torch.as_tensor(xh))
        return probe.min_det(buf) > 0

    xh, info = inputs.config_mesh(name, basis_nodes(p), is_valid=valid)
    ndof = probe.ndof
    probe.close()
    del buf
    x0 = torch.as_tensor(xh).cuda()
    x = torch.empty_like(x0)
    vh = inputs.gaussian_vector(ndof, c["vec_seed"])
    v = torch.as_tensor(vh).cuda()
    rng = np.random.default_rng(77)
    nx = ndof // dim
    nodes = np.sort(rng.choice(nx, size=n_sample, replace=False))
    idx = np.concatenate([a * nx + nodes for a in range(dim)])
    res = {"workload": "3D hex box %d^3, Q%d, %d^3 Gauss-Legendre points, mu_303" % (n, p, nq),
           "dofs": ndof, "mesh_tries": info["tries"], "variants": {}}
    sampled = {}
    for storage in ("tensor", "compact"):
        for prec in ("fp64", "mixed"):
            key = "%s_%s" % (storage, prec)
            cv = Context(dim, n, p, nq, precision=prec, storage=storage)
            em, tm, eb, mm = time_actions(cv, x0, v, apply_reps)
            y = torch.empty_like(v)
            cv.hessian_apply(v, y)
            sampled[key] = y.cpu().numpy()[idx]
            sv = S if storage == "tensor" else 13
            r = {"value": round(ndof / (mm / 1e3) / 1e9, 3), "unit": "GDoF/s",
                 "elements_per_workgroup": eb,
                 "roofline": roofline(ne, nqe, sv, ndof, 8 if prec == "fp64" else 4, em, tm)}
            r["roofline"]["median_action_us"] = round(mm * 1e3, 2)
            if storage == "tensor":
                run_steps(cv, x, x0, 1, n_minres)
                acc = run_steps(cv, x, x0, steps, n_minres)
                r["newton_step_ms"] = round(acc["wall_s"] / steps * 1e3, 3)
            x.copy_(x0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep = cv.solve(x, rel_grad_tol=1e-8, max_newton=100)
            torch.cuda.synchronize()
            r["solve_to_1e-8"] = {"seconds": round(time.perf_counter() - t0, 4),
                                  "status": rep["status_name"], "newton_its": rep["newton_its"],
                                  "minres_its": rep["minres_its_total"], "F0": rep["F0"],
                                  "F": rep["F"]}
            r["_x"] = x.clone()
            res["variants"][key] = r
            cv.close()
            log("[bench] %s %s %s: %.2f GDoF/s, frac %.3f" % (name, storage, prec, r["value"],
                                                                r["roofline"]["frac"]))
    ref = res["variants"]["tensor_fp64"]
    worst = 0.0
    for k, r in res["variants"].items():
        sv = r["solve_to_1e-8"]
        sv["rel_final_energy_diff_vs_tensor_fp64"] = abs(sv["F"] - ref["solve_to_1e-8"]["F"]) / abs(
            ref["solve_to_1e-8"]["F"])
        sv["rel_node_diff_vs_tensor_fp64"] = float((r["_x"] - ref["_x"]).norm() / ref["_x"].norm())
        worst = max(worst, sv["rel_final_energy_diff_vs_tensor_fp64"])
    for r in res["variants"].values():
        del r["_x"]
    res["max_rel_final_energy_diff"] = worst
    res["final_energy_within_1e-10"] = bool(worst <= 1e-10)
    return res, (name, xh, vh, nodes, idx, sampled)


def config3_oracle_error(ref):
    """CPU-baseline leg of a 6.44 M-DoF workload: the oracle's Hessian action at the
    sampled DoFs (the oracle evaluates only the elements touching the sampled nodes,
    whose entries equal the full operator's there) and each GPU variant's error
    against it (relative l2 and max-entry measures over the sampled DoFs)."""
    import numpy as np
    import oracle
    from paper_2205_12721_amd import inputs
    name, xh, vh, nodes, idx, sampled = ref
    c = inputs.CONFIGS[name]
    pb = oracle.Problem.box(c["dim"], c["n"], c["p"], c["nq"])  # boundary fixed, as the GPU's
    t0 = time.perf_counter()
    sub = oracle.restrict_to_nodes(pb, nodes)
    yo = sub.hvp(xh, vh)[idx]
    out = {"sampled_nodes": int(nodes.size), "oracle_seconds": round(time.perf_counter() - t0, 2)}
    for k, y in sampled.items():
        d = y - yo
        out[k] = {"rel_l2": float(np.linalg.norm(d) / np.linalg.norm(yo)),
                  "rel_max": float(np.abs(d).max() / np.abs(yo).max())}
    return out


def batch_leg(count, sequential=True):
    """256 independent hex meshes (log-uniform sizes, p = 1..4, n_q = p+2, mu_303):
    one batched mixed-precision solve (one graph launch per Newton step) vs
    one-mesh-at-a-time FP64 solves (skipped with sequential=False)."""
    import torch
    from paper_2205_12721_amd import inputs
    from paper_2205_12721_amd.tmop import Context, basis_nodes, batch_solve, request, solve_params
    specs = inputs.batch_specs(count, seed=5)
    xs = [inputs.perturbed_box(3, s["n"], s["p"], basis_nodes(s["p"]), s["seed"], recipe="smooth",
                               amp=0.05)[0] for s in specs]
    ndof = sum(x.size for x in xs)
    reqs = [request(3, s["n"], s["p"], s["nq"], precision="mixed", storage="compact") for s in specs]
    sps = [solve_params(rel_grad_tol=1e-8, max_newton=100) for _ in specs]
    xd = [torch.as_tensor(x).cuda() for x in xs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = batch_solve(reqs, xd, sps)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    if not sequential:
        return {"meshes": count, "dofs_total": int(ndof), "batched_mixed_s": round(tb, 4),
                "solved_batched": sum(1 for r in reps if r["status"] == 0),
                "newton_its_batched": int(sum(r["newton_its"] for r in reps))}
    t0 = time.perf_counter()
    seq = []
    for s, x in zip(specs, xs):
        ctx = Context(3, s["n"], s["p"], s["nq"])
        xs1 = torch.as_tensor(x).cuda()
        seq.append(ctx.solve(xs1, rel_grad_tol=1e-8, max_newton=100))
        ctx.close()
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    ok = [k for k in range(count) if reps[k]["status"] == 0 and seq[k]["status"] == 0]
    dF = [abs(reps[k]["F"] - seq[k]["F"]) / max(abs(seq[k]["F"]), 1e-300) for k in ok]
    return {
        "meshes": count, "dofs_total": int(ndof),
        "batched_mixed_s": round(tb, 4), "sequential_fp64_s": round(ts, 4),
        "speedup": round(ts / tb, 2),
        "solved_batched": sum(1 for r in reps if r["status"] == 0),
        "solved_sequential": sum(1 for r in seq if r["status"] == 0),
        "max_rel_final_energy_diff": float(max(dF)) if dF else None,
        "newton_its_batched": int(sum(r["newton_its"] for r in reps)),
        "newton_its_sequential": int(sum(r["newton_its"] for r in seq)),
    }


# Served pools: resident MINRES Lanczos vectors on, with an HBM budget of 4x
# the requests' base regions (room for every resident slot's vectors).
SERVE_BUDGET_FACTOR = 4.0


def serve_leg(rates, nreq):
    """The served stream (Poisson arrivals of mixed 2D/3D requests, the same
    requests at every rate, arrival times one unit-rate stream divided by the
    rate) through the pool, and the same stream through a one-at-a-time FP64
    loop, at every rate: p50/p99 latency (every request counted, a failed one at
    the time its result was known) and solves/s of both."""
    from paper_2205_12721_amd import inputs, serve
    base = inputs.serving_stream(1.0, count=nreq, seed=6, same_requests=True)
    t0 = time.perf_counter()
    xs = serve.make_inputs(base)
    gen_s = time.perf_counter() - t0
    budget = serve.budget_for(base, factor=SERVE_BUDGET_FACTOR, cap=64 << 30)
    r3 = lambda v: None if v is None else round(v, 3)  # noqa: E731
    rows = []
    for rate in rates:
        reqs = [dict(r, t_arrive=r["t_arrive"] / rate) for r in base]
        s, _ = serve.serve(reqs, xs, budget, max_slots=min(512, nreq), lanczos_bank=True)
        q, _ = serve.sequential(reqs, xs)
        rows.append({
            "rate_per_s": rate, "requests": nreq,
            "p50_ms": r3(s["p50_ms"]), "p99_ms": r3(s["p99_ms"]),
            "solves_per_s": r3(s["solves_per_s"]), "solved": s["solved"], "ticks": s["ticks"],
            "solved_p99_ms": r3(s["solved_p99_ms"]),
            "sequential_fp64": {"p50_ms": r3(q["p50_ms"]), "p99_ms": r3(q["p99_ms"]),
                                "solves_per_s": r3(q["solves_per_s"]), "solved": q["solved"]},
        })
        log("[bench] serve rate", rate, "p50", rows[-1]["p50_ms"], "p99", rows[-1]["p99_ms"],
            "sequential p50", rows[-1]["sequential_fp64"]["p50_ms"], "p99",
            rows[-1]["sequential_fp64"]["p99_ms"])
    return {"requests_per_rate": nreq, "budget_bytes": budget,
            "redrawn_inputs": int(sum(r["redraws"] for r in base)),
            "input_generation_s": round(gen_s, 2),
            "latency_rule": "arrival to result-ready (end of the tick that finished the solve); "
                            "every request counted, a failed one at the time its result was known",
            "max_newton": 200, "rel_grad_tol": 1e-8, "sweep": rows}


# Sec. 4.1, Table tab_kershaw_baseline: GPU runs on 4 V100s with (PA*) and without
# (PA) the Jacobi preconditioner, for context: (seconds, Newton its, MINRES its)
KERSHAW_PAPER = {
    True: {1: (0.4, 11, 203), 2: (0.9, 18, 507), 3: (3.9, 41, 1536), 4: (8.5, 70, 3110)},
    False: {1: (0.5, 19, 284), 2: (1.7, 29, 1107), 3: (4.7, 44, 2060), 4: (7.8, 67, 3139)},
}


def kershaw_leg(orders, storage="compact", cuts=()):
    """Kershaw benchmark (Sec. 4.1): 24^3 hexes, eps_y = eps_z = 0.3, 9^3 points per
    element, mu_303, at most 50 MINRES iterations per Newton step, with the Jacobi
    preconditioner ("PA*") and without ("PA"), stop at |g|/|g0| <= 1e-10; boundary nodes
    slide along their faces.  Gauss-Legendre points, and for the unpreconditioned solve
    also the 9-point Gauss-Lobatto rule ("PA_gll"); with ``cuts`` also the preconditioned
    solve with MINRES cut at that many iterations per Newton step ("PA*_minresN").  Time to
    solution on one GPU, FP64, next to the paper's 4-V100 numbers (context, not a
    like-for-like target)."""
    import torch
    from paper_2205_12721_amd import inputs
    from paper_2205_12721_amd.tmop import Context, basis_nodes
    ns = (24, 24, 24)
    res = {"storage": storage}
    rows = [(True, "PA*", "gl", 50), (False, "PA", "gl", 50), (False, "PA_gll", "gll", 50)]
    rows += [(True, "PA*_minres%d" % c, "gl", c) for c in cuts]
    for jac, key, quad, max_minres in rows:
        res[key] = {}
        for p in orders:
            mask = torch.as_tensor(inputs.sliding_mask(ns, p)).cuda()
            ctx = Context(3, ns, p, 9, ess=mask, storage=storage, quad=quad)
            x0 = torch.as_tensor(inputs.kershaw_nodes(ns, p, basis_nodes(p), 0.3, 0.3)).cuda()
            x = x0.clone()
            ctx.solve(x, rel_grad_tol=1e-10, max_newton=1, max_minres=2)  # warm-up
            x.copy_(x0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep = ctx.solve(x, rel_grad_tol=1e-10, max_newton=300, max_minres=max_minres, jacobi=jac)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ctx.close()
            pt, pn, pm = KERSHAW_PAPER[jac].get(p, (None, None, None))
            res[key]["p%d" % p] = {
                "dofs": 3 * (24 * p + 1) ** 3, "seconds": round(dt, 3),
                "status": rep["status_name"], "newton_its": rep["newton_its"],
                "minres_its": rep["minres_its_total"], "F0": rep["F0"], "F": rep["F"],
                "g_rel": rep["g_norm"] / rep["g0_norm"],
                "paper_4xV100_seconds": pt, "paper_newton_its": pn, "paper_minres_its": pm,
            }
    return res


def apply_only(args):
    """Only the Hessian action on a workload's mesh (for rocprofv3 runs)."""
    import torch

    from paper_2205_12721_amd import inputs
    from paper_2205_12721_amd.tmop import Context, basis_nodes
    st = ["tensor", "compact"] if args.storage == "both" else [args.storage]
    pr = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    ckw = {}
    if args.workload in KERSHAW_WORKLOADS:
        dim, n, p, nq = 3, (24, 24, 24), KERSHAW_WORKLOADS[args.workload], 9
        ckw["ess"] = torch.as_tensor(inputs.sliding_mask(n, p)).cuda()
        xh = inputs.kershaw_nodes(n, p, basis_nodes(p), 0.3, 0.3)
        vec_seed = 200 + p
    else:
        c = inputs.CONFIGS[args.workload]
        dim, n, p, nq = c["dim"], c["n"], c["p"], c["nq"]
        probe = Context(dim, n, p, nq)
        buf = torch.empty(probe.ndof, dtype=torch.float64, device="cuda")

        def valid(xh):
            buf.copy_(torch.as_tensor(xh))
            return probe.min_det(buf) > 0

        xh, _ = inputs.config_mesh(args.workload, basis_nodes(p), is_valid=valid)
        probe.close()
        vec_seed = c["vec_seed"]
    x = torch.as_tensor(xh).cuda()
    v = torch.as_tensor(inputs.gaussian_vector(x.numel(), vec_seed)).cuda()
    y = torch.empty_like(v)
    out = {}
    for s in st:
        for q in pr:
            ctx = Context(dim, n, p, nq, precision=q, storage=s, **ckw)
            ctx.hessian_setup(x)
            ctx.hessian_apply(v, y)
            if args.all_kernels:
                # the other element kernels of the path, reps calls each
                for _ in range(args.reps):
                    ctx.energy(x)
                    ctx.gradient(x, y)
                    ctx.hessian_setup(x)
                    ctx.hessian_diag(y)
                if args.mfma and q == "fp64" and dim == 3 and nq <= 5:
                    # and with the forward sweeps on the matrix cores
                    ctx.set_sweeps("mfma")
                    for _ in range(args.reps):
                        ctx.energy(x)
                        ctx.gradient(x, y)
                        ctx.hessian_setup(x)
                    ctx.set_sweeps("pencil")
                    ctx.hessian_setup(x)
            elem, tot = ctx.time_apply(v, y, args.reps)
            out["%s_%s" % (s, q)] = dict(elem_us=round(elem * 1e3, 2), total_us=round(tot * 1e3, 2),
                                         elements_per_workgroup=ctx.tile_epb())
            log("[apply-only]", s, q, out["%s_%s" % (s, q)])
            ctx.close()
    if args.copy_ref:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_ref_bytes_each_way"] = src.numel() * 8
    print(json.dumps(dict(workload=args.workload, dofs=int(x.numel()), actions=out)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--minres", type=int, default=20)
    ap.add_argument("--apply-reps", type=int, default=30)
    ap.add_argument("--workload", default="c2",
                    choices=sorted(WORKLOADS) + sorted(KERSHAW_WORKLOADS),
                    help="kershaw1..4 only with --apply-only")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-copy-bw", action="store_true")
    ap.add_argument("--batch-meshes", type=int, default=256)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-rates", default="50,100,200,500,1000,2000",
                    help="arrival rates (req/s) of the served stream")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--config3", default="c3a,c3b",
                    help="6.44 M-DoF workloads to run beside the headline; empty to skip")
    ap.add_argument("--config3-steps", type=int, default=3)
    ap.add_argument("--kershaw-orders", default="1,2,3,4")
    ap.add_argument("--no-kershaw", action="store_true")
    ap.add_argument("--kershaw-minres-cuts", default="20",
                    help="MINRES iteration caps of extra preconditioned Kershaw rows; empty for none")
    ap.add_argument("--apply-only", action="store_true",
                    help="time only the Hessian action (for profilers); see the module docstring")
    ap.add_argument("--reps", type=int, default=10, help="--apply-only: actions per timing")
    ap.add_argument("--storage", default="both", choices=["tensor", "compact", "both"])
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"])
    ap.add_argument("--copy-ref", action="store_true")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched solve (no sequential loop), for profilers")
    ap.add_argument("--all-kernels", action="store_true",
                    help="--apply-only: also run energy, gradient, setup and diagonal reps times")
    ap.add_argument("--mfma", action="store_true",
                    help="--apply-only --all-kernels: also run energy, gradient and FP64 setup "
                         "with the forward sweeps on the matrix cores")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(a mesh would shard by element slabs with one interface exchange per "
              "action, independent meshes by HBM budget); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2205_12721_amd import inputs
    from paper_2205_12721_amd.tmop import Context, basis_nodes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.apply_only:
        apply_only(args)
        return
    if args.batch_only:
        # the batched solve alone, for profilers
        print(json.dumps(batch_leg(args.batch_meshes, sequential=False)), flush=True)
        return
    if args.workload not in WORKLOADS:
        sys.exit("--workload %s runs with --apply-only only" % args.workload)
    cfg = WORKLOADS[args.workload]
    cname, dim, n, p, nq = cfg
    S = dim * dim * (dim * dim + 1) // 2

    log("[bench] workload", cfg)
    ctx = Context(dim, n, p, nq, precision="fp64")
    probe = torch.empty(ctx.ndof, dtype=torch.float64, device="cuda")

    def valid(xh):
        probe.copy_(torch.as_tensor(xh))
        return ctx.min_det(probe) > 0

    xh, info = inputs.config_mesh(cname, basis_nodes(p), is_valid=valid)
    log("[bench] mesh ready, tries", info["tries"], "ndof", ctx.ndof)
    x0 = torch.as_tensor(xh).cuda()
    x = torch.empty_like(x0)
    ne = int(np.prod([n] * dim))
    nqe = nq ** dim

    v0 = torch.as_tensor(inputs.gaussian_vector(ctx.ndof, inputs.CONFIGS[cname]["vec_seed"])).cuda()

    # FP64: Newton steps (the whole path), then standalone actions for the metric
    run_steps(ctx, x, x0, args.warmup, args.minres)
    log("[bench] fp64 warmup done")
    acc = run_steps(ctx, x, x0, args.steps, args.minres)
    log("[bench] fp64 timed steps done")
    inst = instrumented_steps(ctx, x, x0, args.minres)
    napp = max(inst["n_apply"], 1)
    elem_ms, tot_ms, epb, med_ms = time_actions(ctx, x0, v0, args.apply_reps)
    # the metric: N_dof over the median time of one tmop_hessian_apply
    gdofs = ctx.ndof / (med_ms / 1e3) / 1e9
    rf = roofline(ne, nqe, S, ctx.ndof, 8, elem_ms, tot_ms, traffic_for("tensor_fp64", cname, epb))
    rf["median_action_us"] = round(med_ms * 1e3, 2)
    kl = kernel_leg(ctx, x0, ne, nqe, S, dim, p, nq)
    # the same forward sweeps on the FP64 matrix cores (tmop_set_sweeps)
    if nq <= 5 and dim == 3:
        ctx.set_sweeps("mfma")
        km = kernel_leg(ctx, x0, ne, nqe, S, dim, p, nq)
        ctx.set_sweeps("pencil")
        kl["mfma_forward_sweeps"] = {k: km[k] for k in ("setup", "gradient", "energy")}
    # action FLOP: forward and backward sweeps plus the d^2 x d^2 point product
    act_flop = 2.0 * ne * (2 * sweep_fma(dim, p, nq) + nqe * (dim * dim) ** 2)
    kl["action_GFLOP_s"] = round(act_flop / (tot_ms / 1e3) / 1e9, 2)
    log("[bench] kernel leg done")
    ms_step = acc["wall_s"] / args.steps * 1e3

    out = {
        "metric": "PA TMOP Hessian-apply GDoF/s + %HBM roofline (FP64 vs mixed); p99 solve ms",
        "value": round(gdofs, 3),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "3D hex box %d^3, Q%d, %d^3 Gauss-Legendre points, mu_303, ideal target; "
                        "one Newton step with %d Jacobi-MINRES iterations per step"
                        % (n, p, nq, args.minres) if dim == 3 else
                        "2D quad box %d^2, Q%d, %d^2 points, mu_2" % (n, p, nq),
            "elements": ne, "order": p, "nq1d": nq, "dofs": ctx.ndof,
            "minres_per_step": args.minres, "mesh_seed": inputs.CONFIGS[cname]["seed"],
            "actions_timed": args.apply_reps, "elements_per_workgroup": epb,
        },
        "roofline": rf,
        "kernels": kl,
        "step_gdof_s": round(ctx.ndof * args.minres / (ms_step / 1e3) / 1e9, 3),
        "phases_ms_per_step": {k: round(acc[k] / args.steps, 3)
                               for k in ("t_setup_ms", "t_minres_ms", "t_linesearch_ms")},
        # the action inside MINRES: element kernel + the gather fused with the
        # first Lanczos vector update (HIP events around each, in two more
        # steps after the timed ones; the timed steps record no events)
        "apply_in_minres_us": round(inst["t_apply_ms"] / napp * 1e3, 2),
    }

    variants = [("compact", "fp64")]
    if not args.no_mixed:
        variants = [("tensor", "mixed"), ("compact", "fp64"), ("compact", "mixed")]
    for storage, prec in variants:
        cv = Context(dim, n, p, nq, precision=prec, storage=storage)
        run_steps(cv, x, x0, args.warmup, args.minres)
        av = run_steps(cv, x, x0, args.steps, args.minres)
        iv = instrumented_steps(cv, x, x0, args.minres)
        log("[bench] %s %s timed steps done" % (storage, prec))
        em, tm, eb, mm = time_actions(cv, x0, v0, args.apply_reps)
        sv = S if storage == "tensor" else (13 if dim == 3 else 8)
        key = "%s_%s" % (storage, prec)
        out[key] = {
            "value": round(cv.ndof / (mm / 1e3) / 1e9, 3), "unit": "GDoF/s",
            "dtype": "f64" if prec == "fp64" else "f32 action / f64 rest",
            "storage": storage, "values_per_point": sv,
            "ms_per_step": round(av["wall_s"] / args.steps * 1e3, 3),
            "apply_in_minres_us": round(iv["t_apply_ms"] / max(iv["n_apply"], 1) * 1e3, 2),
            "elements_per_workgroup": eb,
            "roofline": roofline(ne, nqe, sv, cv.ndof, 8 if prec == "fp64" else 4, em, tm,
                                 traffic_for(key, cname, eb)),
        }
        out[key]["roofline"]["median_action_us"] = round(mm * 1e3, 2)
        cv.close()

    c3_refs = []
    if args.config3:
        out["config3"] = {}
        for name in [w for w in args.config3.split(",") if w]:
            out["config3"][name], r = config3_leg(name, args.apply_reps, args.config3_steps,
                                                  args.minres)
            c3_refs.append(r)
            log("[bench] config3 %s done" % name)

    if not args.no_batch:
        out["batch"] = batch_leg(args.batch_meshes)
        log("[bench] batch leg done")
    if not args.no_serve:
        rates = [float(r) for r in args.serve_rates.split(",") if r]
        out["serve"] = serve_leg(rates, args.serve_requests)
        log("[bench] serve leg done")

    if not args.no_kershaw:
        out["kershaw"] = kershaw_leg([int(v) for v in args.kershaw_orders.split(",") if v],
                                     cuts=[int(v) for v in args.kershaw_minres_cuts.split(",") if v])
        log("[bench] kershaw leg done")

    out["config1"] = config1_leg(not args.no_cpu_baseline)
    log("[bench] config1 done")

    if not args.no_copy_bw:
        bw = copy_bandwidth(torch)
        out["copy_bw_GBs"] = round(bw, 1)
        out["roofline"]["frac_of_copy_bw"] = round(rf["achieved"] / bw, 4)

    if not args.no_cpu_baseline:
        v = inputs.gaussian_vector(ctx.ndof, inputs.CONFIGS[cname]["vec_seed"])
        out["cpu_baseline"], y_oracle = cpu_baseline(cfg, xh, v, args.cpu_seconds)
        log("[bench] cpu baseline done")
        if not args.no_precision:
            out["precision"] = precision_leg(cfg, x0, v, y_oracle)
            log("[bench] precision leg done")
        for r in c3_refs:
            out["config3"][r[0]]["hvp_err_vs_oracle_sampled"] = config3_oracle_error(r)
            log("[bench] config3 %s oracle comparison done" % r[0])

    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
