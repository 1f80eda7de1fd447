"""Run only the Hessian action on a benchmark mesh, for profilers.

    python -m paper_2205_12721_amd.profile_apply [--workload c2] [--reps 10]
        [--storage tensor|compact|both] [--precision fp64|mixed|both] [--copy-ref]

Sets up the mesh (seeded, as in bench.py), one Hessian setup per variant, then
``reps`` actions back to back on the library's stream, and prints the mean
device time per action (HIP events).  ``--copy-ref`` also runs a plain
device-to-device copy of 1 GiB (a kernel of known traffic, to scale hardware
byte counters).
"""
import argparse
import json
import sys

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--storage", default="both")
    ap.add_argument("--precision", default="both")
    ap.add_argument("--copy-ref", action="store_true")
    a = ap.parse_args(argv)
    import torch

    from . import inputs
    from .tmop import Context, basis_nodes
    c = inputs.CONFIGS[a.workload]
    dim, n, p, nq = c["dim"], c["n"], c["p"], c["nq"]
    st = ["tensor", "compact"] if a.storage == "both" else [a.storage]
    pr = ["fp64", "mixed"] if a.precision == "both" else [a.precision]
    probe = Context(dim, n, p, nq)
    buf = torch.empty(probe.ndof, dtype=torch.float64, device="cuda")

    def valid(xh):
        buf.copy_(torch.as_tensor(xh))
        return probe.min_det(buf) > 0

    xh, _ = inputs.config_mesh(a.workload, basis_nodes(p), is_valid=valid)
    probe.close()
    x = torch.as_tensor(xh).cuda()
    v = torch.as_tensor(inputs.gaussian_vector(x.numel(), c["vec_seed"])).cuda()
    y = torch.empty_like(v)
    out = {}
    for s in st:
        for q in pr:
            ctx = Context(dim, n, p, nq, precision=q, storage=s)
            ctx.hessian_setup(x)
            ctx.hessian_apply(v, y)
            elem, tot = ctx.time_apply(v, y, a.reps)
            out["%s_%s" % (s, q)] = dict(elem_us=round(elem * 1e3, 2), total_us=round(tot * 1e3, 2))
            ctx.close()
    if a.copy_ref:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_ref_bytes_each_way"] = src.numel() * 8
    print(json.dumps(dict(workload=a.workload, dofs=int(x.numel()), actions=out)))
    sys.stdout.flush()


if __name__ == "__main__":
    main()
