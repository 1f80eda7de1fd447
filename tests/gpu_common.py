"""Shared helpers of the GPU parity tests: the same seeded mesh handed to the
oracle (CPU, FP64) and to the HIP library through its C ABI."""
import sys

import numpy as np

import oracle
from oracle import basis
from paper_2205_12721_amd import inputs

TOL64 = 1e-11   # relative, energy / gradient / Hessian action / diagonal in FP64
TOLX = 1e-9     # relative, final node positions of a full solve


def rel(a, b):
    """Relative error of a against b: the larger of the l2 measure
    |a - b|_2 / |b|_2 over all entries and the entrywise measure
    max|a - b| / max|b|.  The second catches an error confined to a few
    entries, which the l2 measure over millions of entries would dilute."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = a - b
    nb = np.linalg.norm(b)
    mb = np.abs(b).max() if b.size else 0.0
    e2 = np.linalg.norm(d) / (nb if nb > 0 else 1.0)
    ei = (np.abs(d).max() if d.size else 0.0) / (mb if mb > 0 else 1.0)
    return float(np.max([e2, ei]))  # NaN propagates


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_case(dim, ns, p, nq, recipe="smooth", amp=0.05, seed=1, constrain="boundary", W=None):
    """Oracle problem and a perturbed mesh accepted by the oracle's det test."""
    pb = oracle.Problem.box(dim, ns, p, nq, W=W, constrain=constrain)
    x, _ = inputs.perturbed_box(dim, ns, p, basis.gll_nodes(p), seed, recipe=recipe, amp=amp,
                                is_valid=lambda x: pb.min_det(x) > 0)
    return pb, x


def to_dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)
