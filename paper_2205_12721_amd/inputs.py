"""Seeded synthetic inputs: perturbed structured quad/hex meshes and vectors.

This module holds only the input recipe (node placement, perturbation,
random draws).  It computes nothing of the optimisation method itself: the
1D node positions inside an element are passed in by the caller, and the
det(J) > 0 acceptance test of a draw is a caller-supplied predicate, so the
product path and the oracle each bring their own.

Layout of a node vector: float64, SoA by component, x[c*N_x + g] with the
global node index g lexicographic on the (n_k p + 1) grid, first axis
fastest.

Recipes (the paper's own meshes are the Kershaw family of Sec. 4.1 and a
production ALE mesh; these perturbed boxes stand in for them):

* ``interior_jitter``: uniform mesh of [0,1]^d; every coordinate of every
  interior node moved by U[-a h, a h] (h = 1/n per axis).
* ``smooth``: uniform mesh plus a smooth displacement
  u_c(x) = (0.2 h / 4) sum_{k<4} s_ck prod_j sin(pi m_ckj x_j)
  with m in {1,2,3} and s in {-1,+1} drawn from the seed (it vanishes on the
  boundary), plus U[-a, a] jitter on every node, with the jitter component
  normal to a boundary face removed (boundary nodes slide only along their
  face/edge; corners do not move).

Jitter amplitude: a = amp * h * p * g_min, where g_min is the smallest gap
between adjacent 1D element nodes on [0,1] (p * g_min = 1 for p <= 2, 0.83
for p = 3, 0.69 for p = 4), so the jitter is the same fraction of the closest
node spacing at every order.
* ``pin``: the ``smooth`` geometry class but with interior-only jitter, so the
  uniform grid is the optimum of every shape metric with fixed boundary.

A draw whose predicate fails is redrawn from the continuing random stream
(up to ``max_tries``).
"""
import math

import numpy as np

CONFIGS = {
    # 2D 8x8 Q2, 4x4 Gauss-Legendre points, mu_2, interior jitter 0.15 h
    "c1": dict(dim=2, n=8, p=2, nq=4, metric=2, seed=1, vec_seed=101,
               recipe="interior_jitter", amp=0.15),
    # 3D 24^3 Q3, 5^3 points, mu_303, smooth + tangential jitter
    "c2": dict(dim=3, n=24, p=3, nq=5, metric=303, seed=2, vec_seed=102,
               recipe="smooth", amp=0.05),
    # 3D 64^3 Q2 and 32^3 Q4, p+2 points per direction
    "c3a": dict(dim=3, n=64, p=2, nq=4, metric=303, seed=3, vec_seed=103,
                recipe="smooth", amp=0.05),
    "c3b": dict(dim=3, n=32, p=4, nq=6, metric=303, seed=4, vec_seed=104,
                recipe="smooth", amp=0.05),
}


def grid_shape(ns, p):
    return [int(n) * p + 1 for n in ns]


def grid_coords(ns, p):
    """Integer grid coordinates G[k, g] of every global node (first axis fastest)."""
    dim = len(ns)
    M = grid_shape(ns, p)
    return np.indices(tuple(M[::-1])).reshape(dim, -1)[::-1].copy()


def uniform_nodes(ns, p, nodes1d):
    """Node vector (dim*N_x) of the uniform mesh of [0,1]^dim.

    Grid coordinate g_k = e_k p + j lies at (e_k + nodes1d[j]) / n_k.
    """
    nodes1d = np.asarray(nodes1d, dtype=np.float64)
    if len(nodes1d) != p + 1:
        raise ValueError("need p+1 one-dimensional node positions")
    G = grid_coords(ns, p)
    dim = len(ns)
    out = []
    for k in range(dim):
        g = G[k]
        e = np.minimum(g // p, ns[k] - 1)
        j = g - e * p
        out.append((e + nodes1d[j]) / ns[k])
    return np.concatenate(out)


def boundary_component_mask(ns, p):
    """(dim, N_x) bool: True where grid coordinate k is on the low/high face of axis k."""
    G = grid_coords(ns, p)
    M = grid_shape(ns, p)
    return np.stack([(G[k] == 0) | (G[k] == M[k] - 1) for k in range(len(ns))])


def smooth_displacement(ns, x, rng, amp=0.2):
    """u_c(x) = (amp h_c / 4) sum_k s_ck prod_j sin(pi m_ckj x_j); draws m, s from rng."""
    dim = len(ns)
    nx = x.size // dim
    X = x.reshape(dim, nx)
    m = rng.integers(1, 4, size=(dim, 4, dim))
    s = rng.integers(0, 2, size=(dim, 4)) * 2 - 1
    u = np.zeros((dim, nx))
    for c in range(dim):
        h = 1.0 / ns[c]
        for k in range(4):
            term = np.full(nx, float(s[c, k]))
            for j in range(dim):
                term *= np.sin(math.pi * m[c, k, j] * X[j])
            u[c] += term
        u[c] *= amp * h / 4.0
    return u.ravel()


def perturbed_box(dim, n, p, nodes1d, seed, recipe="smooth", amp=0.05,
                  is_valid=None, max_tries=100):
    """Seeded perturbed box mesh.  Returns (x, info) with info['tries']."""
    ns = (n,) * dim if np.isscalar(n) else tuple(int(v) for v in n)
    rng = np.random.default_rng(seed)
    x0 = uniform_nodes(ns, p, nodes1d)
    nx = x0.size // dim
    bmask = boundary_component_mask(ns, p)
    interior = ~np.any(bmask, axis=0)
    base = x0.copy()
    if recipe == "smooth":
        base = x0 + smooth_displacement(ns, x0, rng)
    elif recipe not in ("interior_jitter", "pin"):
        raise ValueError("unknown recipe %r" % recipe)
    gap = float(np.min(np.diff(np.asarray(nodes1d, dtype=np.float64)))) * p
    hs = np.array([gap / v for v in ns])
    for t in range(1, max_tries + 1):
        jit = rng.uniform(-1.0, 1.0, size=(dim, nx)) * (amp * hs)[:, None]
        if recipe == "smooth":
            jit[bmask] = 0.0            # no motion normal to a boundary face
        else:
            jit[:, ~interior] = 0.0     # boundary nodes stay put
        x = base + jit.ravel()
        if is_valid is None or is_valid(x):
            return x, dict(tries=t, shape=ns)
    raise RuntimeError("no valid draw after %d tries" % max_tries)


def config_mesh(name, nodes1d, is_valid=None, n_override=None):
    """Mesh of a named configuration (see CONFIGS)."""
    c = CONFIGS[name]
    n = c["n"] if n_override is None else n_override
    return perturbed_box(c["dim"], n, c["p"], nodes1d, c["seed"], recipe=c["recipe"],
                         amp=c["amp"], is_valid=is_valid)


def gaussian_vector(ndof, seed, fixed=None):
    """N(0,1) vector with entries on fixed DoFs zeroed."""
    v = np.random.default_rng(seed).standard_normal(ndof)
    if fixed is not None:
        v[np.asarray(fixed, dtype=bool)] = 0.0
    return v


def batch_specs(count=256, seed=5):
    """Per-mesh specs of the batched workload: log2 E ~ U[3,12], n = clamp(round(2^(log2E/3)),2,16),
    p ~ U{1..4}, n_q = p + 2, one child seed per mesh."""
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for k, ss in enumerate(children):
        rng = np.random.default_rng(ss)
        l2e = rng.uniform(3.0, 12.0)
        n = int(min(16, max(2, round(2.0 ** (l2e / 3.0)))))
        p = int(rng.integers(1, 5))
        mseed = int(rng.integers(0, 2 ** 31 - 1))
        out.append(dict(index=k, dim=3, n=n, p=p, nq=p + 2, metric=303, seed=mseed))
    return out


def serving_stream(rate, count=2000, seed=6, max_n3=48, same_requests=False):
    """Poisson arrival stream of mixed 2D/3D requests.

    Inter-arrival ~ Exp(rate); 50% 2D (mu_2) / 50% 3D (mu_303); element count
    lognormal with median 512 and sigma 1 (log space), truncated to
    [2^d, 48^3]; n = round(E^(1/d)); p ~ U{1..4}; n_q = p + 2.
    With ``same_requests`` the draw does not depend on the rate: every rate
    sees the same requests in the same order, with arrival times that are one
    unit-rate Poisson stream divided by the rate.
    """
    rng = np.random.default_rng([seed] if same_requests else [seed, int(rate)])
    t = 0.0
    reqs = []
    for k in range(count):
        gap = rng.exponential(1.0) / rate if same_requests else rng.exponential(1.0 / rate)
        t += gap
        dim = 2 if rng.uniform() < 0.5 else 3
        E = float(np.exp(rng.normal(math.log(512.0), 1.0)))
        E = min(max(E, 2.0 ** dim), float(max_n3) ** 3)
        n = max(2, int(round(E ** (1.0 / dim))))
        p = int(rng.integers(1, 5))
        reqs.append(dict(id=k, t_arrive=t, dim=dim, n=n, p=p, nq=p + 2,
                         metric=2 if dim == 2 else 303,
                         seed=int(rng.integers(0, 2 ** 31 - 1))))
    return reqs


# ---------------------------------------------------------------------------
# Kershaw meshes (Sec. 4.1; the mesh is fixed by the generator the paper's
# appendix lists, restated here): x is unchanged; y (and z) is moved by a map
# that is piecewise linear in t with a kink at t = 1/2.  At the left end the
# map L packs the elements towards t = 0 ... y-slope eps for t < 1/2 at the low
# side of the box ... at the right end the mirror map R packs them at the
# opposite corner, so the high-aspect-ratio elements (aspect 1/eps) sit in
# opposite corners of the first and last of six equal layers in x.  In
# between, the map blends the two with a weight s(x) made of clamped quintic
# smoothsteps: 0 -> 1 across the second layer, back 1 -> 0 across the third
# and fourth together, 0 -> 1 across the fifth.  eps = 1 gives the uniform
# mesh; t = 0 and t = 1 stay put, so boundary nodes only move tangentially.
# ---------------------------------------------------------------------------

def _quintic_step(u):
    """Smoothstep 10u^3 - 15u^4 + 6u^5 on [0, 1], clamped to 0 / 1 outside."""
    u = np.clip(u, 0.0, 1.0)
    return u ** 3 * (10.0 - 15.0 * u + 6.0 * u * u)


def kershaw_blend(x):
    """Weight s(x) of the right-end map: 0 on the first layer, rising across the
    second, falling across the third and fourth, rising across the fifth, 1 on
    the sixth (layers of width 1/6 in x)."""
    x = np.asarray(x, dtype=np.float64)
    return _quintic_step(6.0 * x - 1.0) - _quintic_step(3.0 * x - 1.0) + _quintic_step(6.0 * x - 4.0)


def kershaw_map(x, t, eps):
    """Image of coordinate t (y or z) at abscissa x for anisotropy eps:
    Y = L(t) + (R(t) - L(t)) s(x), with L and R the piecewise-linear maps of
    [0, 1] onto itself through (1/2, eps/2) and (1/2, 1 - eps/2)."""
    t = np.asarray(t, dtype=np.float64)
    knots = [0.0, 0.5, 1.0]
    L = np.interp(t, knots, [0.0, 0.5 * eps, 1.0])
    R = np.interp(t, knots, [0.0, 1.0 - 0.5 * eps, 1.0])
    return L + (R - L) * kershaw_blend(x)


def kershaw_nodes(ns, p, nodes1d, eps_y=0.3, eps_z=0.3):
    """Kershaw node vector (3D) of an ns = (n_x, n_y, n_z) box of order p; n_x must be a
    multiple of 6 and n_y, n_z multiples of 2 for the layers to align with elements."""
    x = uniform_nodes(ns, p, nodes1d)
    nx = x.size // 3
    X, Y, Z = x[:nx], x[nx:2 * nx], x[2 * nx:]
    return np.concatenate([X, kershaw_map(X, Y, eps_y), kershaw_map(X, Z, eps_z)])


def sliding_mask(ns, p):
    """uint8 mask (dim*N_x): component c of a node is fixed iff the node lies on a face
    normal to axis c, so boundary nodes slide along their faces (edges: along the edge;
    corners fixed)."""
    return boundary_component_mask(ns, p).astype(np.uint8).ravel()
