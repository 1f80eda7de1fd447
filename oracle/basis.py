"""Oracle: 1D bases, quadrature and the dense reference tables.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``gll_nodes``   -- the p+1 nodes of the 1D Lagrange basis on [0,1]
  (Sec. 3.1 speaks of "standard 1D Lagrange polynomials in [0,1]" without
  naming the node set; this build reads it as Gauss-Lobatto-Legendre points,
  which coincide with equispaced points for p <= 2).
* ``gl_rule``     -- the n_q-point Gauss-Legendre rule mapped to [0,1]
  (Sec. 3.1, tensor-product quadrature built from a 1D rule).
* ``gll_rule``    -- the n_q-point Gauss-Lobatto-Legendre rule on [0,1]
  (the other 1D rule the library offers; the paper does not name its rule).
* ``lagrange``    -- l_j(x) and l_j'(x) from the product formula.
* ``tables_1d``   -- B_qi = l_i(chi_q), G_qi = l_i'(chi_q)  (Sec. 3.1, eq. eq_B_G_1D).
* ``dense_tables``-- d wbar_i / d xbar_b at every tensor quadrature point as an
  explicit product over axes (Sec. 3.1, eq. eqn_basis_tensor and the
  derivative display after it), with lexicographic local numbering
  i = i1 + n_i*i2 + n_i^2*i3 (0-based form of the paper's formula).
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def gll_nodes(p):
    """p+1 Gauss-Lobatto-Legendre points on [0,1], ascending."""
    if p < 1:
        raise ValueError("order p must be >= 1")
    if p == 1:
        t = np.array([-1.0, 1.0])
    else:
        # interior GLL points are the roots of P_p'(t) on (-1,1)
        cp = np.zeros(p + 1)
        cp[p] = 1.0
        interior = np.sort(np.real(npleg.legroots(npleg.legder(cp))))
        # polish the roots with Newton steps on P_p'
        d1 = npleg.legder(cp)
        d2 = npleg.legder(cp, 2)
        for _ in range(5):
            interior = interior - npleg.legval(interior, d1) / npleg.legval(interior, d2)
        t = np.concatenate([[-1.0], interior, [1.0]])
    x = 0.5 * (t + 1.0)
    # enforce exact symmetry about 1/2
    x = 0.5 * (x + (1.0 - x[::-1]))
    return x


def gl_rule(nq):
    """n_q-point Gauss-Legendre rule on [0,1]: (points, weights), weights sum to 1."""
    t, w = npleg.leggauss(nq)
    return 0.5 * (t + 1.0), 0.5 * w


def gll_rule(nq):
    """n_q-point Gauss-Lobatto-Legendre rule on [0,1] (n_q >= 2): the end points and
    the roots of P_{n-1}', weights 2 / (n (n-1) P_{n-1}(t)^2) on [-1,1], halved."""
    if nq < 2:
        raise ValueError("a Gauss-Lobatto rule needs at least 2 points")
    x = gll_nodes(nq - 1)
    c = np.zeros(nq)
    c[nq - 1] = 1.0
    P = npleg.legval(2.0 * x - 1.0, c)
    return x, 1.0 / (nq * (nq - 1.0) * P * P)


def quad_rule(nq, rule="gl"):
    """The 1D rule by name: "gl" (Gauss-Legendre) or "gll" (Gauss-Lobatto-Legendre)."""
    if rule == "gl":
        return gl_rule(nq)
    if rule == "gll":
        return gll_rule(nq)
    raise ValueError("unknown quadrature rule %r" % (rule,))


def lagrange(nodes, pts):
    """Values and derivatives of the Lagrange polynomials on ``nodes`` at ``pts``.

    Returns (L, dL) with L[k, j] = l_j(pts[k]), dL[k, j] = l_j'(pts[k]).
    l_j(x) = prod_{m != j} (x - x_m)/(x_j - x_m); the derivative is the sum over
    the dropped factor (product rule).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    pts = np.atleast_1d(np.asarray(pts, dtype=np.float64))
    n = len(nodes)
    L = np.ones((len(pts), n))
    dL = np.zeros((len(pts), n))
    for j in range(n):
        for m in range(n):
            if m == j:
                continue
            L[:, j] *= (pts - nodes[m]) / (nodes[j] - nodes[m])
        for r in range(n):
            if r == j:
                continue
            term = np.full(len(pts), 1.0 / (nodes[j] - nodes[r]))
            for m in range(n):
                if m == j or m == r:
                    continue
                term = term * (pts - nodes[m]) / (nodes[j] - nodes[m])
            dL[:, j] += term
    return L, dL


def tables_1d(p, nq, rule="gl"):
    """B (nq x (p+1)) and G (nq x (p+1)) at the points of the 1D rule."""
    chi, _ = quad_rule(nq, rule)
    return lagrange(gll_nodes(p), chi)


def dense_tables(dim, p, nq, rule="gl"):
    """Weights w_q (N_q) and dphi[b, q, i] = d wbar_i/d xbar_b (dim x N_q x N_p).

    Quadrature points q = q1 + nq*q2 (+ nq^2*q3), nodes i = i1 + ni*i2 (+ ni^2*i3),
    both lexicographic with the first axis fastest.
    """
    ni = p + 1
    chi, w1 = quad_rule(nq, rule)
    B, G = lagrange(gll_nodes(p), chi)
    NQ = nq ** dim
    NP = ni ** dim
    wq = np.zeros(NQ)
    dphi = np.zeros((dim, NQ, NP))
    for q in range(NQ):
        qs = [(q // nq ** k) % nq for k in range(dim)]
        wq[q] = np.prod([w1[qk] for qk in qs])
        for i in range(NP):
            iis = [(i // ni ** k) % ni for k in range(dim)]
            for b in range(dim):
                val = 1.0
                for k in range(dim):
                    val *= (G if k == b else B)[qs[k], iis[k]]
                dphi[b, q, i] = val
    return wq, dphi


def dense_values(dim, p, nq, rule="gl"):
    """phi[q, i] = wbar_i(xbar_q) (N_q x N_p), same orderings as dense_tables."""
    ni = p + 1
    chi, _ = quad_rule(nq, rule)
    B, _ = lagrange(gll_nodes(p), chi)
    NQ = nq ** dim
    NP = ni ** dim
    phi = np.ones((NQ, NP))
    for q in range(NQ):
        qs = [(q // nq ** k) % nq for k in range(dim)]
        for i in range(NP):
            iis = [(i // ni ** k) % ni for k in range(dim)]
            for k in range(dim):
                phi[q, i] *= B[qs[k], iis[k]]
    return phi
