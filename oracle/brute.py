"""Exhaustive minimum enclosing ball of a few balls (numpy, FP64).

TEST INFRASTRUCTURE ONLY: pins the ripALM oracle on tiny instances.

Independent of ripALM.  The optimal ball touches a support set S of at most
d+1 input balls whose centers are affinely independent, its center lies in
the affine hull of those centers, and ||c - c_i|| = r - r_i on S (the KKT
conditions of the SOCP form, Section 2, with u_i > 0 only on S).  For every
subset S this module solves those equations in closed form, keeps the
candidates that enclose every ball, and returns the smallest.  Since any
enclosing ball has radius >= r*, and the optimum is among the candidates,
the minimum over enclosing candidates is the optimum.
"""
import itertools

import numpy as np


def candidates_for(Cs, Rs):
    """All balls (r, c) with c in aff(Cs) and ||c - c_i|| = r - r_i for the
    given centers Cs (k x d) and radii Rs; empty if the centers are
    affinely dependent."""
    k, d = Cs.shape
    c0, r0 = Cs[0], Rs[0]
    if k == 1:
        return [(r0, c0.copy())]
    A = (Cs[1:] - c0).T  # d x (k-1)
    G = 2.0 * A.T @ A
    if np.linalg.matrix_rank(G, tol=1e-12 * max(1.0, np.abs(G).max())) < k - 1:
        return []
    # 2 a_j^T A lam = ||a_j||^2 + 2 r (r_j - r0) - r_j^2 + r0^2
    b = np.einsum("ij,ij->j", A, A) - Rs[1:] ** 2 + r0 ** 2
    e = 2.0 * (Rs[1:] - r0)
    p = np.linalg.solve(G, b)
    q = np.linalg.solve(G, e)
    Ap, Aq = A @ p, A @ q
    # ||A p + r A q||^2 = (r - r0)^2
    qa = Aq @ Aq - 1.0
    qb = 2.0 * (Ap @ Aq + r0)
    qc = Ap @ Ap - r0 ** 2
    roots = []
    if abs(qa) < 1e-14:
        if abs(qb) > 0:
            roots = [-qc / qb]
    else:
        disc = qb * qb - 4 * qa * qc
        if disc >= -1e-12 * max(1.0, qb * qb):
            sq = np.sqrt(max(disc, 0.0))
            roots = [(-qb + sq) / (2 * qa), (-qb - sq) / (2 * qa)]
    out = []
    for r in roots:
        if r < Rs.max() - 1e-12:
            continue
        out.append((r, c0 + A @ (p + r * q)))
    return out


def meb(C, R=None, rel=1e-10):
    """Exact minimum enclosing ball by enumeration.  Returns (r, c, S)."""
    C = np.asarray(C, dtype=np.float64)
    m, d = C.shape
    R = np.zeros(m) if R is None else np.asarray(R, dtype=np.float64)
    scale = np.abs(C).max() + R.max() + 1.0
    best = None
    for k in range(1, min(m, d + 1) + 1):
        for S in itertools.combinations(range(m), k):
            S = list(S)
            for r, c in candidates_for(C[S], R[S]):
                reach = np.linalg.norm(C - c, axis=1) + R
                if reach.max() <= r + rel * scale:
                    if best is None or r < best[0]:
                        best = (r, c, S)
    return best
