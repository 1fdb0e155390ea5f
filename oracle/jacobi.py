"""One-sided (Hestenes) Jacobi SVD -- TEST INFRASTRUCTURE ONLY.

An independent cross-check for the rank-1 update oracle on small inputs: it
never uses the update structure, only the explicit matrix A^. Column pairs of
G = A^T (n x m, n >= m) are rotated until mutually orthogonal; the column norms
are the singular values. Pairs are visited in round-robin (tournament) order so
that each step rotates m/2 disjoint pairs at once.
"""
from __future__ import annotations

import numpy as np

U64 = 2.0 ** -53


def _tournament(q: int):
    """Rounds of disjoint pairs covering every pair of 0..q-1 once (q even)."""
    players = list(range(q))
    rounds = []
    for _ in range(q - 1):
        rounds.append([(players[k], players[q - 1 - k]) for k in range(q // 2)])
        players = [players[0]] + [players[-1]] + players[1:-1]
    return rounds


def jacobi_svd(A: np.ndarray, max_sweeps: int = 60):
    """SVD of A (m x n, m <= n) as U (m x m), s (m, descending), Vm (n x m)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m > n:
        raise ValueError("need m <= n")
    q = m + (m % 2)                       # pad to an even number of columns
    G = np.zeros((n, q))
    G[:, :m] = A.T
    J = np.eye(q)
    rounds = _tournament(q)
    for _ in range(max_sweeps):
        rotated = False
        for rnd in rounds:
            p = np.array([x for x, _ in rnd])
            r = np.array([y for _, y in rnd])
            gp, gr = G[:, p], G[:, r]
            alpha = np.sum(gp * gp, axis=0)
            beta = np.sum(gr * gr, axis=0)
            gamma = np.sum(gp * gr, axis=0)
            act = np.abs(gamma) > 2.0 * U64 * np.sqrt(alpha * beta)
            act &= gamma != 0.0
            if not np.any(act):
                continue
            rotated = True
            zeta = np.where(act, (beta - alpha) / np.where(act, 2.0 * gamma, 1.0), 0.0)
            t = np.where(act, np.sign(zeta) / (np.abs(zeta) + np.sqrt(1.0 + zeta * zeta)), 0.0)
            t = np.where(act & (zeta == 0.0), 1.0, t)
            c = 1.0 / np.sqrt(1.0 + t * t)
            s = c * t
            G[:, p], G[:, r] = c * gp - s * gr, s * gp + c * gr
            jp, jr = J[:, p].copy(), J[:, r].copy()
            J[:, p], J[:, r] = c * jp - s * jr, s * jp + c * jr
        if not rotated:
            break
    G, J = G[:, :m], J[:m, :m]
    sv = np.sqrt(np.sum(G * G, axis=0))
    order = np.argsort(-sv, kind="stable")
    sv, G, J = sv[order], G[:, order], J[:, order]
    W = np.where(sv[None, :] > 0, G / np.where(sv > 0, sv, 1.0)[None, :], 0.0)
    # A^T = W diag(s) J^T  =>  A = J diag(s) W^T
    return J, sv, W
