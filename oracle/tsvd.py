"""Truncated-SVD solution of each +-k_m pair (test infrastructure, FP64, CPU).

Paper, Section 3.1: each decoupled system of eqs. Split is solved by the
singular value decomposition of its matrix, with the reciprocal of every
singular value below a tolerance replaced by zero.  For the real form
A^ = [Re A; Im A] (real unknowns x+-, Section 2.1) the singular values s_j
and right singular vectors v_j of A^ are the square roots and eigenvectors of
the Gram G = A^T A^ = Re(A^H A), and the truncated solution is

    x = sum_{s_j >= sigma} v_j (u_j . b^) / s_j = sum_{s_j^2 >= sigma^2} v_j (v_j . c) / s_j^2,

with c = A^T b^ = Re(A^H b).  The paper's tolerance is an absolute sigma = 1
on a scale it does not state; here the tolerance is relative,
sigma^2 = tol_rel^2 * ||G||_F (the Frobenius norm of the Gram, which bounds
the largest s_j^2 from above).  An empty pair gives x = 0; a self-conjugate
k_m keeps x- = 0, as in the damped solve.  The eigen-decomposition is
numpy.linalg.eigh.
"""
from __future__ import annotations

import numpy as np

from .rows import row_values
from .solve import INFO_EMPTY, INFO_OK, normal_equations

__all__ = ["tsvd_threshold", "tsvd_gram", "tsvd_pair", "tsvd_solve"]


def tsvd_threshold(G, tol_rel):
    """sigma^2 = tol_rel^2 ||G||_F."""
    return float(tol_rel) ** 2 * float(np.linalg.norm(G))


def tsvd_gram(G, c, tol_rel):
    """Truncated solution from the Gram: x (k, nz) for right-hand sides c (k, nz),
    the eigenvalues (ascending) and sigma^2."""
    tau2 = tsvd_threshold(G, tol_rel)
    w, V = np.linalg.eigh(G)
    keep = w >= tau2
    Vk = V[:, keep]
    x = ((Vk.T @ np.atleast_2d(c).T) / w[keep][:, None]).T @ Vk.T
    return x, w, tau2


def tsvd_pair(s, p, A, d0, d1, tol_rel):
    """x (2, nz), info, eigenvalues and sigma^2 of one pair."""
    nz = s.nz
    if p.n_rows == 0:
        return np.zeros((2, nz)), INFO_EMPTY, np.zeros(0), 0.0
    G, c, _ = normal_equations(A, d0, d1)
    x, w, tau2 = tsvd_gram(G, c, tol_rel)
    if p.self_conjugate:
        x[1] = 0.0
    return x, INFO_OK, w, tau2


def tsvd_solve(s, pl, data, tabs, tol_rel, pairs=None):
    """V~ (n_km, nz) complex128 in fftfreq order and per-pair details."""
    pairs = pl.pairs if pairs is None else pairs
    V = np.zeros((pl.n_km, s.nz), np.complex128)
    info = []
    for p, (d0, d1) in zip(pairs, data):
        A = row_values(s, p, tabs.lookup) if p.n_rows else None
        x, inf, w, tau2 = tsvd_pair(s, p, A, d0, d1, tol_rel)
        V[p.u] = x[0] + 1j * x[1]
        if not p.self_conjugate:
            V[p.u_neg] = x[0] - 1j * x[1]
        info.append(dict(x=x, info=inf, eig=w, tau2=tau2))
    return V, info
