"""Restriction of the solution to a disk in (k_m, k_z) (test infrastructure,
FP64, CPU).

Paper, Section 3.1: the depth integrals of eqs. Split are rewritten over the
vertical wavenumber k_z, with M and V~ replaced by their Fourier transforms
over z, and V~(k_x, k_z) is kept only inside the disk |k| <= 2.2 w_max / c0
(w_max the largest angular frequency used).  The horizontal wavenumber of the
model is the pair's k_m, so at one pair the kept vertical wavenumbers are
those with k_z^2 + |k_m|^2 <= K^2.

On the survey of parallel lines (Section 2.2) the subproblem is a pair
(k_m, k_y), the model's horizontal wavenumber is (k_m, k_y), and the disk is
taken in (|(k_m, k_y)|, k_z).

Readings: the transform over z is the discrete one on the inversion's depth
grid (nz depths at spacing dz, k_z,j = 2 pi j / (nz dz) for the fftfreq
indices j), and c0, undefined for a layered reference, is the velocity of the
top layer.  A real unknown x(z) restricted to a symmetric set of k_z is a
combination of the real basis 1, cos(k_z,j z_n), sin(k_z,j z_n) (and (-1)^n
at the Nyquist index), orthonormalised; with F the nz x n_keep matrix of that
basis the pair's system A x = b becomes (A F) y = b, x = F y, and the
truncated SVD is taken of A F (Gram F^T G F, right-hand sides F^T c).
"""
from __future__ import annotations

import numpy as np

from .rows import row_values
from .solve import INFO_EMPTY, INFO_OK, normal_equations
from .tsvd import tsvd_gram

__all__ = ["kz_disk_radius", "pair_km2", "kz_kept", "kz_basis", "kz_tsvd_solve"]

TWO_PI = 2.0 * np.pi


def kz_disk_radius(s, factor=2.2):
    """K = factor * 2 pi f_max / c0, c0 the top layer's velocity."""
    return factor * (TWO_PI * float(np.max(s.freqs))) / float(s.vel[0])


def _signed(u, N):
    return u if u < (N + 1) // 2 else u - N


def pair_km2(s, u):
    """|k_m|^2 of the k_m index u (fftfreq order; 3D: u = ux N + uy; parallel
    lines: u = ux N_y + c, |(k_m, k_y)|^2)."""
    N = s.n_mid
    dk = TWO_PI / (N * s.d_mid)
    if getattr(s, "n_line", 0):
        Ny = s.n_line
        ux, c = divmod(u, Ny)
        kx = _signed(ux, N) * dk
        ky = _signed(c, Ny) * (TWO_PI / (Ny * s.d_line))
        return kx * kx + ky * ky
    if getattr(s, "dim", 2) == 3:
        ux, uy = divmod(u, N)
        kx = _signed(ux, N) * dk
        ky = _signed(uy, N) * dk
        return kx * kx + ky * ky
    k = _signed(u, N) * dk
    return k * k


def kz_kept(nz, dz, km2, K):
    """Non-negative k_z indices j (0 <= j <= nz/2) with k_z,j^2 + km2 <= K^2."""
    dkz = TWO_PI / (nz * dz)
    K2 = K * K
    out = []
    for j in range(nz // 2 + 1):
        kz = j * dkz
        if kz * kz + km2 <= K2:
            out.append(j)
    return out


def kz_basis(nz, dz, km2, K):
    """Orthonormal real basis (nz, n_keep) of the kept discrete Fourier modes."""
    n = np.arange(nz)
    cols = []
    for j in kz_kept(nz, dz, km2, K):
        if j == 0:
            cols.append(np.full(nz, 1.0 / np.sqrt(nz)))
        elif 2 * j == nz:
            cols.append(np.cos(np.pi * n) / np.sqrt(nz))
        else:
            ph = TWO_PI * j * n / nz
            cols.append(np.sqrt(2.0 / nz) * np.cos(ph))
            cols.append(np.sqrt(2.0 / nz) * np.sin(ph))
    return np.stack(cols, axis=1) if cols else np.zeros((nz, 0))


def kz_tsvd_solve(s, pl, data, tabs, tol_rel, K, pairs=None):
    """Truncated-SVD solution restricted to the disk of radius K:
    V~ (n_km, nz) complex128 in fftfreq order and per-pair details (x, info,
    the eigenvalues of F^T G F, sigma^2 and the number of kept columns).
    Survey of parallel lines: `tabs` is the table of
    oracle.lines3d.line_tables and `pl` its plan."""
    if getattr(s, "n_line", 0):
        from .lines3d import line_row_values

        def rows_of(p):
            return line_row_values(s, p, tabs)
    else:
        def rows_of(p):
            return row_values(s, p, tabs.lookup)
    pairs = pl.pairs if pairs is None else pairs
    nz = s.nz
    V = np.zeros((pl.n_km, nz), np.complex128)
    info = []
    for p, (d0, d1) in zip(pairs, data):
        F = kz_basis(nz, s.dz, pair_km2(s, p.u), K)
        x = np.zeros((2, nz))
        w, tau2, inf = np.zeros(0), 0.0, INFO_EMPTY
        if p.n_rows:
            inf = INFO_OK
            if F.shape[1]:
                A = rows_of(p)
                G, c, _ = normal_equations(A, d0, d1)
                y, w, tau2 = tsvd_gram(F.T @ G @ F, c @ F, tol_rel)
                x = y @ F.T
                if p.self_conjugate:
                    x[1] = 0.0
        V[p.u] = x[0] + 1j * x[1]
        if not p.self_conjugate:
            V[p.u_neg] = x[0] - 1j * x[1]
        info.append(dict(x=x, info=inf, eig=w, tau2=tau2, n_keep=F.shape[1]))
    return V, info
