"""Finite aperture (test infrastructure, FP64, CPU).

Paper, Section 2.1, eq. M: with the offsets limited to |h| <= b, each datum at
offset wavenumber k_h is a sinc-weighted integral over k_h' of the
infinite-aperture integrand.  On the periodic line (N positions at dx) the
same statement is exact and discrete: the records are kept only where the
full offset satisfies |x_R - x_S| <= 2 b, and at the pair of k_m index u the
transformed datum at receiver index a becomes

    d_W(a) = sum_a' S(a - a') d(a'),   S(m) = (1/N) sum_o w(o) e^{-2 pi i m o / N},

with w the 0/1 window over the signed offset index o = R - S (S(m) is the
discrete sinc; for a symmetric window it is real and even).  The partner
datum at -u is convolved over the same receiver index.  The windowed system
is (S A) x = d_W, and since the circulant S is an orthogonal projector its
normal equations have the Gram Re(A^H S A) and the right-hand sides
Re(A^H d_W).  Rows cut as evanescent are zero in A.

Survey of parallel lines (Section 2.2): the decoupled 3D equation carries
the same sinc over the offset wavenumber.  Each line is a 2D line of N_x
positions whose records are kept where |x_R - x_S| <= 2 b; the window does
not depend on the line, so at the pair (k_m, k_y) it is the same circulant
S over the receiver index, applied to the line rows (oracle.lines3d).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .rows import row_values
from .solve import INFO_EMPTY, INFO_OK

__all__ = ["offset_window", "window_kernel", "aperture_rows", "aperture_data", "aperture_solve"]


def offset_window(s, b_max):
    """w(o) over the fftfreq-order offset index o: |o dx| <= 2 b_max."""
    N = s.n_mid
    o = np.fft.fftfreq(N, 1.0 / N)
    return (np.abs(o) * s.d_mid <= 2.0 * b_max).astype(np.float64)


def window_kernel(w):
    """S(m) for m in [0, N): the DFT of the window over N (real for a
    symmetric window)."""
    N = w.shape[0]
    m = np.arange(N)
    o = np.fft.fftfreq(N, 1.0 / N)
    Sm = (np.exp(-2j * np.pi * np.outer(m, o) / N) @ w) / N
    return Sm


def aperture_rows(s, p, A, Sm):
    """The windowed rows S A of one pair: rows of one frequency are mixed by
    S(a - a') over their receiver indices a."""
    N = s.n_mid
    B = np.zeros_like(A)
    a = p.key0[:, 0]
    for f in np.unique(p.f):
        sel = np.nonzero(p.f == f)[0]
        K = Sm[(a[sel][:, None] - a[sel][None, :]) % N]
        B[sel] = K @ A[sel]
    return B


def aperture_data(s, pl, data, b_max, pairs=None):
    """The windowed data d_W = S d of every pair: the data (d+, d-) of one
    frequency are mixed by S(a - a') over their receiver indices a, as the
    rows are (the records windowed in full offset, with the data outside the
    kept rows taken as zero)."""
    Sm = window_kernel(offset_window(s, b_max))
    pairs = pl.pairs if pairs is None else pairs
    out = []
    for p, (d0, d1) in zip(pairs, data):
        if not p.n_rows:
            out.append((d0.copy(), d1.copy()))
            continue
        B = aperture_rows(s, p, np.stack([d0, d1], axis=1), Sm)
        out.append((B[:, 0].copy(), B[:, 1].copy()))
    return out


def aperture_solve(s, pl, data, tabs, b_max, lambda_rel=None, pairs=None):
    """Damped solve of the windowed system: (Re(A^H S A) + lambda I) x =
    Re(A^H b+-), lambda = lambda_rel tr / nz, with b+- formed from `data`,
    which are the windowed data d_W (aperture_data) for the windowed system.
    V~ (n_km, nz) and per-pair details.  2D line: `tabs` from
    oracle.solve.gtables; survey of parallel lines: the table of
    oracle.lines3d.line_tables and its plan."""
    if getattr(s, "n_line", 0):
        from .lines3d import line_row_values

        def rows_of(p):
            return line_row_values(s, p, tabs)
    elif getattr(s, "dim", 2) == 2:
        def rows_of(p):
            return row_values(s, p, tabs.lookup)
    else:
        raise ValueError("the 2D line survey and the survey of parallel lines only")
    lam_rel = s.lambda_rel if lambda_rel is None else lambda_rel
    Sm = window_kernel(offset_window(s, b_max))
    pairs = pl.pairs if pairs is None else pairs
    V = np.zeros((pl.n_km, s.nz), np.complex128)
    info = []
    for p, (d0, d1) in zip(pairs, data):
        x = np.zeros((2, s.nz))
        inf, G = INFO_EMPTY, None
        if p.n_rows:
            A = rows_of(p)
            B = aperture_rows(s, p, A, Sm)
            G = (A.conj().T @ B).real
            bp, bm = 0.5 * (d0 + d1), (d0 - d1) / 2j
            c = np.stack([(A.conj().T @ bp).real, (A.conj().T @ bm).real])
            lam = lam_rel * np.trace(G) / s.nz
            fac = scipy.linalg.cho_factor(G + lam * np.eye(s.nz), lower=True)
            x = scipy.linalg.cho_solve(fac, c.T).T
            if p.self_conjugate:
                x[1] = 0.0
            inf = INFO_OK
        V[p.u] = x[0] + 1j * x[1]
        if not p.self_conjugate:
            V[p.u_neg] = x[0] - 1j * x[1]
        info.append(dict(x=x, info=inf, gram=G))
    return V, info
