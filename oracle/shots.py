"""The transforms on either side of the decoupled problems (test
infrastructure, FP64, CPU).

Paper, Section 2.1: the method works on the data Fourier-transformed over
receiver and source positions, and the solution is the model's transform over
the horizontal coordinate.  On the periodic line of N positions (spacing
dx) the transformed datum at receiver wavenumber index a and source index b is

    d~(a, b) = dx * sum_{R, S} D(x_R, x_S) e^{-2 pi i (a R + b S) / N},

the convention under which the packed rows equal brute-force space-domain
Born data (pinned through oracle.born), and the model is the inverse of the
unnormalised DFT over x (over x and y in 3D) that defines V~:

    V(x_n, z) = Re (1/N) sum_u V~(u, z) e^{2 pi i u n / N}.

Both are numpy FFTs; the packing follows each row's (a, b) key and its -k_m
partner (-b, -a).

3D areal survey (Section 2.2).  A row of k_m index q and k_h index n has, in
units of dk/2 (dk = 2 pi / (N d_mid)), receiver wavenumber q + 2n and source
wavenumber q - 2n per axis: half-grid wavenumbers of the N-periodic grid.
They are whole-grid wavenumbers of a survey of twice the period, so the
records are those of a full-coverage periodic areal survey on the 2N x 2N
grid (spacing d_mid), D[f, Rx, Ry, Sx, Sy], whose transform

    F(a, b) = d_mid^2 sum_{R, S} D(x_R, x_S) e^{-2 pi i (a . R + b . S) / 2N}

at a = q + 2n, b = q - 2n (mod 2N per axis) is 4 times the row's datum at
+k_m, and at (-b, -a) 4 times the datum at -k_m: the N-periodic model seen
on the 2N grid has its spectrum at the even indices 2q only, 4 times the
N-grid spectrum there.  (The pin compares these rows with brute-force
space-domain Born data of the model repeated 2 x 2 times.)

3D survey of parallel lines (Section 2.2; oracle.lines3d): records
D[f, j, R, S] of line j, receiver R and source S; the datum of key
(a, b, c) is d_mid sum_{j, R, S} D e^{-2 pi i (a R + b S) / N_x}
e^{-2 pi i c j / N_y}, and a row of pair (u, c) keyed (a, b, c) has its
-k partner at (-b, -a, -c).
"""
from __future__ import annotations

import numpy as np

__all__ = ["shots_to_rows", "model_from_spectrum"]


def shots_to_rows(s, pl, D, pairs=None):
    """Shot records -> list of (d+, d-) per pair, in the oracle's row order.

    2D line: D (n_freq, N, N) [f, receiver, source].  3D areal: D (n_freq,
    2N, 2N, 2N, 2N) [f, Rx, Ry, Sx, Sy], the doubled periodic survey.  3D
    parallel lines: D (n_freq, N_y, N_x, N_x) [f, line, receiver, source]."""
    pairs = pl.pairs if pairs is None else pairs
    if getattr(s, "n_line", 0):
        return _line_rows(s, D, pairs)
    if getattr(s, "dim", 2) == 3:
        return _areal_rows(s, D, pairs)
    F = s.d_mid * np.fft.fft2(np.asarray(D, np.complex128), axes=(1, 2))
    out = []
    for p in pairs:
        d0 = F[p.f, p.key0[:, 0], p.key0[:, 1]]
        d1 = F[p.f, p.key1[:, 0], p.key1[:, 1]]
        out.append((d0, d1))
    return out


def _signed(u, N):
    return u if u < (N + 1) // 2 else u - N


def _areal_rows(s, D, pairs):
    N, nh = s.n_mid, s.n_off
    M = 2 * N
    D = np.asarray(D, np.complex128).reshape(len(s.freqs), M, M, M, M)
    F = (s.d_mid ** 2) * np.fft.fftn(D, axes=(1, 2, 3, 4))
    out = []
    for p in pairs:
        ux, uy = divmod(p.u, N)
        qx, qy = _signed(ux, N), _signed(uy, N)
        n = p.key0[:, 1]
        nx, ny = n // nh - nh // 2, n % nh - nh // 2
        ax, ay = (qx + 2 * nx) % M, (qy + 2 * ny) % M
        bx, by = (qx - 2 * nx) % M, (qy - 2 * ny) % M
        d0 = F[p.f, ax, ay, bx, by] / 4.0
        d1 = F[p.f, (-bx) % M, (-by) % M, (-ax) % M, (-ay) % M] / 4.0
        out.append((d0, d1))
    return out


def model_from_spectrum(s, V):
    """V~ (n_km, nz) in fftfreq order -> the real model: (N, nz) in 2D,
    (N, N, nz) in 3D, (N_x, N_y, nz) on the survey of parallel lines (k_m
    index ux N_y + c, the inverse DFT over x and over the line index)."""
    V = np.asarray(V, np.complex128)
    if getattr(s, "n_line", 0):
        return np.real(np.fft.ifft2(V.reshape(s.n_mid, s.n_line, -1), axes=(0, 1)))
    if getattr(s, "dim", 2) == 3:
        N = s.n_mid
        return np.real(np.fft.ifft2(V.reshape(N, N, -1), axes=(0, 1)))
    return np.real(np.fft.ifft(V, axis=0))


def _line_rows(s, D, pairs):
    Ny, N = s.n_line, s.n_mid
    D = np.asarray(D, np.complex128).reshape(len(s.freqs), Ny, N, N)
    F = s.d_mid * np.fft.fftn(D, axes=(1, 2, 3))
    out = []
    for p in pairs:
        d0 = F[p.f, p.key0[:, 2], p.key0[:, 0], p.key0[:, 1]]
        d1 = F[p.f, p.key1[:, 2], p.key1[:, 0], p.key1[:, 1]]
        out.append((d0, d1))
    return out
