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
"""
from __future__ import annotations

import numpy as np

__all__ = ["shots_to_rows", "model_from_spectrum"]


def shots_to_rows(s, pl, D, pairs=None):
    """2D: shot records D (n_freq, N, N) [f, receiver, source] -> list of
    (d+, d-) per pair, in the oracle's row order."""
    if getattr(s, "dim", 2) != 2:
        raise ValueError("shot records of the 2D line survey only")
    F = s.d_mid * np.fft.fft2(np.asarray(D, np.complex128), axes=(1, 2))
    pairs = pl.pairs if pairs is None else pairs
    out = []
    for p in pairs:
        d0 = F[p.f, p.key0[:, 0], p.key0[:, 1]]
        d1 = F[p.f, p.key1[:, 0], p.key1[:, 1]]
        out.append((d0, d1))
    return out


def model_from_spectrum(s, V):
    """V~ (n_km, nz) in fftfreq order -> the real model: (N, nz) in 2D,
    (N, N, nz) in 3D."""
    V = np.asarray(V, np.complex128)
    if getattr(s, "dim", 2) == 3:
        N = s.n_mid
        return np.real(np.fft.ifft2(V.reshape(N, N, -1), axes=(0, 1)))
    return np.real(np.fft.ifft(V, axis=0))
