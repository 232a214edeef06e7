"""The decoupled 1D problems: wavenumbers, the evanescent cut, pairs and rows.

Paper, Section 2.1: after the Fourier transform over midpoint and offset and
the substitution w -> w + i eps, the data at one midpoint wavenumber k_m
depend only on V~(k_m, z) (eq. DMV) through the kernel M (eq. M), which is a
product of two reference Green's functions at k_r = (k_m + k_h)/2 and
k_s = (k_m - k_h)/2 (eq. COV).  Discretised on a depth grid (Section 3.1), one
datum -- a row -- is

    A[(f, k_r, k_s), i] = w_f^2 dz g(z_i; |k_r|, w_f) g(z_i; |k_s|, w_f).

The finite-aperture sinc of eq. M is dropped (infinite-aperture limit).  Rows
with an evanescent wavenumber are cut: a row is kept iff
|k_r| <= kappa * 2 pi f / c_top and |k_s| <= kappa * 2 pi f / c_top, where
c_top is the velocity of the layer holding the sources.  Several frequencies
are stacked into one system (Section 3.1).

Because g depends on |k| only, M(k_m) = M(-k_m) (the symmetry after eq. M),
so the problems at +k_m and -k_m share one row set; they form a *pair*.

2D (split-spread, periodic line of N positions, every source recorded by every
receiver): the DFT of the data over receiver and source positions couples
receiver wavenumber index a and source index b only through a + b = u (mod N),
the k_m index.  Rows of problem u are (f, a) with b = wrap(u - a); the row of
-u with the same k_h = k_a - k_b is (f, -b, -a).

3D (areal reading): k_m on an N_m x N_m grid with spacing dk, k_h on an
N_h x N_h grid with spacing 2 dk (offset extent half the midpoint extent).  In
units of dk/2, k_r = q_u + 2n and k_s = q_u - 2n for the signed k_m index q_u
and k_h index n; the row of -u is the same n with the same A.

Canonical row order inside a pair: frequency, then (2D) signed a ascending, or
(3D) n_x then n_y ascending.  Pairs are listed by their representative k_m
index u (fftfreq order) ascending, u <= its negative.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = ["Pair", "Plan", "plan", "kmax_of", "row_values"]

TWO_PI = 2.0 * np.pi


def kmax_of(f_hz, kappa, ctop):
    """Largest kept horizontal wavenumber at each frequency (evanescent cut)."""
    return kappa * (TWO_PI * np.asarray(f_hz, np.float64)) / ctop


@dataclasses.dataclass
class Pair:
    u: int                 # representative k_m index (fftfreq order; 3D flattened)
    u_neg: int             # index of -k_m
    f: np.ndarray          # (R,) frequency index per row
    kr: np.ndarray         # (R,) |k_r|
    ks: np.ndarray         # (R,) |k_s|
    key0: np.ndarray       # (R, nk) integer key of the datum at +k_m
    key1: np.ndarray       # (R, nk) integer key of the datum at -k_m (partner row)

    @property
    def self_conjugate(self) -> bool:
        return self.u == self.u_neg

    @property
    def n_rows(self) -> int:
        return int(self.f.shape[0])


@dataclasses.dataclass
class Plan:
    n_km: int
    pairs: list
    ctop: float
    kmax: np.ndarray
    index: list = None     # survey pair index of each listed pair (all pairs: 0..P-1)


def _ctop(s):
    return float(s.vel[0])


def _plan2d(s, only):
    N = s.n_mid
    dk = TWO_PI / (N * s.d_mid)
    kmax = kmax_of(s.freqs, s.kappa, _ctop(s))
    qs = np.arange(-(N // 2), N - N // 2)          # signed a, ascending
    pairs, index = [], []
    for u in range(N // 2 + 1):
        if only is not None and u not in only:
            continue
        index.append(u)
        un = (-u) % N
        fl, al, bl = [], [], []
        for f in range(s.n_freq):
            b = (u - qs) % N
            b = np.where(b < (N + 1) // 2, b, b - N)
            keep = (np.abs(qs) * dk <= kmax[f]) & (np.abs(b) * dk <= kmax[f])
            a_k, b_k = qs[keep], b[keep]
            fl.append(np.full(a_k.shape, f))
            al.append(a_k)
            bl.append(b_k)
        f_ = np.concatenate(fl).astype(np.int64)
        a_ = np.concatenate(al).astype(np.int64)
        b_ = np.concatenate(bl).astype(np.int64)
        # partner datum at -k_m with the same k_h: (-b, -a) (fftfreq indices)
        pa = (-b_) % N
        pb = (-a_) % N
        key0 = np.stack([a_ % N, b_ % N], axis=1)
        key1 = np.stack([pa, pb], axis=1)
        pairs.append(Pair(u, un, f_, np.abs(a_) * dk, np.abs(b_) * dk, key0, key1))
    return Plan(N, pairs, _ctop(s), kmax, index)


def _plan3d(s, only):
    N, Nh = s.n_mid, s.n_off
    if abs(Nh * s.d_off - N * s.d_mid / 2) > 1e-9 * N * s.d_mid:
        raise ValueError("3D areal reading needs N_h*dh = N_m*dm/2")
    dk = TWO_PI / (N * s.d_mid)
    hh = (0.5 * dk) * (0.5 * dk)
    kmax = kmax_of(s.freqs, s.kappa, _ctop(s))
    kmax2 = kmax * kmax
    ns = np.arange(-(Nh // 2), Nh - Nh // 2)
    nx, ny = np.meshgrid(ns, ns, indexing="ij")
    nx, ny = nx.ravel(), ny.ravel()
    pairs, index = [], []
    gp = -1   # survey pair index
    for u in range(N * N):
        ux, uy = divmod(u, N)
        un = ((-ux) % N) * N + ((-uy) % N)
        if un < u:
            continue
        gp += 1
        if only is not None and gp not in only:
            continue
        index.append(gp)
        qx = ux if ux < (N + 1) // 2 else ux - N
        qy = uy if uy < (N + 1) // 2 else uy - N
        sr = (qx + 2 * nx) ** 2 + (qy + 2 * ny) ** 2
        ss = (qx - 2 * nx) ** 2 + (qy - 2 * ny) ** 2
        fl, rl, sl, nl = [], [], [], []
        for f in range(s.n_freq):
            keep = (sr * hh <= kmax2[f]) & (ss * hh <= kmax2[f])
            idx = np.nonzero(keep)[0]
            fl.append(np.full(idx.shape, f))
            rl.append(sr[idx])
            sl.append(ss[idx])
            nl.append(idx)
        f_ = np.concatenate(fl).astype(np.int64)
        sr_ = np.concatenate(rl).astype(np.float64)
        ss_ = np.concatenate(sl).astype(np.float64)
        n_ = np.concatenate(nl).astype(np.int64)
        key0 = np.stack([np.full(n_.shape, u), n_], axis=1)
        key1 = np.stack([np.full(n_.shape, un), n_], axis=1)
        pairs.append(Pair(u, un, f_, np.sqrt(sr_) * (0.5 * dk), np.sqrt(ss_) * (0.5 * dk),
                          key0, key1))
    return Plan(N * N, pairs, _ctop(s), kmax, index)


def plan(s, only=None) -> Plan:
    """Enumerate pairs and rows of a survey (see module docstring).  ``only``:
    a set of survey pair indices (the pair order above) to list, e.g. a sample
    of a survey too large to enumerate whole; ``Plan.index`` gives each listed
    pair's survey index."""
    only = None if only is None else set(int(i) for i in only)
    if s.dim == 2:
        return _plan2d(s, only)
    if s.dim == 3:
        return _plan3d(s, only)
    raise ValueError("dim must be 2 or 3")


def row_values(s, pair: Pair, gfun):
    """Complex rows A (R, nz) of one pair.

    gfun(f_idx, kvals) -> g (len(kvals), nz) at frequency index f_idx.
    """
    from .green import omega
    A = np.zeros((pair.n_rows, s.nz), np.complex128)
    for f in np.unique(pair.f):
        sel = np.nonzero(pair.f == f)[0]
        kk = np.concatenate([pair.kr[sel], pair.ks[sel]])
        uk, inv = np.unique(kk, return_inverse=True)
        gt = gfun(int(f), uk)
        gr = gt[inv[: sel.shape[0]]]
        gs = gt[inv[sel.shape[0]:]]
        w = omega(s.freqs[f], s.eps)
        A[sel] = (w * w * s.dz) * gr * gs
    return A
