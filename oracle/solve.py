"""Forward data, the damped normal equations and the recombined estimate.

Paper, Section 2.1, eqs. DMV, VSym and Split: the data at +k_m and -k_m are
combined as b+ = (d(k_m) + d(-k_m))/2 and b- = (d(k_m) - d(-k_m))/(2i); both
satisfy M x = b with the SAME kernel M and REAL unknowns x+ = Re V~(k_m),
x- = Im V~(k_m), which guarantees V~(-k_m) = conj V~(k_m) (eq. VSym).

For a real unknown and a complex matrix the least-squares normal equations
are Re(A^H A) x = Re(A^H b).  The paper solves each small system by a
truncated SVD (Section 3.1) and names Tikhonov damping as the next step
(Section 4); this oracle uses Tikhonov damping relative to the trace,

    (G + lambda I) x = c,   G = Re(A^H A),  c = Re(A^H b),
    lambda = lambda_rel * tr(G) / nz,

solved by a Cholesky factorisation (scipy.linalg.cho_factor).  A pair with no
rows gets V~ = 0.  A self-conjugate k_m (k_m = -k_m on the grid) has a real
V~: only x+ is solved and x- = 0.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg

from edt_inputs import noise, vhat
from .green import green, omega
from .rows import plan, row_values

__all__ = ["GTables", "gtables", "forward", "noise_scale", "add_noise", "synth_data",
           "normal_equations", "solve_pair", "solve", "pack", "INFO_OK", "INFO_EMPTY"]

INFO_OK = 0
INFO_EMPTY = -1


@dataclasses.dataclass
class GTables:
    """g(z; |k|, w_f) for every (f, |k|) some row needs, per frequency."""
    k: dict        # f -> sorted unique |k| values
    g: dict        # f -> complex128 (len(k), nz)

    def lookup(self, f, kvals):
        idx = np.searchsorted(self.k[f], kvals)
        assert np.array_equal(self.k[f][idx], kvals), "wavenumber missing from table"
        return self.g[f][idx]


def gtables(s, pl, vel=None, pairs=None):
    vel = s.vel if vel is None else vel
    pairs = pl.pairs if pairs is None else pairs
    ks = {}
    for p in pairs:
        for f in np.unique(p.f):
            sel = p.f == f
            ks.setdefault(int(f), []).append(np.concatenate([p.kr[sel], p.ks[sel]]))
    tk, tg = {}, {}
    for f, parts in ks.items():
        uk = np.unique(np.concatenate(parts))
        tk[f] = uk
        tg[f] = green(vel, s.zif, omega(s.freqs[f], s.eps), uk, s.z)
    return GTables(tk, tg)


def forward(s, pl, vh, tabs, pairs=None):
    """Clean Born data (d at +k_m, d at -k_m) per pair: d = A V~ (eq. DMV)."""
    pairs = pl.pairs if pairs is None else pairs
    out = []
    for p in pairs:
        if p.n_rows == 0:
            out.append((np.zeros(0, np.complex128), np.zeros(0, np.complex128)))
            continue
        A = row_values(s, p, tabs.lookup)
        out.append((A @ vh[p.u], A @ vh[p.u_neg]))
    return out


def noise_scale(s, pl, clean, pairs=None):
    """Per-frequency noise modulus: noise_rel * max |d| over all kept data."""
    pairs = pl.pairs if pairs is None else pairs
    mx = np.zeros(s.n_freq)
    for p, (d0, d1) in zip(pairs, clean):
        if p.n_rows == 0:
            continue
        m = np.maximum(np.abs(d0), np.abs(d1))
        np.maximum.at(mx, p.f, m)
    return s.noise_rel * mx


def add_noise(s, pl, clean, scale, pairs=None):
    """Add scale_f * n(seed, f, key) to every datum (counter-based noise)."""
    pairs = pl.pairs if pairs is None else pairs
    out = []
    for p, (d0, d1) in zip(pairs, clean):
        if p.n_rows == 0 or s.noise_rel == 0.0:
            out.append((d0.copy(), d1.copy()))
            continue
        n0 = noise(s.seed, p.f, *p.key0.T)
        n1 = noise(s.seed, p.f, *p.key1.T)
        out.append((d0 + scale[p.f] * n0, d1 + scale[p.f] * n1))
    return out


def synth_data(s, pl=None, tabs=None):
    """Noisy Born data of the survey's model; returns (plan, tables, data, scale)."""
    pl = plan(s) if pl is None else pl
    tabs = gtables(s, pl) if tabs is None else tabs
    clean = forward(s, pl, vhat(s), tabs)
    scale = noise_scale(s, pl, clean)
    return pl, tabs, add_noise(s, pl, clean, scale), scale


def normal_equations(A, d0, d1):
    """G = Re(A^H A), c = [Re(A^H b+), Re(A^H b-)], and tr(G)."""
    bp = 0.5 * (d0 + d1)
    bm = (d0 - d1) / 2j
    G = (A.conj().T @ A).real
    c = np.stack([(A.conj().T @ bp).real, (A.conj().T @ bm).real])
    return G, c, float(np.trace(G))


def solve_pair(s, p, A, d0, d1, lambda_rel=None, return_gram=False):
    """x (2, nz), info, lambda, trace for one pair (and the Gram G if
    return_gram)."""
    lam_rel = s.lambda_rel if lambda_rel is None else lambda_rel
    nz = s.nz
    if p.n_rows == 0:
        out = (np.zeros((2, nz)), INFO_EMPTY, 0.0, 0.0)
        return out + (np.zeros((nz, nz)),) if return_gram else out
    G, c, tr = normal_equations(A, d0, d1)
    lam = lam_rel * tr / nz
    fac = scipy.linalg.cho_factor(G + lam * np.eye(nz), lower=True)
    x = scipy.linalg.cho_solve(fac, c.T).T
    if p.self_conjugate:
        x[1] = 0.0
    return (x, INFO_OK, lam, tr, G) if return_gram else (x, INFO_OK, lam, tr)


def solve(s, pl, data, tabs, lambda_rel=None, pairs=None):
    """V~ estimate (n_km, nz) complex128 in fftfreq order, plus per-pair details."""
    pairs = pl.pairs if pairs is None else pairs
    V = np.zeros((pl.n_km, s.nz), np.complex128)
    info = []
    for p, (d0, d1) in zip(pairs, data):
        A = row_values(s, p, tabs.lookup) if p.n_rows else None
        x, inf, lam, tr = solve_pair(s, p, A, d0, d1, lambda_rel)
        V[p.u] = x[0] + 1j * x[1]
        if not p.self_conjugate:
            V[p.u_neg] = x[0] - 1j * x[1]
        info.append(dict(x=x, info=inf, lam=lam, trace=tr))
    return V, info


def pack(pl, data, pairs=None):
    """Concatenate per-pair data into rows (R, 2) and offsets (P+1,)."""
    pairs = pl.pairs if pairs is None else pairs
    off = np.zeros(len(pairs) + 1, np.int64)
    off[1:] = np.cumsum([p.n_rows for p in pairs])
    d = np.zeros((off[-1], 2), np.complex128)
    for i, (d0, d1) in enumerate(data):
        d[off[i]:off[i + 1], 0] = d0
        d[off[i]:off[i + 1], 1] = d1
    return d, off
