"""The 3D survey of many parallel 2D lines (test infrastructure, FP64, CPU).

Paper, Section 2.2 (eqs. Born3D, Invariant3D and the decoupled 3D equation
after them): the sources and receivers of each line lie along x at one y, and
the lines cover |y| <= c.  Transforming the data over midpoint, offset and
the line coordinate y, and letting both survey extents go to infinity, each
pair (k_m, k_y) is an independent 1D problem whose kernel is an integral
over the second offset wavenumber k_h'' (the y wavenumbers of the receiver
and source Green's functions differ by k_y but are otherwise free, since a
source and its receivers share one y).  The argument printed as k_m' in the
two Green's functions of that equation is read as the offset wavenumber k_h'
(the change of variables of eq. COV), and the aperture b is taken to
infinity as in the 2D rows.

Discrete, periodic statement used here.  N_x positions at dx along each line
(period L_x), N_y lines at dy (period L_y); on every line each source is
recorded by each receiver.  The data transform is

    d~(a, b, c) = dx sum_{R, S, j} D(x_R, x_S, y_j) e^{-2 pi i (a R + b S) / N_x} e^{-2 pi i c j / N_y},

and the subproblem of k_m index u and k_y index c has one row per frequency
f and receiver index a (source index b = u - a), whose value is

    A[(f, a), z] = (w_f^2 dz / L_y) sum_q g(z; |(k_a, k_q)|) g(z; |(k_b, k_{q - c})|),

the sum over the N_y wavenumber indices q of the periodic lines being the
discrete k_h'' quadrature (weight 2 pi / L_y over 2 pi).  With this
normalisation d~(a, b, c) = sum_i A[(f, a), z_i] V^(u, c, z_i), V^ the
unnormalised DFT of the model over x and y: exact up to rounding for the
periodic Born data (pinned by brute force in tests/test_oracle_lines3d.py).

Evanescent cut: a term q is kept iff |(k_a, k_q)| and |(k_b, k_{q-c})| are
both <= kappa 2 pi f / c_top (squared lengths compared in FP64, each written
as (n dk)*(n dk) + (m dk')*(m dk') with no fused multiply-add); a row is kept
iff one of its terms is.  The row of the pair's -k partner with the same
offset is (-b, -a) at (-u, -c); it has the same value (the sum over q is
over the whole periodic grid, so it can be re-indexed), so the two data
form one +-k pair as in the 2D split (eqs. VSym, Split).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .green import green, omega

__all__ = ["LinePair", "LinePlan", "plan_lines", "line_row_values", "line_tables", "forward_lines",
           "vhat_lines", "solve_lines"]

TWO_PI = 2.0 * np.pi


@dataclasses.dataclass
class LinePair:
    u: int                 # flattened k index ux * N_y + c of the representative
    u_neg: int             # index of the partner (-ux, -c)
    ux: int                # k_m index (fftfreq order)
    c: int                 # k_y index (fftfreq order)
    f: np.ndarray          # (R,) frequency index per row
    a: np.ndarray          # (R,) signed receiver wavenumber index
    b: np.ndarray          # (R,) signed source wavenumber index, b = u - a (wrapped)
    mask: np.ndarray       # (R,) uint64: bit (q + N_y/2) set iff term q is kept
    key0: np.ndarray       # (R, 3): (a, b, c) fftfreq indices of the datum at +k
    key1: np.ndarray       # (R, 3): (-b, -a, -c), the partner datum at -k

    @property
    def self_conjugate(self) -> bool:
        return self.u == self.u_neg

    @property
    def n_rows(self) -> int:
        return int(self.f.shape[0])


@dataclasses.dataclass
class LinePlan:
    n_km: int
    pairs: list
    ctop: float
    kmax: np.ndarray
    index: list


def _signed(n, N):
    return n if n < (N + 1) // 2 else n - N


def plan_lines(s, only=None) -> LinePlan:
    """Pairs and rows of the line survey s (fields n_mid = N_x, d_mid = dx,
    n_line = N_y, d_line = dy); pairs listed by their flattened index k =
    ux N_y + c ascending, k <= its partner's.  ``only``: survey pair indices."""
    Nx, Ny = int(s.n_mid), int(s.n_line)
    dkx = TWO_PI / (Nx * s.d_mid)
    dky = TWO_PI / (Ny * s.d_line)
    kmax = s.kappa * (TWO_PI * np.asarray(s.freqs, np.float64)) / float(s.vel[0])
    only = None if only is None else set(int(i) for i in only)
    qs = np.arange(-(Ny // 2), Ny - Ny // 2)
    pairs, index = [], []
    gp = -1
    for k in range(Nx * Ny):
        ux, c = divmod(k, Ny)
        kn = ((-ux) % Nx) * Ny + ((-c) % Ny)
        if kn < k:
            continue
        gp += 1
        if only is not None and gp not in only:
            continue
        index.append(gp)
        qc = _signed(c, Ny)
        fl, al, bl, ml = [], [], [], []
        for f in range(s.n_freq):
            K2 = kmax[f] * kmax[f]
            for a in range(-(Nx // 2), Nx - Nx // 2):
                b = _signed((ux - a) % Nx, Nx)
                m = 0
                for q in qs:
                    p = _signed(int(q - qc) % Ny, Ny)
                    kr2 = (a * dkx) * (a * dkx) + (q * dky) * (q * dky)
                    ks2 = (b * dkx) * (b * dkx) + (p * dky) * (p * dky)
                    if kr2 <= K2 and ks2 <= K2:
                        m |= 1 << int(q + Ny // 2)
                if m:
                    fl.append(f)
                    al.append(a)
                    bl.append(b)
                    ml.append(m)
        f_ = np.asarray(fl, np.int64)
        a_ = np.asarray(al, np.int64)
        b_ = np.asarray(bl, np.int64)
        key0 = np.stack([a_ % Nx, b_ % Nx, np.full(a_.shape, c)], axis=1) if a_.size else np.zeros((0, 3), np.int64)
        key1 = (np.stack([(-b_) % Nx, (-a_) % Nx, np.full(a_.shape, (-c) % Ny)], axis=1)
                if a_.size else np.zeros((0, 3), np.int64))
        pairs.append(LinePair(k, kn, ux, c, f_, a_, b_, np.asarray(ml, np.uint64), key0, key1))
    return LinePlan(Nx * Ny, pairs, float(s.vel[0]), kmax, index)


def line_tables(s, vel=None):
    """g(z; |(k_a, k_q)|, w_f) for every |a| <= N_x/2, |q| <= N_y/2 and frequency:
    array (n_freq, N_x/2 + 1, N_y/2 + 1, nz) complex128."""
    vel = s.vel if vel is None else vel
    Nx, Ny = int(s.n_mid), int(s.n_line)
    dkx = TWO_PI / (Nx * s.d_mid)
    dky = TWO_PI / (Ny * s.d_line)
    ia = np.arange(Nx // 2 + 1)
    iq = np.arange(Ny // 2 + 1)
    K = np.sqrt((ia[:, None] * dkx) ** 2 + (iq[None, :] * dky) ** 2).ravel()
    out = np.zeros((s.n_freq, ia.size, iq.size, s.nz), np.complex128)
    for f in range(s.n_freq):
        out[f] = green(vel, s.zif, omega(s.freqs[f], s.eps), K, s.z).reshape(ia.size, iq.size, s.nz)
    return out


def line_row_values(s, p: LinePair, tab):
    """Rows A (R, nz) of one pair: the sum over the kept terms q of the
    products of the receiver and source Green's functions."""
    Nx, Ny = int(s.n_mid), int(s.n_line)
    qc = _signed(p.c, Ny)
    A = np.zeros((p.n_rows, s.nz), np.complex128)
    Ly = Ny * s.d_line
    for r in range(p.n_rows):
        f, a, b, m = int(p.f[r]), int(p.a[r]), int(p.b[r]), int(p.mask[r])
        acc = np.zeros(s.nz, np.complex128)
        for bit in range(Ny):
            if not (m >> bit) & 1:
                continue
            q = bit - Ny // 2
            pq = _signed((q - qc) % Ny, Ny)
            acc += tab[f, abs(a), abs(q)] * tab[f, abs(b), abs(pq)]
        w = omega(s.freqs[f], s.eps)
        A[r] = (w * w * s.dz / Ly) * acc
    return A


def vhat_lines(s):
    """Unnormalised DFT of the model V (N_x, N_y, nz) over x and y, flattened
    to (N_x N_y, nz) with index ux N_y + c."""
    vh = np.fft.fft2(s.v_true, axes=(0, 1))
    return vh.reshape(s.n_mid * s.n_line, s.nz)


def forward_lines(s, pl: LinePlan, vh, tab):
    """Clean data (d at +k, d at -k) per pair: d = A V~."""
    out = []
    for p in pl.pairs:
        if p.n_rows == 0:
            out.append((np.zeros(0, np.complex128), np.zeros(0, np.complex128)))
            continue
        A = line_row_values(s, p, tab)
        out.append((A @ vh[p.u], A @ vh[p.u_neg]))
    return out


def solve_lines(s, pl: LinePlan, data, tab, lambda_rel=None):
    """Damped solve of every pair (the normal equations of oracle.solve on the
    line rows): V~ (N_x N_y, nz) and per-pair details."""
    from .solve import solve_pair
    V = np.zeros((pl.n_km, s.nz), np.complex128)
    info = []
    for p, (d0, d1) in zip(pl.pairs, data):
        A = line_row_values(s, p, tab) if p.n_rows else None
        x, inf, lam, tr = solve_pair(s, p, A, d0, d1, lambda_rel)
        V[p.u] = x[0] + 1j * x[1]
        if not p.self_conjugate:
            V[p.u_neg] = x[0] - 1j * x[1]
        info.append(dict(x=x, info=inf, lam=lam, trace=tr))
    return V, info
