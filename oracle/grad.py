"""Gradient of a loss on V~ with respect to the data, the damping and the
layer velocities of the reference medium.

The forward map is the one in oracle.solve (paper, Section 2.1, eqs. DMV,
Split; Tikhonov damping named in Section 4):

    b+ = (d0 + d1)/2,  b- = (d0 - d1)/(2i),  Ah = [Re A; Im A],
    H = Ah^T Ah + lambda I,  lambda = lambda_rel tr(Ah^T Ah)/nz,
    x+- = H^{-1} Ah^T bh+-,   V~(u) = x+ + i x-,  V~(-u) = x+ - i x-.

Given gV = dL/dRe V~ + i dL/dIm V~ (the complex-gradient convention of
PyTorch), the adjoint is, per pair:

    gx+ = Re gV(u) + Re gV(-u),   gx- = Im gV(u) - Im gV(-u)
    y+- = H^{-1} gx+-
    dL/dlambda = -sum y^T x
    dL/dbh+-   = Ah y+-
    dL/dAh     = sum [(bh - Ah x) y^T - (Ah y) x^T] + dL/dlambda * (2 lambda_rel/nz) Ah

and with A = w^2 dz g(k_r) g(k_s) (holomorphic in g) the table gradient is
gbar(k_r) += conj(w^2 dz g(k_s)) Abar and symmetrically, Abar = dL/dRe A +
i dL/dIm A.  Finally dL/dc_l = sum Re(conj(gbar) dg/dc_l) with dg/dc_l taken
in forward mode (oracle.green.green_tangent).  The evanescent-cut mask is held
fixed.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .green import green_tangent, omega
from .rows import row_values
from .solve import GTables

__all__ = ["grad", "grad_lines"]


def grad(s, pl, data, gV, lambda_rel=None, vel=None, pairs=None):
    """Returns dict(d=[(gd0, gd1) per pair], lambda_rel=float, vel=array,
    lambda_terms=array, lambda_abs=array): lambda_terms[p] = tr(G_p)/nz *
    dL/dlambda_p, the per-pair terms whose sum is dL/dlambda_rel, and
    lambda_abs[p] = tr(G_p)/nz * sum |y * x|, the magnitude a rounding error of
    the dot product -y.x is relative to."""
    lam_rel = s.lambda_rel if lambda_rel is None else lambda_rel
    vel = s.vel if vel is None else np.asarray(vel, np.float64)
    pairs = pl.pairs if pairs is None else pairs
    nz = s.nz
    # tables of g and dg/dc_l (forward mode, all layers)
    ks = {}
    for p in pairs:
        for f in np.unique(p.f):
            sel = p.f == f
            ks.setdefault(int(f), []).append(np.concatenate([p.kr[sel], p.ks[sel]]))
    tk, tg, tdg, tbar = {}, {}, {}, {}
    for f, parts in ks.items():
        uk = np.unique(np.concatenate(parts))
        g, dg = green_tangent(vel, s.zif, omega(s.freqs[f], s.eps), uk, s.z)
        tk[f], tg[f], tdg[f] = uk, g, dg
        tbar[f] = np.zeros_like(g)
    tabs = GTables(tk, tg)

    gd = []
    glam = 0.0
    lterms = []
    labs = []
    for p, (d0, d1) in zip(pairs, data):
        if p.n_rows == 0:
            gd.append((np.zeros(0, np.complex128), np.zeros(0, np.complex128)))
            lterms.append(0.0)
            labs.append(0.0)
            continue
        A = row_values(s, p, tabs.lookup)
        bp = 0.5 * (d0 + d1)
        bm = (d0 - d1) / 2j
        G = (A.conj().T @ A).real
        tr = float(np.trace(G))
        lam = lam_rel * tr / nz
        fac = scipy.linalg.cho_factor(G + lam * np.eye(nz), lower=True)
        c = np.stack([(A.conj().T @ bp).real, (A.conj().T @ bm).real])
        x = scipy.linalg.cho_solve(fac, c.T).T
        gx = np.zeros((2, nz))
        if p.self_conjugate:
            gx[0] = gV[p.u].real
        else:
            gx[0] = gV[p.u].real + gV[p.u_neg].real
            gx[1] = gV[p.u].imag - gV[p.u_neg].imag
        y = scipy.linalg.cho_solve(fac, gx.T).T
        if p.self_conjugate:
            y[1] = 0.0
        dlam = -float(np.sum(y * x))
        glam += dlam * tr / nz
        lterms.append(dlam * tr / nz)
        labs.append(float(np.sum(np.abs(y * x))) * tr / nz)
        Ay = A @ y.T                      # (R, 2): dL/db+-, complex
        gbp, gbm = Ay[:, 0], Ay[:, 1]
        gd.append((0.5 * gbp + 0.5j * gbm, 0.5 * gbp - 0.5j * gbm))
        # dL/dAh assembled directly in complex form: Abar = dL/dReA + i dL/dImA
        Ax = A @ x.T                      # (R, 2)
        res = np.stack([bp, bm], axis=1) - Ax
        Abar = res @ y - Ay @ x + dlam * (2.0 * lam_rel / nz) * A
        # chain into the g table
        for f in np.unique(p.f):
            sel = np.nonzero(p.f == f)[0]
            w = omega(s.freqs[f], s.eps)
            ir = np.searchsorted(tk[f], p.kr[sel])
            is_ = np.searchsorted(tk[f], p.ks[sel])
            gr, gs = tg[f][ir], tg[f][is_]
            ab = Abar[sel]
            np.add.at(tbar[f], ir, np.conj(w * w * s.dz * gs) * ab)
            np.add.at(tbar[f], is_, np.conj(w * w * s.dz * gr) * ab)
    gvel = np.zeros(vel.shape[0])
    for f in tk:
        gvel += np.einsum("kz,lkz->l", np.conj(tbar[f]), tdg[f]).real
    return dict(d=gd, lambda_rel=glam, vel=gvel, lambda_terms=np.array(lterms),
                lambda_abs=np.array(labs))


def grad_lines(s, pl, data, gV, lambda_rel=None, vel=None):
    """The same gradient on the survey of parallel lines (Section 2.2;
    oracle.lines3d): a row is A = (w^2 dz / L_y) sum_q g(k_a, k_q) g(k_b, k_{q-c})
    over its kept terms, so a row's Abar flows to both factors of every term:
    gbar(k_a, k_q) += conj(w^2 dz / L_y g(k_b, k_{q-c})) Abar and symmetrically.
    Returns dict(d=[(gd0, gd1) per pair], lambda_rel=float, vel=array)."""
    from .lines3d import _signed as signed, line_row_values
    lam_rel = s.lambda_rel if lambda_rel is None else lambda_rel
    vel = s.vel if vel is None else np.asarray(vel, np.float64)
    Nx, Ny, nz = int(s.n_mid), int(s.n_line), s.nz
    Ly = Ny * s.d_line
    dkx = 2.0 * np.pi / (Nx * s.d_mid)
    dky = 2.0 * np.pi / (Ny * s.d_line)
    ia, iq = np.arange(Nx // 2 + 1), np.arange(Ny // 2 + 1)
    K = np.sqrt((ia[:, None] * dkx) ** 2 + (iq[None, :] * dky) ** 2).ravel()
    shape = (ia.size, iq.size, nz)
    tab = np.zeros((s.n_freq,) + shape, np.complex128)
    dtab = np.zeros((s.n_freq, len(vel)) + shape, np.complex128)
    for f in range(s.n_freq):
        g, dg = green_tangent(vel, s.zif, omega(s.freqs[f], s.eps), K, s.z)
        tab[f] = g.reshape(shape)
        dtab[f] = dg.reshape((len(vel),) + shape)
    tbar = np.zeros_like(tab)
    gd = []
    glam = 0.0
    for p, (d0, d1) in zip(pl.pairs, data):
        if p.n_rows == 0:
            gd.append((np.zeros(0, np.complex128), np.zeros(0, np.complex128)))
            continue
        A = line_row_values(s, p, tab)
        bp = 0.5 * (d0 + d1)
        bm = (d0 - d1) / 2j
        G = (A.conj().T @ A).real
        tr = float(np.trace(G))
        lam = lam_rel * tr / nz
        fac = scipy.linalg.cho_factor(G + lam * np.eye(nz), lower=True)
        c = np.stack([(A.conj().T @ bp).real, (A.conj().T @ bm).real])
        x = scipy.linalg.cho_solve(fac, c.T).T
        gx = np.zeros((2, nz))
        if p.self_conjugate:
            gx[0] = gV[p.u].real
        else:
            gx[0] = gV[p.u].real + gV[p.u_neg].real
            gx[1] = gV[p.u].imag - gV[p.u_neg].imag
        y = scipy.linalg.cho_solve(fac, gx.T).T
        if p.self_conjugate:
            y[1] = 0.0
        dlam = -float(np.sum(y * x))
        glam += dlam * tr / nz
        Ay = A @ y.T
        gd.append((0.5 * Ay[:, 0] + 0.5j * Ay[:, 1], 0.5 * Ay[:, 0] - 0.5j * Ay[:, 1]))
        res = np.stack([bp, bm], axis=1) - A @ x.T
        Abar = res @ y - Ay @ x + dlam * (2.0 * lam_rel / nz) * A
        qc = signed(p.c, Ny)
        for r in range(p.n_rows):
            f, a, b, m = int(p.f[r]), abs(int(p.a[r])), abs(int(p.b[r])), int(p.mask[r])
            w = omega(s.freqs[f], s.eps)
            W = w * w * s.dz / Ly
            for bit in range(Ny):
                if not (m >> bit) & 1:
                    continue
                q = bit - Ny // 2
                pq = abs(signed((q - qc) % Ny, Ny))
                tbar[f, a, abs(q)] += np.conj(W * tab[f, b, pq]) * Abar[r]
                tbar[f, b, pq] += np.conj(W * tab[f, a, abs(q)]) * Abar[r]
    gvel = np.einsum("fabz,flabz->l", np.conj(tbar), dtab).real
    return dict(d=gd, lambda_rel=glam, vel=gvel)
