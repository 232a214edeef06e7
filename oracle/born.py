"""Brute-force space-domain Born data on tiny periodic grids.

Paper, Section 2.1, eq. Born: D(x_R, x_S) = w^2 int dx int dz
G(x_R, 0; x, z) V(x, z) G(x, z; x_S, 0), with a laterally invariant reference
(eq. Invariant).  On a periodic line of N points (spacing dx, period L) the
reference Green's function is the image-summed field

    G_per(x, z) = (1/L) sum_{q in [-N/2, N/2)} e^{i k_q x} g(z; |k_q|),

and the integral becomes a Riemann sum over the same grid in x and the depth
cells z_i.  This module evaluates that double sum directly, point by point,
with no transform of the data; it is the independent check that the
wavenumber-domain rows (oracle.rows) carry the right indexing, pairing and
constants.
"""
from __future__ import annotations

import numpy as np

from .green import green, omega

__all__ = ["gper_2d", "born_2d", "gper_3d", "born_3d", "gper_rect", "born_lines"]


def gper_2d(vel, zif, w, N, dx, z):
    """G_per(x_n, z_i) for n in [0, N): shape (N, nz)."""
    L = N * dx
    q = np.arange(-(N // 2), N - N // 2)
    k = 2 * np.pi * q / L
    g = green(vel, zif, w, np.abs(k), z)            # (N, nz), row q
    x = np.arange(N) * dx
    ph = np.exp(1j * np.outer(x, k))               # (N_x, N_q)
    return ph @ g / L


def born_2d(vel, zif, f_hz, eps, V, dx, z, dz):
    """D[R, S] = w^2 dx dz sum_n sum_i G_per(x_R - x_n, z_i) V(x_n, z_i) G_per(x_n - x_S, z_i)."""
    N = V.shape[0]
    w = omega(f_hz, eps)
    Gp = gper_2d(vel, zif, w, N, dx, z)             # depends on (x mod L)
    D = np.zeros((N, N), np.complex128)
    for R in range(N):
        for S in range(N):
            acc = 0.0 + 0.0j
            for n in range(N):
                gr = Gp[(R - n) % N]
                gs = Gp[(n - S) % N]
                acc += np.sum(gr * V[n] * gs)
            D[R, S] = w * w * dx * dz * acc
    return D


def gper_3d(vel, zif, w, N, dx, z):
    """G_per on an N x N periodic surface grid: shape (N, N, nz), index (x, y)."""
    L = N * dx
    q = np.fft.fftfreq(N, d=1.0 / N)                # signed, fftfreq order
    kx, ky = np.meshgrid(2 * np.pi * q / L, 2 * np.pi * q / L, indexing="ij")
    kabs = np.hypot(kx, ky).ravel()
    uk, inv = np.unique(kabs, return_inverse=True)
    g = green(vel, zif, w, uk, z)[inv].reshape(N, N, -1)
    # G_per(x) = (1/L^2) sum_q e^{i k.x} g(|k|) = (N^2/L^2) * ifft2(g)
    return np.fft.ifft2(g, axes=(0, 1)) * (N * N) / (L * L)


def born_3d(vel, zif, f_hz, eps, V, dx, z, dz):
    """Full-coverage areal survey on an N x N periodic grid (every source to
    every receiver): D[R, S] = w^2 dx^2 dz sum_x sum_i G_per(x_R - x) V(x) G_per(x - S),
    with R, S, x flattened (x*N + y).  The x-sum is written as a product of
    the explicit (circulant) Green's matrices, one depth at a time."""
    N = V.shape[0]
    w = omega(f_hz, eps)
    Gp = gper_3d(vel, zif, w, N, dx, z)
    ix = np.arange(N)
    dxi = (ix[:, None] - ix[None, :]) % N           # (R_x - x_x) mod N
    D = np.zeros((N * N, N * N), np.complex128)
    for i in range(z.shape[0]):
        Gm = Gp[dxi[:, None, :, None], dxi[None, :, None, :], i].reshape(N * N, N * N)
        D += Gm @ (V[:, :, i].reshape(-1)[:, None] * Gm)
    return w * w * dx * dx * dz * D


def gper_rect(vel, zif, w, Nx, dx, Ny, dy, z):
    """G_per on an N_x x N_y periodic surface grid (spacings dx, dy): shape
    (N_x, N_y, nz), index (x, y); G_per(x, y) = (1/(L_x L_y)) sum_q e^{i k.x} g(|k|)."""
    Lx, Ly = Nx * dx, Ny * dy
    kx = 2 * np.pi * np.fft.fftfreq(Nx, d=1.0 / Nx) / Lx
    ky = 2 * np.pi * np.fft.fftfreq(Ny, d=1.0 / Ny) / Ly
    KX, KY = np.meshgrid(kx, ky, indexing="ij")
    kabs = np.hypot(KX, KY).ravel()
    uk, inv = np.unique(kabs, return_inverse=True)
    g = green(vel, zif, w, uk, z)[inv].reshape(Nx, Ny, -1)
    return np.fft.ifft2(g, axes=(0, 1)) * (Nx * Ny) / (Lx * Ly)


def born_lines(vel, zif, f_hz, eps, V, dx, dy, z, dz):
    """3D survey of parallel lines (paper eq. Born3D): V on an (N_x, N_y, nz)
    periodic grid, sources and receivers of line j at y_j, every source to
    every receiver of its own line:
        D[R, S, j] = w^2 dx dy dz sum_{n, m, i} G_per(x_R - x_n, y_j - y_m, z_i)
                     V(x_n, y_m, z_i) G_per(x_n - x_S, y_m - y_j, z_i)."""
    Nx, Ny, nz = V.shape
    w = omega(f_hz, eps)
    Gp = gper_rect(vel, zif, w, Nx, dx, Ny, dy, z)
    ix, iy = np.arange(Nx), np.arange(Ny)
    D = np.zeros((Nx, Nx, Ny), np.complex128)
    for j in range(Ny):
        for i in range(nz):
            Gr = Gp[(ix[:, None, None] - ix[None, :, None]) % Nx, (j - iy[None, None, :]) % Ny, i]   # [R, n, m]
            Gs = Gp[(ix[:, None, None] - ix[None, None, :]) % Nx, ((iy - j) % Ny)[None, :, None], i]  # [n, m, S]
            D[:, :, j] += np.einsum("rnm,nm,nms->rs", Gr, V[:, :, i], Gs)
    return w * w * dx * dy * dz * D
