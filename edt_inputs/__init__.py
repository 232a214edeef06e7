"""Seeded synthetic inputs for extended diffraction tomography (EDT).

This module is the one piece shared by the FP64 oracle and the GPU harness. It
holds no arithmetic of the method itself: it only fixes survey geometry, draws
the layered reference medium, draws the scattering-potential model V(x, z), and
supplies counter-based Gaussian noise.  Everything that maps V to data or data
to V (Green's functions, Born rows, normal equations) lives elsewhere, twice:
once in ``oracle/`` and once in the HIP library.

Workloads follow the paper's setting (Section 3.1): 2D surface reflection
surveys with sources and receivers at z = 0, data in the frequency domain with
a complex frequency w + i*eps (eps = 0.15 1/s as in Section 3.1), a reference
velocity that depends on depth only, and a dimensionless perturbation V.
The five named workloads (``make_config(1..5)``) are seeded, synthetic
stand-ins at the sizes the benchmark is quoted on; no public data set is used.

Conventions
-----------
* Horizontal positions x_n = n*dx, periodic with period L = N*dx.
* Horizontal wavenumbers are held in numpy ``fftfreq`` order: index n in
  [0, N) has signed integer q = n for n < (N+1)//2 and q = n - N otherwise, and
  k = q * 2*pi/L.
* Depth samples are cell centres z_i = z0 + i*dz with z0 = dz/2.
* A layer stack is (vel[0..L-1], zif[0..L-2]): layer 0 extends upward to
  -infinity and holds the sources (so zif[0] > 0), layer L-1 is a half space.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = ["Survey", "make_config", "make_custom", "make_lines", "staircase_layers",
           "vhat", "noise", "signed_index", "CONFIG_NAMES"]

EPS_DEFAULT = 0.15  # imaginary part of the angular frequency, 1/s (Section 3.1)

CONFIG_NAMES = {
    1: "2d-gradient-N64-nz64-nf32",
    2: "2d-8layer-N512-nz256-nf128",
    3: "2d-8layer-N512-nz128-nf64-grad",
    4: "3d-areal-128x128-kh64x64-nz200-nf96",
    5: "3d-areal-256x256-kh96x96-nz400-nf160",
}


@dataclasses.dataclass
class Survey:
    """One synthetic survey: geometry, frequencies, reference medium, model."""
    name: str
    dim: int                     # 2: split-spread line survey; 3: areal survey
    n_mid: int                   # 2D: N surface positions; 3D: N_m per axis
    d_mid: float                 # 2D: dx; 3D: midpoint spacing per axis
    n_off: int                   # 3D: N_h offset wavenumbers per axis (2D: 0)
    d_off: float                 # 3D: half-offset spacing (2D: 0.0)
    freqs: np.ndarray            # Hz, float64
    eps: float                   # imaginary frequency, 1/s
    nz: int
    dz: float
    z0: float
    kappa: float                 # evanescent cut factor
    vel: np.ndarray              # layer velocities, m/s
    zif: np.ndarray              # interface depths, m (len = n_layers - 1)
    lambda_rel: float
    noise_rel: float             # noise modulus relative to max |d| per frequency
    seed: int
    v_true: Optional[np.ndarray]  # 2D: (N, nz); 3D: (N, N, nz); lines: (N, N_y, nz); real float64
    data_c64: bool = False       # data rows delivered as complex64
    n_line: int = 0              # 3D line survey: number of parallel lines N_y (0: not a line survey)
    d_line: float = 0.0          # 3D line survey: line spacing dy

    @property
    def n_layers(self) -> int:
        return int(self.vel.shape[0])

    @property
    def n_freq(self) -> int:
        return int(self.freqs.shape[0])

    @property
    def n_km(self) -> int:
        if self.n_line:
            return self.n_mid * self.n_line
        return self.n_mid if self.dim == 2 else self.n_mid * self.n_mid

    @property
    def z(self) -> np.ndarray:
        return self.z0 + self.dz * np.arange(self.nz, dtype=np.float64)


def signed_index(n: np.ndarray, N: int) -> np.ndarray:
    """fftfreq-order index -> signed integer wavenumber index."""
    n = np.asarray(n)
    return np.where(n < (N + 1) // 2, n, n - N)


def staircase_layers(vfun, nz: int, dz: float):
    """Cell-wise constant medium: cell i = [i*dz, (i+1)*dz) at vfun(z_i).

    Cell 0 extends upward to -infinity and cell nz-1 downward to +infinity.
    Returns (vel[nz], zif[nz-1]).
    """
    zc = (np.arange(nz) + 0.5) * dz
    vel = np.asarray(vfun(zc), dtype=np.float64)
    zif = (np.arange(1, nz) * dz).astype(np.float64)
    return vel, zif


def _blobs(rng, N, dx, nz, dz, n_blobs=4, sigma=30.0, amp=0.05):
    """Sum of Gaussian blobs, random sign, centres uniform over the box.

    The x distance uses the minimum image of the periodic line.
    """
    L = N * dx
    Z = nz * dz
    cx = rng.uniform(0.0, L, n_blobs)
    cz = rng.uniform(0.0, Z, n_blobs)
    sgn = np.where(rng.uniform(size=n_blobs) < 0.5, -1.0, 1.0)
    x = np.arange(N) * dx
    z = (np.arange(nz) + 0.5) * dz
    v = np.zeros((N, nz))
    for b in range(n_blobs):
        ddx = x - cx[b]
        ddx = ddx - L * np.round(ddx / L)
        ddz = z - cz[b]
        v += sgn[b] * amp * np.exp(-(ddx[:, None] ** 2 + ddz[None, :] ** 2) / (2 * sigma ** 2))
    return v


def _smooth(rng, shape, spacing, ell=40.0, std=0.03):
    """Gaussian-filtered white noise rescaled to a given standard deviation.

    Horizontal axes wrap (periodic survey); depth reflects.
    """
    from scipy.ndimage import gaussian_filter
    w = rng.normal(0.0, std, size=shape)
    sig = [ell / s for s in spacing]
    modes = ["wrap"] * (len(shape) - 1) + ["reflect"]
    v = gaussian_filter(w, sigma=sig, mode=modes)
    v -= v.mean()
    v *= std / max(v.std(), 1e-300)
    return v


def _layers(rng, n, vlo, vhi, tlo=100.0, thi=600.0):
    vel = rng.uniform(vlo, vhi, n)
    thick = rng.uniform(tlo, thi, n - 1)
    return vel.astype(np.float64), np.cumsum(thick).astype(np.float64)


def make_config(i: int, with_model: bool = True) -> Survey:
    """The five named synthetic workloads, seeded with seed = i.

    Draw order: velocities, thicknesses, then the model V.  Data noise is
    counter-based (see ``noise``) and does not consume the generator stream.
    """
    if i == 1:
        N, dx, nz, dz = 64, 10.0, 64, 10.0
        vel, zif = staircase_layers(lambda z: 1500.0 + 0.5 * z, nz, dz)
        rng = np.random.default_rng(1)
        v = _blobs(rng, N, dx, nz, dz) if with_model else None
        return Survey(CONFIG_NAMES[1], 2, N, dx, 0, 0.0, np.linspace(5.0, 40.0, 32),
                      EPS_DEFAULT, nz, dz, dz / 2, 1.0, vel, zif, 1e-3, 0.0, 1, v)
    if i in (2, 3):
        rng = np.random.default_rng(2)
        vel, zif = _layers(rng, 8, 1500.0, 4000.0)
        N, dx = 512, 12.5
        nz, nf = (256, 128) if i == 2 else (128, 64)
        dz = 8.0
        v = _smooth(rng, (N, nz), (dx, dz)) if with_model else None
        return Survey(CONFIG_NAMES[i], 2, N, dx, 0, 0.0, np.linspace(3.0, 60.0, nf),
                      EPS_DEFAULT, nz, dz, dz / 2, 1.0, vel, zif, 1e-3, 0.05, i, v)
    if i == 4:
        rng = np.random.default_rng(4)
        vel, zif = _layers(rng, 6, 1600.0, 3800.0)
        Nm, dm, Nh = 128, 12.5, 64
        nz, dz = 200, 10.0
        v = _smooth(rng, (Nm, Nm, nz), (dm, dm, dz)) if with_model else None
        return Survey(CONFIG_NAMES[4], 3, Nm, dm, Nh, Nm * dm / (2 * Nh),
                      np.linspace(4.0, 48.0, 96), EPS_DEFAULT, nz, dz, dz / 2, 1.0,
                      vel, zif, 1e-3, 0.05, 4, v)
    if i == 5:
        rng = np.random.default_rng(5)
        vel, zif = _layers(rng, 12, 1500.0, 4500.0)
        Nm, dm, Nh = 256, 12.5, 96
        nz, dz = 400, 10.0
        v = _smooth(rng, (Nm, Nm, nz), (dm, dm, dz)) if with_model else None
        return Survey(CONFIG_NAMES[5], 3, Nm, dm, Nh, Nm * dm / (2 * Nh),
                      np.linspace(3.0, 60.0, 160), EPS_DEFAULT, nz, dz, dz / 2, 1.0,
                      vel, zif, 1e-3, 0.05, 5, v, data_c64=True)
    raise ValueError(f"unknown config {i}")


def make_custom(*, dim=2, N=32, dx=12.5, Nh=0, nz=24, dz=10.0, freqs=(5.0, 10.0, 15.0),
                vel=(2000.0,), zif=(), eps=EPS_DEFAULT, kappa=1.0, lambda_rel=1e-3,
                noise_rel=0.0, seed=0, model="smooth", data_c64=False,
                name="custom") -> Survey:
    """A small survey for tests; model is 'smooth', 'blobs', 'zero' or None."""
    rng = np.random.default_rng(seed)
    shape = (N, nz) if dim == 2 else (N, N, nz)
    spacing = (dx, dz) if dim == 2 else (dx, dx, dz)
    if model == "smooth":
        v = _smooth(rng, shape, spacing, ell=2.0 * max(dx, dz))
    elif model == "blobs":
        assert dim == 2
        v = _blobs(rng, N, dx, nz, dz, sigma=2.0 * max(dx, dz))
    elif model == "zero":
        v = np.zeros(shape)
    else:
        v = None
    d_off = (N * dx / (2 * Nh)) if dim == 3 else 0.0
    return Survey(name, dim, N, dx, Nh if dim == 3 else 0, d_off,
                  np.asarray(freqs, dtype=np.float64), float(eps), nz, dz, dz / 2,
                  float(kappa), np.asarray(vel, dtype=np.float64),
                  np.asarray(zif, dtype=np.float64), float(lambda_rel), float(noise_rel),
                  int(seed), v, data_c64)


def make_square_experiment(*, depth=1500.0, two_layer=False, freqs=(1.0, 2.0, 3.0, 4.0, 5.0), N=800,
                           tol_scale=None, seed=0) -> Survey:
    """The numerical examples of Section 3.2: a 2D line of N positions at 50 m
    (N = 800: the 40 km survey), depths 800-4000 m at 50 m, sources and
    receivers at z = 0, imaginary frequency 0.15 1/s; reference water
    (1500 m/s), or water above 1 km over 4000 m/s; model V = 1 inside a
    1 km square centred at x = 0 and the given depth, 0 elsewhere."""
    dx, dz, z0, nz = 50.0, 50.0, 800.0, 65
    vel = (1500.0, 4000.0) if two_layer else (1500.0,)
    zif = (1000.0,) if two_layer else ()
    n = np.arange(N)
    x = np.where(n < (N + 1) // 2, n, n - N) * dx
    z = z0 + dz * np.arange(nz)
    inside_x = (x >= -500.0) & (x < 500.0)
    inside_z = (z >= depth - 500.0) & (z < depth + 500.0)
    v = (inside_x[:, None] & inside_z[None, :]).astype(np.float64)
    return Survey("square", 2, N, dx, 0, 0.0, np.asarray(freqs, np.float64), EPS_DEFAULT, nz, dz, z0, 1.0,
                  np.asarray(vel, np.float64), np.asarray(zif, np.float64), 0.0, 0.0, int(seed), v, False)


def make_lines(*, Nx=16, dx=25.0, Ny=8, dy=50.0, nz=6, dz=20.0, freqs=(6.0, 11.0), vel=(1800.0, 2600.0),
               zif=(45.0,), eps=EPS_DEFAULT, kappa=1.0, lambda_rel=1e-3, noise_rel=0.0, seed=0,
               model="smooth", name="lines") -> Survey:
    """A 3D survey of N_y parallel 2D lines (Section 2.2): along each line
    N_x positions at dx, every source recorded by every receiver of its line;
    lines dy apart, periodic in y.  Model V on the (N_x, N_y, nz) grid."""
    rng = np.random.default_rng(seed)
    shape = (Nx, Ny, nz)
    if model == "smooth":
        v = _smooth(rng, shape, (dx, dy, dz), ell=2.0 * max(dx, dz))
    elif model == "zero":
        v = np.zeros(shape)
    else:
        v = None
    return Survey(name, 3, Nx, dx, 0, 0.0, np.asarray(freqs, dtype=np.float64), float(eps), nz, dz, dz / 2,
                  float(kappa), np.asarray(vel, dtype=np.float64), np.asarray(zif, dtype=np.float64),
                  float(lambda_rel), float(noise_rel), int(seed), v, False, int(Ny), float(dy))


def vhat(s: Survey) -> np.ndarray:
    """Unnormalised horizontal DFT of the model, fftfreq order.

    2D: shape (N, nz); 3D: shape (N*N, nz) with k_m index u = ux*N + uy.
    """
    if s.dim == 2:
        return np.fft.fft(s.v_true, axis=0)
    vh = np.fft.fft2(s.v_true, axes=(0, 1))
    return vh.reshape(s.n_km, s.nz)


# ---------------------------------------------------------------- noise ----
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea & Flood 2014), vectorised on uint64."""
    with np.errstate(over="ignore"):
        z = (x + np.uint64(0x9E3779B97F4A7C15)) & _M64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
        return z ^ (z >> np.uint64(31))


def noise(seed: int, f_idx, *keys) -> np.ndarray:
    """Counter-based standard complex normal numbers, E|n|^2 = 1.

    The value depends only on (seed, f_idx, *keys) -- integer arrays that
    broadcast together -- so any subset of data samples can be drawn in any
    order.  A SplitMix64 hash chain gives two uniforms, Box-Muller turns them
    into (xi1 + i*xi2)/sqrt(2).
    """
    arrs = np.broadcast_arrays(np.asarray(f_idx, dtype=np.int64),
                               *[np.asarray(k, dtype=np.int64) for k in keys])
    h = _splitmix64(np.full(arrs[0].shape, np.uint64(seed) + np.uint64(0x5EED), dtype=np.uint64))
    for a in arrs:
        h = _splitmix64(h ^ a.astype(np.uint64))
    h1 = _splitmix64(h ^ np.uint64(1))
    h2 = _splitmix64(h ^ np.uint64(2))
    u1 = ((h1 >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)
    u2 = ((h2 >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)
    r = np.sqrt(-2.0 * np.log(u1))
    return (r * np.cos(2 * np.pi * u2) + 1j * r * np.sin(2 * np.pi * u2)) / np.sqrt(2.0)
