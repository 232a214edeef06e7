"""Reference Green's function of a depth-dependent (layered) medium.

Paper, Section 2.1: the reference Green's function solves the Helmholtz
equation with a point source, (w^2/c0(z)^2) G + lap G = -delta, for an acoustic
constant-density medium.  Lateral invariance (eq. Invariant) makes its
horizontal Fourier transform depend only on |k| (the evenness stated after
eq. M).  With G(x, z) = (1/2pi) int dk e^{ikx} g(z; |k|) the 1D problem is

    g'' + k_z(z)^2 g = -delta(z),   k_z^2 = w^2/c0(z)^2 - k^2,

for a source at depth 0, radiation (outgoing/decaying) conditions at +-inf,
and g, g' continuous at every interface.  The frequency is complex,
w = 2 pi f + i eps (Section 2.1, the substitution w -> w + i eps), so
Im(w^2) > 0 and the principal square root gives Im k_z > 0 on every layer.

The layered solution is built with the generalised reflection-coefficient
recursion (Kennett 1983; Chew 1990, Sec. 2.1): every exponential carries a
non-negative distance times i k_z, so nothing grows.  Layers are numbered
0..L-1 from the top; interface j (depth zif[j]) separates layers j and j+1;
layer 0 extends to -inf and holds the source, layer L-1 is a half space.

Forward-mode derivatives with respect to the layer velocities are carried by a
small dual-number type, so the same code path yields g and dg/dc_m.
"""
from __future__ import annotations

import numpy as np

__all__ = ["Dual", "omega", "kz", "green", "green_with_deriv", "green_tangent", "layer_of"]


def omega(f_hz, eps):
    """Complex angular frequency 2 pi f + i eps."""
    return 2.0 * np.pi * np.asarray(f_hz, dtype=np.float64) + 1j * eps


class Dual:
    """Complex value with tangents along several directions.

    ``v`` has shape S; ``d`` has shape (ndir,) + S.
    """
    __slots__ = ("v", "d")

    def __init__(self, v, d):
        self.v = v
        self.d = d

    @staticmethod
    def const(v, ndir):
        v = np.asarray(v, dtype=np.complex128)
        return Dual(v, np.zeros((ndir,) + v.shape, dtype=np.complex128))

    def _lift(self, o):
        """Lift o to a Dual and broadcast both operands to one value shape."""
        if not isinstance(o, Dual):
            o = np.asarray(o, dtype=np.complex128)
            o = Dual(o, np.zeros((self.d.shape[0],) + o.shape, dtype=np.complex128))
        shp = np.broadcast_shapes(self.v.shape, o.v.shape)
        nd = self.d.shape[0]

        def bc(x):
            v = np.broadcast_to(x.v, shp)
            d = x.d.reshape((nd,) + (1,) * (len(shp) - x.v.ndim) + x.v.shape)
            return Dual(v, np.broadcast_to(d, (nd,) + shp))
        return bc(self), bc(o)

    def __add__(self, o):
        a, b = self._lift(o)
        return Dual(a.v + b.v, a.d + b.d)
    __radd__ = __add__

    def __sub__(self, o):
        a, b = self._lift(o)
        return Dual(a.v - b.v, a.d - b.d)

    def __rsub__(self, o):
        a, b = self._lift(o)
        return Dual(b.v - a.v, b.d - a.d)

    def __neg__(self):
        return Dual(-self.v, -self.d)

    def __mul__(self, o):
        a, b = self._lift(o)
        return Dual(a.v * b.v, a.d * b.v + a.v * b.d)
    __rmul__ = __mul__

    def __truediv__(self, o):
        a, b = self._lift(o)
        q = a.v / b.v
        return Dual(q, (a.d - q * b.d) / b.v)

    def __rtruediv__(self, o):
        a, b = self._lift(o)
        q = b.v / a.v
        return Dual(q, (b.d - q * a.d) / a.v)

    def exp(self):
        e = np.exp(self.v)
        return Dual(e, self.d * e)


def _exp(x):
    return x.exp() if isinstance(x, Dual) else np.exp(x)


def kz(w, c, k):
    """Vertical wavenumber sqrt(w^2/c^2 - k^2) on the branch Im k_z > 0."""
    q = np.sqrt(np.asarray(w, dtype=np.complex128) ** 2 / c ** 2 - np.asarray(k) ** 2 + 0j)
    # principal sqrt of an upper-half-plane number lies in the first quadrant
    return q


def layer_of(z, zif):
    """Index of the layer containing depth z; a depth on an interface belongs below."""
    return np.searchsorted(np.asarray(zif), np.asarray(z), side="right")


def _recursion(kl, zif):
    """Generalised reflection coefficients Rh[j] (j=0..L-2) and rho[j] (j=1..L-1).

    kl: list of L arrays (or Duals) of vertical wavenumbers per layer.
    """
    L = len(kl)
    Rh = [None] * max(L - 1, 0)
    rho = [None] * L
    if L == 1:
        return Rh, rho
    rho[L - 1] = 0.0
    for j in range(L - 2, -1, -1):
        r = (kl[j] - kl[j + 1]) / (kl[j] + kl[j + 1])
        if j == L - 2:
            Rh[j] = r
        else:
            Rh[j] = (r + rho[j + 1]) / (1.0 + r * rho[j + 1])
        if j >= 1:
            h = zif[j] - zif[j - 1]
            rho[j] = Rh[j] * _exp(2j * kl[j] * h)
    return Rh, rho


def _amplitudes(kl, zif, Rh, rho):
    """Down-going amplitudes b[j] at the top of layer j (j = 1..L-1)."""
    L = len(kl)
    b = [None] * L
    if L == 1:
        return b
    b[1] = (1j / (2.0 * kl[0])) * _exp(1j * kl[0] * zif[0]) * (1.0 + Rh[0]) / (1.0 + rho[1])
    for j in range(1, L - 1):
        h = zif[j] - zif[j - 1]
        b[j + 1] = b[j] * _exp(1j * kl[j] * h) * (1.0 + Rh[j]) / (1.0 + rho[j + 1])
    return b


def _eval(kl, zif, Rh, b, j, z, deriv=False):
    """g (or dg/dz) in layer j at depths z (1D array)."""
    L = len(kl)
    k = kl[j]
    if j == 0:
        zz = np.abs(z)
        sg = np.sign(z)
        up = _exp(1j * k * zz)
        if L == 1:
            if deriv:
                return (1j / (2.0 * k)) * (1j * k * sg) * up
            return (1j / (2.0 * k)) * up
        refl = Rh[0] * _exp(1j * k * (2.0 * zif[0] - z))
        if deriv:
            return (1j / (2.0 * k)) * (1j * k * sg * up - 1j * k * refl)
        return (1j / (2.0 * k)) * (up + refl)
    if j == L - 1:
        e = _exp(1j * k * (z - zif[L - 2]))
        return b[j] * (1j * k) * e if deriv else b[j] * e
    dn = _exp(1j * k * (z - zif[j - 1]))
    upg = Rh[j] * _exp(1j * k * (2.0 * zif[j] - zif[j - 1] - z))
    if deriv:
        return b[j] * (1j * k) * (dn - upg)
    return b[j] * (dn + upg)


def _green_core(kl, zif, z, deriv=False):
    Rh, rho = _recursion(kl, zif)
    b = _amplitudes(kl, zif, Rh, rho)
    lay = layer_of(z, zif)
    out = None
    for j in np.unique(lay):
        sel = np.nonzero(lay == j)[0]
        val = _eval(kl, zif, Rh, b, int(j), z[sel], deriv)
        if out is None:
            if isinstance(val, Dual):
                shp = val.v.shape[:-1] + (z.shape[0],)
                out = Dual(np.zeros(shp, np.complex128),
                           np.zeros((val.d.shape[0],) + shp, np.complex128))
            else:
                out = np.zeros(np.shape(val)[:-1] + (z.shape[0],), np.complex128)
        if isinstance(val, Dual):
            out.v[..., sel] = val.v
            out.d[..., sel] = val.d
        else:
            out[..., sel] = val
    return out


def green(vel, zif, w, k, z):
    """g(z; |k|, w) for a 1D array of wavenumbers k and depths z.

    Returns complex128 of shape (len(k), len(z)).
    """
    vel = np.asarray(vel, np.float64)
    zif = np.asarray(zif, np.float64)
    k = np.asarray(k, np.float64)[:, None]
    z = np.asarray(z, np.float64)
    kl = [kz(w, c, k) for c in vel]
    return _green_core(kl, zif, z)


def green_with_deriv(vel, zif, w, k, z, side=None):
    """(g, dg/dz) at depths z; ``side`` in {None,'above','below'} picks the layer
    formula used at an interface depth ('above' = layer above the interface)."""
    vel = np.asarray(vel, np.float64)
    zif = np.asarray(zif, np.float64)
    k = np.asarray(k, np.float64)[:, None]
    z = np.asarray(z, np.float64)
    kl = [kz(w, c, k) for c in vel]
    Rh, rho = _recursion(kl, zif)
    b = _amplitudes(kl, zif, Rh, rho)
    lay = layer_of(z, zif) if side != "above" else np.searchsorted(zif, z, side="left")
    g = np.zeros((k.shape[0], z.shape[0]), np.complex128)
    dg = np.zeros_like(g)
    for j in np.unique(lay):
        sel = np.nonzero(lay == j)[0]
        g[:, sel] = _eval(kl, zif, Rh, b, int(j), z[sel])
        dg[:, sel] = _eval(kl, zif, Rh, b, int(j), z[sel], deriv=True)
    return g, dg


def green_tangent(vel, zif, w, k, z, dirs=None):
    """g and its derivatives with respect to layer velocities (forward mode).

    dirs: list of layer indices to differentiate along (default: all).
    Returns (g[len(k), len(z)], dg[len(dirs), len(k), len(z)]).
    dk_l/dc_l = -w^2 / (c_l^3 k_l) since k_l^2 = w^2/c_l^2 - k^2.
    """
    vel = np.asarray(vel, np.float64)
    zif = np.asarray(zif, np.float64)
    k = np.asarray(k, np.float64)[:, None]
    z = np.asarray(z, np.float64)
    if dirs is None:
        dirs = list(range(vel.shape[0]))
    nd = len(dirs)
    kl = []
    for l, c in enumerate(vel):
        kv = kz(w, c, k)
        d = np.zeros((nd,) + kv.shape, np.complex128)
        for t, m in enumerate(dirs):
            if m == l:
                d[t] = -(w ** 2) / (c ** 3 * kv)
        kl.append(Dual(kv, d))
    out = _green_core(kl, zif, z)
    return out.v, out.d
