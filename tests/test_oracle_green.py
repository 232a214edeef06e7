"""Pins of the oracle's reference Green's function (paper Section 2.1, the
reference Helmholtz equation with a point source, and eq. Invariant).

Each test checks the generalised-reflection recursion against something that
does not share its algebra: textbook closed forms, the ODE and its interface
conditions evaluated directly, a 50-digit transfer-matrix (propagator)
solution, and the space-domain Green's function via the Weyl integral.
"""
import numpy as np
import pytest

from oracle.green import green, green_tangent, green_with_deriv, omega, kz

W = omega(12.0, 0.15)


def test_homogeneous_closed_form_through_recursion():
    # several interfaces with no contrast: every reflection coefficient is zero,
    # so the recursion must collapse to g = i e^{i kz |z|} / (2 kz)
    z = np.linspace(1.0, 1500.0, 300)
    k = np.array([0.0, 0.005, 0.02, 0.04, 0.06])      # includes evanescent ones
    g = green([1750.0] * 5, [100.0, 333.0, 700.0, 1200.0], W, k, z)
    q = np.sqrt(W ** 2 / 1750.0 ** 2 - k[:, None] ** 2 + 0j)
    ref = 1j * np.exp(1j * q * z) / (2 * q)
    assert np.max(np.abs(g - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_two_layer_closed_form():
    # reflection R = (k1-k2)/(k1+k2), transmission T = 2k1/(k1+k2)
    c1, c2, zeta = 1500.0, 4000.0, 1000.0
    z = np.linspace(1.0, 2500.0, 400)
    k = np.array([0.0, 0.01, 0.03, 0.049])
    g = green([c1, c2], [zeta], W, k, z)
    k1 = np.sqrt(W ** 2 / c1 ** 2 - k[:, None] ** 2 + 0j)
    k2 = np.sqrt(W ** 2 / c2 ** 2 - k[:, None] ** 2 + 0j)
    R = (k1 - k2) / (k1 + k2)
    T = 2 * k1 / (k1 + k2)
    above = (1j / (2 * k1)) * (np.exp(1j * k1 * z) + R * np.exp(1j * k1 * (2 * zeta - z)))
    below = (1j / (2 * k1)) * T * np.exp(1j * k1 * zeta) * np.exp(1j * k2 * (z - zeta))
    ref = np.where(z < zeta, above, below)
    assert np.max(np.abs(g - ref)) <= 1e-13 * np.max(np.abs(ref))


LAYERS = ([2154.0, 2246.0, 3536.0, 1730.0, 3000.0, 3321.0, 1970.0, 1638.0],
          [237.0, 666.0, 1047.0, 1222.0, 1539.0, 1973.0, 2285.0])


@pytest.mark.parametrize("f", [3.0, 25.0, 60.0])
def test_interface_continuity_and_source_jump(f):
    vel, zif = LAYERS
    w = omega(f, 0.15)
    kmax = 2 * np.pi * f / vel[0]
    k = np.linspace(0.0, kmax, 7)
    zi = np.asarray(zif)
    ga, da = green_with_deriv(vel, zif, w, k, zi, side="above")
    gb, db = green_with_deriv(vel, zif, w, k, zi, side="below")
    scale = np.max(np.abs(ga), axis=1, keepdims=True)
    assert np.max(np.abs(ga - gb) / scale) <= 1e-12
    dscale = np.max(np.abs(da), axis=1, keepdims=True)
    assert np.max(np.abs(da - db) / dscale) <= 1e-12
    # jump of g' across the source at z = 0 is -1 (the -delta source term)
    _, dp = green_with_deriv(vel, zif, w, k, np.array([1e-12]))
    _, dm = green_with_deriv(vel, zif, w, k, np.array([-1e-12]))
    assert np.max(np.abs((dp - dm)[:, 0] + 1.0)) <= 1e-9


def test_ode_residual_inside_layers():
    vel, zif = LAYERS
    f = 20.0
    w = omega(f, 0.15)
    k = np.array([0.0, 0.02, 0.05])
    h = 1e-3
    z = np.array([100.0, 400.0, 900.0, 1100.0, 1400.0, 1800.0, 2100.0, 2600.0])
    _, d_p = green_with_deriv(vel, zif, w, k, z + h)
    _, d_m = green_with_deriv(vel, zif, w, k, z - h)
    g, _ = green_with_deriv(vel, zif, w, k, z)
    lay = np.searchsorted(zif, z, side="right")
    c = np.asarray(vel)[lay]
    q2 = w ** 2 / c[None, :] ** 2 - k[:, None] ** 2
    res = (d_p - d_m) / (2 * h) + q2 * g
    assert np.max(np.abs(res) / (np.abs(q2 * g) + 1e-300)) <= 1e-6


def test_flux_conservation_without_damping():
    # at eps = 0 and a propagating k the energy flux Im(conj(g) g') is the same
    # constant in every layer below the source (no sources or sinks there)
    vel, zif = LAYERS
    w = omega(30.0, 0.0)
    k = np.array([0.0, 0.01, 0.02])          # propagating in every layer
    z = np.array([10.0, 300.0, 800.0, 1100.0, 1300.0, 1700.0, 2000.0, 2500.0, 4000.0])
    g, dg = green_with_deriv(vel, zif, w, k, z)
    flux = np.imag(np.conj(g) * dg)
    assert np.max(np.abs(flux - flux[:, :1]) / np.abs(flux[:, :1])) <= 1e-11


def _propagator_mp(vel, zif, f, eps, k, z, dps=50):
    """Independent 50-digit solution by transfer matrices, bottom to top."""
    import mpmath as mp
    mp.mp.dps = dps
    w = 2 * mp.pi * mp.mpf(f) + 1j * mp.mpf(eps)
    ks = [mp.sqrt(w ** 2 / mp.mpf(c) ** 2 - mp.mpf(k) ** 2) for c in vel]
    ks = [q if mp.im(q) > 0 else -q for q in ks]
    L = len(vel)
    bounds = [mp.mpf(b) for b in zif]

    def state_at(zq):
        """(g, g') at depth zq >= 0 of the solution that radiates downward in
        the bottom half space, e^{i k_L (z - zif[-1])}, propagated upward."""
        zq = mp.mpf(zq)
        if L == 1:
            e = mp.exp(1j * ks[0] * zq)
            return e, 1j * ks[0] * e
        zb = bounds[-1]
        if zq >= zb:
            e = mp.exp(1j * ks[-1] * (zq - zb))
            return e, 1j * ks[-1] * e
        gv, dv = mp.mpc(1), 1j * ks[-1]
        zc = zb
        for j in range(L - 2, -1, -1):
            top = bounds[j - 1] if j >= 1 else zq
            tgt = max(top, zq)
            d = zc - tgt
            q = ks[j]
            cs, sn = mp.cos(q * d), mp.sin(q * d)
            gv, dv = cs * gv - sn / q * dv, q * sn * gv + cs * dv
            zc = tgt
            if tgt == zq:
                break
        return gv, dv

    g0, d0 = state_at(0)
    C = -1 / (d0 + 1j * ks[0] * g0)
    out = []
    for zq in z:
        gv, _ = state_at(zq)
        out.append(complex(C * gv))
    return np.array(out)


@pytest.mark.parametrize("k", [0.0, 0.012, 0.03])
def test_against_50_digit_propagator(k):
    vel = [2000.0, 2600.0, 1700.0, 3200.0]
    zif = [150.0, 420.0, 610.0]
    z = np.array([5.0, 149.0, 151.0, 300.0, 500.0, 609.0, 700.0, 1200.0])
    f = 15.0
    ref = _propagator_mp(vel, zif, f, 0.15, k, z)
    g = green(vel, zif, omega(f, 0.15), np.array([k]), z)[0]
    assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_weyl_integral_homogeneous():
    # (i/4) H0^(1)(k0 r) = (1/2pi) int dk e^{ikx} g(z;|k|): invert the x-transform
    # numerically at strong damping so the x-integral converges absolutely.
    from scipy.integrate import quad
    from scipy.special import hankel1
    c, f = 2000.0, 8.0
    w = 2 * np.pi * f * (1 + 0.2j)
    k0 = w / c
    for k, z in [(0.0, 300.0), (0.01, 200.0), (0.02, 500.0)]:
        def fr(x, part):
            v = 0.25j * hankel1(0, k0 * np.hypot(x, z)) * np.cos(k * x)
            return v.real if part == 0 else v.imag
        X = 60000.0
        re = 2 * quad(fr, 0, X, args=(0,), limit=4000, epsabs=1e-16, epsrel=1e-13)[0]
        im = 2 * quad(fr, 0, X, args=(1,), limit=4000, epsabs=1e-16, epsrel=1e-13)[0]
        g = green([c], [], w, np.array([k]), np.array([z]))[0, 0]
        assert abs((re + 1j * im) - g) <= 1e-10 * abs(g)


def test_tangent_derivative_matches_fd():
    vel, zif = LAYERS
    w = omega(17.0, 0.15)
    k = np.array([0.0, 0.02, 0.045])
    z = np.linspace(4.0, 2500.0, 60)
    g, dg = green_tangent(vel, zif, w, k, z)
    for m in range(len(vel)):
        h = 1e-6 * vel[m]
        vp = list(vel)
        vm = list(vel)
        vp[m] += h
        vm[m] -= h
        fd = (green(vp, zif, w, k, z) - green(vm, zif, w, k, z)) / (2 * h)
        assert np.max(np.abs(fd - dg[m])) <= 1e-6 * np.max(np.abs(dg[m])) + 1e-300


def test_branch_has_positive_imaginary_part():
    k = np.linspace(0, 0.2, 50)
    for c in (1500.0, 4000.0):
        q = kz(omega(10.0, 0.15), c, k)
        assert np.all(q.imag > 0)
