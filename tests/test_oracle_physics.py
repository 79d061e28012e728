"""Pins of the oracle's equations of motion (Sec. 2.1: the Hamiltonian and
the force f(t, y)) and of whole trajectories against closed forms, invariants
and independent computations: the Hamiltonian's gradient, the harmonic trap,
free flight, the Mathieu equation (brute-force RK4 and the textbook edge of
its first stability region), two-body conservation laws with the trap off,
the head-on elastic collision and the classical deflection integral."""
import dataclasses
import math

import numpy as np
import pytest
from scipy import integrate, optimize

from paper_2509_12381_amd import workload as W

STATUS = {"escaped": 1, "tmax": 2, "maxsteps": 3, "hmin": 4, "nonfinite": 5}
O = W.OBS


def _liyb(**kw):
    s = W.liyb_system()
    return dataclasses.replace(s, **kw)


def _untrapped(**kw):
    return _liyb(a=(0.0, 0.0, 0.0), q=(0.0, 0.0, 0.0), omega_rf=0.0, **kw)


def _hamiltonian(s, t, y):
    """Sec. 2.1 Hamiltonian, written for complex-step differentiation."""
    xi, vi, xa, va = y[0:3], y[3:6], y[6:9], y[9:12]
    d = xi - xa
    r = np.sqrt(np.sum(d * d))
    h = 0.5 * s.m_atom * np.sum(va * va) + 0.5 * s.m_ion * np.sum(vi * vi)
    h = h - s.Cn / r**s.n + s.Cm / r**s.m
    for k in range(3):
        h = h + (s.a[k] + 2 * s.q[k] * math.cos(s.omega_rf * t)) * s.m_ion * s.omega_rf**2 / 8 * xi[k] ** 2
    return h


@pytest.mark.parametrize("n,m", [(4, 8), (6, 12), (4, 6), (3, 7)])
@pytest.mark.parametrize("r", [9.0, 40.0, 3000.0])
def test_force_is_minus_gradient_of_hamiltonian(aio, r, n, m):
    """For the configuration's C4/C8 and other exponents (Sec. 4.1), with the
    well at 10 a0 and 4.1e-3 E_h deep."""
    cn = 4.1e-3 * 10.0**n / (1.0 - n / m)
    s = _liyb(a=(1e-3, 2e-3, -3e-3), n=n, m=m, Cn=cn, Cm=n * cn * 10.0 ** (m - n) / m)
    rng = np.random.default_rng(int(r))
    y = rng.standard_normal(12) * np.array([50, 50, 50, 1e-7, 1e-7, 1e-7] * 2)
    u = rng.standard_normal(3)
    y[6:9] = y[0:3] + r * u / np.linalg.norm(u)
    t = 1.234e10
    f = aio.force(s, t, y)
    np.testing.assert_array_equal(f[0:3], y[3:6])
    np.testing.assert_array_equal(f[6:9], y[9:12])
    for k, mass in ((0, s.m_ion), (6, s.m_atom)):
        for c in range(3):
            yc = y.astype(complex)
            hstep = 1e-20 * max(1.0, abs(y[k + c]))
            yc[k + c] += 1j * hstep
            dH = _hamiltonian(s, t, yc).imag / hstep
            assert f[k + 3 + c] == pytest.approx(-dH / mass, rel=1e-12, abs=1e-30)
    assert aio.energy(s, t, y) == pytest.approx(_hamiltonian(s, t, y), rel=1e-13)


def test_harmonic_trap_closed_form(aio):
    # q = 0, Omega = 2, a_k = w_k^2 gives the harmonic trap (Sec. 4.1)
    w = np.array([0.3, 0.7, 1.1])
    s = _liyb(Cn=0.0, Cm=0.0, a=tuple(w**2), q=(0.0, 0.0, 0.0), omega_rf=2.0, r_exit=0.0)
    y0 = np.zeros(12)
    y0[0:3] = [1.0, -2.0, 0.5]
    y0[3:6] = [0.2, 0.1, -0.3]
    y0[6:9] = [1e6, 0, 0]
    T = 25.0
    yf, ob, rc = aio.integrate_one(s, 0.0, T, y0, 1e-11, 1e-13)
    assert rc == 0 and ob[O["status"]] == STATUS["tmax"] and ob[O["tend"]] == T
    x = y0[0:3] * np.cos(w * T) + y0[3:6] / w * np.sin(w * T)
    v = -y0[0:3] * w * np.sin(w * T) + y0[3:6] * np.cos(w * T)
    np.testing.assert_allclose(yf[0:3], x, rtol=0, atol=1e-8)
    np.testing.assert_allclose(yf[3:6], v, rtol=0, atol=1e-8)


def test_free_atom_moves_on_a_straight_line(aio):
    s = _liyb(Cn=0.0, Cm=0.0, r_exit=0.0)
    y0 = np.zeros(12)
    y0[0:3] = [100.0, -50.0, 30.0]
    y0[6:9] = [5e4, 2e4, -1e4]
    y0[9:12] = [-3e-7, 1e-7, 2e-7]
    T = W.rf_periods(s, 7.3)
    yf, ob, _ = aio.integrate_one(s, 0.0, T, y0, 1e-8, 1e-10)
    np.testing.assert_allclose(yf[6:9], y0[6:9] + y0[9:12] * T, rtol=1e-13)
    np.testing.assert_allclose(yf[9:12], y0[9:12], rtol=1e-14)
    assert ob[O["angle"]] < 1e-12 and ob[O["transfer"]] < 1e-15


def _mathieu_rk4(a, q, omega, x0, v0, T, nsteps):
    """Brute-force classical RK4 for x'' = -(a + 2q cos(omega t)) omega^2/4 x."""
    h = T / nsteps
    x, v, t = np.array(x0, float), np.array(v0, float), 0.0
    a, q = np.asarray(a), np.asarray(q)
    acc = lambda tt, xx: -(a + 2 * q * np.cos(omega * tt)) * omega**2 / 4 * xx
    for _ in range(nsteps):
        k1x, k1v = v, acc(t, x)
        k2x, k2v = v + h / 2 * k1v, acc(t + h / 2, x + h / 2 * k1x)
        k3x, k3v = v + h / 2 * k2v, acc(t + h / 2, x + h / 2 * k2x)
        k4x, k4v = v + h * k3v, acc(t + h, x + h * k3x)
        x = x + h / 6 * (k1x + 2 * k2x + 2 * k3x + k4x)
        v = v + h / 6 * (k1v + 2 * k2v + 2 * k3v + k4v)
        t += h
    return x, v


def test_ion_alone_follows_mathieu_equation(aio):
    s = _liyb(Cn=0.0, Cm=0.0, r_exit=0.0)
    y0 = np.zeros(12)
    y0[0:3] = [3000.0, -5000.0, 2000.0]
    y0[3:6] = [5e-8, 2e-8, -7e-8]
    y0[6:9] = [1e8, 0, 0]
    T = W.rf_periods(s, 3.0)
    yf, ob, _ = aio.integrate_one(s, 0.0, T, y0, 1e-12, 1e-14)
    x, v = _mathieu_rk4(s.a, s.q, s.omega_rf, y0[0:3], y0[3:6], T, 12000)
    np.testing.assert_allclose(yf[0:3], x, rtol=0, atol=1e-7 * np.abs(y0[0:3]).max())
    np.testing.assert_allclose(yf[3:6], v, rtol=0, atol=1e-7 * np.abs(v).max())


def _monodromy(aio, qz):
    s = _liyb(Cn=0.0, Cm=0.0, r_exit=0.0, a=(0.0, 0.0, 0.0), q=(0.0, 0.0, qz))
    T = W.rf_periods(s, 1.0)
    cols = []
    for x0, v0 in ((1.0, 0.0), (0.0, s.omega_rf)):
        y0 = np.zeros(12)
        y0[2], y0[5] = x0, v0
        y0[6:9] = [1e8, 0, 0]
        yf, _, _ = aio.integrate_one(s, 0.0, T, y0, 1e-12, 1e-30)
        cols.append([yf[2], yf[5] / s.omega_rf])
    return np.array(cols).T


@pytest.mark.parametrize("q,stable", [(0.2, True), (0.9, True), (0.92, False), (1.0, False)])
def test_mathieu_stability_edge(aio, q, stable):
    # first stability region of x'' + (a - 2q cos 2 tau) x = 0 at a = 0 ends at
    # |q| = 0.908; the Wronskian of the linear system is constant (det M = 1)
    M = _monodromy(aio, q)
    assert np.linalg.det(M) == pytest.approx(1.0, abs=1e-9)
    assert (abs(np.trace(M)) < 2.0) == stable


def _two_body_state(b, R0, v0, along=(0.0, 0.0, -1.0), side=(1.0, 0.0, 0.0)):
    y0 = np.zeros(12)
    along, side = np.array(along), np.array(side)
    y0[6:9] = -math.sqrt(R0**2 - b**2) * along + b * side
    y0[9:12] = v0 * along
    return y0


def _invariants(s, y):
    P = s.m_ion * y[3:6] + s.m_atom * y[9:12]
    L = s.m_ion * np.cross(y[0:3], y[3:6]) + s.m_atom * np.cross(y[6:9], y[9:12])
    return P, L


@pytest.mark.parametrize("b", [150.0, 1500.0])
def test_two_body_conservation_trap_off(aio, b):
    s = _untrapped(r_exit=3000.0)
    y0 = _two_body_state(b=b, R0=3000.0, v0=2e-6)
    y0[3:6] = [1e-8, -2e-8, 3e-8]
    yf, ob, _ = aio.integrate_one(s, 0.0, 1e15, y0, 1e-12, 1e-24)
    assert ob[O["status"]] == STATUS["escaped"]
    E0, E1 = aio.energy(s, 0.0, y0), aio.energy(s, 0.0, yf)
    # errors are relative to the largest energy met on the way: the kinetic
    # energy at the bottom of the well, D_e = C4^2 / (4 C8), for a close pass
    scale = s.Cn**2 / (4 * s.Cm) if ob[O["rmin"]] < 50 else abs(E0)
    assert abs(E1 - E0) < 100 * 1e-12 * scale
    P0, L0 = _invariants(s, y0)
    P1, L1 = _invariants(s, yf)
    # linear invariants are kept by every Runge-Kutta method up to rounding,
    # which accumulates at most linearly in the number of steps
    pscale = max(s.m_ion * np.abs(y0[3:6]).max(), s.m_atom * np.abs(y0[9:12]).max())
    nst = ob[O["nsteps"]] + ob[O["nfailed"]]
    np.testing.assert_allclose(P1, P0, rtol=0, atol=8 * nst * np.finfo(float).eps * pscale)
    np.testing.assert_allclose(L1, L0, rtol=0, atol=1e-12 * scale / abs(E0) * np.abs(L0).max())
    # centre of mass moves on a straight line
    M = s.m_ion + s.m_atom
    cm0 = (s.m_ion * y0[0:3] + s.m_atom * y0[6:9]) / M
    cm1 = (s.m_ion * yf[0:3] + s.m_atom * yf[6:9]) / M
    np.testing.assert_allclose(cm1, cm0 + P0 / M * ob[O["tend"]], rtol=0, atol=1e-9 * 3000)


def test_head_on_elastic_collision(aio):
    # b = 0, ion at rest, trap off: a one-dimensional elastic collision.  The
    # centre of mass keeps m_a v0 / M; the relative velocity reverses with the
    # speed that energy conservation gives at the final separation.
    s = _untrapped(r_exit=5000.0)
    v0 = math.sqrt(3 * W.KB * 1e-3 / s.m_atom)
    y0 = W.head_on_state(s, 5000.0, 1e-3, 0.4, 1.1)
    yf, ob, _ = aio.integrate_one(s, 0.0, 1e14, y0, 1e-13, 1e-26)
    u = y0[6:9] / 5000.0
    mi, ma = s.m_ion, s.m_atom
    M, mu = mi + ma, mi * ma / (mi + ma)
    V = lambda r: -s.Cn / r**4 + s.Cm / r**8
    erel = 0.5 * mu * v0**2 + V(5000.0)
    r_end = ob[O["dist"]]
    vrel = math.sqrt(2 * (erel - V(r_end)) / mu) * u        # atom minus ion, outgoing
    vcm = -ma * v0 / M * u
    # amplification of rtol through the well depth: D_e / E_rel ~ 1e6
    np.testing.assert_allclose(yf[9:12], vcm + mi / M * vrel, rtol=1e-6)
    np.testing.assert_allclose(yf[3:6], vcm - ma / M * vrel, rtol=1e-6)
    assert ob[O["status"]] == STATUS["escaped"]
    assert ob[O["bounces"]] == 1 and ob[O["lifetime"]] == 0.0
    assert ob[O["angle"]] == pytest.approx(math.pi, abs=1e-7)
    assert ob[O["transfer"]] == pytest.approx(2 * mu * v0, rel=1e-4)
    rt = optimize.brentq(lambda r: -s.Cn / r**4 + s.Cm / r**8 - erel, 5.0, 10.0)
    assert rt < ob[O["rmin"]] < rt * 1.01
    assert 0 < ob[O["position"]] < 100.0
    assert ob[O["ke"]] == pytest.approx(0.5 * mi * np.sum(yf[3:6] ** 2), rel=1e-15)


def _swept_angle_integral(s, y0, r_end):
    mu = s.m_ion * s.m_atom / (s.m_ion + s.m_atom)
    rho = y0[6:9] - y0[0:3]
    vrel = y0[9:12] - y0[3:6]
    r0 = np.linalg.norm(rho)
    V = lambda r: -s.Cn / r**s.n + s.Cm / r**s.m
    E = 0.5 * mu * vrel @ vrel + V(r0)
    L = mu * np.linalg.norm(np.cross(rho, vrel))
    rad = lambda r: 2.0 / mu * (E - V(r)) - L**2 / (mu**2 * r**2)
    # outermost turning point (b is well above the capture radius)
    rt = optimize.brentq(rad, 0.5 * np.linalg.norm(np.cross(rho, vrel)) / np.linalg.norm(vrel),
                         r0 * 0.999999, xtol=1e-14, rtol=1e-15)

    def piece(r_out):
        # r = rt + u^2 removes the inverse square-root singularity at rt
        g = lambda u: 2 * u * (L / (mu * (rt + u * u) ** 2)) / math.sqrt(rad(rt + u * u))
        val, _ = integrate.quad(g, 0.0, math.sqrt(r_out - rt), epsabs=0, epsrel=1e-13, limit=400)
        return val

    return piece(r0) + piece(r_end)


@pytest.mark.parametrize("b", [800.0, 2000.0])
def test_deflection_matches_quadrature(aio, b):
    s = _untrapped(r_exit=1e4)
    v0 = math.sqrt(3 * W.KB * 1e-3 / s.m_atom)
    y0 = _two_body_state(b=b, R0=1e4, v0=v0)
    yf, ob, _ = aio.integrate_one(s, 0.0, 1e15, y0, 1e-12, 1e-24)
    assert ob[O["status"]] == STATUS["escaped"]
    rho0, rho1 = y0[6:9] - y0[0:3], yf[6:9] - yf[0:3]
    swept = math.atan2(np.linalg.norm(np.cross(rho0, rho1)), rho0 @ rho1)
    expect = _swept_angle_integral(s, y0, np.linalg.norm(rho1))
    assert expect < math.pi
    assert swept == pytest.approx(expect, abs=1e-8)
