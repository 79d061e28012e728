"""Pins of the oracle's ode45 stepper and step-size control (Fig. 2, the
algorithm shared by ode45 and ode45gpu; Sec. 3.1: the step shrinks when the
error estimate exceeds the tolerance and may grow otherwise).

What fixes each value here: the stability polynomial of the Dormand-Prince
pair, exact quadrature of polynomials, the observed convergence orders 5 and
4, closed-form solutions of linear problems, and invariants of the driver.
The control constants themselves (safety 0.8, exponent 1/5, shrink floor 0.1,
halving after a repeated failure, growth cap 5, 1.1 stretch, 16 eps(t) floor)
are ode45's documented rule; no MATLAB is available, so agreement with
MATLAB's own step sequence is parity unpinned."""
import math
from fractions import Fraction

import numpy as np
import pytest

R5 = [1.0, 1.0, 1 / 2, 1 / 6, 1 / 24, 1 / 120, 1 / 600]   # stability polynomial


def _matpoly(coeffs, M):
    out = np.zeros_like(M)
    P = np.eye(len(M))
    for c in coeffs:
        out = out + c * P
        P = P @ M
    return out


def _embedded_coeffs(aio):
    t = aio.tableau()
    a = [[Fraction(x).limit_denominator(10**6) for x in row] for row in t["a"]]
    bh = [Fraction(x).limit_denominator(10**6) for x in t["bhat"]]
    coeffs, v = [1.0], [Fraction(1)] * 7
    for _ in range(7):
        coeffs.append(float(sum(w * x for w, x in zip(bh, v))))
        v = [sum(a[i][j] * v[j] for j in range(7)) for i in range(7)]
    return coeffs


def test_attempt_on_linear_system_is_stability_polynomial(aio):
    rng = np.random.default_rng(3)
    M = rng.standard_normal((6, 6))
    y = rng.standard_normal(6)
    for h in (0.05, 0.2, 0.5):
        ynew, eps = aio.linear_attempt(M, 0.0, h, y)
        expect = _matpoly(R5, h * M) @ y
        np.testing.assert_allclose(ynew, expect, rtol=1e-12, atol=1e-13 * np.abs(expect).max())
        yhat = ynew - h * eps
        expect_hat = _matpoly(_embedded_coeffs(aio), h * M) @ y
        np.testing.assert_allclose(yhat, expect_hat, rtol=1e-12,
                                   atol=1e-13 * np.abs(expect_hat).max())


def test_attempt_scalar_against_exp(aio):
    # local error of one step on y' = lam y is O(z^6) with leading term
    # (1/600 - 1/720) z^6 = z^6 / 3600
    lam = -1.3
    for h in (0.01, 0.02, 0.04):
        ynew, _ = aio.linear_attempt(np.array([[lam]]), 0.0, h, np.array([1.0]))
        z = lam * h
        err = ynew[0] - math.exp(z)
        assert abs(err - z**6 / 3600) <= 0.05 * abs(z**6 / 3600) + 4e-16


@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4])
def test_polynomial_quadrature_and_stage_times(aio, deg):
    # y' = p(t): the fifth-order weights integrate degree <= 4 exactly, the
    # embedded fourth-order weights degree <= 3, and stage times enter through c
    coef = np.arange(1, deg + 2, dtype=float)
    p = np.polynomial.Polynomial(coef)
    P = p.integ()
    t, h = 0.7, 0.3
    ynew, eps = aio.rhs_attempt(lambda tt, y: np.array([p(tt)]), t, h, np.array([2.0]))
    assert ynew[0] == pytest.approx(2.0 + P(t + h) - P(t), rel=1e-14)
    if deg <= 3:
        assert abs(eps[0]) < 1e-13
    else:
        assert abs(eps[0]) > 1e-6


def _kepler(t, y):
    r3 = (y[0] ** 2 + y[1] ** 2) ** 1.5
    return np.array([y[2], y[3], -y[0] / r3, -y[1] / r3])


def _fixed_steps(aio, fun, y0, T, n, embedded=False):
    y, t, h = np.array(y0, float), 0.0, T / n
    for _ in range(n):
        ynew, eps = aio.rhs_attempt(fun, t, h, y)
        y = ynew - h * eps if embedded else ynew
        t += h
    return y


@pytest.mark.parametrize("embedded,order", [(False, 5), (True, 4)])
def test_observed_convergence_order(aio, embedded, order):
    # eccentric Kepler orbit: a nonlinear system that exercises all trees
    y0 = [0.5, 0.0, 0.0, math.sqrt(3.0)]           # e = 0.5, pericentre
    T = 2.0
    sols = [_fixed_steps(aio, _kepler, y0, T, n, embedded) for n in (40, 80, 160, 320)]
    d = [np.linalg.norm(sols[i] - sols[i + 1]) for i in range(3)]
    rates = [math.log2(d[i] / d[i + 1]) for i in range(2)]
    assert abs(rates[-1] - order) < 0.25, rates


def test_initial_step_rule(aio):
    rtol, thr = 1e-6, 1e-3
    y0 = np.array([2.0, 1e-5, -3.0])
    f0 = np.array([0.1, 4.0, 0.3])
    h = aio.initial_step(y0, f0, 0.0, 100.0, rtol, thr, 10.0)
    rh = np.max(np.abs(f0) / np.maximum(np.abs(y0), thr))
    # uncapped: the weighted first-order increment h f0 equals 0.8 rtol^(1/5)
    assert h * rh == pytest.approx(0.8 * rtol ** 0.2, rel=1e-14)
    # capped by hmax, by the span, and floored at 16 eps(t0)
    assert aio.initial_step(y0, 1e-9 * f0, 0.0, 100.0, rtol, thr, 10.0) == 10.0
    assert aio.initial_step(y0, 1e-9 * f0, 0.0, 3.0, rtol, thr, 10.0) == 3.0
    t0 = 1e6
    assert aio.initial_step(y0, 1e30 * f0, t0, t0 + 1, rtol, thr, 1.0) == 16 * aio.spacing(t0)


def test_spacing_is_eps(aio):
    assert aio.spacing(1.0) == np.finfo(float).eps
    assert aio.spacing(0.0) == 5e-324
    for t in (3.7, -1e12, 2.0**40):
        assert aio.spacing(t) == np.spacing(abs(t))


def test_error_norm_scaling(aio):
    eps = np.array([1e-3, -2e-3, 5e-4])
    y = np.array([1.0, 10.0, 1e-9])
    ynew = np.array([-4.0, 1.0, 1e-9])
    err = aio.error_norm(0.5, eps, y, ynew, 1e-2)
    assert err == pytest.approx(0.5 * max(1e-3 / 4.0, 2e-3 / 10.0, 5e-4 / 1e-2))
    assert math.isnan(aio.error_norm(1.0, np.array([np.nan, 1.0]), y[:2], ynew[:2], 1e-2))


def test_failure_and_success_rules(aio):
    # ode45's documented rule (parity with MATLAB unpinned): see module docstring
    rtol, hmin = 1e-6, 1e-12
    assert aio.step_after_failure(1.0, 2 * rtol, rtol, True, hmin) == pytest.approx(0.8 * 0.5 ** 0.2)
    assert aio.step_after_failure(1.0, 1e9 * rtol, rtol, True, hmin) == pytest.approx(0.1)
    assert aio.step_after_failure(1.0, 2 * rtol, rtol, False, hmin) == 0.5
    assert aio.step_after_failure(1e-12, 1e3 * rtol, rtol, True, 5e-13) == 5e-13
    assert aio.step_after_success(1.0, rtol / 32, rtol) == pytest.approx(1.0 / (1.25 * 0.5))
    assert aio.step_after_success(1.0, 0.0, rtol) == 5.0
    assert aio.step_after_success(1.0, rtol, rtol) == pytest.approx(0.8)


def test_driver_invariants_on_decay(aio):
    A = np.array([[-1.0]])
    ys, runs = [], []
    for rtol in (1e-5, 1e-10):
        y, run, th, hh = aio.linear_ode45(A, 0.0, 10.0, np.array([1.0]), rtol, 1e-14,
                                          hist_cap=100000)
        assert run["t_end"] == 10.0 and th[-1] == 10.0
        assert run["status"] == 2
        assert run["nfevals"] == 1 + 6 * (run["nsteps"] + run["nfailed"])
        assert np.all(np.diff(th) > 0) and hh.min() > 0
        assert th[0] == pytest.approx(hh[0])
        ys.append(abs(y[0] - math.exp(-10.0)) / math.exp(-10.0))
        runs.append(run)
    # accepted steps grow like rtol^(-1/5) (10x for 5 decades)
    ratio = runs[1]["nsteps"] / runs[0]["nsteps"]
    assert 7.0 < ratio < 13.0, ratio
    # the global error follows the tolerance
    assert ys[0] < 1e-4 and ys[1] < 1e-9 and ys[1] < 1e-3 * ys[0]


def test_rejections_after_sudden_stiffening(aio):
    fun = lambda t, y: np.array([-(1.0 if t < 1.0 else 60.0) * y[0]])
    y, run, th, hh = aio.rhs_ode45(fun, 0.0, 1.5, np.array([1.0]), 1e-8, 1e-14, hist_cap=10000)
    assert run["nfailed"] > 0 and run["status"] == 2 and run["t_end"] == 1.5
    exact = math.exp(-1.0) * math.exp(-60.0 * 0.5)
    assert y[0] == pytest.approx(exact, rel=1e-3)
    # step sizes after the switch are much smaller than before it
    assert hh[(th > 1.05) & (th < 1.2)].max() < 0.5 * hh[(th > 0.5) & (th < 0.95)].min()


def test_blow_up_ends_with_step_floor(aio):
    # y' = y^2, y(0) = 1 blows up at t = 1: the step collapses to 16 eps(t)
    y, run, _, _ = aio.rhs_ode45(lambda t, y: y * y, 0.0, 2.0, np.array([1.0]), 1e-6, 1e-6)
    assert run["status"] == 4
    assert abs(run["t_end"] - 1.0) < 1e-3
    assert run["h_next"] <= 16 * aio.spacing(run["t_end"])
    assert y[0] > 1e9


def test_rtol_floor_warning(aio):
    y, run, _, _ = aio.linear_ode45(np.array([[-1.0]]), 0.0, 1.0, np.array([1.0]), 1e-17, 1e-20)
    assert run["rc"] == 1 and run["rtol_raised"] == 1
    assert y[0] == pytest.approx(math.exp(-1.0), rel=1e-12)
