"""Pins of the sphere-motion oracle (App. B, Basset-Boussinesq-Oseen equation
of a sphere settling from rest): the implicit Euler scheme against closed
forms that share none of its code.

* Without the history and added-mass terms the equation is linear with an
  exponential solution; the scheme converges to it at first order.
* With both, the Laplace transform gives a closed form in Faddeeva functions
  (``stokes_exact``); the scheme converges to it, and the closed form has the
  initial slope kappa g / (kappa + 1/2) and the t^(-1/2) approach to the
  terminal speed that the transform predicts at small s.
* With the Clift-Gauvin drag and no history, the terminal speed balances the
  weight against 1/2 C_D pi r^2 u^2, solved here by bisection."""
import math

import numpy as np
import pytest

from oracle import bbo

KAPPA, NU, R, G = 2.7, 0.032, 8.0, 1.0e-5
K = 9.0 * NU / (2.0 * R * R)
UT = KAPPA * G / K


def test_without_history_is_the_exponential_at_first_order():
    errs = []
    for dt in (1.0, 0.5, 0.25):
        n = int(2000 / dt)
        u = bbo.settle(KAPPA, G, NU, R, dt, n, history=False, added_mass=False)
        t = dt * np.arange(n + 1)
        errs.append(np.abs(u - UT * (1.0 - np.exp(-K * t / KAPPA))).max() / UT)
    assert errs[-1] < 5e-5
    for a, b in zip(errs, errs[1:]):
        assert 1.8 < a / b < 2.2


def test_scheme_converges_to_the_laplace_closed_form():
    errs = []
    for dt in (4.0, 1.0, 0.25):
        n = int(4000 / dt)
        u = bbo.settle(KAPPA, G, NU, R, dt, n)
        t = dt * np.arange(n + 1)
        errs.append(np.abs(u - bbo.stokes_exact(KAPPA, G, NU, R, t)).max() / UT)
    assert errs[-1] < 5e-5
    for a, b in zip(errs, errs[1:]):
        assert 3.2 < a / b < 4.8


def test_closed_form_limits():
    # u(0) = 0 and initial acceleration kappa g / (kappa + 1/2)
    t = np.array([0.0, 1e-6, 2e-6])
    u = bbo.stokes_exact(KAPPA, G, NU, R, t)
    assert abs(u[0]) < 1e-18
    slope = u[1] / t[1]
    assert abs(slope / (KAPPA * G / (KAPPA + 0.5)) - 1.0) < 2e-3
    # small s: U ~ (u_T / s)(1 - (beta / k) sqrt(s)) -> u_T - u ~ u_T beta / (k sqrt(pi t))
    beta = 9.0 / (2.0 * R) * math.sqrt(NU)
    for tl in (1e7, 1e9):
        gap = UT - bbo.stokes_exact(KAPPA, G, NU, R, np.array([tl]))[0]
        assert abs(gap * K * math.sqrt(math.pi * tl) / (beta * UT) - 1.0) < 2e-2


def test_clift_gauvin_terminal_speed_balances_the_weight():
    g = 2.4e-6
    n = 40000
    u = bbo.settle(KAPPA, g, NU, R, 1.0, n, history=False, drag="clift_gauvin")
    # kappa g (4/3) pi r^3 = 1/2 C_D(Re) pi r^2 u^2, Re = 2 r u / nu, by bisection
    def residual(v):
        re = 2.0 * R * v / NU
        cd = 24.0 / re * (1.0 + 0.15 * re ** 0.687) + 0.42 / (1.0 + 4.25e4 * re ** -1.16)
        return KAPPA * g * 4.0 / 3.0 * R - 0.5 * cd * v * v
    lo, hi = 1e-6, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if residual(mid) > 0:
            lo = mid
        else:
            hi = mid
    assert u[-1] == pytest.approx(0.5 * (lo + hi), rel=1e-6)
    assert bbo.terminal_speed(KAPPA, g, NU, R, "clift_gauvin") == pytest.approx(0.5 * (lo + hi), rel=1e-9)
    # the Stokes drag would be lower: the corrected speed is below the Stokes one
    assert u[-1] < KAPPA * g / K
    # a drag scale for a given terminal speed reproduces that speed, and
    # scaling the drag up slows the sphere
    c = bbo.drag_scale_for(0.9 * u[-1], KAPPA, g, NU, R, "clift_gauvin")
    assert c > 1.0
    assert bbo.terminal_speed(KAPPA, g, NU, R, "clift_gauvin", c) == pytest.approx(0.9 * u[-1], rel=1e-9)
    us = bbo.settle(KAPPA, g, NU, R, 1.0, n, history=False, drag="clift_gauvin", drag_scale=c)
    assert us[-1] == pytest.approx(0.9 * u[-1], rel=1e-6)


# ------------------------------------------------------------ rotation
KR, RR, NUR, TQ = 100.0, 8.0, 0.1, 1e-3
IR = KR * 4.0 / 3.0 * math.pi * RR ** 3 * 0.4 * RR * RR
K0R = 8.0 * math.pi * NUR * RR ** 3


def test_spin_up_without_history_is_the_exponential():
    errs = []
    for dt in (40.0, 20.0, 10.0):
        n = int(4 * IR / K0R / dt)
        w = bbo.spin_up(IR, TQ, NUR, RR, dt, n, history=False)
        t = dt * np.arange(n + 1)
        errs.append(np.abs(w - TQ / K0R * (1.0 - np.exp(-K0R * t / IR))).max() / (TQ / K0R))
    assert errs[-1] < 5e-4
    for a, b in zip(errs, errs[1:]):
        assert 1.8 < a / b < 2.2


def test_spin_up_converges_to_the_laplace_closed_form():
    errs = []
    for dt in (40.0, 10.0, 2.5):
        n = int(4 * IR / K0R / dt)
        w = bbo.spin_up(IR, TQ, NUR, RR, dt, n)
        t = dt * np.arange(n + 1)
        errs.append(np.abs(w - bbo.spin_up_exact(IR, TQ, NUR, RR, t)).max() / (TQ / K0R))
    assert errs[-1] < 2e-4
    for a, b in zip(errs, errs[1:]):
        assert 3.2 < a / b < 4.8


def test_spin_up_closed_form_limits():
    w = bbo.spin_up_exact(IR, TQ, NUR, RR, np.array([0.0, 1e-3, 1e10]))
    assert abs(w[0]) < 1e-20
    assert abs(w[1] / 1e-3 / (TQ / IR) - 1.0) < 1e-3     # initial slope T / I
    assert abs(w[2] / (TQ / K0R) - 1.0) < 1e-8          # steady rotlet: T = 8 pi nu r^3 w
    # the history terms slow the approach: below the exponential at one relaxation time
    t1 = IR / K0R
    assert bbo.spin_up_exact(IR, TQ, NUR, RR, np.array([t1]))[0] < TQ / K0R * (1.0 - math.exp(-1.0))
