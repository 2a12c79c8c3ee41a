"""FP64 reference of the sphere-motion equation of App. B: a sphere settling
from rest under the Basset-Boussinesq-Oseen (BBO) equation, the curve the
paper compares its transient settling velocity with (Sec. 3.1).

TEST INFRASTRUCTURE ONLY (tests and the benchmark's measurement legs); the
product path never imports it.

The equation as printed, in lattice units (fluid density 1), with u the
settling speed (positive downward):

    (kappa + 1/2) du/dt = kappa g - (9 nu / (2 r^2)) u
                          - (9 / (2 r)) sqrt(nu / pi) int_0^t u'(s) / sqrt(t - s) ds

Readings:
* the printed density symbol in the prefactor is the density ratio kappa, and
  the printed v in the drag term is the sphere speed u;
* the weight is kappa g without buoyancy, as in the translational update of
  Sec. 2.3;
* for finite Reynolds numbers the paper turns the drag curve of Sec. 3.2 into
  a trajectory through this equation; the Stokes drag term is then multiplied
  by C_D(Re) Re / 24 with Re = 2 r u / nu (``drag="clift_gauvin"``).

``settle`` integrates it with the implicit Euler scheme the paper names (time
step dt, the history integral with u' constant on each step, the drag
correction at the new speed by fixed-point iteration).  ``stokes_exact`` is the
closed-form solution of the Stokes form from its Laplace transform, an
independent check of the scheme.
"""
from __future__ import annotations

import math

import numpy as np


def clift_gauvin_cd(re):
    """Drag coefficient of Sec. 3.2 (Clift & Gauvin 1971)."""
    return 24.0 / re * (1.0 + 0.15 * re ** 0.687) + 0.42 / (1.0 + 4.25e4 * re ** -1.16)


def drag_factor(u, r, nu, drag):
    """Multiplier of the Stokes drag: 1, or C_D(Re) Re / 24."""
    if drag == "stokes":
        return 1.0
    re = 2.0 * r * abs(u) / nu
    if re < 1e-12:
        return 1.0
    return clift_gauvin_cd(re) * re / 24.0


def settle(kappa, g, nu, r, dt, nsteps, history=True, added_mass=True, drag="stokes", drag_scale=1.0):
    """Speeds u_0 = 0, u_1 .. u_nsteps at t_n = n dt (implicit Euler).

    With m = kappa (+ 1/2 for the added mass), k = 9 nu / (2 r^2) phi(u_n),
    c = (9 / (2 r)) sqrt(nu / pi) (0 without the history term) and
    H_n = sum_j (u_j - u_{j-1}) / dt * 2 (sqrt(t_n - t_{j-1}) - sqrt(t_n - t_j)),
    each step solves m (u_n - u_{n-1}) / dt = kappa g - k u_n - c H_n for u_n;
    H_n is linear in u_n through its last interval.  drag_scale multiplies
    the drag term (a drag law scaled to a given terminal speed)."""
    m = kappa + (0.5 if added_mass else 0.0)
    k0 = 9.0 * nu / (2.0 * r * r) * drag_scale
    c = 9.0 / (2.0 * r) * math.sqrt(nu / math.pi) if history else 0.0
    u = np.zeros(nsteps + 1)
    du = np.zeros(nsteps + 1)          # du[j] = u_j - u_{j-1}
    sq = np.sqrt(dt * np.arange(nsteps + 1))   # sqrt(t_n - t_j) = sq[n - j]
    cl = 2.0 / math.sqrt(dt)           # the last interval's weight: 2 sqrt(dt) / dt
    # interval j < n of H_n weighs du_j by wt[n - j], wt[i] = 2 (sqrt((i+1) dt) - sqrt(i dt)) / dt
    wt = np.zeros(nsteps + 1)
    wt[1:nsteps] = 2.0 * (sq[2:nsteps + 1] - sq[1:nsteps]) / dt
    for n in range(1, nsteps + 1):
        # the completed intervals j = 1 .. n-1 of the history integral
        hprev = float(np.dot(du[n - 1:0:-1], wt[1:n])) if c and n > 1 else 0.0
        un = u[n - 1]
        for _ in range(50):
            k = k0 * drag_factor(un, r, nu, drag)
            new = (kappa * g + (m / dt + c * cl) * u[n - 1] - c * hprev) / (m / dt + k + c * cl)
            if abs(new - un) <= 1e-15 * max(1.0, abs(new)):
                un = new
                break
            un = new
        u[n] = un
        du[n] = u[n] - u[n - 1]
    return u


def stokes_exact(kappa, g, nu, r, t, added_mass=True):
    """Closed form of the Stokes BBO equation from rest.

    The Laplace transform gives U(s) = kappa g / (s (m s + beta sqrt(s) + k))
    with m = kappa + 1/2, k = 9 nu / (2 r^2), beta = (9 / (2 r)) sqrt(nu).
    With p1, p2 the roots of m p^2 + beta p + k and the transform pair
    1 / (s (sqrt(s) - a)) <-> -(1 - exp(a^2 t) erfc(-a sqrt(t))) / a:
    u(t) = kappa g / (m (p1 - p2)) [-(1 - E(p1)) / p1 + (1 - E(p2)) / p2],
    E(p) = exp(p^2 t) erfc(-p sqrt(t)) = w(-i p sqrt(t)) (Faddeeva w)."""
    from scipy.special import wofz
    m = kappa + (0.5 if added_mass else 0.0)
    k = 9.0 * nu / (2.0 * r * r)
    beta = 9.0 / (2.0 * r) * math.sqrt(nu)
    disc = complex(beta * beta - 4.0 * m * k)
    p1 = (-beta + np.sqrt(disc)) / (2.0 * m)
    p2 = (-beta - np.sqrt(disc)) / (2.0 * m)
    t = np.asarray(t, dtype=float)
    rt = np.sqrt(t)
    e1 = wofz(-1j * p1 * rt)
    e2 = wofz(-1j * p2 * rt)
    u = kappa * g / (m * (p1 - p2)) * (-(1.0 - e1) / p1 + (1.0 - e2) / p2)
    return u.real


def terminal_speed(kappa, g, nu, r, drag="stokes", drag_scale=1.0):
    """The speed at which the (scaled) drag balances the weight kappa g:
    drag_scale (9 nu / (2 r^2)) phi(u) u = kappa g, by bisection."""
    k0 = 9.0 * nu / (2.0 * r * r) * drag_scale
    lo, hi = 0.0, kappa * g / k0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if k0 * drag_factor(mid, r, nu, drag) * mid < kappa * g:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def drag_scale_for(u_target, kappa, g, nu, r, drag="stokes"):
    """The drag scale whose terminal speed is u_target (the weight over the
    unscaled drag at that speed)."""
    k0 = 9.0 * nu / (2.0 * r * r)
    return kappa * g / (k0 * drag_factor(u_target, r, nu, drag) * u_target)
