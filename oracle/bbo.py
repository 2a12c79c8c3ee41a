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


# ------------------------------------------------------------ rotation
# The rotational equation of App. B (Basset; Feuillebois & Lasek): a sphere of
# moment of inertia I spun up from rest by a constant torque T, fluid
# density 1, K0 = 8 pi nu r^3:
#
#   I dw/dt = T - K0 w - K0 (r / (3 sqrt(pi nu))) int_0^t w'(s) / sqrt(t - s) ds
#               + (K0 / 3) int_0^t w'(s) exp(a (t - s)) erfc(sqrt(a (t - s))) ds,
#   a = nu / r^2.
#
# Its Laplace transform is the unsteady Stokes torque on a rotating sphere,
# K0 W (1 + lam r + lam^2 r^2 / 3) / (1 + lam r) with lam = sqrt(s / nu).

def _erfc_kernel_integral(a, tau):
    """G(tau) = int_0^tau exp(a x) erfc(sqrt(a x)) dx
    = (exp(a tau) erfc(sqrt(a tau)) - 1 + 2 sqrt(a tau / pi)) / a."""
    from scipy.special import erfcx
    x = np.sqrt(a * np.asarray(tau, dtype=float))
    return (erfcx(x) - 1.0 + 2.0 * x / math.sqrt(math.pi)) / a


def spin_up(I, T, nu, r, dt, nsteps, history=True):
    """Angular speeds w_0 = 0, w_1 .. w_nsteps at t_n = n dt (implicit Euler,
    w' constant on each step: the 1/sqrt kernel integrates as in settle, the
    exp-erfc kernel through its antiderivative G)."""
    K0 = 8.0 * math.pi * nu * r ** 3
    c1 = r / (3.0 * math.sqrt(math.pi * nu)) if history else 0.0
    c2 = 1.0 / 3.0 if history else 0.0
    a = nu / (r * r)
    w = np.zeros(nsteps + 1)
    dw = np.zeros(nsteps + 1)
    sq = np.sqrt(dt * np.arange(nsteps + 1))
    wt1 = np.zeros(nsteps + 1)
    wt1[1:nsteps] = 2.0 * (sq[2:nsteps + 1] - sq[1:nsteps]) / dt
    Gs = _erfc_kernel_integral(a, dt * np.arange(nsteps + 1))
    wt2 = np.zeros(nsteps + 1)
    wt2[1:nsteps] = (Gs[2:nsteps + 1] - Gs[1:nsteps]) / dt
    l1, l2 = 2.0 / math.sqrt(dt), Gs[1] / dt     # the last interval's weights
    for n in range(1, nsteps + 1):
        h1 = float(np.dot(dw[n - 1:0:-1], wt1[1:n])) if n > 1 else 0.0
        h2 = float(np.dot(dw[n - 1:0:-1], wt2[1:n])) if n > 1 else 0.0
        # I (w_n - w_{n-1}) / dt = T - K0 w_n - K0 c1 (h1 + l1 dw_n) + K0 c2 (h2 + l2 dw_n)
        lhs = I / dt + K0 + K0 * c1 * l1 - K0 * c2 * l2
        rhs = T + (I / dt + K0 * c1 * l1 - K0 * c2 * l2) * w[n - 1] - K0 * c1 * h1 + K0 * c2 * h2
        w[n] = rhs / lhs
        dw[n] = w[n] - w[n - 1]
    return w


def spin_up_exact(I, T, nu, r, t):
    """Closed form from the Laplace transform.  With p = sqrt(s) and
    b = sqrt(nu) / r, W(s) = (T / I) (p + b) / (p^2 C(p)), C the cubic
    p^3 + (b + K0 / (3 b I)) p^2 + (K0 / I) p + K0 b / I with roots p_i; by
    partial fractions w(t) = (T / I) sum_i A_i (-(1 - E(p_i)) / p_i),
    A_i = (p_i + b) / prod_{j != i} (p_i - p_j), E(p) = exp(p^2 t) erfc(-p sqrt(t))."""
    from scipy.special import wofz
    K0 = 8.0 * math.pi * nu * r ** 3
    b = math.sqrt(nu) / r
    roots = np.roots([1.0, b + K0 / (3.0 * b * I), K0 / I, K0 * b / I]).astype(complex)
    t = np.asarray(t, dtype=float)
    rt = np.sqrt(t)
    out = np.zeros(t.shape, dtype=complex)
    for i, pi in enumerate(roots):
        Ai = (pi + b) / np.prod([pi - pj for j, pj in enumerate(roots) if j != i])
        out += Ai * (-(1.0 - wofz(-1j * pi * rt)) / pi)
    return (T / I * out).real
