"""Pins of the oracle's lattice, equilibrium, off-equilibrium and collision
(Sec. 2.1 and App. A) against mathematics independent of its code:
Maxwellian moments, Hermite orthogonality under the lattice weights,
brute-force full-tensor Hermite sums and conservation laws."""
import itertools
import math
import os

import numpy as np
import pytest

CS2 = 1.0 / 3.0
HERE = os.path.dirname(os.path.abspath(__file__))


def h1d(m, x):
    """One-dimensional Hermite polynomials of variance cs^2 up to order 2."""
    return (1.0, float(x), x * x - CS2)[m]


def multi_indices():
    return [(a, b, c) for c in range(3) for b in range(3) for a in range(3)]


def counts(idx):
    return tuple(sum(1 for a in idx if a == d) for d in range(3))


PRINTED = [(0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 2, 2), (1, 2, 2), (1, 1, 2), (0, 1, 2),
           (0, 0, 1, 1), (0, 0, 2, 2), (1, 1, 2, 2), (0, 1, 2, 2), (0, 1, 1, 2), (0, 0, 1, 2),
           (0, 0, 1, 2, 2), (0, 0, 1, 1, 2), (0, 1, 1, 2, 2), (0, 0, 1, 1, 2, 2)]


def test_weights_golden(orc):
    xi, w = orc.lattice()
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "d3q27_weights.txt")) if l[0] != "#"]
    for sq, cnt, num, den in rows:
        sel = (xi ** 2).sum(1) == int(sq)
        assert sel.sum() == int(cnt)
        assert np.allclose(w[sel], int(num) / int(den), rtol=0, atol=1e-16)
    # direction convention i = 9(xi_z+1) + 3(xi_y+1) + (xi_x+1); opposite = 26 - i
    for i in range(27):
        assert i == 9 * (xi[i, 2] + 1) + 3 * (xi[i, 1] + 1) + (xi[i, 0] + 1)
        assert (xi[26 - i] == -xi[i]).all()


def test_lattice_isotropy(orc):
    xi, w = orc.lattice()
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(w @ xi, 0, atol=1e-16)
    assert np.allclose((w[:, None, None] * xi[:, :, None] * xi[:, None, :]).sum(0), CS2 * np.eye(3), atol=1e-16)
    # fourth-order isotropy of the Gaussian: E[x^2 y^2] = cs^4
    assert abs((w * xi[:, 0] ** 2 * xi[:, 1] ** 2).sum() - CS2 ** 2) < 1e-16


def test_hermite_tensor_equals_product_and_is_orthogonal(orc):
    """The oracle's tensor Hermite polynomials (three-term recurrence) equal
    the products of 1-D Hermite polynomials for index strings with each
    index at most twice, and are orthogonal under the weights with norm
    prod m_d! cs^(2 m_d)."""
    xi, w = orc.lattice()
    tuples = [()] + [(a,) for a in range(3)] + [(a, b) for a in range(3) for b in range(3)] + PRINTED
    for idx in tuples:
        m = counts(idx)
        for i in range(27):
            ref = np.prod([h1d(m[d], xi[i, d]) for d in range(3)])
            assert abs(orc.hermite(i, idx) - ref) < 1e-14, (idx, i)
    for m in multi_indices():
        for mp in multi_indices():
            s = sum(w[i] * np.prod([h1d(m[d], xi[i, d]) * h1d(mp[d], xi[i, d]) for d in range(3)])
                    for i in range(27))
            norm = np.prod([math.factorial(m[d]) * CS2 ** m[d] for d in range(3)]) if m == mp else 0.0
            assert abs(s - norm) < 1e-15


def maxwell_moment(rho, u, a):
    """Raw moment E[prod xi_d^a_d] of rho times a Gaussian with mean u and
    variance cs^2, for a_d <= 2."""
    out = rho
    for d in range(3):
        out *= (1.0, u[d], CS2 + u[d] ** 2)[a[d]]
    return out


@pytest.mark.parametrize("seed", range(6))
def test_equilibrium_has_maxwellian_moments(orc, seed):
    """All 27 raw moments of f^(0) (App. A) equal those of the Maxwellian
    rho N(u, cs^2): 27 independent conditions, so they fix f^(0) fully."""
    rng = np.random.default_rng(seed)
    rho = 1 + 0.1 * rng.standard_normal()
    u = 0.15 * rng.standard_normal(3)
    f0 = orc.feq(CS2 * (rho - 1.0), u)
    xi, _ = orc.lattice()
    for a in multi_indices():
        mom = (f0 * np.prod(xi ** np.array(a), axis=1)).sum()
        assert abs(mom - maxwell_moment(rho, u, a)) < 1e-14, a


def closed_form_a1(P1, u, idx):
    """a_1^(n) unrolled: sum over index pairs (j<k) of P1_{a_j a_k} prod_{l != j,k} u_{a_l}."""
    n = len(idx)
    s = 0.0
    for j in range(n):
        for k in range(j + 1, n):
            prod = P1[idx[j], idx[k]]
            for l in range(n):
                if l not in (j, k):
                    prod *= u[idx[l]]
            s += prod
    return s


def random_p1(rng):
    A = rng.standard_normal((3, 3)) * 1e-3
    return A + A.T


@pytest.mark.parametrize("seed", range(4))
def test_a1_recursion_symmetric_and_unrolled(orc, seed):
    """The recursion of App. A is written with a distinguished last index; the
    tensor it defines must be fully symmetric and equal the pair sum it
    unrolls to."""
    rng = np.random.default_rng(seed)
    P1, u = random_p1(rng), 0.1 * rng.standard_normal(3)
    for n in range(2, 7):
        for idx in itertools.product(range(3), repeat=n):
            if max(counts(idx)) > 2:
                continue
            v = orc.a1(P1, u, idx)
            assert abs(v - closed_form_a1(P1, u, idx)) < 1e-17
            for perm in set(itertools.permutations(idx)):
                assert abs(orc.a1(P1, u, perm) - v) < 1e-17


@pytest.mark.parametrize("seed", range(6))
def test_offequilibrium_moments_and_projections(orc, seed):
    """f^(1) carries no mass or momentum, its second moment is P^(1), and its
    Hermite projection onto every D3Q27-supported polynomial of order >= 2
    recovers the corresponding a_1 coefficient (orthogonality)."""
    rng = np.random.default_rng(100 + seed)
    P1, u = random_p1(rng), 0.1 * rng.standard_normal(3)
    f1 = orc.fneq(P1, u)
    xi, _ = orc.lattice()
    assert abs(f1.sum()) < 1e-18
    assert np.allclose(f1 @ xi, 0, atol=1e-18)
    second = (f1[:, None, None] * xi[:, :, None] * xi[:, None, :]).sum(0)
    assert np.allclose(second, P1, atol=1e-17, rtol=0)
    for m in multi_indices():
        if sum(m) < 2:
            continue
        idx = tuple(d for d in range(3) for _ in range(m[d]))
        proj = sum(f1[i] * np.prod([h1d(m[d], xi[i, d]) for d in range(3)]) for i in range(27))
        assert abs(proj - closed_form_a1(P1, u, idx)) < 1e-17, m


@pytest.mark.parametrize("seed", range(3))
def test_bruteforce_full_tensor_hermite_sums(orc, seed):
    """Direct evaluation of f^(0) and f^(1) as full tensor contractions
    w_i sum_n 1/(n! cs^2n) H^(n)_i : a^(n) over every index string the
    lattice supports (each index at most twice), with no multi-index
    bookkeeping, matches the oracle's term-by-term sums."""
    rng = np.random.default_rng(200 + seed)
    rho = 1 + 0.05 * rng.standard_normal()
    u = 0.1 * rng.standard_normal(3)
    P1 = random_p1(rng)
    xi, w = orc.lattice()
    f0 = np.zeros(27)
    f1 = np.zeros(27)
    for n in range(0, 7):
        for idx in itertools.product(range(3), repeat=n):
            m = counts(idx)
            if max(m, default=0) > 2:
                continue
            Hn = np.array([np.prod([h1d(m[d], xi[i, d]) for d in range(3)]) for i in range(27)])
            a0 = rho * np.prod([u[a] for a in idx])
            f0 += w * Hn * a0 / (math.factorial(n) * CS2 ** n)
            if n >= 2:
                f1 += w * Hn * closed_form_a1(P1, u, idx) / (math.factorial(n) * CS2 ** n)
    assert np.allclose(orc.feq(CS2 * (rho - 1), u), f0, rtol=0, atol=1e-14)
    assert np.allclose(orc.fneq(P1, u), f1, rtol=0, atol=1e-16)


def random_cell(orc, rng, amp=0.05):
    _, w = orc.lattice()
    return w * (1 + amp * rng.standard_normal(27))


def test_rest_state_is_fixed_point(orc):
    _, w = orc.lattice()
    for tau in (0.51, 0.6, 1.0, 1.7):
        assert np.allclose(orc.collide_cell(w, None, tau), w, rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", range(8))
def test_collision_conservation_and_stress_relaxation(orc, seed):
    """Mass is conserved; momentum changes by tau rho h (the forced rule of
    Sec. 2.2 read literally: f^(0) at u + tau h, f^(1) without momentum);
    the second moment relaxes to rho(cs^2 I + u~u~) + (1 - 1/tau) P^(1)."""
    rng = np.random.default_rng(300 + seed)
    xi, w = orc.lattice()
    f = random_cell(orc, rng)
    tau = rng.uniform(0.51, 2.0)
    h = 1e-3 * rng.standard_normal(3) if seed % 2 else np.zeros(3)
    out = orc.collide_cell(f, h, tau)
    rho = f.sum()
    u = (f @ xi) / rho
    assert abs(out.sum() - rho) < 1e-15
    assert np.allclose(out @ xi, rho * (u + tau * h), atol=1e-16, rtol=0)
    f0 = orc.feq(CS2 * (rho - 1), u)
    P1 = ((f - f0)[:, None, None] * xi[:, :, None] * xi[:, None, :]).sum(0)
    ut = u + tau * h
    second = (out[:, None, None] * xi[:, :, None] * xi[:, None, :]).sum(0)
    expect = rho * (CS2 * np.eye(3) + np.outer(ut, ut)) + (1 - 1 / tau) * P1
    assert np.allclose(second, expect, atol=1e-15, rtol=0)


@pytest.mark.parametrize("seed", range(6))
def test_momentum_exact_variant_adds_rho_h(orc, seed):
    """Momentum-exact variant of the forced rule: the momentum added per step
    is exactly rho h (not tau rho h); mass and the second moment are those of
    the rule as printed; at tau = 1 the two coincide."""
    rng = np.random.default_rng(900 + seed)
    xi, w = orc.lattice()
    f = random_cell(orc, rng)
    tau = rng.uniform(0.51, 2.0)
    h = 1e-3 * rng.standard_normal(3)
    lit = orc.collide_cell(f, h, tau)
    ex = orc.collide_cell(f, h, tau, forcing=1)
    rho = f.sum()
    u = (f @ xi) / rho
    assert abs(ex.sum() - rho) < 1e-15
    assert np.allclose(ex @ xi, rho * (u + h), atol=1e-16, rtol=0)
    sec = lambda g: (g[:, None, None] * xi[:, :, None] * xi[:, None, :]).sum(0)
    assert np.allclose(sec(ex), sec(lit), atol=1e-15, rtol=0)
    assert np.allclose(orc.collide_cell(f, h, 1.0, forcing=1), orc.collide_cell(f, h, 1.0), atol=1e-17, rtol=0)
    assert np.array_equal(orc.collide_cell(f, None, tau, forcing=1), orc.collide_cell(f, None, tau))


@pytest.mark.parametrize("seed", range(4))
def test_bgk_comparison_collision(orc, seed):
    """BGK (collision 1, for comparison): every moment of the off-equilibrium
    part relaxes by the same factor 1 - 1/tau (third- and fourth-order ones
    too, which the regularized rule filters); mass and momentum as in the
    regularized rule; on a state whose off-equilibrium is the regularized
    second-order one the two collisions agree."""
    rng = np.random.default_rng(700 + seed)
    xi, w = orc.lattice()
    f = random_cell(orc, rng)
    tau = rng.uniform(0.51, 1.8)
    h = 1e-3 * rng.standard_normal(3)
    rho = f.sum()
    u = (f @ xi) / rho
    bgk = orc.collide_cell(f, h, tau, collision=1)
    rr = orc.collide_cell(f, h, tau)
    assert abs(bgk.sum() - rho) < 1e-15
    assert np.allclose(bgk @ xi, rho * (u + tau * h), atol=1e-16, rtol=0)
    neq_in = f - orc.feq(CS2 * (rho - 1), u)
    neq_bgk = bgk - orc.feq(CS2 * (rho - 1), u + tau * h)
    neq_rr = rr - orc.feq(CS2 * (rho - 1), u + tau * h)
    for mono in [(1, 1, 1), (2, 1, 0), (2, 2, 0), (2, 1, 1), (2, 2, 2)]:
        psi = xi[:, 0] ** mono[0] * xi[:, 1] ** mono[1] * xi[:, 2] ** mono[2]
        assert abs(psi @ neq_bgk - (1 - 1 / tau) * (psi @ neq_in)) < 1e-15
    # the random state has higher-order off-equilibrium content that RR drops
    psi = xi[:, 0] * xi[:, 1] * xi[:, 2]
    assert abs(psi @ neq_rr - (1 - 1 / tau) * (psi @ neq_in)) > 1e-6
    # pure regularized off-equilibrium: both rules coincide
    P1 = (neq_in[:, None, None] * xi[:, :, None] * xi[:, None, :]).sum(0)
    g = orc.feq(CS2 * (rho - 1), u) + orc.fneq(P1, u)
    assert np.allclose(orc.collide_cell(g, h, tau, collision=1), orc.collide_cell(g, h, tau), atol=1e-15, rtol=0)


def test_tau_one_is_equilibrium(orc):
    rng = np.random.default_rng(7)
    xi, _ = orc.lattice()
    f = random_cell(orc, rng)
    h = 1e-3 * rng.standard_normal(3)
    rho = f.sum()
    u = (f @ xi) / rho
    assert np.allclose(orc.collide_cell(f, h, 1.0), orc.feq(CS2 * (rho - 1), u + h), atol=1e-16, rtol=0)


def test_stress_definition_parts(orc):
    """sigma = -p I + (1/(2 tau) - 1) P^(1): at equilibrium only -p I is left,
    and its deviatoric part scales with 1/(2 tau) - 1."""
    rng = np.random.default_rng(11)
    xi, w = orc.lattice()
    rho = 1.02
    u = np.array([0.01, -0.02, 0.015])
    f0 = orc.feq(CS2 * (rho - 1), u)
    sig, r, uu = orc.stress_cell(f0, 0.8)
    assert np.allclose(sig, -CS2 * (rho - 1) * np.eye(3), atol=1e-16)
    assert abs(r - rho) < 1e-15 and np.allclose(uu, u, atol=1e-16)
    f = random_cell(orc, rng)
    s1, _, _ = orc.stress_cell(f, 0.6)
    s2, _, _ = orc.stress_cell(f, 1.5)
    p = CS2 * (f.sum() - 1)
    d1, d2 = s1 + p * np.eye(3), s2 + p * np.eye(3)
    assert np.allclose(d1 * (1 / 3.0 - 1), d2 * (1 / 1.2 - 1), atol=1e-16)
    assert np.allclose(s1, s1.T, atol=1e-18)
