"""Cube-symmetry equivariance of the oracle's time step (the lattice and the
collision of Sec. 2.1 / App. A have the symmetry of the cube): for every one
of the 48 rotations and reflections sigma of the cube, acting on space and on
the velocity directions together, collide(sigma f) = sigma collide(f) for a
single cell (forced rule included, with the force rotated too), and a whole
periodic step commutes with sigma on a cubic box.  A coefficient attached to
the wrong index, or an asymmetric term, breaks it."""
import itertools

import numpy as np
import pytest

from paper_2408_15115_amd import workloads as W


def symmetries():
    """The 48 signed permutation matrices."""
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            M = np.zeros((3, 3), int)
            for a in range(3):
                M[a, perm[a]] = signs[a]
            out.append(M)
    return out


def direction_map(xi, M):
    """Index j of the direction M xi_i, for each i."""
    lookup = {tuple(v): j for j, v in enumerate(xi)}
    return np.array([lookup[tuple(M @ v)] for v in xi])


def test_there_are_48_distinct_symmetries():
    S = symmetries()
    assert len({tuple(M.ravel()) for M in S}) == 48


def test_single_cell_collision_is_equivariant(orc):
    xi, w = orc.lattice()
    rng = np.random.default_rng(5)
    f = w * (1.0 + 0.1 * rng.standard_normal(27))
    h = rng.standard_normal(3) * 1e-3
    for forcing in (0, 1):
        C = orc.collide_cell(f, h, 0.73, forcing=forcing)
        for M in symmetries():
            j = direction_map(xi, M)
            fs = np.empty(27)
            fs[j] = f                      # (sigma f)_{M xi_i} = f_i
            Cs = orc.collide_cell(fs, M @ h, 0.73, forcing=forcing)
            assert np.allclose(Cs[j], C, rtol=0, atol=1e-15)


def test_periodic_grid_step_commutes_with_the_cube_group(orc):
    xi, _ = orc.lattice()
    n, tau = 6, 0.8
    f = W.random_populations(9, n, n, n, amp=0.05)      # (z, y, x, 27)
    out = orc.stream_grid(orc.collide_grid(f, tau))
    grid = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1)   # (z, y, x) indices
    for M in symmetries()[::5]:
        j = direction_map(xi, M)
        # sigma acts on positions r = (x, y, z) by r -> M r (mod n)
        r = grid[..., ::-1]                            # (x, y, z) at each (z, y, x)
        rs = (r @ M.T) % n
        fs = np.empty_like(f)
        tmp = np.empty_like(f)
        tmp[rs[..., 2], rs[..., 1], rs[..., 0]] = f
        fs[..., j] = tmp
        outs = orc.stream_grid(orc.collide_grid(fs, tau))
        ref = np.empty_like(out)
        ref_tmp = np.empty_like(out)
        ref_tmp[rs[..., 2], rs[..., 1], rs[..., 0]] = out
        ref[..., j] = ref_tmp
        assert np.allclose(outs, ref, rtol=0, atol=1e-15)
