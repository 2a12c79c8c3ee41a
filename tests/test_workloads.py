"""The seeded input generators: meshes, marker areas and normals, mass
properties and lattice scaling against analytic values."""
import math

import numpy as np
import pytest

from paper_2408_15115_amd import workloads as W


@pytest.mark.parametrize("freq", [1, 4, 16, 35])
def test_geodesic_counts_and_closure(freq):
    V, F = W.geodesic_sphere(freq)
    assert len(V) == 10 * freq * freq + 2 and len(F) == 20 * freq * freq
    assert np.allclose(np.linalg.norm(V, axis=1), 1.0)
    # closed 2-manifold: every edge shared by exactly two triangles, Euler characteristic 2
    edges = np.sort(np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]]), axis=1)
    _, cnt = np.unique(edges, axis=0, return_counts=True)
    assert (cnt == 2).all()
    assert len(V) - len(cnt) + len(F) == 2


def test_marker_areas_sum_to_mesh_area_and_normals_point_out():
    V, F = W.ellipsoid_mesh(32, 32, 16, 12)
    dS, n = W.vertex_areas_normals(V, F)
    tri = 0.5 * np.linalg.norm(np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]]), axis=1)
    assert abs(dS.sum() - tri.sum()) < 1e-9 * tri.sum()
    assert (np.einsum("ij,ij->i", n, V) > 0).all()
    # closed surface: sum dS n ~ 0
    assert np.linalg.norm((dS[:, None] * n).sum(0)) < 1e-3 * dS.sum()


def test_mesh_mass_properties_converge_to_ellipsoid():
    a, b, c = 32.0, 24.0, 16.0
    V, F = W.ellipsoid_mesh(a, b, c, 35)
    vol, cen, J = W.mesh_mass_properties(V, F)
    assert abs(vol / (4 / 3 * math.pi * a * b * c) - 1) < 2e-3
    assert np.allclose(cen, 0, atol=1e-9)
    ref = np.diag([(b * b + c * c) / 5, (a * a + c * c) / 5, (a * a + b * b) / 5])
    assert np.allclose(J, ref, rtol=4e-3, atol=1e-9)


def test_mass_properties_exact_for_a_cube():
    # unit cube [0,1]^3 as 12 outward triangles
    V = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)], float)
    F = np.array([[0, 2, 1], [1, 2, 3], [4, 5, 6], [5, 7, 6], [0, 1, 4], [1, 5, 4],
                  [2, 6, 3], [3, 6, 7], [0, 4, 2], [2, 4, 6], [1, 3, 5], [3, 7, 5]])
    vol, cen, J = W.mesh_mass_properties(V, F)
    assert abs(vol - 1) < 1e-14 and np.allclose(cen, 0.5)
    assert np.allclose(J, np.eye(3) / 6)


def test_sphere_case_matches_its_description():
    case, body = W.case_sphere48()
    assert (case["nx"], case["ny"], case["nz"], case["tau"]) == (48, 48, 48, 0.6)
    assert body["x_body"].shape == (400, 3)
    assert abs(body["dS"].sum() - 4 * math.pi * 16) < 1e-9
    assert np.allclose(np.linalg.norm(body["x_body"], axis=1), 4.0)
    assert np.allclose(body["r0"], 23.5)


def test_tall_ellipsoid_case_scaling():
    case, body = W.case_ellipsoid_tall()
    assert body["x_body"].shape == (12252, 3)
    assert abs(case["d_eq"] - 50.80) < 0.01
    assert abs(case["tau"] - (3 * 0.02 * case["d_eq"] / 100 + 0.5)) < 1e-12
    assert abs(case["gravity"] / 2.392e-6 - 1) < 2e-3
    # tilted: the body z axis leans 5..30 degrees from vertical
    tilt = math.degrees(math.acos(body["d0"][2, 2]))
    assert 5 <= tilt <= 30
    assert case["h_ini"] - case["h_end"] == 64


def test_batch_is_seeded_and_in_range():
    a = W.batch_cases(6)
    b = W.batch_cases(6)
    for (ca, ba), (cb, bb) in zip(a, b):
        assert ca == cb and np.array_equal(ba["x_body"], bb["x_body"])
        assert 64 <= ca["nx"] <= 192 and ca["nz"] <= 384
        assert 0.5 < ca["tau"] <= 1.0 + 1e-12
        assert ca["sponge"] == round(0.08 * ca["nz"])
