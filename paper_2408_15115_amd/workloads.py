"""Seeded synthetic inputs: cases, particle surface meshes and markers.

Both the library and the FP64 CPU oracle consume these inputs; this module
imports nothing else of the package and holds none of the time-step
arithmetic.  It builds only what a user of the solver would prepare before
the first step:

* the domain descriptor (box size, relaxation time, walls, sponge, window);
* the particle's surface markers: positions and outward normals in the body
  frame and the area ``dS_k`` of each marker.  For a triangulated surface the
  markers are the mesh vertices and ``dS_k`` is one third of the area of the
  triangles sharing the vertex (Sec. 2.2); a Fibonacci point set on a sphere
  gets the uniform share 4 pi R^2 / M;
* the body's volume and inertia-per-mass tensor J/m about its centre of mass
  (Sec. 2.3), analytic for spheres and ellipsoids and from signed tetrahedra
  for meshes;
* the lattice scaling of Sec. 3: the terminal velocity is 0.02 in lattice
  units, nu = v_T d / Re, tau = 3 nu + 1/2 (Sec. 2.1 viscosity relation), and
  gravity follows from the Clift-Gauvin drag law (Sec. 3.2) so that the
  weight balances the drag at v_T.

Lattice units: dx = dt = rho_f = 1; z is vertical and gravity points along -z.
"""
from __future__ import annotations

import math

import numpy as np

BC_PERIODIC, BC_FREESLIP, BC_NOSLIP, BC_PRESSURE = 0, 1, 2, 3
V_TERMINAL_LU = 0.02
# Where the force and torque of Sec. 2.2 are evaluated: the stress integral on
# the parallel surface this many cells outside the markers (with that
# surface's own areas).  0 evaluates it at the markers, as printed; there the
# 4-point stencil straddles the surface and averages the outer stress with
# that of the rigidly moving inner fluid, and a sphere in Stokes flow reads a
# third to a half of its drag.  Three cells out the stencil sees only fluid.
FORCE_OFFSET = 3.0

# D3Q27 weights w_i = prod_d w1(xi_d), w1(0) = 2/3, w1(+-1) = 1/6; direction
# i = 9*(xi_z+1) + 3*(xi_y+1) + (xi_x+1).  Only used to draw random
# near-rest population fields.
_W1 = {-1: 1.0 / 6.0, 0: 2.0 / 3.0, 1: 1.0 / 6.0}
D3Q27_W = np.array([_W1[i % 3 - 1] * _W1[(i // 3) % 3 - 1] * _W1[i // 9 - 1] for i in range(27)])
# D3Q19 (the comparison lattice): the D3Q27 directions without the eight
# corners, same order; weights 1/3, 1/18, 1/36.
D3Q19_XI = np.array([[i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1] for i in range(27)
                     if abs(i % 3 - 1) + abs((i // 3) % 3 - 1) + abs(i // 9 - 1) < 3], np.float64)
D3Q19_W = np.array([{0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0}[int(np.abs(v).sum())] for v in D3Q19_XI])


# ---------------------------------------------------------------- meshes
def icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    return v, f


def geodesic_sphere(freq: int):
    """Class-I geodesic sphere of frequency ``freq``: 10 freq^2 + 2 unit-radius
    vertices, 20 freq^2 outward-oriented triangles."""
    V0, F0 = icosahedron()
    key = {}
    verts = []
    n = freq

    def vid(a, b, c, i, j):
        # integer barycentric key: shared edge/corner points get one id
        k = tuple(sorted((int(v), int(wt)) for v, wt in ((a, n - i - j), (b, i), (c, j)) if wt))
        if k not in key:
            p = (V0[a] * (n - i - j) + V0[b] * i + V0[c] * j) / n
            key[k] = len(verts)
            verts.append(p / np.linalg.norm(p))
        return key[k]

    tris = []
    for a, b, c in F0:
        grid = {}
        for i in range(n + 1):
            for j in range(n + 1 - i):
                grid[(i, j)] = vid(a, b, c, i, j)
        for i in range(n):
            for j in range(n - i):
                tris.append((grid[(i, j)], grid[(i + 1, j)], grid[(i, j + 1)]))
                if i + j < n - 1:
                    tris.append((grid[(i + 1, j)], grid[(i + 1, j + 1)], grid[(i, j + 1)]))
    V = np.array(verts)
    F = np.array(tris, dtype=np.int64)
    # orient every triangle outward
    cen = V[F].mean(axis=1)
    nrm = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    flip = np.einsum("ij,ij->i", nrm, cen) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def vertex_areas_normals(V, F):
    """Per-vertex area (one third of the incident triangle areas, Sec. 2.2) and
    unit normal (area-weighted incident face normals, outward)."""
    e1 = V[F[:, 1]] - V[F[:, 0]]
    e2 = V[F[:, 2]] - V[F[:, 0]]
    cr = np.cross(e1, e2)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    dS = np.zeros(len(V))
    nrm = np.zeros_like(V)
    for k in range(3):
        np.add.at(dS, F[:, k], area / 3.0)
        np.add.at(nrm, F[:, k], 0.5 * cr)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return dS, nrm


def mesh_mass_properties(V, F):
    """Volume, centroid and inertia-per-mass J/m = (1/V) int (|x|^2 I - x x) dV
    about the centroid, for a closed outward-oriented triangle mesh (signed
    tetrahedra from the origin, exact for polyhedra)."""
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    vol6 = np.einsum("ij,ij->i", a, np.cross(b, c))
    vol = vol6.sum() / 6.0
    cen = ((a + b + c) * vol6[:, None]).sum(0) / (24.0 * vol)
    # second moments int x_i x_j dV over each tetrahedron (0, a, b, c)
    S = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            s = (2 * (a[:, i] * a[:, j] + b[:, i] * b[:, j] + c[:, i] * c[:, j])
                 + a[:, i] * b[:, j] + a[:, j] * b[:, i] + a[:, i] * c[:, j] + a[:, j] * c[:, i]
                 + b[:, i] * c[:, j] + b[:, j] * c[:, i])
            S[i, j] = (s * vol6).sum() / 120.0
    S = S / vol - np.outer(cen, cen)          # central second moments per volume
    J = np.trace(S) * np.eye(3) - S
    return vol, cen, J


def fibonacci_sphere(n: int, R: float):
    """Fibonacci point set: z_k = 1 - (2k+1)/n, azimuth k pi (3 - sqrt 5)."""
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    rho = np.sqrt(1.0 - z * z)
    ph = k * math.pi * (3.0 - math.sqrt(5.0))
    nrm = np.stack([rho * np.cos(ph), rho * np.sin(ph), z], axis=1)
    return R * nrm, nrm, np.full(n, 4.0 * math.pi * R * R / n)


def real_sph_harm(l, m, theta, phi):
    from scipy.special import sph_harm_y
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    y = sph_harm_y(l, abs(m), theta, phi)
    return math.sqrt(2.0) * (np.real(y) if m > 0 else np.imag(y)) * (-1) ** m


# ---------------------------------------------------------------- bodies
def _body(kappa, volume, Jm, xb, nb, dS, r0, d0=None, v0=None, w0=None):
    return {"kappa": float(kappa), "volume": float(volume), "J_over_m": np.asarray(Jm, np.float64),
            "x_body": np.ascontiguousarray(xb, np.float64), "n_body": np.ascontiguousarray(nb, np.float64),
            "dS": np.ascontiguousarray(dS, np.float64), "r0": np.asarray(r0, np.float64),
            "d0": np.eye(3) if d0 is None else np.asarray(d0, np.float64),
            "v0": np.zeros(3) if v0 is None else np.asarray(v0, np.float64),
            "w0": np.zeros(3) if w0 is None else np.asarray(w0, np.float64)}


def _with_force_surface(body, delta, dS_offset):
    """Attach the parallel surface at distance delta outside the markers on
    which the force may be evaluated: its marker areas (input geometry)."""
    if delta > 0.0:
        body["force_offset"] = float(delta)
        body["dS_offset"] = np.ascontiguousarray(dS_offset, np.float64)
    return body


def sphere_fibonacci_body(R, n, kappa, r0, force_offset=FORCE_OFFSET, **kw):
    xb, nb, dS = fibonacci_sphere(n, R)
    b = _body(kappa, 4.0 / 3.0 * math.pi * R ** 3, 0.4 * R * R * np.eye(3), xb, nb, dS, r0, **kw)
    return _with_force_surface(b, force_offset, dS * ((R + force_offset) / R) ** 2)


def mesh_body(V, F, kappa, r0, force_offset=FORCE_OFFSET, **kw):
    """Markers at the vertices of a closed triangle mesh.  With force_offset
    > 0 (the default) the mesh is also offset along the vertex normals by
    that distance and the vertex areas of the offset mesh are attached."""
    vol, cen, Jm = mesh_mass_properties(V, F)
    Vc = V - cen
    dS, nb = vertex_areas_normals(Vc, F)
    b = _body(kappa, vol, Jm, Vc, nb, dS, r0, **kw)
    if force_offset > 0.0:
        dSo, _ = vertex_areas_normals(Vc + force_offset * nb, F)
        _with_force_surface(b, force_offset, dSo)
    return b


def ellipsoid_mesh(a, b, c, freq):
    V, F = geodesic_sphere(freq)
    return V * np.array([a, b, c]), F


def perturbed_sphere_mesh(rng, freq=16, lmax=6, amp=0.15):
    """Unit geodesic sphere with radius 1 + s sum_{l=1..lmax} sum_m c_lm Y_lm,
    c_lm ~ N(0,1), s set so the largest |perturbation| is ``amp``."""
    V, F = geodesic_sphere(freq)
    theta = np.arccos(np.clip(V[:, 2], -1, 1))
    phi = np.arctan2(V[:, 1], V[:, 0])
    pert = np.zeros(len(V))
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            pert += rng.standard_normal() * real_sph_harm(l, m, theta, phi)
    pert *= amp / np.abs(pert).max()
    return V * (1.0 + pert)[:, None], F


def rotation_matrix(axis, angle):
    axis = np.asarray(axis, np.float64)
    axis = axis / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * K @ K


# ---------------------------------------------------------------- physics scaling
def clift_gauvin_cd(re):
    """Clift-Gauvin drag coefficient (Sec. 3.2)."""
    return 24.0 / re * (1.0 + 0.15 * re ** 0.687) + 0.42 / (1.0 + 4.25e4 * re ** -1.16)


# viscosity at tau = 1: nu = (tau - 1/2) / 3
TAU_MAX_BATCH_NU = (1.0 - 0.5) / 3.0


def lattice_scaling(d_eq, re, kappa, v_t=V_TERMINAL_LU):
    """nu, tau and gravity for a body of volume-equivalent diameter d_eq that
    should settle at v_t with Reynolds number re (weight without buoyancy,
    as in the translational update of Sec. 2.3)."""
    nu = v_t * d_eq / re
    tau = 3.0 * nu + 0.5
    g = 3.0 * clift_gauvin_cd(re) * v_t ** 2 / (4.0 * kappa * d_eq)
    return nu, tau, g


# ---------------------------------------------------------------- cases
def make_case(nx, ny, nz, tau, bc_zlo=BC_FREESLIP, bc_zhi=BC_FREESLIP, sponge=0, gravity=0.0,
              h_ini=0.0, h_end=0.0, ibm_cycles=4, u_wall=(0.0, 0.0)):
    return {"nx": int(nx), "ny": int(ny), "nz": int(nz), "tau": float(tau), "bc_zlo": int(bc_zlo),
            "bc_zhi": int(bc_zhi), "sponge": int(sponge), "gravity": float(gravity),
            "h_ini": float(h_ini), "h_end": float(h_end), "ibm_cycles": int(ibm_cycles),
            "u_wall_lo": float(u_wall[0]), "u_wall_hi": float(u_wall[1])}


def case_sphere48(n=48, markers=400, R=4.0, tau=0.6, kappa=2.0, gravity=1e-5):
    """Plain-method case: D3Q27 RR on 48^3, tau 0.6, periodic x/y, free-slip
    top/bottom, one sphere (D = 8) of 400 Fibonacci markers, density ratio 2,
    gravity 1e-5, at rest at the box centre."""
    c = (n - 1) / 2.0
    case = make_case(n, n, n, tau, BC_FREESLIP, BC_FREESLIP, 0, gravity)
    body = sphere_fibonacci_body(R, markers, kappa, [c, c, c])
    return case, body


def case_ellipsoid_tall(seed=2408, nx=256, ny=256, nz=768, semi=(32.0, 32.0, 16.0), freq=35,
                        kappa=2.7, re=100.0, sponge_frac=0.08, drop=64):
    """Scale case: 256x256x768 falling-frame box, oblate ellipsoid 32/32/16
    meshed by a frequency-35 geodesic sphere (12,252 markers), density ratio
    2.7, Re 100, random initial tilt (5..30 degrees about a horizontal axis)."""
    rng = np.random.default_rng(seed)
    V, F = ellipsoid_mesh(*semi, freq)
    d_eq = 2.0 * (semi[0] * semi[1] * semi[2]) ** (1.0 / 3.0)
    nu, tau, g = lattice_scaling(d_eq, re, kappa)
    az = rng.uniform(0.0, 2.0 * math.pi)
    ang = math.radians(rng.uniform(5.0, 30.0))
    Rm = rotation_matrix([math.cos(az), math.sin(az), 0.0], ang)
    z0 = 0.75 * nz
    r0 = [(nx - 1) / 2.0, (ny - 1) / 2.0, z0]
    body = mesh_body(V, F, kappa, r0, d0=Rm.T)
    case = make_case(nx, ny, nz, tau, BC_FREESLIP, BC_FREESLIP, int(round(sponge_frac * nz)), g,
                     h_ini=z0, h_end=z0 - drop)
    case["nu"], case["re"], case["d_eq"] = nu, re, d_eq
    return case, body


def _freq_for_area(area, target_dS=0.5):
    return max(4, int(round(math.sqrt(area / target_dS / 10.0))))


def case_sphere_settling(D=16.0, re=5.0, kappa=2.7, force_offset=FORCE_OFFSET, w_d=10, h_d=30, domain="free-slip",
                         v_t=None, h_ini_d=None, h_end_d=None, sponge_d=None):
    """A sphere of diameter D (lattice units) settling from rest in a
    w = w_d D by w_d D by h = h_d D box (the paper's w* = 10, h* = 30 domain of
    its low-Re sphere cases): periodic x/y, free-slip top and bottom (or, with
    domain="paper", the Sec. 3 layout: no-slip bottom, constant-pressure top),
    sponge 0.08 h, window re-injection from 0.75 h by 4 D (or from h_ini_d D
    down to h_end_d D, sponge sponge_d D, as in Table 2).  Gravity from the
    Clift-Gauvin drag so that the unbounded terminal velocity is v_T (0.02,
    lowered to keep tau <= 1, unless given).  Markers at the vertices of a
    geodesic mesh with mean area about 0.5.  Returns (case, body, v_T)."""
    R = D / 2.0
    w, h = int(round(w_d * D)), int(round(h_d * D))
    V, F = geodesic_sphere(_freq_for_area(4 * math.pi * R * R))
    if v_t is None:
        v_t = min(V_TERMINAL_LU, re * TAU_MAX_BATCH_NU / D)
    nu, tau, g = lattice_scaling(D, re, kappa, v_t)
    z0 = 0.75 * h if h_ini_d is None else h_ini_d * D
    z1 = z0 - 4 * D if h_end_d is None else h_end_d * D
    sponge = int(round(0.08 * h)) if sponge_d is None else int(round(sponge_d * D))
    body = mesh_body(V * R, F, kappa, [(w - 1) / 2.0, (w - 1) / 2.0, z0], force_offset=force_offset)
    lo, hi = (BC_NOSLIP, BC_PRESSURE) if domain == "paper" else (BC_FREESLIP, BC_FREESLIP)
    case = make_case(w, w, h, tau, lo, hi, sponge, g, h_ini=z0, h_end=z1)
    case["re"], case["d_eq"], case["v_terminal"] = re, D, v_t
    return case, body, v_t


def batch_cases(n_cases=64, seed0=2408, max_h=384):
    """Batched form: independent settling cases of uneven boxes (64^3 up to
    192x192x384): spheres, spheroids and perturbed geodesic spheres, density
    ratios log-uniform in 1.5..1000, Re log-uniform in 0.5..300.  The lattice
    terminal velocity is 0.02, lowered where that would put tau above 1 (the
    relaxation time the sponge reaches at the top), so that tau <= 1."""
    out = []
    for i in range(n_cases):
        rng = np.random.default_rng(seed0 + i)
        w = 32 * int(rng.integers(2, 7))
        h = min(max_h, 32 * int(round(w * float(rng.choice([1.0, 1.5, 2.0])) / 32.0)))
        shape = i % 3
        D = rng.uniform(8.0, 24.0)
        kappa = math.exp(rng.uniform(math.log(1.5), math.log(1000.0)))
        re = math.exp(rng.uniform(math.log(0.5), math.log(300.0)))
        z0 = 0.75 * h
        r0 = [(w - 1) / 2.0, (w - 1) / 2.0, z0]
        if shape == 0:
            R = D / 2.0
            V, F = geodesic_sphere(_freq_for_area(4 * math.pi * R * R))
            body = mesh_body(V * R, F, kappa, r0)
        elif shape == 1:
            aspect = math.exp(rng.uniform(math.log(0.3), math.log(3.0)))
            a = D / 2.0 / aspect ** (1.0 / 3.0)
            c = a * aspect
            area = 4 * math.pi * max(a, c) ** 2
            V, F = ellipsoid_mesh(a, a, c, min(_freq_for_area(area), 24))
            q = rng.standard_normal(4)
            q /= np.linalg.norm(q)
            Rm = rotation_matrix(q[1:], 2 * math.acos(min(1.0, abs(q[0]))))
            body = mesh_body(V, F, kappa, r0, d0=Rm.T)
        else:
            V, F = perturbed_sphere_mesh(rng)
            vol, _, _ = mesh_mass_properties(V, F)
            scale = D / 2.0 / (3.0 * vol / (4.0 * math.pi)) ** (1.0 / 3.0)
            body = mesh_body(V * scale, F, kappa, r0)
        # keep the stencils of the force surface two cells inside the walls:
        # start at most 0.75 h high and re-inject 32 rows lower, or above
        # R_b + force offset + 4
        rb = float(np.linalg.norm(body["x_body"], axis=1).max()) + body.get("force_offset", 0.0)
        z_start = min(z0, h - rb - 4.0)
        z_end = max(z_start - 32.0, rb + 4.0)
        body["r0"] = np.array([body["r0"][0], body["r0"][1], z_start])
        v_t = min(V_TERMINAL_LU, re * TAU_MAX_BATCH_NU / D)
        nu, tau, g = lattice_scaling(D, re, kappa, v_t)
        case = make_case(w, w, h, tau, BC_FREESLIP, BC_FREESLIP, int(round(0.08 * h)), g,
                         h_ini=z_start, h_end=z_end if z_start - z_end >= 1.0 else 0.0)
        case["re"], case["d_eq"], case["shape"] = re, D, ("sphere", "spheroid", "irregular")[shape]
        out.append((case, body))
    return out


# ---------------------------------------------------------------- random states
def smooth_noise(rng, shape, n_modes=4, kmax=2):
    """Sum of a few random low-wavenumber periodic modes, values in about [-1, 1]."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros(shape)
    for _ in range(n_modes):
        k = rng.integers(-kmax, kmax + 1, size=3)
        ph = rng.uniform(0, 2 * math.pi)
        out += np.cos(2 * math.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz) + ph)
    return out / n_modes


def taylor_green_populations(n, U0):
    """Initial state of the 3-D Taylor-Green vortex on an n^3 periodic box:
    density 1, u = U0 (sin a cos b cos c, -cos a sin b cos c, 0) with
    (a, b, c) = 2 pi (x, y, z) / n, populations from the second-order
    Maxwellian expansion w_i (1 + 3 xi.u + 9/2 (xi.u)^2 - 3/2 u^2).  Layout
    (nz, ny, nx, 27)."""
    t = 2 * math.pi * np.arange(n) / n
    c, b, a = np.meshgrid(t, t, t, indexing="ij")
    u = np.stack([U0 * np.sin(a) * np.cos(b) * np.cos(c), -U0 * np.cos(a) * np.sin(b) * np.cos(c),
                  np.zeros_like(a)], axis=-1)
    xi = np.array([[i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1] for i in range(27)], np.float64)
    xu = u @ xi.T
    uu = (u * u).sum(-1, keepdims=True)
    return D3Q27_W * (1.0 + 3.0 * xu + 4.5 * xu * xu - 1.5 * uu)


def couette_populations(nx, ny, nz, U):
    """Plane Couette flow between no-slip walls halfway outside the first and
    last rows moving at -U and +U in x: u_x(z) = U (2 (z + 1/2) / nz - 1),
    density 1, populations from the second-order Maxwellian expansion.
    Layout (27, nz, ny, nx)."""
    ux = U * (2.0 * (np.arange(nz) + 0.5) / nz - 1.0)
    xi_x = np.array([i % 3 - 1 for i in range(27)], np.float64)
    f = D3Q27_W[:, None] * (1.0 + 3.0 * xi_x[:, None] * ux[None, :] + 4.5 * (xi_x[:, None] * ux[None, :]) ** 2
                            - 1.5 * ux[None, :] ** 2)
    return np.ascontiguousarray(np.broadcast_to(f[:, :, None, None], (27, nz, ny, nx)))


def taylor_green_populations19(n, U0):
    """The same Taylor-Green state on the D3Q19 lattice.  Layout (nz, ny, nx, 19)."""
    t = 2 * math.pi * np.arange(n) / n
    c, b, a = np.meshgrid(t, t, t, indexing="ij")
    u = np.stack([U0 * np.sin(a) * np.cos(b) * np.cos(c), -U0 * np.cos(a) * np.sin(b) * np.cos(c),
                  np.zeros_like(a)], axis=-1)
    xu = u @ D3Q19_XI.T
    uu = (u * u).sum(-1, keepdims=True)
    return D3Q19_W * (1.0 + 3.0 * xu + 4.5 * xu * xu - 1.5 * uu)


def random_populations19(seed, nx, ny, nz, amp=0.02):
    """Near-rest D3Q19 field f_i = w_i (1 + amp * eta_i(x)), smooth random
    eta_i.  Layout (nz, ny, nx, 19)."""
    rng = np.random.default_rng(seed)
    f = np.empty((nz, ny, nx, 19))
    for i in range(19):
        f[..., i] = D3Q19_W[i] * (1.0 + amp * smooth_noise(rng, (nz, ny, nx)))
    return f


def random_populations(seed, nx, ny, nz, amp=0.02):
    """Near-rest population field f_i = w_i (1 + amp * eta_i(x)) with smooth
    random eta_i.  Layout (nz, ny, nx, 27)."""
    rng = np.random.default_rng(seed)
    f = np.empty((nz, ny, nx, 27))
    for i in range(27):
        f[..., i] = D3Q27_W[i] * (1.0 + amp * smooth_noise(rng, (nz, ny, nx)))
    return f


def random_vectors(seed, n, scale=1.0):
    return np.random.default_rng(seed).standard_normal((n, 3)) * scale
