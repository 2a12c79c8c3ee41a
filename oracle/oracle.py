"""ctypes wrapper of the FP64 CPU oracle (``orc.c``).

Test infrastructure only: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product path never imports it.  This module only
marshals numpy arrays into the C functions; every formula lives in ``orc.c``
(see its header for the paper passages each function follows).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "orc.c")
SRC19_PATH = os.path.join(_HERE, "orc19.c")     # the D3Q19 comparison lattice
# A test of the pins themselves may point this at a build with a planted mistake.
_OVERRIDE = os.environ.get("ORACLE_LIB_OVERRIDE")

BC_PERIODIC, BC_FREESLIP, BC_NOSLIP, BC_PRESSURE = 0, 1, 2, 3
STORAGE = {"f64": 0, "f32": 0, "f16": 1, "bf16": 2}   # stored-state precision of the oracle (f32: not modelled)


def build(force: bool = False) -> str:
    """Compile orc.c with gcc (-O2, OpenMP, strict IEEE: no fast-math)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(
            os.path.getmtime(SRC_PATH), os.path.getmtime(SRC19_PATH)):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               SRC_PATH, SRC19_PATH, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _OVERRIDE:
            L = C.CDLL(_OVERRIDE)
        else:
            build()
            L = C.CDLL(LIB_PATH)
        P = C.POINTER
        d, i32 = C.c_double, C.c_int32
        pd, pi = P(d), P(i32)
        L.orc_init.restype = None
        L.orc_lattice.argtypes = [pi, pd]
        L.orc_hermite.argtypes = [i32, pi, i32]
        L.orc_hermite.restype = d
        L.orc_feq.argtypes = [d, pd, pd]
        L.orc_fneq.argtypes = [pd, pd, pd]
        L.orc_a1.argtypes = [pd, pd, pi, i32]
        L.orc_a1.restype = d
        L.orc_collide_cell.argtypes = [pd, pd, d, pd]
        L.orc_collide_cell_v.argtypes = [pd, pd, d, i32, pd]
        L.orc_collide_cell_m.argtypes = [pd, pd, d, i32, i32, pd]
        L.orc_stress_cell.argtypes = [pd, d, pd, pd, pd]
        L.orc_phi.argtypes = [d]
        L.orc_phi.restype = d
        L.orc_tau_at.argtypes = [i32, d, i32, i32]
        L.orc_tau_at.restype = d
        L.orc_collide_grid.argtypes = [pi, d, i32, pd, pd, pd]
        L.orc_collide_grid_v.argtypes = [pi, d, i32, i32, pd, pd, pd]
        L.orc_collide_grid_m.argtypes = [pi, d, i32, i32, i32, pd, pd, pd]
        L.orc_stream_grid.argtypes = [pi, i32, i32, pd, pd]
        L.orc_stream_grid_w.argtypes = [pi, i32, i32, pd, pd, pd]
        L.orc_sim_set_walls.argtypes = [C.c_void_p, pd]
        L.orc_interp.argtypes = [pi, pd, i32, i32, pd, pd]
        L.orc_interp.restype = i32
        L.orc_spread.argtypes = [pi, i32, pd, pd, pd, pd]
        L.orc_spread.restype = i32
        L.orc_body_advance.argtypes = [pd, pd, pd]
        L.orc_sim_new.argtypes = [pi, pi, pd, i32, pd, pd, pd, pd]
        L.orc_sim_new.restype = C.c_void_p
        L.orc_sim_free.argtypes = [C.c_void_p]
        L.orc_sim_set_force_surface.argtypes = [C.c_void_p, d, pd]
        L.orc_sim_set_torque.argtypes = [C.c_void_p, pd]
        L.orc_sim_set_fluid_force.argtypes = [C.c_void_p, pd]
        L.orc_sim_set_storage.argtypes = [C.c_void_p, i32, d, pi]
        L.orc_round_format.argtypes = [d, i32]
        L.orc_round_format.restype = d
        L.orc_quantize.argtypes = [i32, C.c_int64, pd]
        L.orc19_lattice.argtypes = [pi, pd]
        L.orc19_feq.argtypes = [d, pd, pd]
        L.orc19_f1.argtypes = [pd, pd, pd]
        L.orc19_collide_cell.argtypes = [pd, d, i32, pd]
        L.orc19_run.argtypes = [i32, i32, i32, d, i32, pd, i32]
        L.orc19_collide_grid.argtypes = [i32, i32, i32, d, i32, pd]
        L.orc19_stream.argtypes = [i32, i32, i32, pd]
        L.orc_sim_set_f.argtypes = [C.c_void_p, pd]
        L.orc_sim_get_f.argtypes = [C.c_void_p, pd]
        L.orc_sim_get_h.argtypes = [C.c_void_p, pd]
        L.orc_sim_get_post_collision.argtypes = [C.c_void_p, pd]
        L.orc_sim_step.argtypes = [C.c_void_p, i32]
        L.orc_sim_step.restype = i32
        L.orc_sim_get_body.argtypes = [C.c_void_p, pd]
        L.orc_sim_get_markers.argtypes = [C.c_void_p, pd, pd, pd, pd]
        L.orc_num_threads.restype = i32
        L.orc_set_threads.argtypes = [i32]
        L.orc_init()
        _lib = L
    return _lib


def _pd(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _pi(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


# ------------------------------------------------------------- per-cell ops
def lattice():
    xi = np.zeros((27, 3), np.int32)
    w = np.zeros(27)
    lib().orc_lattice(_pi(xi), _pd(w))
    return xi, w


def hermite(i, idx):
    al = np.ascontiguousarray(idx, dtype=np.int32)
    return lib().orc_hermite(int(i), _pi(al), len(al))


def feq(p, u):
    out = np.zeros(27)
    lib().orc_feq(float(p), _pd(_f64(u)), _pd(out))
    return out


def fneq(P1, u):
    out = np.zeros(27)
    lib().orc_fneq(_pd(_f64(P1, (9,))), _pd(_f64(u)), _pd(out))
    return out


def a1(P1, u, idx):
    al = np.ascontiguousarray(idx, dtype=np.int32)
    return lib().orc_a1(_pd(_f64(P1, (9,))), _pd(_f64(u)), _pi(al), len(al))


def collide_cell(f, h, tau, forcing=0, collision=0):
    """Forced collision of one cell (Sec. 2.2); forcing 1 = momentum-exact
    variant; collision 1 = BGK (raw off-equilibrium) for comparison."""
    out = np.zeros(27)
    hp = _pd(_f64(h)) if h is not None else None
    lib().orc_collide_cell_m(_pd(_f64(f)), hp, float(tau), int(forcing), int(collision), _pd(out))
    return out


def stress_cell(f, tau):
    sig = np.zeros(9)
    rho = np.zeros(1)
    u = np.zeros(3)
    lib().orc_stress_cell(_pd(_f64(f)), float(tau), _pd(sig), _pd(rho), _pd(u))
    return sig.reshape(3, 3), rho[0], u


def phi(r):
    return lib().orc_phi(float(r))


def tau_at(nz, tau0, sponge, z):
    return lib().orc_tau_at(int(nz), float(tau0), int(sponge), int(z))


def round_format(x, storage):
    """x rounded to the nearest binary16 / bfloat16 value (ties to even)."""
    return lib().orc_round_format(float(x), STORAGE[storage])


def quantize(f, storage):
    """Populations (..., 27) as the reduced-precision store holds them:
    w_i + q(s_i (f_i - w_i)) / s_i with s_i = 2^(14 + 2 |xi_i|^2)."""
    f = np.array(f, np.float64, order="C")
    lib().orc_quantize(STORAGE[storage], f.size // 27, _pd(f))
    return f


# ------------------------------------------------------------- grid ops
# Grid arrays are (nz, ny, nx, ncomp) in the oracle's own layout.
def collide_grid(f, tau0, sponge=0, h=None, forcing=0, collision=0):
    f = _f64(f)
    nz, ny, nx, _ = f.shape
    dims = np.array([nx, ny, nz], np.int32)
    out = np.zeros_like(f)
    hp = _pd(_f64(h)) if h is not None else None
    lib().orc_collide_grid_m(_pi(dims), float(tau0), int(sponge), int(forcing), int(collision), _pd(f), hp,
                             _pd(out))
    return out


def stream_grid(C_, bc_lo=BC_PERIODIC, bc_hi=BC_PERIODIC, u_wall=(0.0, 0.0)):
    """Pull-streaming with the z wall rules; u_wall = x velocities of no-slip
    bottom and top walls."""
    C_ = _f64(C_)
    nz, ny, nx, _ = C_.shape
    dims = np.array([nx, ny, nz], np.int32)
    out = np.zeros_like(C_)
    uw = _f64(u_wall)
    lib().orc_stream_grid_w(_pi(dims), int(bc_lo), int(bc_hi), _pd(uw), _pd(C_), _pd(out))
    return out


def interp(field, X):
    field = _f64(field)
    nz, ny, nx, nc = field.shape
    X = _f64(X)
    M = X.shape[0]
    out = np.zeros((M, nc))
    rc = lib().orc_interp(_pi(np.array([nx, ny, nz], np.int32)), _pd(field), nc, M, _pd(X), _pd(out))
    if rc:
        raise ValueError("marker stencil leaves the domain in z")
    return out


def spread(shape, X, h, dS):
    nz, ny, nx = shape
    X, h, dS = _f64(X), _f64(h), _f64(dS)
    out = np.zeros((nz, ny, nx, 3))
    rc = lib().orc_spread(_pi(np.array([nx, ny, nz], np.int32)), X.shape[0], _pd(X), _pd(h), _pd(dS), _pd(out))
    if rc:
        raise ValueError("marker stencil leaves the domain in z")
    return out


def body_advance(state, F, T, kappa, volume, J_over_m, gravity):
    """state: dict r, d (3x3 rows), v, w.  Returns the advanced copy."""
    st = np.concatenate([np.ravel(state["r"]), np.ravel(state["d"]), np.ravel(state["v"]), np.ravel(state["w"])])
    st = _f64(st)
    FT = _f64(np.concatenate([np.ravel(F), np.ravel(T)]))
    prm = _f64(np.concatenate([[kappa, volume], np.ravel(J_over_m), [gravity]]))
    lib().orc_body_advance(_pd(st), _pd(FT), _pd(prm))
    return {"r": st[0:3].copy(), "d": st[3:12].reshape(3, 3).copy(), "v": st[12:15].copy(), "w": st[15:18].copy()}


# ------------------------------------------------------------ D3Q19 lattice
def lattice19():
    """(xi (19, 3) int, w (19,)) of the D3Q19 comparison lattice."""
    xi = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    lib().orc19_lattice(_pi(xi), _pd(w))
    return xi, w


def feq19(rho, u):
    out = np.zeros(19)
    lib().orc19_feq(float(rho), _pd(_f64(u)), _pd(out))
    return out


def f1_19(P1, u):
    out = np.zeros(19)
    lib().orc19_f1(_pd(_f64(P1, (3, 3))), _pd(_f64(u)), _pd(out))
    return out


def collide19(f, tau, collision=0):
    out = np.zeros(19)
    lib().orc19_collide_cell(_pd(_f64(f)), float(tau), int(collision), _pd(out))
    return out


def run19(f, tau, nsteps, collision=0):
    """nsteps of the D3Q19 fluid step on a periodic box; f is (nz, ny, nx, 19)."""
    f = np.array(f, np.float64, order="C")
    nz, ny, nx, q = f.shape
    assert q == 19
    lib().orc19_run(nx, ny, nz, float(tau), int(collision), _pd(f), int(nsteps))
    return f


def collide_grid19(f, tau, collision=0):
    """The D3Q19 collision on every cell of an (nz, ny, nx, 19) field."""
    f = np.array(f, np.float64, order="C")
    nz, ny, nx, q = f.shape
    assert q == 19
    lib().orc19_collide_grid(nx, ny, nz, float(tau), int(collision), _pd(f))
    return f


def stream19(f):
    """Periodic pull-streaming of an (nz, ny, nx, 19) field."""
    f = np.array(f, np.float64, order="C")
    nz, ny, nx, q = f.shape
    assert q == 19
    lib().orc19_stream(nx, ny, nz, _pd(f))
    return f


# ------------------------------------------------------------- simulation
class OracleSim:
    """The full coupled time iteration (Table 1) on one case.

    ``case`` and ``body`` are the plain dicts produced by the workload
    generators (keys: nx ny nz tau bc_zlo bc_zhi sponge gravity h_ini h_end
    ibm_cycles, and optionally forcing: 0 = forced rule as printed, 1 =
    momentum-exact variant; kappa volume J_over_m r0 d0 v0 w0 x_body n_body
    dS, and optionally force_offset > 0 with dS_offset: the stress integral
    on the parallel surface at that distance outside the markers)."""

    def __init__(self, case: dict, body: dict | None):
        L = lib()
        self.nx, self.ny, self.nz = int(case["nx"]), int(case["ny"]), int(case["nz"])
        dims = np.array([self.nx, self.ny, self.nz], np.int32)
        ip = np.array([case.get("bc_zlo", 0), case.get("bc_zhi", 0), case.get("sponge", 0),
                       case.get("ibm_cycles", 4), case.get("forcing", 0), case.get("collision", 0)], np.int32)
        dp = _f64([case["tau"], case.get("gravity", 0.0), case.get("h_ini", 0.0), case.get("h_end", 0.0)])
        if body is None:
            M = 0
            xb = nb = np.zeros((1, 3))
            dS = np.zeros(1)
            bp = _f64(np.concatenate([[1.0, 1.0], np.eye(3).ravel(), np.zeros(3), np.eye(3).ravel(),
                                      np.zeros(3), np.zeros(3)]))
        else:
            xb, nb, dS = _f64(body["x_body"]), _f64(body["n_body"]), _f64(body["dS"])
            M = xb.shape[0]
            bp = _f64(np.concatenate([[body["kappa"], body["volume"]], np.ravel(body["J_over_m"]),
                                      np.ravel(body["r0"]), np.ravel(body["d0"]), np.ravel(body["v0"]),
                                      np.ravel(body["w0"])]))
        self.M = M
        self._keep = (dims, ip, dp, xb, nb, dS, bp)
        self._p = L.orc_sim_new(_pi(dims), _pi(ip), _pd(dp), M, _pd(xb), _pd(nb), _pd(dS), _pd(bp))
        if case.get("u_wall_lo", 0.0) != 0.0 or case.get("u_wall_hi", 0.0) != 0.0:
            uw = _f64([case.get("u_wall_lo", 0.0), case.get("u_wall_hi", 0.0)])
            self._keep = self._keep + (uw,)
            L.orc_sim_set_walls(self._p, _pd(uw))
        if body is not None and body.get("torque") is not None:
            tq = _f64(body["torque"])
            self._keep = self._keep + (tq,)
            L.orc_sim_set_torque(self._p, _pd(tq))
        if body is not None and body.get("force_offset", 0.0) > 0.0:
            dSo = _f64(body["dS_offset"])
            self._keep = self._keep + (dSo,)
            L.orc_sim_set_force_surface(self._p, float(body["force_offset"]), _pd(dSo))

    def set_storage(self, storage, box=None):
        """Store the post-collision state in "f16" or "bf16" (the build's
        precision form).  box = (rb, (ex, ey, ez)) keeps the cells
        floor(r_a - rb) - 3 ... + e_a - 1 around the body in FP64."""
        rb, edges = box if box is not None else (0.0, (0, 0, 0))
        e = np.array(edges, np.int32)
        self._keep = self._keep + (e,)
        lib().orc_sim_set_storage(self._p, STORAGE[storage], float(rb), _pi(e))

    def set_fluid_force(self, g):
        """A uniform force per unit mass on the whole fluid, added to the
        immersed force in every collision."""
        gf = _f64(g)
        self._keep = self._keep + (gf,)
        lib().orc_sim_set_fluid_force(self._p, _pd(gf))

    def __del__(self):
        if getattr(self, "_p", None):
            lib().orc_sim_free(self._p)
            self._p = None

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def step(self, n: int = 1):
        rc = lib().orc_sim_step(self._p, int(n))
        if rc:
            raise RuntimeError("oracle step failed: marker stencil left the domain")

    def set_populations(self, f):
        f = _f64(f, (self.nz, self.ny, self.nx, 27))
        lib().orc_sim_set_f(self._p, _pd(f))

    def populations(self):
        out = np.zeros((self.nz, self.ny, self.nx, 27))
        lib().orc_sim_get_f(self._p, _pd(out))
        return out

    def immersed_force(self):
        out = np.zeros((self.nz, self.ny, self.nx, 3))
        lib().orc_sim_get_h(self._p, _pd(out))
        return out

    def post_collision(self):
        out = np.zeros((self.nz, self.ny, self.nx, 27))
        lib().orc_sim_get_post_collision(self._p, _pd(out))
        return out

    def body_state(self) -> dict:
        o = np.zeros(34)
        lib().orc_sim_get_body(self._p, _pd(o))
        return {"r": o[0:3].copy(), "d": o[3:12].reshape(3, 3).copy(), "v": o[12:15].copy(),
                "w": o[15:18].copy(), "F": o[18:21].copy(), "T": o[21:24].copy(),
                "F_pressure": o[24:27].copy(), "ibm_residual": o[27], "steps": int(o[28]),
                "shifts": int(o[29]), "pending_shift": int(o[30])}

    def markers(self):
        M = max(self.M, 1)
        X, N, U, H = (np.zeros((M, 3)) for _ in range(4))
        lib().orc_sim_get_markers(self._p, _pd(X), _pd(N), _pd(U), _pd(H))
        return X[: self.M], N[: self.M], U[: self.M], H[: self.M]


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))
