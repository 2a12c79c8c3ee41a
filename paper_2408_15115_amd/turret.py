"""Python binding of libturret (include/turret.h): ctypes argument marshalling.

The functions below carry the C names and do nothing but convert arguments;
every step of the time iteration runs in the library's HIP kernels.  PyTorch
only provides the device buffers and the stream.  If the library has not
been built the import of this module fails: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libturret.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "turret.h")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_F32, LBM_F16, LBM_BF16 = 0, 1, 2
STORAGE = {"f32": LBM_F32, "f16": LBM_F16, "bf16": LBM_BF16}
ELEM_BYTES = {LBM_F32: 4, LBM_F16: 2, LBM_BF16: 2}
ERRNAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EHIP", -4: "LBM_EUNSTABLE", -5: "LBM_ESTATE"}


class lbm_case(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("bc_zlo", C.c_int32),
                ("bc_zhi", C.c_int32), ("sponge_cells", C.c_int32), ("tau", C.c_double),
                ("gravity", C.c_double), ("h_ini", C.c_double), ("h_end", C.c_double)]


class lbm_body(C.Structure):
    _fields_ = [("n_markers", C.c_int32), ("x_body", C.POINTER(C.c_double)), ("n_body", C.POINTER(C.c_double)),
                ("dS", C.POINTER(C.c_double)), ("kappa", C.c_double), ("volume", C.c_double),
                ("J_over_m", C.c_double * 9), ("r0", C.c_double * 3), ("d0", C.c_double * 9),
                ("v0", C.c_double * 3), ("w0", C.c_double * 3)]


class lbm_options(C.Structure):
    _fields_ = [("storage", C.c_int32), ("ibm_cycles", C.c_int32), ("block", C.c_int32),
                ("schedule", C.c_int32), ("persist_wgs", C.c_int32), ("reserved", C.c_int32 * 3)]


class lbm_buffers(C.Structure):
    _fields_ = [("pop_a", C.c_void_p), ("pop_b", C.c_void_p), ("aux", C.c_void_p)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
_lib = C.CDLL(LIB_PATH)

_P = C.POINTER
_ctx = C.c_void_p
_sig = {
    "lbm_required_bytes": (C.c_int32, [_P(lbm_case), _P(lbm_body), C.c_int32, _P(lbm_options), _P(C.c_int64)]),
    "lbm_init": (C.c_int32, [_P(lbm_case), _P(lbm_body), C.c_int32, _P(lbm_options), _P(lbm_buffers),
                             _P(C.c_int64), C.c_void_p, _P(_ctx)]),
    "body_advance": (C.c_int32, [_ctx]),
    "lbm_step": (C.c_int32, [_ctx]),
    "ibm_couple": (C.c_int32, [_ctx]),
    "window_shift": (C.c_int32, [_ctx]),
    "lbm_run": (C.c_int32, [_ctx, C.c_int32]),
    "lbm_graph_capture": (C.c_int32, [_ctx, C.c_int32]),
    "lbm_graph_launch": (C.c_int32, [_ctx]),
    "lbm_get_populations": (C.c_int32, [_ctx, C.c_int32, _P(C.c_double)]),
    "lbm_set_populations": (C.c_int32, [_ctx, C.c_int32, _P(C.c_double)]),
    "body_get_state": (C.c_int32, [_ctx, C.c_int32, _P(C.c_double)]),
    "lbm_save": (C.c_int32, [_ctx, C.c_char_p]),
    "lbm_load": (C.c_int32, [_ctx, C.c_char_p]),
    "lbm_pop_offset": (C.c_int64, [_ctx, C.c_int32]),
    "lbm_current_buffer": (C.c_void_p, [_ctx]),
    "lbm_stream_copy": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "lbm_destroy": (C.c_int32, [_ctx]),
    "lbm_last_error": (C.c_char_p, [_ctx]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


def exported_symbols():
    return list(_sig)


class TurretError(RuntimeError):
    def __init__(self, where, code, msg):
        super().__init__(f"{where}: {ERRNAMES.get(code, code)}: {msg}")
        self.code = code


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_case(d: dict) -> lbm_case:
    return lbm_case(int(d["nx"]), int(d["ny"]), int(d["nz"]), int(d.get("bc_zlo", 0)), int(d.get("bc_zhi", 0)),
                    int(d.get("sponge", 0)), float(d["tau"]), float(d.get("gravity", 0.0)),
                    float(d.get("h_ini", 0.0)), float(d.get("h_end", 0.0)))


def make_body(d: dict | None, keep: list) -> lbm_body:
    if d is None:
        return lbm_body()
    xb = np.ascontiguousarray(d["x_body"], np.float64)
    nb = np.ascontiguousarray(d["n_body"], np.float64)
    dS = np.ascontiguousarray(d["dS"], np.float64)
    keep += [xb, nb, dS]
    b = lbm_body()
    b.n_markers = xb.shape[0]
    b.x_body, b.n_body, b.dS = _dptr(xb), _dptr(nb), _dptr(dS)
    b.kappa, b.volume = float(d["kappa"]), float(d["volume"])
    b.J_over_m[:] = [float(v) for v in np.ravel(d["J_over_m"])]
    b.r0[:] = [float(v) for v in np.ravel(d["r0"])]
    b.d0[:] = [float(v) for v in np.ravel(d["d0"])]
    b.v0[:] = [float(v) for v in np.ravel(d["v0"])]
    b.w0[:] = [float(v) for v in np.ravel(d["w0"])]
    return b


def make_options(storage="f32", ibm_cycles=4, block=256, schedule=0, persist_wgs=0) -> lbm_options:
    o = lbm_options()
    o.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    o.ibm_cycles, o.block, o.schedule, o.persist_wgs = int(ibm_cycles), int(block), int(schedule), int(persist_wgs)
    return o


def required_bytes(cases, bodies=None, **opts):
    keep = []
    ca = (lbm_case * len(cases))(*[make_case(c) for c in cases])
    ba = (lbm_body * len(cases))(*[make_body(b, keep) for b in bodies]) if bodies is not None else None
    out = (C.c_int64 * 3)()
    o = make_options(**opts)
    rc = lbm_required_bytes(ca, ba, len(cases), C.byref(o), out)
    if rc:
        raise TurretError("lbm_required_bytes", rc, lbm_last_error(None).decode())
    return [int(v) for v in out]


def stream_copy(dst, src, nbytes, stream=None):
    """Device-to-device streaming copy through the library's copy kernel."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = lbm_stream_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), int(nbytes),
                         C.c_void_p(st.cuda_stream))
    if rc:
        raise TurretError("lbm_stream_copy", rc, lbm_last_error(None).decode())


class Solver:
    """One context over torch-allocated device buffers (argument marshalling
    only).  ``cases``/``bodies`` are lists of the workload dicts."""

    def __init__(self, cases, bodies=None, storage="f32", ibm_cycles=4, block=256, schedule=0,
                 persist_wgs=0, stream=None, device="cuda"):
        import torch

        self.torch = torch
        self.n = len(cases)
        self._keep = []
        self._cases = (lbm_case * self.n)(*[make_case(c) for c in cases])
        self._bodies = ((lbm_body * self.n)(*[make_body(b, self._keep) for b in bodies])
                        if bodies is not None else None)
        self._opt = make_options(storage, ibm_cycles, block, schedule, persist_wgs)
        self.dims = [(int(c["nx"]), int(c["ny"]), int(c["nz"])) for c in cases]
        sizes = (C.c_int64 * 3)()
        rc = lbm_required_bytes(self._cases, self._bodies, self.n, C.byref(self._opt), sizes)
        if rc:
            raise TurretError("lbm_required_bytes", rc, lbm_last_error(None).decode())
        self.sizes = [int(v) for v in sizes]
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.bufs = [torch.empty(max(s, 1), dtype=torch.uint8, device=device) for s in self.sizes]
        b = lbm_buffers(self.bufs[0].data_ptr(), self.bufs[1].data_ptr(), self.bufs[2].data_ptr())
        self._ctx = _ctx()
        rc = lbm_init(self._cases, self._bodies, self.n, C.byref(self._opt), C.byref(b), sizes,
                      C.c_void_p(self.stream.cuda_stream), C.byref(self._ctx))
        if rc:
            raise TurretError("lbm_init", rc, lbm_last_error(None).decode())

    def _chk(self, where, rc):
        if rc:
            raise TurretError(where, rc, lbm_last_error(self._ctx).decode())

    # --- the step sequence (Table 1)
    def body_advance(self):
        self._chk("body_advance", body_advance(self._ctx))

    def lbm_step(self):
        self._chk("lbm_step", lbm_step(self._ctx))

    def ibm_couple(self):
        self._chk("ibm_couple", ibm_couple(self._ctx))

    def window_shift(self):
        self._chk("window_shift", window_shift(self._ctx))

    def run(self, nsteps=1):
        self._chk("lbm_run", lbm_run(self._ctx, int(nsteps)))

    def graph_capture(self, steps=2):
        self._chk("lbm_graph_capture", lbm_graph_capture(self._ctx, int(steps)))

    def graph_launch(self):
        self._chk("lbm_graph_launch", lbm_graph_launch(self._ctx))

    # --- host copies
    def populations(self, case=0):
        nx, ny, nz = self.dims[case]
        out = np.empty((27, nz, ny, nx))
        self._chk("lbm_get_populations", lbm_get_populations(self._ctx, case, _dptr(out)))
        return out

    def set_populations(self, f, case=0):
        nx, ny, nz = self.dims[case]
        f = np.ascontiguousarray(f, np.float64).reshape(27, nz, ny, nx)
        self._chk("lbm_set_populations", lbm_set_populations(self._ctx, case, _dptr(f)))

    def body_state(self, case=0, check=True):
        o = np.zeros(32)
        rc = body_get_state(self._ctx, case, _dptr(o))
        if check:
            self._chk("body_get_state", rc)
        return {"r": o[0:3].copy(), "d": o[3:12].reshape(3, 3).copy(), "v": o[12:15].copy(),
                "w": o[15:18].copy(), "F": o[18:21].copy(), "T": o[21:24].copy(),
                "F_pressure": o[24:27].copy(), "ibm_residual": o[27], "steps": int(o[28]),
                "shifts": int(o[29]), "z0": int(o[30]), "err": int(o[31])}

    def save(self, path):
        self._chk("lbm_save", lbm_save(self._ctx, str(path).encode()))

    def load(self, path):
        self._chk("lbm_load", lbm_load(self._ctx, str(path).encode()))

    def pop_offset(self, case=0):
        return int(lbm_pop_offset(self._ctx, case))

    def current_buffer(self):
        return int(lbm_current_buffer(self._ctx))

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            lbm_destroy(self._ctx)
            self._ctx = _ctx()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
