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
LIB_PATH = os.environ.get("TURRET_LIB") or os.path.join(HERE, "libturret.so")   # TURRET_LIB: another build
HEADER = os.path.join(os.path.dirname(HERE), "include", "turret.h")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_F32, LBM_F16, LBM_BF16, LBM_MOM = 0, 1, 2, 3
LBM_WARM_NONE, LBM_WARM_PREVIOUS, LBM_WARM_MLP = 0, 1, 2
MLP_IN = 16   # network inputs (LBM_MLP_IN)
FEAT_NORMAL = 12   # first of the three normal components among the features
MLP_PARAMS = MLP_IN * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3
STORAGE = {"f32": LBM_F32, "f16": LBM_F16, "bf16": LBM_BF16, "mom": LBM_MOM}
ELEM_BYTES = {LBM_F32: 4, LBM_F16: 2, LBM_BF16: 2, LBM_MOM: 4}
ERRNAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EHIP", -4: "LBM_EUNSTABLE", -5: "LBM_ESTATE"}


class lbm_case(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("bc_zlo", C.c_int32),
                ("bc_zhi", C.c_int32), ("sponge_cells", C.c_int32), ("tau", C.c_double),
                ("gravity", C.c_double), ("h_ini", C.c_double), ("h_end", C.c_double),
                ("u_wall", C.c_double * 2)]


class lbm_body(C.Structure):
    _fields_ = [("n_markers", C.c_int32), ("x_body", C.POINTER(C.c_double)), ("n_body", C.POINTER(C.c_double)),
                ("dS", C.POINTER(C.c_double)), ("kappa", C.c_double), ("volume", C.c_double),
                ("J_over_m", C.c_double * 9), ("r0", C.c_double * 3), ("d0", C.c_double * 9),
                ("v0", C.c_double * 3), ("w0", C.c_double * 3), ("force_offset", C.c_double),
                ("dS_offset", C.POINTER(C.c_double)), ("torque", C.c_double * 3)]


class lbm_options(C.Structure):
    _fields_ = [("storage", C.c_int32), ("ibm_cycles", C.c_int32), ("block", C.c_int32),
                ("schedule", C.c_int32), ("persist_wgs", C.c_int32), ("tile_order", C.c_int32),
                ("ibm_diag", C.c_int32), ("forcing", C.c_int32), ("serial_ibm", C.c_int32),
                ("collision", C.c_int32), ("lattice", C.c_int32), ("fine_box", C.c_int32)]


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
    "lbm_set_schedule": (C.c_int32, [_ctx, _P(lbm_options)]),
    "lbm_graph_capture": (C.c_int32, [_ctx, C.c_int32]),
    "lbm_graph_launch": (C.c_int32, [_ctx]),
    "lbm_get_populations": (C.c_int32, [_ctx, C.c_int32, _P(C.c_double)]),
    "lbm_set_populations": (C.c_int32, [_ctx, C.c_int32, _P(C.c_double)]),
    "lbm_get_populations_noalloc": (C.c_int32, [_ctx, C.c_int32, C.c_void_p]),
    "body_get_state": (C.c_int32, [_ctx, C.c_int32, _P(C.c_double)]),
    "lbm_log_read": (C.c_int32, [_ctx, C.c_int32, _P(C.c_double), C.c_int32, _P(C.c_int32), _P(C.c_int64)]),
    "lbm_save": (C.c_int32, [_ctx, C.c_char_p]),
    "lbm_load": (C.c_int32, [_ctx, C.c_char_p]),
    "lbm_pop_offset": (C.c_int64, [_ctx, C.c_int32]),
    "lbm_plane_stride": (C.c_int64, [_ctx, C.c_int32]),
    "lbm_current_buffer": (C.c_void_p, [_ctx]),
    "lbm_stream_copy": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "mlp_required_bytes": (C.c_int32, [C.c_int32, _P(C.c_int64)]),
    "mlp_create": (C.c_int32, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, _P(C.c_void_p)]),
    "mlp_set_params": (C.c_int32, [C.c_void_p, _P(C.c_float)]),
    "mlp_get_params": (C.c_int32, [C.c_void_p, _P(C.c_float)]),
    "mlp_forward": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "mlp_grad": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "mlp_train_step": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float, C.c_void_p]),
    "mlp_destroy": (C.c_int32, [C.c_void_p]),
    "mlp_last_error": (C.c_char_p, [C.c_void_p]),
    "lbm_set_warm_start": (C.c_int32, [_ctx, C.c_int32, C.c_void_p, C.c_int32]),
    "lbm_set_ibm_gate": (C.c_int32, [_ctx, C.c_int32, C.c_double]),
    "lbm_ibm_samples": (C.c_int32, [_ctx, C.c_void_p, C.c_void_p]),
    "lbm_marker_count": (C.c_int32, [_ctx]),
    "lbm_ibm_stats": (C.c_int32, [_ctx, C.c_int32, _P(C.c_double)]),
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
    c = lbm_case(int(d["nx"]), int(d["ny"]), int(d["nz"]), int(d.get("bc_zlo", 0)), int(d.get("bc_zhi", 0)),
                 int(d.get("sponge", 0)), float(d["tau"]), float(d.get("gravity", 0.0)),
                 float(d.get("h_ini", 0.0)), float(d.get("h_end", 0.0)))
    c.u_wall[0], c.u_wall[1] = float(d.get("u_wall_lo", 0.0)), float(d.get("u_wall_hi", 0.0))
    return c


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
    if d.get("torque") is not None:
        b.torque[:] = [float(v) for v in np.ravel(d["torque"])]
    if d.get("force_offset", 0.0) > 0.0:
        b.force_offset = float(d["force_offset"])
        if d.get("dS_offset") is not None:   # else NULL: the library rejects the body
            dSo = np.ascontiguousarray(d["dS_offset"], np.float64)
            keep.append(dSo)
            b.dS_offset = _dptr(dSo)
    return b


def make_options(storage="f32", ibm_cycles=4, block=256, schedule=0, persist_wgs=0, tile_order=0,
                 ibm_diag=0, forcing=0, serial_ibm=0, collision=0, lattice=27, fine_box=0) -> lbm_options:
    o = lbm_options()
    o.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    o.ibm_cycles, o.block, o.schedule, o.persist_wgs = int(ibm_cycles), int(block), int(schedule), int(persist_wgs)
    o.tile_order, o.ibm_diag, o.forcing, o.serial_ibm = int(tile_order), int(ibm_diag), int(forcing), int(serial_ibm)
    o.collision, o.lattice, o.fine_box = int(collision), int(lattice), int(fine_box)
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
                 persist_wgs=0, tile_order=0, ibm_diag=0, forcing=0, serial_ibm=0, collision=0, stream=None,
                 device="cuda", lattice=27, fine_box=None):
        # FP16/BF16 storage keeps the full-precision box around each body
        # unless told otherwise
        if fine_box is None:
            fine_box = int(storage in ("f16", "bf16") and bodies is not None
                           and any(b is not None and len(b["x_body"]) > 0 for b in bodies))
        import torch

        self.torch = torch
        self.n = len(cases)
        self._keep = []
        self._cases = (lbm_case * self.n)(*[make_case(c) for c in cases])
        self._bodies = ((lbm_body * self.n)(*[make_body(b, self._keep) for b in bodies])
                        if bodies is not None else None)
        self._opt = make_options(storage, ibm_cycles, block, schedule, persist_wgs, tile_order, ibm_diag, forcing,
                                 serial_ibm, collision, lattice, fine_box)
        self.q = 19 if lattice == 19 else 27
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

    def set_schedule(self, block=256, schedule=0, persist_wgs=0, tile_order=0):
        o = make_options(self._opt.storage, self._opt.ibm_cycles, block, schedule, persist_wgs, tile_order,
                         self._opt.ibm_diag, self._opt.forcing, self._opt.serial_ibm, self._opt.collision,
                         self._opt.lattice, self._opt.fine_box)
        self._chk("lbm_set_schedule", lbm_set_schedule(self._ctx, C.byref(o)))
        self._opt = o

    def graph_capture(self, steps=2):
        self._chk("lbm_graph_capture", lbm_graph_capture(self._ctx, int(steps)))

    def graph_launch(self):
        self._chk("lbm_graph_launch", lbm_graph_launch(self._ctx))

    # --- host copies
    def populations(self, case=0):
        nx, ny, nz = self.dims[case]
        out = np.empty((self.q, nz, ny, nx))
        self._chk("lbm_get_populations", lbm_get_populations(self._ctx, case, _dptr(out)))
        return out

    def populations_noalloc(self, out, case=0):
        """lbm_get_populations_noalloc into a device tensor ``out`` of
        q * nx * ny * nz float64 values (asynchronous on the stream)."""
        nx, ny, nz = self.dims[case]
        assert out.dtype == self.torch.float64 and out.is_cuda and out.is_contiguous()
        assert out.numel() >= self.q * nx * ny * nz
        self._chk("lbm_get_populations_noalloc", lbm_get_populations_noalloc(self._ctx, case, C.c_void_p(out.data_ptr())))

    def set_populations(self, f, case=0):
        nx, ny, nz = self.dims[case]
        f = np.ascontiguousarray(f, np.float64).reshape(self.q, nz, ny, nx)
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

    LOG_CAPACITY = 1024

    def log_read(self, case=0, max_records=LOG_CAPACITY):
        """Step records of the case not read before, oldest first, as an
        (n, 32) array in the layout of body_get_state, and the number of
        records overwritten before they were read."""
        out = np.zeros((max(int(max_records), 1), 32))
        n, lost = C.c_int32(0), C.c_int64(0)
        self._chk("lbm_log_read", lbm_log_read(self._ctx, int(case), _dptr(out), int(max_records), C.byref(n),
                                               C.byref(lost)))
        return out[:n.value].copy(), int(lost.value)

    # --- learned warm start
    def set_warm_start(self, mode, mlp=None, cycles=4):
        mp = C.c_void_p(mlp._m.value) if mlp is not None else None
        self._chk("lbm_set_warm_start", lbm_set_warm_start(self._ctx, int(mode), mp, int(cycles)))

    def set_ibm_gate(self, case, threshold):
        self._chk("lbm_set_ibm_gate", lbm_set_ibm_gate(self._ctx, int(case), float(threshold)))

    def marker_count(self):
        return int(lbm_marker_count(self._ctx))

    def ibm_samples(self):
        """(features, targets) of the last ibm_couple as new device tensors.
        The library writes them on the context's stream; the caller's current
        stream is made to wait for that before they are returned."""
        torch = self.torch
        M = self.marker_count()
        cur = torch.cuda.current_stream()
        with torch.cuda.stream(self.stream):
            f = torch.empty((M, MLP_IN), dtype=torch.float32, device="cuda")
            t = torch.empty((M, 3), dtype=torch.float32, device="cuda")
            self._chk("lbm_ibm_samples", lbm_ibm_samples(self._ctx, C.c_void_p(f.data_ptr()),
                                                         C.c_void_p(t.data_ptr())))
        cur.wait_stream(self.stream)
        f.record_stream(cur)
        t.record_stream(cur)
        return f, t

    def ibm_stats(self, case=0):
        o = np.zeros(24)
        self._chk("lbm_ibm_stats", lbm_ibm_stats(self._ctx, case, _dptr(o)))
        return {"resid": o[0], "resid_hist": o[1:9].copy(), "resid_hist_fallback": o[9:17].copy(),
                "accepts": int(o[17]), "rejects": int(o[18]), "fallback": int(o[19]),
                "warm_cycles_accepted": int(o[20])}

    def save(self, path):
        self._chk("lbm_save", lbm_save(self._ctx, str(path).encode()))

    def load(self, path):
        self._chk("lbm_load", lbm_load(self._ctx, str(path).encode()))

    def pop_offset(self, case=0):
        return int(lbm_pop_offset(self._ctx, case))

    def plane_stride(self, case=0):
        return int(lbm_plane_stride(self._ctx, case))

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


def mlp_init_params(seed):
    """He-uniform weights (bound sqrt(6 / fan_in)) and zero biases, FP32, in
    the library's flat layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((MLP_IN, 64), (64, 64), (64, 3)):
        b = np.sqrt(6.0 / fan_in)
        parts += [rng.uniform(-b, b, size=fan_out * fan_in), np.zeros(fan_out)]
    return np.concatenate(parts).astype(np.float32)


class MLP:
    """The warm-start network object over a torch device buffer (marshalling
    only; all arithmetic runs in the library's kernels)."""

    def __init__(self, max_batch=65536, params=None, seed=0, stream=None):
        import torch

        self.torch = torch
        self.max_batch = int(max_batch)
        nb = C.c_int64()
        if mlp_required_bytes(self.max_batch, C.byref(nb)):
            raise TurretError("mlp_required_bytes", LBM_EINVAL, mlp_last_error(None).decode())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.buf = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        self._m = C.c_void_p()
        rc = mlp_create(C.c_void_p(self.buf.data_ptr()), nb.value, self.max_batch,
                        C.c_void_p(self.stream.cuda_stream), C.byref(self._m))
        if rc:
            raise TurretError("mlp_create", rc, mlp_last_error(None).decode())
        self.set_params(mlp_init_params(seed) if params is None else params)

    def _chk(self, where, rc):
        if rc:
            raise TurretError(where, rc, mlp_last_error(self._m).decode())

    def set_params(self, params):
        a = np.ascontiguousarray(params, np.float32)
        assert a.size == MLP_PARAMS
        self._chk("mlp_set_params", mlp_set_params(self._m, a.ctypes.data_as(C.POINTER(C.c_float))))

    def params(self):
        a = np.empty(MLP_PARAMS, np.float32)
        self._chk("mlp_get_params", mlp_get_params(self._m, a.ctypes.data_as(C.POINTER(C.c_float))))
        return a

    def forward(self, X, out=None):
        X = X.contiguous()
        Y = out if out is not None else self.torch.empty((X.shape[0], 3), dtype=self.torch.float32, device="cuda")
        if Y.shape != (X.shape[0], 3) or Y.dtype != self.torch.float32 or not Y.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor of shape (n, 3)")
        self._chk("mlp_forward", mlp_forward(self._m, C.c_void_p(X.data_ptr()), X.shape[0], C.c_void_p(Y.data_ptr())))
        return Y

    def grad(self, X, Tg):
        X, Tg = X.contiguous(), Tg.contiguous()
        g = self.torch.empty(MLP_PARAMS, dtype=self.torch.float32, device="cuda")
        loss = self.torch.empty(1, dtype=self.torch.float32, device="cuda")
        self._chk("mlp_grad", mlp_grad(self._m, C.c_void_p(X.data_ptr()), C.c_void_p(Tg.data_ptr()), X.shape[0],
                                       C.c_void_p(g.data_ptr()), C.c_void_p(loss.data_ptr())))
        return g, loss

    def train_step(self, X, Tg, lr=1e-3, loss=None):
        lp = C.c_void_p(loss.data_ptr()) if loss is not None else None
        self._chk("mlp_train_step", mlp_train_step(self._m, C.c_void_p(X.data_ptr()), C.c_void_p(Tg.data_ptr()),
                                                   X.shape[0], float(lr), lp))

    def close(self):
        if getattr(self, "_m", None) is not None and self._m.value:
            mlp_destroy(self._m)
            self._m = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
