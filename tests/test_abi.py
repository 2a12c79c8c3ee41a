"""The C-ABI library loads, exports every function include/turret.h declares,
and rejects invalid arguments on the host before touching the GPU."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2408_15115_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "turret.h")
LIB = os.path.join(ROOT, "paper_2408_15115_amd", "libturret.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["lbm_init", "lbm_step", "ibm_couple", "body_advance", "window_shift", "lbm_required_bytes",
              "lbm_graph_capture", "lbm_graph_launch", "body_get_state", "lbm_destroy", "lbm_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first"
    lib = C.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert set(declared_functions()) <= exported


def test_binding_covers_the_header():
    from paper_2408_15115_amd import turret as T
    assert set(declared_functions()) == set(T.exported_symbols())


def test_required_bytes_of_the_sphere_case():
    from paper_2408_15115_amd import turret as T
    case, body = W.case_sphere48()
    a, b, aux = T.required_bytes([case], [body])
    plane = 48 ** 3 + 256          # direction planes staggered by 1 KB (256 four-byte elements)
    assert a == b == 27 * plane * 4
    a16, _, _ = T.required_bytes([case], [body], storage="f16")
    assert a16 == 27 * (48 ** 3 + 512) * 2   # the 1 KB stagger is 512 two-byte elements
    assert aux > 400 * 8 * 3


@pytest.mark.parametrize("mutate,needle", [
    (lambda c, b: c.update(tau=0.5), "tau"),
    (lambda c, b: c.update(nx=7), "dimension"),
    (lambda c, b: c.update(sponge=1), "sponge"),
    (lambda c, b: b.update(r0=np.array([23.5, 23.5, 4.0])), "wall"),
    (lambda c, b: c.update(bc_zlo=0), "periodic"),
    (lambda c, b: c.update(nx=12, ny=12), "region"),
    (lambda c, b: b.update(torque=np.array([0.0, np.nan, 0.0])), "torque"),
])
def test_invalid_cases_rejected_on_host(mutate, needle):
    from paper_2408_15115_amd import turret as T
    case, body = W.case_sphere48()
    mutate(case, body)
    with pytest.raises(T.TurretError) as e:
        T.required_bytes([case], [body])
    assert e.value.code == T.LBM_EINVAL
    assert needle in str(e.value)


def test_init_rejects_null_buffers_without_gpu():
    from paper_2408_15115_amd import turret as T
    case, body = W.case_sphere48()
    keep = []
    ca = (T.lbm_case * 1)(T.make_case(case))
    ba = (T.lbm_body * 1)(T.make_body(body, keep))
    o = T.make_options()
    bufs = T.lbm_buffers(None, None, None)
    sizes = (C.c_int64 * 3)(1, 1, 1)
    ctx = C.c_void_p()
    rc = T.lbm_init(ca, ba, 1, C.byref(o), C.byref(bufs), sizes, None, C.byref(ctx))
    assert rc == T.LBM_EINVAL and not ctx.value
    assert b"NULL" in T.lbm_last_error(None)


def test_bad_options_rejected():
    from paper_2408_15115_amd import turret as T
    case, body = W.case_sphere48()
    for kw in ({"storage": 7}, {"block": 96}, {"schedule": 5}, {"ibm_cycles": 40}, {"forcing": 2},
               {"serial_ibm": 3}, {"collision": 2}, {"ibm_diag": 2}, {"tile_order": 3}):
        with pytest.raises(T.TurretError):
            T.required_bytes([case], [body], **kw)


def test_force_surface_checks():
    """A body with force_offset > 0 needs the offset areas, keeps its offset
    points two cells inside the z walls, and gets a larger region."""
    from paper_2408_15115_amd import turret as T
    case, body = W.case_sphere48()
    assert body["force_offset"] == W.FORCE_OFFSET == 3.0        # the default reading
    at_markers = W.sphere_fibonacci_body(4.0, 400, 2.0, body["r0"], force_offset=0.0)
    _, _, aux0 = T.required_bytes([case], [at_markers])
    b = W.sphere_fibonacci_body(4.0, 400, 2.0, body["r0"], force_offset=3.0)
    _, _, aux1 = T.required_bytes([case], [b])
    assert aux1 > aux0
    nod = dict(b)
    nod.pop("dS_offset")
    with pytest.raises(T.TurretError) as e:
        T.required_bytes([case], [nod])
    assert "dS_offset" in str(e.value)
    low = W.sphere_fibonacci_body(4.0, 400, 2.0, [23.5, 23.5, 7.0], force_offset=3.0)
    with pytest.raises(T.TurretError) as e:
        T.required_bytes([case], [low])
    assert "wall" in str(e.value)


def test_pressure_wall_accepted_and_unknown_wall_rejected():
    from paper_2408_15115_amd import turret as T
    case, body = W.case_sphere48()
    T.required_bytes([dict(case, bc_zlo=W.BC_NOSLIP, bc_zhi=W.BC_PRESSURE)], [body])
    with pytest.raises(T.TurretError):
        T.required_bytes([dict(case, bc_zhi=4)], [body])


def test_degenerate_and_maximum_sizes_on_host():
    """No case at all, a box of 2^31 cells or more, and a particle-free case
    next to a particle case."""
    from paper_2408_15115_amd import turret as T
    case, body = W.case_sphere48()
    with pytest.raises(T.TurretError) as e:
        T.required_bytes([], [])
    assert "at least one case" in str(e.value)
    with pytest.raises(T.TurretError) as e:
        T.required_bytes([dict(case, nx=2048, ny=1024, nz=1024)], None)
    assert "2^31" in str(e.value)
    a = T.required_bytes([case, case], [body, None])
    b = T.required_bytes([case], [body])
    assert a[0] == 2 * b[0] and a[2] >= b[2]


def test_d3q19_lattice_option():
    """The D3Q19 comparison lattice: 19 planes per case, FP32 storage and
    schedule 0 only, fluid-only, periodic z, no sponge."""
    from paper_2408_15115_amd import turret as T
    case = W.make_case(24, 20, 16, 0.6, W.BC_PERIODIC, W.BC_PERIODIC, 0)
    a, b, _ = T.required_bytes([case], None, lattice=19)
    plane = 24 * 20 * 16 + 256
    assert a == b == 19 * plane * 4
    assert T.required_bytes([case], None)[0] == 27 * plane * 4
    bad = [({"storage": "f16"}, "FP32"), ({"schedule": 1}, "schedule 0"), ({"lattice": 21}, "lattice")]
    for kw, needle in bad:
        with pytest.raises(T.TurretError) as e:
            T.required_bytes([case], None, **dict({"lattice": 19}, **kw))
        assert needle in str(e.value)
    for c in (dict(case, bc_zlo=W.BC_FREESLIP, bc_zhi=W.BC_FREESLIP), dict(case, sponge=2)):
        with pytest.raises(T.TurretError) as e:
            T.required_bytes([c], None, lattice=19)
        assert "periodic z" in str(e.value)
    sc, sb = W.case_sphere48()
    sc = dict(sc, bc_zlo=W.BC_PERIODIC, bc_zhi=W.BC_PERIODIC)
    with pytest.raises(T.TurretError) as e:
        T.required_bytes([sc], [sb], lattice=19)
    assert "fluid-only" in str(e.value)


def test_moment_storage_option():
    """Moment storage: 10 FP32 planes per case; D3Q27 regularized,
    schedule 0 only, any z walls, with or without a particle."""
    from paper_2408_15115_amd import turret as T
    case = W.make_case(24, 20, 40, 0.6, W.BC_PERIODIC, W.BC_PERIODIC, 0)
    cells = 24 * 20 * 40
    plane = (cells + 127) // 128 * 128 + 256   # staggered direction planes
    a, b, _ = T.required_bytes([case], None, storage="mom")
    assert a == b == 10 * plane * 4
    T.required_bytes([dict(case, sponge=6)], None, storage="mom")
    bad = [({"collision": 1}, "collision 0"), ({"schedule": 2}, "schedule 0"), ({"lattice": 19}, "FP32")]
    for kw, needle in bad:
        with pytest.raises(T.TurretError) as e:
            T.required_bytes([case], None, **dict({"storage": "mom"}, **kw))
        assert needle in str(e.value)
    T.required_bytes([dict(case, bc_zlo=W.BC_NOSLIP, bc_zhi=W.BC_PRESSURE)], None, storage="mom")
    sc, sb = W.case_sphere48()
    a_mom, _, aux_mom = T.required_bytes([sc], [sb], storage="mom")
    a_pop, _, aux_pop = T.required_bytes([sc], [sb])
    assert a_mom < a_pop / 2 and aux_mom > aux_pop   # the expanded region rides in the auxiliary buffer


def test_moving_wall_checks():
    from paper_2408_15115_amd import turret as T
    case = W.make_case(16, 16, 16, 0.7, W.BC_NOSLIP, W.BC_NOSLIP, 0, u_wall=(-0.05, 0.05))
    T.required_bytes([case], None)
    for bad, needle in ((dict(case, bc_zhi=W.BC_FREESLIP), "no-slip"), (dict(case, u_wall_lo=0.3), "0.2"),
                        (dict(case, u_wall_hi=float("nan")), "finite")):
        with pytest.raises(T.TurretError) as e:
            T.required_bytes([bad], None)
        assert needle in str(e.value)
