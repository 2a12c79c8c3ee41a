"""Pins of the oracle's model of reduced-precision storage (the build's
precision form; the paper has none): each stored population is
w_i + q(s_i (f_i - w_i)) / s_i with s_i = 2^(14 + 2 |xi_i|^2) and q the rounding to
IEEE binary16 or to bfloat16, to nearest with ties to even.

The rounding is checked against numpy's double-to-half conversion and
against torch's float-to-bfloat16 conversion (on values that are exact in
float32, so that conversion rounds once), including ties, subnormals and
overflow; the stored field against the same rounding applied by hand; and
the quantized time step against collide, round, stream done step by step."""
import numpy as np
import pytest

from paper_2408_15115_amd import workloads as W

# storage scale s_i = 2^(14 + 2 |xi_i|^2) of the FP16/BF16 store
SCALE = np.array([2.0 ** (14 + 2 * ((i % 3 - 1) ** 2 + ((i // 3) % 3 - 1) ** 2 + (i // 9 - 1) ** 2)) for i in range(27)])


def test_binary16_rounding_is_numpys(orc):
    rng = np.random.default_rng(0)
    x = rng.standard_normal(20000) * np.exp(rng.uniform(-22.0, 12.0, 20000))
    x = np.concatenate([x, [65504.0, 65519.99, 65520.0, -65520.0, 2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -26,
                            1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11, 0.0, -0.0]])
    ours = np.array([orc.round_format(v, "f16") for v in x])
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(ours, ref)
    # the listed ties round to even
    assert orc.round_format(1 + 2.0 ** -11, "f16") == 1.0
    assert orc.round_format(1 + 3 * 2.0 ** -11, "f16") == 1 + 2.0 ** -9
    assert np.isinf(orc.round_format(65520.0, "f16"))


def test_bfloat16_rounding_is_torchs(orc):
    import torch
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-30.0, 30.0, 20000))).astype(np.float32)
    # exact ties between two bfloat16 neighbours: mantissa bit 16 set, lower bits clear
    t = (rng.integers(1 << 23, 1 << 24, 200) | 1 << 15) & ~0x7FFF
    ties = (t.astype(np.uint32) | (127 << 23)).view(np.float32)
    x = np.concatenate([x, ties]).astype(np.float64)
    ours = np.array([orc.round_format(v, "bf16") for v in x])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).double().numpy()
    assert np.array_equal(ours, ref)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_stored_field_is_the_rounded_scaled_deviation(orc, storage):
    _, w = orc.lattice()
    f = W.random_populations(3, 6, 5, 4, amp=0.05)
    q = orc.quantize(f, storage)
    s = SCALE.reshape(w.shape)
    x = s * (f - w)
    want = w + np.vectorize(lambda v: orc.round_format(v, storage))(x) / s
    assert np.array_equal(q, want)
    # the rest state is exact, and rounding twice changes nothing
    assert np.array_equal(orc.quantize(np.broadcast_to(w, (3, 27)), storage), np.broadcast_to(w, (3, 27)))
    assert np.allclose(orc.quantize(q, storage), q, rtol=0, atol=1e-17)
    # one rounding is within half a unit of the format
    p = 11 if storage == "f16" else 8
    ulp = 2.0 ** (np.floor(np.log2(np.abs(x))) - (p - 1))
    assert np.all(np.abs(s * (q - f)) <= 0.5 * ulp * (1 + 1e-12))


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_quantized_step_is_collide_round_stream(orc, storage):
    n, nz, tau = 10, 12, 0.7
    case = W.make_case(n, n, nz, tau, W.BC_FREESLIP, W.BC_FREESLIP, 0)
    f = orc.quantize(W.random_populations(5, n, n, nz, amp=0.05), storage)
    s = orc.OracleSim(case, None)
    s.set_storage(storage)
    s.set_populations(f)
    s.step(3)
    g = f
    for _ in range(3):
        g = orc.stream_grid(orc.quantize(orc.collide_grid(g, tau), storage), W.BC_FREESLIP, W.BC_FREESLIP)
    assert np.array_equal(s.populations(), g)
    assert np.array_equal(s.post_collision(), orc.quantize(orc.collide_grid(g, tau), storage))


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_full_precision_box_around_the_body(orc, storage):
    """With a box, the cells of the cube floor(r - rb) - 3 .. + edge - 1
    around the body keep the unrounded collision; the others are rounded."""
    n, nz, tau = 20, 28, 0.7
    case = W.make_case(n, n, nz, tau, W.BC_FREESLIP, W.BC_FREESLIP, 0, 2e-5)
    body = W.sphere_fibonacci_body(3.0, 200, 2.0, [n - 2.3, 4.6, 13.2], w0=np.array([0.0, 1e-3, 2e-3]))
    rb, edge = 6.02, (18, 17, 19)          # reaches across the periodic x edge
    s = orc.OracleSim(case, body)
    s.set_storage(storage, (rb, edge))
    s.step(3)
    C = s.post_collision()
    direct = orc.collide_grid(s.populations(), tau, 0, h=s.immersed_force())
    r = s.body_state()["r"]
    lo = np.floor(r - rb).astype(int) - 3
    z, y, x = np.meshgrid(np.arange(nz), np.arange(n), np.arange(n), indexing="ij")
    inside = (((x - lo[0]) % n) < edge[0]) & (((y - lo[1]) % n) < edge[1]) & ((z - lo[2]) >= 0) & ((z - lo[2]) < edge[2])
    assert 0 < inside.sum() < inside.size
    assert np.array_equal(C[inside], direct[inside])
    assert np.array_equal(C[~inside], orc.quantize(direct[~inside], storage))
