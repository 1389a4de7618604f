"""Kernel-level parity on the GPU: every kernel kind and dtype against the FP64 oracle, through
the C ABI (one-kernel DAGs), at shapes that span several tiles and ragged tails."""
import numpy as np
import pytest

import paper_2009_07482_amd as psc
from oracle.bf16 import round_bf16, round_f32
from gpu_helpers import one_kernel_spec, normwise, oracle_outputs, uniform

pytestmark = pytest.mark.gpu

GEMM_SHAPES = [(1, 1, 1), (17, 33, 29), (64, 64, 64), (100, 64, 257), (513, 70, 130), (256, 512, 64),
               (512, 64, 512), (0, 8, 8), (8, 8, 0)]


def _run(spec, inputs, **kw):
    out, _ = psc.run_spec(spec, inputs, **kw)
    return out["C"]


@pytest.mark.parametrize("m,n,k", GEMM_SHAPES)
@pytest.mark.parametrize("tile", list(range(psc.psc_gemm_tile_count())))
def test_gemm_f32(m, n, k, tile):
    print(f"gemm f32 {m}x{n}x{k} tile {tile}", flush=True)
    spec = one_kernel_spec("gemm", [(m, k), (k, n), (m, n)], ["f32"] * 3, alpha=0.5, tile=tile)
    inp = {"A": uniform(1, (m, k)), "B": uniform(2, (k, n))}
    got = _run(spec, inp)
    ref = oracle_outputs(spec, inp)["C"]
    assert got.shape == (m, n)
    if m and n:
        assert normwise(got, ref) < 1e-5


@pytest.mark.parametrize("m,n,k", [(64, 64, 64), (130, 250, 97), (512, 512, 512)])
@pytest.mark.parametrize("tile", [0, 1, 3, 6, 9, 12, 13, 14, 15])
def test_gemm_f32_ternary_exact(m, n, k, tile):
    g = np.random.default_rng(3)
    spec = one_kernel_spec("gemm", [(m, k), (k, n), (m, n)], ["f32"] * 3, tile=tile)
    inp = {"A": g.integers(-1, 2, (m, k)).astype(np.float32), "B": g.integers(-1, 2, (k, n)).astype(np.float32)}
    got = _run(spec, inp)
    np.testing.assert_array_equal(got, oracle_outputs(spec, inp)["C"])


@pytest.mark.parametrize("m,n,k", GEMM_SHAPES + [(1024, 64, 1024), (1024, 1024, 64), (512, 256, 512), (256, 256, 192),
                                   (512, 512, 320), (80, 48, 2112)])
@pytest.mark.parametrize("tile", list(range(psc.psc_gemm_tile_count())))
@pytest.mark.parametrize("cdt", ["f32", "bf16"])
def test_gemm_bf16(m, n, k, tile, cdt):
    print(f"gemm bf16 {m}x{n}x{k} tile {tile} out {cdt}", flush=True)
    spec = one_kernel_spec("gemm", [(m, k), (k, n), (m, n)], ["bf16", "bf16", cdt], alpha=0.125, tile=tile)
    inp = {"A": uniform(4, (m, k)), "B": uniform(5, (k, n))}
    got = _run(spec, inp)
    if not (m and n):
        return
    exact = oracle_outputs(spec, inp)["C"]
    emul = oracle_outputs(spec, inp, emulate=True)["C"]
    assert normwise(got, exact) < 2e-2
    # against the storage-emulating oracle: FP32 accumulation and at most one output rounding
    assert normwise(got, emul) < (5e-3 if cdt == "bf16" else 1e-5)


@pytest.mark.parametrize("tile", [0, 12, 16, 17, 18, 19])
def test_gemm_bf16_ternary_exact(tile):
    # integer products and sums below 2^8 in magnitude are exact in bf16 storage and fp32 sums
    g = np.random.default_rng(6)
    m, n, k = 96, 160, 200
    spec = one_kernel_spec("gemm", [(m, k), (k, n), (m, n)], ["bf16", "bf16", "f32"], tile=tile)
    inp = {"A": g.integers(-1, 2, (m, k)).astype(np.float32), "B": g.integers(-1, 2, (k, n)).astype(np.float32)}
    np.testing.assert_array_equal(_run(spec, inp), oracle_outputs(spec, inp)["C"])


@pytest.mark.parametrize("tile", [16, 20, 21])
@pytest.mark.parametrize("m,n,k", [(256, 256, 64), (512, 768, 448), (768, 512, 1024)])
def test_gemm_bf16_whole_tile_exact(tile, m, n, k):
    # the 256 x 256 tiles run only on whole tiles: check that the launch kept the tile, and that
    # every element is exact (integer operands, sums below 2^8 in magnitude)
    g = np.random.default_rng(8)
    spec = one_kernel_spec("gemm", [(m, k), (k, n), (m, n)], ["bf16", "bf16", "f32"], tile=tile)
    inp = {"A": g.integers(-1, 2, (m, k)).astype(np.float32), "B": g.integers(-1, 2, (k, n)).astype(np.float32)}
    runner = psc.SpecRunner(spec, "coarse")
    try:
        psc.psc_sched_prepare(runner.sched)
        assert psc.psc_sched_kernel_tile(runner.sched, 0) == tile
    finally:
        runner.close()
    np.testing.assert_array_equal(_run(spec, inp), oracle_outputs(spec, inp)["C"])


@pytest.mark.parametrize("r,c", [(1, 1), (64, 64), (512, 64), (64, 512), (130, 257), (1024, 64), (0, 5),
                                 (136, 264), (72, 200), (8, 4104), (256, 384), (200, 136)])
@pytest.mark.parametrize("dt", ["f32", "bf16"])
@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4])
def test_transpose_exact(r, c, dt, tile):
    spec = one_kernel_spec("transpose", [(r, c), (c, r)], [dt, dt], tile=tile)
    a = uniform(7, (r, c))
    got = _run(spec, {"A": a})
    want = round_bf16(a.T) if dt == "bf16" else a.T.astype(np.float64)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("r,c", [(1, 1), (4, 256), (512, 512), (1024, 1024), (37, 2048), (3, 2500), (77, 1000),
                                 (5, 3), (6, 300), (9, 1996)])
@pytest.mark.parametrize("idt,odt", [("f32", "f32"), ("f32", "bf16"), ("bf16", "bf16"), ("bf16", "f32")])
def test_softmax(r, c, idt, odt):
    print(f"softmax {r}x{c} {idt}->{odt}", flush=True)
    spec = one_kernel_spec("softmax", [(r, c), (r, c)], [idt, odt])
    x = (np.random.default_rng(8).standard_normal((r, c)) * 3).astype(np.float32)
    got = _run(spec, {"A": x})
    exact = oracle_outputs(spec, {"A": x})["C"]
    emul = oracle_outputs(spec, {"A": x}, emulate=True)["C"]
    # the emulating oracle rounds the BF16 input as the host does and the output to its dtype;
    # what remains is FP32 exponentials and sums (~1e-7) and, for BF16 output, the rare rounding
    # decision they flip
    assert normwise(got, emul) < (1e-5 if odt == "f32" else 1e-3)
    if idt == "f32":
        assert normwise(got, exact) < (1e-5 if odt == "f32" else 2e-2)
    np.testing.assert_allclose(got.astype(np.float64).sum(axis=1), 1.0, atol=1e-5 if odt == "f32" else 1e-2 * max(1, c / 512))


def test_softmax_shift_invariance_and_constant_rows():
    spec = one_kernel_spec("softmax", [(8, 300), (8, 300)], ["f32", "f32"])
    x = np.zeros((8, 300), np.float32)
    np.testing.assert_allclose(_run(spec, {"A": x}), np.full((8, 300), 1 / 300), rtol=1e-6)
    x = uniform(9, (8, 300), -5, 5)
    np.testing.assert_allclose(_run(spec, {"A": x + 64.0}), _run(spec, {"A": x}), rtol=2e-5, atol=1e-8)
    x = np.zeros((2, 300), np.float32)
    x[:, 7] = 200.0
    spec = one_kernel_spec("softmax", [(2, 300), (2, 300)], ["f32", "f32"])
    want = np.zeros((2, 300))
    want[:, 7] = 1.0
    np.testing.assert_array_equal(_run(spec, {"A": x}), want)


@pytest.mark.parametrize("r,c", [(1, 1), (256, 256), (129, 1000), (0, 3), (3, 2056), (7, 4104)])
@pytest.mark.parametrize("idt,odt", [("f32", "f32"), ("bf16", "bf16"), ("bf16", "f32"), ("f32", "bf16")])
def test_add_exact(r, c, idt, odt):
    spec = one_kernel_spec("add", [(r, c), (r, c), (r, c)], [idt, idt, odt])
    a, b = uniform(10, (r, c)), uniform(11, (r, c))
    got = _run(spec, {"A": a, "B": b})
    if idt == "bf16":
        a, b = round_bf16(a), round_bf16(b)
    s = a.astype(np.float64) + b.astype(np.float64)
    want = round_bf16(round_f32(s)) if odt == "bf16" else round_f32(s)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_add_and_transpose_on_column_windows(dt):
    """Kernels on views: aligned leading dimension, ragged width (the vector kernels' tail path)."""
    R, W, C = 5, 1008, 1001
    bufs = [{"name": "A", "dtype": dt, "rows": R, "cols": W, "view_of": None, "row_off": 0, "col_off": 0},
            {"name": "B", "dtype": dt, "rows": R, "cols": W, "view_of": None, "row_off": 0, "col_off": 0},
            {"name": "Cr", "dtype": dt, "rows": R, "cols": W, "view_of": None, "row_off": 0, "col_off": 0},
            {"name": "Av", "dtype": dt, "rows": R, "cols": C, "view_of": "A", "row_off": 0, "col_off": 0},
            {"name": "Bv", "dtype": dt, "rows": R, "cols": C, "view_of": "B", "row_off": 0, "col_off": 0},
            {"name": "Cv", "dtype": dt, "rows": R, "cols": C, "view_of": "Cr", "row_off": 0, "col_off": 0},
            {"name": "T", "dtype": dt, "rows": C, "cols": R, "view_of": None, "row_off": 0, "col_off": 0}]
    kers = [{"name": "add", "kind": "add", "inputs": ["Av", "Bv"], "outputs": ["Cv"], "alpha": 1.0, "tile": 0},
            {"name": "tr", "kind": "transpose", "inputs": ["Av"], "outputs": ["T"], "alpha": 1.0, "tile": 0}]
    spec = {"buffers": bufs, "kernels": kers, "edges": [], "component": [0, 0]}
    a, b = uniform(12, (R, W)), uniform(13, (R, W))
    out, _ = psc.run_spec(spec, {"A": a, "B": b})
    if dt == "bf16":
        a, b = round_bf16(a), round_bf16(b)
    s_ = a[:, :C].astype(np.float64) + b[:, :C].astype(np.float64)
    want = round_bf16(round_f32(s_)) if dt == "bf16" else round_f32(s_)
    np.testing.assert_array_equal(out["Cv"], want)
    np.testing.assert_array_equal(out["T"], a[:, :C].T.astype(np.float64))


# Outputs of 256 MiB and more take the streaming (non-temporal) variants; ragged edges on both axes.
@pytest.mark.parametrize("dt,r,c", [("f32", 8200, 8216), ("bf16", 10000, 13432)])
@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4])
def test_transpose_large_streaming(dt, r, c, tile):
    print(f"transpose {r}x{c} {dt} tile {tile}", flush=True)
    spec = one_kernel_spec("transpose", [(r, c), (c, r)], [dt, dt], tile=tile)
    a = uniform(14, (r, c))
    got = _run(spec, {"A": a})
    want = round_bf16(a.T) if dt == "bf16" else a.T.astype(np.float64)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("idt,odt,r,c", [("f32", "f32", 8200, 8200), ("bf16", "bf16", 8200, 16400)])
def test_add_large_streaming(idt, odt, r, c):
    spec = one_kernel_spec("add", [(r, c), (r, c), (r, c)], [idt, idt, odt])
    a, b = uniform(15, (r, c)), uniform(16, (r, c))
    got = _run(spec, {"A": a, "B": b})
    if idt == "bf16":
        a, b = round_bf16(a), round_bf16(b)
    s = a.astype(np.float64) + b.astype(np.float64)
    want = round_bf16(round_f32(s)) if odt == "bf16" else round_f32(s)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("idt,odt,r,c", [("f32", "f32", 65600, 1024), ("f32", "bf16", 65560, 2048),
                                           ("bf16", "bf16", 65540, 2048)])
def test_softmax_large_streaming(idt, odt, r, c):
    print(f"softmax {r}x{c} {idt}->{odt}", flush=True)
    spec = one_kernel_spec("softmax", [(r, c), (r, c)], [idt, odt])
    x = (np.random.default_rng(17).standard_normal((r, c)) * 3).astype(np.float32)
    got = _run(spec, {"A": x})
    exact = oracle_outputs(spec, {"A": x})["C"]
    assert normwise(got, exact) < (1e-5 if (idt, odt) == ("f32", "f32") else 2e-2)
