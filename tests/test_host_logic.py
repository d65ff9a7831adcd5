"""Host-side logic without a GPU: layout helpers, the byte counts the
benchmark reports, the seeded input generators and the tuner's candidates."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_aligned_stride():
    from paper_1111_1129_amd.lattice import ROW_ALIGN, aligned_stride
    for n in (1, 63, 64, 65, 17263, 7797209):
        s = aligned_stride(n)
        assert s >= n and s % ROW_ALIGN == 0 and s - n < ROW_ALIGN
    # 128-byte rows for the narrowest storage (FP16)
    assert ROW_ALIGN * 2 % 128 == 0


def test_candidate_strides_are_aligned_and_large_enough():
    from paper_1111_1129_amd.tune import candidate_strides
    for n in (17263, 148691, 7797209, 107371203):
        c = candidate_strides(n)
        assert c == sorted(c) and len(c) == len(set(c))
        assert all(s >= n and s % 64 == 0 for s in c)
        assert all(19 * s < 2 ** 32 for s in c)


def test_sweep_byte_counts():
    """Per-update algorithmic bytes: 19 loads + 19 stores of a PDF plus the
    adjacency (18 uint32, or 18 int16 codes + one 80-byte record per 256
    cells; every other step in place)."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.sweep_bytes("f64", "full") == 376
    assert bench.sweep_bytes("f32s", "full") == 224
    assert bench.sweep_bytes("f16s", "full") == 148
    assert bench.sweep_bytes("f64", "c16") == pytest.approx(304 + 36 + 80 / 256)
    assert bench.sweep_bytes("f64", "inplace") == pytest.approx(304 + 36)
    assert bench.sweep_bytes("f16s", "inplace_c16") == pytest.approx(76 + (36 + 80 / 256) / 2)
    # 8-bit codes: by the shares of cells in narrow tiles and in tiles with escapes
    assert bench.sweep_bytes("f64", "c8", 1.0, 0.0) == pytest.approx(304 + 18 + 80 / 256)
    assert bench.sweep_bytes("f64", "c8", 0.9, 0.0) == pytest.approx(304 + 0.9 * 18 + 0.1 * 36
                                                                     + 80 / 256)
    assert bench.sweep_bytes("f64", "c8", 0.0, 1.0) == pytest.approx(304 + 72 + 80 / 256)
    assert bench.sweep_bytes("f64", "c16", 0.0, 0.25) == pytest.approx(304 + 0.75 * 36 + 18
                                                                      + 80 / 256)
    assert bench.sweep_bytes("f64", "c8") == bench.sweep_bytes("f64", "c16")
    for kind in bench.SWEEP_KERNELS:
        assert bench.sweep_bytes("f64", kind) > bench.sweep_bytes("f32", kind) > \
            bench.sweep_bytes("f16s", kind)


def test_bench_refuses_more_than_one_gpu():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in json.loads(res.stdout.strip().splitlines()[-1])["error"]


def test_input_generators_are_seeded_and_sized():
    from paper_1111_1129_amd import inputs as I
    a = I.packing_small(1)
    b = I.packing_small(1)
    assert np.array_equal(a.flags, b.flags)
    assert int(a.flags.sum()) == 17263            # the recorded count of this seed
    assert not np.array_equal(a.flags, I.packing_small(2).flags)
    ch = I.channel(100)
    assert ch.flags.shape == (100, 100, 500) and int(ch.flags.sum()) == 500 * 98 * 98
    r = I.random_flags(3, 5, 6, 7, 0.5)
    assert r.flags.shape == (7, 6, 5) and r.flags.dtype == np.uint8


def test_crop_sample_keeps_aspect_and_fraction():
    torch = pytest.importorskip("torch")
    from paper_1111_1129_amd.tune import crop_sample
    f = torch.zeros((64, 32, 128), dtype=torch.uint8)
    c = crop_sample(f, 0.125)
    assert tuple(c.shape) == (32, 16, 64)
    assert c.is_contiguous()


def test_device_build_flags_fix_the_rounding():
    """Device code is built without floating-point contraction (every sweep
    variant then rounds each product and sum on its own, the basis of their
    bitwise equality) and without packed FP32 instructions; the profile hash
    covers these flags."""
    import importlib
    build = importlib.import_module("paper_1111_1129_amd.build")
    flags = build.compile_flags()
    assert "-ffp-contract=off" in flags
    assert not any(f.startswith("-ffp-contract=") and f != "-ffp-contract=off" for f in flags)
    i = flags.index("-packed-fp32-ops")
    assert flags[i - 3:i] == ["-Xclang", "-target-feature", "-Xclang"]
    assert not any("fast-math" in f or f.startswith("-Ofast") for f in flags)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    h = bench.kernel_source_hash("c8")
    orig = build.compile_flags
    try:
        build.compile_flags = lambda: [f.replace("=off", "=on") for f in orig()]
        assert bench.kernel_source_hash("c8") != h
    finally:
        build.compile_flags = orig
    assert bench.kernel_source_hash("c8") == h
