"""The C-ABI library loads, exports every entry point include/lbm.h declares,
and rejects bad arguments on the host (CPU only: no kernel is launched)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")
LIB = os.path.join(ROOT, "paper_1111_1129_amd", "liblbm.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("liblbm.so is not built: run python -m paper_1111_1129_amd.build")
    return C.CDLL(LIB)


def test_header_declares_the_five_calls():
    names = declared_functions()
    for fn in ("lbm_build_adjacency", "lbm_init", "lbm_step", "lbm_step_adjoint", "lbm_moments"):
        assert fn in names


def test_every_declared_symbol_is_exported(lib):
    for fn in declared_functions():
        assert hasattr(lib, fn), fn


def test_version_and_status_strings(lib):
    lib.lbm_version.restype = C.c_int32
    assert lib.lbm_version() >= 10000
    lib.lbm_status_string.restype = C.c_char_p
    lib.lbm_status_string.argtypes = [C.c_int32]
    for s in range(0, -8, -1):
        assert lib.lbm_status_string(s) not in (None, b"unknown status")
    assert lib.lbm_status_string(-99) == b"unknown status"


def test_struct_layouts():
    from paper_1111_1129_amd import _native as N
    assert C.sizeof(N.lbm_geom) == 24
    assert C.sizeof(N.lbm_params) == 48
    assert C.sizeof(N.lbm_segment) == 24


def test_host_side_argument_errors(lib):
    """Validation happens before any launch, so these run without a GPU."""
    from paper_1111_1129_amd import _native as N
    P = C.c_void_p
    nf = C.c_int64(0)
    ws = C.c_size_t(0)
    lib.lbm_build_adjacency.restype = C.c_int32
    lib.lbm_build_adjacency.argtypes = [C.POINTER(N.lbm_geom), P, C.c_int64, C.c_int64, P, P, P,
                                        C.c_int64, C.POINTER(C.c_int64), P,
                                        C.POINTER(C.c_size_t), P]
    g = N.lbm_geom(0, 4, 4, 0, 0, 0)
    assert lib.lbm_build_adjacency(C.byref(g), None, 0, 0, None, None, None, 0, C.byref(nf),
                                   None, C.byref(ws), None) == N.LBM_EINVAL
    g = N.lbm_geom(4, 4, 4, 0, 7, 0)  # unknown ordering
    assert lib.lbm_build_adjacency(C.byref(g), None, 0, 0, None, None, None, 0, C.byref(nf),
                                   None, C.byref(ws), None) == N.LBM_EINVAL
    g = N.lbm_geom(4, 4, 4, 0, 1, 0)  # blocking factor 0
    assert lib.lbm_build_adjacency(C.byref(g), None, 0, 0, None, None, None, 0, C.byref(nf),
                                   None, C.byref(ws), None) == N.LBM_EINVAL
    g = N.lbm_geom(2048, 1024, 1024, 0, 0, 0)  # 2^31 cells: the paper's 2^31 limit
    assert lib.lbm_build_adjacency(C.byref(g), None, 0, 0, None, None, None, 0, C.byref(nf),
                                   None, C.byref(ws), None) == N.LBM_EOVERFLOW
    # workspace size query touches nothing on the device
    g = N.lbm_geom(32, 32, 32, 1, 2, 0)
    ws = C.c_size_t(0)
    assert lib.lbm_build_adjacency(C.byref(g), None, 0, 0, None, None, None, 0, C.byref(nf),
                                   None, C.byref(ws), None) == N.LBM_OK
    assert ws.value >= 32 ** 3 * 4

    lib.lbm_step.restype = C.c_int32
    lib.lbm_step.argtypes = [C.POINTER(N.lbm_params), C.c_int32, P, C.c_int32, C.c_int64,
                             C.c_int64, P, P, P, P, C.c_int32, C.c_int32, P,
                             C.POINTER(C.c_size_t), P]
    dummy = P(4096)
    good = N.make_params(0.8, 3 / 16, (1e-6, 0, 0), "f64")
    zero = C.c_size_t(0)

    def step(p, n=10, stride=10, n_params=1, a=dummy, b=P(8192)):
        return lib.lbm_step(C.byref(p), n_params, None, 0, n, stride, dummy, None, a, b, 1, 0, None,
                            C.byref(zero), None)

    assert step(N.make_params(0.5, 3 / 16)) == N.LBM_EINVAL          # tau+ = 1/2
    assert step(N.make_params(0.8, 0.0)) == N.LBM_EINVAL             # tau- = 1/2
    assert step(N.make_params(0.8, 3 / 16, (float("nan"), 0, 0))) == N.LBM_EINVAL
    assert step(N.make_params(0.8, 3 / 16, storage=9)) == N.LBM_EINVAL
    assert step(N.make_params(0.8, 3 / 16, flags=3 << 8)) == N.LBM_EINVAL  # chunk not 2^k
    assert step(N.make_params(0.8, 3 / 16, flags=1 << 20)) == N.LBM_EINVAL  # unknown flag bit
    assert step(good, n=10, stride=5) == N.LBM_EINVAL                # stride < n
    assert step(good, n_params=0) == N.LBM_EINVAL
    assert step(good, a=dummy, b=dummy) == N.LBM_EINVAL              # in-place not allowed
    assert step(good, n=10, stride=(1 << 32) // 19 + 1) == N.LBM_EOVERFLOW
    # strides whose product with 19 would overflow int64 are refused, not wrapped
    for big in ((1 << 63) - 1, (1 << 63) // 2, (1 << 63) // 19 + 1):
        assert step(good, n=10, stride=big) == N.LBM_EOVERFLOW
        g = N.lbm_geom(4, 4, 4, 0, 0, 0)
        ws = C.c_size_t(1 << 20)
        assert lib.lbm_build_adjacency(C.byref(g), P(4096), 0, big, None, P(4096), P(4096), 64,
                                       C.byref(nf), P(4096), C.byref(ws), None) == N.LBM_EOVERFLOW
    # persistent size query
    ws = C.c_size_t(0)
    assert lib.lbm_step(C.byref(good), 1, None, 0, 10, 10, dummy, None, dummy, P(8192), 5, 1,
                        None, C.byref(ws), None) == N.LBM_OK and ws.value > 0
    # bad segments: overlapping / outside [0, n)
    segs = (N.lbm_segment * 2)(N.lbm_segment(0, 6, 0, 0), N.lbm_segment(5, 5, 0, 0))
    assert lib.lbm_step(C.byref(good), 1, C.cast(segs, P), 2, 10, 10, dummy, None, dummy,
                        P(8192), 1, 0, None, C.byref(zero), None) == N.LBM_EINVAL

    lib.lbm_step_adjoint.restype = C.c_int32
    lib.lbm_step_adjoint.argtypes = [C.POINTER(N.lbm_params), C.c_int64, C.c_int64, P, P, P, P,
                                     P, P, P]
    f32 = N.make_params(0.8, 3 / 16, storage="f32")
    assert lib.lbm_step_adjoint(C.byref(f32), 10, 10, dummy, dummy, None, dummy, dummy, None,
                                None) == N.LBM_EINVAL


def test_compressed_adjacency_argument_errors(lib):
    from paper_1111_1129_amd import _native as N
    P = C.c_void_p
    lib.lbm_compress_adjacency.restype = C.c_int32
    lib.lbm_compress_adjacency.argtypes = [C.c_int64, C.c_int64, P, P, P, C.POINTER(C.c_int64),
                                           P, C.POINTER(C.c_size_t), P]
    esc = C.c_int64(0)
    ws = C.c_size_t(0)
    assert lib.lbm_compress_adjacency(10, 10, None, None, None, C.byref(esc), None, C.byref(ws),
                                      None) == N.LBM_OK and ws.value == 8 * 257  # partial sums
    assert lib.lbm_compress_adjacency(10, 10, None, None, None, C.byref(esc), None, None,
                                      None) == N.LBM_EINVAL
    small = C.c_size_t(8)
    assert lib.lbm_compress_adjacency(10, 10, P(4096), P(4096), P(4096), C.byref(esc), P(4096),
                                      C.byref(small), None) == N.LBM_EWORKSPACE
    ok = C.c_size_t(ws.value)
    assert lib.lbm_compress_adjacency(10, 5, P(4096), P(4096), P(4096), C.byref(esc), P(4096),
                                      C.byref(ok), None) == N.LBM_EINVAL       # stride < n
    assert lib.lbm_compress_adjacency(0, 5, P(4096), P(4096), P(4096), C.byref(esc), P(4096),
                                      C.byref(ok), None) == N.LBM_EINVAL       # empty list
    assert lib.lbm_compress_adjacency(10, 10, None, P(4096), P(4096), C.byref(esc), P(4096),
                                      C.byref(ok), None) == N.LBM_EINVAL

    lib.lbm_step_c16.restype = C.c_int32
    lib.lbm_step_c16.argtypes = [C.POINTER(N.lbm_params), C.c_int64, C.c_int64, P, P, P, P, P, P,
                                 C.c_int32, P]
    good = N.make_params(0.8, 3 / 16, (1e-6, 0, 0), "f64")
    d = P(4096)

    def step(p=good, n=10, stride=10, codes=d, a=d, b=P(8192), steps=1):
        return lib.lbm_step_c16(C.byref(p), n, stride, codes, d, d, None, a, b, steps, None)

    assert step(p=N.make_params(0.5, 3 / 16)) == N.LBM_EINVAL
    assert step(codes=None) == N.LBM_EINVAL
    assert step(b=d) == N.LBM_EINVAL                   # in place
    assert step(stride=5) == N.LBM_EINVAL
    assert step(steps=-1) == N.LBM_EINVAL
    assert step(stride=(1 << 32) // 19 + 1) == N.LBM_EOVERFLOW
    assert step(steps=0) == N.LBM_OK                  # nothing to do, nothing launched


def test_inplace_argument_errors(lib):
    from paper_1111_1129_amd import _native as N
    P = C.c_void_p
    lib.lbm_step_inplace.restype = C.c_int32
    lib.lbm_step_inplace.argtypes = [C.POINTER(N.lbm_params), C.c_int64, C.c_int64, P, P, P, P,
                                     P, C.c_int32, C.c_int32, P]
    good = N.make_params(0.8, 3 / 16, (1e-6, 0, 0), "f64")
    d = P(4096)

    def step(p=good, n=10, stride=10, adj=d, codes=None, recs=None, f=d, phase=0, steps=1):
        return lib.lbm_step_inplace(C.byref(p), n, stride, adj, codes, recs, None, f, phase,
                                    steps, None)

    assert step(p=N.make_params(0.8, 0.0)) == N.LBM_EINVAL
    assert step(adj=None) == N.LBM_EINVAL
    assert step(f=None) == N.LBM_EINVAL
    assert step(phase=2) == N.LBM_EINVAL
    assert step(codes=d) == N.LBM_EINVAL          # codes without their tile records
    assert step(recs=d) == N.LBM_EINVAL
    assert step(stride=9) == N.LBM_EINVAL
    assert step(steps=-2) == N.LBM_EINVAL
    assert step(stride=(1 << 32) // 19 + 1) == N.LBM_EOVERFLOW
    assert step(steps=0) == N.LBM_OK


C_CLIENT = r"""
#include <stdio.h>
#include <string.h>
#include "lbm.h"

int main(void) {
    size_t ws = 0;
    int64_t esc = 0;
    lbm_params p;
    memset(&p, 0, sizeof p);
    p.tau_plus = 0.8;
    p.magic = 3.0 / 16.0;
    p.storage = LBM_F64;
    if (lbm_version() < 10000) return 1;
    if (strcmp(lbm_status_string(LBM_OK), "unknown status") == 0) return 2;
    if (lbm_compress_adjacency(10, 10, NULL, NULL, NULL, &esc, NULL, &ws, NULL) != LBM_OK) return 3;
    if (ws != 8 * 257) return 4;
    p.tau_plus = 0.5; /* tau+ = 1/2 is rejected on the host */
    if (lbm_step_inplace(&p, 10, 10, (const uint32_t*)0x1000, NULL, NULL, NULL, (void*)0x2000, 0, 1,
                         NULL) != LBM_EINVAL) return 5;
    printf("c client ok %d\n", lbm_version());
    return 0;
}
"""


def test_c_client_compiles_links_and_runs(tmp_path):
    """The header is plain C and the library's host-side entry points work
    from a C program (no GPU call is made)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "client.c"
    src.write_text(C_CLIENT)
    exe = tmp_path / "client"
    libdir = os.path.dirname(LIB)
    res = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", f"-I{os.path.dirname(HEADER)}",
                          str(src), "-o", str(exe), f"-L{libdir}", "-llbm",
                          f"-Wl,-rpath,{libdir}", "-Wl,-rpath,/opt/rocm/lib"],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert run.returncode == 0, (run.returncode, run.stdout, run.stderr)
    assert "c client ok" in run.stdout


def test_adjoint_c16_argument_errors(lib):
    from paper_1111_1129_amd import _native as N
    P = C.c_void_p
    lib.lbm_step_adjoint_c16.restype = C.c_int32
    lib.lbm_step_adjoint_c16.argtypes = [C.POINTER(N.lbm_params), C.c_int64, C.c_int64, P, P, P,
                                         P, P, P, P, P, P]
    f64 = N.make_params(0.8, 3 / 16, storage="f64s")
    d = P(4096)

    def call(p=f64, n=10, stride=10, codes=d, recs=d, lam_next=d):
        return lib.lbm_step_adjoint_c16(C.byref(p), n, stride, codes, recs, d, d, None, lam_next,
                                        d, None, None)

    assert call(p=N.make_params(0.8, 3 / 16, storage="f32")) == N.LBM_EINVAL   # FP64 only
    assert call(codes=None) == N.LBM_EINVAL
    assert call(recs=None) == N.LBM_EINVAL
    assert call(lam_next=None) == N.LBM_EINVAL          # no seed through this entry
    assert call(n=0) == N.LBM_EINVAL
    assert call(stride=9) == N.LBM_EINVAL
    assert call(stride=(1 << 32) // 19 + 1) == N.LBM_EOVERFLOW


def test_adjoint_c8_argument_errors(lib):
    from paper_1111_1129_amd import _native as N
    P = C.c_void_p
    lib.lbm_step_adjoint_c8.restype = C.c_int32
    lib.lbm_step_adjoint_c8.argtypes = [C.POINTER(N.lbm_params), C.c_int64, C.c_int64, P, P, P,
                                        P, P, P, P, P, P, P]
    f64 = N.make_params(0.8, 3 / 16, storage="f64s")
    d = P(4096)

    def call(p=f64, n=10, stride=10, codes8=d, codes=d, recs=d, lam_next=d):
        return lib.lbm_step_adjoint_c8(C.byref(p), n, stride, codes8, codes, recs, d, d, None,
                                       lam_next, d, None, None)

    assert call(p=N.make_params(0.8, 3 / 16, storage="f16s")) == N.LBM_EINVAL  # FP64 only
    assert call(codes8=None) == N.LBM_EINVAL
    assert call(codes=None) == N.LBM_EINVAL
    assert call(recs=None) == N.LBM_EINVAL
    assert call(lam_next=None) == N.LBM_EINVAL          # no seed through this entry
    assert call(n=0) == N.LBM_EINVAL
    assert call(stride=9) == N.LBM_EINVAL
    assert call(stride=(1 << 32) // 19 + 1) == N.LBM_EOVERFLOW


def test_c8_argument_errors(lib):
    from paper_1111_1129_amd import _native as N
    P = C.c_void_p
    lib.lbm_step_c8.restype = C.c_int32
    lib.lbm_step_c8.argtypes = [C.POINTER(N.lbm_params), C.c_int64, C.c_int64, P, P, P, P, P, P,
                                P, C.c_int32, P]
    prm = N.make_params(0.8, 3 / 16)
    d, e = P(4096), P(8192)

    def step(c8=d, c16=d, recs=d, fa=d, fb=e, n=10, stride=10, steps=1):
        return lib.lbm_step_c8(C.byref(prm), n, stride, c8, c16, recs, d, None, fa, fb, steps,
                               None)

    assert step(c8=None) == N.LBM_EINVAL
    assert step(c16=None) == N.LBM_EINVAL
    assert step(recs=None) == N.LBM_EINVAL
    assert step(fb=d) == N.LBM_EINVAL                  # in place is not allowed here
    assert step(steps=-1) == N.LBM_EINVAL
    assert step(stride=9) == N.LBM_EINVAL
    assert step(n=0, stride=0) == N.LBM_OK             # nothing to do, no launch
    lib.lbm_narrow_codes.restype = C.c_int32
    lib.lbm_narrow_codes.argtypes = [C.c_int64, C.c_int64, P, P, P, C.POINTER(C.c_int64), P,
                                     C.POINTER(C.c_size_t), P]
    ws = C.c_size_t(0)
    cnt = C.c_int64(0)
    assert lib.lbm_narrow_codes(10, 10, d, d, d, C.byref(cnt), None, C.byref(ws), None) == N.LBM_OK
    assert ws.value == 8 * 257
    small = C.c_size_t(8)
    assert lib.lbm_narrow_codes(10, 10, d, d, d, C.byref(cnt), d, C.byref(small),
                                None) == N.LBM_EWORKSPACE
    assert lib.lbm_narrow_codes(10, 10, None, d, d, C.byref(cnt), d, C.byref(ws),
                                None) == N.LBM_EINVAL
    assert lib.lbm_narrow_codes(0, 0, d, d, d, C.byref(cnt), d, C.byref(ws), None) == N.LBM_EINVAL


def test_inplace_c8_argument_errors(lib):
    from paper_1111_1129_amd import _native as N
    P = C.c_void_p
    lib.lbm_step_inplace_c8.restype = C.c_int32
    lib.lbm_step_inplace_c8.argtypes = [C.POINTER(N.lbm_params), C.c_int64, C.c_int64, P, P, P,
                                        P, P, P, C.c_int32, C.c_int32, P]
    prm = N.make_params(0.8, 3 / 16)
    d = P(4096)

    def step(adj=d, c8=d, c16=d, recs=d, f=d, phase=0, steps=1, n=10, stride=10):
        return lib.lbm_step_inplace_c8(C.byref(prm), n, stride, adj, c8, c16, recs, None, f,
                                       phase, steps, None)

    for kw in ({"adj": None}, {"c8": None}, {"c16": None}, {"recs": None}, {"f": None},
               {"phase": 2}, {"steps": -1}, {"stride": 9}):
        assert step(**kw) == N.LBM_EINVAL, kw
    assert step(steps=0) == N.LBM_OK  # nothing to do, no launch


def test_parameter_set_and_batch_argument_errors(lib):
    """Per-segment parameter sets (lbm_step, lbm_step_batch, lbm_moments,
    lbm_objective): every rule is checked on the host before any launch."""
    from paper_1111_1129_amd import _native as N
    P, I32, I64, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    lib.lbm_step.restype = I32
    lib.lbm_step.argtypes = [C.POINTER(N.lbm_params), I32, P, I32, I64, I64, P, P, P, P, I32, I32,
                             P, C.POINTER(SZ), P]
    lib.lbm_step_batch.restype = I32
    lib.lbm_step_batch.argtypes = [C.POINTER(N.lbm_params), I32, P, I32, I64, I64, P, P, P, P, P,
                                   P, P, I32, I32, P, C.POINTER(SZ), P]
    lib.lbm_moments.restype = I32
    lib.lbm_moments.argtypes = [C.POINTER(N.lbm_params), I32, I64, I64, P, P, P, P, P, I32, P, P,
                                C.POINTER(SZ), P]
    lib.lbm_objective.restype = I32
    lib.lbm_objective.argtypes = [C.POINTER(N.lbm_params), I32, I64, I64, P, P, P, I32, P, P,
                                  C.POINTER(SZ), P]
    d, e = P(4096), P(8192)
    good = N.make_params(0.8, 3 / 16, (1e-6, 0, 0), "f32")

    def params(*ps):
        arr = (N.lbm_params * len(ps))(*ps)
        return C.cast(arr, C.POINTER(N.lbm_params)), arr

    def segs(*ts):
        return C.cast((N.lbm_segment * len(ts))(*[N.lbm_segment(*t, 0) for t in ts]), P)

    two, _keep = params(good, N.make_params(0.9, 3 / 16, (2e-6, 0, 0), "f32"))
    ws = C.c_size_t(1 << 20)

    def step(p=two, n_params=2, sg=None, n_seg=0, n=1000, stride=1024, persistent=0,
             workspace=d, wsb=ws):
        return lib.lbm_step(p, n_params, sg, n_seg, n, stride, d, None, d, e, 1, persistent,
                            workspace, C.byref(wsb), None)

    # size query: a segment selecting set 1 needs the table
    q = C.c_size_t(0)
    assert step(sg=segs((0, 300, 0), (512, 400, 1)), n_seg=2, workspace=None, wsb=q) == N.LBM_OK
    assert q.value >= 256 + 2 * 96 + 4 * 4
    # a set index outside [0, n_params)
    assert step(sg=segs((0, 300, 0), (512, 400, 2)), n_seg=2) == N.LBM_EINVAL
    assert step(sg=segs((0, 300, -1)), n_seg=1) == N.LBM_EINVAL
    # sets differ and a segment does not start on a 256-cell tile
    assert step(sg=segs((0, 300, 0), (300, 400, 1)), n_seg=2) == N.LBM_EINVAL
    assert step(sg=segs((0, 300, 1), (400, 400, 0)), n_seg=2) == N.LBM_EINVAL
    # out of order / overlapping / past n
    assert step(sg=segs((512, 100, 1), (0, 100, 0)), n_seg=2) == N.LBM_EINVAL
    assert step(sg=segs((0, 600, 0), (512, 100, 1)), n_seg=2) == N.LBM_EINVAL
    assert step(sg=segs((768, 300, 1)), n_seg=1) == N.LBM_EINVAL
    # workspace smaller than the query
    small = C.c_size_t(q.value - 1)
    assert step(sg=segs((0, 300, 0), (512, 400, 1)), n_seg=2, wsb=small) == N.LBM_EWORKSPACE
    # sets that differ in storage or launch flags
    other, _k2 = params(good, N.make_params(0.9, 3 / 16, (0, 0, 0), "f64"))
    assert step(p=other) == N.LBM_EINVAL
    flagged, _k3 = params(good, N.make_params(0.9, 3 / 16, (0, 0, 0), "f32", flags=1))
    assert step(p=flagged) == N.LBM_EINVAL
    bad, _k4 = params(good, N.make_params(0.5, 3 / 16, (0, 0, 0), "f32"))
    assert step(p=bad) == N.LBM_EINVAL
    assert step(n_params=65537) == N.LBM_EINVAL  # beyond the documented limit (host check only)
    # the finite check is a known flag
    chk, _k5 = params(N.make_params(0.8, 3 / 16, (0, 0, 0), "f32", flags=N.FLAG_CHECK_FINITE))
    assert step(p=chk, n_params=1, n=0, stride=0) == N.LBM_OK

    # lbm_step_batch: codes8 needs codes, codes need tile records
    def batch(c8=None, c16=None, recs=None):
        return lib.lbm_step_batch(two, 2, None, 0, 1000, 1024, c8, c16, recs, d, None, d, e, 1, 0,
                                  d, C.byref(ws), None)
    assert batch(c8=d) == N.LBM_EINVAL
    assert batch(c16=d) == N.LBM_EINVAL
    assert batch(recs=d) == N.LBM_EINVAL
    assert lib.lbm_step_batch(two, 2, None, 0, 0, 0, d, d, d, d, None, d, e, 1, 0, d,
                              C.byref(ws), None) == N.LBM_OK  # nothing to do
    # persistent size query through the batch entry point
    q2 = C.c_size_t(0)
    assert lib.lbm_step_batch(two, 2, None, 0, 1000, 1024, None, None, None, d, None, d, e, 3, 1,
                              None, C.byref(q2), None) == N.LBM_OK and q2.value >= 256

    # lbm_moments / lbm_objective take the sets too
    tot = C.c_size_t(0)
    assert lib.lbm_moments(two, 2, 1000, 1024, d, d, None, None, segs((0, 300, 0), (512, 400, 1)),
                           2, d, None, C.byref(tot), None) == N.LBM_OK and tot.value > 0
    assert lib.lbm_moments(two, 2, 1000, 1024, d, d, None, None, segs((0, 300, 3)), 1, d, None,
                           C.byref(tot), None) == N.LBM_EINVAL
    assert lib.lbm_moments(two, 0, 1000, 1024, d, d, None, None, None, 0, d, None, C.byref(tot),
                           None) == N.LBM_EINVAL
    assert lib.lbm_moments(other, 2, 1000, 1024, d, d, None, None, None, 0, d, d, C.byref(ws),
                           None) == N.LBM_EINVAL  # storages differ
    assert lib.lbm_objective(two, 2, 1000, 1024, d, d, None, 0, None, d, C.byref(ws),
                             None) == N.LBM_EINVAL  # J missing
    assert lib.lbm_objective(two, 2, 1000, 1024, d, d, None, 0, d, None, C.byref(tot),
                             None) == N.LBM_OK and tot.value > 0  # size query



def test_init_argument_errors(lib):
    """lbm_init refuses a non-finite density or initial velocity on the host."""
    from paper_1111_1129_amd import _native as N
    P = C.c_void_p
    lib.lbm_init.restype = C.c_int32
    lib.lbm_init.argtypes = [C.POINTER(N.lbm_params), C.c_int64, C.c_int64, P, C.c_double, P, P]
    p = N.make_params(0.8, 3 / 16, (1e-6, 0, 0), "f64")
    d = P(4096)
    nan_u = (C.c_double * 3)(0.0, float("nan"), 0.0)
    inf_u = (C.c_double * 3)(float("inf"), 0.0, 0.0)
    assert lib.lbm_init(C.byref(p), 10, 10, d, float("nan"), None, None) == N.LBM_EINVAL
    assert lib.lbm_init(C.byref(p), 10, 10, d, 1.0, C.cast(nan_u, P), None) == N.LBM_EINVAL
    assert lib.lbm_init(C.byref(p), 10, 10, d, 1.0, C.cast(inf_u, P), None) == N.LBM_EINVAL
    assert lib.lbm_init(C.byref(p), 10, 10, None, 1.0, None, None) == N.LBM_EINVAL
    assert lib.lbm_init(C.byref(N.make_params(0.8, 3 / 16, storage=9)), 10, 10, d, 1.0, None,
                        None) == N.LBM_EINVAL
    assert lib.lbm_init(C.byref(p), 10, 9, d, 1.0, None, None) == N.LBM_EINVAL  # stride < n


def test_check_adjacency_arguments_and_query(lib):
    from paper_1111_1129_amd import _native as N
    P = C.c_void_p
    res = (C.c_int64 * 2)(7, 7)
    ws = C.c_size_t(0)
    lib.lbm_check_adjacency.restype = C.c_int32
    lib.lbm_check_adjacency.argtypes = [C.c_int64, C.c_int64, C.c_int64, P,
                                        C.POINTER(C.c_int64), P, C.POINTER(C.c_size_t), P]
    assert lib.lbm_check_adjacency(0, 1000, 1024, None, res, None, C.byref(ws), None) == N.LBM_OK
    assert ws.value >= 18 * 1000 * 4 + 16  # the slot counts and two counters
    assert lib.lbm_check_adjacency(-1, 10, 10, None, res, None, C.byref(ws), None) == N.LBM_EINVAL
    assert lib.lbm_check_adjacency(0, -1, 10, None, res, None, C.byref(ws), None) == N.LBM_EINVAL
    assert lib.lbm_check_adjacency(8, 10, 10, None, res, None, C.byref(ws), None) == N.LBM_EINVAL
    assert lib.lbm_check_adjacency(0, 10, (1 << 32) // 19 + 1, None, res, None, C.byref(ws),
                                   None) == N.LBM_EOVERFLOW
    assert lib.lbm_check_adjacency(0, 10, 10, None, res, None, None, None) == N.LBM_EINVAL
    big = C.c_size_t(1 << 20)
    assert lib.lbm_check_adjacency(0, 10, 10, None, res, P(4096), C.byref(big),
                                   None) == N.LBM_EINVAL          # NULL adj
    small = C.c_size_t(8)
    assert lib.lbm_check_adjacency(0, 10, 10, P(4096), res, P(4096), C.byref(small),
                                   None) == N.LBM_EWORKSPACE
    # an empty list needs no launch: valid, nothing counted
    assert lib.lbm_check_adjacency(0, 0, 0, P(4096), res, P(4096), C.byref(big), None) == N.LBM_OK
    assert (res[0], res[1]) == (0, 0)
