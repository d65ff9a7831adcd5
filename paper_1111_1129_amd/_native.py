"""ctypes binding of ``liblbm.so`` (the C ABI declared in include/lbm.h).

Argument marshalling only: every function here forwards to the entry point of
the same name.  Torch tensors are passed as raw device pointers and the
current torch stream as the HIP stream.  torch is imported before the library
is loaded so that the library binds to the same HIP runtime instance as torch.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import torch  # noqa: F401  (loads the HIP runtime the library must share)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ECAPACITY, LBM_EOVERFLOW, LBM_EWORKSPACE, LBM_EHIP, LBM_EBARRIER = \
    0, -1, -2, -3, -4, -5, -6
LBM_ENONFINITE = -7
ORDERS = {"lex": 0, "blocked": 1, "morton1": 2, "morton2": 3, "random": 4, "hilbert": 5}
STORAGES = {"f64": 0, "f64s": 1, "f32": 2, "f32s": 3, "f16s": 4, "f16s12": 5}
STORAGE_DTYPE = {0: torch.float64, 1: torch.float64, 2: torch.float32, 3: torch.float32,
                 4: torch.float16, 5: torch.float16}  # 5 holds 2^12 (f - w) as FP16
F16_SCALE = 4096.0  # factor of the scaled shifted FP16 storage
FLAG_NONTEMPORAL = 1
FLAG_CHECK_FINITE = 2
FLAG_XCD_CHUNK_SHIFT = 8
SEGMENT_ALIGN = 256  # segments with their own parameter sets start on a sweep tile

ENTRY_POINTS = ("lbm_build_adjacency", "lbm_init", "lbm_step", "lbm_step_batch",
                "lbm_step_adjoint", "lbm_moments", "lbm_objective", "lbm_moments_noalloc",
                "lbm_partition_stats", "lbm_compress_adjacency", "lbm_step_c16",
                "lbm_step_inplace", "lbm_step_adjoint_c16", "lbm_step_adjoint_c8",
                "lbm_narrow_codes", "lbm_step_c8", "lbm_step_inplace_c8", "lbm_check_adjacency",
                "lbm_version", "lbm_status_string")


class lbm_geom(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("periodic", C.c_uint32), ("order", C.c_int32), ("order_param", C.c_uint32)]


class lbm_params(C.Structure):
    _fields_ = [("tau_plus", C.c_double), ("magic", C.c_double), ("force", C.c_double * 3),
                ("storage", C.c_int32), ("flags", C.c_int32)]


class lbm_segment(C.Structure):
    _fields_ = [("base", C.c_int64), ("n", C.c_int64), ("param_index", C.c_int32),
                ("pad", C.c_int32)]


class LbmError(RuntimeError):
    def __init__(self, fn: str, status: int):
        self.status = status
        super().__init__(f"{fn} failed: {status} ({status_string(status)})")


_lock = threading.Lock()
_lib = None


def load(path: str = LIB_PATH):
    """Load the library (once).  Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with "
                               "`python -m paper_1111_1129_amd.build` (hipcc, gfx950)")
        lib = C.CDLL(path)
        P, I32, I64, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        lib.lbm_build_adjacency.restype = I32
        lib.lbm_build_adjacency.argtypes = [C.POINTER(lbm_geom), P, I64, I64, P, P, P, I64,
                                            C.POINTER(C.c_int64), P, C.POINTER(SZ), P]
        lib.lbm_init.restype = I32
        lib.lbm_init.argtypes = [C.POINTER(lbm_params), I64, I64, P, C.c_double, P, P]
        lib.lbm_step.restype = I32
        lib.lbm_step.argtypes = [C.POINTER(lbm_params), I32, P, I32, I64, I64, P, P, P, P, I32,
                                 I32, P, C.POINTER(SZ), P]
        lib.lbm_step_batch.restype = I32
        lib.lbm_step_batch.argtypes = [C.POINTER(lbm_params), I32, P, I32, I64, I64, P, P, P, P,
                                       P, P, P, I32, I32, P, C.POINTER(SZ), P]
        lib.lbm_objective.restype = I32
        lib.lbm_objective.argtypes = [C.POINTER(lbm_params), I32, I64, I64, P, P, P, I32, P, P,
                                      C.POINTER(SZ), P]
        lib.lbm_moments_noalloc.restype = I32
        lib.lbm_moments_noalloc.argtypes = [C.POINTER(lbm_params), I32, I64, I64, P, P, P, P, P,
                                            I32, P, P]
        lib.lbm_step_adjoint.restype = I32
        lib.lbm_step_adjoint.argtypes = [C.POINTER(lbm_params), I64, I64, P, P, P, P, P, P, P]
        lib.lbm_moments.restype = I32
        lib.lbm_moments.argtypes = [C.POINTER(lbm_params), I32, I64, I64, P, P, P, P, P, I32, P,
                                    P, C.POINTER(SZ), P]
        lib.lbm_partition_stats.restype = I32
        lib.lbm_partition_stats.argtypes = [I64, I64, P, I64, P, P, P, P, C.POINTER(SZ), P]
        lib.lbm_compress_adjacency.restype = I32
        lib.lbm_compress_adjacency.argtypes = [I64, I64, P, P, P, C.POINTER(C.c_int64), P,
                                               C.POINTER(SZ), P]
        lib.lbm_step_c16.restype = I32
        lib.lbm_step_c16.argtypes = [C.POINTER(lbm_params), I64, I64, P, P, P, P, P, P, I32, P]
        lib.lbm_step_inplace.restype = I32
        lib.lbm_step_inplace.argtypes = [C.POINTER(lbm_params), I64, I64, P, P, P, P, P, I32, I32,
                                         P]
        lib.lbm_step_adjoint_c16.restype = I32
        lib.lbm_step_adjoint_c16.argtypes = [C.POINTER(lbm_params), I64, I64, P, P, P, P, P, P,
                                             P, P, P]
        lib.lbm_step_adjoint_c8.restype = I32
        lib.lbm_step_adjoint_c8.argtypes = [C.POINTER(lbm_params), I64, I64, P, P, P, P, P, P,
                                            P, P, P, P]
        lib.lbm_check_adjacency.restype = I32
        lib.lbm_check_adjacency.argtypes = [I64, I64, I64, P, C.POINTER(C.c_int64), P,
                                            C.POINTER(SZ), P]
        lib.lbm_narrow_codes.restype = I32
        lib.lbm_narrow_codes.argtypes = [I64, I64, P, P, P, C.POINTER(C.c_int64), P,
                                         C.POINTER(SZ), P]
        lib.lbm_step_c8.restype = I32
        lib.lbm_step_c8.argtypes = [C.POINTER(lbm_params), I64, I64, P, P, P, P, P, P, P, I32, P]
        lib.lbm_step_inplace_c8.restype = I32
        lib.lbm_step_inplace_c8.argtypes = [C.POINTER(lbm_params), I64, I64, P, P, P, P, P, P,
                                            I32, I32, P]
        lib.lbm_version.restype = I32
        lib.lbm_version.argtypes = []
        lib.lbm_status_string.restype = C.c_char_p
        lib.lbm_status_string.argtypes = [I32]
        _lib = lib
        return lib


def status_string(status: int) -> str:
    return load().lbm_status_string(status).decode()


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _check(fn, status):
    if status != LBM_OK:
        raise LbmError(fn, status)


def make_params(tau_plus=0.8, magic=3.0 / 16.0, force=(0.0, 0.0, 0.0), storage="f64",
                flags=0) -> lbm_params:
    st = STORAGES[storage] if isinstance(storage, str) else int(storage)
    return lbm_params(float(tau_plus), float(magic), (C.c_double * 3)(*map(float, force)),
                      st, int(flags))


def make_segments(segs):
    """ctypes array of segments from (base, n) or (base, n, param_index) tuples."""
    if not segs:
        return None, 0
    arr = (lbm_segment * len(segs))(*[lbm_segment(int(t[0]), int(t[1]),
                                                  int(t[2]) if len(t) > 2 else 0, 0)
                                      for t in segs])
    return arr, len(segs)


def make_param_array(params):
    """(pointer-compatible array, count) of one lbm_params or a list of them."""
    if isinstance(params, lbm_params):
        return params, 1
    arr = (lbm_params * len(params))(*params)
    return arr, len(params)


# ---------------------------------------------------------------------------
# entry points, same names as the C ABI
# ---------------------------------------------------------------------------

def lbm_build_adjacency(geom: lbm_geom, flag, base, stride, index_of, cell_of, adj, cap,
                        workspace=None, ws_bytes=None, stream=None, query=False):
    """Returns (status, n_fluid, ws_bytes).  With query=True only the workspace
    size is computed."""
    lib = load()
    nf = C.c_int64(0)
    ws = C.c_size_t(0 if ws_bytes is None else ws_bytes)
    st = lib.lbm_build_adjacency(C.byref(geom), _ptr(flag), base, stride, _ptr(index_of),
                                 _ptr(cell_of), _ptr(adj), cap, C.byref(nf),
                                 None if query else _ptr(workspace), C.byref(ws),
                                 _stream(stream))
    return st, nf.value, ws.value


def lbm_init(params: lbm_params, n, stride, f, rho0=1.0, u0=None, stream=None):
    lib = load()
    u = None if u0 is None else (C.c_double * 3)(*map(float, u0))
    return lib.lbm_init(C.byref(params), n, stride, _ptr(f), float(rho0),
                        None if u is None else C.cast(u, C.c_void_p), _stream(stream))


def lbm_step(params, n, stride, adj, ns, f_a, f_b, n_steps, persistent=0,
             segments=None, workspace=None, ws_bytes=0, stream=None, query=False):
    """params: one lbm_params or a list (parameter sets named by the segments'
    third entry).  Returns (status, ws_bytes)."""
    lib = load()
    seg, n_seg = make_segments(segments)
    prm, n_params = make_param_array(params)
    ws = C.c_size_t(ws_bytes)
    st = lib.lbm_step(C.cast(C.pointer(prm), C.POINTER(lbm_params)), n_params, seg, n_seg, n,
                      stride, _ptr(adj), _ptr(ns), _ptr(f_a), _ptr(f_b), n_steps, persistent,
                      None if query else _ptr(workspace), C.byref(ws), _stream(stream))
    return st, ws.value


def lbm_step_batch(params, n, stride, codes8, codes, tile_records, adj, ns, f_a, f_b, n_steps,
                   persistent=0, segments=None, workspace=None, ws_bytes=0, stream=None,
                   query=False):
    """lbm_step over the adjacency codes.  Returns (status, ws_bytes)."""
    lib = load()
    seg, n_seg = make_segments(segments)
    prm, n_params = make_param_array(params)
    ws = C.c_size_t(ws_bytes)
    st = lib.lbm_step_batch(C.cast(C.pointer(prm), C.POINTER(lbm_params)), n_params, seg, n_seg,
                            n, stride, _ptr(codes8), _ptr(codes), _ptr(tile_records), _ptr(adj),
                            _ptr(ns), _ptr(f_a), _ptr(f_b), n_steps, persistent,
                            None if query else _ptr(workspace), C.byref(ws), _stream(stream))
    return st, ws.value


def lbm_step_adjoint(params: lbm_params, n, stride, adj, f_t, ns, lam_next, lam_t, grad_ns,
                     stream=None):
    lib = load()
    return lib.lbm_step_adjoint(C.byref(params), n, stride, _ptr(adj), _ptr(f_t), _ptr(ns),
                                _ptr(lam_next), _ptr(lam_t), _ptr(grad_ns), _stream(stream))


def lbm_moments(params, n, stride, adj, f, rho, u, segments, totals,
                workspace=None, ws_bytes=0, stream=None, query=False):
    lib = load()
    seg, n_seg = make_segments(segments)
    prm, n_params = make_param_array(params)
    ws = C.c_size_t(ws_bytes)
    st = lib.lbm_moments(C.cast(C.pointer(prm), C.POINTER(lbm_params)), n_params, n, stride,
                         _ptr(adj), _ptr(f), _ptr(rho), _ptr(u), seg, n_seg, _ptr(totals),
                         None if query else _ptr(workspace), C.byref(ws), _stream(stream))
    return st, ws.value


def lbm_moments_noalloc(params, n, stride, adj, f, rho, u, segments, totals, stream=None):
    lib = load()
    seg, n_seg = make_segments(segments)
    prm, n_params = make_param_array(params)
    return lib.lbm_moments_noalloc(C.cast(C.pointer(prm), C.POINTER(lbm_params)), n_params, n,
                                   stride, _ptr(adj), _ptr(f), _ptr(rho), _ptr(u), seg, n_seg,
                                   _ptr(totals), _stream(stream))


def lbm_objective(params, n, stride, adj, f, segments, J, workspace=None, ws_bytes=0,
                  stream=None, query=False):
    lib = load()
    seg, n_seg = make_segments(segments)
    prm, n_params = make_param_array(params)
    ws = C.c_size_t(ws_bytes)
    st = lib.lbm_objective(C.cast(C.pointer(prm), C.POINTER(lbm_params)), n_params, n, stride,
                           _ptr(adj), _ptr(f), seg, n_seg, _ptr(J),
                           None if query else _ptr(workspace), C.byref(ws), _stream(stream))
    return st, ws.value


def lbm_check_adjacency(base, n, stride, adj, workspace=None, ws_bytes=0, stream=None,
                        query=False):
    """Returns (status, (entries out of range, slots not referenced once), ws_bytes)."""
    lib = load()
    res = (C.c_int64 * 2)(0, 0)
    ws = C.c_size_t(ws_bytes)
    st = lib.lbm_check_adjacency(base, n, stride, _ptr(adj), res,
                                 None if query else _ptr(workspace), C.byref(ws),
                                 None if query else _stream(stream))
    return st, (int(res[0]), int(res[1])), ws.value


def lbm_partition_stats(n, stride, adj, n_chunks, remote_links, neighbours, interface_cells,
                        workspace=None, ws_bytes=0, stream=None, query=False):
    lib = load()
    ws = C.c_size_t(ws_bytes)
    st = lib.lbm_partition_stats(n, stride, _ptr(adj), n_chunks, _ptr(remote_links),
                                 _ptr(neighbours), _ptr(interface_cells),
                                 None if query else _ptr(workspace), C.byref(ws),
                                 None if query else _stream(stream))
    return st, ws.value


def lbm_compress_adjacency(n, stride, adj, codes, tile_records, workspace=None, ws_bytes=0,
                           stream=None, query=False):
    """Returns (status, n_escapes, ws_bytes).  Synchronizes the stream."""
    lib = load()
    ws = C.c_size_t(ws_bytes)
    esc = C.c_int64(0)
    st = lib.lbm_compress_adjacency(n, stride, _ptr(adj), _ptr(codes), _ptr(tile_records),
                                    C.byref(esc), None if query else _ptr(workspace),
                                    C.byref(ws), None if query else _stream(stream))
    return st, esc.value, ws.value


def lbm_step_c16(params: lbm_params, n, stride, codes, tile_records, adj, ns, f_a, f_b, n_steps,
                 stream=None):
    return load().lbm_step_c16(C.byref(params), n, stride, _ptr(codes), _ptr(tile_records),
                               _ptr(adj), _ptr(ns), _ptr(f_a), _ptr(f_b), int(n_steps),
                               _stream(stream))


def lbm_narrow_codes(n, stride, codes, tile_records, codes8, workspace=None, ws_bytes=0,
                     stream=None, query=False):
    """Returns (status, n_narrow_tiles, ws_bytes).  Synchronizes the stream."""
    lib = load()
    ws = C.c_size_t(ws_bytes)
    cnt = C.c_int64(0)
    st = lib.lbm_narrow_codes(n, stride, _ptr(codes), _ptr(tile_records), _ptr(codes8),
                              C.byref(cnt), None if query else _ptr(workspace), C.byref(ws),
                              None if query else _stream(stream))
    return st, cnt.value, ws.value


def lbm_step_c8(params: lbm_params, n, stride, codes8, codes, tile_records, adj, ns, f_a, f_b,
                n_steps, stream=None):
    return load().lbm_step_c8(C.byref(params), n, stride, _ptr(codes8), _ptr(codes),
                              _ptr(tile_records), _ptr(adj), _ptr(ns), _ptr(f_a), _ptr(f_b),
                              int(n_steps), _stream(stream))


def lbm_step_inplace(params: lbm_params, n, stride, adj, codes, tile_records, ns, f, phase,
                     n_steps, stream=None):
    return load().lbm_step_inplace(C.byref(params), n, stride, _ptr(adj), _ptr(codes),
                                   _ptr(tile_records), _ptr(ns), _ptr(f), int(phase),
                                   int(n_steps), _stream(stream))


def lbm_step_adjoint_c16(params: lbm_params, n, stride, codes, tile_records, adj, f_t, ns,
                         lam_next, lam_t, grad_ns, stream=None):
    return load().lbm_step_adjoint_c16(C.byref(params), n, stride, _ptr(codes),
                                       _ptr(tile_records), _ptr(adj), _ptr(f_t), _ptr(ns),
                                       _ptr(lam_next), _ptr(lam_t), _ptr(grad_ns),
                                       _stream(stream))


def lbm_step_adjoint_c8(params: lbm_params, n, stride, codes8, codes, tile_records, adj, f_t,
                        ns, lam_next, lam_t, grad_ns, stream=None):
    return load().lbm_step_adjoint_c8(C.byref(params), n, stride, _ptr(codes8), _ptr(codes),
                                      _ptr(tile_records), _ptr(adj), _ptr(f_t), _ptr(ns),
                                      _ptr(lam_next), _ptr(lam_t), _ptr(grad_ns),
                                      _stream(stream))


def lbm_step_inplace_c8(params: lbm_params, n, stride, adj, codes8, codes, tile_records, ns, f,
                        phase, n_steps, stream=None):
    return load().lbm_step_inplace_c8(C.byref(params), n, stride, _ptr(adj), _ptr(codes8),
                                      _ptr(codes), _ptr(tile_records), _ptr(ns), _ptr(f),
                                      int(phase), int(n_steps), _stream(stream))


def lbm_version() -> int:
    return load().lbm_version()
