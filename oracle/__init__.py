"""CPU oracle for the list-based D3Q19 TRT lattice Boltzmann hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, double-precision
statement of what the method computes, written from the paper (Wittmann,
Zeiser, Hager, Wellein, "Domain decomposition and locality optimization for
large-scale lattice Boltzmann simulations") and from the standard TRT
literature where the paper is silent.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the GPU library never does,
and the two share no code (the C source here has its own velocity set, keys
and collision).

The arithmetic lives in ``lbm_oracle.c`` / ``trt_step.inc`` (C99, FP64,
floating-point contraction off, OpenMP over independent cells only).  This
module compiles it with gcc on first use and wraps it with ctypes; the only
thing done in Python is argument marshalling, plus the storage rounding of the
reduced-precision forms (numpy's IEEE round-to-nearest-even conversions).

Parity status of each function (what pins it) is listed in the test-suite
(tests/test_oracle_*.py); every function here is pinned by at least one
closed form, invariant, special case or brute-force check.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "lbm_oracle.c"), os.path.join(_HERE, "trt_step.inc")]
_LIB_PATH = os.path.join(_HERE, "_liblbm_oracle.so")
_lock = threading.Lock()
_lib = None

ORDERS = {"lex": 0, "blocked": 1, "morton1": 2, "morton2": 3, "random": 4, "hilbert": 5}
OK, EINVAL, ECAPACITY, EOVERFLOW = 0, -1, -2, -3


# LBM_ORACLE_SANITIZE=1: build and load a copy instrumented with
# AddressSanitizer and UndefinedBehaviorSanitizer (host code only; the process
# must preload libasan, see tests/test_oracle_sanitized.py).
_SANITIZE = os.environ.get("LBM_ORACLE_SANITIZE") == "1"
_SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
              "-fno-omit-frame-pointer", "-g"]
if _SANITIZE:
    _LIB_PATH = os.path.join(_HERE, "_liblbm_oracle_san.so")


def compile_library(out: str | None = None, sanitize: bool | None = None) -> str:
    """Compile the oracle's C source with gcc (always recompiles)."""
    sanitize = _SANITIZE if sanitize is None else sanitize
    out = out or _LIB_PATH
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", *(_SAN_FLAGS if sanitize else []), "-o", out + ".tmp", _SRC[0], "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        stale = (not os.path.exists(_LIB_PATH)
                 or any(os.path.getmtime(s) > os.path.getmtime(_LIB_PATH) for s in _SRC))
        if stale:
            compile_library()
        lib = C.CDLL(_LIB_PATH)
        P, I64, I32, U64, D = C.c_void_p, C.c_int64, C.c_int, C.c_uint64, C.c_double
        lib.orc_splitmix64.restype = U64
        lib.orc_splitmix64.argtypes = [U64]
        lib.orc_feistel.restype = U64
        lib.orc_feistel.argtypes = [U64, I32, U64]
        lib.orc_feistel_half_bits.restype = I32
        lib.orc_feistel_half_bits.argtypes = [U64]
        lib.orc_key.restype = U64
        lib.orc_key.argtypes = [I32, U64, I64, I64, I64, I64, I64, I64]
        lib.orc_build.restype = I32
        lib.orc_build.argtypes = [I64, I64, I64, C.c_uint32, I32, U64, P, I64, I64, P, P, P,
                                  I64, C.POINTER(C.c_int64)]
        lib.orc_rates.restype = None
        lib.orc_rates.argtypes = [D, D, C.POINTER(D), C.POINTER(D)]
        lib.orc_init.restype = None
        lib.orc_init.argtypes = [I64, I64, I64, I32, D, P, P]
        for name in ("orc_step", "orc_step_c"):
            fn = getattr(lib, name)
            fn.restype = None
            fn.argtypes = [D, D, P, I64, I64, I64, P, P, P, P]
        for name in ("orc_moments", "orc_moments_c"):
            fn = getattr(lib, name)
            fn.restype = None
            fn.argtypes = [P, I32, I64, I64, I64, P, P, P, P, I64, P]
        lib.orc_step_adjoint.restype = None
        lib.orc_step_adjoint.argtypes = [D, D, P, I64, I64, I64, P, P, P, P, P, P]
        lib.orc_velocity.restype = I32
        lib.orc_velocity.argtypes = [I32, C.POINTER(C.c_int)]
        lib.orc_weight.restype = D
        lib.orc_weight.argtypes = [I32]
        lib.orc_set_threads.restype = None
        lib.orc_set_threads.argtypes = [I32]
        lib.orc_max_threads.restype = I32
        lib.orc_max_threads.argtypes = []
        _lib = lib
        return lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def set_threads(n: int):
    """Set the OpenMP thread count used by the step loops."""
    _load().orc_set_threads(int(n))


def max_threads() -> int:
    return _load().orc_max_threads()


# ---------------------------------------------------------------------------
# velocity set (for tests that need to read it back)
# ---------------------------------------------------------------------------

def velocity(i: int):
    c = (C.c_int * 3)()
    opp = _load().orc_velocity(i, c)
    return (c[0], c[1], c[2]), opp


def weight(i: int) -> float:
    return _load().orc_weight(i)


# ---------------------------------------------------------------------------
# numbering and sparse representation
# ---------------------------------------------------------------------------

def splitmix64(x: int) -> int:
    return _load().orc_splitmix64(x)


def feistel(seed: int, h: int, v: int) -> int:
    return _load().orc_feistel(seed, h, v)


def feistel_half_bits(n_box: int) -> int:
    return _load().orc_feistel_half_bits(n_box)


def key(order, param, dims, x, y, z) -> int:
    nx, ny, nz = dims
    return _load().orc_key(ORDERS.get(order, order), param, nx, ny, nz, x, y, z)


@dataclasses.dataclass
class Sparse:
    n_fluid: int
    stride: int
    base: int
    index_of: np.ndarray   # int32 [n_box], -1 = solid
    cell_of: np.ndarray    # int32 [n_fluid]
    adj: np.ndarray | None  # uint32 [18][stride] (only this geometry's columns written)


def build(flags: np.ndarray, periodic: int, order="lex", param: int = 0, base: int = 0,
          stride: int | None = None, adj_out: np.ndarray | None = None) -> Sparse:
    """Compaction + adjacency of one geometry (see orc_build in lbm_oracle.c)."""
    lib = _load()
    flags = np.ascontiguousarray(flags, dtype=np.uint8)
    nz, ny, nx = flags.shape
    nf = C.c_int64(0)
    rc = lib.orc_build(nx, ny, nz, periodic, ORDERS.get(order, order), param, _ptr(flags),
                       0, 0, None, None, None, 0, C.byref(nf))
    if rc != OK:
        raise ValueError(f"orc_build count pass failed: {rc}")
    n = nf.value
    if stride is None:
        stride = base + n
    index_of = np.empty(nx * ny * nz, dtype=np.int32)
    cell_of = np.empty(max(n, 1), dtype=np.int32)
    adj = adj_out if adj_out is not None else np.zeros((18, stride), dtype=np.uint32)
    assert adj.dtype == np.uint32 and adj.shape == (18, stride) and adj.flags.c_contiguous
    rc = lib.orc_build(nx, ny, nz, periodic, ORDERS.get(order, order), param, _ptr(flags),
                       base, stride, _ptr(index_of), _ptr(cell_of), _ptr(adj), n, C.byref(nf))
    if rc != OK:
        raise ValueError(f"orc_build failed: {rc}")
    return Sparse(n, stride, base, index_of, cell_of[:n], adj)


# ---------------------------------------------------------------------------
# flow step
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class TRT:
    tau_plus: float = 0.8
    magic: float = 3.0 / 16.0
    force: tuple = (0.0, 0.0, 0.0)

    def rates(self):
        sp, sm = C.c_double(), C.c_double()
        _load().orc_rates(self.tau_plus, self.magic, C.byref(sp), C.byref(sm))
        return sp.value, sm.value

    def G(self):
        return np.asarray(self.force, dtype=np.float64)


def init(n: int, stride: int | None = None, shifted: bool = False, rho0: float = 1.0,
         u0=(0.0, 0.0, 0.0), f: np.ndarray | None = None, n0: int = 0) -> np.ndarray:
    """Equilibrium state f[19][stride] for cells [n0, n0 + n)."""
    stride = stride if stride is not None else n0 + n
    if f is None:
        f = np.zeros((19, stride), dtype=np.float64)
    u = np.asarray(u0, dtype=np.float64)
    _load().orc_init(n0, n0 + n, stride, int(shifted), rho0, _ptr(u), _ptr(f))
    return f


def step(prm: TRT, adj: np.ndarray, src: np.ndarray, dst: np.ndarray, ns=None,
         n0: int = 0, n1: int | None = None):
    """One TRT pull step over cells [n0, n1): dst = step(src)."""
    stride = src.shape[1]
    n1 = stride if n1 is None else n1
    G = prm.G()
    assert src.flags.c_contiguous and dst.flags.c_contiguous and adj.shape[1] == stride
    if np.iscomplexobj(src) or np.iscomplexobj(ns):
        src = src.astype(np.complex128, copy=False)
        assert dst.dtype == np.complex128
        nsc = None if ns is None else np.ascontiguousarray(ns, dtype=np.complex128)
        _load().orc_step_c(prm.tau_plus, prm.magic, _ptr(G), n0, n1, stride, _ptr(adj),
                           _ptr(nsc), _ptr(src), _ptr(dst))
    else:
        assert src.dtype == np.float64 and dst.dtype == np.float64
        nsr = None if ns is None else np.ascontiguousarray(ns, dtype=np.float64)
        _load().orc_step(prm.tau_plus, prm.magic, _ptr(G), n0, n1, stride, _ptr(adj),
                         _ptr(nsr), _ptr(src), _ptr(dst))
    return dst


def run(prm: TRT, adj: np.ndarray, f: np.ndarray, n_steps: int, ns=None, n0: int = 0,
        n1: int | None = None) -> np.ndarray:
    """n_steps pull steps from state f (not modified); returns the final state."""
    a = f.copy()
    b = np.empty_like(a)
    if n1 is not None:
        b[:] = a
    for _ in range(n_steps):
        step(prm, adj, a, b, ns=ns, n0=n0, n1=n1)
        a, b = b, a
    return a


def round_storage(f: np.ndarray, storage: str) -> np.ndarray:
    """Round an FP64 state to a storage type (IEEE round to nearest even) and
    widen it back: 'f64', 'f32', 'f16s' (FP16 goes through FP32 first, as a
    kernel with FP32 arithmetic and FP16 storage rounds), 'f16s12' (FP16 of
    2^12 times the value: exact scaling, the same two roundings)."""
    if storage in ("f64", "f64s"):
        return f.copy()
    if storage in ("f32", "f32s"):
        return f.astype(np.float32).astype(np.float64)
    if storage == "f16s":
        return f.astype(np.float32).astype(np.float16).astype(np.float64)
    if storage == "f16s12":
        up = (f * 4096.0).astype(np.float32)
        return up.astype(np.float16).astype(np.float64) / 4096.0
    raise KeyError(storage)


# ---------------------------------------------------------------------------
# moments
# ---------------------------------------------------------------------------

def moments(prm: TRT, adj: np.ndarray, f: np.ndarray, shifted: bool = False, n0: int = 0,
            n1: int | None = None):
    """(rho[n], u[3][n], totals[4]) of a stored state over cells [n0, n1)."""
    stride = f.shape[1]
    n1 = stride if n1 is None else n1
    G = prm.G()
    cplx = np.iscomplexobj(f)
    dt = np.complex128 if cplx else np.float64
    rho = np.zeros(stride, dtype=dt)
    u = np.zeros((3, stride), dtype=dt)
    tot = np.zeros(4, dtype=dt)
    fn = _load().orc_moments_c if cplx else _load().orc_moments
    fn(_ptr(G), int(shifted), n0, n1, stride, _ptr(adj), _ptr(np.ascontiguousarray(f)),
       _ptr(rho), _ptr(u), stride, _ptr(tot))
    return rho[n0:n1], u[:, n0:n1], tot


def objective(prm: TRT, adj, f, shifted=False, n0=0, n1=None):
    """J = mean over the listed cells of u_x = j_x + G_x/2."""
    n1 = f.shape[1] if n1 is None else n1
    return moments(prm, adj, f, shifted, n0, n1)[2][1] / (n1 - n0)


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------

def adjoint_step(prm: TRT, adj, f_t, ns, lam_next, lam_t, grad, n0=0, n1=None):
    """lam_t = (d f^{t+1}/d f^t)^T lam_next; grad += (d f^{t+1}/d ns)^T lam_next.
    lam_next None writes the objective's seed lam^T."""
    stride = f_t.shape[1]
    n1 = stride if n1 is None else n1
    G = prm.G()
    _load().orc_step_adjoint(prm.tau_plus, prm.magic, _ptr(G), n0, n1, stride, _ptr(adj),
                             _ptr(f_t), _ptr(ns), _ptr(lam_next), _ptr(lam_t), _ptr(grad))


def gradient(prm: TRT, adj, f0, ns, n_steps: int, shifted=False):
    """(J, dJ/dns) after n_steps from f0, by storing every state and sweeping
    the adjoint backwards (no checkpointing: small cases only)."""
    states = [f0.copy()]
    for _ in range(n_steps):
        nxt = np.empty_like(f0)
        step(prm, adj, states[-1], nxt, ns=ns)
        states.append(nxt)
    J = objective(prm, adj, states[-1], shifted)
    lam = np.zeros_like(f0)
    adjoint_step(prm, adj, states[-1], ns, None, lam, None)
    grad = np.zeros(f0.shape[1])
    lam_prev = np.empty_like(f0)
    for t in range(n_steps - 1, -1, -1):
        adjoint_step(prm, adj, states[t], ns, lam, lam_prev, grad)
        lam, lam_prev = lam_prev, lam
    return J, grad


def complex_step_derivative(prm: TRT, adj, f0, ns, direction, n_steps: int, shifted=False,
                            h: float = 1e-30) -> float:
    """dJ/dns . direction by complex-step differentiation of the forward run."""
    nsc = ns.astype(np.complex128) + 1j * h * np.asarray(direction, dtype=np.float64)
    a = f0.astype(np.complex128)
    b = np.empty_like(a)
    for _ in range(n_steps):
        step(prm, adj, a, b, ns=nsc)
        a, b = b, a
    return float(objective(prm, adj, a, shifted).imag / h)


# ---------------------------------------------------------------------------
# communication analysis of a list cut into chunks (paper Sec. 2, Sec. 7)
# ---------------------------------------------------------------------------

def chunk_bounds(n: int, G: int) -> np.ndarray:
    """Start of each of G chunks of an n-cell list, plus n: chunk k is
    [floor(k n / G), floor((k+1) n / G))."""
    return np.array([(k * n) // G for k in range(G + 1)], dtype=np.int64)


def partition_stats(adj: np.ndarray, n: int, G: int):
    """(remote_links[G], neighbours[G], interface_cells[G]) by definition:
    entry k of cell m streams from cell src when the slot's direction is k+1;
    it is a remote link when src's chunk differs from m's."""
    stride = adj.shape[1]
    bounds = chunk_bounds(n, G)
    cells = np.arange(n)
    own = np.searchsorted(bounds, cells, side="right") - 1
    remote = np.zeros(G, dtype=np.int64)
    pairs = set()
    has_remote = np.zeros(n, dtype=bool)
    for k in range(18):
        slot = adj[k, :n].astype(np.int64)
        streams = slot // stride == k + 1
        src = slot - (k + 1) * stride
        src_chunk = np.where(streams, np.searchsorted(bounds, np.where(streams, src, 0),
                                                      side="right") - 1, own)
        cross = streams & (src_chunk != own)
        remote += np.bincount(own[cross], minlength=G)
        has_remote |= cross
        pairs.update(zip(own[cross].tolist(), src_chunk[cross].tolist()))
    neighbours = np.zeros(G, dtype=np.int64)
    for a, _ in pairs:
        neighbours[a] += 1
    interface = np.bincount(own[has_remote], minlength=G)
    return remote, neighbours, interface
