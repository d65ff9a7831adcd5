"""Python-level objects over the C ABI: Lattice (sparse representation),
State (PDF arrays + parameters) and Batch (many geometries in shared arrays).

Every numeric step runs in the HIP library; this module allocates device
memory with torch and passes pointers and the current stream.
"""
from __future__ import annotations

import dataclasses

import torch

from . import _native as N


ROW_ALIGN = 64  # elements: 128 B rows for FP16 storage, 512 B for FP64


def aligned_stride(n: int, align: int = ROW_ALIGN) -> int:
    """Smallest row stride >= n that starts every [19][stride] row on a
    128-byte boundary.  Unaligned rows make each wave's 512-byte store span
    partial cache lines, which HBM serves as read-modify-write."""
    return max(align, (n + align - 1) // align * align)


@dataclasses.dataclass
class Lattice:
    """Sparse representation of one geometry (paper Sec. 2-3)."""

    dims: tuple             # (nx, ny, nz)
    periodic: int
    order: str
    param: int
    n_fluid: int
    base: int
    stride: int
    index_of: torch.Tensor  # int32 [n_box], -1 = solid
    cell_of: torch.Tensor   # int32 [n_fluid]
    adj: torch.Tensor       # int32 storage of uint32 [18][stride]

    @property
    def device(self):
        return self.adj.device


def _geom(dims, periodic, order, param):
    nx, ny, nz = dims
    o = N.ORDERS[order] if isinstance(order, str) else int(order)
    return N.lbm_geom(int(nx), int(ny), int(nz), int(periodic), o, int(param))


def count_fluid(flags: torch.Tensor, periodic=0, order="lex", param=0, stream=None) -> int:
    """N_f of a flag field (count-only pass of lbm_build_adjacency)."""
    nz, ny, nx = flags.shape
    g = _geom((nx, ny, nz), periodic, order, param)
    idx = torch.empty(nx * ny * nz, dtype=torch.int32, device=flags.device)
    st, _, ws = N.lbm_build_adjacency(g, flags, 0, 0, idx, None, None, 0, query=True)
    N._check("lbm_build_adjacency", st)
    wsb = torch.empty(max(ws, 1), dtype=torch.uint8, device=flags.device)
    st, nf, _ = N.lbm_build_adjacency(g, flags, 0, 0, idx, None, None, 0, wsb, ws, stream)
    N._check("lbm_build_adjacency", st)
    return nf


def build(flags: torch.Tensor, periodic: int = 0, order: str = "lex", param: int = 0,
          base: int = 0, stride: int | None = None, adj: torch.Tensor | None = None,
          stream=None) -> Lattice:
    """Assemble the sparse representation of a flag field on the GPU.

    flags: uint8 [nz][ny][nx] on the device, nonzero = fluid.
    base/stride/adj: place this geometry at columns [base, base + N_f) of an
    existing [18][stride] adjacency (batched use); by default a new array with
    stride = aligned_stride(base + N_f) is allocated.
    """
    assert flags.dtype == torch.uint8 and flags.is_cuda and flags.is_contiguous()
    nz, ny, nx = flags.shape
    g = _geom((nx, ny, nz), periodic, order, param)
    dev = flags.device
    index_of = torch.empty(nx * ny * nz, dtype=torch.int32, device=dev)
    st, _, ws = N.lbm_build_adjacency(g, flags, base, 0, index_of, None, None, 0, query=True)
    N._check("lbm_build_adjacency", st)
    wsb = torch.empty(max(ws, 1), dtype=torch.uint8, device=dev)
    st, nf, _ = N.lbm_build_adjacency(g, flags, base, 0, index_of, None, None, 0, wsb, ws, stream)
    N._check("lbm_build_adjacency", st)
    if stride is None:
        stride = aligned_stride(base + nf)
    if adj is None:
        adj = torch.zeros((18, stride), dtype=torch.int32, device=dev)
    assert adj.shape == (18, stride) and adj.dtype == torch.int32 and adj.is_contiguous()
    cell_of = torch.empty(max(nf, 1), dtype=torch.int32, device=dev)
    st, nf2, _ = N.lbm_build_adjacency(g, flags, base, stride, index_of, cell_of, adj, nf, wsb, ws,
                                       stream)
    N._check("lbm_build_adjacency", st)
    assert nf2 == nf
    return Lattice((nx, ny, nz), periodic, order, param, nf, base, stride, index_of, cell_of[:nf],
                   adj)


@dataclasses.dataclass
class State:
    """PDF ping-pong arrays [19][stride] and the TRT parameters."""

    lattice: Lattice
    params: N.lbm_params
    f: torch.Tensor                 # current state
    g: torch.Tensor                 # the other array
    ns: torch.Tensor | None = None  # float64 [stride] solid fraction (PBB) or None
    n: int = 0                      # number of listed cells the sweep covers
    steps: int = 0

    @property
    def storage(self) -> int:
        return self.params.storage


def params(tau_plus=0.8, magic=3.0 / 16.0, force=(0.0, 0.0, 0.0), storage="f64",
           nontemporal=False, xcd_chunk=0) -> N.lbm_params:
    """TRT parameters.  xcd_chunk: consecutive list tiles per XCD (a power of
    two; 1 = hardware round robin, 0 = one contiguous eighth per XCD)."""
    assert xcd_chunk >= 0 and xcd_chunk & (xcd_chunk - 1) == 0 and xcd_chunk < 256
    flags = (N.FLAG_NONTEMPORAL if nontemporal else 0) | (xcd_chunk << N.FLAG_XCD_CHUNK_SHIFT)
    return N.make_params(tau_plus, magic, force, storage, flags)


def init(lat: Lattice, prm: N.lbm_params, rho0: float = 1.0, u0=None, ns: torch.Tensor | None = None,
         n: int | None = None, stream=None) -> State:
    """Equilibrium state for the listed cells [0, n) (default: base + N_f)."""
    n = lat.base + lat.n_fluid if n is None else n
    dt = N.STORAGE_DTYPE[prm.storage]
    # both arrays in one allocation: their relative placement is fixed
    pair = torch.empty((2, 19, lat.stride), dtype=dt, device=lat.device)
    f, g = pair[0], pair[1]
    st = N.lbm_init(prm, n, lat.stride, f, rho0, u0, stream)
    N._check("lbm_init", st)
    if ns is not None:
        assert ns.dtype == torch.float64 and ns.numel() >= n and ns.is_contiguous()
    return State(lat, prm, f, g, ns, n, 0)


def set_state(state: State, f: torch.Tensor):
    """Overwrite the current PDFs (same shape and dtype)."""
    state.f.copy_(f)


def step(state: State, n_steps: int = 1, persistent: bool = False, segments=None, stream=None):
    """Advance the state by n_steps sweeps (one launch per step, or one
    persistent cooperative launch)."""
    lat = state.lattice
    ws = None
    wsn = 0
    if persistent:
        st, wsn = N.lbm_step(state.params, state.n, lat.stride, lat.adj, state.ns, state.f, state.g,
                             n_steps, 1, segments, query=True)
        N._check("lbm_step", st)
        ws = torch.empty(wsn, dtype=torch.uint8, device=lat.device)
    st, _ = N.lbm_step(state.params, state.n, lat.stride, lat.adj, state.ns, state.f, state.g,
                       n_steps, int(persistent), segments, ws, wsn, stream)
    N._check("lbm_step", st)
    if n_steps % 2 == 1:
        state.f, state.g = state.g, state.f
    state.steps += n_steps
    return state


def moments(state: State, fields: bool = True, segments=None, stream=None):
    """(rho [n], u [3][n], totals [n_seg or 1][4]) in FP64 on the device."""
    assert getattr(state, "phase", 0) == 0, "in-place state must be in phase 0 (an even step count)"
    lat = state.lattice
    n = state.n
    dev = lat.device
    rho = torch.empty(n, dtype=torch.float64, device=dev) if fields else None
    u = torch.empty((3, n), dtype=torch.float64, device=dev) if fields else None
    nseg = len(segments) if segments else 1
    totals = torch.empty((nseg, 4), dtype=torch.float64, device=dev)
    st, wsn = N.lbm_moments(state.params, n, lat.stride, lat.adj, state.f, rho, u, segments,
                            totals, query=True)
    N._check("lbm_moments", st)
    ws = torch.empty(max(wsn, 1), dtype=torch.uint8, device=dev)
    st, _ = N.lbm_moments(state.params, n, lat.stride, lat.adj, state.f, rho, u, segments, totals,
                          ws, wsn, stream)
    N._check("lbm_moments", st)
    return rho, u, totals


def partition_stats(lat: Lattice, n_chunks: int, n: int | None = None, stream=None):
    """(remote_links int64[G], neighbours int32[G], interface_cells int32[G])
    of cutting the list [0, n) into n_chunks near-equal chunks (paper Sec. 2,
    Sec. 7 / Fig. 7)."""
    n = lat.base + lat.n_fluid if n is None else n
    dev = lat.device
    remote = torch.empty(n_chunks, dtype=torch.int64, device=dev)
    nb = torch.empty(n_chunks, dtype=torch.int32, device=dev)
    iface = torch.empty(n_chunks, dtype=torch.int32, device=dev)
    st, wsn = N.lbm_partition_stats(n, lat.stride, lat.adj, n_chunks, remote, nb, iface, query=True)
    N._check("lbm_partition_stats", st)
    ws = torch.empty(wsn, dtype=torch.uint8, device=dev)
    st, _ = N.lbm_partition_stats(n, lat.stride, lat.adj, n_chunks, remote, nb, iface, ws, wsn,
                                  stream)
    N._check("lbm_partition_stats", st)
    return remote, nb, iface


@dataclasses.dataclass
class Compressed:
    """16-bit adjacency codes of a lattice (lbm_compress_adjacency), and
    their 8-bit form in the tiles that allow it (lbm_narrow_codes)."""

    codes: torch.Tensor         # int16 [18][stride]
    tile_records: torch.Tensor  # int32 [ceil(n / 256)][20]: 18 offsets, escapes, narrow flag
    n: int
    n_escapes: int
    codes8: torch.Tensor | None = None  # int8 [18][stride] after narrow()
    n_narrow: int = 0                   # narrow tiles

    @property
    def n_tiles(self) -> int:
        return (self.n + 255) // 256


def compress(lat: Lattice, n: int | None = None, stream=None) -> Compressed:
    """Re-encode adj[:, :n] as int16 offsets from per-tile bases (lossless)."""
    n = lat.base + lat.n_fluid if n is None else n
    dev = lat.device
    codes = torch.empty((18, lat.stride), dtype=torch.int16, device=dev)
    toff = torch.empty(((n + 255) // 256, 20), dtype=torch.int32, device=dev)
    st, _, wsn = N.lbm_compress_adjacency(n, lat.stride, lat.adj, codes, toff, query=True)
    N._check("lbm_compress_adjacency", st)
    ws = torch.empty(wsn, dtype=torch.uint8, device=dev)
    st, esc, _ = N.lbm_compress_adjacency(n, lat.stride, lat.adj, codes, toff, ws, wsn, stream)
    N._check("lbm_compress_adjacency", st)
    return Compressed(codes, toff, n, esc)


def narrow(comp: Compressed, stream=None) -> Compressed:
    """Add the 8-bit codes of the tiles whose codes fit one byte (sets word 19
    of every tile record); returns comp."""
    dev = comp.codes.device
    S = comp.codes.shape[1]
    codes8 = torch.empty((18, S), dtype=torch.int8, device=dev)
    st, _, wsn = N.lbm_narrow_codes(comp.n, S, comp.codes, comp.tile_records, codes8, query=True)
    N._check("lbm_narrow_codes", st)
    ws = torch.empty(wsn, dtype=torch.uint8, device=dev)
    st, cnt, _ = N.lbm_narrow_codes(comp.n, S, comp.codes, comp.tile_records, codes8, ws, wsn,
                                    stream)
    N._check("lbm_narrow_codes", st)
    comp.codes8, comp.n_narrow = codes8, cnt
    return comp


def step_c8(state: State, comp: Compressed, n_steps: int = 1, stream=None):
    """As step(), reading 8-bit codes in narrow tiles and 16-bit codes
    elsewhere (results bitwise equal)."""
    lat = state.lattice
    assert comp.codes8 is not None, "narrow(comp) first"
    assert comp.n == state.n and comp.codes.shape[1] == lat.stride
    st = N.lbm_step_c8(state.params, state.n, lat.stride, comp.codes8, comp.codes,
                       comp.tile_records, lat.adj, state.ns, state.f, state.g, n_steps, stream)
    N._check("lbm_step_c8", st)
    if n_steps % 2 == 1:
        state.f, state.g = state.g, state.f
    state.steps += n_steps
    return state


def step_c16(state: State, comp: Compressed, n_steps: int = 1, stream=None):
    """As step(), reading the 16-bit codes (results bitwise equal)."""
    lat = state.lattice
    assert comp.n == state.n and comp.codes.shape[1] == lat.stride
    st = N.lbm_step_c16(state.params, state.n, lat.stride, comp.codes, comp.tile_records, lat.adj,
                        state.ns, state.f, state.g, n_steps, stream)
    N._check("lbm_step_c16", st)
    if n_steps % 2 == 1:
        state.f, state.g = state.g, state.f
    state.steps += n_steps
    return state


class StepGraph:
    """n_steps sweeps of a State captured once in a HIP graph and replayed as
    one graph launch, for geometries so small that launching a sweep costs
    about as much as the sweep.  n_steps is even, so each replay leaves the
    result in state.f.  The sweeps read the full list (comp None), the
    16-bit codes, or the 8-bit codes where comp has been narrowed; results
    are bitwise those of the same eager calls.  The captured work is kernel
    launches only (no allocation, no memset); the buffers and parameters are
    fixed at capture."""

    def __init__(self, state: State, n_steps: int, comp: Compressed | None = None):
        assert n_steps > 0 and n_steps % 2 == 0, "an even step count"
        lat = state.lattice
        if comp is not None:
            assert comp.n == state.n and comp.codes.shape[1] == lat.stride
        self.state, self.n_steps, self.comp = state, n_steps, comp
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):  # launches go to the capturing stream
            self._launch()

    def _launch(self):
        st, lat, comp = self.state, self.state.lattice, self.comp
        if comp is None:
            rc, _ = N.lbm_step(st.params, st.n, lat.stride, lat.adj, st.ns, st.f, st.g,
                               self.n_steps)
            N._check("lbm_step", rc)
        elif comp.codes8 is None:
            N._check("lbm_step_c16", N.lbm_step_c16(st.params, st.n, lat.stride, comp.codes,
                                                    comp.tile_records, lat.adj, st.ns, st.f,
                                                    st.g, self.n_steps))
        else:
            N._check("lbm_step_c8", N.lbm_step_c8(st.params, st.n, lat.stride, comp.codes8,
                                                  comp.codes, comp.tile_records, lat.adj, st.ns,
                                                  st.f, st.g, self.n_steps))

    def replay(self) -> State:
        self.graph.replay()
        self.state.steps += self.n_steps
        return self.state


@dataclasses.dataclass
class InplaceState:
    """One PDF array [19][stride] stepped in place (lbm_step_inplace).

    phase 0: slot (i, m) holds the post-collision f*_i(m), the layout of
    State.f (moments() and step() expect it); phase 1: slot (opp(i), m) holds
    the population arriving at m in direction i."""

    lattice: Lattice
    params: N.lbm_params
    f: torch.Tensor
    ns: torch.Tensor | None = None
    n: int = 0
    phase: int = 0
    steps: int = 0


def init_inplace(lat: Lattice, prm: N.lbm_params, rho0: float = 1.0, u0=None,
                 ns: torch.Tensor | None = None, n: int | None = None,
                 stream=None) -> InplaceState:
    n = lat.base + lat.n_fluid if n is None else n
    f = torch.empty((19, lat.stride), dtype=N.STORAGE_DTYPE[prm.storage], device=lat.device)
    N._check("lbm_init", N.lbm_init(prm, n, lat.stride, f, rho0, u0, stream))
    if ns is not None:
        assert ns.dtype == torch.float64 and ns.numel() >= n and ns.is_contiguous()
    return InplaceState(lat, prm, f, ns, n, 0, 0)


def step_inplace(state: InplaceState, n_steps: int = 1, comp: Compressed | None = None,
                 stream=None, c8: bool = False) -> InplaceState:
    """n_steps in-place sweeps; with comp the gather-scatter steps read the
    16-bit codes, with c8 also the 8-bit codes of narrow tiles (results
    bitwise the same)."""
    lat = state.lattice
    codes = recs = None
    if comp is not None:
        assert comp.n == state.n and comp.codes.shape[1] == lat.stride
        codes, recs = comp.codes, comp.tile_records
    if c8:
        assert comp is not None and comp.codes8 is not None, "narrow(comp) first"
        st = N.lbm_step_inplace_c8(state.params, state.n, lat.stride, lat.adj, comp.codes8, codes,
                                   recs, state.ns, state.f, state.phase, n_steps, stream)
        N._check("lbm_step_inplace_c8", st)
    else:
        st = N.lbm_step_inplace(state.params, state.n, lat.stride, lat.adj, codes, recs,
                                state.ns, state.f, state.phase, n_steps, stream)
        N._check("lbm_step_inplace", st)
    state.phase = (state.phase + n_steps) % 2
    state.steps += n_steps
    return state


class Batch:
    """Many geometries in one set of [19][S] / [18][S] arrays.

    Geometry k occupies columns [base_k, base_k + N_k); its adjacency entries
    carry its base, so one sweep over [0, sum N_k) advances all of them.
    """

    def __init__(self, flags_list, periodic_list, order="lex", param=0, device="cuda",
                 stride: int | None = None, counts=None):
        if counts is None:
            counts = [count_fluid(fl, per, order, param) for fl, per in zip(flags_list, periodic_list)]
        self.counts = list(counts)
        self.bases = [sum(counts[:k]) for k in range(len(counts))]
        self.total = sum(counts)
        self.stride = aligned_stride(self.total) if stride is None else stride
        assert self.stride >= self.total
        self.adj = torch.zeros((18, self.stride), dtype=torch.int32, device=device)
        self.lattices = []
        for fl, per, b in zip(flags_list, periodic_list, self.bases):
            self.lattices.append(build(fl, per, order, param, base=b, stride=self.stride,
                                       adj=self.adj))
        self.segments = list(zip(self.bases, self.counts))
        first = self.lattices[0]
        self.lattice = Lattice(first.dims, first.periodic, order, param, self.total, 0,
                               self.stride, first.index_of, first.cell_of, self.adj)

    def init(self, prm, rho0=1.0, u0=None, ns=None):
        return init(self.lattice, prm, rho0, u0, ns, n=self.total)
