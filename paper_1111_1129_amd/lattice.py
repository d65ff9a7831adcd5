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
    index_of: torch.Tensor | None  # int32 [n_box], -1 = solid (None for a batch)
    cell_of: torch.Tensor | None   # int32 [n_fluid] (None for a batch)
    adj: torch.Tensor              # int32 storage of uint32 [18][stride]

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
    """PDF ping-pong arrays [19][stride] and the TRT parameters: one parameter
    set, or a list of sets that the segments (base, n, set index) select."""

    lattice: Lattice
    params: N.lbm_params | list
    f: torch.Tensor                 # current state
    g: torch.Tensor                 # the other array
    ns: torch.Tensor | None = None  # float64 [stride] solid fraction (PBB) or None
    n: int = 0                      # number of listed cells the sweep covers
    steps: int = 0
    segments: list | None = None    # default segments of step() / moments()

    @property
    def first_params(self) -> N.lbm_params:
        return self.params[0] if isinstance(self.params, list) else self.params

    @property
    def storage(self) -> int:
        return self.first_params.storage


def params(tau_plus=0.8, magic=3.0 / 16.0, force=(0.0, 0.0, 0.0), storage="f64",
           nontemporal=False, xcd_chunk=0) -> N.lbm_params:
    """TRT parameters.  xcd_chunk: consecutive list tiles per XCD (a power of
    two; 1 = hardware round robin, 0 = one contiguous eighth per XCD)."""
    assert xcd_chunk >= 0 and xcd_chunk & (xcd_chunk - 1) == 0 and xcd_chunk < 256
    flags = (N.FLAG_NONTEMPORAL if nontemporal else 0) | (xcd_chunk << N.FLAG_XCD_CHUNK_SHIFT)
    return N.make_params(tau_plus, magic, force, storage, flags)


def init(lat: Lattice, prm, rho0: float = 1.0, u0=None, ns: torch.Tensor | None = None,
         n: int | None = None, stream=None, segments=None) -> State:
    """Equilibrium state for the listed cells [0, n) (default: base + N_f).
    prm: one parameter set, or a list of sets (one storage type) that the
    segments select."""
    n = lat.base + lat.n_fluid if n is None else n
    first = prm[0] if isinstance(prm, list) else prm
    dt = N.STORAGE_DTYPE[first.storage]
    # both arrays in one allocation: their relative placement is fixed
    pair = torch.empty((2, 19, lat.stride), dtype=dt, device=lat.device)
    f, g = pair[0], pair[1]
    st = N.lbm_init(first, n, lat.stride, f, rho0, u0, stream)
    N._check("lbm_init", st)
    if ns is not None:
        assert ns.dtype == torch.float64 and ns.numel() >= n and ns.is_contiguous()
    return State(lat, prm, f, g, ns, n, 0, segments)


def _needs_workspace(persistent: bool, segments) -> bool:
    """A persistent launch, or segments selecting parameter sets other than 0,
    read a table / barrier block from the caller's workspace."""
    return bool(persistent) or any(len(t) > 2 and t[2] != 0 for t in (segments or ()))


def _hold(t: torch.Tensor | None, stream) -> torch.Tensor | None:
    """A scratch tensor allocated on torch's current stream but used by work
    queued on `stream`: keep its memory from being handed out again until
    that work is done (it is freed when the caller returns, before the
    asynchronous kernels have run)."""
    if t is not None and stream is not None:
        t.record_stream(stream)
    return t


def _step_workspace(state: State, persistent: bool, segments, query, stream=None):
    if not _needs_workspace(persistent, segments):
        return None, 0
    st, wsn = query()
    N._check("lbm_step", st)
    ws = torch.empty(max(wsn, 1), dtype=torch.uint8, device=state.lattice.device)
    return _hold(ws, stream), wsn


def set_state(state: State, f: torch.Tensor):
    """Overwrite the current PDFs (same shape and dtype)."""
    state.f.copy_(f)


def step(state: State, n_steps: int = 1, persistent: bool = False, segments=None, stream=None):
    """Advance the state by n_steps sweeps (one launch per step, or one
    persistent cooperative launch)."""
    lat = state.lattice
    segments = state.segments if segments is None else segments
    ws, wsn = _step_workspace(state, persistent, segments, lambda: N.lbm_step(
        state.params, state.n, lat.stride, lat.adj, state.ns, state.f, state.g, n_steps, 1,
        segments, query=True), stream)
    st, _ = N.lbm_step(state.params, state.n, lat.stride, lat.adj, state.ns, state.f, state.g,
                       n_steps, int(persistent), segments, ws, wsn, stream)
    N._check("lbm_step", st)
    if n_steps % 2 == 1:
        state.f, state.g = state.g, state.f
    state.steps += n_steps
    return state


def moments(state: State, fields: bool = True, segments=None, stream=None,
            check_finite: bool = False):
    """(rho [n], u [3][n], totals [n_seg or 1][4]) in FP64 on the device.
    With segments, rho and u are written in the segments' columns only (the
    padding between tile-aligned batch members is left as allocated).
    check_finite: the library reads the totals back and raises LbmError
    (LBM_ENONFINITE) if one is NaN or infinite."""
    assert getattr(state, "phase", 0) == 0, "in-place state must be in phase 0 (an even step count)"
    lat = state.lattice
    segments = getattr(state, "segments", None) if segments is None else segments
    params = state.params
    if check_finite:
        params = _with_flag(params, N.FLAG_CHECK_FINITE)
    n = state.n
    dev = lat.device
    rho = torch.empty(n, dtype=torch.float64, device=dev) if fields else None
    u = torch.empty((3, n), dtype=torch.float64, device=dev) if fields else None
    nseg = len(segments) if segments else 1
    totals = torch.empty((nseg, 4), dtype=torch.float64, device=dev)
    st, wsn = N.lbm_moments(params, n, lat.stride, lat.adj, state.f, rho, u, segments,
                            totals, query=True)
    N._check("lbm_moments", st)
    ws = _hold(torch.empty(max(wsn, 1), dtype=torch.uint8, device=dev), stream)
    st, _ = N.lbm_moments(params, n, lat.stride, lat.adj, state.f, rho, u, segments, totals,
                          ws, wsn, stream)
    N._check("lbm_moments", st)
    return rho, u, totals


def _with_flag(params, flag: int):
    """Copies of the parameter set(s) with `flag` added to their flags."""
    def one(p):
        q = N.lbm_params.from_buffer_copy(p)
        q.flags |= flag
        return q
    return [one(p) for p in params] if isinstance(params, list) else one(params)


def objective(state: State, segments=None, stream=None) -> torch.Tensor:
    """J [n_seg or 1] (FP64, device): per segment the mean x velocity
    (j_x + G_x/2) over its cells, the mean flux whose gradient the adjoint
    computes (lbm_objective)."""
    assert getattr(state, "phase", 0) == 0, "in-place state must be in phase 0 (an even step count)"
    lat = state.lattice
    segments = getattr(state, "segments", None) if segments is None else segments
    nseg = len(segments) if segments else 1
    J = torch.empty(nseg, dtype=torch.float64, device=lat.device)
    st, wsn = N.lbm_objective(state.params, state.n, lat.stride, lat.adj, state.f, segments, J,
                              query=True)
    N._check("lbm_objective", st)
    ws = _hold(torch.empty(max(wsn, 1), dtype=torch.uint8, device=lat.device), stream)
    st, _ = N.lbm_objective(state.params, state.n, lat.stride, lat.adj, state.f, segments, J, ws,
                            wsn, stream)
    N._check("lbm_objective", st)
    return J


def check_adjacency(lat: Lattice, stream=None) -> tuple[int, int]:
    """(entries out of range, slots not referenced exactly once) of the
    lattice's own columns (lbm_check_adjacency; (0, 0) for a valid list)."""
    st, _, wsn = N.lbm_check_adjacency(lat.base, lat.n_fluid, lat.stride, lat.adj, query=True)
    N._check("lbm_check_adjacency", st)
    ws = torch.empty(wsn, dtype=torch.uint8, device=lat.device)
    st, res, _ = N.lbm_check_adjacency(lat.base, lat.n_fluid, lat.stride, lat.adj, ws, wsn,
                                       stream)
    N._check("lbm_check_adjacency", st)
    return res


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
    ws = _hold(torch.empty(wsn, dtype=torch.uint8, device=dev), stream)
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


def _step_coded(state: State, comp: Compressed, codes8, n_steps, persistent, segments, stream):
    lat = state.lattice
    assert comp.n == state.n and comp.codes.shape[1] == lat.stride
    segments = state.segments if segments is None else segments
    if persistent or isinstance(state.params, list) or segments:
        # lbm_step_batch: per-segment parameter sets and / or one persistent launch
        ws, wsn = _step_workspace(state, persistent, segments, lambda: N.lbm_step_batch(
            state.params, state.n, lat.stride, codes8, comp.codes, comp.tile_records, lat.adj,
            state.ns, state.f, state.g, n_steps, 1, segments, query=True), stream)
        st, _ = N.lbm_step_batch(state.params, state.n, lat.stride, codes8, comp.codes,
                                 comp.tile_records, lat.adj, state.ns, state.f, state.g, n_steps,
                                 int(persistent), segments, ws, wsn, stream)
        N._check("lbm_step_batch", st)
    elif codes8 is not None:
        st = N.lbm_step_c8(state.params, state.n, lat.stride, codes8, comp.codes,
                           comp.tile_records, lat.adj, state.ns, state.f, state.g, n_steps, stream)
        N._check("lbm_step_c8", st)
    else:
        st = N.lbm_step_c16(state.params, state.n, lat.stride, comp.codes, comp.tile_records,
                            lat.adj, state.ns, state.f, state.g, n_steps, stream)
        N._check("lbm_step_c16", st)
    if n_steps % 2 == 1:
        state.f, state.g = state.g, state.f
    state.steps += n_steps
    return state


def step_c8(state: State, comp: Compressed, n_steps: int = 1, stream=None,
            persistent: bool = False, segments=None):
    """As step(), reading 8-bit codes in narrow tiles and 16-bit codes
    elsewhere (results bitwise equal); persistent / per-segment parameter
    sets go through lbm_step_batch."""
    assert comp.codes8 is not None, "narrow(comp) first"
    return _step_coded(state, comp, comp.codes8, n_steps, persistent, segments, stream)


def step_c16(state: State, comp: Compressed, n_steps: int = 1, stream=None,
             persistent: bool = False, segments=None):
    """As step(), reading the 16-bit codes (results bitwise equal)."""
    return _step_coded(state, comp, None, n_steps, persistent, segments, stream)


class StepGraph:
    """n_steps sweeps of a State captured once in a HIP graph and replayed as
    one graph launch: for geometries so small that launching a sweep costs
    about as much as the sweep, and for a batch that has to advance many
    steps in one launch (every step keeps the hardware's dynamic workgroup
    dispatch, which the persistent launch gives up).  n_steps is even, so
    each replay leaves the result in state.f.  The sweeps read the full list
    (comp None), the 16-bit codes, or the 8-bit codes where comp has been
    narrowed; a batch whose segments select parameter sets goes through
    lbm_step_batch with a workspace allocated before the capture.  Results
    are bitwise those of the same eager calls.  The captured work is kernel
    launches only (no allocation, no memset); the buffers and parameters are
    fixed at capture."""

    def __init__(self, state: State, n_steps: int, comp: Compressed | None = None):
        assert n_steps > 0 and n_steps % 2 == 0, "an even step count"
        lat = state.lattice
        if comp is not None:
            assert comp.n == state.n and comp.codes.shape[1] == lat.stride
        self.state, self.n_steps, self.comp = state, n_steps, comp
        self.ws, self.wsn = None, 0
        if _needs_workspace(False, state.segments):
            codes8, codes, recs = self._codes()
            rc, self.wsn = N.lbm_step_batch(state.params, state.n, lat.stride, codes8, codes, recs,
                                            lat.adj, state.ns, state.f, state.g, n_steps, 0,
                                            state.segments, query=True)
            N._check("lbm_step_batch", rc)
            self.ws = torch.empty(max(self.wsn, 1), dtype=torch.uint8, device=lat.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):  # launches go to the capturing stream
            self._launch()

    def _codes(self):
        comp = self.comp
        if comp is None:
            return None, None, None
        return comp.codes8, comp.codes, comp.tile_records

    def _launch(self):
        st, lat, comp = self.state, self.state.lattice, self.comp
        if self.ws is not None:
            codes8, codes, recs = self._codes()
            rc, _ = N.lbm_step_batch(st.params, st.n, lat.stride, codes8, codes, recs, lat.adj,
                                     st.ns, st.f, st.g, self.n_steps, 0, st.segments, self.ws,
                                     self.wsn)
            N._check("lbm_step_batch", rc)
        elif comp is None:
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
    carry its base, so one sweep over [0, total) advances all of them.  With
    tile_align, every base is a multiple of 256 (the sweep tile), which lets
    the members run with their own parameter sets (init with a list); the
    columns between members are then padding that no segment claims.
    """

    def __init__(self, flags_list, periodic_list, order="lex", param=0, device="cuda",
                 stride: int | None = None, counts=None, tile_align: bool = False):
        if counts is None:
            counts = [count_fluid(fl, per, order, param) for fl, per in zip(flags_list, periodic_list)]
        self.counts = list(counts)
        align = N.SEGMENT_ALIGN if tile_align else 1
        self.bases, b = [], 0
        for c in self.counts:
            self.bases.append(b)
            b = (b + c + align - 1) // align * align
        self.total = self.bases[-1] + self.counts[-1] if self.counts else 0
        self.stride = aligned_stride(self.total) if stride is None else stride
        assert self.stride >= self.total
        self.adj = torch.zeros((18, self.stride), dtype=torch.int32, device=device)
        self.lattices = []
        for fl, per, b in zip(flags_list, periodic_list, self.bases):
            self.lattices.append(build(fl, per, order, param, base=b, stride=self.stride,
                                       adj=self.adj))
        self.segments = list(zip(self.bases, self.counts))
        first = self.lattices[0]
        # box <-> list maps are per member (self.lattices[k]); the batch has none
        self.lattice = Lattice(first.dims, first.periodic, order, param, self.total, 0,
                               self.stride, None, None, self.adj)

    def init(self, prm, rho0=1.0, u0=None, ns=None):
        """State of the whole batch.  prm: one parameter set for every member,
        or one per member (needs tile_align): member k then runs with prm[k]
        and the state's segments name it."""
        if isinstance(prm, list):
            assert len(prm) == len(self.counts), "one parameter set per member"
            assert all(b % N.SEGMENT_ALIGN == 0 for b in self.bases), "Batch(tile_align=True)"
            segs = [(b, c, k) for k, (b, c) in enumerate(self.segments)]
            return init(self.lattice, list(prm), rho0, u0, ns, n=self.total, segments=segs)
        return init(self.lattice, prm, rho0, u0, ns, n=self.total)


# ---------------------------------------------------------------------------
# checkpoint / restart
# ---------------------------------------------------------------------------

def _params_dict(p: N.lbm_params) -> dict:
    return {"tau_plus": p.tau_plus, "magic": p.magic, "force": list(p.force),
            "storage": p.storage, "flags": p.flags}


def _params_from(d: dict) -> N.lbm_params:
    return N.make_params(d["tau_plus"], d["magic"], d["force"], d["storage"], d["flags"])


def checkpoint(state) -> dict:
    """Host copy of what a restart needs: the geometry and ordering, the box
    cell of every listed cell, the PDFs of the listed cells in list order
    (post-collision values, the layout every sweep starts from), the
    parameters, the solid fraction and the step count.  Plain tensors, ints,
    floats and strings only, so torch.save / torch.load(weights_only=True)
    round-trip it.  A state stepped in place must be in phase 0."""
    assert getattr(state, "phase", 0) == 0, "in-place state must be in phase 0 (an even step count)"
    lat = state.lattice
    assert lat.cell_of is not None, "checkpoint one geometry (a batch member's own lattice)"
    b, n = lat.base, lat.n_fluid
    params = state.params if isinstance(state.params, list) else [state.params]
    return {"dims": list(lat.dims), "periodic": int(lat.periodic), "order": lat.order,
            "param": int(lat.param), "cell_of": lat.cell_of[:n].cpu(),
            "f": state.f[:, b:b + n].cpu(), "params": [_params_dict(p) for p in params],
            "ns": None if state.ns is None else state.ns[b:b + n].cpu(), "steps": int(state.steps)}


def restore(ckpt: dict, flags: torch.Tensor, order: str | None = None, param: int | None = None,
            stride: int | None = None) -> State:
    """Rebuild the sparse representation from the flag field -- in the
    checkpoint's ordering or another one: the paper lets the numbering be
    chosen afresh at every restart (Sec. 8) -- and place each listed cell's
    PDFs at its new index.  Every cell's populations are unchanged, so a run
    continued from here is bitwise the uninterrupted one (up to the order of
    the list)."""
    order = ckpt["order"] if order is None else order
    param = ckpt["param"] if param is None else param
    nz, ny, nx = flags.shape
    if [nx, ny, nz] != list(ckpt["dims"]):
        raise ValueError(f"flag field {nx}x{ny}x{nz} is not the checkpoint's {ckpt['dims']}")
    lat = build(flags, ckpt["periodic"], order, param, stride=stride)
    dev = lat.device
    old_cells = ckpt["cell_of"].to(dev, torch.int64)
    if lat.n_fluid != old_cells.numel():
        raise ValueError("the flag field does not hold the checkpoint's fluid cells")
    new_index = lat.index_of.to(torch.int64)[old_cells]
    if bool((new_index < 0).any()):
        raise ValueError("a checkpointed cell is solid in this flag field")
    params = [_params_from(d) for d in ckpt["params"]]
    ns = None
    if ckpt["ns"] is not None:
        ns = torch.zeros(lat.stride, dtype=torch.float64, device=dev)
        ns[new_index] = ckpt["ns"].to(dev)
    st = init(lat, params if len(params) > 1 else params[0], ns=ns)
    st.f[:, new_index] = ckpt["f"].to(dev)
    st.steps = ckpt["steps"]
    return st
