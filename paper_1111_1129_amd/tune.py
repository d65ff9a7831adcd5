"""Empirical layout tuning for the sweep on the actual geometry.

The paper's conclusion proposes choosing ordering parameters by simulating
samples of the geometry on the target machine (Sec. 8).  On the MI355X the
sweep's sustained HBM bandwidth also depends on where the 19 + 19 PDF rows
and the 18 adjacency rows fall in the HBM channel interleave (set by the row
stride) and on the store policy, so those are tuned the same way: a handful
of candidate strides (all 128-byte aligned) x {plain, nontemporal stores} x
a few workgroup-to-XCD chunk lengths are each timed over a few sweeps, and
the fastest is kept.  Results do not depend on the choice (the
arithmetic per cell is identical); only the speed does.
"""
from __future__ import annotations

import dataclasses

import torch

from . import lattice as L


@dataclasses.dataclass
class Layout:
    stride: int
    nontemporal: bool
    xcd_chunk: int
    mflups: float = 0.0
    table: list = dataclasses.field(default_factory=list)
    finals: dict = dataclasses.field(default_factory=dict)


def _next_pow2(n: int) -> int:
    p = 1
    while p < n:
        p <<= 1
    return p


def candidate_strides(n: int) -> list[int]:
    up = lambda v, a: (v + a - 1) // a * a
    p2 = _next_pow2(n)
    cands = {L.aligned_stride(n), up(n, 1 << 10), up(n, 1 << 16), p2, p2 + (1 << 10), p2 + (1 << 13)}
    return sorted(c for c in cands if c >= n)


SWEEPS = ("full", "c16", "c8", "inplace", "inplace_c16", "inplace_c8")


class Sweeper:
    """One way of stepping a lattice: the two-array sweep over the full
    adjacency list ("full"), over 16-bit codes ("c16") or over 8-bit codes
    where a tile allows them ("c8"), or the in-place sweep on one array over
    the full list or the codes ("inplace", "inplace_c16", "inplace_c8").
    Results are bitwise the same after an even number of steps."""

    def __init__(self, lat, kind: str = "full"):
        assert kind in SWEEPS, kind
        self.lat, self.kind = lat, kind
        self.comp = L.compress(lat) if kind.endswith(("c16", "c8")) else None
        if kind.endswith("c8"):
            L.narrow(self.comp)

    def init(self, prm, **kw):
        if self.kind.startswith("inplace"):
            return L.init_inplace(self.lat, prm, **kw)
        return L.init(self.lat, prm, **kw)

    def step(self, st, n_steps: int):
        if self.kind == "full":
            return L.step(st, n_steps)
        if self.kind == "c16":
            return L.step_c16(st, self.comp, n_steps)
        if self.kind == "c8":
            return L.step_c8(st, self.comp, n_steps)
        return L.step_inplace(st, n_steps, self.comp, c8=self.kind.endswith("c8"))


def _time_sweeps(lat, prm, sweeps, stream, sweeper=None):
    sw = sweeper or Sweeper(lat)
    st = sw.init(prm)
    sw.step(st, 2)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sw.step(st, sweeps)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / sweeps


def tune_layout(flags: torch.Tensor, periodic: int, order: str = "lex", param: int = 0,
                storage: str = "f64", force=(1e-6, 0.0, 0.0), sweeps: int = 6,
                candidates: list[int] | None = None,
                chunks: tuple = (1, 4, 16, 64, 0), finalists: int = 5,
                sweep: str = "full", final_seconds: float = 0.25,
                final_max_sweeps: int = 2000) -> Layout:
    """Time the candidate layouts on this geometry and return the fastest.

    `sweep` names the sweep being tuned (see Sweeper); timed runs use an even
    number of sweeps.

    Two stages: every candidate is timed over `sweeps` sweeps; the best
    configuration of every stride and the best `finalists` overall are timed
    again, twice each and interleaved, each time for about `final_seconds`
    (at least 3 x `sweeps`, at most `final_max_sweeps` sweeps), and the best
    mean wins.  Short bursts alone mis-rank layouts a few percent apart, and
    a layout's rate over a burst of a few milliseconds is not its sustained
    rate over seconds of streaming, so no stride is dropped on its burst
    rate alone.  The returned Layout carries the burst table (`table`) and
    the finalists' sustained rates (`finals`, MFLUPS)."""
    n = L.count_fluid(flags, periodic, order, param)
    cands = candidates or candidate_strides(n)
    sweeps += sweeps % 2
    table = []
    stream = torch.cuda.current_stream()
    for S in cands:
        sw = Sweeper(L.build(flags, periodic, order, param, stride=S), sweep)
        for nt in (False, True):
            for chunk in chunks:
                prm = L.params(0.8, 3.0 / 16.0, force, storage, nontemporal=nt, xcd_chunk=chunk)
                t = _time_sweeps(sw.lat, prm, sweeps, stream, sw)
                table.append((S, nt, chunk, round(n / t / 1e6, 1)))
        del sw
    ranked = sorted(table, key=lambda r: -r[3])
    top = ranked[:max(1, finalists)]
    for S in cands:  # the best configuration of every stride
        row = next(r for r in ranked if r[0] == S)
        if row not in top:
            top.append(row)
    by_stride = {}
    for S, nt, chunk, rate in top:
        k = int(final_seconds * rate * 1e6 / max(n, 1))  # sweeps in final_seconds at the burst rate
        k = max(3 * sweeps, min(final_max_sweeps, k))
        by_stride.setdefault(S, []).append((nt, chunk, k + k % 2))
    totals = {}
    for _ in range(2):
        for S, cfgs in by_stride.items():
            sw = Sweeper(L.build(flags, periodic, order, param, stride=S), sweep)
            for nt, chunk, k in cfgs:
                prm = L.params(0.8, 3.0 / 16.0, force, storage, nontemporal=nt, xcd_chunk=chunk)
                t = _time_sweeps(sw.lat, prm, k, stream, sw)
                totals[(S, nt, chunk)] = totals.get((S, nt, chunk), 0.0) + t
            del sw
    (S, nt, chunk), tsum = min(totals.items(), key=lambda kv: kv[1])
    best = Layout(S, nt, chunk, n / (tsum / 2) / 1e6)
    best.table = table
    best.finals = {key: round(n / (t / 2) / 1e6, 1) for key, t in totals.items()}
    return best


def tune_sweep(flags: torch.Tensor, periodic: int, order: str = "lex", param: int = 0,
               storage: str = "f64", force=(1e-6, 0.0, 0.0), sweeps: int = 6,
               kinds=SWEEPS, candidates: list[int] | None = None):
    """Pick the sweep kind (full list, 16-bit or 8-bit codes, in place, in
    place over codes) and its layout: each kind's layout is tuned, and the fastest kind
    wins.  Which one that is depends on the storage form and the ordering
    (codes pay off where tiles are escape-free; in place where the PDF bytes
    dominate).  Returns (kind, Layout, {kind: MFLUPS})."""
    rates = {}
    best = None
    for kind in kinds:
        lay = tune_layout(flags, periodic, order, param, storage, force, sweeps=sweeps,
                          candidates=candidates, sweep=kind)
        rates[kind] = round(lay.mflups, 1)
        if best is None or lay.mflups > best[1].mflups:
            best = (kind, lay)
    return best[0], best[1], rates


ORDER_CANDIDATES = (("lex", 0), ("blocked", 8), ("blocked", 16), ("blocked", 32),
                    ("blocked", 64), ("morton2", 0), ("hilbert", 0))


def crop_sample(flags: torch.Tensor, fraction: float) -> torch.Tensor:
    """Central sub-box holding about `fraction` of the cells (same aspect)."""
    nz, ny, nx = flags.shape
    f = fraction ** (1.0 / 3.0)
    sz, sy, sx = (max(1, int(round(d * f))) for d in (nz, ny, nx))
    z0, y0, x0 = (nz - sz) // 2, (ny - sy) // 2, (nx - sx) // 2
    return flags[z0:z0 + sz, y0:y0 + sy, x0:x0 + sx].contiguous()


def tune_ordering(flags: torch.Tensor, periodic: int, storage: str = "f64",
                  candidates=ORDER_CANDIDATES, sample: float | None = None,
                  force=(1e-6, 0.0, 0.0), sweeps: int = 4, sweep: str = "full"):
    """Pick the cell ordering (and layout) with the highest sweep rate.

    The paper proposes choosing the blocking factor by simulating samples of
    the geometry (Sec. 8); with `sample` the candidates are timed on the
    central sub-box holding that fraction of the cells, otherwise on the
    whole geometry.  Returns (order, param, Layout, table).
    """
    probe = crop_sample(flags, sample) if sample else flags
    # in a crop the y/z walls may be cut away; periodicity is kept as given
    best = None
    table = []
    for order, param in candidates:
        n = L.count_fluid(probe, periodic, order, param)
        if n == 0:
            continue
        lay = tune_layout(probe, periodic, order, param, storage, force, sweeps=sweeps,
                          candidates=sorted({L.aligned_stride(n), candidate_strides(n)[-3]}),
                          chunks=(1, 0), sweep=sweep)
        table.append((order, param, round(lay.mflups, 1)))
        if best is None or lay.mflups > best[2].mflups:
            best = (order, param, lay)
    order, param, lay = best
    if sample:  # re-tune the layout of the chosen ordering on the full geometry
        lay = tune_layout(flags, periodic, order, param, storage, force, sweeps=sweeps,
                          sweep=sweep)
    return order, param, lay, table


def tune_batch_layout(flags_list, periodic_list, order: str = "lex", param: int = 0,
                      storage: str = "f32", force=(1e-6, 0.0, 0.0), sweeps: int = 6,
                      chunks: tuple = (1, 16, 0)):
    """Layout tuning for a Batch: candidate strides of the concatenated list x
    {plain, nontemporal} x XCD chunk lengths, timed over one-launch-per-step
    sweeps; returns (stride, nontemporal, xcd_chunk, table)."""
    counts = [L.count_fluid(fl, per, order, param) for fl, per in zip(flags_list, periodic_list)]
    total = sum(counts)
    stream = torch.cuda.current_stream()
    best, table = None, []
    for S in candidate_strides(total):
        batch = L.Batch(flags_list, periodic_list, order, param, stride=S, counts=counts)
        for nt in (False, True):
            for chunk in chunks:
                prm = L.params(0.8, 3.0 / 16.0, force, storage, nontemporal=nt, xcd_chunk=chunk)
                st = batch.init(prm)
                L.step(st, 2)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                L.step(st, sweeps)
                e1.record(stream)
                e1.synchronize()
                rate = total * sweeps / (e0.elapsed_time(e1) / 1e3) / 1e6
                table.append((S, nt, chunk, round(rate, 1)))
                if best is None or rate > best[3]:
                    best = (S, nt, chunk, rate)
                del st
        del batch
    return best[0], best[1], best[2], table
