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


def tune_layout(flags: torch.Tensor, periodic: int, order: str = "lex", param: int = 0,
                storage: str = "f64", force=(1e-6, 0.0, 0.0), sweeps: int = 6,
                candidates: list[int] | None = None,
                chunks: tuple = (1, 4, 16, 64, 0)) -> Layout:
    """Time the candidate layouts on this geometry and return the fastest."""
    n = L.count_fluid(flags, periodic, order, param)
    cands = candidates or candidate_strides(n)
    best = None
    table = []
    stream = torch.cuda.current_stream()
    for S in cands:
        lat = L.build(flags, periodic, order, param, stride=S)
        for nt in (False, True):
            for chunk in chunks:
                prm = L.params(0.8, 3.0 / 16.0, force, storage, nontemporal=nt, xcd_chunk=chunk)
                st = L.init(lat, prm)
                L.step(st, 2)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                L.step(st, sweeps)
                e1.record(stream)
                e1.synchronize()
                t = e0.elapsed_time(e1) / 1e3 / sweeps
                mflups = n / t / 1e6
                table.append((S, nt, chunk, round(mflups, 1)))
                if best is None or mflups > best.mflups:
                    best = Layout(S, nt, chunk, mflups)
                del st
        del lat
    best.table = table
    return best
