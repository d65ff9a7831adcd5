"""Gradient of the mean flux (permeability) with respect to a per-cell
partial-bounce-back solid fraction, through the hand-written adjoint step.

Forward: T TRT sweeps from rest with solid fraction ns; J = mean over listed
cells of u_x = j_x + G_x/2 after the last sweep (permeability k = nu J / G_x).
Backward, two schedules over the same kernels (bitwise the same gradient):
  * two-level checkpointing -- the forward keeps the state every k steps;
    the backward walks the segments in reverse, recomputes the states of one
    segment into a buffer, and applies the adjoint step from the last state
    of the segment down to its first.  Memory: ceil(T/k) checkpoints + k
    buffer states; work: one extra forward sweep per step.
  * binomial ("revolve") checkpointing with a fixed number of snapshot slots
    (checkpointing.Revolve): memory snapshots + 3 states, work the optimal
    number of recomputed sweeps for that memory.
"""
from __future__ import annotations

import torch

from . import _native as N
from .checkpointing import Revolve
from .lattice import Compressed, Lattice, compress, init, narrow, objective, step_c8


def codes_of(lat: Lattice, comp: Compressed | None) -> Compressed:
    """The lattice's 16-bit codes with their 8-bit form (built if not given)."""
    comp = compress(lat) if comp is None else comp
    return narrow(comp) if comp.codes8 is None else comp


def forward_states(lat: Lattice, prm, ns: torch.Tensor, T: int, k: int,
                   comp: Compressed | None = None):
    """Run T steps from rest; return (J, checkpoints at 0, k, 2k, ..., final state).

    The sweeps read the 8-bit adjacency codes where a tile allows them and
    the 16-bit codes elsewhere (bitwise the same states as the sweep over the
    full list, fewer bytes)."""
    comp = codes_of(lat, comp)
    st = init(lat, prm, ns=ns)
    ckpts = []
    t = 0
    while t < T:
        ckpts.append(st.f.clone())
        n = min(k, T - t)
        step_c8(st, comp, n)
        t += n
    J = objective(st)[0]  # mean x velocity, formed in the library (lbm_objective)
    return J, ckpts, st


def adjoint_gradient(lat: Lattice, prm, ns: torch.Tensor, T: int, k: int, ckpts=None,
                     comp: Compressed | None = None):
    """dJ/dns [stride] (float64) by checkpointed reverse sweeps (the segment
    recomputation and the adjoint steps read the 8-bit codes in narrow tiles
    and the 16-bit codes elsewhere, as the forward does)."""
    comp = codes_of(lat, comp)
    if ckpts is None:
        _, ckpts, _ = forward_states(lat, prm, ns, T, k, comp)
    S, n = lat.stride, lat.n_fluid
    dev = lat.device
    lam = torch.empty((19, S), dtype=torch.float64, device=dev)
    lam_prev = torch.empty_like(lam)
    grad = torch.zeros(S, dtype=torch.float64, device=dev)
    N._check("lbm_step_adjoint", N.lbm_step_adjoint(prm, n, S, lat.adj, None, ns, None, lam, None))
    buf = [torch.empty_like(ckpts[0]) for _ in range(k)]
    nseg = len(ckpts)
    for s in range(nseg - 1, -1, -1):
        t0 = s * k
        t1 = min(t0 + k, T)
        buf[0].copy_(ckpts[s])
        for j in range(1, t1 - t0):
            st = N.lbm_step_c8(prm, n, S, comp.codes8, comp.codes, comp.tile_records, lat.adj,
                               ns, buf[j - 1], buf[j], 1)
            N._check("lbm_step_c8", st)
        for t in range(t1 - 1, t0 - 1, -1):
            rc = N.lbm_step_adjoint_c8(prm, n, S, comp.codes8, comp.codes, comp.tile_records,
                                       lat.adj, buf[t - t0], ns, lam, lam_prev, grad)
            N._check("lbm_step_adjoint_c8", rc)
            lam, lam_prev = lam_prev, lam
    return grad


def adjoint_gradient_revolve(lat: Lattice, prm, ns: torch.Tensor, T: int, snapshots: int,
                             comp: Compressed | None = None, stats: dict | None = None):
    """dJ/dns [stride] (float64) with binomial checkpointing: the reverse
    sweep starts from the initial state alone and keeps at most `snapshots`
    intermediate states (plus the initial one, a work state and the sweep's
    second array); the states are recomputed by the schedule of
    checkpointing.Revolve.  Bitwise the two-level gradient.  stats, if
    given, receives the forward sweeps the schedule ran."""
    comp = codes_of(lat, comp)
    S, n = lat.stride, lat.n_fluid
    dev = lat.device
    st0 = init(lat, prm, ns=ns)
    plan = Revolve(T, snapshots)
    slots = [st0.f] + [torch.empty_like(st0.f) for _ in range(snapshots + 1)]
    spare = st0.g  # the sweep's second array
    lam = torch.empty((19, S), dtype=torch.float64, device=dev)
    lam_prev = torch.empty_like(lam)
    grad = torch.zeros(S, dtype=torch.float64, device=dev)
    N._check("lbm_step_adjoint", N.lbm_step_adjoint(prm, n, S, lat.adj, None, ns, None, lam, None))
    lams = [lam, lam_prev]
    swept = [0]

    def sweeps(src, dst, k):
        rc = N.lbm_step_c8(prm, n, S, comp.codes8, comp.codes, comp.tile_records, lat.adj, ns,
                           src, dst, k)
        N._check("lbm_step_c8", rc)

    def advance(src, dst, t, k):
        # no copy: the first sweep reads slot src, the rest alternate between
        # slot dst and the spare array so that the last one writes slot dst
        a, b = (slots[dst], spare) if (k - 1) % 2 == 0 else (spare, slots[dst])
        sweeps(slots[src], a, 1)
        if k > 1:
            sweeps(a, b, k - 1)  # k - 1 sweeps from a end in b if odd, in a if even
        swept[0] += k

    def adjoint(slot, t):
        rc = N.lbm_step_adjoint_c8(prm, n, S, comp.codes8, comp.codes, comp.tile_records, lat.adj,
                                   slots[slot], ns, lams[0], lams[1], grad)
        N._check("lbm_step_adjoint_c8", rc)
        lams.reverse()

    plan.run(advance, adjoint)
    assert swept[0] == plan.forward_steps
    if stats is not None:
        stats["forward_sweeps"] = swept[0]
        stats["states_held"] = snapshots + 3
    return grad


class PermeabilityFn(torch.autograd.Function):
    """J = PermeabilityFn.apply(ns, lattice, params, T, k[, snapshots]): mean x
    velocity after T sweeps; backward returns dJ/dns via the adjoint, with
    two-level checkpoints every k steps, or, if snapshots is given, with
    binomial checkpointing in that many snapshot slots (k unused)."""

    @staticmethod
    def forward(ctx, ns, lat, prm, T, k, *snapshots_arg):
        if prm.storage not in (N.STORAGES["f64"], N.STORAGES["f64s"]):
            raise ValueError("the adjoint needs FP64 storage")
        snapshots = snapshots_arg[0] if snapshots_arg else None
        ctx.n_inputs = 5 + len(snapshots_arg)
        nsd = ns.detach().contiguous()
        if snapshots is None:
            J, ckpts, _ = forward_states(lat, prm, nsd, T, k)
        else:
            J, ckpts = forward_states(lat, prm, nsd, T, max(T, 1))[0], None
        ctx.lat, ctx.prm, ctx.T, ctx.k, ctx.snapshots = lat, prm, T, k, snapshots
        ctx.ckpts = ckpts
        ctx.save_for_backward(nsd)
        return J

    @staticmethod
    def backward(ctx, gJ):
        (ns,) = ctx.saved_tensors
        if ctx.snapshots is None:
            grad = adjoint_gradient(ctx.lat, ctx.prm, ns, ctx.T, ctx.k, ctx.ckpts)
        else:
            grad = adjoint_gradient_revolve(ctx.lat, ctx.prm, ns, ctx.T, ctx.snapshots)
        ctx.ckpts = None
        return (grad * gJ,) + (None,) * (ctx.n_inputs - 1)
