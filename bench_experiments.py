"""Measurement experiments of bench.py (``python bench.py --experiment NAME``).

Each prints one JSON line per configuration.  All inputs are the seeded
synthetic workloads of paper_1111_1129_amd.inputs; every timed number is the
average duration of the kernels measured with HIP events on the launch
stream.
"""
from __future__ import annotations

import json
import time

import numpy as np
import torch

from paper_1111_1129_amd import _native as N
from paper_1111_1129_amd import adjoint as AD
from paper_1111_1129_amd import inputs as I
from paper_1111_1129_amd import lattice as L
from paper_1111_1129_amd.tune import Sweeper, tune_layout, tune_ordering, candidate_strides

from bench import PDF_SIZE, code_mix, sweep_bytes  # one definition of the per-update byte counts

BYTES = {"f64": 376, "f64s": 376, "f32": 224, "f32s": 224, "f16s": 148, "f16s12": 148}
PEAK = 8000.0


def emit(d):
    print(json.dumps(d), flush=True)


def timed(fn):
    """Seconds for fn() on the current stream (HIP events)."""
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    out = fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3, out


def quick_layout(flags, periodic, order, param, storage, force=(1e-6, 0.0, 0.0)):
    n = L.count_fluid(flags, periodic, order, param)
    cands = sorted({L.aligned_stride(n), candidate_strides(n)[-3]})
    return tune_layout(flags, periodic, order, param, storage, force, sweeps=4,
                       candidates=cands, chunks=(1, 0))


def dev_flags(g):
    return torch.from_numpy(np.ascontiguousarray(g.flags)).cuda()


# ---------------------------------------------------------------------------
def precision(a):
    """FP64 vs FP32 / shifted storage: speed and velocity error against FP64."""
    g = I.workload("large_packing", scale=a.scale)
    flags = dev_flags(g)
    sweeps = 500
    forms = ["f64", "f64s", "f32", "f32s", "f16s", "f16s12"]
    layouts = {st: tune_layout(flags, g.periodic, "lex", 0, st, sweeps=4) for st in forms}
    t_ref_codes = {}
    for gx in (1e-6, 1e-5, 1e-4):
        ref = None
        t_ref = None
        for st in forms:
            lay = layouts[st]
            lat = L.build(flags, g.periodic, "lex", stride=lay.stride)
            prm = L.params(0.8, 3 / 16, (gx, 0, 0), st, nontemporal=lay.nontemporal,
                           xcd_chunk=lay.xcd_chunk)
            state = L.init(lat, prm)
            L.step(state, 2)
            state = L.init(lat, prm)
            t, _ = timed(lambda: L.step(state, sweeps))
            _, u, tot = L.moments(state)
            n = lat.n_fluid
            rec = {"experiment": "precision", "workload": f"large_packing/{a.scale}",
                   "n_fluid": n, "sweeps": sweeps, "storage": st, "gx": gx,
                   "mflups": round(n * sweeps / t / 1e6, 1),
                   "gbs": round(BYTES[st] * n * sweeps / t / 1e9, 1),
                   "hbm_frac": round(BYTES[st] * n * sweeps / t / 1e9 / PEAK, 4),
                   "stride": lat.stride, "nt": lay.nontemporal, "chunk": lay.xcd_chunk,
                   "mass": float(tot[0, 0]), "mean_ux": float(tot[0, 1]) / n}
            if gx == 1e-6:
                # the same sweeps over the adjacency codes, two arrays and in
                # place (bitwise the same state after the even sweep count)
                for kind in ("c16", "c8", "inplace_c8"):
                    sw = Sweeper(lat, kind)
                    sc = sw.init(prm)
                    sw.step(sc, 2)
                    sc = sw.init(prm)
                    tc, _ = timed(lambda: sw.step(sc, sweeps))
                    rec[f"mflups_{kind}"] = round(n * sweeps / tc / 1e6, 1)
                    rec[f"{kind}_equal"] = bool(torch.equal(sc.f[:, :n], state.f[:, :n]))
                    if st == "f64":
                        t_ref_codes[kind] = tc
                    else:
                        rec[f"speedup_{kind}_vs_f64_{kind}"] = round(t_ref_codes[kind] / tc, 3)
                    del sc, sw
            if st == "f64":
                ref, t_ref = u.clone(), t
            else:
                d = u - ref
                rec["speedup_vs_f64"] = round(t_ref / t, 3)
                rec["u_rel_l2"] = float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(ref))
                rec["u_rel_max"] = float(d.abs().max() / ref.abs().max())
                rec["ux_mean_rel"] = float((u[0].mean() - ref[0].mean()) / ref[0].mean())
            emit(rec)
            del lat, state, u
            torch.cuda.empty_cache()
    precision_vs_oracle(a)


def precision_vs_oracle(a, scale=4, sweeps=500):
    """Every storage form against the FP64 oracle itself, on the 1/4-edge
    crop of the precision workload (128 x 128 x 256, porosity 0.4), plus the
    oracle's own rate on the host cores."""
    import oracle as O
    g = I.workload("large_packing", scale=scale)
    sp = O.build(g.flags, g.periodic, "lex")
    n = sp.n_fluid
    oprm = O.TRT(0.8, 3 / 16, (1e-6, 0.0, 0.0))
    f = O.init(n)
    t0 = time.perf_counter()
    f = O.run(oprm, sp.adj, f, sweeps)
    t_cpu = time.perf_counter() - t0
    _, u_orc, _ = O.moments(oprm, sp.adj, f)
    u_orc = torch.from_numpy(np.ascontiguousarray(u_orc)).cuda()
    flags = dev_flags(g)
    lat = L.build(flags, g.periodic, "lex")
    for st in ("f64", "f64s", "f32", "f32s", "f16s", "f16s12"):
        prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), st)
        state = L.init(lat, prm)
        L.step(state, sweeps)
        _, u, _ = L.moments(state)
        d = u - u_orc
        emit({"experiment": "precision_vs_oracle", "workload": f"large_packing/{scale}",
              "n_fluid": n, "sweeps": sweeps, "storage": st, "gx": 1e-6,
              "u_rel_l2_vs_oracle": float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(u_orc)),
              "u_rel_max_vs_oracle": float(d.abs().max() / u_orc.abs().max()),
              "cpu_baseline": {"value": round(n * sweeps / t_cpu / 1e6, 2), "unit": "MFLUPS",
                               "cores": O.max_threads(), "kind": "oracle",
                               "sample": f"{sweeps} FP64 sweeps of the {n}-cell crop"}})


# Algorithmic bytes of one adjoint cell-step: f^t gathered (19 x 8),
# lambda^{t+1} read (19 x 8), lambda^t scattered (19 x 8), the solid fraction
# (8), the gradient read and written (16), plus the adjacency: 18 uint32, or
# 18 int16 codes and one 80-byte record per 256 cells.
ADJ_BYTES_FULL = 3 * 152 + 8 + 16 + 72
ADJ_BYTES_C16 = 3 * 152 + 8 + 16 + 36 + 80 / 256


def adj_bytes_c8(narrow: float, escape: float) -> float:
    """Bytes per cell-step of the adjoint over 8-bit codes: 18 int8 codes in
    narrow tiles, 18 int16 elsewhere, the uint32 list in escape tiles."""
    return (3 * 152 + 8 + 16 + 18 * narrow + 36 * (1 - narrow - escape) + 72 * escape
            + 80 / 256)


# ---------------------------------------------------------------------------
def adjoint(a):
    """Gradient of the mean flux w.r.t. the PBB solid fraction: adjoint with
    two-level checkpointing vs central finite differences on 32 cells."""
    n_edge = 128 // a.scale
    g = I.pbb_box(4, n=n_edge)
    flags = dev_flags(g)
    # layout of the adjoint kernel (over the 8-/16-bit codes, as the gradient
    # uses it): row stride x store policy x XCD mapping, each timed over 20
    # adjoint steps; the fastest is used for the run
    n = L.count_fluid(flags, g.periodic, "lex")
    table = []
    for S in sorted({L.aligned_stride(n), candidate_strides(n)[-2]}):
        lat = L.build(flags, g.periodic, "lex", stride=S)
        comp = L.narrow(L.compress(lat))
        nsl = torch.zeros(S, dtype=torch.float64, device="cuda")
        nsl[:n] = 0.5
        for nt in (False, True):
            for chunk in (1, 4, 16, 0):
                prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), "f64s", nontemporal=nt, xcd_chunk=chunk)
                st = L.init(lat, prm, ns=nsl)
                lam = torch.zeros((19, S), dtype=torch.float64, device="cuda")
                lam2 = torch.empty_like(lam)
                gr = torch.zeros(S, dtype=torch.float64, device="cuda")

                def adj_steps(reps):
                    for _ in range(reps):
                        N.lbm_step_adjoint_c8(prm, n, S, comp.codes8, comp.codes,
                                              comp.tile_records, lat.adj, st.f, nsl, lam, lam2,
                                              gr)
                adj_steps(1)
                t, _ = timed(lambda: adj_steps(20))
                table.append((S, nt, chunk, round(t / 20 * 1e6, 1)))
                del st, lam, lam2, gr
        del lat, comp
    S_best, nt_best, chunk_best, _ = min(table, key=lambda r: r[3])
    lat = L.build(flags, g.periodic, "lex", stride=S_best)
    comp = L.narrow(L.compress(lat))
    n, S = lat.n_fluid, lat.stride
    cell = lat.cell_of.cpu().numpy()
    ns_host = np.zeros(S)
    ns_host[:n] = g.ns.ravel()[cell]
    ns = torch.from_numpy(ns_host).cuda()
    prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), "f64s", nontemporal=nt_best, xcd_chunk=chunk_best)
    T, k = 500, 22
    t_fwd, (J, ckpts, _) = timed(lambda: AD.forward_states(lat, prm, ns, T, k, comp))
    t_bwd, grad = timed(lambda: AD.adjoint_gradient(lat, prm, ns, T, k, ckpts, comp))
    states_two_level = len(ckpts) + k  # checkpoints + the segment buffer
    # binomial checkpointing: the same gradient with fewer states held
    revolve = []
    for snaps in (4, 10, 42):
        stats = {}
        t_rev, g_rev = timed(lambda: AD.adjoint_gradient_revolve(lat, prm, ns, T, snaps, comp,
                                                                 stats=stats))
        revolve.append({"snapshots": snaps, "states_held": stats["states_held"],
                        "forward_sweeps": stats["forward_sweeps"],
                        "backward_s": round(t_rev, 4),
                        "bitwise_two_level": bool(torch.equal(g_rev, grad))})
        del g_rev
    grad = grad.cpu().numpy()[:n]
    # adjoint kernel alone, over the 8-bit codes, the 16-bit codes and the full list
    narrow, escape = code_mix(comp)
    bytes_c8 = adj_bytes_c8(narrow, escape)
    lam = torch.zeros((19, S), dtype=torch.float64, device="cuda")
    lam2 = torch.empty_like(lam)
    gr = torch.zeros(S, dtype=torch.float64, device="cuda")

    def c16_steps(reps):
        for _ in range(reps):
            N.lbm_step_adjoint_c16(prm, n, S, comp.codes, comp.tile_records, lat.adj, ckpts[0],
                                   ns, lam, lam2, gr)

    def c8_steps(reps):
        for _ in range(reps):
            N.lbm_step_adjoint_c8(prm, n, S, comp.codes8, comp.codes, comp.tile_records, lat.adj,
                                  ckpts[0], ns, lam, lam2, gr)

    def full_steps(reps):
        for _ in range(reps):
            N.lbm_step_adjoint(prm, n, S, lat.adj, ckpts[0], ns, lam, lam2, gr)
    c8_steps(1)
    t_adj, _ = timed(lambda: c8_steps(20))
    t_adj /= 20
    c16_steps(1)
    t_adj_c16, _ = timed(lambda: c16_steps(20))
    t_adj_c16 /= 20
    full_steps(1)
    t_adj_full, _ = timed(lambda: full_steps(20))
    t_adj_full /= 20
    del ckpts
    torch.cuda.empty_cache()

    def ux_of(nsv):
        st = L.init(lat, prm, ns=nsv)
        L.step(st, T)
        _, u, _ = L.moments(st)
        return u[0]

    def dJ(e):
        # J(ns + e) - J(ns - e) from the per-cell velocity difference: the
        # two runs' x velocities are subtracted cell by cell before summing,
        # so the difference is not quantised at one ulp of J as a difference
        # of two rounded means would be.
        return float((ux_of(ns + e) - ux_of(ns - e)).sum()) / n

    rng = np.random.default_rng(44)
    inner = np.flatnonzero((ns_host[:n] > 0.05) & (ns_host[:n] < 0.95))
    cells = rng.choice(inner, 32, replace=False)
    hs = (1e-2, 1e-3, 1e-4, 1e-5)
    fds = {h: [] for h in hs}
    t0 = time.perf_counter()
    for c in cells:
        for h in hs:
            e = torch.zeros(S, dtype=torch.float64, device="cuda")
            e[int(c)] = h
            fds[h].append(dJ(e) / (2 * h))
    t_fd = time.perf_counter() - t0
    g32 = grad[cells]
    per_h = {h: np.abs(g32 - np.array(v)) / np.abs(np.array(v)) for h, v in fds.items()}
    # Richardson: central differences have an h^2 leading error, so
    # (4 D(h/10) - ...) -- here the classic 2-point combination of h and h/10
    rich = (100 * np.array(fds[1e-3]) - np.array(fds[1e-2])) / 99
    per_h["richardson_1e-2_1e-3"] = np.abs(g32 - rich) / np.abs(rich)
    errs = per_h[1e-4]
    import oracle as O
    osp = O.build(g.flags, g.periodic, "lex")
    oprm = O.TRT(0.8, 3 / 16, (1e-6, 0.0, 0.0))
    ons = np.ascontiguousarray(g.ns.ravel()[osp.cell_of])
    of = O.init(osp.n_fluid, shifted=True)
    og = np.empty_like(of)
    ol, ol2, ogr = np.zeros_like(of), np.zeros_like(of), np.zeros(osp.n_fluid)
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        O.step(oprm, osp.adj, of, og, ns=ons)
    t_of = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        O.adjoint_step(oprm, osp.adj, of, ons, ol, ol2, ogr)
    t_oa = (time.perf_counter() - t0) / reps
    cpu = {"value": round(osp.n_fluid / (t_of + t_oa) / 1e6, 2), "unit": "M cell-steps/s",
           "cores": O.max_threads(), "kind": "oracle",
           "sample": f"{reps} forward + {reps} adjoint FP64 steps of the same box",
           "forward_step_s": round(t_of, 4), "adjoint_step_s": round(t_oa, 4)}
    emit({"experiment": "adjoint", "workload": f"pbb_box {n_edge}^3", "n_fluid": n, "steps": T,
          "checkpoint_every": k, "J_mean_ux": float(J), "forward_s": round(t_fwd, 4),
          "backward_s": round(t_bwd, 4), "backward_over_forward": round(t_bwd / t_fwd, 2),
          "two_level_states_held": states_two_level, "revolve": revolve,
          "layout": [S, nt_best, chunk_best], "layout_table_us": table,
          "adjoint_step_us": round(t_adj * 1e6, 1), "adjoint_codes": "8-bit",
          "narrow_cells": round(narrow, 4), "escape_cells": round(escape, 4),
          "adjoint_bytes_per_cell": round(bytes_c8, 2),
          "adjoint_gbs": round(bytes_c8 * n / t_adj / 1e9, 1),
          "adjoint_hbm_frac": round(bytes_c8 * n / t_adj / 1e9 / PEAK, 4),
          "adjoint_c16_step_us": round(t_adj_c16 * 1e6, 1),
          "adjoint_c16_gbs": round(ADJ_BYTES_C16 * n / t_adj_c16 / 1e9, 1),
          "adjoint_full_list_step_us": round(t_adj_full * 1e6, 1),
          "adjoint_full_list_gbs": round(ADJ_BYTES_FULL * n / t_adj_full / 1e9, 1),
          "fd_cells": 32, "fd_h": 1e-4, "fd_rel_err_max": float(errs.max()),
          "fd_rel_err_median": float(np.median(errs)), "fd_pass_1e-6": int((errs <= 1e-6).sum()),
          "fd_by_h": {str(h): {"max": float(v.max()), "median": float(np.median(v)),
                               "pass_1e-6": int((v <= 1e-6).sum())} for h, v in per_h.items()},
          "grad_abs_median": float(np.median(np.abs(g32))), "fd_seconds": round(t_fd, 1),
          "cpu_baseline": cpu,
          "cells": [{"cell": int(c), "ns": float(ns_host[c]), "adjoint": float(g32[i]),
                     **{f"fd_{h:g}": float(fds[h][i]) for h in hs}} for i, c in enumerate(cells)]})


# ---------------------------------------------------------------------------
def batched(a):
    """64 uneven geometries: one persistent launch vs one launch per step over
    the concatenated list vs separate per-geometry launches."""
    count = max(1, 64 // a.scale)
    geoms = I.batch_packings(count=count)
    flags = [dev_flags(g) for g in geoms]
    steps = 200
    from paper_1111_1129_amd.tune import tune_batch_layout
    for storage in ("f32", "f32s"):
        S, nt, chunk, _tab = tune_batch_layout(flags, [g.periodic for g in geoms], "lex", 0, storage)
        batch = L.Batch(flags, [g.periodic for g in geoms], "lex", stride=S)
        prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), storage, nontemporal=nt, xcd_chunk=chunk)
        tot_n = batch.total
        st = batch.init(prm)
        L.step(st, 2)
        st = batch.init(prm)
        t_step, _ = timed(lambda: L.step(st, steps))
        f_step = st.f[:, :tot_n].clone()
        stp = batch.init(prm)
        t_pers, _ = timed(lambda: L.step(stp, steps, persistent=True, segments=batch.segments))
        same = bool(torch.equal(stp.f[:, :tot_n], f_step))
        # the same concatenated list swept over 16-bit adjacency codes (tiles
        # that straddle two geometries escape to the full list)
        comp = L.compress(batch.lattice, n=tot_n)
        stc = batch.init(prm)
        L.step_c16(stc, comp, 2)
        stc = batch.init(prm)
        t_c16, _ = timed(lambda: L.step_c16(stc, comp, steps))
        same_c16 = bool(torch.equal(stc.f[:, :tot_n], f_step))
        del stc
        # and over 8-bit codes where a tile allows them
        L.narrow(comp)
        stc = batch.init(prm)
        L.step_c8(stc, comp, 2)
        stc = batch.init(prm)
        t_c8, _ = timed(lambda: L.step_c8(stc, comp, steps))
        same_c8 = bool(torch.equal(stc.f[:, :tot_n], f_step))
        del stc
        # one persistent launch over the 8-bit codes (lbm_step_batch)
        stc = batch.init(prm)
        L.step_c8(stc, comp, 2, persistent=True)
        stc = batch.init(prm)
        t_c8p, _ = timed(lambda: L.step_c8(stc, comp, steps, persistent=True))
        same_c8p = bool(torch.equal(stc.f[:, :tot_n], f_step))
        del stc
        # every member with its own tau+ and force: members on 256-cell tiles,
        # one persistent launch over the 8-bit codes
        tb = L.Batch(flags, [g.periodic for g in geoms], "lex", stride=S, tile_align=True)
        prms = [L.params(0.6 + 0.6 * k / max(1, count - 1), 3 / 16, (1e-6 * (1 + k % 3), 0, 0),
                         storage, nontemporal=nt, xcd_chunk=chunk) for k in range(count)]
        tcomp = L.narrow(L.compress(tb.lattice, n=tb.total))
        stm = tb.init(prms)
        L.step_c8(stm, tcomp, 2, persistent=True)
        stm = tb.init(prms)
        t_mp, _ = timed(lambda: L.step_c8(stm, tcomp, steps, persistent=True))
        stm2 = tb.init(prms)
        t_ms, _ = timed(lambda: L.step_c8(stm2, tcomp, steps))
        same_m = bool(torch.equal(stm.f[:, :tb.total], stm2.f[:, :tb.total]))
        # all steps in one graph launch (the per-step launches captured once)
        stg = tb.init(prms)
        graph = L.StepGraph(stg, steps, tcomp)
        graph.replay()
        stg2 = tb.init(prms)
        stg.f.copy_(stg2.f)
        t_mg, _ = timed(graph.replay)
        same_g = bool(torch.equal(stg.f[:, :tb.total], stm2.f[:, :tb.total]))
        del stm, stm2, stg, stg2, graph, tcomp, tb
        solos = []
        for fl, g in zip(flags, geoms):
            lat = L.build(fl, g.periodic, "lex")
            solos.append(L.init(lat, prm))

        def separate():
            for _ in range(steps):
                for s_ in solos:
                    L.step(s_, 1)

        t_sep, _ = timed(separate)
        _, _, tot = L.moments(st, fields=False, segments=batch.segments)
        cpu = None
        if storage == "f32":
            import oracle as O
            oprm = O.TRT(0.8, 3 / 16, (1e-6, 0.0, 0.0))
            t_cpu, cells = 0.0, 0
            for g in geoms:
                osp = O.build(g.flags, g.periodic, "lex")
                of = O.init(osp.n_fluid)
                og = np.empty_like(of)
                t0 = time.perf_counter()
                O.step(oprm, osp.adj, of, og)
                t_cpu += time.perf_counter() - t0
                cells += osp.n_fluid
            cpu = {"value": round(cells / t_cpu / 1e6, 2), "unit": "MFLUPS",
                   "cores": O.max_threads(), "kind": "oracle",
                   "sample": "one FP64 sweep of every member geometry"}
        emit({"experiment": "batched", "geometries": count, "n_fluid_total": tot_n,
              "cpu_baseline": cpu, "layout": [S, nt, chunk],
              "edge_min": min(g.dims[0] for g in geoms), "edge_max": max(g.dims[0] for g in geoms),
              "storage": storage, "steps": steps,
              "mflups_persistent": round(tot_n * steps / t_pers / 1e6, 1),
              "mflups_launch_per_step": round(tot_n * steps / t_step / 1e6, 1),
              "mflups_separate_launches": round(tot_n * steps / t_sep / 1e6, 1),
              "mflups_c16_per_step": round(tot_n * steps / t_c16 / 1e6, 1),
              "c16_escapes": comp.n_escapes, "c16_equals_per_step": same_c16,
              "mflups_c8_per_step": round(tot_n * steps / t_c8 / 1e6, 1),
              "c8_narrow_tiles": comp.n_narrow, "tiles": comp.n_tiles,
              "c8_equals_per_step": same_c8,
              "mflups_c8_persistent": round(tot_n * steps / t_c8p / 1e6, 1),
              "c8_persistent_equals_per_step": same_c8p,
              "mflups_c8_persistent_member_params": round(tot_n * steps / t_mp / 1e6, 1),
              "mflups_c8_per_step_member_params": round(tot_n * steps / t_ms / 1e6, 1),
              "member_params_persistent_equals_per_step": same_m,
              "mflups_c8_graph_member_params": round(tot_n * steps / t_mg / 1e6, 1),
              "member_params_graph_equals_per_step": same_g,
              "persistent_equals_per_step": same,
              "gbs_persistent": round(BYTES[storage] * tot_n * steps / t_pers / 1e9, 1),
              "gbs_launch_per_step": round(BYTES[storage] * tot_n * steps / t_step / 1e9, 1),
              "mass_finite": bool(torch.isfinite(tot).all())})
        del batch, st, stp, solos
        torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
def orderings(a):
    """Sweep and assembly speed vs cell ordering (the paper's Fig. 4 study on
    one GPU): lexicographic, blocking factors, Z curves, random."""
    g, desc = (I.packing_tube(2), "tube_packing") if a.workload == "tube_packing" else \
        (I.channel(100), "channel")
    flags = dev_flags(g)
    sweeps = 200
    cases = [("lex", 0)] + [("blocked", b) for b in (2, 4, 8, 16, 32, 64, 100)] + \
        [("morton1", 0), ("morton2", 0), ("hilbert", 0), ("random", 22)]
    for order, param in cases:
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lat = L.build(flags, g.periodic, order, param)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        t_asm = float(np.median(ts))
        lay = quick_layout(flags, g.periodic, order, param, "f64")
        lat = L.build(flags, g.periodic, order, param, stride=lay.stride)
        prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), "f64", nontemporal=lay.nontemporal,
                       xcd_chunk=lay.xcd_chunk)
        st = L.init(lat, prm)
        L.step(st, 2)
        t, _ = timed(lambda: L.step(st, sweeps))
        n = lat.n_fluid
        emit({"experiment": "orderings", "workload": desc, "n_fluid": n, "order": order,
              "param": param, "mflups": round(n * sweeps / t / 1e6, 1),
              "gbs": round(376 * n * sweeps / t / 1e9, 1),
              "hbm_frac": round(376 * n * sweeps / t / 1e9 / PEAK, 4),
              "stride": lay.stride, "nt": lay.nontemporal, "chunk": lay.xcd_chunk,
              "assembly_ms": round(t_asm * 1e3, 2),
              "assembly_mcells_per_s": round(flags.numel() / t_asm / 1e6, 1),
              # flag read + index_of write per box cell, cell_of + adjacency per fluid cell
              "assembly_gbs": round((5 * flags.numel() + 76 * n) / t_asm / 1e9, 1)})
        del lat, st
        torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
def partitions(a):
    """The paper's Fig. 7 analysis on one GPU: neighbour chunks and remote
    links per chunk when the list is cut into G chunks, per ordering, for
    the paper's 500x100x100 channel and for the tube packing."""
    for name, g in (("channel", I.channel(100)), ("tube_packing", I.packing_tube(2))):
        flags = dev_flags(g)
        for order, param in [("lex", 0), ("blocked", 8), ("blocked", 32), ("blocked", 100),
                             ("morton1", 0), ("morton2", 0), ("hilbert", 0)]:
            lat = L.build(flags, g.periodic, order, param)
            for G in (8, 64, 512, 3072):
                t, (r, nb, ifc) = timed(lambda: L.partition_stats(lat, G))
                r, nb = r.double(), nb.double()
                emit({"experiment": "partitions", "workload": name, "n_fluid": lat.n_fluid,
                      "order": order, "param": param, "chunks": G,
                      "cells_per_chunk": lat.n_fluid / G,
                      "neighbours_mean": round(float(nb.mean()), 2),
                      "neighbours_max": int(nb.max()),
                      "remote_links_mean": round(float(r.mean()), 1),
                      "remote_links_max": int(r.max()),
                      "remote_links_total": int(r.sum()),
                      "interface_cells_mean": round(float(ifc.double().mean()), 1),
                      "analysis_ms": round(t * 1e3, 3)})
            del lat


def ordering_tuner(a):
    """Automatic choice of ordering: candidates timed on a 1/8 sample of the
    geometry (the paper's proposal, Sec. 8) and on the whole geometry."""
    g = I.packing_tube(2)
    flags = dev_flags(g)
    for sample in (0.125, None):
        t0 = time.perf_counter()
        order, param, lay, table = tune_ordering(flags, g.periodic, "f64", sample=sample)
        dt = time.perf_counter() - t0
        emit({"experiment": "ordering_tuner", "sample": sample, "chosen": [order, param],
              "layout": [lay.stride, lay.nontemporal, lay.xcd_chunk],
              "full_geometry_mflups": round(lay.mflups, 1), "tuning_s": round(dt, 2),
              "candidates": table})


# ---------------------------------------------------------------------------
def bytes_resident(storage, kind):
    """HBM bytes per cell held by the arrays a sweep needs."""
    pdf = 19 * PDF_SIZE[storage] * (1 if kind.startswith("inplace") else 2)
    return pdf + 72 + (36 if kind.endswith(("c16", "c8")) else 0) + (18 if kind.endswith("c8") else 0)


def compressed(a):
    """Byte reduction: the sweep over 16-bit adjacency codes, over 8-bit codes
    where a tile allows them, and the in-place sweep (one PDF array), each
    against the two-array sweep over the full uint32 list: speed per storage
    form and ordering, bitwise equality of the results after the same (even)
    number of sweeps."""
    sweeps = 400
    kinds = ("full", "c16", "c8", "inplace", "inplace_c16", "inplace_c8")
    tube = I.packing_tube(2)
    cases = [("tube_packing", tube, "lex", 0),
             ("tube_packing", tube, "blocked", 16),
             ("tube_packing", tube, "morton2", 0),
             ("tube_packing", tube, "hilbert", 0),
             (f"large_packing/{a.scale}", I.workload("large_packing", scale=a.scale), "lex", 0)]
    for name, g, order, param in cases:
        flags = dev_flags(g)
        for storage in ("f64", "f32s", "f16s"):
            lay = tune_layout(flags, g.periodic, order, param, storage, sweeps=4)
            lat = L.build(flags, g.periodic, order, param, stride=lay.stride)
            n = lat.n_fluid
            t_asm, comp = timed(lambda: L.compress(lat))
            t_narrow, _ = timed(lambda: L.narrow(comp))  # word 19: read by c8 only
            narrow, escape = code_mix(comp)
            res = {}
            for kind in kinds:
                best = None
                for nt, chunk in ((lay.nontemporal, lay.xcd_chunk), (True, 1), (False, 1),
                                  (True, 0), (False, 0)):
                    prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), storage, nontemporal=nt,
                                   xcd_chunk=chunk)
                    if kind in ("full", "c16", "c8"):
                        def run(k, st):
                            if kind == "full":
                                return L.step(st, k)
                            if kind == "c8":
                                return L.step_c8(st, comp, k)
                            return L.step_c16(st, comp, k)
                        make = L.init
                    else:
                        def run(k, st):
                            return L.step_inplace(st, k, None if kind == "inplace" else comp,
                                                  c8=kind == "inplace_c8")
                        make = L.init_inplace
                    st = make(lat, prm)
                    run(2, st)
                    st = make(lat, prm)
                    t, _ = timed(lambda: run(sweeps, st))
                    if best is None or t < best[0]:
                        best = (t, nt, chunk, st.f[:, :n].clone())
                    del st
                    torch.cuda.empty_cache()
                res[kind] = best
            tf = res["full"][0]
            rec = {"experiment": "compressed", "workload": name, "order": order, "n_fluid": n,
                   "storage": storage, "sweeps": sweeps, "stride": lat.stride,
                   "escapes": comp.n_escapes, "compress_ms": round(t_asm * 1e3, 2),
                   "narrow_ms": round(t_narrow * 1e3, 2), "narrow_cells": round(narrow, 4),
                   "escape_cells": round(escape, 4)}
            for kind in kinds:
                t, nt, chunk, f = res[kind]
                bpu = sweep_bytes(storage, kind, narrow, escape)
                rec[kind] = {"mflups": round(n * sweeps / t / 1e6, 1),
                             "speedup": round(tf / t, 3),
                             "bytes_per_update": round(bpu, 2),
                             "gbs": round(bpu * n * sweeps / t / 1e9, 1),
                             "hbm_frac": round(bpu * n * sweeps / t / 1e9 / PEAK, 4),
                             "resident_bytes_per_cell": bytes_resident(storage, kind),
                             "layout": [nt, chunk],
                             "bitwise_equal_full": bool(torch.equal(f, res["full"][3]))}
            emit(rec)
            del lat, comp, res
            torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
def oracle_rates(a):
    """The plain FP64 oracle on the host cores, one thread and all threads:
    sweep rate on the small packing and on the tube for each ordering, and the
    forward and adjoint step rates on the PBB box (the CPU side of every GPU
    number; no GPU work)."""
    import oracle as O
    all_threads = O.max_threads()
    prm = O.TRT(0.8, 3 / 16, (1e-6, 0.0, 0.0))
    cases = [("small_packing", I.packing_small(1), [("lex", 0)], 50),
             ("tube_packing", I.packing_tube(2),
              [("lex", 0), ("blocked", 16), ("morton1", 0), ("morton2", 0), ("random", 22)], 2)]
    for name, g, orders, steps in cases:
        for order, param in orders:
            sp = O.build(g.flags, g.periodic, order, param)
            n = sp.n_fluid
            rec = {"experiment": "oracle_rates", "workload": name, "order": order, "param": param,
                   "n_fluid": n, "steps": steps}
            for threads in (1, all_threads):
                O.set_threads(threads)
                f = O.init(n)
                h = np.empty_like(f)
                O.step(prm, sp.adj, f, h)
                t0 = time.perf_counter()
                for _ in range(steps):
                    O.step(prm, sp.adj, f, h)
                    f, h = h, f
                dt = time.perf_counter() - t0
                rec[f"mflups_{threads}_threads"] = round(n * steps / dt / 1e6, 2)
            emit(rec)
            del sp
    g = I.pbb_box(4)
    sp = O.build(g.flags, g.periodic, "lex")
    n = sp.n_fluid
    ns_list = np.ascontiguousarray(g.ns.reshape(-1)[sp.cell_of[:n].astype(np.int64)],
                                   dtype=np.float64)
    f = O.init(n, shifted=True)
    h = np.empty_like(f)
    lam = np.zeros_like(f)
    lam2 = np.zeros_like(f)
    grad = np.zeros(n)
    rec = {"experiment": "oracle_rates", "workload": "pbb_box 128^3", "n_fluid": n, "steps": 3}
    for threads in (1, all_threads):
        O.set_threads(threads)
        t0 = time.perf_counter()
        for _ in range(3):
            O.step(prm, sp.adj, f, h, ns=ns_list)
            f, h = h, f
        t_fwd = time.perf_counter() - t0
        O.adjoint_step(prm, sp.adj, f, ns_list, None, lam, grad)
        t0 = time.perf_counter()
        for _ in range(3):
            O.adjoint_step(prm, sp.adj, f, ns_list, lam, lam2, grad)
            lam, lam2 = lam2, lam
        t_adj = time.perf_counter() - t0
        rec[f"forward_mcells_per_s_{threads}_threads"] = round(n * 3 / t_fwd / 1e6, 2)
        rec[f"adjoint_mcells_per_s_{threads}_threads"] = round(n * 3 / t_adj / 1e6, 2)
    O.set_threads(all_threads)
    emit(rec)


# ---------------------------------------------------------------------------
def pbb(a):
    """The sweep with partial bounce-back (one more FP64 value per cell: the
    solid fraction) on the tube with a uniform random field and on the PBB box
    with its smoothed field: full list, 16-bit and 8-bit codes."""
    cases = [("tube_packing", I.packing_tube(2), None), ("pbb_box 128^3", I.pbb_box(4), "field")]
    sweeps = 400
    for name, g, kind in cases:
        flags = dev_flags(g)
        for storage in ("f64", "f64s"):
            lay = tune_layout(flags, g.periodic, "lex", 0, storage, sweeps=4)
            lat = L.build(flags, g.periodic, "lex", stride=lay.stride)
            n, S = lat.n_fluid, lat.stride
            ns = torch.zeros(S, dtype=torch.float64, device="cuda")
            if kind == "field":
                ns[:n] = torch.from_numpy(g.ns.ravel()[lat.cell_of.cpu().numpy()]).cuda()
            else:
                ns[:n] = torch.rand(n, dtype=torch.float64,
                                    generator=torch.Generator().manual_seed(7)).cuda()
            prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), storage, nontemporal=lay.nontemporal,
                           xcd_chunk=lay.xcd_chunk)
            comp = L.narrow(L.compress(lat))  # word 19 is read by the c8 sweep only
            narrow, escape = code_mix(comp)
            res = {}
            for sweep in ("full", "c16", "c8"):
                st = L.init(lat, prm, ns=ns)
                step = {"full": lambda k: L.step(st, k), "c16": lambda k: L.step_c16(st, comp, k),
                        "c8": lambda k: L.step_c8(st, comp, k)}[sweep]
                step(2)
                t, _ = timed(lambda: step(sweeps))
                byt = sweep_bytes(storage, sweep, narrow, escape) + 8  # + the solid fraction
                res[sweep] = {"mflups": round(n * sweeps / t / 1e6, 1),
                              "bytes_per_update": round(byt, 2),
                              "hbm_frac": round(byt * n * sweeps / t / 1e9 / PEAK, 4)}
                del st
            emit({"experiment": "pbb", "workload": name, "n_fluid": n, "storage": storage,
                  "sweeps": sweeps, "layout": [lay.stride, lay.nontemporal, lay.xcd_chunk],
                  "narrow_cells": round(narrow, 4), "escape_cells": round(escape, 4), **res})
            del lat, comp, ns
            torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
def launch_overhead(a):
    """Where the persistent launch pays: geometries small enough that a sweep
    takes about as long as launching it (the 32^3 packing, 17 k cells) up to
    the tube (7.8 M cells); one launch per step vs one persistent launch vs
    the per-step launches captured once in a HIP graph and replayed."""
    cases = [("small_packing", I.packing_small(1), 4000),
             ("packing_64", I.packing_small(1, n=64, radius=8.0), 2000),
             ("packing_128", I.packing_small(1, n=128, radius=16.0), 1000),
             ("tube_packing", I.packing_tube(2), 200)]
    for name, g, steps in cases:
        flags = dev_flags(g)
        lat = L.build(flags, g.periodic, "lex")
        n = lat.n_fluid
        for storage in ("f64", "f32"):
            prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), storage, nontemporal=True, xcd_chunk=1)
            a1 = L.init(lat, prm)
            L.step(a1, 10)
            t_step, _ = timed(lambda: L.step(a1, steps))
            a2 = L.init(lat, prm)
            L.step(a2, 10, persistent=True)
            t_pers, _ = timed(lambda: L.step(a2, steps, persistent=True))
            a3 = L.init(lat, prm)
            L.step(a3, 10)
            chunk = min(steps, 200)  # steps per captured graph
            graph = L.StepGraph(a3, chunk)
            graph.replay()

            def replays():
                for _ in range(steps // chunk):
                    graph.replay()
            t_graph, _ = timed(replays)
            ref = L.init(lat, prm)  # the same step count eagerly
            L.step(ref, a3.steps)
            graph_equal = bool(torch.equal(ref.f[:, :n], a3.f[:, :n]))
            del ref
            emit({"experiment": "launch_overhead", "workload": name, "n_fluid": n,
                  "storage": storage, "steps": steps,
                  "us_per_step_launch": round(t_step / steps * 1e6, 2),
                  "us_per_step_persistent": round(t_pers / steps * 1e6, 2),
                  "mflups_launch": round(n * steps / t_step / 1e6, 1),
                  "mflups_persistent": round(n * steps / t_pers / 1e6, 1),
                  "persistent_speedup": round(t_step / t_pers, 3),
                  "us_per_step_graph": round(t_graph / steps * 1e6, 2),
                  "graph_speedup": round(t_step / t_graph, 3),
                  "equal": bool(torch.equal(a1.f[:, :n], a2.f[:, :n])),
                  "graph_equal": graph_equal})
            del a1, a2, a3, graph
        del lat
        torch.cuda.empty_cache()
