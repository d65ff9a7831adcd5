"""Throughput of the list-based D3Q19 TRT lattice Boltzmann hot path on one MI355X.

One benchmark "step" is one pass of the whole hot path over the workload:
assembly of the sparse representation from the flag field (numbering,
compaction, adjacency, adjacency codes), equilibrium initialisation, SWEEPS
pull sweeps, and the FP64 moments/totals of the final state.  The flag field
is resident in HBM before the timed region.  value = fluid-lattice updates per
second of the whole job (MFLUPS, counting fluid cells only, as the paper's
FLUP/s in Sec. 7), in double precision.

Default workload (the precision configuration): a 512 x 512 x 1024 box with
1-cell walls on the y and z faces, periodic in x, filled with overlapping
spheres of radius uniform in [8, 16] to porosity 0.40 (seed 3,
107,371,203 fluid cells), D3Q19 TRT with tau+ = 0.8, magic 3/16, body force
g_x = 1e-6, 500 sweeps from rest, FP64 storage, lexicographic ordering.  The
sweep reads the adjacency as 8-bit codes in the tiles whose codes fit a byte
and as 16-bit codes elsewhere (``--sweep c8``; results are bitwise those of
the sweep over the full uint32 list, ``--sweep full``).

After the timed loop the same 500 sweeps run once in every other storage
form (shifted FP64, FP32, shifted FP32, shifted FP16 with FP32 arithmetic,
and shifted FP16 holding 2^12 (f - w) so that small deviations stay normal);
the line's ``precision`` object gives each form's sweep rate, its speed-up
over the FP64 sweep and the relative L2 and max error of its velocity field
against the FP64 run's.  At this size the parity-checked FP64 GPU run stands
in for the oracle (its host arrays would need about 42 GB and hours); the
oracle itself runs 500 sweeps of a central crop of the same flag field (the
CPU baseline) and every form's error against it on that crop is reported too.

``--workload tube_packing`` runs the 256^3 tube of the ordering study instead
(1000 sweeps).  Experiments (``--experiment``, one JSON line per
configuration, see bench_experiments.py): precision (all forms at three force
levels), adjoint, batched, orderings, partitions, ordering_tuner, compressed,
oracle_rates, pbb, launch_overhead.

Besides the one JSON line the run reports, for the dominant kernel (the
sweep), the achieved HBM bandwidth from its algorithmic bytes (19 PDFs read +
19 written + the adjacency: 18 uint32 entries, or 18 int16 / int8 codes and
an 80-byte record per 256 cells, per fluid cell) and its average launch time
measured with HIP events on the launch stream, and a CPU baseline: the plain
FP64 oracle timed on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "MFLUPS and % of HBM peak, D3Q19 TRT sparse sweep; FP64 vs FP32/FP16 at stated error"
HBM_PEAK_GBS = 8000.0
BYTES_PER_FLUP = {"f64": 376, "f64s": 376, "f32": 224, "f32s": 224, "f16s": 148, "f16s12": 148}
PDF_SIZE = {"f64": 8, "f64s": 8, "f32": 4, "f32s": 4, "f16s": 2, "f16s12": 2}
SWEEP_KERNELS = {"full": ("k_trt", "trt.hip"), "c16": ("k_trt_c16", "compress.hip"),
                 "c8": ("k_trt_c8", "compress.hip"),
                 "inplace": ("k_gather_scatter + k_local", "inplace.hip"),
                 "inplace_c16": ("k_gather_scatter + k_local", "inplace.hip"),
                 "inplace_c8": ("k_gather_scatter + k_local", "inplace.hip")}


def sweep_bytes(storage: str, kind: str, narrow: float = 0.0, escape: float = 0.0) -> float:
    """Algorithmic bytes per cell update: 19 PDF loads + 19 stores, plus the
    adjacency: 18 uint32 (full list), or per cell of a tile 18 int8 codes
    (narrow tile, c8 only), 18 int16 codes, or 18 uint32 (tile with escapes),
    plus an 80-byte tile record per 256 cells.  narrow / escape are the
    shares of cells in narrow tiles and in tiles with escapes.  The in-place
    sweep reads the adjacency every other step."""
    if kind.endswith("c8"):
        adj = 18 * narrow + 36 * (1 - narrow - escape) + 72 * escape + 80 / 256
    elif kind.endswith("c16"):
        adj = 36 * (1 - escape) + 72 * escape + 80 / 256
    else:
        adj = 72.0
    if kind.startswith("inplace"):
        adj /= 2
    return 38 * PDF_SIZE[storage] + adj


def code_mix(comp) -> tuple[float, float]:
    """(share of cells in narrow tiles, share in tiles with escapes)."""
    if comp is None:
        return 0.0, 0.0
    rec = comp.tile_records.cpu().numpy()
    cells = np.full(len(rec), 256, dtype=np.int64)
    cells[-1] = comp.n - 256 * (len(rec) - 1)
    narrow = float(cells[rec[:, 19] != 0].sum()) / comp.n if comp.codes8 is not None else 0.0
    return narrow, float(cells[rec[:, 18] != 0].sum()) / comp.n


def kernel_sources(kind: str):
    return ["paper_1111_1129_amd/csrc/" + SWEEP_KERNELS[kind][1],
            "paper_1111_1129_amd/csrc/lbm_device.hpp"]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large_packing",
                    choices=["tube_packing", "small_packing", "large_packing", "channel"])
    ap.add_argument("--sweeps", type=int, default=0,
                    help="sweeps per pass (0: 500 for large_packing, else 1000)")
    ap.add_argument("--precision", type=int, default=1,
                    help="after the timed loop run the other storage forms once and report "
                         "speed-up and velocity error vs FP64 (headline only)")
    ap.add_argument("--order", default="lex")
    ap.add_argument("--param", type=int, default=0)
    ap.add_argument("--storage", default="f64", choices=list(BYTES_PER_FLUP))
    ap.add_argument("--sweep", default="c8", choices=list(SWEEP_KERNELS) + ["auto"],
                    help="full: two arrays, uint32 adjacency; c16: two arrays, 16-bit codes; "
                         "c8: two arrays, 8-bit codes where a tile allows them, else 16-bit; "
                         "inplace / inplace_c16 / inplace_c8: one PDF array; auto: the fastest kind "
                         "on this geometry (tuned before the timed region, with --layout tuned)")
    ap.add_argument("--layout", default="tuned", choices=["tuned", "aligned", "given"],
                    help="tuned: time candidate row strides / store policies on the geometry "
                         "first (excluded from the timed region); aligned: 128-byte aligned "
                         "stride, plain stores, contiguous eighth per XCD; given: --stride/--nt/--chunk")
    ap.add_argument("--stride", type=int, default=0, help="row stride for --layout given")
    ap.add_argument("--nt", type=int, default=1, help="nontemporal stores for --layout given")
    ap.add_argument("--chunk", type=int, default=0,
                    help="consecutive tiles per XCD for --layout given (0 = one eighth each)")
    ap.add_argument("--experiment", default="headline",
                    choices=["headline", "precision", "adjoint", "batched", "orderings",
                             "partitions", "ordering_tuner", "compressed", "oracle_rates", "pbb", "launch_overhead"],
                    help="headline: the JSON line below; the others print one JSON line per "
                         "configuration (see the module docstring)")
    ap.add_argument("--scale", type=int, default=1,
                    help="divide the large packing's (and the experiments' workloads') edge "
                         "lengths by this (quick checks)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample (0 = skip)")
    return ap.parse_args()


def code_only(text: str) -> str:
    """C++ source with comments, trailing blanks and empty lines removed."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def kernel_source_hash(kind: str) -> str:
    """Hash of the sweep's code (kernel file + device header, comments
    ignored) and of the device compile flags (include paths left out): a
    profile summary is trusted only while it matches."""
    import importlib
    build = importlib.import_module("paper_1111_1129_amd.build")
    h = hashlib.sha256()
    h.update(" ".join(f for f in build.compile_flags() if not f.startswith("-I")).encode())
    for rel in kernel_sources(kind):
        with open(os.path.join(ROOT, rel)) as fh:
            h.update(code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def profile_name(kind: str, storage: str, workload: str, order: str, what: str) -> str:
    return os.path.join(ROOT, "profiles", f"sweep_{kind}_{storage}_{workload}_{order}_{what}.txt")


def traffic_from_profile(kind: str, workload: str, order: str, storage: str):
    """HBM bytes per sweep launch from the committed PMC summary, if it was
    taken on the current kernel source (else None)."""
    path = profile_name(kind, storage, workload, order, "pmc")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_source_hash(kind):
        return None
    return float(m_bytes.group(1))


def make_workload(name: str, scale: int = 1):
    from paper_1111_1129_amd import inputs as I
    if name == "large_packing" and scale > 1:  # edges and radii divided by scale
        return (I.workload("large_packing", scale=scale),
                f"{512 // scale}x{512 // scale}x{1024 // scale} box, walls y/z, periodic x, "
                f"overlapping spheres r~U[{8 / scale:g},{16 / scale:g}] to porosity 0.40, seed 3")
    if name == "tube_packing":
        return I.packing_tube(2), "256^3 tube D=240, RSA spheres r=12, seed 2"
    if name == "small_packing":
        return I.packing_small(1), "32^3 box, RSA spheres r=4, seed 1"
    if name == "large_packing":
        return (I.workload("large_packing"),
                "512x512x1024 box, walls y/z, periodic x, overlapping spheres r~U[8,16] "
                "to porosity 0.40, seed 3")
    if name == "channel":
        return I.channel(100), "500x100x100 empty channel"
    raise KeyError(name)


def central_crop(flags: np.ndarray, edge_div: int) -> np.ndarray:
    """Central sub-box with every edge divided by edge_div (a sample of the
    same flag field for the oracle)."""
    nz, ny, nx = flags.shape
    sz, sy, sx = max(1, nz // edge_div), max(1, ny // edge_div), max(1, nx // edge_div)
    z0, y0, x0 = (nz - sz) // 2, (ny - sy) // 2, (nx - sx) // 2
    return np.ascontiguousarray(flags[z0:z0 + sz, y0:y0 + sy, x0:x0 + sx])


def cpu_baseline(geom, order, param, storage, target_s, crop_div=1, sweeps=0):
    """The oracle's FP64 sweep timed on the host cores.

    crop_div == 1: sweeps of the whole geometry until target_s has passed.
    crop_div > 1: exactly `sweeps` sweeps from rest of the central crop with
    every edge divided by crop_div (the full geometry's host arrays would not
    fit a bounded sample); the oracle's final state is returned as well, for
    the reduced-precision forms' error on the same crop.
    Returns (baseline dict, (crop flags, oracle sparse, oracle state) or None)."""
    import oracle as O
    flags = geom.flags if crop_div == 1 else central_crop(geom.flags, crop_div)
    sp = O.build(flags, geom.periodic, order, param)
    prm = O.TRT(0.8, 3.0 / 16.0, (1e-6, 0.0, 0.0))
    f = O.init(sp.n_fluid, shifted=storage.endswith("s"))
    g = np.empty_like(f)
    O.step(prm, sp.adj, f, g)  # warm (page-in)
    f = O.init(sp.n_fluid, shifted=storage.endswith("s"))
    steps = 0
    t0 = time.perf_counter()
    while True:
        O.step(prm, sp.adj, f, g)
        f, g = g, f
        steps += 1
        if (sweeps and steps >= sweeps) or (not sweeps and time.perf_counter() - t0 >= target_s):
            break
    dt = time.perf_counter() - t0
    if crop_div == 1:
        sample = (f"{steps} FP64 sweeps of the same geometry ({sp.n_fluid} fluid cells, "
                  f"{order}), {dt:.1f} s, OpenMP over cells")
    else:
        nz, ny, nx = flags.shape
        sample = (f"{steps} FP64 sweeps from rest of the central {nx}x{ny}x{nz} crop of the "
                  f"same flag field (1/{crop_div ** 3} of the box, {sp.n_fluid} fluid cells, "
                  f"{order}), {dt:.1f} s, OpenMP over cells")
    base = {"value": round(sp.n_fluid * steps / dt / 1e6, 2), "unit": "MFLUPS",
            "cores": O.max_threads(), "kind": "oracle", "sample": sample}
    return base, (None if crop_div == 1 else (flags, sp, f, prm))


def rel_errors(u, ref):
    """(relative L2, max |u - ref| / max |ref|) of two [3][n] velocity fields."""
    import torch
    d = u - ref
    return (float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(ref)),
            float(d.abs().max() / ref.abs().max()))


def print_finals(what: str, layout) -> None:
    """The tuner's finalists and their sustained rates (stderr)."""
    for (S, nt, chunk), rate in sorted(layout.finals.items(), key=lambda kv: -kv[1]):
        print(f"tune final {what}: stride={S} nt={int(nt)} chunk={chunk}: {rate:.0f} MFLUPS",
              file=sys.stderr)


def run_form(flags, geom, a, storage, kind, sweeps, layout=None):
    """One storage form: tune its layout (unless given), sweep `sweeps` times
    from rest, return (seconds per sweep, u [3][n] FP64, Layout)."""
    import torch
    from paper_1111_1129_amd import lattice as L
    from paper_1111_1129_amd.tune import Layout, Sweeper, tune_layout
    if layout is None:
        layout = (tune_layout(flags, geom.periodic, a.order, a.param, storage, sweep=kind)
                  if a.layout == "tuned" else Layout(None, False, 0))
        print_finals(f"{storage} {kind}", layout)
    lat = L.build(flags, geom.periodic, a.order, a.param, stride=layout.stride)
    sw = Sweeper(lat, kind)
    prm = L.params(0.8, 3.0 / 16.0, (1e-6, 0.0, 0.0), storage, nontemporal=layout.nontemporal,
                   xcd_chunk=layout.xcd_chunk)
    st = sw.init(prm)
    sw.step(st, 2)
    st = sw.init(prm)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sw.step(st, sweeps)
    e1.record(stream)
    e1.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / sweeps
    _, u, _ = L.moments(st)
    narrow, escape = code_mix(sw.comp)
    bpf = sweep_bytes(storage, kind, narrow, escape)
    del st, sw, lat
    return t, u, layout, bpf


def precision_leg(flags, geom, a, sweeps, u_ref, t_ref):
    """Every other storage form once over the same sweeps: rate, speed-up over
    the FP64 sweep, velocity error vs the FP64 run."""
    import torch
    forms = {}
    for storage in ("f64s", "f32", "f32s", "f16s", "f16s12"):
        kinds = (a.sweep,) if storage.startswith("f64") else (a.sweep, "inplace_c8")
        rec = {}
        for kind in dict.fromkeys(kinds):
            if kind.startswith("inplace") and sweeps % 2:
                continue
            t, u, lay, bpf = run_form(flags, geom, a, storage, kind, sweeps)
            l2, mx = rel_errors(u, u_ref)
            r = {"mflups": round(u.shape[1] / t / 1e6, 1), "speedup_vs_f64": round(t_ref / t, 3),
                 "hbm_frac": round(bpf * u.shape[1] / t / 1e9 / HBM_PEAK_GBS, 4),
                 "bytes_per_flup": round(bpf, 2), "u_rel_l2": float(f"{l2:.3e}"),
                 "u_rel_max": float(f"{mx:.3e}"),
                 "layout": {"stride": lay.stride, "nontemporal": lay.nontemporal,
                            "xcd_chunk": lay.xcd_chunk}}
            rec[kind] = r
            del u
            torch.cuda.empty_cache()
        best = max(rec, key=lambda k: rec[k]["mflups"])
        forms[storage] = dict(rec[best], sweep=best,
                              **{f"mflups_{k}": rec[k]["mflups"] for k in rec if k != best})
        print(f"precision {storage}: {forms[storage]}", file=sys.stderr, flush=True)
    return forms


def crop_vs_oracle(crop, geom, a, sweeps):
    """Every storage form on the oracle's crop: velocity error vs the oracle."""
    import torch
    import oracle as O
    flags_np, sp, f_orc, prm = crop
    _, u_orc, _ = O.moments(prm, sp.adj, f_orc)
    u_orc = torch.from_numpy(np.ascontiguousarray(u_orc)).cuda()
    flags = torch.from_numpy(flags_np).cuda()
    from paper_1111_1129_amd.tune import Layout
    out = {}
    for storage in ("f64", "f64s", "f32", "f32s", "f16s", "f16s12"):
        _, u, _, _ = run_form(flags, geom, a, storage, a.sweep, sweeps, Layout(None, False, 0))
        l2, mx = rel_errors(u, u_orc)
        out[storage] = {"u_rel_l2": float(f"{l2:.3e}"), "u_rel_max": float(f"{mx:.3e}")}
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (one MI355X); "
                                   "--gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_1111_1129_amd import _native as N
    from paper_1111_1129_amd import lattice as L

    N.load()
    if a.experiment != "headline":
        import bench_experiments
        getattr(bench_experiments, a.experiment)(a)
        return
    if not a.sweeps:
        a.sweeps = 500 if a.workload == "large_packing" else 1000
    dev = torch.device("cuda:0")
    geom, desc = make_workload(a.workload, a.scale)
    print(f"workload {a.workload}: {geom.n_fluid} fluid cells", file=sys.stderr, flush=True)
    flags = torch.from_numpy(np.ascontiguousarray(geom.flags)).to(dev)
    lay = None
    if a.sweep == "auto":
        if a.layout != "tuned":
            print(json.dumps({"error": "--sweep auto needs --layout tuned"}))
            sys.exit(2)
        from paper_1111_1129_amd.tune import tune_sweep
        kind, lay, rates = tune_sweep(flags, geom.periodic, a.order, a.param, a.storage)
        if kind.startswith("inplace") and a.sweeps % 2:  # needs an even sweep count
            kind, lay = max(("c8", "c16", "full"), key=lambda k: rates.get(k, 0.0)), None
        print("sweep kinds (MFLUPS): %s -> %s" % (rates, kind), file=sys.stderr)
        a.sweep = kind
    if a.layout == "tuned":
        from paper_1111_1129_amd.tune import tune_layout
        if lay is None:
            lay = tune_layout(flags, geom.periodic, a.order, a.param, a.storage, sweep=a.sweep)
        stride, nt, chunk = lay.stride, lay.nontemporal, lay.xcd_chunk
        for row in lay.table:
            print("tune stride=%d nt=%d chunk=%d: %.0f MFLUPS" % row, file=sys.stderr)
        print_finals(f"{a.storage} {a.sweep}", lay)
    elif a.layout == "given":
        stride, nt, chunk = (a.stride or None), bool(a.nt), a.chunk
    else:
        stride, nt, chunk = None, False, 0
    prm = L.params(0.8, 3.0 / 16.0, (1e-6, 0.0, 0.0), a.storage, nontemporal=nt, xcd_chunk=chunk)
    stream = torch.cuda.current_stream()
    from paper_1111_1129_amd.tune import Layout, Sweeper
    if a.sweep.startswith("inplace") and a.sweeps % 2:
        print(json.dumps({"error": "the in-place sweep needs an even --sweeps"}))
        sys.exit(2)

    def one_pass(ev=None):
        lat = L.build(flags, geom.periodic, a.order, a.param, stride=stride)
        sw = Sweeper(lat, a.sweep)  # builds the codes for the c16 / c8 kinds
        st = sw.init(prm)
        if ev is not None:
            ev[0].record(stream)
        sw.step(st, a.sweeps)
        if ev is not None:
            ev[1].record(stream)
        _, _, totals = L.moments(st, fields=False)
        return lat, sw, st, totals

    for k in range(a.warmup):
        one_pass()
        print(f"warmup pass {k + 1}/{a.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        lat, sw, st, totals = one_pass(events[k])
        if (k + 1) % 5 == 0 or k + 1 == a.steps:
            print(f"timed pass {k + 1}/{a.steps} queued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_fluid = lat.n_fluid
    sweep_ms = np.mean([e0.elapsed_time(e1) for e0, e1 in events])
    launch_s = sweep_ms / 1e3 / a.sweeps
    tot = totals.cpu().numpy()[0]
    if not np.isfinite(tot).all():
        print(json.dumps({"error": "non-finite totals", "totals": tot.tolist()}))
        sys.exit(1)

    flups = n_fluid * a.sweeps * a.steps
    value = flups / wall / 1e6
    narrow, escape = code_mix(sw.comp)
    bpf = sweep_bytes(a.storage, a.sweep, narrow, escape)
    achieved = bpf * n_fluid / launch_s / 1e9
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "MFLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.storage.startswith("f64") else "f32",  # arithmetic type
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: {desc}", "n_fluid": n_fluid,
                   "sweeps_per_step": a.sweeps, "order": a.order, "order_param": a.param,
                   "storage": a.storage, "sweep": a.sweep,
                   "code_tiles": {"narrow_cells": round(narrow, 4), "escape_cells": round(escape, 4)},
                   "tau_plus": 0.8, "magic": 0.1875, "force_x": 1e-6,
                   "layout": a.layout, "row_stride": lat.stride, "nontemporal": nt,
                   "xcd_chunk": chunk},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profile(a.sweep, a.workload, a.order, a.storage),
                     "kernel": SWEEP_KERNELS[a.sweep][0] + " (one sweep launch)",
                     "bytes_per_flup": round(bpf, 2),
                     "sweep_mflups": round(n_fluid / launch_s / 1e6, 1),
                     "avg_launch_us": round(launch_s * 1e6, 2)},
        "cpu_baseline": None,
    }
    if a.precision and a.storage == "f64":
        # reference velocity of the FP64 run (the last timed pass's state)
        _, u_ref, _ = L.moments(st)
        del lat, sw, st
        torch.cuda.empty_cache()
        forms = precision_leg(flags, geom, a, a.sweeps, u_ref, launch_s)
        line["precision"] = {
            "reference": f"the FP64 run ({a.sweep} sweep, {a.sweeps} sweeps from rest, g_x = 1e-6) "
                         "stands in for the oracle at this size; its sweep is parity-checked "
                         "against the oracle (1e-12) on the tube, the crop and sampled ranges of "
                         "this workload",
            "f64": {"mflups": round(n_fluid / launch_s / 1e6, 1), "sweep": a.sweep,
                    "hbm_frac": round(achieved / HBM_PEAK_GBS, 4)},
            **forms}
        del u_ref
        torch.cuda.empty_cache()
    if a.cpu_seconds > 0:
        crop_div = 4 if a.workload == "large_packing" else 1
        base, crop = cpu_baseline(geom, a.order, a.param, a.storage, a.cpu_seconds, crop_div,
                                  a.sweeps if crop_div > 1 else 0)
        line["cpu_baseline"] = base
        if crop is not None and "precision" in line:
            line["precision"]["vs_oracle_on_crop"] = crop_vs_oracle(crop, geom, a, a.sweeps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
