"""Degenerate inputs on the batched / persistent / parameter-set paths: lists
shorter than a wave or a tile, odd step counts, empty and single-cell
members, zero steps; every case against the one-launch-per-step sweep
(bitwise) and, where it is cheap, against the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1111_1129_amd import _native as N
from paper_1111_1129_amd import inputs as I
from paper_1111_1129_amd import lattice as L

from gpu_helpers import dev_flags, oracle_params, print_case, random_state, rel_err_f64

pytestmark = pytest.mark.gpu


def tiny(n_target, seed):
    rng = np.random.default_rng(seed)
    flags = np.zeros((12, 12, 12), dtype=np.uint8)
    flags.ravel()[rng.choice(flags.size, n_target, replace=False)] = 1
    return I.Geometry("tiny", flags, 7)


@pytest.mark.parametrize("n_target", [1, 63, 64, 65, 255, 256, 257, 700])
@pytest.mark.parametrize("steps", [1, 4, 7])
def test_persistent_tiny_lists_over_codes(n_target, steps):
    """A persistent launch (full list and 8-bit codes) on lists of one cell
    up to under three tiles, odd and even step counts: bitwise the per-step
    sweep, and within 1e-12 of the oracle."""
    g = tiny(n_target, n_target + 17)
    lat = L.build(dev_flags(g), g.periodic, "lex")
    n = lat.n_fluid
    print_case("persistent tiny", n, steps)
    prm = L.params(0.9, 0.25, (1e-3, -1e-3, 5e-4), "f64")
    f0 = torch.from_numpy(random_state(n, 3, stride=lat.stride)).cuda()
    ref = L.init(lat, prm)
    ref.f.copy_(f0)
    L.step(ref, steps)
    comp = L.narrow(L.compress(lat))
    for kind in ("full", "c8"):
        st = L.init(lat, prm)
        st.f.copy_(f0)
        if kind == "full":
            L.step(st, steps, persistent=True)
        else:
            L.step_c8(st, comp, steps, persistent=True)
        assert torch.equal(st.f[:, :n], ref.f[:, :n]), kind
    sp = O.build(g.flags, g.periodic, "lex", stride=lat.stride)
    orc = O.run(oracle_params(prm), sp.adj, f0.cpu().numpy(), steps, n0=0, n1=n)
    assert rel_err_f64(ref.f.cpu().numpy()[:, :n], orc[:, :n]) <= 1e-12


def test_member_sets_with_empty_and_single_cell_members():
    """A batch whose members are a packing, an empty segment, a single cell
    and another packing, each with its own parameter set: members equal their
    solo runs in both launch forms; the empty member's objective is NaN."""
    geoms = [I.packing_boolean(90, 20, 20, 20, 2.0, 4.0, 0.5), tiny(1, 5),
             I.packing_boolean(91, 17, 17, 17, 2.0, 3.0, 0.45)]
    batch = L.Batch([dev_flags(g) for g in geoms], [g.periodic for g in geoms], "lex",
                    tile_align=True)
    prms = [L.params(0.7 + 0.2 * k, 3 / 16, (1e-5 * (k + 1), 0, 0), "f64") for k in range(3)]
    # an empty segment between the members, selecting set 1
    segs = [(batch.bases[0], batch.counts[0], 0), (batch.bases[1], 0, 1),
            (batch.bases[1], batch.counts[1], 1), (batch.bases[2], batch.counts[2], 2)]
    print_case("member sets edge", batch.counts)
    outs = []
    for persistent in (False, True):
        st = L.init(batch.lattice, list(prms), n=batch.total, segments=segs)
        L.step(st, 9, persistent=persistent)
        outs.append(st)
    assert torch.equal(outs[0].f[:, :batch.total], outs[1].f[:, :batch.total])
    for k, (g, prm) in enumerate(zip(geoms, prms)):
        lat = L.build(dev_flags(g), g.periodic, "lex")
        solo = L.init(lat, prm)
        L.step(solo, 9)
        b, c = batch.bases[k], batch.counts[k]
        assert torch.equal(outs[0].f[:, b:b + c], solo.f[:, :c]), k
    J = L.objective(outs[0])
    assert J.shape == (4,) and torch.isnan(J[1]) and torch.isfinite(J[[0, 2, 3]]).all()


def test_zero_steps_and_empty_list_are_no_ops():
    g = I.packing_small(1)
    lat = L.build(dev_flags(g), g.periodic, "lex")
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f32")
    st = L.init(lat, prm)
    n = lat.n_fluid
    # the listed columns only: the padding up to the row stride is never
    # written and may hold NaN bit patterns, which compare unequal
    before = st.f[:, :n].clone()
    comp = L.narrow(L.compress(lat))
    L.step(st, 0, persistent=True)
    L.step_c8(st, comp, 0, persistent=True)
    L.step(st, 0, segments=[(0, n, 0)])
    assert torch.equal(st.f[:, :n], before)
    # n = 0 with parameter sets: nothing is launched, nothing is read
    rc, _ = N.lbm_step([prm, prm], 0, lat.stride, lat.adj, None, st.f, st.g, 3, 0, None)
    assert rc == N.LBM_OK
    assert torch.equal(st.f[:, :n], before)


def test_all_cells_in_one_member_with_set_one():
    """Set 1 for the only segment and set 0 unused: the sweep must read set 1
    everywhere (tile index table filled for every tile)."""
    g = I.packing_small(1)
    lat = L.build(dev_flags(g), g.periodic, "lex")
    n = lat.n_fluid
    unused = L.params(0.6, 3 / 16, (0, 0, 0), "f64")
    used = L.params(0.95, 3 / 16, (2e-5, 0, 0), "f64")
    st = L.init(lat, [unused, used], segments=[(0, n, 1)])
    L.step(st, 6)
    ref = L.init(lat, used)
    L.step(ref, 6)
    assert torch.equal(st.f[:, :n], ref.f[:, :n])


def test_calls_on_a_side_stream():
    """Steps with parameter sets, moments and the objective queued on a
    stream other than torch's current one, while the current stream
    allocates and writes memory (which would take over any workspace freed
    too early): results equal the same calls on the current stream."""
    geoms = [I.packing_boolean(92, 24, 24, 24, 2.0, 4.0, 0.5),
             I.packing_boolean(93, 20, 20, 20, 2.0, 3.0, 0.45)]
    batch = L.Batch([dev_flags(g) for g in geoms], [g.periodic for g in geoms], "lex",
                    tile_align=True)
    prms = [L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64"), L.params(1.1, 3 / 16, (2e-5, 0, 0), "f64")]
    segs = [(batch.bases[k], batch.counts[k], k) for k in range(2)]
    print_case("side stream", batch.counts)
    ref = L.init(batch.lattice, list(prms), n=batch.total, segments=segs)
    L.step(ref, 6)
    _, u_ref, tot_ref = L.moments(ref)
    J_ref = L.objective(ref)
    side = torch.cuda.Stream()
    st = L.init(batch.lattice, list(prms), n=batch.total, segments=segs)
    side.wait_stream(torch.cuda.current_stream())  # the state's init ran on the current stream
    L.step(st, 6, stream=side)
    _, u, tot = L.moments(st, stream=side)
    J = L.objective(st, stream=side)
    junk = [torch.full((1 << 20,), 7, dtype=torch.uint8, device="cuda") for _ in range(64)]
    side.synchronize()
    del junk
    assert torch.equal(st.f[:, :batch.total], ref.f[:, :batch.total])
    for b, c, _ in segs:  # fields are written in the members' columns only
        assert torch.equal(u[:, b:b + c], u_ref[:, b:b + c])
    assert torch.equal(tot, tot_ref) and torch.equal(J, J_ref)
