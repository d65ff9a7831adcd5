"""Sweeps captured in a HIP graph: every replay, with eager work and
synchronisations between replays, ends in bitwise the state of the same
eager calls."""
import pytest
import torch

from paper_1111_1129_amd import inputs as I
from paper_1111_1129_amd import lattice as L

from gpu_helpers import dev_flags, print_case

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("codes", ["full", "c16", "c8"])
@pytest.mark.parametrize("storage", ["f64", "f16s"])
def test_graph_replays_match_eager_steps(codes, storage):
    g = I.packing_small(1)
    print_case("graph", codes, storage)
    lat = L.build(dev_flags(g), g.periodic, "lex", 0)
    n = lat.n_fluid
    comp = None
    if codes != "full":
        comp = L.compress(lat)
        if codes == "c8":
            L.narrow(comp)
    prm = L.params(0.8, 3 / 16, (1e-5, 2e-6, 0), storage, nontemporal=True, xcd_chunk=1)
    ref = L.init(lat, prm)
    st = L.init(lat, prm)
    graph = L.StepGraph(st, 10, comp)
    assert st.steps == 0  # capture runs nothing
    for r in range(4):
        graph.replay()
        L.step(ref, 10)                          # eager work between replays
        _, _, tot = L.moments(st, fields=False)  # eager library work on the graph's state
        torch.cuda.synchronize()
        assert torch.equal(st.f[:, :n], ref.f[:, :n]), r
        assert torch.isfinite(tot).all()
    assert st.steps == 40


@pytest.mark.parametrize("codes", ["full", "c8"])
def test_graph_of_a_batch_with_parameter_sets(codes):
    """A batch whose members keep their own tau+ and force, captured once:
    every replay equals the same eager steps, bitwise."""
    geoms = [I.packing_boolean(40 + k, e, e, e, 2.0, 4.0, 0.5) for k, e in enumerate((19, 26, 13))]
    batch = L.Batch([dev_flags(g) for g in geoms], [g.periodic for g in geoms], "lex",
                    tile_align=True)
    prms = [L.params(0.7 + 0.15 * k, 3 / 16, (1e-5 * (k + 1), 0, 0), "f32s") for k in range(3)]
    comp = None
    if codes == "c8":
        comp = L.narrow(L.compress(batch.lattice, n=batch.total))
    print_case("graph batch", codes, batch.total)
    ref = batch.init(prms)
    st = batch.init(prms)
    graph = L.StepGraph(st, 8, comp)
    for r in range(3):
        graph.replay()
        if comp is None:
            L.step(ref, 8)
        else:
            L.step_c8(ref, comp, 8)
        torch.cuda.synchronize()
        assert torch.equal(st.f[:, :batch.total], ref.f[:, :batch.total]), r


def test_graph_with_partial_bounce_back():
    g = I.pbb_box(4, n=24)
    lat = L.build(dev_flags(g), g.periodic, "lex", 0)
    n, S = lat.n_fluid, lat.stride
    ns = torch.zeros(S, dtype=torch.float64, device="cuda")
    ns[:n] = torch.from_numpy(g.ns.ravel()[lat.cell_of.cpu().numpy()]).cuda()
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64s")
    comp = L.narrow(L.compress(lat))
    ref = L.init(lat, prm, ns=ns)
    st = L.init(lat, prm, ns=ns)
    graph = L.StepGraph(st, 6, comp)
    for r in range(3):
        graph.replay()
        L.step_c8(ref, comp, 6)
        torch.cuda.synchronize()
        assert torch.equal(st.f[:, :n], ref.f[:, :n]), r
