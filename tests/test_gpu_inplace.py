"""In-place sweep (one PDF array): after an even number of steps it is
bitwise the two-array sweep, and so within the FP64 tolerance of the oracle;
odd step counts continue correctly."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1111_1129_amd import inputs as I
from paper_1111_1129_amd import lattice as L

from gpu_helpers import dev_flags, oracle_params, print_case, random_state, rel_err_f64

pytestmark = pytest.mark.gpu


def two_array(lat, prm, f0, steps, ns=None):
    st = L.init(lat, prm, ns=ns)
    if f0 is not None:
        st.f.copy_(f0)
    L.step(st, steps)
    return st.f[:, :lat.n_fluid]


def one_array(lat, prm, f0, steps, ns=None, comp=None, split=None, c8=False):
    st = L.init_inplace(lat, prm, ns=ns)
    if f0 is not None:
        st.f.copy_(f0)
    for k in (split or [steps]):
        L.step_inplace(st, k, comp, c8=c8)
    assert st.phase == steps % 2
    return st


@pytest.mark.parametrize("storage", ["f64", "f64s", "f32", "f32s", "f16s", "f16s12"])
@pytest.mark.parametrize("codes", ["adj", "c16", "c8"])
def test_even_steps_bitwise_equal_two_array(storage, codes):
    """Lexicographic order of a fully periodic box: narrow, 16-bit and escape
    tiles in one list."""
    g = I.random_flags(11, 64, 64, 48, 0.7)
    print_case("inplace", storage, codes, "random_flags 64x64x48 periodic xyz")
    lat = L.build(dev_flags(g), 7, "lex", 0)
    comp = None if codes == "adj" else L.compress(lat)
    if codes == "c8":
        L.narrow(comp)
        assert 0 < comp.n_narrow < comp.n_tiles and comp.n_escapes > 0
    prm = L.params(0.8, 3 / 16, (1e-5, 2e-6, 0), storage)
    ref = two_array(lat, prm, None, 10)
    st = one_array(lat, prm, None, 10, comp=comp, c8=codes == "c8")
    assert torch.equal(st.f[:, :lat.n_fluid], ref)


@pytest.mark.parametrize("split", [[1, 1], [3, 5], [7, 1, 2]])
def test_odd_step_counts_continue(split):
    """Stops in phase 1 are resumed; the total is even, so the result is the
    two-array state."""
    g = I.packing_small(1)
    print_case("inplace", "split", split)
    lat = L.build(dev_flags(g), g.periodic, "morton2", 0)
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64", nontemporal=True, xcd_chunk=1)
    f0 = torch.from_numpy(random_state(lat.n_fluid, 6, stride=lat.stride)).cuda()
    total = sum(split)
    ref = two_array(lat, prm, f0, total)
    st = one_array(lat, prm, f0, total, split=split)
    assert torch.equal(st.f[:, :lat.n_fluid], ref)


def test_vs_oracle_with_pbb_and_escapes():
    """Random ordering: most codes escape, so the full-list path of the
    gather-scatter step runs too; PBB blends with the bounce-back."""
    g = I.random_flags(11, 64, 64, 48, 0.7)
    print_case("inplace", "oracle", "random_flags 64x64x48 random order, pbb")
    lat = L.build(dev_flags(g), g.periodic, "random", 9)
    sp = O.build(g.flags, g.periodic, "random", 9, stride=lat.stride)
    n = sp.n_fluid
    comp = L.compress(lat)
    assert comp.n_escapes > 0
    ns_h = np.zeros(lat.stride)
    ns_h[:n] = np.random.default_rng(8).uniform(0, 1, n)
    ns = torch.from_numpy(ns_h).cuda()
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64s")
    f0 = random_state(n, 9, amp=1e-3, shifted=True, stride=lat.stride)
    st = one_array(lat, prm, torch.from_numpy(f0).cuda(), 24, ns=ns, comp=comp)
    orc = O.run(oracle_params(prm), sp.adj, f0, 24, ns=ns_h, n0=0, n1=n)
    assert rel_err_f64(st.f.cpu().numpy()[:, :n], orc[:, :n], shifted=True) <= 1e-12


@pytest.mark.parametrize("n_target", [1, 255, 257])
@pytest.mark.parametrize("c8", [False, True])
def test_tiny_lists(n_target, c8):
    flags = np.zeros((8, 8, 8), dtype=np.uint8)
    flags.ravel()[:n_target] = 1
    print_case("inplace", "tiny", n_target, "c8" if c8 else "c16")
    lat = L.build(torch.from_numpy(flags).cuda(), 7, "lex", 0)
    prm = L.params(0.8, 3 / 16, (1e-4, 0, 0), "f64")
    f0 = torch.from_numpy(random_state(lat.n_fluid, 4, stride=lat.stride)).cuda()
    ref = two_array(lat, prm, f0, 4)
    comp = L.compress(lat)
    if c8:
        L.narrow(comp)
    st = one_array(lat, prm, f0, 4, comp=comp, c8=c8)
    assert torch.equal(st.f[:, :lat.n_fluid], ref)


def test_c8_vs_oracle_with_pbb():
    """In place over 8-bit codes (with 16-bit and escape tiles in the list)
    against the oracle, partial bounce-back on."""
    g = I.random_flags(12, 64, 64, 48, 0.7)
    print_case("inplace", "oracle c8", "random_flags 64x64x48 periodic xyz, pbb")
    lat = L.build(dev_flags(g), 7, "lex", 0)
    sp = O.build(g.flags, 7, "lex", 0, stride=lat.stride)
    n = sp.n_fluid
    comp = L.narrow(L.compress(lat))
    assert 0 < comp.n_narrow < comp.n_tiles and comp.n_escapes > 0
    ns_h = np.zeros(lat.stride)
    ns_h[:n] = np.random.default_rng(18).uniform(0, 1, n)
    ns = torch.from_numpy(ns_h).cuda()
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64s")
    f0 = random_state(n, 19, amp=1e-3, shifted=True, stride=lat.stride)
    st = one_array(lat, prm, torch.from_numpy(f0).cuda(), 24, ns=ns, comp=comp, c8=True)
    orc = O.run(oracle_params(prm), sp.adj, f0, 24, ns=ns_h, n0=0, n1=n)
    assert rel_err_f64(st.f.cpu().numpy()[:, :n], orc[:, :n], shifted=True) <= 1e-12


def test_batch_of_geometries():
    """Cells of several geometries in one list: each scatters only into its own."""
    geoms = I.batch_packings(count=4, l_min=24, l_max=40)
    flags = [dev_flags(g) for g in geoms]
    print_case("inplace", "batch", 4)
    batch = L.Batch(flags, [g.periodic for g in geoms], "lex")
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f32s")
    ref = batch.init(prm)
    L.step(ref, 6)
    st = L.init_inplace(batch.lattice, prm, n=batch.total)
    L.step_inplace(st, 6)
    assert torch.equal(st.f[:, :batch.total], ref.f[:, :batch.total])


def test_full_size_tube():
    g = I.packing_tube(2)
    print_case("inplace", "tube", "256^3")
    lat = L.build(dev_flags(g), g.periodic, "lex", 0)
    comp = L.compress(lat)
    prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), "f64", nontemporal=True, xcd_chunk=1)
    ref = two_array(lat, prm, None, 20).clone()
    st = one_array(lat, prm, None, 20, comp=comp)
    torch.cuda.synchronize()
    assert torch.equal(st.f[:, :lat.n_fluid], ref)
    _, _, tot = L.moments(st, fields=False)
    assert abs(float(tot[0, 0]) / lat.n_fluid - 1.0) < 1e-12  # mass is conserved
    del st
    L.narrow(comp)
    st = one_array(lat, prm, None, 20, comp=comp, c8=True)
    torch.cuda.synchronize()
    assert torch.equal(st.f[:, :lat.n_fluid], ref)


def test_sweeper_kinds_and_tuner():
    """Every sweep kind the tuner and the benchmark use ends in the same state;
    the tuner returns an aligned stride and a valid store/XCD choice."""
    from paper_1111_1129_amd.tune import SWEEPS, Sweeper, tune_layout
    g = I.packing_small(1)
    flags = dev_flags(g)
    print_case("inplace", "sweeper kinds + tuner")
    lat = L.build(flags, g.periodic, "lex", 0)
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f32s")
    finals = []
    for kind in SWEEPS:
        sw = Sweeper(lat, kind)
        st = sw.init(prm)
        sw.step(st, 6)
        finals.append(st.f[:, :lat.n_fluid].clone())
    for f in finals[1:]:
        assert torch.equal(f, finals[0])
    lay = tune_layout(flags, g.periodic, "lex", 0, "f32s", sweeps=2, chunks=(1, 0), finalists=2,
                      sweep="c16")
    assert lay.stride >= lat.n_fluid and lay.stride % 64 == 0
    assert lay.xcd_chunk in (1, 0) and lay.mflups > 0
    # every candidate stride reaches the sustained finals
    from paper_1111_1129_amd.tune import candidate_strides
    assert {key[0] for key in lay.finals} == set(candidate_strides(lat.n_fluid))
    assert (lay.stride, lay.nontemporal, lay.xcd_chunk) in lay.finals
