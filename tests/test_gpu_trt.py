"""GPU TRT sweep, moments and reduced-precision storage vs the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1111_1129_amd import inputs as I
from paper_1111_1129_amd import lattice as L

from gpu_helpers import W, dev_flags, oracle_params, print_case, random_state, rel_err_f64

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-12  # relative, on unshifted PDF values


def pair(g, order="lex", param=0):
    """GPU lattice and oracle sparse representation with the same row stride."""
    lat = L.build(dev_flags(g), g.periodic, order, param)
    return O.build(g.flags, g.periodic, order, param, stride=lat.stride), lat


@pytest.fixture(scope="module")
def small():
    g = I.packing_small(1)
    sp, lat = pair(g)
    return g, sp, lat


def run_gpu(lat, prm, f0, steps, ns=None, persistent=False):
    st = L.init(lat, prm, ns=ns)
    st.f.copy_(torch.from_numpy(f0))
    L.step(st, steps, persistent=persistent)
    return st


def orun(prm, sp, f0, steps, ns=None):
    return O.run(oracle_params(prm), sp.adj, f0, steps, ns=ns, n0=0, n1=sp.n_fluid)


def cells(a, n):
    return a[:, :n]


@pytest.mark.parametrize("storage", ["f64", "f64s"])
def test_small_packing_100_steps_from_rest(small, storage):
    g, sp, lat = small
    shifted = storage == "f64s"
    prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), storage)
    print_case("trt", storage, "small_packing", 100)
    st = L.init(lat, prm)
    n = sp.n_fluid
    f0 = O.init(n, stride=lat.stride, shifted=shifted)
    np.testing.assert_array_equal(cells(st.f.cpu().numpy(), n), cells(f0, n))
    L.step(st, 100)
    orc = orun(prm, sp, f0, 100)
    assert rel_err_f64(cells(st.f.cpu().numpy(), n), cells(orc, n), shifted) <= TOL_F64


def test_small_packing_random_state_ragged_n(small):
    g, sp, lat = small
    assert sp.n_fluid % 256 != 0  # a ragged last workgroup
    prm = L.params(0.8, 3 / 16, (1e-4, 2e-5, -1e-5), "f64")
    n = sp.n_fluid
    f0 = random_state(n, 1, stride=lat.stride)
    st = run_gpu(lat, prm, f0, 37)
    orc = orun(prm, sp, f0, 37)
    assert rel_err_f64(cells(st.f.cpu().numpy(), n), cells(orc, n)) <= TOL_F64


@pytest.mark.parametrize("order,param", [("blocked", 8), ("morton2", 0), ("random", 5)])
def test_other_orderings(order, param):
    g = I.packing_small(1)
    sp, lat = pair(g, order, param)
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64")
    n = sp.n_fluid
    f0 = random_state(n, 2, stride=lat.stride)
    st = run_gpu(lat, prm, f0, 20)
    orc = orun(prm, sp, f0, 20)
    assert rel_err_f64(cells(st.f.cpu().numpy(), n), cells(orc, n)) <= TOL_F64


@pytest.mark.parametrize("n_target", [1, 63, 64, 65, 255, 257, 700])
def test_tiny_lists(n_target):
    """Lists shorter than a wave, exactly a wave, just above, and ragged."""
    rng = np.random.default_rng(n_target)
    flags = np.zeros((12, 12, 12), dtype=np.uint8)
    idx = rng.choice(flags.size, n_target, replace=False)
    flags.ravel()[idx] = 1
    g = I.Geometry("tiny", flags, 7)
    sp, lat = pair(g, "morton1")
    prm = L.params(0.9, 0.25, (1e-3, -1e-3, 5e-4), "f64")
    n = sp.n_fluid
    f0 = random_state(n, 3, stride=lat.stride)
    st = run_gpu(lat, prm, f0, 5)
    orc = orun(prm, sp, f0, 5)
    assert rel_err_f64(cells(st.f.cpu().numpy(), n), cells(orc, n)) <= TOL_F64


def test_pbb(small):
    g, sp, lat = small
    rng = np.random.default_rng(4)
    n = sp.n_fluid
    ns = np.zeros(lat.stride)
    ns[:n] = rng.uniform(0, 1, n)
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64s")
    f0 = random_state(n, 5, amp=1e-3, shifted=True, stride=lat.stride)
    st = run_gpu(lat, prm, f0, 25, ns=torch.from_numpy(ns).cuda())
    orc = orun(prm, sp, f0, 25, ns=ns)
    assert rel_err_f64(cells(st.f.cpu().numpy(), n), cells(orc, n), shifted=True) <= TOL_F64


def test_launch_variants_are_bitwise_identical(small):
    """Nontemporal stores, the XCD chunk mapping and the persistent launch change
    only where/how cells are processed, not their arithmetic."""
    g, sp, lat = small
    n = sp.n_fluid
    f0 = random_state(n, 6, stride=lat.stride)
    outs = []
    for nt, chunk, pers in [(False, 0, False), (True, 0, False), (False, 1, False), (True, 4, False),
                            (False, 2, False), (False, 0, True), (True, 0, True)]:
        prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64", nontemporal=nt, xcd_chunk=chunk)
        outs.append(cells(run_gpu(lat, prm, f0, 9, persistent=pers).f.cpu().numpy(), n))
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


def test_rest_mass_and_uniform_force_on_gpu():
    g = I.packing_small(1)
    lat = L.build(dev_flags(g), g.periodic, "lex")
    n = lat.n_fluid
    st = L.init(lat, L.params(0.8, 3 / 16, (0, 0, 0), "f64s"))
    L.step(st, 50)
    assert not st.f[:, :n].any().item()  # shifted rest state is exactly preserved
    prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), "f64")
    st = L.init(lat, prm)
    m0 = st.f[:, :n].sum().item()
    L.step(st, 100)
    assert abs(st.f[:, :n].sum().item() - m0) <= 1e-12 * m0
    # all-fluid periodic box forced from rest: u = (t + 1/2) G
    box = I.all_fluid(6, 5, 4)
    latb = L.build(dev_flags(box), 7, "lex")
    G = (1e-5, -2e-5, 3e-5)
    stb = L.init(latb, L.params(0.8, 3 / 16, G, "f64s"))
    L.step(stb, 20)
    _, u, tot = L.moments(stb)
    expect = 20.5 * np.array(G)
    np.testing.assert_allclose(u.cpu().numpy().T, np.tile(expect, (latb.n_fluid, 1)), rtol=1e-13)


def test_poiseuille_on_gpu():
    H = 8
    g = I.plate_channel(H, nx=3, nz=2)
    lat = L.build(dev_flags(g), g.periodic, "lex")
    gx = 1e-6
    st = L.init(lat, L.params(0.8, 3 / 16, (gx, 0, 0), "f64s"))
    L.step(st, 16000)
    _, u, _ = L.moments(st)
    y = (lat.cell_of.cpu().numpy() // 3) % (H + 2)
    exact = gx / (2 * 0.1) * (y - 0.5) * (H + 0.5 - y)
    np.testing.assert_allclose(u[0].cpu().numpy(), exact, rtol=1e-9)


def encode(f64: np.ndarray, storage: str) -> np.ndarray:
    """Host values -> the array a storage form keeps (exactly representable
    inputs: round_storage first)."""
    if storage == "f16s12":
        return (f64 * 4096.0).astype(np.float16)
    dt = {"f64": np.float64, "f64s": np.float64, "f32": np.float32, "f32s": np.float32,
          "f16s": np.float16}[storage]
    return f64.astype(dt)


def decode(stored: np.ndarray, storage: str) -> np.ndarray:
    out = stored.astype(np.float64)
    return out / 4096.0 if storage == "f16s12" else out


def storage_shifted(storage: str) -> bool:
    return storage in ("f64s", "f32s", "f16s", "f16s12")


@pytest.mark.parametrize("storage", ["f64", "f64s", "f32", "f16s", "f16s12"])
def test_moments_vs_oracle(small, storage):
    g, sp, lat = small
    shifted = storage_shifted(storage)
    prm = L.params(0.8, 3 / 16, (1e-5, 2e-6, 0), storage)
    n = sp.n_fluid
    f0 = O.round_storage(random_state(n, 7, amp=1e-2, shifted=shifted, stride=lat.stride), storage)
    st = L.init(lat, prm)
    st.f.copy_(torch.from_numpy(encode(f0, storage)))
    rho, u, tot = L.moments(st)
    orho, ou, otot = O.moments(oracle_params(prm), sp.adj, f0, shifted, 0, n)
    np.testing.assert_allclose(rho.cpu().numpy(), orho, rtol=1e-14, atol=0)
    np.testing.assert_allclose(u.cpu().numpy(), ou, rtol=0, atol=1e-16)
    t = tot.cpu().numpy()[0]
    np.testing.assert_allclose(t[0], otot[0], rtol=1e-15)
    np.testing.assert_allclose(t[1:], otot[1:], rtol=0, atol=1e-15 * np.abs(ou).sum())


def test_moments_segments_and_determinism(small):
    g, sp, lat = small
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64")
    f = random_state(sp.n_fluid, 8, stride=lat.stride)
    st = L.init(lat, prm)
    st.f.copy_(torch.from_numpy(f))
    n = sp.n_fluid
    segs = [(0, 1000), (1000, 1), (1001, n - 1001)]
    _, _, t1 = L.moments(st, segments=segs)
    _, _, t2 = L.moments(st, segments=segs)
    assert torch.equal(t1, t2)
    for k, (b, c) in enumerate(segs):
        _, _, ot = O.moments(oracle_params(prm), sp.adj, f, False, b, b + c)
        np.testing.assert_allclose(t1[k].cpu().numpy(), ot, rtol=1e-13, atol=1e-18)


def storage_ulp(x: np.ndarray, storage: str) -> np.ndarray:
    """Spacing of the storage grid at |x| (FP64 values)."""
    if storage == "f16s12":
        return np.spacing(np.abs(x * 4096.0).astype(np.float16)).astype(np.float64) / 4096.0
    dt = np.float16 if storage == "f16s" else np.float32
    return np.spacing(np.abs(x).astype(dt)).astype(np.float64)


@pytest.mark.parametrize("storage", ["f32", "f32s", "f16s", "f16s12"])
def test_reduced_precision_one_step(small, storage):
    """One step from a stored FP32/FP16 state: the GPU computes in FP32, the
    oracle in FP64 on the same widened inputs and rounds to the storage type.
    Bound: one storage ulp of the result (the rounding decision may differ)
    plus the FP32 evaluation error, 64 eps32 of the largest value involved."""
    g, sp, lat = small
    shifted = storage_shifted(storage)
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), storage)
    n = sp.n_fluid
    f0 = O.round_storage(random_state(n, 9, amp=2e-2, shifted=shifted, stride=lat.stride), storage)
    st = L.init(lat, prm)
    st.f.copy_(torch.from_numpy(encode(f0, storage)))
    L.step(st, 1)
    gpu = cells(decode(st.f.cpu().numpy(), storage), n)
    exact = cells(orun(prm, sp, f0, 1), n)
    f0 = cells(f0, n)
    orc = O.round_storage(exact, storage)
    scale = np.abs(f0).max() if shifted else 1.0
    tol = storage_ulp(exact, storage) + 64 * np.finfo(np.float32).eps * scale
    assert (np.abs(gpu - orc) <= tol).all()
    # and the result is not trivially the input
    assert np.abs(gpu - f0).max() > 10 * tol.max()


def test_scaled_fp16_keeps_small_deviations():
    """At body force 1e-6 the deviations f - w fall below FP16's normal range;
    the scaled form keeps them, the plain shifted form rounds them to a
    subnormal grid: after 200 sweeps its velocity is far closer to FP64's."""
    g = I.packing_small(1)
    lat = L.build(dev_flags(g), g.periodic, "lex")
    u = {}
    for storage in ("f64s", "f16s", "f16s12"):
        st = L.init(lat, L.params(0.8, 3 / 16, (1e-6, 0, 0), storage))
        L.step(st, 200)
        u[storage] = L.moments(st)[1]
    err = {k: float(torch.linalg.vector_norm(u[k] - u["f64s"]) / torch.linalg.vector_norm(u["f64s"]))
           for k in ("f16s", "f16s12")}
    print_case("scaled fp16 error", err)
    assert err["f16s12"] < 0.2 * err["f16s"]


def sampled_step_vs_oracle(lat, sp, prm, st, advance, ranges, seed):
    """One GPU step (`advance`) from a seeded state, compared on sampled cell
    ranges with the oracle's step of the same state.

    The state is the rest weights everywhere except the slots the sampled
    cells read -- located through the oracle's own adjacency `sp` -- which get
    seeded random values; both sides take their inputs from that one table,
    and the oracle steps the sampled cells through an identity adjacency."""
    S = lat.stride
    # distinct cells (ranges may overlap): every slot then belongs to one cell
    cells = np.unique(np.concatenate([np.arange(a, b) for a, b in ranges])).astype(np.int64)
    k = cells.size
    slots = np.empty((19, k), dtype=np.int64)
    slots[0] = cells                                   # rest population: own slot of row 0
    slots[1:] = sp.adj[:, cells].astype(np.int64)      # the oracle's pull adjacency
    rows = slots // S
    rng = np.random.default_rng(seed)
    vals = W[rows] * (1.0 + 0.02 * rng.standard_normal(slots.shape))
    w_dev = torch.from_numpy(W).cuda()
    st.f.copy_(w_dev[:, None].expand(19, S))
    st.f.view(-1)[torch.from_numpy(slots.ravel()).cuda()] = torch.from_numpy(vals.ravel()).cuda()
    advance()
    got = st.f[:, torch.from_numpy(cells).cuda()].cpu().numpy()
    ident = ((np.arange(1, 19, dtype=np.uint64)[:, None] * k + np.arange(k, dtype=np.uint64)[None, :])
             .astype(np.uint32))
    orc = np.zeros_like(vals)
    O.step(oracle_params(prm), ident, np.ascontiguousarray(vals), orc)
    return rel_err_f64(got, orc)


@pytest.mark.parametrize("sweep,stride,chunk", [("c8", 8396800, 4), ("c16", 8389632, 1)])
def test_full_size_tube_sampled_step(sweep, stride, chunk):
    """The full 256^3 tube in the benchmark's launch configurations (sweep
    over 8-bit codes in narrow tiles: row stride 2^23 + 8192, nontemporal
    stores, XCD chunk 4; over 16-bit codes: 2^23 + 1024, chunk 1): one GPU
    step from a seeded state compared on sampled cell ranges (head, middle,
    ragged tail) with the oracle; then 20 more steps conserve mass."""
    g = I.packing_tube(2)
    lat = L.build(dev_flags(g), g.periodic, "lex", stride=stride)
    sp = O.build(g.flags, g.periodic, "lex", stride=lat.stride)
    n = lat.n_fluid
    assert n == sp.n_fluid
    prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), "f64", nontemporal=True, xcd_chunk=chunk)
    print_case("tube full size", sweep, n)
    comp = L.compress(lat)
    if sweep == "c8":
        L.narrow(comp)
        assert comp.n_narrow > 0.8 * comp.n_tiles
        advance = lambda k: L.step_c8(st, comp, k)  # noqa: E731
    else:
        advance = lambda k: L.step_c16(st, comp, k)  # noqa: E731
    st = L.init(lat, prm)
    ranges = [(0, 4096), (n // 3, n // 3 + 3000), (n // 2 + 17, n // 2 + 5000), (n - 2049, n)]
    err = sampled_step_vs_oracle(lat, sp, prm, st, lambda: advance(1), ranges, 10)
    assert err <= TOL_F64
    mass0 = float(st.f[:, :n].sum())
    advance(20)
    assert abs(float(st.f[:, :n].sum()) - mass0) <= 1e-12 * mass0


def test_full_size_tube_whole_state_10_sweeps():
    """The full 256^3 tube (7,797,209 cells) in the tuned launch configuration
    of its sweep over 8-bit codes (row stride 2^23 + 8192, nontemporal
    stores, XCD chunk 4): 10 FP64 sweeps from a seeded random state, every
    one of the 19 x 7,797,209 PDFs within 1e-12 of the oracle."""
    g = I.packing_tube(2)
    lat = L.build(dev_flags(g), g.periodic, "lex", stride=8396800)
    sp = O.build(g.flags, g.periodic, "lex", stride=lat.stride)
    n = lat.n_fluid
    assert n == sp.n_fluid == 7797209
    print_case("tube whole state", n)
    comp = L.narrow(L.compress(lat))
    prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), "f64", nontemporal=True, xcd_chunk=4)
    f0 = random_state(n, 31, stride=lat.stride)
    st = L.init(lat, prm)
    st.f.copy_(torch.from_numpy(f0))
    L.step_c8(st, comp, 10)
    got = st.f.cpu().numpy()
    del st
    orc = orun(prm, sp, f0, 10)
    assert rel_err_f64(cells(got, n), cells(orc, n)) <= TOL_F64


@pytest.fixture(scope="module")
def large():
    """The 512x512x1024 packing (107 M cells) on the GPU and its oracle
    sparse representation, built once on the host."""
    g = I.workload("large_packing")
    lat = L.build(dev_flags(g), g.periodic, "lex")
    sp = O.build(g.flags, g.periodic, "lex", stride=lat.stride)
    assert sp.n_fluid == lat.n_fluid
    comp = L.narrow(L.compress(lat))
    assert 0 < comp.n_narrow < comp.n_tiles
    yield lat, sp, comp
    del lat, sp, comp
    torch.cuda.empty_cache()


def special_ranges(lat, comp):
    """Cell ranges that a sample of the large packing must cover besides its
    head, middle and tail: a tile read through 16-bit codes (not narrow), and
    a row next to the y = 0 wall in the middle plane (bounce-back from the
    wall layer; the head and tail planes lie next to the z walls)."""
    rec = comp.tile_records.cpu().numpy()
    wide = np.flatnonzero((rec[:, 19] == 0) & (rec[:, 18] == 0))
    assert wide.size > 0
    t = int(wide[wide.size // 2])
    nx, ny, nz = lat.dims
    index_of = lat.index_of.cpu().numpy()
    row = index_of[nx * (1 + ny * (nz // 2)):nx * (2 + ny * (nz // 2))]
    first = int(row[row >= 0].min())
    return [(t * 256, min(t * 256 + 256, lat.n_fluid)), (first, first + 512)]


def test_large_packing_full_size_sampled_step(large):
    """The 512x512x1024 packing (107 M cells) at full size: one GPU step over
    8-bit codes (16-bit in the tiles that need them) from a seeded state,
    compared on sampled ranges with the oracle (whose sparse representation
    of the whole box is built on the host)."""
    lat, sp, comp = large
    n = lat.n_fluid
    print_case("large packing full size", n)
    prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), "f64", nontemporal=True, xcd_chunk=64)
    st = L.init(lat, prm)
    ranges = [(0, 4096), (n // 2, n // 2 + 4096), (n - 3001, n)] + special_ranges(lat, comp)
    err = sampled_step_vs_oracle(lat, sp, prm, st, lambda: L.step_c8(st, comp, 1), ranges, 11)
    assert err <= TOL_F64
    del st


@pytest.mark.parametrize("storage", ["f32s", "f16s"])
def test_large_packing_full_size_sampled_step_reduced(large, storage):
    """The same in shifted FP32 / FP16 storage (FP32 arithmetic), in the
    launch configuration of the precision experiment: the oracle computes in
    FP64 from the same stored values and rounds to the storage type; bound as
    for the one-step test on the small packing (one storage ulp + 64 eps32 of
    the largest stored value)."""
    lat, sp, comp = large
    n, S = lat.n_fluid, lat.stride
    print_case("large packing full size", storage, n)
    prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), storage, nontemporal=True, xcd_chunk=1)
    st = L.init(lat, prm)
    dt = np.float16 if storage == "f16s" else np.float32
    ranges = [(0, 4096), (n // 3, n // 3 + 3000), (n - 2049, n)] + special_ranges(lat, comp)
    cells_ = np.unique(np.concatenate([np.arange(a, b) for a, b in ranges])).astype(np.int64)
    k = cells_.size
    slots = np.empty((19, k), dtype=np.int64)
    slots[0] = cells_
    slots[1:] = sp.adj[:, cells_].astype(np.int64)
    rng = np.random.default_rng(12)
    vals = (W[slots // S] * 2e-2 * rng.standard_normal(slots.shape)).astype(dt)  # h = f - w
    st.f.zero_()  # shifted rest state everywhere
    st.f.view(-1)[torch.from_numpy(slots.ravel()).cuda()] = torch.from_numpy(vals.ravel()).cuda()
    L.step_c8(st, comp, 1)
    got = st.f[:, torch.from_numpy(cells_).cuda()].cpu().numpy().astype(np.float64)
    ident = ((np.arange(1, 19, dtype=np.uint64)[:, None] * k + np.arange(k, dtype=np.uint64)[None, :])
             .astype(np.uint32))
    exact = np.zeros((19, k))
    O.step(oracle_params(prm), ident, np.ascontiguousarray(vals.astype(np.float64)), exact)
    orc = O.round_storage(exact, storage)
    ulp = np.spacing(np.abs(exact).astype(dt)).astype(np.float64)
    tol = ulp + 64 * np.finfo(np.float32).eps * np.abs(vals.astype(np.float64)).max()
    assert (np.abs(got - orc) <= tol).all()
    assert np.abs(got - vals.astype(np.float64)).max() > 10 * tol.max()  # it moved
    del st


def test_large_packing_cropped_vs_oracle():
    """The 512x512x1024 Boolean packing at 1/4 edge (128x128x256, porosity
    0.4): bit-exact assembly and 10 FP64 sweeps within 1e-12 of the oracle."""
    g = I.workload("large_packing", scale=4)
    sp, lat = pair(g)
    np.testing.assert_array_equal(lat.adj.cpu().numpy().view(np.uint32)[:, :sp.n_fluid],
                                  sp.adj[:, :sp.n_fluid])
    prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), "f64")
    n = sp.n_fluid
    f0 = random_state(n, 11, stride=lat.stride)
    st = run_gpu(lat, prm, f0, 10)
    orc = orun(prm, sp, f0, 10)
    assert rel_err_f64(cells(st.f.cpu().numpy(), n), cells(orc, n)) <= TOL_F64
