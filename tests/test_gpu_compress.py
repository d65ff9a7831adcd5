"""16-bit adjacency codes: lossless on every ordering, and the sweep that reads
them gives bitwise the results of the sweep over the full adjacency list (and
so the oracle's, within the FP64 tolerance)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1111_1129_amd import inputs as I
from paper_1111_1129_amd import lattice as L

from gpu_helpers import adj_u32, dev_flags, oracle_params, print_case, random_state, rel_err_f64

pytestmark = pytest.mark.gpu

BOUNCE, ESCAPE = -32768, -32767


def opp(i):
    return i + 1 if i % 2 == 1 else i - 1


def decode(codes, toff, adj, n, stride):
    """Slots named by the codes (host side), escapes resolved through adj."""
    m = np.arange(n, dtype=np.int64)
    out = np.empty((18, n), dtype=np.int64)
    for k in range(18):
        i = k + 1
        c = codes[k, :n].astype(np.int64)
        t = toff[m // 256, k].astype(np.int64)
        out[k] = np.where(c == BOUNCE, opp(i) * stride + m,
                          np.where(c == ESCAPE, adj[k, :n].astype(np.int64),
                                   i * stride + m + t + c))
    return out


def check_codes(lat, comp):
    n, S = comp.n, lat.stride
    adj = adj_u32(lat)
    codes = comp.codes.cpu().numpy()
    toff = comp.tile_records.cpu().numpy()
    np.testing.assert_array_equal(decode(codes, toff, adj, n, S), adj[:, :n].astype(np.int64))
    # escapes only where a streaming entry does not fit the 16-bit range
    m = np.arange(n, dtype=np.int64)
    esc = 0
    for k in range(18):
        i = k + 1
        a = adj[k, :n].astype(np.int64)
        streams = a // S == i
        d = a - i * S - m - toff[m // 256, k]
        fits = (d >= -32766) & (d <= 32767)
        c = codes[k, :n]
        assert np.all((c == BOUNCE) == ~streams)
        assert np.all((c == ESCAPE) == (streams & ~fits))
        esc += int(np.sum(c == ESCAPE))
    assert esc == comp.n_escapes
    # tile records: escapes per tile, then a zero word
    tiles = (n + 255) // 256
    per_tile = np.zeros(tiles, dtype=np.int64)
    np.add.at(per_tile, m // 256, np.sum(codes[:, :n] == ESCAPE, axis=0))
    np.testing.assert_array_equal(toff[:, 18], per_tile)
    assert np.all(toff[:, 19] == 0)
    return esc


@pytest.mark.parametrize("order,param", [("lex", 0), ("blocked", 8), ("morton1", 0),
                                         ("morton2", 0), ("hilbert", 0), ("random", 3)])
def test_codes_are_lossless(order, param):
    g = I.packing_small(1)
    print_case("compress", order, "small_packing")
    lat = L.build(dev_flags(g), g.periodic, order, param)
    comp = L.compress(lat)
    esc = check_codes(lat, comp)
    if order == "lex":
        assert esc == 0  # plane offsets of a 32^3 box are far inside the range


def test_many_escapes_and_ragged_tail():
    """A random ordering of a 64^3 box scatters neighbours over the whole
    list, so most streaming entries escape; the sweep still matches."""
    g = I.random_flags(11, 64, 64, 48, 0.7)
    print_case("compress", "random", "random_flags 64x64x48")
    lat = L.build(dev_flags(g), g.periodic, "random", 9)
    comp = L.compress(lat)
    esc = check_codes(lat, comp)
    assert esc > 0.5 * lat.n_fluid
    assert lat.n_fluid % 256 != 0
    prm = L.params(0.8, 3 / 16, (1e-5, 2e-6, 0), "f64")
    f0 = random_state(lat.n_fluid, 3, stride=lat.stride)
    a = L.init(lat, prm)
    a.f.copy_(torch.from_numpy(f0))
    b = L.init(lat, prm)
    b.f.copy_(torch.from_numpy(f0))
    L.step(a, 7)
    L.step_c16(b, comp, 7)
    assert torch.equal(a.f[:, :lat.n_fluid], b.f[:, :lat.n_fluid])


@pytest.mark.parametrize("n_target", [1, 255, 256, 257])
def test_tiny_lists(n_target):
    """Lists shorter than a tile, exactly a tile, and one cell over."""
    flags = np.zeros((8, 8, 8), dtype=np.uint8)
    flags.ravel()[:n_target] = 1
    print_case("compress", "tiny", n_target)
    lat = L.build(torch.from_numpy(flags).cuda(), 7, "lex", 0)
    assert lat.n_fluid == n_target
    comp = L.compress(lat)
    check_codes(lat, comp)
    prm = L.params(0.8, 3 / 16, (1e-4, 0, 0), "f64")
    f0 = random_state(lat.n_fluid, 4, stride=lat.stride)
    a = L.init(lat, prm)
    a.f.copy_(torch.from_numpy(f0))
    b = L.init(lat, prm)
    b.f.copy_(torch.from_numpy(f0))
    L.step(a, 3)
    L.step_c16(b, comp, 3)
    assert torch.equal(a.f[:, :lat.n_fluid], b.f[:, :lat.n_fluid])


def test_small_packing_vs_oracle_with_pbb():
    g = I.packing_small(1)
    print_case("compress", "oracle", "small_packing", "pbb")
    lat = L.build(dev_flags(g), g.periodic, "lex", 0)
    sp = O.build(g.flags, g.periodic, "lex", 0, stride=lat.stride)
    n = sp.n_fluid
    comp = L.compress(lat)
    ns_h = np.zeros(lat.stride)
    ns_h[:n] = np.random.default_rng(7).uniform(0, 1, n)
    ns = torch.from_numpy(ns_h).cuda()
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64s")
    f0 = random_state(n, 5, amp=1e-3, shifted=True, stride=lat.stride)
    st = L.init(lat, prm, ns=ns)
    st.f.copy_(torch.from_numpy(f0))
    L.step_c16(st, comp, 25)
    orc = O.run(oracle_params(prm), sp.adj, f0, 25, ns=ns_h, n0=0, n1=n)
    assert rel_err_f64(st.f.cpu().numpy()[:, :n], orc[:, :n], shifted=True) <= 1e-12


@pytest.mark.parametrize("storage", ["f64", "f64s", "f32", "f32s", "f16s", "f16s12"])
def test_bitwise_equal_to_full_list_sweep(storage):
    g = I.packing_small(1)
    print_case("compress", "bitwise", storage)
    lat = L.build(dev_flags(g), g.periodic, "morton2", 0)
    comp = L.compress(lat)
    for nt, chunk in ((False, 0), (True, 1)):
        prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), storage, nontemporal=nt, xcd_chunk=chunk)
        a = L.init(lat, prm)
        b = L.init(lat, prm)
        L.step(a, 11)
        L.step_c16(b, comp, 11)
        assert torch.equal(a.f[:, :lat.n_fluid], b.f[:, :lat.n_fluid]), (storage, nt, chunk)


def test_full_size_tube_bitwise():
    g = I.packing_tube(2)
    print_case("compress", "tube", "256^3")
    lat = L.build(dev_flags(g), g.periodic, "lex", 0)
    comp = L.compress(lat)
    assert comp.n_escapes == 0
    # lossless on sampled tiles (the whole list would be 140 M entries)
    rng = np.random.default_rng(0)
    tiles = rng.choice((lat.n_fluid + 255) // 256, 64, replace=False)
    adj = lat.adj
    toff = comp.tile_records.cpu().numpy()
    for t in tiles:
        lo, hi = t * 256, min(lat.n_fluid, t * 256 + 256)
        a = adj[:, lo:hi].cpu().numpy().view(np.uint32).astype(np.int64)
        c = comp.codes[:, lo:hi].cpu().numpy().astype(np.int64)
        m = np.arange(lo, hi)
        for k in range(18):
            i = k + 1
            slot = np.where(c[k] == BOUNCE, opp(i) * lat.stride + m,
                            i * lat.stride + m + toff[t, k] + c[k])
            np.testing.assert_array_equal(slot, a[k])
    prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), "f64", nontemporal=True, xcd_chunk=1)
    a = L.init(lat, prm)
    b = L.init(lat, prm)
    L.step(a, 20)
    L.step_c16(b, comp, 20)
    torch.cuda.synchronize()
    assert torch.equal(a.f[:, :lat.n_fluid], b.f[:, :lat.n_fluid])


NARROW_BOUNCE = -128


def check_narrow(lat, comp):
    """A tile is narrow exactly when all its live codes are bounce-backs or
    lie in [-127, 127]; its 8-bit codes are the 16-bit ones."""
    n = comp.n
    codes = comp.codes[:, :n].cpu().numpy().astype(np.int64)
    c8 = comp.codes8[:, :n].cpu().numpy().astype(np.int64)
    rec = comp.tile_records.cpu().numpy()
    tiles = comp.n_tiles
    fits = (codes == BOUNCE) | ((codes >= -127) & (codes <= 127))
    ok = np.ones(tiles, dtype=bool)
    np.logical_and.at(ok, np.arange(n) // 256, fits.all(axis=0))
    np.testing.assert_array_equal(rec[:, 19], ok.astype(np.int32))
    assert comp.n_narrow == int(ok.sum())
    narrow_cell = ok[np.arange(n) // 256]
    want = np.where(codes == BOUNCE, NARROW_BOUNCE, codes)
    np.testing.assert_array_equal(c8[:, narrow_cell], want[:, narrow_cell])
    assert np.all(c8[:, ~narrow_cell] == 0)
    assert np.all(rec[ok, 18] == 0)  # no narrow tile has escapes
    return ok


@pytest.mark.parametrize("order,param", [("lex", 0), ("blocked", 8), ("morton2", 0),
                                         ("hilbert", 0), ("random", 3)])
def test_narrow_codes_are_exact(order, param):
    g = I.packing_small(1)
    print_case("narrow", order, "small_packing")
    lat = L.build(dev_flags(g), g.periodic, order, param)
    comp = L.narrow(L.compress(lat))
    ok = check_narrow(lat, comp)
    if order == "lex":
        assert ok.mean() > 0.5  # plane offsets of a 32^3 box stay near the tile base
    if order == "random":
        assert not ok.any()


@pytest.mark.parametrize("storage", ["f64", "f64s", "f32", "f32s", "f16s", "f16s12"])
def test_c8_bitwise_equal_to_full_list_sweep(storage):
    g = I.random_flags(11, 64, 64, 48, 0.7)
    print_case("narrow", "bitwise", storage, "random_flags 64x64x48 periodic xyz")
    lat = L.build(dev_flags(g), 7, "lex", 0)  # narrow, 16-bit and escape tiles
    comp = L.narrow(L.compress(lat))
    assert 0 < comp.n_narrow < comp.n_tiles and comp.n_escapes > 0
    for nt, chunk in ((False, 0), (True, 1)):
        prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), storage, nontemporal=nt, xcd_chunk=chunk)
        a = L.init(lat, prm)
        b = L.init(lat, prm)
        L.step(a, 11)
        L.step_c8(b, comp, 11)
        assert torch.equal(a.f[:, :lat.n_fluid], b.f[:, :lat.n_fluid]), (storage, nt, chunk)


def test_c8_with_escapes_pbb_and_ragged_tail():
    """Narrow tiles, 16-bit tiles and escape tiles (full list) in one list:
    lexicographic order of a fully periodic 64x64x48 box; tiles across a y
    wrap pull from a row and from a plane away (16-bit), tiles across the z
    wrap from the next plane and from the far end of the list (escapes)."""
    g = I.random_flags(11, 64, 64, 48, 0.7)
    print_case("narrow", "mixed", "random_flags 64x64x48 periodic xyz")
    lat = L.build(dev_flags(g), 7, "lex", 0)
    comp = L.narrow(L.compress(lat))
    ok = check_narrow(lat, comp)
    rec = comp.tile_records.cpu().numpy()
    esc = rec[:, 18] > 0
    kinds = (int(ok.sum()), int(esc.sum()), int((~ok & ~esc).sum()))
    print("narrow / escape / wide tiles", kinds)
    assert min(kinds) > 0
    assert lat.n_fluid % 256 != 0
    n = lat.n_fluid
    ns_h = np.zeros(lat.stride)
    ns_h[:n] = np.random.default_rng(8).uniform(0, 1, n)
    ns = torch.from_numpy(ns_h).cuda()
    prm = L.params(0.8, 3 / 16, (1e-5, 2e-6, 0), "f64s")
    f0 = random_state(n, 3, amp=1e-3, shifted=True, stride=lat.stride)
    a = L.init(lat, prm, ns=ns)
    a.f.copy_(torch.from_numpy(f0))
    b = L.init(lat, prm, ns=ns)
    b.f.copy_(torch.from_numpy(f0))
    L.step(a, 7)
    L.step_c8(b, comp, 7)
    assert torch.equal(a.f[:, :n], b.f[:, :n])


@pytest.mark.parametrize("n_target", [1, 255, 256, 257])
def test_c8_tiny_lists(n_target):
    flags = np.zeros((8, 8, 8), dtype=np.uint8)
    flags.ravel()[:n_target] = 1
    print_case("narrow", "tiny", n_target)
    lat = L.build(torch.from_numpy(flags).cuda(), 7, "lex", 0)
    comp = L.narrow(L.compress(lat))
    check_narrow(lat, comp)
    prm = L.params(0.8, 3 / 16, (1e-4, 0, 0), "f64")
    f0 = random_state(lat.n_fluid, 4, stride=lat.stride)
    a = L.init(lat, prm)
    a.f.copy_(torch.from_numpy(f0))
    b = L.init(lat, prm)
    b.f.copy_(torch.from_numpy(f0))
    L.step(a, 3)
    L.step_c8(b, comp, 3)
    assert torch.equal(a.f[:, :lat.n_fluid], b.f[:, :lat.n_fluid])


def test_c8_full_size_tube_bitwise():
    g = I.packing_tube(2)
    print_case("narrow", "tube", "256^3")
    lat = L.build(dev_flags(g), g.periodic, "lex", 0)
    comp = L.narrow(L.compress(lat))
    print("narrow tiles", comp.n_narrow, "of", comp.n_tiles)
    assert comp.n_narrow > 0.8 * comp.n_tiles
    # exact on sampled tiles
    rng = np.random.default_rng(1)
    rec = comp.tile_records.cpu().numpy()
    for t in rng.choice(comp.n_tiles, 64, replace=False):
        lo, hi = t * 256, min(lat.n_fluid, t * 256 + 256)
        c = comp.codes[:, lo:hi].cpu().numpy().astype(np.int64)
        c8 = comp.codes8[:, lo:hi].cpu().numpy().astype(np.int64)
        fits = bool(np.all((c == BOUNCE) | ((c >= -127) & (c <= 127))))
        assert rec[t, 19] == int(fits)
        if fits:
            np.testing.assert_array_equal(c8, np.where(c == BOUNCE, NARROW_BOUNCE, c))
    prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), "f64", nontemporal=True, xcd_chunk=1)
    a = L.init(lat, prm)
    b = L.init(lat, prm)
    L.step(a, 20)
    L.step_c8(b, comp, 20)
    torch.cuda.synchronize()
    assert torch.equal(a.f[:, :lat.n_fluid], b.f[:, :lat.n_fluid])
