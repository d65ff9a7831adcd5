"""GPU assembly (lbm_build_adjacency) vs the oracle: bit-exact index_of,
cell_of and adjacency, at small sizes spanning many tiles and at the full
256^3 tube size."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1111_1129_amd import _native as N
from paper_1111_1129_amd import inputs as I
from paper_1111_1129_amd import lattice as L

from gpu_helpers import adj_u32, dev_flags, print_case

pytestmark = pytest.mark.gpu

ORDERS = [("lex", 0), ("blocked", 16), ("blocked", 3), ("blocked", 1), ("morton1", 0),
          ("morton2", 0), ("random", 22), ("hilbert", 0)]


def assert_same(geom, order, param, base=0, stride=None):
    print_case("assembly", geom.name, geom.dims, order, param, base, stride)
    lat = L.build(dev_flags(geom), geom.periodic, order, param, base=base, stride=stride)
    sp = O.build(geom.flags, geom.periodic, order, param, base=base, stride=lat.stride)
    assert lat.n_fluid == sp.n_fluid
    np.testing.assert_array_equal(lat.index_of.cpu().numpy(), sp.index_of)
    np.testing.assert_array_equal(lat.cell_of.cpu().numpy(), sp.cell_of)
    a = adj_u32(lat)
    np.testing.assert_array_equal(a[:, base:base + sp.n_fluid], sp.adj[:, base:base + sp.n_fluid])
    return lat, sp


@pytest.mark.parametrize("order,param", ORDERS)
def test_small_packing(order, param):
    assert_same(I.packing_small(1), order, param)


def test_exhaustive_2x2x2(dev):
    for bits in range(256):
        flags = np.array([(bits >> k) & 1 for k in range(8)], dtype=np.uint8).reshape(2, 2, 2)
        for periodic in (0, 5, 7):
            for order, param in [("lex", 0), ("blocked", 2), ("morton1", 0), ("morton2", 0),
                                 ("random", 3), ("hilbert", 0)]:
                g = I.Geometry("tiny", flags, periodic)
                lat = L.build(dev_flags(g), periodic, order, param)
                sp = O.build(flags, periodic, order, param, stride=lat.stride)
                assert lat.n_fluid == sp.n_fluid
                np.testing.assert_array_equal(lat.index_of.cpu().numpy(), sp.index_of)
                if sp.n_fluid:
                    np.testing.assert_array_equal(adj_u32(lat)[:, :sp.n_fluid],
                                                  sp.adj[:, :sp.n_fluid])


@pytest.mark.parametrize("seed", range(24))
def test_random_fields(seed):
    rng = np.random.default_rng(1000 + seed)
    dims = [int(v) for v in rng.integers(1, 40, size=3)]
    if seed % 4 == 0:
        dims[int(rng.integers(0, 3))] = 1
    g = I.random_flags(seed, *dims, fluid_fraction=float(rng.uniform(0.1, 0.95)))
    order, param = ORDERS[seed % len(ORDERS)]
    if order == "blocked":
        param = int(rng.choice([1, 2, 3, 5, 7, 64, 1000]))
    assert_same(g, order, param)


def test_base_and_stride_placement():
    g = I.packing_small(1)
    n = g.n_fluid
    assert_same(g, "morton2", 0, base=300, stride=n + 1000)


def test_all_solid_and_single_cell():
    flags = np.zeros((5, 6, 7), dtype=np.uint8)
    g = I.Geometry("empty", flags, 7)
    lat = L.build(dev_flags(g), 7, "morton1")
    assert lat.n_fluid == 0
    assert (lat.index_of.cpu().numpy() == -1).all()
    flags[2, 3, 4] = 1
    lat, _ = assert_same(I.Geometry("one", flags, 0), "lex", 0)
    assert lat.n_fluid == 1


def test_count_only_and_capacity_error():
    g = I.packing_small(1)
    fl = dev_flags(g)
    assert L.count_fluid(fl, g.periodic, "morton1") == g.n_fluid
    nz, ny, nx = g.flags.shape
    geom = N.lbm_geom(nx, ny, nz, g.periodic, 0, 0)
    idx = torch.empty(nx * ny * nz, dtype=torch.int32, device="cuda")
    st, _, ws = N.lbm_build_adjacency(geom, fl, 0, 0, idx, None, None, 0, query=True)
    wsb = torch.empty(ws, dtype=torch.uint8, device="cuda")
    cell = torch.empty(10, dtype=torch.int32, device="cuda")
    st, nf, _ = N.lbm_build_adjacency(geom, fl, 0, 0, idx, cell, None, 10, wsb, ws)
    assert st == N.LBM_ECAPACITY and nf == g.n_fluid
    st, _, _ = N.lbm_build_adjacency(geom, fl, 0, 0, idx, cell, None, 10, wsb, ws - 1)
    assert st == N.LBM_EWORKSPACE


@pytest.fixture(scope="module")
def tube():
    return I.packing_tube(2)


@pytest.mark.parametrize("order,param", [("lex", 0), ("blocked", 16), ("morton1", 0),
                                         ("morton2", 0), ("random", 22), ("hilbert", 0)])
def test_tube_full_size(tube, order, param):
    lat, sp = assert_same(tube, order, param)
    # adjacency is a permutation of the PDF slots (pull streaming is bijective)
    n, S = lat.n_fluid, lat.stride
    a = adj_u32(lat)[:, :n].astype(np.int64)
    # slot i*S + m  ->  dense index i*n + m
    dense = (a // S) * n + a % S
    assert (a % S < n).all()
    counts = np.bincount(dense.ravel(), minlength=19 * n)
    assert counts.shape == (19 * n,)
    assert (counts[:n] == 0).all() and (counts[n:] == 1).all()
    # the library's checked mode reaches the same verdict on the device
    assert L.check_adjacency(lat) == (0, 0)


@pytest.mark.parametrize("order,param", [("lex", 0), ("blocked", 8), ("hilbert", 0)])
@pytest.mark.parametrize("G", [1, 2, 7, 64, 300])
def test_partition_stats_vs_oracle(order, param, G):
    g = I.packing_small(1)
    lat = L.build(dev_flags(g), g.periodic, order, param)
    sp = O.build(g.flags, g.periodic, order, param, stride=lat.stride)
    r, nb, ifc = L.partition_stats(lat, G)
    orr, onb, oifc = O.partition_stats(sp.adj, sp.n_fluid, G)
    np.testing.assert_array_equal(r.cpu().numpy(), orr)
    np.testing.assert_array_equal(nb.cpu().numpy(), onb)
    np.testing.assert_array_equal(ifc.cpu().numpy(), oifc)


def test_partition_stats_tube_3072_chunks(tube):
    """The tube cut into 3072 chunks (the paper's largest process count):
    bit-exact against the oracle's definition."""
    lat = L.build(dev_flags(tube), tube.periodic, "blocked", 16)
    sp = O.build(tube.flags, tube.periodic, "blocked", 16, stride=lat.stride)
    r, nb, ifc = L.partition_stats(lat, 3072)
    orr, onb, oifc = O.partition_stats(sp.adj, sp.n_fluid, 3072)
    np.testing.assert_array_equal(r.cpu().numpy(), orr)
    np.testing.assert_array_equal(nb.cpu().numpy(), onb)
    np.testing.assert_array_equal(ifc.cpu().numpy(), oifc)


@pytest.mark.parametrize("order,param", ORDERS)
def test_checked_mode_accepts_the_assembled_lists(order, param):
    """lbm_check_adjacency: every list the assembly builds has all entries in
    range and references each of its 18 n slots exactly once."""
    g = I.packing_small(1)
    print_case("check adjacency", order, param)
    lat = L.build(dev_flags(g), g.periodic, order, param)
    assert L.check_adjacency(lat) == (0, 0)


def test_checked_mode_on_batch_members_and_corrupted_lists():
    geoms = [I.packing_boolean(60 + k, 20 + 3 * k, 20, 20, 2.0, 4.0, 0.5) for k in range(3)]
    batch = L.Batch([dev_flags(g) for g in geoms], [g.periodic for g in geoms], "morton2",
                    tile_align=True)
    print_case("check adjacency batch", batch.counts)
    for lat in batch.lattices:
        assert L.check_adjacency(lat) == (0, 0)
    lat = batch.lattices[1]
    b, n, S = lat.base, lat.n_fluid, lat.stride
    good = lat.adj.clone()
    # one entry duplicated: one slot referenced twice, another never
    lat.adj[3, b + 100] = lat.adj[3, b + 101]
    assert L.check_adjacency(lat) == (0, 2)
    lat.adj.copy_(good)
    # an entry in row 0 (the implicit rest slot), one past 19 * stride, one in
    # another member's columns: each out of range and its slot left unreferenced
    lat.adj[0, b + 5] = b + 5
    lat.adj[7, b + 9] = -16  # the uint32 entry 0xFFFFFFF0, far past 19 * stride
    lat.adj[2, b + 11] = 3 * S + batch.bases[2]
    assert L.check_adjacency(lat) == (3, 3)
    lat.adj.copy_(good)
    assert L.check_adjacency(lat) == (0, 0)
