"""Pins of the oracle's numbering, compaction and adjacency (CPU only).

Every check compares the oracle with something other than itself: an
independent traversal that visits cells in the ordering's definition order,
a brute-force neighbour search, a closed form, or a count the paper prints.
"""
import itertools
import os

import numpy as np
import pytest

import oracle as O
from paper_1111_1129_amd import inputs as I

ORDERS = ["lex", "blocked", "morton1", "morton2", "random"]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---- independent visiting sequences (test-side, not the oracle's keys) ----

def visit_lex(nx, ny, nz):
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                yield x, y, z


def visit_blocked(nx, ny, nz, b):
    """Blocks in lexicographic order, cells lexicographic inside a block."""
    for Z in range(0, nz, b):
        for Y in range(0, ny, b):
            for X in range(0, nx, b):
                for z in range(Z, min(Z + b, nz)):
                    for y in range(Y, min(Y + b, ny)):
                        for x in range(X, min(X + b, nx)):
                            yield x, y, z


def visit_recursive(nx, ny, nz, fan):
    """Recursive subdivision of the enclosing cube into fan^3 children visited
    with x fastest: fan=2 is the Z curve with 1-bit interleave, fan=4 the
    2-bit-group interleave.  Cells outside the box are skipped."""
    size = 1
    while size < max(nx, ny, nz):
        size *= fan

    def rec(x0, y0, z0, s):
        if x0 >= nx or y0 >= ny or z0 >= nz:
            return
        if s == 1:
            yield x0, y0, z0
            return
        h = s // fan
        for cz in range(fan):
            for cy in range(fan):
                for cx in range(fan):
                    yield from rec(x0 + cx * h, y0 + cy * h, z0 + cz * h, h)

    yield from rec(0, 0, 0, size)


def expected_ranks(flags, seq):
    nz, ny, nx = flags.shape
    idx = -np.ones(nx * ny * nz, dtype=np.int64)
    r = 0
    for x, y, z in seq:
        if flags[z, y, x]:
            idx[x + nx * (y + ny * z)] = r
            r += 1
    return idx


def sequence(order, param, nx, ny, nz):
    if order == "lex":
        return visit_lex(nx, ny, nz)
    if order == "blocked":
        return visit_blocked(nx, ny, nz, param)
    if order == "morton1":
        return visit_recursive(nx, ny, nz, 2)
    if order == "morton2":
        # 2-bit groups need coordinates padded to an even number of bits;
        # fan-4 recursion over the enclosing power-of-4 cube does exactly that
        return visit_recursive(nx, ny, nz, 4)
    raise KeyError(order)


# ---- numbering ------------------------------------------------------------

@pytest.mark.parametrize("dims", [(2, 2, 2), (3, 4, 5), (7, 5, 3), (1, 1, 9), (8, 8, 8),
                                  (5, 9, 6), (16, 4, 4)])
@pytest.mark.parametrize("order,param", [("lex", 0), ("blocked", 1), ("blocked", 2),
                                         ("blocked", 3), ("blocked", 100), ("morton1", 0),
                                         ("morton2", 0)])
def test_ranks_match_visiting_order(dims, order, param):
    nx, ny, nz = dims
    g = I.random_flags(seed=11 + nx * 100 + ny * 10 + nz, nx=nx, ny=ny, nz=nz)
    sp = O.build(g.flags, g.periodic, order, param)
    ref = expected_ranks(g.flags, sequence(order, param, nx, ny, nz))
    np.testing.assert_array_equal(sp.index_of, ref)
    assert sp.n_fluid == g.n_fluid


def test_exhaustive_2x2x2():
    """Every 2x2x2 flag field x every periodic mask x every ordering."""
    for bits in range(256):
        flags = np.array([(bits >> k) & 1 for k in range(8)], dtype=np.uint8).reshape(2, 2, 2)
        for periodic in range(8):
            for order, param in [("lex", 0), ("blocked", 1), ("blocked", 2), ("morton1", 0),
                                 ("morton2", 0), ("random", 7)]:
                sp = O.build(flags, periodic, order, param)
                if order == "random":
                    keys = [O.key(order, param, (2, 2, 2), x, y, z)
                            for x, y, z in visit_lex(2, 2, 2)]
                    ref = -np.ones(8, dtype=np.int64)
                    fl = [k for k, (x, y, z) in zip(keys, visit_lex(2, 2, 2)) if flags[z, y, x]]
                    for lin, (x, y, z) in enumerate(visit_lex(2, 2, 2)):
                        if flags[z, y, x]:
                            ref[lin] = sum(1 for k in fl if k < keys[lin])
                else:
                    ref = expected_ranks(flags, sequence(order, param, 2, 2, 2))
                np.testing.assert_array_equal(sp.index_of, ref)
                check_adjacency_bruteforce(flags, periodic, sp)


def test_closed_forms_all_fluid():
    # all-fluid box, LEX: I_c = linear index
    g = I.all_fluid(5, 3, 4)
    sp = O.build(g.flags, 7, "lex")
    np.testing.assert_array_equal(sp.index_of, np.arange(60))
    # blocking factor 1 is no blocking (paper Sec. 7); so is a block that
    # covers the whole box
    for b in (1, 5, 64):
        np.testing.assert_array_equal(O.build(g.flags, 7, "blocked", b).index_of, np.arange(60))
    # 2-bit groups on a 4^3 box reduce to lexicographic order
    g4 = I.all_fluid(4, 4, 4)
    np.testing.assert_array_equal(O.build(g4.flags, 7, "morton2").index_of, np.arange(64))
    # 1-bit Z curve on a 2^k cube: I_c is the interleaved bit pattern
    g8 = I.all_fluid(8, 8, 8)
    idx = O.build(g8.flags, 7, "morton1").index_of
    for x, y, z in itertools.product(range(8), repeat=3):
        m = sum((((x >> k) & 1) << (3 * k)) | (((y >> k) & 1) << (3 * k + 1))
                | (((z >> k) & 1) << (3 * k + 2)) for k in range(3))
        assert idx[x + 8 * (y + 8 * z)] == m


def test_random_order_is_bijection():
    for n_box in (1, 2, 3, 15, 16, 17, 64, 100, 1000):
        h = O.feistel_half_bits(n_box)
        assert 4 ** h >= n_box and (h == 1 or 4 ** (h - 1) < n_box)
        vals = [O.feistel(12345, h, v) for v in range(4 ** h)]
        assert sorted(vals) == list(range(4 ** h))
    # different seeds give different orders
    g = I.all_fluid(6, 5, 4)
    a = O.build(g.flags, 0, "random", 1).index_of
    b = O.build(g.flags, 0, "random", 2).index_of
    assert sorted(a) == list(range(120)) and not np.array_equal(a, b)


def test_splitmix64_definition():
    """SplitMix64 mixes state + golden gamma with two xorshift-multiply
    rounds; its finaliser is a bijection, so distinct inputs give distinct
    outputs, and state 0 - gamma maps to the finaliser of 0, which is 0."""
    gamma = 0x9E3779B97F4A7C15
    assert O.splitmix64((2 ** 64 - gamma) % 2 ** 64) == 0
    outs = {O.splitmix64(v) for v in range(4096)}
    assert len(outs) == 4096


def test_splitmix64_published_outputs():
    """The published SplitMix64 stream from state 0 (tests/golden): any change
    to a constant or shift of the generator changes these outputs."""
    gamma = 0x9E3779B97F4A7C15
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 5
    for k, out in rows:
        assert O.splitmix64(int(k) * gamma % 2 ** 64) == int(out, 16)


def test_ranks_increase_with_key():
    g = I.random_flags(5, 9, 7, 6, periodic=1)
    for order, param in [("lex", 0), ("blocked", 4), ("morton1", 0), ("morton2", 0),
                         ("random", 99)]:
        sp = O.build(g.flags, g.periodic, order, param)
        nx, ny, nz = g.dims
        keys = []
        for lin in sp.cell_of:
            x, y, z = lin % nx, (lin // nx) % ny, lin // (nx * ny)
            keys.append(O.key(order, param, (nx, ny, nz), x, y, z))
        assert all(a < b for a, b in zip(keys, keys[1:]))
        assert sorted(sp.cell_of.tolist()) == sorted(np.flatnonzero(g.flags.ravel()).tolist())


# ---- adjacency ------------------------------------------------------------

def d3q19():
    cs, opp = [], []
    for i in range(19):
        c, o = O.velocity(i)
        cs.append(c)
        opp.append(o)
    return np.array(cs), np.array(opp)


def test_velocity_set_is_d3q19():
    """The 18 moving links are exactly the nonzero vectors of {-1,0,1}^3 with
    |c|^2 <= 2, opposite pairs are negatives, weights are isotropic."""
    c, opp = d3q19()
    assert tuple(c[0]) == (0, 0, 0)
    expect = {v for v in itertools.product((-1, 0, 1), repeat=3) if 0 < sum(t * t for t in v) <= 2}
    assert {tuple(v) for v in c[1:]} == expect and len(c) == 19
    for i in range(19):
        np.testing.assert_array_equal(c[opp[i]], -c[i])
        assert opp[opp[i]] == i
    w = np.array([O.weight(i) for i in range(19)])
    assert abs(w.sum() - 1) < 1e-15
    # second moment c_s^2 = 1/3, fourth moments of D3Q19 lattice isotropy
    np.testing.assert_allclose((w[:, None, None] * c[:, :, None] * c[:, None, :]).sum(0),
                               np.eye(3) / 3, atol=1e-16)
    assert abs((w * c[:, 0] ** 4).sum() - 1 / 3) < 1e-16
    assert abs((w * c[:, 0] ** 2 * c[:, 1] ** 2).sum() - 1 / 9) < 1e-16


def check_adjacency_bruteforce(flags, periodic, sp):
    c, opp = d3q19()
    nz, ny, nx = flags.shape
    N, S, base = sp.n_fluid, sp.stride, sp.base
    dims = (nx, ny, nz)
    for m in range(N):
        lin = int(sp.cell_of[m])
        p = (lin % nx, (lin // nx) % ny, lin // (nx * ny))
        for i in range(1, 19):
            q = [p[d] - c[i][d] for d in range(3)]
            fluid_up = True
            for d in range(3):
                if not 0 <= q[d] < dims[d]:
                    if periodic >> d & 1:
                        q[d] %= dims[d]
                    else:
                        fluid_up = False
            if fluid_up and flags[q[2], q[1], q[0]]:
                expect = i * S + base + int(sp.index_of[q[0] + nx * (q[1] + ny * q[2])])
            else:
                expect = opp[i] * S + base + m
            assert sp.adj[i - 1, base + m] == expect, (m, i)


@pytest.mark.parametrize("seed", range(6))
def test_adjacency_bruteforce_random(seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = (int(v) for v in rng.integers(1, 7, size=3))
    g = I.random_flags(seed, nx, ny, nz)
    order = ORDERS[seed % 5]
    sp = O.build(g.flags, g.periodic, order, 2 if order == "blocked" else 3)
    check_adjacency_bruteforce(g.flags, g.periodic, sp)


def test_adjacency_offset_base_and_stride():
    g = I.random_flags(3, 5, 4, 3, periodic=5)
    full = O.build(g.flags, g.periodic, "morton1")
    base, stride = 17, full.n_fluid + 40
    sp = O.build(g.flags, g.periodic, "morton1", base=base, stride=stride)
    check_adjacency_bruteforce(g.flags, g.periodic, sp)
    # untouched columns stay zero
    assert not sp.adj[:, :base].any() and not sp.adj[:, base + sp.n_fluid:].any()


def check_permutation_and_symmetry(flags, periodic, sp):
    c, opp = d3q19()
    N, S = sp.n_fluid, sp.stride
    slots = np.concatenate([np.arange(N, dtype=np.int64), sp.adj[:, :N].ravel().astype(np.int64)])
    # pull streaming with bounce-back reads every PDF slot exactly once
    np.testing.assert_array_equal(np.sort(slots), np.arange(19 * N))
    # link symmetry: n pulls i from m  <=>  m pulls opp(i) from n
    a = sp.adj[:, :N].astype(np.int64)
    for k in range(18):
        i = k + 1
        dirn, src = a[k] // S, a[k] % S
        linked = dirn == i
        m = src[linked]
        n = np.flatnonzero(linked)
        back = a[opp[i] - 1, m]
        np.testing.assert_array_equal(back, opp[i] * S + n)
        # bounce-back entries point at the cell's own opposite population
        bb = ~linked
        np.testing.assert_array_equal(dirn[bb], opp[i])
        np.testing.assert_array_equal(src[bb], np.flatnonzero(bb))
    # number of bounce-back entries = number of fluid->blocked links
    nz, ny, nx = flags.shape
    dims = (nx, ny, nz)
    pad_count = 0
    fl = np.argwhere(flags.transpose(2, 1, 0) > 0)  # (x, y, z)
    for i in range(1, 19):
        q = fl - c[i]
        inside = np.ones(len(q), dtype=bool)
        for d in range(3):
            if periodic >> d & 1:
                q[:, d] %= dims[d]
            else:
                inside &= (q[:, d] >= 0) & (q[:, d] < dims[d])
        qq = np.clip(q, 0, np.array(dims) - 1)
        solid = ~inside | (flags[qq[:, 2], qq[:, 1], qq[:, 0]] == 0)
        pad_count += int(solid.sum())
    n_bb = int(sum((a[k] // S != k + 1).sum() for k in range(18)))
    assert n_bb == pad_count


@pytest.mark.parametrize("order,param", [("lex", 0), ("blocked", 8), ("morton1", 0),
                                         ("morton2", 0), ("random", 22)])
def test_permutation_invariant_small_packing(order, param):
    g = I.packing_small(1)
    sp = O.build(g.flags, g.periodic, order, param)
    check_permutation_and_symmetry(g.flags, g.periodic, sp)


def test_channel_fluid_count_matches_paper():
    """The paper's 500 x 100 x 100 empty channel holds about 4.8e6 fluid cells
    (Sec. 7), which 1-cell walls on the y and z faces reproduce exactly."""
    with open(os.path.join(GOLDEN, "paper_counts.txt")) as fh:
        rows = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    stated = {r[0]: float(r[1]) for r in rows}
    g = I.channel(100)
    sp = O.build(g.flags, g.periodic, "lex")
    assert sp.n_fluid == 500 * 98 * 98
    assert abs(sp.n_fluid - stated["channel_500x100x100_fluid"]) <= 0.05e6


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_hilbert_is_a_continuous_curve(k):
    """On a full 2^k cube the Hilbert order visits every cell once, starts at
    the origin, and consecutive cells are face neighbours (the defining
    property of a Hilbert curve; the Z curves fail it)."""
    n = 2 ** k
    g = I.all_fluid(n, n, n)
    sp = O.build(g.flags, 7, "hilbert")
    lin = sp.cell_of.astype(np.int64)
    xyz = np.stack([lin % n, (lin // n) % n, lin // (n * n)], axis=1)
    assert sorted(lin.tolist()) == list(range(n ** 3))
    assert tuple(xyz[0]) == (0, 0, 0)
    steps = np.abs(np.diff(xyz, axis=0)).sum(axis=1)
    assert (steps == 1).all()
    if k >= 2:
        z = O.build(g.flags, 7, "morton1").cell_of.astype(np.int64)
        zxyz = np.stack([z % n, (z // n) % n, z // (n * n)], axis=1)
        assert (np.abs(np.diff(zxyz, axis=0)).sum(axis=1) > 1).any()


def test_hilbert_on_uneven_boxes_is_a_bijection():
    for dims in [(3, 5, 7), (9, 2, 4), (1, 1, 6), (17, 3, 1)]:
        g = I.random_flags(sum(dims), *dims, fluid_fraction=0.7)
        sp = O.build(g.flags, g.periodic, "hilbert")
        check_adjacency_bruteforce(g.flags, g.periodic, sp)
        keys = [O.key("hilbert", 0, dims, l % dims[0], (l // dims[0]) % dims[1],
                      l // (dims[0] * dims[1])) for l in sp.cell_of]
        assert all(a < b for a, b in zip(keys, keys[1:]))
        allk = {O.key("hilbert", 0, dims, x, y, z) for x in range(dims[0])
                for y in range(dims[1]) for z in range(dims[2])}
        assert len(allk) == dims[0] * dims[1] * dims[2]


# ---- chunk communication analysis ----------------------------------------

def test_partition_chunks_are_near_equal():
    """The list is cut into G chunks whose sizes differ by at most one cell
    (paper Sec. 2)."""
    for n, G in [(10, 3), (17263, 7), (100, 100), (5, 5), (1000, 64)]:
        b = O.chunk_bounds(n, G)
        sizes = np.diff(b)
        assert b[0] == 0 and b[-1] == n and sizes.max() - sizes.min() <= 1


def test_partition_stats_special_cases_and_symmetry():
    g = I.packing_small(1)
    sp = O.build(g.flags, g.periodic, "lex")
    n = sp.n_fluid
    # one chunk: nothing is remote
    r, nb, ifc = O.partition_stats(sp.adj, n, 1)
    assert r.sum() == 0 and nb.sum() == 0 and ifc.sum() == 0
    # every cell its own chunk: every streaming entry is remote
    r, nb, ifc = O.partition_stats(sp.adj, n, n)
    S = sp.adj.shape[1]
    streaming = sum(int((sp.adj[k, :n].astype(np.int64) // S == k + 1).sum()) for k in range(18))
    assert r.sum() == streaming
    # pull symmetry: links a<-b and b<-a come in pairs, so the total is even
    # and chunk neighbour relations are symmetric
    for G in (2, 5, 16, 64):
        r, nb, ifc = O.partition_stats(sp.adj, n, G)
        assert r.sum() % 2 == 0 and (ifc <= np.diff(O.chunk_bounds(n, G))).all()
        assert (nb <= G - 1).all() and (r >= ifc).all()


def test_partition_stats_brute_force_small():
    """A 4x3x2 all-fluid periodic box cut in two: count links by walking the
    D3Q19 neighbourhood of every cell by hand."""
    g = I.all_fluid(4, 3, 2)
    sp = O.build(g.flags, 7, "lex")
    n = sp.n_fluid
    c, opp = d3q19()
    G = 2
    b = O.chunk_bounds(n, G)
    chunk = lambda m: int(np.searchsorted(b, m, side="right") - 1)
    expect = np.zeros(G, dtype=np.int64)
    for x in range(4):
        for y in range(3):
            for z in range(2):
                m = x + 4 * (y + 3 * z)
                for i in range(1, 19):
                    u = ((x - c[i][0]) % 4, (y - c[i][1]) % 3, (z - c[i][2]) % 2)
                    src = u[0] + 4 * (u[1] + 3 * u[2])
                    if chunk(src) != chunk(m):
                        expect[chunk(m)] += 1
    r, nb, _ = O.partition_stats(sp.adj, n, G)
    np.testing.assert_array_equal(r, expect)
    assert list(nb) == [1, 1]
