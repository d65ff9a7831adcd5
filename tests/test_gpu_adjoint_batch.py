"""GPU adjoint vs the oracle adjoint, the autograd Function, and batched
geometries vs solo runs."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1111_1129_amd import _native as N
from paper_1111_1129_amd import adjoint as AD
from paper_1111_1129_amd import inputs as I
from paper_1111_1129_amd import lattice as L

from gpu_helpers import dev_flags, oracle_params, print_case, random_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pbb():
    g = I.pbb_box(4, n=12)
    lat = L.build(dev_flags(g), g.periodic, "lex", stride=None)
    sp = O.build(g.flags, g.periodic, "lex", stride=lat.stride)
    ns = np.zeros(lat.stride)
    ns[:sp.n_fluid] = g.ns.ravel()[sp.cell_of]
    return g, sp, lat, ns


def ogradient(prm, sp, ns, T):
    """Oracle (J, dJ/dns) on the listed cells, from the dense (stride = n) form."""
    n = sp.n_fluid
    dense = O.build(I.pbb_box(4, n=12).flags, 1, "lex")
    assert dense.n_fluid == n
    return O.gradient(oracle_params(prm), dense.adj, O.init(n, shifted=True), ns[:n].copy(), T,
                      shifted=True)


def test_adjoint_step_vs_oracle(pbb):
    g, sp, lat, ns = pbb
    n, S = sp.n_fluid, lat.stride
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64s")
    op = oracle_params(prm)
    f = random_state(n, 1, amp=1e-3, shifted=True, stride=S)
    lam = np.zeros((19, S))
    lam[:, :n] = np.random.default_rng(2).standard_normal((19, n))
    o_lam, o_grad = np.zeros((19, S)), np.zeros(S)
    O.adjoint_step(op, sp.adj, f, ns, lam, o_lam, o_grad, 0, n)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g_lam = torch.zeros((19, S), dtype=torch.float64, device="cuda")
    g_grad = torch.zeros(S, dtype=torch.float64, device="cuda")
    rc = N.lbm_step_adjoint(prm, n, S, lat.adj, d(f), d(ns), d(lam), g_lam, g_grad)
    assert rc == 0
    gl, gg = g_lam.cpu().numpy()[:, :n], g_grad.cpu().numpy()[:n]
    ol, og = o_lam[:, :n], o_grad[:n]
    np.testing.assert_allclose(gl, ol, rtol=0, atol=1e-13 * np.abs(ol).max())
    np.testing.assert_allclose(gg, og, rtol=0, atol=1e-13 * np.abs(og).max())
    # seed
    seed = torch.zeros((19, S), dtype=torch.float64, device="cuda")
    assert N.lbm_step_adjoint(prm, n, S, lat.adj, None, None, None, seed, None) == 0
    o_seed = np.zeros((19, S))
    O.adjoint_step(op, sp.adj, f, ns, None, o_seed, None, 0, n)
    np.testing.assert_array_equal(seed.cpu().numpy()[:, :n], o_seed[:, :n])


def test_adjoint_launch_options_are_bitwise_identical():
    """Store policy and workgroup-to-XCD mapping change only the speed."""
    g = I.pbb_box(4, n=40)
    print_case("adjoint", "launch options", "pbb_box 40^3")
    lat = L.build(dev_flags(g), g.periodic, "lex")
    n, S = lat.n_fluid, lat.stride
    ns = torch.zeros(S, dtype=torch.float64, device="cuda")
    ns[:n] = torch.from_numpy(g.ns.ravel()[lat.cell_of.cpu().numpy()]).cuda()
    f = torch.from_numpy(random_state(n, 3, amp=1e-3, shifted=True, stride=S)).cuda()
    lam = torch.zeros((19, S), dtype=torch.float64, device="cuda")
    lam[:, :n] = torch.randn((19, n), dtype=torch.float64, generator=torch.Generator().manual_seed(5)).cuda()
    outs = []
    for nt, chunk in ((False, 0), (True, 1), (False, 4), (True, 0)):
        prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64s", nontemporal=nt, xcd_chunk=chunk)
        lt = torch.zeros((19, S), dtype=torch.float64, device="cuda")
        gr = torch.zeros(S, dtype=torch.float64, device="cuda")
        assert N.lbm_step_adjoint(prm, n, S, lat.adj, f, ns, lam, lt, gr) == 0
        outs.append((lt[:, :n].clone(), gr[:n].clone()))
    for lt, gr in outs[1:]:
        assert torch.equal(lt, outs[0][0]) and torch.equal(gr, outs[0][1])


@pytest.mark.parametrize("order", ["lex", "morton2", "random"])
def test_adjoint_over_codes_is_bitwise_the_adjoint(order):
    """The adjoint step reading 16-bit codes, and reading 8-bit codes in
    narrow tiles, equals the plain adjoint step bit for bit.  On this box the
    lexicographic order has only narrow tiles, the 2-bit Z curve a mix of
    16-bit and escape tiles, the random order escapes almost everywhere, so
    every branch of both coded kernels runs."""
    g = I.pbb_box(4, n=64)
    print_case("adjoint c16 / c8", order, "pbb_box 64^3")
    lat = L.build(dev_flags(g), g.periodic, order, 5 if order == "random" else 0)
    n, S = lat.n_fluid, lat.stride
    comp = L.narrow(L.compress(lat))
    rec = comp.tile_records.cpu().numpy()
    if order == "lex":
        assert rec[:, 19].all()
    if order == "morton2":
        assert (rec[:, 18] > 0).any() and (rec[:, 18] == 0).any() and not rec[:, 19].any()
    if order == "random":
        assert comp.n_escapes > 0
    ns = torch.zeros(S, dtype=torch.float64, device="cuda")
    ns[:n] = torch.from_numpy(g.ns.ravel()[lat.cell_of.cpu().numpy()]).cuda()
    f = torch.from_numpy(random_state(n, 3, amp=1e-3, shifted=True, stride=S)).cuda()
    lam = torch.zeros((19, S), dtype=torch.float64, device="cuda")
    lam[:, :n] = torch.randn((19, n), dtype=torch.float64,
                             generator=torch.Generator().manual_seed(6)).cuda()
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64s")
    for sf in (ns, None):  # with and without partial bounce-back
        outs = []
        for form in ("full", "c16", "c8"):
            lt = torch.zeros((19, S), dtype=torch.float64, device="cuda")
            gr = torch.zeros(S, dtype=torch.float64, device="cuda")
            gr_arg = gr if sf is not None else None
            if form == "c16":
                rc = N.lbm_step_adjoint_c16(prm, n, S, comp.codes, comp.tile_records, lat.adj, f,
                                            sf, lam, lt, gr_arg)
            elif form == "c8":
                rc = N.lbm_step_adjoint_c8(prm, n, S, comp.codes8, comp.codes, comp.tile_records,
                                           lat.adj, f, sf, lam, lt, gr_arg)
            else:
                rc = N.lbm_step_adjoint(prm, n, S, lat.adj, f, sf, lam, lt, gr_arg)
            assert rc == 0
            outs.append((lt[:, :n].clone(), gr[:n].clone()))
        for lt, gr in outs[1:]:
            assert torch.equal(outs[0][0], lt) and torch.equal(outs[0][1], gr)


@pytest.mark.parametrize("order", ["lex", "morton2", "random"])
def test_adjoint_scatter_is_a_permutation(order):
    """lambda^t starts as NaN in every slot; one adjoint step writes 19 values
    per cell through the adjacency, so if every one of the 19 n listed slots
    is finite afterwards, the 19 n writes hit 19 n distinct slots: each slot
    exactly once.  For the full list, the 16-bit and the 8-bit codes."""
    g = I.pbb_box(4, n=40)
    print_case("adjoint scatter permutation", order, "pbb_box 40^3")
    lat = L.build(dev_flags(g), g.periodic, order, 5 if order == "random" else 0)
    n, S = lat.n_fluid, lat.stride
    comp = L.narrow(L.compress(lat))
    f = torch.from_numpy(random_state(n, 4, amp=1e-3, shifted=True, stride=S)).cuda()
    lam = torch.zeros((19, S), dtype=torch.float64, device="cuda")
    lam[:, :n] = torch.rand((19, n), dtype=torch.float64,
                            generator=torch.Generator().manual_seed(7)).cuda()
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64s")
    for form in ("full", "c16", "c8"):
        lt = torch.full((19, S), float("nan"), dtype=torch.float64, device="cuda")
        if form == "c16":
            rc = N.lbm_step_adjoint_c16(prm, n, S, comp.codes, comp.tile_records, lat.adj, f,
                                        None, lam, lt, None)
        elif form == "c8":
            rc = N.lbm_step_adjoint_c8(prm, n, S, comp.codes8, comp.codes, comp.tile_records,
                                       lat.adj, f, None, lam, lt, None)
        else:
            rc = N.lbm_step_adjoint(prm, n, S, lat.adj, f, None, lam, lt, None)
        assert rc == 0
        assert torch.isfinite(lt[:, :n]).all(), form
        assert torch.isnan(lt[:, n:]).all(), form  # nothing outside the list


def test_gradient_vs_oracle_with_checkpoints(pbb):
    g, sp, lat, ns = pbb
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64s")
    T, k = 23, 5
    n = sp.n_fluid
    nsd = torch.from_numpy(ns).cuda()
    J_gpu, _, _ = AD.forward_states(lat, prm, nsd, T, k)
    grad_gpu = AD.adjoint_gradient(lat, prm, nsd, T, k).cpu().numpy()[:n]
    J, grad = ogradient(prm, sp, ns, T)
    assert abs(J_gpu.item() - J) <= 1e-12 * abs(J)
    assert np.abs(grad_gpu - grad).max() <= 1e-12 * np.abs(grad).max()


@pytest.mark.parametrize("snapshots", [0, 1, 3, 8, 30])
def test_revolve_gradient_is_bitwise_two_level(pbb, snapshots):
    """Binomial checkpointing with 0 to 30 snapshot slots delivers the same
    states in the same order as two-level checkpointing, so the gradient is
    bitwise the same; it runs exactly the schedule's optimal number of
    forward sweeps."""
    from paper_1111_1129_amd.checkpointing import revolve_closed_form
    g, sp, lat, ns = pbb
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64s")
    T, k = 23, 5
    print_case("revolve", snapshots, T)
    nsd = torch.from_numpy(ns).cuda()
    ref = AD.adjoint_gradient(lat, prm, nsd, T, k)
    stats = {}
    grad = AD.adjoint_gradient_revolve(lat, prm, nsd, T, snapshots, stats=stats)
    assert torch.equal(grad, ref)
    assert stats["forward_sweeps"] == revolve_closed_form(T, snapshots + 1)


def test_permeability_autograd_revolve(pbb):
    g, sp, lat, ns = pbb
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64s")
    nsd = torch.from_numpy(ns).cuda().requires_grad_(True)
    J = AD.PermeabilityFn.apply(nsd, lat, prm, 12, 4, 2)  # 2 snapshot slots
    J.backward()
    _, grad = ogradient(prm, sp, ns, 12)
    g = nsd.grad.cpu().numpy()[:sp.n_fluid]
    assert np.abs(g - grad).max() <= 1e-12 * np.abs(grad).max()


def test_permeability_autograd(pbb):
    g, sp, lat, ns = pbb
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64s")
    nsd = torch.from_numpy(ns).cuda().requires_grad_(True)
    J = AD.PermeabilityFn.apply(nsd, lat, prm, 12, 4)
    J.backward()
    _, grad = ogradient(prm, sp, ns, 12)
    g = nsd.grad.cpu().numpy()[:sp.n_fluid]
    assert np.abs(g - grad).max() <= 1e-12 * np.abs(grad).max()


def test_batched_equals_solo():
    geoms = [I.packing_boolean(50 + k, L_, L_, L_, 2.0, 4.0, p)
             for k, (L_, p) in enumerate([(17, 0.5), (24, 0.4), (9, 0.6)])]
    batch = L.Batch([dev_flags(g) for g in geoms], [g.periodic for g in geoms], "morton2")
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f32")
    st = batch.init(prm)
    L.step(st, 13)
    fb = st.f.cpu().numpy()[:, :batch.total]
    stp = batch.init(prm)
    L.step(stp, 13, persistent=True, segments=batch.segments)
    np.testing.assert_array_equal(stp.f.cpu().numpy()[:, :batch.total], fb)
    _, _, tot = L.moments(st, fields=False, segments=batch.segments)
    for k, g in enumerate(geoms):
        print_case("batched member", k, g.dims)
        lat = L.build(dev_flags(g), g.periodic, "morton2")
        solo = L.init(lat, prm)
        L.step(solo, 13)
        b, c = batch.segments[k]
        np.testing.assert_array_equal(fb[:, b:b + c], solo.f.cpu().numpy()[:, :c])
        _, _, ts = L.moments(solo, fields=False)
        np.testing.assert_array_equal(tot[k].cpu().numpy(), ts[0].cpu().numpy())


def test_batched_over_codes_equals_per_step():
    """A lexicographic batch of uneven packings swept over 16-bit and over
    8-bit codes (tiles straddling two members included) ends in the state of
    the full-list sweep, two arrays and in place."""
    geoms = [I.packing_boolean(60 + k, L_, L_, L_, 2.0, 4.0, p)
             for k, (L_, p) in enumerate([(40, 0.5), (33, 0.4), (21, 0.6), (48, 0.45)])]
    batch = L.Batch([dev_flags(g) for g in geoms], [g.periodic for g in geoms], "lex")
    print_case("batched codes", batch.total)
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f32s")
    ref = batch.init(prm)
    L.step(ref, 12)
    comp = L.compress(batch.lattice, n=batch.total)
    s16 = batch.init(prm)
    L.step_c16(s16, comp, 12)
    L.narrow(comp)
    assert comp.n_narrow > 0
    s8 = batch.init(prm)
    L.step_c8(s8, comp, 12)
    one = L.init_inplace(batch.lattice, prm, n=batch.total)
    L.step_inplace(one, 12, comp, c8=True)
    for st in (s16, s8, one):
        assert torch.equal(st.f[:, :batch.total], ref.f[:, :batch.total])


@pytest.fixture(scope="module")
def full_batch():
    """The 64 packings of the batched workload (38.4 M cells) in one batch."""
    geoms = I.batch_packings()
    batch = L.Batch([dev_flags(g) for g in geoms], [g.periodic for g in geoms], "lex")
    yield geoms, batch
    del batch
    torch.cuda.empty_cache()


def test_batch_full_size_persistent_step_vs_oracle(full_batch):
    """The 64-packing batch of the batched experiment (38.4 M cells) at full
    size, one persistent-launch FP32 step from a seeded state: the head and
    the ragged tail of every member against the oracle.  The slots each
    sampled cell reads come from the oracle's own adjacency of the member,
    placed at the member's columns; FP32 bound as for the one-step test of
    the small packing (one FP32 ulp + 64 eps32)."""
    from gpu_helpers import W
    geoms, batch = full_batch
    lat, S = batch.lattice, batch.lattice.stride
    print_case("batch full size", len(geoms), batch.total)
    cells, slots = [], []
    for g, (base, cnt) in zip(geoms, batch.segments):
        sp = O.build(g.flags, g.periodic, "lex")
        assert sp.n_fluid == cnt
        Sk = sp.adj.shape[1]
        m = np.concatenate([np.arange(0, min(256, cnt)), np.arange(max(cnt - 200, 256), cnt)])
        a = sp.adj[:, m].astype(np.int64)
        cells.append(base + m)
        slots.append(np.vstack([base + m, (a // Sk) * S + base + a % Sk]))
    cells = np.concatenate(cells)
    slots = np.concatenate(slots, axis=1)
    k = cells.size
    rng = np.random.default_rng(21)
    vals = (W[slots // S] * (1.0 + 0.02 * rng.standard_normal(slots.shape))).astype(np.float32)
    prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), "f32", nontemporal=True, xcd_chunk=16)
    st = batch.init(prm)
    st.f.copy_(torch.from_numpy(W.astype(np.float32)).cuda()[:, None].expand(19, S))
    st.f.view(-1)[torch.from_numpy(slots.ravel()).cuda()] = torch.from_numpy(vals.ravel()).cuda()
    L.step(st, 1, persistent=True, segments=batch.segments)
    got = st.f[:, torch.from_numpy(cells).cuda()].cpu().numpy().astype(np.float64)
    ident = ((np.arange(1, 19, dtype=np.uint64)[:, None] * k + np.arange(k, dtype=np.uint64)[None, :])
             .astype(np.uint32))
    exact = np.zeros((19, k))
    O.step(oracle_params(prm), ident, np.ascontiguousarray(vals.astype(np.float64)), exact)
    orc = O.round_storage(exact, "f32")
    tol = np.spacing(np.abs(exact).astype(np.float32)).astype(np.float64) + 64 * np.finfo(np.float32).eps
    assert (np.abs(got - orc) <= tol).all()


def test_batch_full_size_persistent_steps_equal_per_step(full_batch):
    """The full 64-packing batch from a seeded state: 4 FP32 steps in one
    persistent launch (the grid barrier between steps runs 3 times at this
    size) give the same bits as 4 launches of one step each, in the batched
    experiment's launch configuration and with the hardware round robin."""
    geoms, batch = full_batch
    S, n = batch.stride, batch.total
    print_case("batch full size persistent", n)
    gen = torch.Generator(device="cuda").manual_seed(23)
    w = torch.tensor([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12, dtype=torch.float32, device="cuda")
    f0 = w[:, None] * (1 + 0.02 * torch.randn((19, S), generator=gen, device="cuda",
                                               dtype=torch.float32))
    for nt, chunk in ((True, 16), (False, 1)):
        prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), "f32", nontemporal=nt, xcd_chunk=chunk)
        a = batch.init(prm)
        a.f.copy_(f0)
        L.step(a, 4)
        b = batch.init(prm)
        b.f.copy_(f0)
        L.step(b, 4, persistent=True, segments=batch.segments)
        assert torch.equal(a.f[:, :n], b.f[:, :n]), (nt, chunk)
        del a, b


def test_adjoint_vs_central_differences_full_size():
    """128^3 box with a partial-bounce-back field, 500 shifted-FP64 steps,
    checkpoints every 22 steps: the adjoint gradient of the mean flux matches
    central differences (h = 1e-4, per-cell velocity differences) within 1e-6
    on all 32 cells drawn with seed 44 from 0.05 < ns < 0.95."""
    g = I.pbb_box(4, n=128)
    lat = L.build(dev_flags(g), g.periodic, "lex")
    n, S = lat.n_fluid, lat.stride
    ns_host = np.zeros(S)
    ns_host[:n] = g.ns.ravel()[lat.cell_of.cpu().numpy()]
    ns = torch.from_numpy(ns_host).cuda()
    prm = L.params(0.8, 3 / 16, (1e-6, 0, 0), "f64s")
    T, k = 500, 22
    grad = AD.adjoint_gradient(lat, prm, ns, T, k).cpu().numpy()

    def ux(nsv):
        st = L.init(lat, prm, ns=nsv)
        L.step(st, T)
        return L.moments(st)[1][0]

    rng = np.random.default_rng(44)
    inner = np.flatnonzero((ns_host[:n] > 0.05) & (ns_host[:n] < 0.95))
    for c in rng.choice(inner, 32, replace=False):
        h = 1e-4
        e = torch.zeros(S, dtype=torch.float64, device="cuda")
        e[int(c)] = h
        fd = float((ux(ns + e) - ux(ns - e)).sum()) / n / (2 * h)
        print_case("fd cell", int(c), grad[c], fd)
        assert abs(grad[c] - fd) <= 1e-6 * abs(fd)


def test_persistent_full_grid_equals_per_step():
    """A persistent launch large enough to fill the device (every workgroup
    slot the grid barrier relies on) gives the same bits as one launch per
    step, for FP32 and for FP64 with partial bounce-back."""
    g = I.packing_tube(2)
    lat = L.build(dev_flags(g), g.periodic, "lex")
    n = lat.n_fluid
    ns = torch.rand(lat.stride, dtype=torch.float64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(3))
    for storage, nsv in (("f32", None), ("f64s", ns)):
        prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), storage)
        a = L.init(lat, prm, ns=nsv)
        L.step(a, 7)
        b = L.init(lat, prm, ns=nsv)
        L.step(b, 7, persistent=True)
        assert torch.equal(a.f[:, :n], b.f[:, :n]), storage
