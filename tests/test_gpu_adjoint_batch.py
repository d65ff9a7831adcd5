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
    sp = O.build(g.flags, g.periodic, "lex")
    lat = L.build(dev_flags(g), g.periodic, "lex")
    ns = np.ascontiguousarray(g.ns.ravel()[sp.cell_of])
    return g, sp, lat, ns


def test_adjoint_step_vs_oracle(pbb):
    g, sp, lat, ns = pbb
    n = sp.n_fluid
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64s")
    op = oracle_params(prm)
    f = random_state(n, 1, amp=1e-3, shifted=True)
    lam = np.random.default_rng(2).standard_normal((19, n))
    o_lam, o_grad = np.zeros((19, n)), np.zeros(n)
    O.adjoint_step(op, sp.adj, f, ns, lam, o_lam, o_grad)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g_lam = torch.empty((19, n), dtype=torch.float64, device="cuda")
    g_grad = torch.zeros(n, dtype=torch.float64, device="cuda")
    rc = N.lbm_step_adjoint(prm, n, n, lat.adj, d(f), d(ns), d(lam), g_lam, g_grad)
    assert rc == 0
    np.testing.assert_allclose(g_lam.cpu().numpy(), o_lam, rtol=0, atol=1e-13 * np.abs(o_lam).max())
    np.testing.assert_allclose(g_grad.cpu().numpy(), o_grad, rtol=0, atol=1e-13 * np.abs(o_grad).max())
    # seed
    seed = torch.empty((19, n), dtype=torch.float64, device="cuda")
    assert N.lbm_step_adjoint(prm, n, n, lat.adj, None, None, None, seed, None) == 0
    o_seed = np.zeros((19, n))
    O.adjoint_step(op, sp.adj, f, ns, None, o_seed, None)
    np.testing.assert_array_equal(seed.cpu().numpy(), o_seed)


def test_gradient_vs_oracle_with_checkpoints(pbb):
    g, sp, lat, ns = pbb
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64s")
    T, k = 23, 5
    nsd = torch.from_numpy(ns).cuda()
    J_gpu, _, _ = AD.forward_states(lat, prm, nsd, T, k)
    grad_gpu = AD.adjoint_gradient(lat, prm, nsd, T, k).cpu().numpy()
    J, grad = O.gradient(oracle_params(prm), sp.adj, O.init(sp.n_fluid, shifted=True), ns, T,
                         shifted=True)
    assert abs(J_gpu.item() - J) <= 1e-12 * abs(J)
    assert np.abs(grad_gpu - grad).max() <= 1e-12 * np.abs(grad).max()


def test_permeability_autograd(pbb):
    g, sp, lat, ns = pbb
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64s")
    nsd = torch.from_numpy(ns).cuda().requires_grad_(True)
    J = AD.PermeabilityFn.apply(nsd, lat, prm, 12, 4)
    J.backward()
    _, grad = O.gradient(oracle_params(prm), sp.adj, O.init(sp.n_fluid, shifted=True), ns, 12,
                         shifted=True)
    assert np.abs(nsd.grad.cpu().numpy() - grad).max() <= 1e-12 * np.abs(grad).max()


def test_batched_equals_solo():
    geoms = [I.packing_boolean(50 + k, L_, L_, L_, 2.0, 4.0, p)
             for k, (L_, p) in enumerate([(17, 0.5), (24, 0.4), (9, 0.6)])]
    batch = L.Batch([dev_flags(g) for g in geoms], [g.periodic for g in geoms], "morton2")
    prm = L.params(0.8, 3 / 16, (1e-5, 0, 0), "f32")
    st = batch.init(prm)
    L.step(st, 13)
    fb = st.f.cpu().numpy()
    stp = batch.init(prm)
    L.step(stp, 13, persistent=True, segments=batch.segments)
    np.testing.assert_array_equal(stp.f.cpu().numpy(), fb)
    _, _, tot = L.moments(st, fields=False, segments=batch.segments)
    for k, g in enumerate(geoms):
        print_case("batched member", k, g.dims)
        lat = L.build(dev_flags(g), g.periodic, "morton2")
        solo = L.init(lat, prm)
        L.step(solo, 13)
        b, c = batch.segments[k]
        np.testing.assert_array_equal(fb[:, b:b + c], solo.f.cpu().numpy())
        _, _, ts = L.moments(solo, fields=False)
        np.testing.assert_array_equal(tot[k].cpu().numpy(), ts[0].cpu().numpy())
