"""Pins of the oracle's adjoint step (CPU only).

The adjoint is checked against complex-step differentiation of the oracle's
own forward step (exact to rounding, an independent route to the same
derivative), by the dot-product identity <lam, D v> = <D^T lam, v> for one
step, and against central finite differences.
"""
import numpy as np
import pytest

import oracle as O
from paper_1111_1129_amd import inputs as I


def small_case(n=8, seed=4):
    g = I.pbb_box(seed=seed, n=n)
    sp = O.build(g.flags, g.periodic, "lex")
    ns = np.ascontiguousarray(g.ns.ravel()[sp.cell_of])
    return g, sp, ns


def test_seed_is_objective_gradient():
    _, sp, ns = small_case()
    prm = O.TRT(0.8, 3 / 16, (1e-5, 0, 0))
    rng = np.random.default_rng(1)
    f = O.init(sp.n_fluid, shifted=True) + 1e-4 * rng.standard_normal((19, sp.n_fluid))
    lam = np.zeros_like(f)
    O.adjoint_step(prm, sp.adj, f, ns, None, lam, None)
    v = rng.standard_normal(f.shape)
    h = 1e-30
    dJ = O.objective(prm, sp.adj, f.astype(np.complex128) + 1j * h * v, shifted=True).imag / h
    assert abs((lam * v).sum() - dJ) <= 1e-13 * abs(dJ)


@pytest.mark.parametrize("with_ns", [False, True])
def test_dot_product_one_step(with_ns):
    """<lam, D_f v> + <lam, D_ns dns> = <D_f^T lam, v> + <grad, dns>, with the
    forward tangent D v taken by complex step through the forward step."""
    _, sp, ns = small_case()
    if not with_ns:
        ns_used = None
    else:
        ns_used = ns
    prm = O.TRT(0.8, 3 / 16, (2e-5, -1e-5, 3e-6))
    rng = np.random.default_rng(2)
    N = sp.n_fluid
    w = np.array([O.weight(i) for i in range(19)])
    f = w[:, None] * (1 + 0.05 * rng.standard_normal((19, N)))
    lam = rng.standard_normal((19, N))
    v = rng.standard_normal((19, N))
    dns = rng.standard_normal(N) if with_ns else np.zeros(N)
    h = 1e-30
    out = np.empty((19, N), dtype=np.complex128)
    ns_c = None if ns_used is None else ns_used + 1j * h * dns
    O.step(prm, sp.adj, f + 1j * h * v, out, ns=ns_c)
    lhs = (lam * (out.imag / h)).sum()
    lam_t = np.zeros_like(f)
    grad = np.zeros(N)
    O.adjoint_step(prm, sp.adj, f, ns_used, lam, lam_t, grad)
    rhs = (lam_t * v).sum() + (grad * dns).sum()
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), abs(lam * v).sum())


def test_adjoint_scatter_covers_every_slot_once():
    """Each lambda^t slot is written by exactly one (cell, direction): fill
    lambda^{t+1} with NaN-free values and check no slot keeps the sentinel."""
    _, sp, ns = small_case()
    prm = O.TRT(0.8, 3 / 16, (1e-5, 0, 0))
    N = sp.n_fluid
    f = O.init(N, shifted=True)
    lam = np.ones((19, N))
    lam_t = np.full((19, N), np.nan)
    O.adjoint_step(prm, sp.adj, f, ns, lam, lam_t, np.zeros(N))
    assert np.isfinite(lam_t).all()


def test_gradient_matches_complex_step():
    _, sp, ns = small_case()
    prm = O.TRT(0.8, 3 / 16, (1e-5, 0, 0))
    f0 = O.init(sp.n_fluid, shifted=True)
    T = 30
    J, grad = O.gradient(prm, sp.adj, f0, ns, T, shifted=True)
    rng = np.random.default_rng(3)
    for _ in range(2):
        d = rng.standard_normal(sp.n_fluid)
        cs = O.complex_step_derivative(prm, sp.adj, f0, ns, d, T, shifted=True)
        assert abs(grad @ d - cs) <= 1e-12 * abs(cs)
    for cell in rng.choice(sp.n_fluid, 3, replace=False):
        e = np.zeros(sp.n_fluid)
        e[cell] = 1.0
        cs = O.complex_step_derivative(prm, sp.adj, f0, ns, e, T, shifted=True)
        assert abs(grad[cell] - cs) <= 1e-11 * abs(cs) + 1e-24


def test_gradient_matches_central_differences():
    _, sp, ns = small_case()
    prm = O.TRT(0.8, 3 / 16, (1e-5, 0, 0))
    f0 = O.init(sp.n_fluid, shifted=True)
    T = 30
    _, grad = O.gradient(prm, sp.adj, f0, ns, T, shifted=True)
    rng = np.random.default_rng(5)
    inner = np.flatnonzero((ns > 0.05) & (ns < 0.95))
    for cell in rng.choice(inner, 4, replace=False):
        h = 1e-4
        Jp = O.objective(prm, sp.adj, O.run(prm, sp.adj, f0, T, ns=ns + h * (np.arange(len(ns)) == cell)), True)
        Jm = O.objective(prm, sp.adj, O.run(prm, sp.adj, f0, T, ns=ns - h * (np.arange(len(ns)) == cell)), True)
        fd = (Jp - Jm) / (2 * h)
        assert abs(grad[cell] - fd) <= 1e-6 * abs(fd)
