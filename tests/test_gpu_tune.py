"""The ordering tuner (the paper's proposal to pick the numbering by
simulating samples of the geometry on the target machine, Sec. 8) on the
full tube: it returns one of its candidates with an aligned layout, and the
sparse representation built in the chosen ordering is the oracle's, bit for
bit."""
import numpy as np
import pytest

import oracle as O
from paper_1111_1129_amd import inputs as I
from paper_1111_1129_amd import lattice as L
from paper_1111_1129_amd.tune import ORDER_CANDIDATES, tune_ordering

from gpu_helpers import adj_u32, dev_flags, print_case

pytestmark = pytest.mark.gpu


def test_tune_ordering_on_tube_sample():
    g = I.packing_tube(2)
    flags = dev_flags(g)
    print_case("tune_ordering tube sample 1/8")
    order, param, lay, table = tune_ordering(flags, g.periodic, sample=1 / 8)
    assert (order, param) in ORDER_CANDIDATES
    assert {(o, p) for o, p, _ in table} == set(ORDER_CANDIDATES)
    assert all(r > 0 for _, _, r in table)
    assert lay.mflups > 0 and lay.stride % L.ROW_ALIGN == 0
    lat = L.build(flags, g.periodic, order, param, stride=lay.stride)
    n = lat.n_fluid
    assert lay.stride >= n
    sp = O.build(g.flags, g.periodic, order, param, stride=lat.stride)
    assert sp.n_fluid == n
    np.testing.assert_array_equal(lat.index_of.cpu().numpy(), sp.index_of)
    np.testing.assert_array_equal(lat.cell_of.cpu().numpy(), sp.cell_of)
    np.testing.assert_array_equal(adj_u32(lat)[:, :n], sp.adj[:, :n])
