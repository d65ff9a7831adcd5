"""The largest row stride the 32-bit slot index allows (19 * stride < 2^32):
every sweep form, placed at that stride, gives bitwise the state it gives
at a small stride, so no slot arithmetic near the top row overflows."""
import numpy as np
import pytest
import torch

from paper_1111_1129_amd import inputs as I
from paper_1111_1129_amd import lattice as L
from paper_1111_1129_amd.tune import SWEEPS, Sweeper

from gpu_helpers import dev_flags, print_case

pytestmark = pytest.mark.gpu

# the largest multiple of 64 (128-byte FP16 rows) with 19 * stride < 2^32
MAX_STRIDE = ((2 ** 32 - 1) // 19) // 64 * 64


def test_max_stride_constant():
    assert 19 * MAX_STRIDE < 2 ** 32 <= 19 * (MAX_STRIDE + 64)


@pytest.mark.parametrize("storage", ["f16s", "f64"])
def test_every_sweep_at_the_largest_stride(storage):
    g = I.packing_small(1)
    flags = dev_flags(g)
    prm = L.params(0.8, 3 / 16, (1e-5, 2e-6, 0), storage, nontemporal=True, xcd_chunk=1)
    small = L.build(flags, g.periodic, "lex", 0)
    n = small.n_fluid
    ref = L.init(small, prm)
    L.step(ref, 6)
    want = ref.f[:, :n].clone()
    del ref, small
    print_case("largest stride", storage, MAX_STRIDE, n)
    lat = L.build(flags, g.periodic, "lex", 0, stride=MAX_STRIDE)
    assert lat.stride == MAX_STRIDE and lat.n_fluid == n
    # the adjacency names slots in the top rows: the last row starts at 17 * stride
    adj = lat.adj[:, :n].cpu().numpy().view(np.uint32).astype(np.int64)
    assert adj.max() >= 17 * MAX_STRIDE
    for kind in SWEEPS:
        sw = Sweeper(lat, kind)
        st = sw.init(prm)
        sw.step(st, 6)
        torch.cuda.synchronize()
        assert torch.equal(st.f[:, :n], want), kind
        del st, sw
        torch.cuda.empty_cache()
