"""Kill and resume: a run interrupted after 50 of 100 steps, its checkpoint
written by one process and read back by another, continues bitwise into the
uninterrupted run -- also when the restart picks another numbering, which the
paper allows at every restart (Sec. 8)."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

from paper_1111_1129_amd import inputs as I
from paper_1111_1129_amd import lattice as L

from gpu_helpers import dev_flags, print_case

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys, torch
sys.path.insert(0, {root!r})
from paper_1111_1129_amd import inputs as I, lattice as L
g = I.packing_boolean(5, 40, 36, 32, 2.0, 5.0, 0.45)
flags = torch.from_numpy(g.flags).cuda()
lat = L.build(flags, g.periodic, "lex")
ns = torch.linspace(0, 0.3, lat.stride, dtype=torch.float64, device="cuda")
st = L.init(lat, L.params(0.8, 3 / 16, (1e-5, 2e-6, 0.0), {storage!r}), ns=ns)
L.step(st, 50)
torch.save(L.checkpoint(st), {path!r})
print("saved", st.steps, flush=True)
"""


@pytest.mark.parametrize("storage,order", [("f64", "lex"), ("f64", "morton2"),
                                           ("f16s", "hilbert")])
def test_resume_in_new_process_equals_uninterrupted(tmp_path, storage, order):
    print_case("resume", storage, order)
    g = I.packing_boolean(5, 40, 36, 32, 2.0, 5.0, 0.45)
    flags = dev_flags(g)
    lat = L.build(flags, g.periodic, "lex")
    ns = torch.linspace(0, 0.3, lat.stride, dtype=torch.float64, device="cuda")
    ref = L.init(lat, L.params(0.8, 3 / 16, (1e-5, 2e-6, 0.0), storage), ns=ns)
    L.step(ref, 100)

    path = str(tmp_path / "ckpt.pt")
    res = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, storage=storage,
                                                               path=path)],
                         capture_output=True, text=True, timeout=300)
    assert res.returncode == 0 and "saved 50" in res.stdout, res.stderr[-2000:]
    ck = torch.load(path, weights_only=True)
    st = L.restore(ck, flags, order=order)
    assert st.steps == 50 and st.lattice.order == order
    L.step(st, 50)
    # back to the reference's (lexicographic) list order
    n = lat.n_fluid
    idx = st.lattice.index_of.to(torch.int64)[lat.cell_of.to(torch.int64)]
    assert torch.equal(st.f[:, idx], ref.f[:, :n])


def test_restore_rejects_another_geometry():
    g = I.packing_boolean(5, 40, 36, 32, 2.0, 5.0, 0.45)
    lat = L.build(dev_flags(g), g.periodic, "lex")
    st = L.init(lat, L.params(0.8, 3 / 16, (1e-5, 0, 0), "f64"))
    ck = L.checkpoint(st)
    other = I.packing_boolean(6, 40, 36, 32, 2.0, 5.0, 0.45)
    with pytest.raises(ValueError):
        L.restore(ck, dev_flags(other))
    with pytest.raises(ValueError):
        L.restore(ck, dev_flags(I.packing_boolean(5, 40, 36, 31, 2.0, 5.0, 0.45)))
