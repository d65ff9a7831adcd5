"""Shared helpers for the GPU parity tests (test side only)."""
import numpy as np
import torch

import oracle as O

W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def dev_flags(geom):
    return torch.from_numpy(np.ascontiguousarray(geom.flags)).cuda()


def adj_u32(lat):
    return lat.adj.cpu().numpy().view(np.uint32)


def rel_err_f64(gpu: np.ndarray, orc: np.ndarray, shifted: bool = False) -> float:
    """max |f_gpu - f_orc| / |f_orc| over unshifted values (f >= ~0.01)."""
    if shifted:
        gpu = gpu + W[:, None]
        orc = orc + W[:, None]
    return float(np.max(np.abs(gpu - orc) / np.abs(orc)))


def random_state(n, seed, amp=0.02, shifted=False, stride=None):
    rng = np.random.default_rng(seed)
    stride = n if stride is None else stride
    f = np.zeros((19, stride))
    f[:, :n] = W[:, None] * (1.0 + amp * rng.standard_normal((19, n)))
    if shifted:
        f[:, :n] -= W[:, None]
    return f


def oracle_params(prm):
    return O.TRT(prm.tau_plus, prm.magic, tuple(prm.force))


def print_case(*args):
    print("CASE", *args, flush=True)
