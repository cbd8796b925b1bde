"""Shared helpers of the GPU parity tests (inputs from synth, expected values
from oracle, results from the HIP library through its C-ABI binding)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def gpu_available():
    return torch.cuda.is_available()


requires_gpu = pytest.mark.skipif(not gpu_available(), reason="needs a ROCm GPU")


def lib():
    import paper_1007_4591_amd as B
    return B


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    return t.to(dtype) if dtype is not None else t


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def leaf_boxes(tree, pos):
    """Lower and upper corners of the leaf box of each point (from the tree's
    root cube and leaf level; a point's leaf is fixed when the tree is built)."""
    inf = tree.info
    sL = inf["side"] / 2 ** inf["leaf_level"]
    lo = np.asarray(inf["lo"])
    c = np.floor((np.asarray(pos) - lo) / sL)
    return lo + c * sL, lo + (c + 1) * sL, sL
