"""Device memory returned to the driver instead of cached: with a 1 MB cache
limit every block of a destroyed tree goes back through hipFree, and the
next build allocates afresh.  Products must be bitwise those of the first
build.  The cache limit is read once per process, so the case runs in a
child process (the parent only waits for it)."""
import os
import subprocess
import sys

import pytest

from gpu_common import requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np, torch, synth
import paper_1007_4591_amd as B
p = synth.blobby(4)
x = torch.as_tensor(np.random.default_rng(5).normal(size=p.n_panels), device="cuda")
outs = []
for rep in range(3):
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params(ncrit=16))
    outs.append([B.fmm_matvec(t, op, prec, x).cpu().numpy() for op in (B.OP_A, B.OP_AT) for prec in (B.FP64, B.FP32)])
    B.tree_destroy(t)
    print("rep", rep, "done", flush=True)
same = all(np.array_equal(a, b) for o in outs[1:] for a, b in zip(outs[0], o))
print("BITWISE" if same else "DIFFERENT", flush=True)
"""


def test_uncached_rebuild_is_bitwise():
    env = dict(os.environ, BEMFMM_CACHE_LIMIT_MB="1")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True, text=True, timeout=110)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0
    assert "BITWISE" in r.stdout
