"""The library loaded before torch in a fresh process: the binding must
still run on torch's HIP runtime (streams and memory come from torch)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, ROOT)
from paper_2006_07057_amd import _lib
_lib.lib()                      # before anything imports torch here
import numpy as np
import torch
from paper_2006_07057_amd import api
rng = np.random.default_rng(0)
X = torch.from_numpy(rng.standard_normal((300, 3)).astype(np.float32)).cuda()
U = torch.from_numpy(rng.standard_normal((127, 3)).astype(np.float32)).cuda()
Phi, ls = api.features_arccos(X, U, 1, 1.5, 0.5)
P2, s2 = api.features(X, U[:124].contiguous(), 0.5, 8.0)
torch.cuda.synchronize()
assert bool(torch.isfinite(Phi).all()) and bool(torch.isfinite(P2).all())
print("child ok", flush=True)
""".replace("ROOT", repr(ROOT))


@pytest.mark.gpu
def test_library_loaded_before_torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = subprocess.run([sys.executable, "-c", CHILD], capture_output=True, text=True,
                       timeout=240, cwd=ROOT)
    assert p.returncode == 0 and "child ok" in p.stdout, (p.stdout[-2000:], p.stderr[-2000:])
