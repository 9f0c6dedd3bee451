"""Regression: importing the package before torch must leave both on one
HIP runtime (the binding loads torch before libmxr.so)."""
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_package_first_then_torch():
    code = ("import paper_2410_08747_amd as m, torch, numpy as np\n"
            "x = torch.tensor(np.ones((2, 5)), device='cuda')\n"
            "mean, rel = m.batch_means(x, 10)\n"
            "torch.cuda.synchronize()\n"
            "assert abs(mean.sum().item() - 0.5) < 1e-12\n"
            "print('ok')\n")
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr
