"""The Python example of README.md runs as written (a plate with a hole
under a normal traction, read-outs included)."""
import os
import re

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example_runs(gpu):
    with open(os.path.join(ROOT, "README.md")) as fh:
        code = re.search(r"```python\n(.*?)```", fh.read(), re.S).group(1)
    ns = {}
    exec(compile(code, "README.md", "exec"), ns)
    from paper_2208_13769_amd import lbm

    assert ns["status"] == lbm.LBM_OK and ns["diag"].steps == 416
    u, W = ns["u"], ns["W"]
    assert np.all(np.isfinite(u)) and 0.0 < np.abs(u).max() < 0.1
    assert np.all(u[:, 24:56, 24:56] == 0.0) and np.all(W[24:56, 24:56] == 0.0)  # the hole
    ns["s"].close()
