"""The quick-start example of the README runs as written: the CIR workload
with 10^6 protons through the binding, and its observer intensities are
finite, non-negative and not all zero, with finite batch errors."""
import os
import re

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_quick_start():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, re.S)
    assert len(blocks) == 1
    ns = {}
    exec(compile(blocks[0], "README.md", "exec"), ns)
    j, sigma = ns["j"], ns["sigma"]
    print(f"bins {j.size}, nonzero {(j > 0).sum()}, max {j.max():.3e}")
    assert np.isfinite(j).all() and np.isfinite(sigma).all()
    assert (j >= 0).all() and (j > 0).sum() > 10
