"""The usage example of README.md runs as written (8^4 doublet: operator,
mixed CG, action and gradient) and its solve reaches the stated residual."""
import os
import re

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example_runs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, re.S)
    assert blocks, "README has no python example"
    ns = {}
    exec(compile(blocks[0], "README.md example", "exec"), ns)
    res = ns["res"]
    assert res["status"] == 0 and res["true_rel_res_normal"] <= 1e-10, res
    grad = ns["Ur"].grad
    assert grad is not None and torch.isfinite(grad).all()
    assert ns["x_canonical"].shape == ns["b"].shape
