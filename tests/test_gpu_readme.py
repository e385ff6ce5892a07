"""The usage example of README.md runs as written (headline workload: tuning,
moments bound to the plan, forward with checkpoints, adjoint with the shared
source's gradient, finalized statistics)."""
import os
import re

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example_runs(gpu_lib):
    with open(os.path.join(ROOT, "README.md")) as f:
        blocks = re.findall(r"```python\n(.*?)```", f.read(), re.S)
    assert blocks, "README.md has no python example"
    scope = {}
    exec(compile(blocks[0], "README.md", "exec"), scope)
    import torch
    torch.cuda.synchronize()
    u_out, g_in, summary = scope["u_out"], scope["g_in"], scope["summary"]
    assert u_out.shape == (64, 1024, 1024) and g_in.shape == (1024, 1024)
    assert bool(torch.isfinite(torch.view_as_real(u_out)).all()) and bool(torch.isfinite(torch.view_as_real(g_in)).all())
    assert summary["count"] == 64
