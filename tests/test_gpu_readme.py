"""The usage example in README.md runs as written on the GPU (the documented calls,
including the workspace reservation that compute calls need)."""
import os
import re

import pytest
import torch

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example_runs():
    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, flags=re.S)
    assert blocks, "README.md has no python example"
    for code in blocks:
        exec(compile(code, "README.md", "exec"), {"__name__": "readme_example"})
    torch.cuda.synchronize()
