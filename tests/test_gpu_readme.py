"""The README's Python example runs as written and prints what it says: -12 for the
Majumdar-Ghosh point of the L = 32 J1-J2 chain, and a mixed-dimension ring energy."""
import contextlib
import io
import os
import re

import pytest

pytestmark = pytest.mark.gpu


def test_readme_python_example():
    text = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "README.md")).read()
    code = re.search(r"```python\n(.*?)```", text, re.S).group(1)
    buf = io.StringIO()
    with contextlib.redirect_stdout(buf):
        exec(compile(code, "README.md", "exec"), {})
    lines = [ln for ln in buf.getvalue().splitlines() if ln.strip()]
    print(lines)
    assert abs(float(lines[0]) + 12.0) <= 1e-6  # E0 = -3L/8 at J2/J1 = 1/2
    assert float(lines[1]) < 0.0
