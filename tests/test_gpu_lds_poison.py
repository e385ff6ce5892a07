"""The LDS-poison check: the test build of the library fills every LDS array
with NaN before each kernel uses it.  Every kernel family's outputs (forward,
adjoint, screens, moments and statistics, AR step, receiver, uneven batch)
must be the same bits as the product build's, and finite: no kernel reads LDS
that it did not write first."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2604_07248_amd import build

from gpu_helpers import say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_poisoned_lds_gives_the_same_bits(gpu_lib, tmp_path):
    if not os.path.exists(build.POISON_LIB):
        pytest.fail("libturpy_poison.so is not built (run __graft_entry__.build())")
    sys.path.insert(0, HERE)
    import lds_poison_cases
    ref = lds_poison_cases.run_cases()
    out = str(tmp_path / "poison.npz")
    env = dict(os.environ, TURPY_LIBRARY=build.POISON_LIB)
    say("[poison] child process with the poison build")
    res = subprocess.run([sys.executable, "-u", os.path.join(HERE, "lds_poison_cases.py"), out], env=env,
                         capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-3000:]
    got = np.load(out)
    assert sorted(got.files) == sorted(ref)
    for name, want in ref.items():
        have = got[name]
        assert np.isfinite(have).all(), name
        assert have.shape == want.shape and np.array_equal(have.view(np.uint8), want.view(np.uint8)), name
    say(f"[poison] {len(ref)} outputs bitwise equal")
