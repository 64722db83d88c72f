"""The bounds-checked build (libmgs_checked.so, MGS_CHECK_BOUNDS): every render path run
through it reports no index outside its bound, and its images and gradients equal the normal
library's bit for bit (the checks change no result); a planted pair count below the lists'
extent (all reads still inside the list buffer) is reported as a list read past the count."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

from gpu_helpers import say

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

HERE = os.path.dirname(os.path.abspath(__file__))
WORKER = os.path.join(HERE, "gpu_bounds_worker.py")


def _run(tmp_path, which):
    out = tmp_path / f"{which}.npz"
    env = dict(os.environ, MGS_LIBRARY=which)
    r = subprocess.run([sys.executable, "-u", WORKER, str(out)], capture_output=True, text=True, env=env,
                       timeout=500)
    say(f"  {which}: {r.stdout.strip().splitlines()[-1] if r.stdout.strip() else r.stderr[-500:]}")
    assert r.returncode == 0, r.stderr[-2000:]
    return r.stdout, np.load(out)


def test_checked_build_reports_no_out_of_bounds_index(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("test_checked_build_reports_no_out_of_bounds_index")
    out_c, imgs_c = _run(tmp_path, "checked")
    assert "checked=1 flags=0x0 " in out_c
    assert "planted=0x8" in out_c            # MGS_BOUNDS_LIST_READ, and nothing else
    out_n, imgs_n = _run(tmp_path, "normal")
    assert "checked=0 " in out_n
    assert sorted(imgs_c.files) == sorted(imgs_n.files)
    for k in imgs_c.files:
        assert np.array_equal(imgs_c[k], imgs_n[k]), k
