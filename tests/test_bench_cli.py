"""bench.py's one-GPU contract, checked on the host: a request for more than
one GPU (by flag or by a launcher's WORLD_SIZE) ends before anything touches
a device, with a message that says why."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("argv, env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}),
                                       ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ)
    e.update(env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], capture_output=True, text=True,
                       env=e, cwd=ROOT, timeout=120)
    assert r.returncode == 1
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
