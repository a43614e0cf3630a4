"""The benchmark's contract that needs no GPU: more than one GPU (by flag or by the
launcher's WORLD_SIZE) is refused with a JSON message before anything else runs; and the
host-side helpers of its roofline."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, capture_output=True, text=True,
                       timeout=120, env=e, cwd=ROOT)
    assert r.returncode == 2, (r.returncode, r.stderr[-500:])
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_width_mix_of_the_gather_ceiling():
    sys.path.insert(0, ROOT)
    import bench
    # 15 kept products of 64 columns and one refresh of all 96: mean 66
    mix = bench.width_mix(66.0, 96, 32)
    assert set(mix) == {64, 96}
    assert abs(mix[64] - 15 / 16) < 1e-12 and abs(mix[96] - 1 / 16) < 1e-12
    assert bench.width_mix(64.0, 96, 32) == {64: 1.0}
    assert bench.width_mix(96.0, 96, 32) == {96: 1.0}
    assert bench.width_mix(194.0, 194, 65) == {194: 1.0}  # no kept product (the Laplacian)
