"""bench.py on the host: more than one GPU is refused with a JSON
explanation before anything touches a device; the autotuner's probe size
and the lookup of the committed counter profiles."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_tune_probe_covers_one_wave():
    # the probe asks for every q-sample up to the limit (the library keeps
    # one q-wave of them) and sizes its steps to ~6e9 field-site updates of
    # at most one wave, 3 to 40 steps
    sys.path.insert(0, ROOT)
    import bench
    import workloads as w
    def geom(n):
        return w.Geometry(comp=np.zeros((n, n, n), np.uint32),
                          comp_phase=np.zeros(1, np.uint8), n_phase=1, dx=1.0)
    big = {"gG0": [[0.0, 0.0, 1.0]] * 256, "q_geom": [0] * 256, "bc": [0, 0, 0],
           "geoms": [geom(256)]}
    Qt, K = bench.tune_probe(big, bench.TUNE_Q)
    assert Qt == 256 and K == 3
    small = dict(big, gG0=big["gG0"][:2], q_geom=[0, 0], geoms=[geom(8)])
    assert bench.tune_probe(small, bench.TUNE_Q) == (2, 40)


def test_traffic_profile_matches_source_and_launch():
    # the committed counter profile of the benchmark's step kernel is read
    # for the launches it was taken in, and only for the current source
    sys.path.insert(0, ROOT)
    import bench
    sha = bench.source_hash(bench.KERNEL_SRC)
    with open(bench.TRAFFIC_FILES[("cfg3a", "k_step")]) as fh:
        t = json.load(fh)
    launches = [t["launch"]] + [o["launch"] for o in t.get("other_launches", [])]
    for L in launches:
        v = bench.traffic_for(("cfg3a", "k_step"), sha, L)
        assert v is not None and 1.0 <= v / t["algorithmic_bytes_per_step"] < 1.3
    assert bench.traffic_for(("cfg3a", "k_step"), "0" * 16, launches[0]) is None
    assert bench.traffic_for(("cfg3a", "k_step"), sha, {"tile": 9, "zc": 9, "xcd": 9}) is None
