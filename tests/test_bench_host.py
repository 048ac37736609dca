"""Host-side checks of bench.py that need no GPU: the one-GPU contract, the
workload's shape and the roofline's algorithmic bytes per flip."""
import importlib.util
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_main_workload_shape():
    b = load_bench()
    W, T, Bn = b.workload()
    assert W.shape == (800, 800) and W.dtype == np.int16
    assert np.array_equal(W, W.T)
    assert (T, Bn) == (80, 8000)
    # max-cut map: W_ii = -deg_w(i), so every row of W sums to zero
    assert np.all(W.astype(np.int64).sum(axis=1) == 0)
    # one flip reads one row of W: n sizeof(W) algorithmic bytes
    assert W.shape[0] * W.dtype.itemsize == 1600


def test_profile_summaries_name_their_commands():
    prof = os.path.join(ROOT, "profiles")
    for f in sorted(os.listdir(prof)):
        text = open(os.path.join(prof, f)).read()
        assert "rocprofv3" in text, f
        assert "bench.py" in text, f
