"""Host side of the benchmark script: its one-GPU contract and the CPU baselines it reports beside the GPU
figures (the oracle timed on the host cores), on tiny models so that no GPU is needed."""
import os
import subprocess
import sys

import numpy as np

import bench
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_refused_before_any_gpu_work():
    for extra, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + extra, cwd=ROOT,
                           capture_output=True, text=True, timeout=120, env={**os.environ, **env})
        assert r.returncode == 2
        assert "one GPU only" in r.stderr
        assert r.stdout == ""


def test_host_cpu_info_fields():
    info = bench.host_cpu_info()
    assert set(info) == {"cpu_model", "logical_cpus", "physical_cores"}
    assert info["logical_cpus"] >= 1
    assert info["physical_cores"] is None or 1 <= info["physical_cores"] <= info["logical_cpus"]


def test_cpu_baseline_object():
    """The matvec baseline: the keys of the bench line's cpu_baseline object, a positive rate, and the
    sampled rows' values equal to the oracle's full matvec on those rows."""
    from oracle import mf
    m, x = W.config(2, reduced=8)                       # D = 216
    cb, rows, y_rows = bench.cpu_baseline(m, x, rep_s=0.05, one_core_rep_s=0.05)
    for k in ("value", "unit", "cores", "kind", "sample", "one_core", "timing"):
        assert k in cb
    assert cb["kind"] == "oracle" and cb["unit"] == "matvecs/s"
    assert cb["value"] > 0 and cb["one_core"]["value"] > 0 and cb["cores"] >= 1
    assert np.array_equal(y_rows, mf.matvec(m, x)[rows])


def test_cpu_lanczos_baseline_object():
    """The Lanczos baseline: seconds per step of the oracle's FP64 Lanczos, and the alpha comparison
    against a run given to it (here the oracle's own recurrence, so the difference is zero)."""
    from oracle import lanczos as olz
    from oracle import mf
    m, x = W.config(2, reduced=8)
    ref = olz.lanczos(lambda v: mf.matvec(m, v), x, 3)
    cb = bench.cpu_lanczos_baseline(m, x, gpu_alpha=ref["alpha"], steps=3)
    assert cb["kind"] == "oracle" and cb["unit"] == "s per Lanczos step" and cb["value"] > 0
    assert cb["max_abs_alpha_diff_vs_gpu"] == 0.0
