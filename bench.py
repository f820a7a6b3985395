"""Throughput of the matrix-free map y = H x on one MI355X.

Workload: the periodic mixed-spin ferrimagnetic ring, 20 sites alternating s = 1/2 and s = 1
(D = 2^10 * 3^10 = 60,466,176), XXZ bonds J_xy = 1.0, J_z = 1.2, single-ion anisotropy 0.5 (S_z)^2 on
the s = 1 sites, field 0.1 S_z; complex128 state drawn from seed 2, already resident in HBM.  A step is
one plain FP64 (complex128) H x.

Prints one JSON line: matvecs/s, the roofline of the matvec kernel (algorithmic bytes 2 * D * 16 per
launch over the mean launch time, measured with HIP events on the launch stream, against 8 TB/s), the
HBM traffic read from committed rocprofv3 counters when they were taken on the same kernel, and the
CPU oracle timed on a bounded sample of rows on the host cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--profile]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "H·x matvecs/s + effective HBM GB/s; FP32/batched vs plain FP64 at stated err"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_ferrimagnetic_ring_N20_c128.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_fingerprint(plan, dtype) -> str:
    """Hash of the kernel source the plan launches (counters are valid only for the same kernel)."""
    info = plan.kernel_info(dtype)
    if info["kind"] == "specialized":
        src = plan.kernel_source(dtype)
    else:
        src = "generic"
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def cpu_baseline(model, x_host, target_s: float = 12.0):
    """The oracle's FP64 matvec on a contiguous sample of rows, on the host cores; scaled to
    matvecs/s of the full vector."""
    import numpy as np
    from oracle import mf
    D = model.dim
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    # calibrate on a short sample, then run about target_s seconds of rows
    rows = np.arange(D // 3, D // 3 + 200_000, dtype=np.int64)
    t0 = time.perf_counter()
    mf.matvec(model, x_host, rows=rows)
    dt = time.perf_counter() - t0
    n = int(min(D, max(200_000, 200_000 * target_s / max(dt, 1e-6))))
    start = (D - n) // 2
    rows = np.arange(start, start + n, dtype=np.int64)
    t0 = time.perf_counter()
    y_rows = mf.matvec(model, x_host, rows=rows)
    dt = time.perf_counter() - t0
    rows_per_s = n / dt
    return dict(value=rows_per_s / D, unit="matvecs/s", cores=threads, kind="oracle",
                sample=f"rows [{start}, {start + n}) of D={D} ({n} rows, {dt:.1f} s), plain C "
                       f"App-A row loop, FP64, OpenMP over rows"), rows, y_rows


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", action="store_true", help="short run for a profiler: no CPU leg")
    ap.add_argument("--kernel", default="auto", choices=["auto", "generic", "specialized"])
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the matvec is measured on one GPU's share; "
              "a multi-GPU run is not part of this build (--gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2606_02169_amd.plan import Plan

    if not torch.cuda.is_available():
        print("bench.py needs a GPU (the HIP library has no CPU path)", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    t0 = time.perf_counter()
    model, x_host = W.config(2)
    log(f"inputs: {model.name} D={model.dim} generated in {time.perf_counter() - t0:.1f} s")
    D = model.dim
    plan = Plan.from_model(model, device=dev)
    plan.set_kernel(args.kernel)
    plan.prepare(torch.complex128)
    info = plan.kernel_info(torch.complex128)
    log(f"kernel: {info}")
    x = torch.from_numpy(x_host).to(dev)
    y = torch.empty_like(x)
    theta = torch.as_tensor(model.theta, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)

    if args.profile:
        # a plain copy of known size (x -> y, 2 * D * 16 bytes of HBM traffic) in the same process, so
        # profiler counters of the matvec can be scaled by what they read for a pure stream
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        plan.matvec(theta, x, out=y)
    torch.cuda.synchronize()

    K = args.steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for i in range(K):
        ev[i][0].record(stream)
        plan.matvec(theta, x, out=y)
        ev[i][1].record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    launch_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = total_ms / K
    mean_launch_ms = float(np.mean(launch_ms))
    alg_bytes = 2 * D * 16
    achieved = alg_bytes / (mean_launch_ms * 1e-3) / 1e9
    log(f"timed {K} steps: {ms_per_step:.4f} ms/step, launch mean {mean_launch_ms:.4f} ms "
        f"(min {min(launch_ms):.4f}, max {max(launch_ms):.4f})")

    traffic = None
    fp = kernel_fingerprint(plan, torch.complex128)
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        if rec.get("kernel_fingerprint") == fp:
            traffic = rec.get("hbm_bytes_per_launch")

    out = {
        "metric": METRIC,
        "value": 1000.0 / ms_per_step,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "ferrimagnetic_ring_N20_c128", "sites": "20 (s=1/2, s=1 alternating), periodic",
                   "D": D, "couplings": "Jxy=1.0 Jz=1.2 D_si=0.5 hz=0.1", "seed": 2,
                   "kernel": info["kind"]},
        "effective_GBps": achieved,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": alg_bytes, "mean_launch_ms": mean_launch_ms,
                     "kernel_fingerprint": fp},
    }

    if not (args.no_cpu_baseline or args.profile):
        # oracle timing and a sampled parity check of the timed output (the oracle is a baseline only)
        cb, rows, y_rows = cpu_baseline(model, x_host)
        y_gpu = y[torch.from_numpy(rows).to(dev)].cpu().numpy()
        err = float(np.linalg.norm(y_gpu - y_rows) / np.linalg.norm(y_rows))
        out["cpu_baseline"] = cb
        out["sampled_rel_err_vs_oracle"] = err
        log(f"cpu baseline: {cb}; sampled rel err {err:.3e}")
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
