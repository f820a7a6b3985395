"""Throughput of the matrix-free map y = H x on one MI355X.

Default workload (the headline line): the periodic mixed-spin ferrimagnetic ring, 20 sites alternating
s = 1/2 and s = 1 (D = 2^10 * 3^10 = 60,466,176), XXZ bonds J_xy = 1.0, J_z = 1.2, single-ion anisotropy
0.5 (S_z)^2 on the s = 1 sites, field 0.1 S_z; complex128 state drawn from seed 2, resident in HBM.  A
step is one plain FP64 (complex128) H x.  Prints one JSON line: matvecs/s, the roofline of the matvec
kernel (algorithmic bytes 2 * D * 16 per launch over the mean launch time, measured with HIP events on
the launch stream, against 8 TB/s), the HBM traffic from committed rocprofv3 counters when they were
taken on the same kernel, and the CPU oracle timed on the host cores.

Other workloads (one JSON line each; not part of the headline):
  --workload torus      4x4 periodic spin-1 Heisenberg (D = 3^16): the matvec alone, c64 and c128
  --workload lanczos4x4  4x4 periodic spin-1 Heisenberg (D = 3^16): FP32 (c64) matvec inside the FP64
                         Lanczos against the plain FP64 form: steps and wall time to 1e-5 relative
                         ground-energy error, end to end and matvec only
  --workload lanczos_ring20  100 Lanczos steps on the headline ring (basis 97.7 GB), plain FP64 and
                         FP32-in-FP64, each reorthogonalisation, beside the sector Lanczos energies of
                         every digit sum
  --workload batched     256 open mixed chains x 8 c64 vectors in one persistent hipGraph launch,
                         against separate plain c64 and c128 calls per vector
  --workload adjoint     Tavis-Cummings (12 spins + boson cut at 64): forward and adjoint times and
                         gradient error against the oracle
  --workload paper       the paper's chain testbeds (spin-1 ring N=15, mixed ring (1/2)^6(1)^6(3/2)^6):
                         matvecs/s and a Lanczos ground state, beside the paper's CPU figures
  --workload propagate   Chebyshev time propagation on the ring: terms per step, time per term
  --workload sector      S_z = 0 sectors of the ring and of C1: sector matvec and sector Lanczos
  --workload stream      stream ceilings of the GPU (standalone probe): reads by footprint and cache
                         policy, copies, window gathers
  --workload chain12     12-site spin-1/2 Heisenberg chain (D = 4096): H x and a 50-step Lanczos, eager
                         and replayed from a HIP graph
  --workload sweep       parameter sweep: the 14-site ring at 256 coupling vectors x 8 c64 vectors in one
                         batched launch, against separate plain calls

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--profile] [--workload W]
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
    src = plan.kernel_source(dtype) if info["kind"] == "specialized" else "generic"
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def cuda_time(fn, stream, reps: int):
    """Mean ms per call over reps back-to-back calls, HIP events on the launch stream."""
    import torch
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def host_cpu_info() -> dict:
    """CPU model, logical CPUs this process may run on, and the physical cores among them (/proc/cpuinfo)."""
    avail = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else list(range(os.cpu_count()))
    model_name, cores = None, set()
    try:
        with open("/proc/cpuinfo") as f:
            blocks = f.read().strip().split("\n\n")
        for b in blocks:
            kv = {}
            for line in b.splitlines():
                if ":" in line:
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
            if int(kv.get("processor", -1)) in avail:
                model_name = model_name or kv.get("model name")
                cores.add((kv.get("physical id", "0"), kv.get("core id", kv.get("processor"))))
    except OSError:
        pass
    return {"cpu_model": model_name, "logical_cpus": len(avail), "physical_cores": len(cores) or None}


def cpu_baseline(model, x_host, rep_s: float = 3.0, one_core_rep_s: float = 2.0):
    """The oracle's FP64 matvec on the host cores, on a bounded sample of the same workload: a contiguous
    block of rows in the middle of the vector sized for about rep_s seconds, timed three times after a
    warm-up (median), on all the threads the oracle uses and again on one thread; scaled to matvecs/s of
    the full vector (rows per second / D).  About 6 rep_s + 6 one_core_rep_s seconds of CPU work."""
    import numpy as np
    from oracle import mf
    D = model.dim

    def block(n):
        n = int(max(1000, min(D, n)))
        start = (D - n) // 2
        return np.arange(start, start + n, dtype=np.int64)

    def median_rate(rows, reps=3):
        mf.matvec(model, x_host, rows=rows)                 # warm-up (thread pool, tables, caches)
        ts = []
        y = None
        for _ in range(reps):
            t0 = time.perf_counter()
            y = mf.matvec(model, x_host, rows=rows)
            ts.append(time.perf_counter() - t0)
        return rows.size / float(np.median(ts)), ts, y

    threads = mf.threads()
    probe = block(200_000)
    r0, _, _ = median_rate(probe, reps=1)
    rows = block(r0 * rep_s)
    rate, ts, y_rows = median_rate(rows)
    mf.threads(1)
    try:
        r1, _, _ = median_rate(block(20_000), reps=1)
        rows1 = block(r1 * one_core_rep_s)
        rate1, ts1, _ = median_rate(rows1)
    finally:
        mf.threads(threads)
    info = host_cpu_info()
    cb = dict(value=rate / D, unit="matvecs/s", cores=threads, kind="oracle",
              sample=f"rows [{rows[0]}, {rows[-1] + 1}) of D={D} ({rows.size} rows), median of 3 timings "
                     f"{', '.join(f'{t:.2f}' for t in ts)} s after a warm-up, scaled to the full vector; "
                     f"oracle row-by-row Kronecker evaluation in C, OpenMP over rows",
              threads=threads, one_core={"value": rate1 / D, "unit": "matvecs/s",
                                         "sample": f"{rows1.size} rows, median of 3 timings "
                                                   f"{', '.join(f'{t:.2f}' for t in ts1)} s"},
              timing="median of 3 after a warm-up", **info)
    return cb, rows, y_rows


def cpu_lanczos_baseline(model, x_host, gpu_alpha=None, steps: int = 3):
    """The oracle's FP64 Lanczos with full CGS2 on the host cores (its matvec on all the oracle's threads,
    the Gram-Schmidt passes in numpy), on a bounded sample of the same run: the first `steps` steps from
    the same start vector, after a one-step warm-up, as seconds per step.  The first steps have the
    shortest Gram-Schmidt passes, so the figure is a lower bound on the oracle's time per step of a longer
    run.  With the GPU's alpha_j of the same run, the largest difference over those steps is reported."""
    import numpy as np
    from oracle import lanczos as olz
    from oracle import mf

    def op(v):
        return mf.matvec(model, v)

    olz.lanczos(op, x_host, 1, explicit_residual=False)
    t0 = time.perf_counter()
    r = olz.lanczos(op, x_host, steps, explicit_residual=False)
    dt = time.perf_counter() - t0
    out = {"value": dt / steps, "unit": "s per Lanczos step", "kind": "oracle", "cores": mf.threads(),
           "sample": f"the first {steps} steps of the same run (full CGS2), after a one-step warm-up; "
                     f"{dt:.2f} s in all", **host_cpu_info()}
    if gpu_alpha is not None:
        k = min(steps, len(gpu_alpha))
        out["max_abs_alpha_diff_vs_gpu"] = float(np.max(np.abs(np.asarray(gpu_alpha[:k]) - r["alpha"][:k])))
    return out


def oracle_residual(model, u, theta):
    """Oracle leg beside the CPU baseline: ||H u - theta u|| of a GPU Ritz vector u (host copy) with the
    oracle's H, and ||u||.  For Hermitian H an eigenvalue lies within ||H u - theta u|| / ||u|| of theta,
    so this certifies a GPU energy independently of the GPU's own residual."""
    import numpy as np
    from oracle import mf
    hu = mf.matvec(model, u)
    return float(np.linalg.norm(hu - theta * u)), float(np.linalg.norm(u))


# ------------------------------------------------------------------------------------------ headline
def bench_ring(args, dev):
    import numpy as np
    import torch

    import workloads as W
    from paper_2606_02169_amd.plan import Plan

    t0 = time.perf_counter()
    model, x_host = W.config(2)
    log(f"inputs: {model.name} D={model.dim} generated in {time.perf_counter() - t0:.1f} s")
    D = model.dim
    plan = Plan.from_model(model, device=dev)
    x = torch.from_numpy(x_host).to(dev)
    y = torch.empty_like(x)
    theta = torch.as_tensor(model.theta, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    if args.kernel == "auto":
        tuned = plan.autotune(theta, x, y)
        log(f"tuned shape: {tuned}")
    else:
        plan.set_kernel(args.kernel)
        plan.prepare(torch.complex128)
    info = plan.kernel_info(torch.complex128)
    log(f"kernel: {info}")

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

    # the stream ceiling of this GPU for the same bytes: a plain device copy of x into a second buffer
    # (read D x 16 B, write D x 16 B), timed the same way after the matvec loop; y keeps H x for the
    # parity check below
    if not args.profile:
        z = torch.empty_like(x)
        for _ in range(2):
            z.copy_(x)
        copy_ms = cuda_time(lambda: z.copy_(x), stream, 10)
        copy_GBps = alg_bytes / (copy_ms * 1e-3) / 1e9
        del z
    else:
        copy_GBps = None

    # HBM traffic is not measured in this run: it is the committed rocprofv3 counter figure (FETCH_SIZE +
    # WRITE_SIZE, scaled by a plain copy) for this exact kernel source, else null
    traffic, traffic_source = None, None
    fp = kernel_fingerprint(plan, torch.complex128)
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        if rec.get("kernel_fingerprint") == fp:
            traffic = rec.get("hbm_bytes_per_launch")
            traffic_source = (f"committed rocprofv3 counters, profiles/{os.path.basename(TRAFFIC_FILE)}, "
                              f"kernel fingerprint {fp}")

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
                   "kernel": {k: info[k] for k in ("kind", "inner_sites", "unrolled_sites", "copies", "block", "grid")}},
        "effective_GBps": achieved,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "traffic_source": traffic_source,
                     "algorithmic_bytes_per_launch": alg_bytes, "mean_launch_ms": mean_launch_ms,
                     "median_launch_ms": float(np.median(launch_ms)),
                     "kernel_fingerprint": fp, "copy_GBps": copy_GBps,
                     "frac_of_copy": achieved / copy_GBps if copy_GBps else None},
    }
    if not (args.no_cpu_baseline or args.profile):
        # oracle timing and a parity check of the timed output (the oracle is a baseline only)
        cb, rows, y_rows = cpu_baseline(model, x_host)
        y_gpu = y[torch.from_numpy(rows).to(dev)].cpu().numpy()
        err = float(np.linalg.norm(y_gpu - y_rows) / np.linalg.norm(y_rows))
        out["cpu_baseline"] = cb
        out["rel_err_vs_oracle"] = err
        out["rel_err_vs_oracle_rows"] = int(rows.size)
        log(f"cpu baseline: {cb}; rel err vs oracle {err:.3e}")
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------------------------------ torus
def bench_torus(args, dev):
    """The 4x4 periodic spin-1 Heisenberg lattice (D = 3^16, 32 bonds with J_b ~ U[0.5, 1.5], seed 3):
    the matvec alone in its FP32 (c64) form and in the plain FP64 (c128) form, each with its autotuned
    shape; algorithmic bytes 2 * D * b per launch (b = 8 or 16).  --dtype picks one form (profiler runs),
    else both are timed."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2606_02169_amd.plan import Plan

    model, x32 = W.config(3)
    D = model.dim
    stream = torch.cuda.current_stream(dev)
    forms = {"c64": (torch.complex64, torch.float32, 8), "c128": (torch.complex128, torch.float64, 16)}
    names = [args.dtype] if args.dtype else ["c64", "c128"]
    out = {"metric": "H·x on the 4x4 periodic spin-1 lattice (D = 3^16): matvecs/s and effective HBM GB/s",
           "workload": "square4x4_spin1_periodic", "D": D, "seed": 3, "forms": {}}
    for name in names:
        cdt, rdt, b = forms[name]
        plan = Plan.from_model(model, device=dev)
        x = torch.from_numpy(x32).to(dev).to(cdt)
        y = torch.empty_like(x)
        th = torch.as_tensor(model.theta, dtype=rdt, device=dev)
        tuned = plan.autotune(th, x, y)
        info = plan.kernel_info(cdt)
        if args.profile:   # plain copy of known size in the same process: scale for the traffic counters
            for _ in range(3):
                y.copy_(x)
            torch.cuda.synchronize()
        for _ in range(args.warmup):
            plan.matvec(th, x, out=y)
        ms = cuda_time(lambda: plan.matvec(th, x, out=y), stream, args.steps)
        alg = 2 * D * b
        res = {"ms_per_matvec": ms, "matvecs_per_s": 1000.0 / ms, "effective_GBps": alg / ms / 1e6,
               "frac_of_peak": alg / ms / 1e6 / PEAK_HBM_GBS, "algorithmic_bytes_per_launch": alg,
               "kernel_fingerprint": kernel_fingerprint(plan, cdt),
               "shape": {k: tuned.get(k) for k in ("variant", "inner_sites", "unrolled_sites", "load_group",
                                                    "unroll_top")},
               "kernel": {k: info[k] for k in ("inner_sites", "unrolled_sites", "copies", "block", "grid",
                                               "super_tiles")}}
        if not args.profile:
            from oracle import mf
            rng = np.random.default_rng(33)
            rows = np.unique(rng.choice(D, 4000, replace=False)).astype(np.int64)
            xin = x.cpu().numpy().astype(np.complex128)
            ref = mf.matvec(model, xin, rows=rows)
            got = y[torch.from_numpy(rows).to(dev)].cpu().numpy()
            res["sampled_rel_err_vs_oracle"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        out["forms"][name] = res
        log(f"{name}: {res}")
        del x, y, plan
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------------------------------ Lanczos
def bench_lanczos(args, dev):
    import numpy as np
    import torch
    from scipy.linalg import eigvalsh_tridiagonal

    import workloads as W
    from paper_2606_02169_amd.plan import Plan

    model, x32 = W.config(3)
    D = model.dim
    v0 = torch.from_numpy(x32.astype(np.complex128)).to(dev)
    th64 = torch.as_tensor(model.theta, dtype=torch.float64, device=dev)
    th32 = th64.float()
    stream = torch.cuda.current_stream(dev)
    pz = Plan.from_model(model, device=dev)
    pc = Plan.from_model(model, device=dev)
    xz = v0.clone()
    yz = torch.empty_like(xz)
    xc = torch.from_numpy(x32).to(dev)
    yc = torch.empty_like(xc)
    log(f"tuned c128: {pz.autotune(th64, xz, yz)}")
    log(f"tuned c64: {pc.autotune(th32, xc, yc)}")
    for _ in range(3):
        pz.matvec(th64, xz, out=yz)
        pc.matvec(th32, xc, out=yc)
    mv_z = cuda_time(lambda: pz.matvec(th64, xz, out=yz), stream, 20)
    mv_c = cuda_time(lambda: pc.matvec(th32, xc, out=yc), stream, 20)
    del xz, yz, xc, yc

    def ritz_curve(alpha, beta, k):
        a = alpha[:k]
        b = beta[: k - 1]
        return np.array([eigvalsh_tridiagonal(a[:i], b[: i - 1], select="i", select_range=(0, 0))[0]
                         for i in range(1, k + 1)])

    def run(plan, prec, m, reorth="cgs2", certify=False):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = plan.lanczos(th64, v0, m, precision=prec, reorth=reorth, theta_c=th32)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res = r["result"].cpu().numpy()
        k = int(res[3])
        out = dict(theta=float(res[0]), resid=float(res[2]), steps=k, seconds=dt,
                   alpha=r["alpha"].cpu().numpy()[:k], beta=r["beta"].cpu().numpy()[:k],
                   passes=[int(c) for c in r["counts"].cpu().numpy()])
        if certify and not args.profile:
            u = r["u"].cpu().numpy()
            del r
            out["oracle_residual"], out["u_norm"] = oracle_residual(model, u, out["theta"])
        return out

    m_ref = args.lanczos_ref_steps
    ref = run(pz, "z", m_ref, reorth=args.lanczos_ref_reorth, certify=True)
    E_ref = ref["theta"]
    log(f"reference: {m_ref} FP64 steps, theta {E_ref!r} residual {ref['resid']:.3e} "
        f"(oracle {ref.get('oracle_residual', float('nan')):.3e}) in {ref['seconds']:.1f} s")
    cpu_lz = None
    if not (args.no_cpu_baseline or args.profile):
        cpu_lz = cpu_lanczos_baseline(model, x32.astype(np.complex128), ref["alpha"])
        log(f"oracle Lanczos on the host: {cpu_lz}")
    out = {"metric": "Lanczos ground energy: FP32 (c64) matvec in FP64 Lanczos vs plain FP64, time to 1e-5",
           "workload": "square4x4_spin1_periodic", "D": D, "seed": 3,
           "reference": {"steps": ref["steps"], "theta": E_ref, "residual": ref["resid"],
                         "oracle_residual": ref.get("oracle_residual"),
                         "certified_within": (ref["oracle_residual"] / ref["u_norm"]) if "u_norm" in ref else None,
                         "reorth": args.lanczos_ref_reorth, "seconds": ref["seconds"]},
           "matvec_ms": {"c128": mv_z, "c64": mv_c}, "forms": {}}
    if cpu_lz is not None:
        out["cpu_baseline"] = cpu_lz
    m = args.lanczos_steps
    forms = args.lanczos_forms.split(",")
    for name, plan, prec, ro in (("fp64", pz, "z", "cgs2"), ("fp32_in_fp64", pc, "c_in_z", "cgs2"),
                                 ("fp64_cgs2_cond", pz, "z", "cgs2_cond"),
                                 ("fp32_in_fp64_cgs2_cond", pc, "c_in_z", "cgs2_cond"),
                                 ("fp64_partial", pz, "z", "partial"),
                                 ("fp32_in_fp64_partial", pc, "c_in_z", "partial")):
        if ro not in forms:
            continue
        full = run(plan, prec, m, ro, certify=True)
        curve = ritz_curve(full["alpha"], full["beta"], full["steps"])
        rel = np.abs(curve - E_ref) / abs(E_ref)
        hit = np.nonzero(rel <= 1e-5)[0]
        k5 = int(hit[0]) + 1 if hit.size else None
        timed = run(plan, prec, k5, ro) if k5 else None
        out["forms"][name] = {
            "reorth": ro, "steps": m, "theta": full["theta"], "rel_err": abs(full["theta"] - E_ref) / abs(E_ref),
            "residual": full["resid"], "oracle_residual": full.get("oracle_residual"), "seconds": full["seconds"],
            "steps_to_1e-5": k5, "seconds_to_1e-5": timed["seconds"] if timed else None,
            "rel_err_at_1e-5_run": (abs(timed["theta"] - E_ref) / abs(E_ref)) if timed else None,
            "matvec_ms": mv_z if prec == "z" else mv_c,
            # second passes taken (cgs2_cond) or passes taken (partial); cgs2 takes two at every step
            "gram_schmidt_passes": (full["passes"][0] if ro == "cgs2_cond" else
                                    full["passes"][1] if ro == "partial" else None)}
        log(f"{name}: {out['forms'][name]}")
    nz = run(pz, "z", m, reorth="none")
    nc = run(pc, "c_in_z", m, reorth="none")
    out["no_reorth"] = {"fp64": {"seconds": nz["seconds"], "rel_err": abs(nz["theta"] - E_ref) / abs(E_ref)},
                        "fp32_in_fp64": {"seconds": nc["seconds"],
                                         "rel_err": abs(nc["theta"] - E_ref) / abs(E_ref)}}
    print(json.dumps(out), flush=True)


def bench_lanczos_ring(args, dev):
    """100 Lanczos steps on the 20-site ferrimagnetic ring from the seeded start vector, plain FP64 and FP32
    matvec inside FP64, with each reorthogonalisation (full CGS2, conditional second pass, partial); the
    full-basis ground energy beside the lowest sector energy (H keeps the digit sum, so its lowest
    eigenvalue is the lowest over all sectors; sector Lanczos in every sector)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2606_02169_amd.plan import Plan, Sector

    model, x = W.config(2)
    D = model.dim
    v0 = torch.from_numpy(x).to(dev)
    cpu_lz = None
    if not (args.no_cpu_baseline or args.profile):
        cpu_lz = cpu_lanczos_baseline(model, x)
        log(f"oracle Lanczos on the host: {cpu_lz}")
    del x
    th64 = torch.as_tensor(model.theta, dtype=torch.float64, device=dev)
    th32 = th64.float()
    m = args.lanczos_steps
    out = {"metric": "Lanczos on the 20-site ferrimagnetic ring (c128 basis): time per step and ground energy",
           "workload": "ferrimagnetic_ring_N20_c128", "D": D, "seed": 2, "steps": m,
           "basis_GB": (m + 1) * D * 16 / 1e9, "forms": {}}
    if cpu_lz is not None:
        out["cpu_baseline"] = cpu_lz
    forms = args.lanczos_forms.split(",")
    for name, prec, ro in (("fp64", "z", "cgs2"), ("fp32_in_fp64", "c_in_z", "cgs2"),
                           ("fp64_cgs2_cond", "z", "cgs2_cond"), ("fp32_in_fp64_cgs2_cond", "c_in_z", "cgs2_cond"),
                           ("fp64_partial", "z", "partial"), ("fp32_in_fp64_partial", "c_in_z", "partial")):
        if ro not in forms:
            continue
        plan = Plan.from_model(model, device=dev)
        y = torch.empty_like(v0)
        plan.autotune(th64, v0, y)
        if prec == "c_in_z":
            xc = v0.to(torch.complex64)
            plan.autotune(th32, xc, torch.empty_like(xc))
            del xc
        del y
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = plan.lanczos(th64, v0, m, precision=prec, reorth=ro, theta_c=th32)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res = r["result"].cpu().numpy()
        passes = [int(c) for c in r["counts"].cpu().numpy()]
        u = r["u"].cpu().numpy() if (ro in ("cgs2", "partial") and not args.profile) else None
        del r   # the basis stays in torch's cache for the next form: no new 98 GB allocation inside a timing
        out["forms"][name] = {"reorth": ro, "seconds": dt, "ms_per_step": dt / max(1, int(res[3])) * 1e3, "E0": float(res[0]),
                              "residual": float(res[2]), "steps": int(res[3])}
        if ro == "cgs2_cond":
            out["forms"][name]["second_passes"] = passes[0]
        elif ro == "partial":
            out["forms"][name]["gram_schmidt_passes"] = passes[1]
        if u is not None:
            ro_res, nu = oracle_residual(model, u, float(res[0]))
            del u
            out["forms"][name]["oracle_residual"] = ro_res
            out["forms"][name]["certified_within"] = ro_res / nu
        log(f"{name}: {out['forms'][name]}")
    torch.cuda.empty_cache()
    if not args.profile and out["forms"]:
        plan = Plan.from_model(model, device=dev)
        sectors = {}
        for Q in range(sum(s.d - 1 for s in model.sites) + 1):
            S = Sector(plan, Q)
            rng = np.random.default_rng(100 + Q)
            xs = torch.from_numpy(W.random_state(S.dim, rng)).to(dev)
            r = S.lanczos(th64, xs, m)
            res = r["result"].cpu().numpy()
            sectors[Q] = {"dim": S.dim, "E0": float(res[0]), "residual": float(res[2])}
            del r, xs, S
            torch.cuda.empty_cache()
        qmin = min(sectors, key=lambda q: sectors[q]["E0"])
        out["sectors"] = sectors
        full = next(f for k, f in out["forms"].items() if k.startswith("fp64"))
        out["lowest_sector"] = {"digit_sum": qmin, "E0": sectors[qmin]["E0"],
                                "full_minus_sector": full["E0"] - sectors[qmin]["E0"]}
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------------------------------ batched
def bench_batched(args, dev):
    import numpy as np
    import torch

    import workloads as W
    from oracle import mf
    from paper_2606_02169_amd.plan import Batch, Plan

    t0 = time.perf_counter()
    models, xs = W.config(4)
    log(f"inputs: {len(models)} lattices, sum D {sum(m.dim for m in models)} in {time.perf_counter() - t0:.1f} s")
    plans = [Plan.from_model(m, device=dev) for m in models]
    B = Batch(plans, 8)
    X = torch.zeros(B.total_elems, dtype=torch.complex64, device=dev)
    for b, x in enumerate(xs):
        B.block(X, b).copy_(torch.from_numpy(np.ascontiguousarray(x)).to(dev))
    Y = torch.empty_like(X)
    th = torch.from_numpy(np.concatenate([m.theta for m in models]).astype(np.float32)).to(dev)
    if args.profile:
        # a short run for profiler counters: the tiles and block the autotuner selects for this workload on
        # MI355X, with the window schedule it selects or another one (--batch-schedule); warm-up and timed
        # graph replays only
        B.set_shape(512, 512, args.batch_schedule)
        shape = B.shape()
    else:
        shape = B.autotune(th, X, Y)
    s = torch.cuda.Stream(device=dev)
    B.capture(th, X, Y, s)
    for _ in range(3):
        B.replay(s)
    s.synchronize()
    K = max(3, args.steps // 5)
    a = torch.cuda.Event(enable_timing=True)
    b_ = torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(K):
        B.replay(s)
    b_.record(s)
    s.synchronize()
    ms_graph = a.elapsed_time(b_) / K
    sumD = sum(m.dim for m in models)
    vec_mv = len(models) * 8
    # errors on sampled rows of every 8th lattice, against the oracle in FP64
    rng = np.random.default_rng(5)
    errs = []
    for bi in range(0, len(models), 8):
        m, x = models[bi], xs[bi]
        r = np.unique(rng.choice(m.dim, min(m.dim, 500), replace=False)).astype(np.int64)
        yb = B.block(Y, bi).cpu().numpy()
        for v in (0, 7):
            ref = mf.matvec(m, x[:, v].astype(np.complex128), rows=r)
            errs.append(float(np.linalg.norm(yb[r, v] - ref) / np.linalg.norm(ref)))
    out = {"metric": "batched vector-matvecs/s (256 lattices x 8 c64 vectors, one persistent hipGraph launch)",
           "workload": "mixed_chains_256x8_c64", "seed": 4, "sum_D": sumD, "vector_matvecs_per_launch": vec_mv,
           "shape": shape, "ms_per_launch": ms_graph, "vector_matvecs_per_s": vec_mv / ms_graph * 1e3,
           "effective_GBps": 2 * sumD * 8 * 8 / (ms_graph * 1e-3) / 1e9,
           "max_rel_err_sampled_vs_fp64_oracle": max(errs)}
    if args.profile:
        print(json.dumps(out), flush=True)
        return
    # separate per-vector launches of the plain forms (contiguous single vectors)
    stream = torch.cuda.current_stream(dev)
    cols_c = [torch.from_numpy(np.ascontiguousarray(x[:, 0])).to(dev) for x in xs]
    outs_c = [torch.empty_like(c) for c in cols_c]
    ths = [torch.as_tensor(m.theta, dtype=torch.float64, device=dev) for m in models]
    ths32 = [t.float() for t in ths]
    for p, c, o, t in zip(plans, cols_c, outs_c, ths32):
        p.matvec(t, c, out=o)

    def sep_c():
        for _ in range(8):
            for p, c, o, t in zip(plans, cols_c, outs_c, ths32):
                p.matvec(t, c, out=o)
    ms_sep_c = cuda_time(sep_c, stream, 1)
    cols_z = [c.to(torch.complex128) for c in cols_c]
    outs_z = [torch.empty_like(c) for c in cols_z]
    for p, c, o, t in zip(plans, cols_z, outs_z, ths):
        p.matvec(t, c, out=o)

    def sep_z():
        for _ in range(8):
            for p, c, o, t in zip(plans, cols_z, outs_z, ths):
                p.matvec(t, c, out=o)
    ms_sep_z = cuda_time(sep_z, stream, 1)
    out["separate_c64_calls"] = {"ms_for_2048": ms_sep_c, "vector_matvecs_per_s": vec_mv / ms_sep_c * 1e3}
    out["separate_c128_calls"] = {"ms_for_2048": ms_sep_z, "vector_matvecs_per_s": vec_mv / ms_sep_z * 1e3}
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------------------------------ adjoint
def bench_adjoint(args, dev):
    import numpy as np
    import torch

    import workloads as W
    from oracle import grad as ograd
    from paper_2606_02169_amd.plan import Plan

    model, x = W.config(5)
    p = Plan.from_model(model, device=dev)
    xt = torch.from_numpy(x).to(dev)
    th = torch.as_tensor(model.theta, dtype=torch.float64, device=dev)
    p.autotune(th, xt)
    stream = torch.cuda.current_stream(dev)
    g = xt / torch.vdot(xt, xt).real
    for _ in range(3):
        p.adjoint(th, xt, g)
    ms_fwd = cuda_time(lambda: p.matvec(th, xt), stream, 50)
    ms_adj = cuda_time(lambda: p.adjoint(th, xt, g), stream, 50)
    # the same calls replayed from HIP graphs of 20 calls each: device time without the Python and
    # allocation overhead of the eager calls above (kernels already built by the warm-up)
    graph_ms = {}
    for name, fn in (("forward", lambda: p.matvec(th, xt)), ("adjoint", lambda: p.adjoint(th, xt, g))):
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            for _ in range(20):
                fn()
        gr.replay()
        torch.cuda.synchronize()
        graph_ms[name] = cuda_time(gr.replay, stream, 10) / 20
    # Rayleigh quotient gradients: dL/dx = 2 (Hx - L x)/<x|x>, dL/dtheta_p = <x|h_p|x>/<x|x>
    y = p.matvec(th, xt)
    L = (torch.vdot(xt, y).real / torch.vdot(xt, xt).real).item()
    gx, gt = p.adjoint(th, xt, g)
    gx = 2 * gx - 2 * L * g                  # dL/dx of Re<x|Hx>/<x|x> through the adjoint
    L_ref, gx_ref, gt_ref = ograd.rayleigh(model, x)
    out = {"metric": "adjoint (grad_x = H g and all coupling gradients) time vs forward matvec",
           "workload": "tavis_cummings_12x64_c128", "D": model.dim, "n_params": model.n_params,
           "forward_ms": ms_fwd, "adjoint_ms": ms_adj, "forward_graph_ms": graph_ms["forward"],
           "adjoint_graph_ms": graph_ms["adjoint"], "adjoint_form": "generated" if p.grad_kernel_ready() else "generic",
           "rel_err_grad_x": float(np.linalg.norm(gx.cpu().numpy() - gx_ref) / np.linalg.norm(gx_ref)),
           "max_abs_err_grad_theta": float(np.max(np.abs(gt.cpu().numpy() - gt_ref))),
           "loss": L, "loss_ref": L_ref}
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------------------------------ propagation
def bench_propagate(args, dev):
    """exp(-i H dt) on the 20-site ring (c128): Chebyshev terms per step, time per step with the fixed H's
    steps merged into one series (the default) and with one series per step, time per term, against the
    plain matvec; invariants (norm, reversal) on the same vector."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2606_02169_amd.plan import Plan

    model, x = W.config(2)
    p = Plan.from_model(model, device=dev)
    xt = torch.from_numpy(x).to(dev)
    del x
    th = torch.as_tensor(model.theta, dtype=torch.float64, device=dev)
    p.autotune(th, xt)
    tuned_cheb = p.autotune(th, xt, kernel="cheb")
    stream = torch.cuda.current_stream(dev)
    dt, steps = 0.05, (2 if args.profile else 4)
    bnd = p.norm_bound(model.theta)
    lo, hi = p.spectral_bounds(th)
    ms_gersh = cuda_time(lambda: p.spectral_bounds(th), stream, 1 if args.profile else 5)
    # the bounds of a 100-step piecewise drive (J_z and h_z modulated) in one pass over the rows
    drive = torch.as_tensor(np.stack([model.theta * np.array([1.0, 1 + 0.3 * np.sin(0.1 * k), 1.0,
                                                              1 + 0.5 * np.cos(0.1 * k)]) for k in range(100)]),
                            dtype=torch.float64, device=dev)
    ms_gersh_drive = cuda_time(lambda: p.spectral_bounds(drive), stream, 1 if args.profile else 3)
    pad = 1e-9 * max(hi - lo, abs(lo), abs(hi))
    bounds = (lo - pad, hi + pad)
    r = p.propagate(th, xt, dt, 1, bounds=bounds)
    nt = r["n_terms"]
    out = torch.empty_like(xt)
    reps = 1 if args.profile else 3
    # the steps of this fixed H are taken as one longer step (exp(-i H dt)^q = exp(-i H q dt)); the same
    # call with one series per step is timed below
    nt_call = p.propagate(th, xt, dt, steps, bounds=bounds, out=out)["n_terms"]
    ms = cuda_time(lambda: p.propagate(th, xt, dt, steps, bounds=bounds, out=out), stream, reps) / steps
    p.set_tuning(cheb_merge=0)
    ms_stepwise = cuda_time(lambda: p.propagate(th, xt, dt, steps, bounds=bounds, out=out), stream, reps) / steps
    x_stepwise = out.clone()
    p.set_tuning(cheb_merge=1)
    nt_norm, ms_norm = None, None
    if not args.profile:
        nt_norm = p.propagate(th, xt, dt, 1, bounds=(-bnd, bnd))["n_terms"]
        p.set_tuning(cheb_merge=0)   # per-step series, as ms_per_step_one_series_per_step
        ms_norm = cuda_time(lambda: p.propagate(th, xt, dt, steps, bounds=(-bnd, bnd), out=out), stream,
                            reps) / steps
        p.set_tuning(cheb_merge=1)
    y = torch.empty_like(xt)
    ms_mv = cuda_time(lambda: p.matvec(th, xt, out=y), stream, 3 if args.profile else 20)
    p.set_tuning(cheb_fused=0, cheb_merge=0)
    ms_two = cuda_time(lambda: p.propagate(th, xt, dt, steps, bounds=bounds, out=out), stream, reps) / steps
    p.set_tuning(cheb_fused=1, cheb_merge=1)
    out = p.propagate(th, xt, dt, steps, bounds=bounds, out=out)["x"]
    back = p.propagate(th, out, -dt, steps, bounds=bounds)["x"]
    res = {"metric": "exp(-i H dt) x by Chebyshev expansion over the matvec (c128)",
           "workload": "ferrimagnetic_ring_N20_c128", "D": model.dim, "dt": dt, "steps": steps,
           "gershgorin_bounds": [lo, hi], "gershgorin_ms": ms_gersh,
           "gershgorin_drive_100_steps": {"one_pass_ms": ms_gersh_drive, "one_vector_per_pass_ms": 100 * ms_gersh},
           "terms_per_step": nt,
           "ms_per_step": ms, "terms_merged_call": nt_call,
           "ms_per_step_one_series_per_step": ms_stepwise, "ms_per_term": ms_stepwise / max(1, nt - 1),
           "merged_vs_stepwise_rel_diff": ((out - x_stepwise).norm() / x_stepwise.norm()).item(),
           "norm_bound": bnd, "norm_bound_terms_per_step": nt_norm,
           "norm_bound_ms_per_step": ms_norm,
           "matvec_ms": ms_mv, "two_pass_ms_per_step": ms_two, "two_pass_ms_per_term": ms_two / max(1, nt - 1),
           "fused_speedup": ms_two / ms_stepwise, "cheb_kernel": {k: tuned_cheb.get(k) for k in
                                                         ("key", "variant", "inner_sites", "unrolled_sites",
                                                          "load_group", "us_per_call")},
           "norm_drift": abs(torch.linalg.vector_norm(out).item() - torch.linalg.vector_norm(xt).item()),
           "reversal_rel_err": ((back - xt).norm() / xt.norm()).item()}
    if not args.profile:
        # a piecewise-constant drive: 100 steps of dt = 0.05, J_z and h_z changed at every step (one series
        # per step; the bounds of all steps from one pass over the rows, included in the time)
        n_drive = 100
        res_out = torch.empty_like(xt)
        t0 = time.perf_counter()
        rd = p.propagate(drive, xt, dt, n_drive, out=res_out)
        torch.cuda.synchronize()
        s_drive = time.perf_counter() - t0
        p.__dict__.pop("_gersh_cache", None)    # time again with the bounds recomputed, not cached
        t0 = time.perf_counter()
        rd = p.propagate(drive, xt, dt, n_drive, out=res_out)
        torch.cuda.synchronize()
        s_drive = time.perf_counter() - t0
        res["driven_100_steps"] = {"seconds": s_drive, "ms_per_step": s_drive / n_drive * 1e3,
                                   "terms": rd["n_terms"], "terms_per_step": rd["n_terms"] / n_drive,
                                   "bounds": list(rd["bounds"]),
                                   "norm_drift": abs(torch.linalg.vector_norm(res_out).item()
                                                     - torch.linalg.vector_norm(xt).item())}
    log(str(res))
    print(json.dumps(res), flush=True)


# ------------------------------------------------------------------------------------------ restricted basis
def bench_sector(args, dev):
    """Fixed-S_z sectors (restricted basis, combinatorial-rank lookup): the 20-site ring's S_z = 0 sector
    and the spin-1 ring N = 15 at S_z = 0, against the full-basis matvec of the same lattice."""
    import numpy as np
    import torch

    import workloads as W
    from oracle import sector as osec
    from paper_2606_02169_amd.plan import Plan, Sector

    out = {"metric": "sector H·x (P H P^T) matvecs/s and sector Lanczos", "cases": {}}
    stream = torch.cuda.current_stream(dev)
    cases = (("ferrimagnetic_ring_N20_Sz0", W.config(2, with_state=False)[0]),
             ("spin1_ring_N15_Sz0", W.paper_c1()))
    for name, model in cases[:1] if args.profile else cases:
        plan = Plan.from_model(model, device=dev)
        Q = Sector.digit_sum_of(model.sites, 0.0)
        S = Sector(plan, Q)
        rng = np.random.default_rng(31)
        x = W.random_state(S.dim, rng)
        xt = torch.from_numpy(x).to(dev)
        th = torch.as_tensor(model.theta, dtype=torch.float64, device=dev)
        y = torch.empty_like(xt)
        for _ in range(3):
            S.matvec(th, xt, out=y)
        ms = cuda_time(lambda: S.matvec(th, xt, out=y), stream, 5 if args.profile else 20)
        if args.profile:
            out["cases"][name] = {"D_sector": S.dim, "sector_matvec_ms": ms}
            continue
        lab = osec.labels(model, Q)
        rows = np.unique(rng.choice(S.dim, 2000, replace=False)).astype(np.int64)
        err = float(np.linalg.norm(y[torch.from_numpy(rows).to(dev)].cpu().numpy()
                                   - osec.matvec(model, Q, x, lab=lab, rows=rows))
                    / np.linalg.norm(osec.matvec(model, Q, x, lab=lab, rows=rows)))
        torch.cuda.synchronize()
        lzs = {}
        for ro in ("cgs2", "partial"):
            t0 = time.perf_counter()
            r = S.lanczos(th, xt, 100, reorth=ro)
            torch.cuda.synchronize()
            dt_lz = time.perf_counter() - t0
            res = r["result"].cpu().numpy()
            lzs[ro] = {"steps": int(res[3]), "reorth": ro, "seconds": dt_lz, "E0": float(res[0]),
                       "residual": float(res[2])}
            if ro == "partial":
                lzs[ro]["gram_schmidt_passes"] = int(r["counts"].cpu().numpy()[1])
            del r
        xf = torch.zeros(model.dim, dtype=torch.complex128, device=dev)
        plan.autotune(th, xf)
        yf = torch.empty_like(xf)
        ms_full = cuda_time(lambda: plan.matvec(th, xf, out=yf), stream, 20)
        # time propagation, 4 steps of dt = 0.05, in the sector and on the full basis (a vector supported
        # on the sector, so both compute the same state), with the same bounds: the sector's own Gershgorin
        # ends (the default), which the plan's contain
        xf.zero_()
        xf[S.labels()] = xt
        sb = S.spectral_bounds(th)
        pb = plan.spectral_bounds(th)
        prop = {"sector_bounds": list(sb), "sector_bounds_ms": cuda_time(lambda: S.spectral_bounds(th), stream, 5),
                "plan_bounds": list(pb), "terms_with_plan_bounds": S.propagate(th, xt, 0.05, 4, bounds=pb)["n_terms"]}
        for where, fn in (("sector", lambda b: S.propagate(th, xt, 0.05, 4, bounds=b)),
                          ("full_basis", lambda b: plan.propagate(th, xf, 0.05, 4, bounds=b))):
            b = fn(None)["bounds"] if where == "sector" else prop["sector"]["bounds"]
            fn(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn(b)
            torch.cuda.synchronize()
            dt_p = time.perf_counter() - t0
            prop[where] = {"seconds": dt_p, "terms": r["n_terms"], "ms_per_term": dt_p / r["n_terms"] * 1e3,
                           "bounds": list(b)}
            if where == "sector":
                ys_prop = r["x"]
            else:
                prop["max_abs_diff_on_sector"] = float((r["x"][S.labels()] - ys_prop).abs().max())
        del xf, yf
        torch.cuda.empty_cache()
        out["cases"][name] = {
            "D_full": model.dim, "D_sector": S.dim, "digit_sum": Q, "sector_matvec_ms": ms,
            "sector_matvecs_per_s": 1000.0 / ms, "sector_rows_per_s": S.dim / ms * 1e3,
            "sector_effective_GBps": 2 * S.dim * 16 / ms / 1e6, "full_matvec_ms": ms_full,
            "sampled_rel_err_vs_oracle": err,
            "lanczos": lzs["cgs2"], "lanczos_partial_reorth": lzs["partial"], "propagate_4x0.05": prop}
        log(f"{name}: {out['cases'][name]}")
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------------------------------ parameter sweep
def bench_sweep(args, dev):
    """A parameter sweep as one batched launch: the 14-site ferrimagnetic ring (D = 279,936) at 256 coupling
    vectors (64 values of J_z times 4 fields h_z), each applied to the same 8 c64 vectors, replayed from a
    HIP graph; against the same 2048 products as separate c64 calls of the plain matvec, one coupling
    vector and one vector per call.  Sampled rows of every 32nd point against the oracle in FP64."""
    import dataclasses

    import numpy as np
    import torch

    import workloads as W
    from oracle import mf
    from paper_2606_02169_amd.plan import Batch, Plan, Sweep

    base = W.ferrimagnetic_ring(14)
    thetas = [np.array([1.0, jz, 0.5, hz]) for hz in (0.0, 0.1, 0.2, 0.3) for jz in np.linspace(0.5, 2.0, 64)]
    models = [dataclasses.replace(base, theta=t) for t in thetas]
    x = W.random_state(base.dim, np.random.default_rng(6), np.complex64, nvec=8)
    plan = Plan.from_model(base, device=dev)
    B = Batch([plan] * len(models), 8)
    X = torch.zeros(B.total_elems, dtype=torch.complex64, device=dev)
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    for b in range(len(models)):
        B.block(X, b).copy_(xd)
    Y = torch.empty_like(X)
    th32 = np.concatenate(thetas).astype(np.float32)
    th = torch.from_numpy(th32).to(dev)
    if args.profile:  # for a profiler: the shape the autotuner selects for this sweep on MI355X, no search
        B.set_shape(512, 512, "xcd_chunk")
        shape = B.shape()
    else:
        shape = B.autotune(th, X, Y)
    s = torch.cuda.Stream(device=dev)
    B.capture(th, X, Y, s)
    for _ in range(3):
        B.replay(s)
    s.synchronize()
    K = 10
    a = torch.cuda.Event(enable_timing=True)
    b_ = torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(K):
        B.replay(s)
    b_.record(s)
    s.synchronize()
    ms_graph = a.elapsed_time(b_) / K
    n_mv = len(models) * 8
    rng = np.random.default_rng(7)
    r = np.unique(rng.choice(base.dim, 2000, replace=False)).astype(np.int64)
    errs = []
    for bi in range(0, len(models), 32):
        m = dataclasses.replace(base, theta=th32[4 * bi: 4 * bi + 4].astype(np.float64))
        yb = B.block(Y, bi).cpu().numpy()
        for v in (0, 7):
            ref = mf.matvec(m, x[:, v].astype(np.complex128), rows=r)
            errs.append(float(np.linalg.norm(yb[r, v] - ref) / np.linalg.norm(ref)))
    # the same sweep with one shared input block (no copy per point; items tile by tile across the points)
    Bs = Batch([plan] * len(models), 8)
    Bs.share_input(True)
    Xs = torch.zeros(Bs.input_elems, dtype=torch.complex64, device=dev)
    Xs[: base.dim * 8].view(base.dim, 8).copy_(xd)
    Ys = torch.empty_like(Y)
    if args.profile:
        Bs.set_shape(512, 512, "windows")
        shape_s = Bs.shape()
    else:
        shape_s = Bs.autotune(th, Xs, Ys)
    Bs.capture(th, Xs, Ys, s)
    for _ in range(3):
        Bs.replay(s)
    s.synchronize()
    a.record(s)
    for _ in range(K):
        Bs.replay(s)
    b_.record(s)
    s.synchronize()
    ms_shared = a.elapsed_time(b_) / K
    same = bool(torch.equal(Ys, Y))
    # the sweep by linearity: the 4 group products h_p X in one batched launch, then the 256 outputs
    # Y_k = sum_p theta_kp h_p X in one combining pass
    sw = Sweep(plan, 8)
    thk = torch.from_numpy(np.stack(thetas).astype(np.float32)).to(dev)
    Yl = torch.empty(len(models) * sw.stride, dtype=torch.complex64, device=dev)
    sw.run(thk, Xs, out=Yl)
    torch.cuda.synchronize()
    ms_lin = cuda_time(lambda: sw.run(thk, Xs, out=Yl), torch.cuda.current_stream(dev), 10)
    lin_err = max(float((sw.block(Yl, k) - Bs.block(Ys, k)).norm() / Bs.block(Ys, k).norm())
                  for k in range(0, len(models), 16))
    if args.profile:
        print(json.dumps({"workload": "ferrimagnetic_ring_N14_sweep_256x8_c64", "shape": shape,
                          "ms_per_launch": ms_graph, "shared_input_shape": shape_s,
                          "shared_input_ms_per_launch": ms_shared, "shared_equals_copies_bitwise": same,
                          "by_linearity_ms": ms_lin, "by_linearity_max_rel_diff": lin_err,
                          "max_rel_err_sampled_vs_fp64_oracle": max(errs)}), flush=True)
        return
    # the same products as separate plain c64 calls
    stream = torch.cuda.current_stream(dev)
    col = torch.from_numpy(np.ascontiguousarray(x[:, 0])).to(dev)
    outc = torch.empty_like(col)
    ths = [torch.from_numpy(th32[4 * k: 4 * k + 4].copy()).to(dev) for k in range(len(models))]
    plan.matvec(ths[0], col, out=outc)

    def separate():
        for _ in range(8):
            for t in ths:
                plan.matvec(t, col, out=outc)
    ms_sep = cuda_time(separate, stream, 1)
    out = {"metric": "parameter sweep: vector-matvecs/s of one lattice at 256 coupling vectors x 8 c64 vectors",
           "workload": "ferrimagnetic_ring_N14_sweep_256x8_c64", "D": base.dim, "points": len(models),
           "vector_matvecs_per_launch": n_mv, "shape": shape, "ms_per_launch": ms_graph,
           "vector_matvecs_per_s": n_mv / ms_graph * 1e3,
           "effective_GBps": 2 * base.dim * len(models) * 8 * 8 / (ms_graph * 1e-3) / 1e9,
           "shared_input": {"shape": shape_s, "ms_per_launch": ms_shared,
                            "vector_matvecs_per_s": n_mv / ms_shared * 1e3,
                            "equals_copies_bitwise": same},
           "by_linearity": {"ms": ms_lin, "vector_matvecs_per_s": n_mv / ms_lin * 1e3,
                            "output_GBps": len(models) * base.dim * 8 * 8 / (ms_lin * 1e-3) / 1e9,
                            "max_rel_diff_vs_direct": lin_err},
           "separate_c64_calls": {"ms_for_2048": ms_sep, "vector_matvecs_per_s": n_mv / ms_sep * 1e3},
           "max_rel_err_sampled_vs_fp64_oracle": max(errs)}
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------------------------------ small chain
def bench_chain12(args, dev):
    """The 12-site spin-1/2 Heisenberg chain (D = 4096, seed 1): one c128 H x and a 50-step Lanczos (CGS2),
    each called eagerly and replayed from a HIP graph.  At this size every kernel is launch-bound, so the
    graph removes the host's launch and marshalling time; the replayed Lanczos equals the eager one
    bitwise (deterministic reductions)."""
    import numpy as np
    import torch

    import workloads as W
    from oracle import kron
    from oracle import lanczos as olz
    from oracle import mf
    from paper_2606_02169_amd.plan import Plan

    model, x = W.config(1)
    p = Plan.from_model(model, device=dev)
    xt = torch.from_numpy(x).to(dev)
    th = torch.as_tensor(model.theta, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    steps = 50
    ref = p.lanczos(th, xt, steps)                      # also builds the generated kernel
    y = p.matvec(th, xt)
    torch.cuda.synchronize()
    ms_mv = cuda_time(lambda: p.matvec(th, xt, out=y), stream, 200)
    ms_lz = cuda_time(lambda: p.lanczos(th, xt, steps), stream, 5)
    gm = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gm):
        for _ in range(20):
            p.matvec(th, xt, out=y)
    gl = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gl):
        out = p.lanczos(th, xt, steps)
    gm.replay()
    gl.replay()
    torch.cuda.synchronize()
    same = bool(torch.equal(out["alpha"], ref["alpha"]) and torch.equal(out["beta"], ref["beta"])
                and torch.equal(out["result"], ref["result"]))
    ms_mv_graph = cuda_time(gm.replay, stream, 20) / 20
    ms_lz_graph = cuda_time(gl.replay, stream, 5)
    res = ref["result"].cpu().numpy()
    ev0 = float(np.linalg.eigvalsh(kron.dense_H(model))[0])
    olz_ref = olz.lanczos(lambda v: mf.matvec(model, v), x, steps)
    out_line = {"metric": "small-lattice H x and Lanczos, eager and replayed from a HIP graph",
                "workload": "heisenberg_chain_N12_c128", "D": model.dim, "seed": 1, "lanczos_steps": steps,
                "matvec_us": ms_mv * 1e3, "matvec_graph_us": ms_mv_graph * 1e3,
                "lanczos_ms": ms_lz, "lanczos_graph_ms": ms_lz_graph,
                "lanczos_graph_equals_eager_bitwise": same,
                "E0": float(res[0]), "residual": float(res[2]), "E0_exact_diag": ev0,
                "E0_oracle_lanczos": float(olz_ref["theta"]),
                "max_abs_alpha_diff_vs_oracle": float(np.max(np.abs(ref["alpha"].cpu().numpy() - olz_ref["alpha"])))}
    print(json.dumps(out_line), flush=True)


# ------------------------------------------------------------------------------------------ stream ceilings
def bench_stream(args, dev):
    """Stream ceilings of this GPU from the standalone probe built beside the library (run as a child
    process): reads of footprints from L2 size to HBM size with the default and the non-temporal cache
    policy, copies, and 8-row window gathers of growing span.  These are the rates the gather kernels'
    L2-miss traffic is compared with."""
    import subprocess
    from paper_2606_02169_amd.build import PROBE
    if not os.path.exists(PROBE):
        print(f"{PROBE} is missing: build with paper_2606_02169_amd.build.build()", file=sys.stderr)
        sys.exit(1)
    r = subprocess.run([PROBE], capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        print(r.stdout + r.stderr, file=sys.stderr)
        sys.exit(r.returncode)
    rows = [json.loads(line) for line in r.stdout.splitlines() if line.startswith("{")]
    out = {"metric": "stream ceilings of one MI355X (GB/s): reads by footprint and cache policy, copy, "
                     "window gathers", "lines": rows}
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------------------------------ paper testbeds
PAPER_TABLE1 = {  # Table I, matrix-free rows (CPU, model not stated, 60 threads): context only
    "spin1_ring_N15": {"matvecs_per_s": 6.137, "eigensolve_s": 29.28, "residual": 2.961e-10},
    "mixed_ring_N18": {"matvecs_per_s": 0.04387, "eigensolve_s": 2748.0, "residual": 7.296e-10},
}


def bench_paper(args, dev):
    import numpy as np
    import torch

    import workloads as W
    from oracle import mf
    from paper_2606_02169_amd.plan import Plan

    out = {"metric": "H·x matvecs/s and Lanczos on the paper's chain testbeds C1 and C2 (synthetic, same lattices)",
           "cases": {}}
    stream = torch.cuda.current_stream(dev)
    for model, seed, m_steps in ((W.paper_c1(), 11, 100), (W.paper_c2(), 12, 60)):
        rng = np.random.default_rng(seed)
        x_host = W.random_state(model.dim, rng)
        D = model.dim
        plan = Plan.from_model(model, device=dev)
        x = torch.from_numpy(x_host).to(dev)
        y = torch.empty_like(x)
        th = torch.as_tensor(model.theta, dtype=torch.float64, device=dev)
        tuned = plan.autotune(th, x, y)
        for _ in range(3):
            plan.matvec(th, x, out=y)
        ms = cuda_time(lambda: plan.matvec(th, x, out=y), stream, 20)
        rows = np.unique(rng.choice(D, 3000, replace=False)).astype(np.int64)
        ref = mf.matvec(model, x_host, rows=rows)
        err = float(np.linalg.norm(y[torch.from_numpy(rows).to(dev)].cpu().numpy() - ref) / np.linalg.norm(ref))
        del y
        torch.cuda.synchronize()
        if args.profile:  # short run for a profiler: the matvec launches only (C1's first, then C2's)
            out["cases"][model.name] = {"D": D, "matvec_ms_c128": ms, "sampled_rel_err_vs_oracle": err,
                                        "kernel": {k: tuned.get(k) for k in ("variant", "inner_sites", "unrolled_sites", "unroll_top")}}
            continue
        lz = {}
        for ro in ("cgs2", "partial"):
            t0 = time.perf_counter()
            r = plan.lanczos(th, x, m_steps, reorth=ro)
            torch.cuda.synchronize()
            lz_s = time.perf_counter() - t0
            res = r["result"].cpu().numpy()
            lz[ro] = {"steps": int(res[3]), "reorth": ro, "seconds": lz_s, "E0": float(res[0]),
                      "residual": float(res[2])}
            if ro == "partial":
                lz[ro]["gram_schmidt_passes"] = int(r["counts"].cpu().numpy()[1])
            del r   # the basis (187 GB for C2) stays in torch's cache for the next run: no new allocation
        torch.cuda.empty_cache()
        paper = PAPER_TABLE1[model.name]
        out["cases"][model.name] = {
            "D": D, "seed": seed, "kernel": {k: tuned.get(k) for k in ("variant", "inner_sites", "unrolled_sites", "unroll_top")},
            "matvec_ms_c128": ms, "matvecs_per_s": 1000.0 / ms, "effective_GBps": 2 * D * 16 / ms / 1e6,
            "sampled_rel_err_vs_oracle": err,
            "lanczos": lz["cgs2"], "lanczos_partial_reorth": lz["partial"],
            "paper_cpu_mf": paper, "matvec_speedup_vs_paper_cpu": (1000.0 / ms) / paper["matvecs_per_s"]}
        log(f"{model.name}: {out['cases'][model.name]}")
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", action="store_true", help="short run for a profiler: no CPU leg")
    ap.add_argument("--kernel", default="auto", choices=["auto", "generic", "specialized"])
    ap.add_argument("--workload", default="ring20", choices=["ring20", "torus", "lanczos4x4", "lanczos_ring20",
                                                              "batched", "adjoint", "paper", "propagate", "sector",
                                                              "stream", "chain12", "sweep"])
    ap.add_argument("--dtype", default=None, choices=["c64", "c128"], help="torus: one element type only")
    ap.add_argument("--lanczos-steps", type=int, default=100)
    ap.add_argument("--lanczos-ref-steps", type=int, default=150)
    ap.add_argument("--lanczos-ref-reorth", default="cgs2", choices=["cgs2", "cgs2_cond", "partial"],
                    help="lanczos4x4: reorthogonalisation of the FP64 reference run")
    ap.add_argument("--batch-schedule", default="windows", choices=["windows", "xcd_chunk", "runs"],
                    help="work schedule of the batched leg under --profile (with the tiles the autotuner picks)")
    ap.add_argument("--lanczos-forms", default="cgs2,cgs2_cond,partial",
                    help="lanczos4x4 / lanczos_ring20: reorthogonalisations to time (comma list)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the matvec is measured on one GPU's share of the work; "
              "runs over several GPUs are not supported (use --gpus 1).", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU (the HIP library has no CPU path)", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    {"ring20": bench_ring, "torus": bench_torus, "lanczos4x4": bench_lanczos, "lanczos_ring20": bench_lanczos_ring, "batched": bench_batched,
     "adjoint": bench_adjoint, "paper": bench_paper, "propagate": bench_propagate,
     "sector": bench_sector, "stream": bench_stream, "chain12": bench_chain12,
     "sweep": bench_sweep}[args.workload](args, dev)


if __name__ == "__main__":
    main()
