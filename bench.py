#!/usr/bin/env python3
"""Throughput of the penalized lattice-Boltzmann step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one pass of the whole hot path: the fused stream-collide-penalize
lattice update, the per-particle momentum sums, Algorithm 1 and the
re-rasterisation of the indicator, on the synthetic 2048x4096 D2Q9
sedimentation workload (500 bodies: 350 disks R=8, 150 ellipses 12x6; inputs
resident in HBM).  The headline value is MLUPS with FP32 population storage;
the same line carries FP64, FP16 and BF16 storage, the 256x256x512 D3Q19
workload, the roofline of the fused kernel (algorithmic bytes over its
event-timed duration), a copy-kernel ceiling measured in the same run, and the
FP64 CPU oracle timed on a bounded sample of the same workload.

Prints ONE JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}
MATH = {"f64": "f64", "f32": "f32", "f16": "f32", "bf16": "f32"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ["paper_2511_01629_amd/csrc/stream_collide.hip", "paper_2511_01629_amd/csrc/node.h",
                  "paper_2511_01629_amd/csrc/lattice.h", "paper_2511_01629_amd/csrc/ctx.h",
                  "paper_2511_01629_amd/csrc/dispatch.h", "paper_2511_01629_amd/csrc/reduce.h"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(key):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != kernel_source_sha():
        return None
    w = t.get("workloads", {}).get(key)
    return None if w is None else w.get("bytes_per_launch")


def _counter_kib(csv_path, kernel_prefix):
    """Mean value (KiB per dispatch) of the counter in a rocprofv3 counter CSV
    over the dispatches of kernels whose name contains kernel_prefix (a
    substring: "k_copy(" to tell the one-array copy from k_copy_arrays)."""
    import csv

    vals = []
    with open(csv_path) as f:
        for r in csv.DictReader(f):
            if kernel_prefix in r["Kernel_Name"]:
                vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no dispatch of {kernel_prefix} in {csv_path}")
    return sum(vals) / len(vals), len(vals)


def record_traffic(root, storages, workload_name, copy_bytes):
    """Turn the FETCH_SIZE and WRITE_SIZE counter runs under root
    (pmc_FETCH_SIZE_<storage>/, pmc_WRITE_SIZE_<storage>/, each holding the
    rocprofv3 run_counter_collection.csv of `bench.py --steps 5 --warmup 2
    --no-modes --no-cpu --storage <storage>`) into profiles/traffic.json:
    HBM bytes per launch of the fused kernel, each counter scaled by what it
    reads for the library's copy kernel on copy_bytes read + copy_bytes written
    in the same run."""
    out = {"source_sha": kernel_source_sha(), "sources": KERNEL_SOURCES, "workloads": {}}
    for st in storages:
        entry = {}
        for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
            path = os.path.join(root, f"pmc_{ctr}_{st}", "run_counter_collection.csv")
            k_kib, k_n = _counter_kib(path, "k_stream_collide")
            c_kib, c_n = _counter_kib(path, "k_copy(")  # the one-array copy, not k_copy_arrays
            scale = copy_bytes / 1024.0 / c_kib
            entry[ctr] = {"kernel_kib": k_kib, "kernel_dispatches": k_n, "copy_kib": c_kib, "copy_dispatches": c_n,
                          "scale": scale, "bytes": k_kib * 1024.0 * scale}
        entry["bytes_per_launch"] = entry["FETCH_SIZE"]["bytes"] + entry["WRITE_SIZE"]["bytes"]
        out["workloads"][f"{workload_name}/{st}"] = entry
        log(f"{workload_name}/{st}: {entry['bytes_per_launch'] / 1e6:.1f} MB per launch "
            f"(read scale {entry['FETCH_SIZE']['scale']:.3f}, write scale {entry['WRITE_SIZE']['scale']:.3f})")
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    log(f"wrote {TRAFFIC_FILE}")


def run_mode(name, storage, steps, warmup, profile=True, fractional=False):
    import torch

    from paper_2511_01629_amd import lbm
    from paper_2511_01629_amd.workloads import workload

    cfg, parts, _, info = workload(name)
    if fractional:  # the same workload with the fractional indicator (disks and spheres only)
        cfg = dict(cfg, fractional=1)
    sim = lbm.Simulation(cfg, parts, storage=storage, device=0)
    N, Q = sim.N, sim.Q
    sim.step(warmup)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    sim.step(steps)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    sim.sync()  # raises if the run went unstable or a body left the box
    out = dict(workload=name, storage=storage, nodes=N, Q=Q, particles=len(parts), steps=steps, ms=ms,
               ms_per_step=ms / steps, mlups=N * steps / (ms * 1e-3) / 1e6)
    if profile:
        sim.profile(True)
        sim.step(steps)
        prof = sim.profile_read()
        sim.profile(False)
        kms, kcnt = prof["stream_collide"]
        k_avg_ms = kms / kcnt
        alg_bytes = 2 * Q * STORAGE_BYTES[storage] * N
        out.update(kernel_avg_us=k_avg_ms * 1e3, kernel_alg_bytes=alg_bytes,
                   kernel_gbs=alg_bytes / (k_avg_ms * 1e-3) / 1e9,
                   breakdown_us={k: (v[0] / max(v[1], 1)) * 1e3 for k, v in prof.items()})
        out["kernel_frac"] = out["kernel_gbs"] / HBM_PEAK_GBS
    out["step_gbs_alg"] = 2 * Q * STORAGE_BYTES[storage] * N * steps / (ms * 1e-3) / 1e9
    sim.close()
    del sim
    torch.cuda.empty_cache()
    if profile:
        # the bandwidth a plain copy reaches with the same access pattern: Q arrays of
        # N elements read and written together, 16-byte lanes
        out["pattern_ceiling_gbs"] = pattern_ceiling(Q, STORAGE_BYTES[storage] * N)
        out["kernel_frac_of_pattern"] = out["kernel_gbs"] / out["pattern_ceiling_gbs"]
    return out


def pattern_ceiling(narrays, bytes_per_array, reps=20):
    """GB/s of lbm_copy_arrays over narrays arrays of bytes_per_array bytes."""
    import torch

    from paper_2511_01629_amd import lbm

    per = (bytes_per_array + 15) // 16 * 16
    a = torch.empty(narrays * per, dtype=torch.uint8, device="cuda")
    b = torch.empty(narrays * per, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream()
    for _ in range(3):
        lbm.copy_arrays(b.data_ptr(), a.data_ptr(), narrays, per, st.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        lbm.copy_arrays(b.data_ptr(), a.data_ptr(), narrays, per, st.cuda_stream)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * narrays * per / (ms * 1e-3) / 1e9


def run_adjoint(name, storage, every, max_steps=None, fractional=False):
    """Forward with checkpoints + hand-written adjoint on the differentiated
    workload; fwd+adj MLUPS counts each node-step once.  max_steps shortens the
    run (profiling)."""
    import torch

    import numpy as np

    from paper_2511_01629_amd import lbm
    from paper_2511_01629_amd.workloads import workload

    cfg, parts, steps, _ = workload(name)
    if fractional:
        cfg = dict(cfg, fractional=1)
    if max_steps:
        steps = min(steps, max_steps)
    sim = lbm.Simulation(cfg, parts, storage=storage, device=0)
    N = sim.N
    seed = np.zeros((len(parts), 3))
    seed[:, 1] = 1.0 / len(parts)
    st = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(st)
    sim.forward_checkpointed(steps, every)
    e1.record(st)
    g_rho, g_tau, g_g = sim.backward(seed)
    e2.record(st)
    torch.cuda.synchronize()
    t_f, t_b = e0.elapsed_time(e1), e1.elapsed_time(e2)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    mlups = N * steps / ((t_f + t_b) * 1e-3) / 1e6
    # algorithmic bytes per node-step: forward 2 Q s, adjoint 2 Q 4 + d 4 (lambda in/out, u);
    # the recomputation of each segment is a checkpointing cost and is not credited
    alg = 2 * 9 * STORAGE_BYTES[storage] + 2 * 9 * 4 + 2 * 4
    return dict(workload=name, storage=storage, steps=steps, checkpoint_every=every, ms_forward=t_f,
                ms_backward=t_b, mlups=mlups, alg_bytes_per_node_step=alg,
                frac=mlups * 1e6 * alg / (HBM_PEAK_GBS * 1e9), grad_tau=g_tau, grad_gmag=g_g,
                grad_rho_s_first=float(g_rho[0]))


COPY_BYTES = 2 << 30  # copy-ceiling buffer: the counter calibration relies on this size


def copy_ceiling(nbytes=COPY_BYTES, reps=20):
    import torch

    from paper_2511_01629_amd import lbm

    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream()
    for _ in range(3):
        lbm.copy(b.data_ptr(), a.data_ptr(), nbytes, st.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        lbm.copy(b.data_ptr(), a.data_ptr(), nbytes, st.cuda_stream)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(name, budget_s):
    """The FP64 oracle as it stands, on the host cores, on the first steps of
    the same workload until `budget_s` seconds of stepping have run."""
    from oracle import oracle as O
    from paper_2511_01629_amd.workloads import workload

    cfg, parts, _, _ = workload(name)
    o = O.Oracle(cfg, parts)
    N = o.N
    o.step(1)  # first touch of every page
    steps, t0 = 0, time.perf_counter()
    while True:
        o.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 10000:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=N * steps / el / 1e6, unit="MLUPS", cores=cores, kind="oracle", cpu=cpu_model(),
                sample=f"{name}: {steps} FP64 steps of the full {N}-node lattice after one warm-up step "
                       f"({el:.1f} s)")


def cpu_baseline_one_thread(name, budget_s):
    """The same on one host thread, in a child process (the oracle's OpenMP
    thread count is fixed when it loads); the child touches no GPU."""
    import subprocess

    code = ("import json, sys; sys.path.insert(0, %r); import bench; "
            "print(json.dumps(bench.cpu_baseline(%r, %r)))" % (ROOT, name, budget_s))
    env = dict(os.environ, OMP_NUM_THREADS="1", HIP_VISIBLE_DEVICES="", ROCR_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        log(f"one-thread baseline failed: {r.stderr[-400:]}")
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="sedimentation_2048x4096")
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--no-modes", action="store_true", help="headline configuration only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the forward + adjoint leg (checkpoint every 100, then every step kept)")
    ap.add_argument("--adj-steps", type=int, default=None, help="shorten the forward + adjoint leg (profiling)")
    ap.add_argument("--record-traffic", metavar="DIR", default=None,
                    help="write profiles/traffic.json from the counter runs under DIR (no GPU needed)")
    args = ap.parse_args()
    if args.record_traffic:
        record_traffic(args.record_traffic, ("f32", "f16"), args.workload, COPY_BYTES)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the library runs on "
              f"one GPU; a multi-GPU run would shard the lattice in slabs with a halo exchange, not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2511_01629_amd import lbm

    lbm.load()
    torch.cuda.init()
    log(f"device: {torch.cuda.get_device_name(0)}")
    if args.adjoint_only:
        for every in (100, 1):
            adj = run_adjoint("adjoint_512x1024", "f32", every, args.adj_steps)
            log(f"every {every}: {adj['mlups']:.0f} MLUPS fwd+adj ({adj['ms_forward']:.1f} ms forward, "
                f"{adj['ms_backward']:.1f} ms backward, {adj['steps']} steps), {adj['frac']:.3f} of roofline")
        return
    log(f"headline {args.workload} {args.storage}: warmup {args.warmup}, steps {args.steps}")
    head = run_mode(args.workload, args.storage, args.steps, args.warmup)
    log(f"  {head['mlups']:.0f} MLUPS, fused kernel {head['kernel_gbs']:.0f} GB/s ({head['kernel_frac']:.3f}), "
        f"{head['Q']}-array copy of the same bytes {head['pattern_ceiling_gbs']:.0f} GB/s")

    modes = {}
    if not args.no_modes:
        for name, storage, steps, frac in ((args.workload, "f64", args.steps // 2, False),
                                           (args.workload, "f16", args.steps, False),
                                           (args.workload, "bf16", args.steps, False),
                                           ("spheres_256x256x512", "f32", 100, False),
                                           ("spheres_256x256x512", "f32", 100, True)):
            key = f"{name}/{storage}" + ("/fractional" if frac else "")
            log(f"mode {key}")
            r = run_mode(name, storage, steps, max(10, args.warmup // 4), fractional=frac)
            modes[key] = {k: r[k] for k in ("mlups", "ms_per_step", "kernel_gbs", "kernel_frac", "kernel_avg_us",
                                            "breakdown_us", "pattern_ceiling_gbs", "kernel_frac_of_pattern")}
            modes[key]["step_frac"] = r["step_gbs_alg"] / HBM_PEAK_GBS
            log(f"  {r['mlups']:.0f} MLUPS, fused kernel {r['kernel_gbs']:.0f} GB/s, "
                f"{r['Q']}-array copy of the same bytes {r['pattern_ceiling_gbs']:.0f} GB/s")
    if not args.no_modes:
        log("forward + adjoint adjoint_512x1024 f32 (5000 steps; checkpoint every 100, and every step kept)")
        for every, frac in ((100, False), (1, False), (100, True)):
            adj = run_adjoint("adjoint_512x1024", "f32", every, args.adj_steps, fractional=frac)
            modes[f"adjoint_512x1024/f32/fwd+adj/every{every}" + ("/fractional" if frac else "")] = adj
            log(f"  every {every}{' fractional' if frac else ''}: {adj['mlups']:.0f} MLUPS fwd+adj "
                f"({adj['ms_forward']:.0f} ms forward, {adj['ms_backward']:.0f} ms backward), "
                f"{adj['frac']:.3f} of roofline")
    log("copy ceiling")
    ceiling = copy_ceiling()
    log(f"  {ceiling:.0f} GB/s")

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(args.workload, args.cpu_seconds)
        log(f"  {cpu['value']:.1f} MLUPS on {cpu['cores']} threads ({cpu['cpu']})")
        one = cpu_baseline_one_thread(args.workload, args.cpu_seconds)
        if one:
            cpu["one_thread"] = {"value": one["value"], "unit": "MLUPS", "cores": 1, "sample": one["sample"]}
            log(f"  {one['value']:.1f} MLUPS on 1 thread")

    key = f"{args.workload}/{args.storage}"
    traffic = measured_traffic(key)
    from paper_2511_01629_amd.workloads import workload

    wcfg = workload(args.workload)[0]
    dims = list(wcfg["n"][:2] if wcfg["lattice"] == "D2Q9" else wcfg["n"])
    line = {
        "metric": "MLUPS & % HBM roofline: FP64 vs FP32 vs FP16-store; fwd+adjoint MLUPS",
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": MATH[args.storage],
        "data": "synthetic (seeded placement, no dataset)",
        "config": {"workload": args.workload, "lattice": wcfg["lattice"], "n": dims, "bodies": head["particles"],
                   "storage": args.storage, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": head["kernel_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["kernel_frac"], "traffic": traffic,
                     "kernel": "k_stream_collide", "alg_bytes_per_launch": head["kernel_alg_bytes"],
                     "avg_launch_us": head["kernel_avg_us"],
                     # the whole step (lattice update + particle side) against the same peak
                     "step_achieved": head["step_gbs_alg"], "step_frac": head["step_gbs_alg"] / HBM_PEAK_GBS,
                     # a plain copy of the same Q arrays (Q streams read and Q written together)
                     "pattern_ceiling": head["pattern_ceiling_gbs"],
                     "frac_of_pattern": head["kernel_frac_of_pattern"]},
        "step_breakdown_us": head["breakdown_us"],
        "copy_ceiling_gbs": ceiling,
        "modes": modes,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
