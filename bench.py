"""Benchmark of the HDArray ApplyKernel hot path on one MI355X.

One step = one ApplyKernel call: communication-set derivation from GDEF,
pack, unpack, the user kernel on every logical device, GDEF update.

Default workload (the one the headline metric is quoted on): jacobi_large,
2-D 5-point Jacobi on 8192 x 8192 fp32, 16 logical devices in a 4 x 4 block
grid, use = own block +-1 (5-point offsets), def = own block, ping-pong
A <- J(B), B <- J(A).  Synthetic U[0,1) inputs (see workloads/).

Prints ONE JSON line.  value = whole-job steps/s with inputs resident in
HBM; roofline = the dominant kernel (the Jacobi kernel over all 16 devices)
measured with HIP events on its own stream during the timed region;
cpu_baseline = the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "ApplyKernel steps/s + pack/unpack GB/s (% HBM peak), plain vs batched/adjoint"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1809_05657_amd/csrc/hd_data.hip"]


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def committed_traffic(name, bytes_alg):
    """HBM traffic per launch from committed rocprofv3 PMC summaries, or None
    when absent or taken on another version of the kernel source."""
    p = os.path.join(ROOT, "profiles", f"{name}_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_hash") != kernel_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def setup_jacobi_large(rt, hd, n):
    from workloads import jacobi_inputs
    A0, B0 = jacobi_inputs(n, 2)
    A, B = rt.create(A0), rt.create(B0)
    p = rt.partition(hd.BLOCK, (n, n), ndev=16)
    offs = [(0, 0), (0, -1), (0, 1), (-1, 0), (1, 0)]
    for k, out, inp in (("jacAB", A, B), ("jacBA", B, A)):
        rt.kernel(k, hd.K_JACOBI2D)
        rt.set_offsets(k, 1, 0, offs)
        rt.set_offsets(k, 0, 1, [(0, 0)])
    rt.write(A, A0, p)
    rt.write(B, B0, p)
    del A0, B0
    return A, B, p


def cpu_baseline_jacobi(n, steps):
    """The oracle as it stands, on a bounded sample: `steps` ApplyKernel
    steps of the same workload (same sizes, partitions, declarations)."""
    import oracle as O
    from workloads import jacobi_inputs
    A0, B0 = jacobi_inputs(n, 2)
    o = O.Oracle()
    A, B = o.create(A0), o.create(B0)
    p = o.partition(O.BLOCK, (n, n), ndev=16)
    offs = [(0, 0), (0, -1), (0, 1), (-1, 0), (1, 0)]
    for k in ("jacAB", "jacBA"):
        o.kernel(k, O.K_JACOBI2D)
        o.set_offsets(k, 1, 0, offs)
        o.set_offsets(k, 0, 1, [(0, 0)])
    o.write(A, A0, p)
    o.write(B, B0, p)
    t0 = time.perf_counter()
    for it in range(steps):
        if it % 2 == 0:
            o.apply("jacAB", p, [A, B])
        else:
            o.apply("jacBA", p, [B, A])
    dt = time.perf_counter() - t0
    o.close()
    return steps / dt, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs the ApplyKernel path on one GPU only (the logical devices are "
              "partitions of one MI355X); multi-GPU runs are not supported.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1809_05657_amd as hd

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    rt = hd.Runtime(stream=stream.cuda_stream)
    n = args.n
    A, B, p = setup_jacobi_large(rt, hd, n)

    def step(i):
        if i % 2 == 0:
            rt.apply("jacAB", p, [A, B])
        else:
            rt.apply("jacBA", p, [B, A])

    for i in range(args.warmup):
        step(i)
    rt.sync()
    torch.cuda.synchronize()
    # timed region: only the user-kernel phase carries an event pair (bit 3)
    rt.profile(1 << 3)
    rt.profile_read()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i)
    rt.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = rt.profile_read()
    kms, kcnt = prof["kernel"]
    # a second pass with every phase timed, for the breakdown and pack/unpack
    rt.profile(0xF)
    for i in range(20):
        step(args.warmup + args.steps + i)
    rt.sync()
    ph = rt.profile_read()
    rt.profile(0)
    st = rt.stats()
    ms_step = dt * 1e3 / args.steps
    bytes_kernel = 2 * 4 * n * n  # read B once, write A once per step
    avg_kernel_ms = kms / max(kcnt, 1)
    achieved = bytes_kernel / (avg_kernel_ms * 1e-3) / 1e9
    pk_ms = ph["pack"][0] / max(ph["pack"][1], 1)
    up_ms = ph["unpack"][0] / max(ph["unpack"][1], 1)
    moved = st["last_bytes"]
    out = {
        "metric": METRIC,
        "value": args.steps / dt,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"jacobi_large: 2-D 5-point Jacobi {n}x{n} fp32, 16 logical devices (4x4 blocks), "
                               f"use = own block +-1 (5-point offsets), def = own block, ping-pong",
                   "n": n, "partitions": 16, "messages_per_step": st["last_messages"],
                   "halo_bytes_per_step": moved},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": committed_traffic("jacobi2d_8192", bytes_kernel),
                     "kernel": "k_jacobi<16,false>", "bytes_per_launch": bytes_kernel,
                     "avg_launch_us": avg_kernel_ms * 1e3},
        "step_hbm_frac": bytes_kernel / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "phases_us": {k: (v[0] / max(v[1], 1)) * 1e3 for k, v in ph.items()},
        "pack_unpack": {"bytes": moved, "pack_GBps": 2 * moved / max(pk_ms * 1e-3, 1e-12) / 1e9,
                        "unpack_GBps": 2 * moved / max(up_ms * 1e-3, 1e-12) / 1e9},
    }
    rt.close()
    if not args.no_cpu_baseline:
        sps, secs = cpu_baseline_jacobi(n, args.cpu_steps)
        out["cpu_baseline"] = {"value": sps, "unit": "steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"{args.cpu_steps} ApplyKernel step(s) of jacobi_large ({n}x{n}, 16 "
                                         f"devices) after setup, single-threaded C oracle, {secs:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
