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
KERNEL_SOURCES = ["paper_1809_05657_amd/csrc/hd_jacobi.hip", "paper_1809_05657_amd/csrc/hd_dev_jacobi.hpp",
                  "paper_1809_05657_amd/csrc/hd_dev_common.hpp"]
# sources of the 3-D stencil, its adjoint and the adjoint's reverse pack / add
S3D_SOURCES = ["paper_1809_05657_amd/csrc/hd_adj.hip", "paper_1809_05657_amd/csrc/hd_data.hip",
               "paper_1809_05657_amd/csrc/hd_dev_data.hpp", "paper_1809_05657_amd/csrc/hd_dev_common.hpp"]


def kernel_hash(sources=KERNEL_SOURCES):
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def committed_traffic(name, kernel, sources=KERNEL_SOURCES):
    """HBM traffic per launch from committed rocprofv3 PMC summaries, or None
    when absent, taken on another version of the kernel source, or on
    another tile shape of the kernel."""
    p = os.path.join(ROOT, "profiles", f"{name}_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_hash") != kernel_hash(sources):
        return None
    return d.get("kernels", {}).get(kernel, {}).get("hbm_bytes_per_launch")


KERNEL_SAMPLE = 4  # every 4th step of a timed loop times its stencil launch
TUNE_CALLS = 36    # calls that cover the runtime's tile-shape timing (4 shapes x 8 calls)


def committed_kernel_avg(name, kernel):
    """Average duration (us) of a kernel in the committed rocprofv3 summary
    profiles/NAME_kernels.txt, or None when absent."""
    p = os.path.join(ROOT, "profiles", f"{name}_kernels.txt")
    if not os.path.exists(p):
        return None
    for line in open(p):
        f = line.split()
        if len(f) == 6 and f[0] == kernel:
            return float(f[3])
    return None


def short_kernel_name(n):
    """A profiler kernel name without namespace, return type, arguments or
    spaces (k_stack_a<4,0>)."""
    n = n.strip('"').replace("void ", "").replace("hd::", "")
    return n.split("(")[0].replace(" ", "")


def pmc_means(folder, counter):
    """Mean value per dispatch of one counter for every kernel of a
    rocprofv3 --pmc CSV output folder: {kernel: (mean, dispatches)}."""
    import csv
    import glob
    acc = {}
    for f in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] != counter:
                    continue
                s = acc.setdefault(short_kernel_name(row["Kernel_Name"]), [0.0, 0])
                s[0] += float(row["Counter_Value"])
                s[1] += 1
    return {k: (v[0] / v[1], v[1]) for k, v in acc.items()}


# algorithmic bytes per launch of the kernels whose traffic is summarised
TRAFFIC_WORKLOADS = {
    "jacobi2d_8192": {"workload": "jacobi_large (8192x8192 fp32, 16 devices 4x4, ping-pong); every tile shape the "
                                  "runtime tries", "sources": KERNEL_SOURCES,
                      "bytes": {k: 8 * 8192 * 8192 for k in ("k_stack_a", "k_stack", "k_jacobi1", "k_strip")},
                      "bench": "python3 bench.py --steps 20 --warmup 3 --no-cpu-baseline --headline-only"},
    "stencil3d_512": {"workload": "stencil3d 512^3 fp32, 8 devices (2x2x2), T=64, checkpoint every 8: forward and "
                                  "adjoint steps", "sources": S3D_SOURCES,
                      "bytes": {"k_s3d": 8 * 512 ** 3, "k_s3d_adj": 12 * 512 ** 3, "adjoint_step": 12 * 512 ** 3},
                      "adjoint_step": ["k_s3d_adj", "k_unpack_add"],
                      "bench": "python3 bench.py --workload stencil3d"},
}


def traffic_summary(name, fetch_dir, write_dir, cal_fetch_dir, cal_write_dir):
    """HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE runs
    (KiB per dispatch), each scaled by what the same counter reads for the
    built-in copy of known size (--workload copy_calib: 256 MiB read and 256
    MiB written per launch)."""
    w = TRAFFIC_WORKLOADS[name]
    n = 8192
    cf = pmc_means(cal_fetch_dir, "FETCH_SIZE")["k_copy"][0] * 1024.0
    cw = pmc_means(cal_write_dir, "WRITE_SIZE")["k_copy"][0] * 1024.0
    ff, fw = 4.0 * n * n / cf, 4.0 * n * n / cw
    fet, wri = pmc_means(fetch_dir, "FETCH_SIZE"), pmc_means(write_dir, "WRITE_SIZE")
    out = {"workload": w["workload"], "kernel_source_hash": kernel_hash(w["sources"]),
           "algorithmic_bytes_per_launch": w["bytes"], "kernels": {},
           "copy_calibration": {"fetch_factor": ff, "write_factor": fw,
                                "fetch_kib_per_dispatch": cf / 1024.0, "write_kib_per_dispatch": cw / 1024.0}}
    for k in sorted(set(fet) & set(wri)):
        if not k.startswith("k_") or k.startswith(("k_runs", "k_tail", "k_gdef", "k_band", "k_heads", "k_compact", "k_init",
                                                        "k_mat", "k_bcast")):
            continue
        hb = fet[k][0] * 1024.0 * ff + wri[k][0] * 1024.0 * fw
        rec = {"fetch_kib_per_dispatch": fet[k][0], "write_kib_per_dispatch": wri[k][0],
               "dispatches": [fet[k][1], wri[k][1]], "hbm_bytes_per_launch": hb}
        alg = w["bytes"].get(k.split("<")[0])
        if alg:
            rec["traffic_over_algorithmic"] = hb / alg
        out["kernels"][k] = rec
    if "adjoint_step" in w:
        parts = [k for k in out["kernels"] if k.split("<")[0] in w["adjoint_step"]]
        if len(parts) == len(w["adjoint_step"]):
            hb = sum(out["kernels"][k]["hbm_bytes_per_launch"] for k in parts)
            out["kernels"]["adjoint_step"] = {"hbm_bytes_per_launch": hb, "of": parts,
                                              "traffic_over_algorithmic": hb / w["bytes"]["adjoint_step"]}
    cmd = w["bench"]
    out["commands"] = [f"rocprofv3 --pmc FETCH_SIZE -f csv -d OUT/fetch -o t -- {cmd}",
                       f"rocprofv3 --pmc WRITE_SIZE -f csv -d OUT/write -o t -- {cmd}",
                       "rocprofv3 --pmc FETCH_SIZE -f csv -d OUT/cal_fetch -o t -- python3 bench.py --workload "
                       "copy_calib --steps 20 --warmup 3",
                       "rocprofv3 --pmc WRITE_SIZE -f csv -d OUT/cal_write -o t -- python3 bench.py --workload "
                       "copy_calib --steps 20 --warmup 3",
                       f"python3 bench.py --traffic {name} OUT/fetch OUT/write OUT/cal_fetch OUT/cal_write"]
    return out


def stencil_kernel_name(st, one, strip, op):
    """Name (as the profiler prints it, without spaces) of the 2-D stencil
    kernel the last call launched, from the shape in the runtime's stats."""
    rows, waves, order = st["stencil_rows"], st["stencil_waves"], st["stencil_order"]
    if rows >= 32:
        return f"{strip}<{rows},{op}>"
    if waves == 4:
        if st["stencil_vec"] == 2:
            return f"k_stack_a<{rows},{op}>"
        return f"k_stack<{rows},{op},{'true' if st['stencil_vec'] else 'false'}>"
    tri = ",false" if op == 0 else ""
    return f"{one}<{rows}{tri},{'true' if order else 'false'}>"


def setup_jacobi_large(rt, hd, n, declare=True):
    from workloads import jacobi_inputs
    A0, B0 = jacobi_inputs(n, 2)
    A, B = rt.create(A0), rt.create(B0)
    p = rt.partition(hd.BLOCK, (n, n), ndev=16)
    offs = [(0, 0), (0, -1), (0, 1), (-1, 0), (1, 0)]
    for k in ("jacAB", "jacBA") if declare else ():
        rt.kernel(k, hd.K_JACOBI2D)
        rt.set_offsets(k, 1, 0, offs)
        rt.set_offsets(k, 0, 1, [(0, 0)])
    rt.write(A, A0, p)
    rt.write(B, B0, p)
    del A0, B0
    return A, B, p


def jacobi64_window(b0, r0, r1, iters):
    """FP64 Jacobi (Sec. 5.1 update on interior cells, boundary copied) of
    the global array b0 after `iters` steps, exact on rows [r0, r1): the
    window carries `iters` extra rows on each side (each step invalidates one
    row at a window edge that is not the array's)."""
    n0, n1 = b0.shape
    w0, w1 = max(0, r0 - iters), min(n0, r1 + iters)
    W = b0[w0:w1].astype(np.float64)
    for _ in range(iters):
        new = W.copy()
        lo = max(1, w0 + 1) - w0          # first window row with both neighbours in the window
        hi = min(n0 - 2, w1 - 2) - w0     # last such row (inclusive)
        if hi >= lo:
            new[lo:hi + 1, 1:n1 - 1] = (((W[lo:hi + 1, 0:n1 - 2] + W[lo:hi + 1, 2:n1]) + W[lo - 1:hi, 1:n1 - 1])
                                        + W[lo + 1:hi + 2, 1:n1 - 1]) * 0.25
        W = new
    return W[r0 - w0:r1 - w0]


def err_stats(x, ref):
    d = np.asarray(x, np.float64) - ref
    return {"max_abs": float(np.max(np.abs(d))), "rms": float(np.sqrt(np.mean(d * d)))}


def fp64_error_jacobi(hd, stream, n, iters=(10, 100), band=(2016, 2080)):
    """The GPU's FP32 Jacobi (jacobi_large layout: 16 devices, 4 x 4 blocks)
    after 10 and 100 steps against FP64 on a band of rows across a block
    boundary (the band's dependence cone computed in FP64 with numpy)."""
    from workloads import jacobi_inputs
    rt = hd.Runtime(stream=stream)
    A, B, p = setup_jacobi_large(rt, hd, n)
    _, B0 = jacobi_inputs(n, 2)
    r0, r1 = band
    res = {"rows": [r0, r1], "iterations": list(iters)}
    done = 0
    for k in iters:
        while done < k:
            if done % 2 == 0:
                rt.apply("jacAB", p, [A, B])
            else:
                rt.apply("jacBA", p, [B, A])
            done += 1
        got = rt.read(A if k % 2 == 1 else B, p)[r0:r1]
        res[str(k)] = err_stats(got, jacobi64_window(B0, r0, r1, k))
    rt.close()
    return res


def s3d64_adjoint(u0, c, T, w):
    """FP64 reverse mode of L = sum(w * u_T) for T 7-point steps (interior
    cells updated, boundary copied): dL/du0 and dL/dc (numpy, whole array)."""
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    n = u0.shape[0]
    I = (slice(1, n - 1),) * 3

    def sh(a, o):
        return a[tuple(slice(1 + d, n - 1 + d) for d in o)]

    us = [u0.astype(np.float64)]
    for _ in range(T):
        u = us[-1]
        v = u.copy()
        acc = c[0] * u[I]
        for e in range(1, 7):
            acc = acc + c[e] * sh(u, offs[e])
        v[I] = acc
        us.append(v)
    g = w.astype(np.float64)
    gc = np.zeros(7)
    for t in reversed(range(T)):
        u = us[t]
        gi = g[I]
        for e in range(7):
            gc[e] += np.sum(gi * sh(u, offs[e]))
        gn = g.copy()
        gn[I] = 0.0
        for e in range(7):
            gn[tuple(slice(1 + d, n - 1 + d) for d in offs[e])] += c[e] * gi
        g = gn
    return g, gc


def adjoint_error_32(hd, stream):
    """Gradient of the 32^3 copy (T = 64, checkpoint every 8) through the
    differentiable stencil against the FP64 adjoint above."""
    import torch
    from paper_1809_05657_amd import autograd as ag
    from workloads import S3D_COEFFS, stencil3d_inputs
    n, T = 32, 64
    u0, w = stencil3d_inputs(n)
    coef = [float(x) for x in S3D_COEFFS]
    rt = hd.Runtime(stream=stream)
    solver = ag.Stencil3D(rt, (n, n, n), ndev=8, T=T, ckpt=8)
    dev = torch.device("cuda:0")
    solver.forward(torch.from_numpy(u0).to(dev), coef)
    g0, cb = solver.backward(torch.from_numpy(w).to(dev))
    g0 = g0.cpu().numpy().astype(np.float64)
    cb = cb.cpu().numpy()
    rt.close()
    g64, gc64 = s3d64_adjoint(u0, np.array(S3D_COEFFS, np.float64), T, w)
    return {"size": f"{n}^3, T={T}, checkpoint every 8",
            "grad_u0_rel_l2": float(np.linalg.norm(g0 - g64) / np.linalg.norm(g64)),
            "grad_coef_max_rel": float(np.max(np.abs(cb - gc64) / np.abs(gc64)))}


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


def bench_matmul(hd, rt, steps, warmup):
    """matmul: C = A.B, 4096^2 fp32, 8 row partitions; the first call gathers
    B (448 MiB through pack/unpack), later calls communicate nothing."""
    from workloads import matmul_inputs
    n = 4096
    a0, b0 = matmul_inputs(n, 3)
    A, B, Cc = rt.create(a0), rt.create(b0), rt.create(shape=(n, n))
    p = rt.partition(hd.ROW, (n, n), ndev=8)
    rt.kernel("gemm", hd.K_MATMUL)
    rt.set_offsets("gemm", 0, 0, [(0, "*")])
    rt.set_offsets("gemm", 1, 0, [("*", 0)])
    rt.set_offsets("gemm", 2, 1, [(0, 0)])
    rt.write(A, a0, p)
    rt.write(B, b0, p)
    rt.sync()
    rt.profile(0xF)
    rt.profile_read()
    rt.apply("gemm", p, [A, B, Cc])
    rt.sync()
    first = rt.profile_read()
    st = rt.stats()
    for _ in range(warmup):
        rt.apply("gemm", p, [A, B, Cc])
    rt.sync()
    rt.profile(1 << 3)
    rt.profile_read()
    t0 = time.perf_counter()
    for _ in range(steps):
        rt.apply("gemm", p, [A, B, Cc])
    rt.sync()
    dt = time.perf_counter() - t0
    kms, kc = rt.profile_read()["kernel"]
    rt.profile(0)
    # FP64 error of C on 64 evenly spaced rows (bound: K 2^-24 (|A||B|)_ij)
    rows = np.linspace(0, n - 1, 64).astype(np.int64)
    cg = rt.read(Cc, p)[rows].astype(np.float64)
    ref = a0[rows].astype(np.float64) @ b0.astype(np.float64)
    bound = n * 2.0 ** -24 * (np.abs(a0[rows]).astype(np.float64) @ np.abs(b0).astype(np.float64))
    fp64 = err_stats(cg, ref)
    fp64["max_over_bound"] = float(np.max(np.abs(cg - ref) / bound))
    fp64["rows_sampled"] = 64
    flops = 2.0 * n ** 3
    tf = flops / (kms / kc * 1e-3) / 1e12
    moved = st["last_bytes"]
    pk = first["pack"][0]
    return {"metric": METRIC, "value": steps / dt, "unit": "steps/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": dt * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "matmul: C=A.B 4096x4096 fp32 U[-1,1), 8 row partitions, use A (0,*), "
                                   "B (*,0), def C (0,0)", "first_step_messages": st["last_messages"],
                       "first_step_bytes": moved, "first_step_ms": sum(v[0] for v in first.values())},
            "roofline": {"bound": "mfma", "achieved": tf, "peak": 157.3, "unit": "TFLOP/s", "frac": tf / 157.3,
                         "traffic": None, "kernel": "k_mm_mfma", "avg_launch_us": kms / kc * 1e3},
            "pack_unpack": {"bytes": moved, "fused_pass_us": pk * 1e3,
                            "GBps": 4 * moved / (pk * 1e-3) / 1e9 if pk else None,
                            "frac_hbm": (4 * moved / (pk * 1e-3) / 1e9) / HBM_PEAK_GBS if pk else None},
            "fp64_error": fp64}


def bench_2mm(hd, rt, steps, warmup):
    """2MM (Sec. 5.1): D = A.B then E = C.D, 4096^2 fp32, 8 partitions, ROW
    and then COL; one iteration = both products.  Reports iterations/s and
    the bytes moved per iteration under each partitioning."""
    from workloads import matmul_inputs
    n, P = 4096, 8
    a0, b0 = matmul_inputs(n, 3)
    c0, _ = matmul_inputs(n, 6)
    res = {}
    for name, lay in (("row", hd.ROW), ("col", hd.COL)):
        A, B, Cm = rt.create(a0), rt.create(b0), rt.create(c0)
        D, E = rt.create(shape=(n, n)), rt.create(shape=(n, n))
        p = rt.partition(lay, (n, n), ndev=P)
        k1, k2 = f"mm1_{name}", f"mm2_{name}"
        for k in (k1, k2):
            rt.kernel(k, hd.K_MATMUL)
            rt.set_offsets(k, 0, 0, [(0, "*")])
            rt.set_offsets(k, 1, 0, [("*", 0)])
            rt.set_offsets(k, 2, 1, [(0, 0)])
        for X, x0 in ((A, a0), (B, b0), (Cm, c0)):
            rt.write(X, x0, p)
        rt.sync()
        moved = []

        def it(track):
            for k, args in ((k1, [A, B, D]), (k2, [Cm, D, E])):
                rt.apply(k, p, args)
                if track:
                    rt.sync()
                    moved.append(rt.stats()["last_bytes"])

        it(True)
        it(True)
        for _ in range(warmup):
            it(False)
        rt.sync()
        t0 = time.perf_counter()
        for _ in range(steps):
            it(False)
        rt.sync()
        dt = time.perf_counter() - t0
        res[name] = {"iterations_per_s": steps / dt, "ms_per_iteration": dt * 1e3 / steps,
                     "first_iteration_bytes": moved[0] + moved[1], "steady_iteration_bytes": moved[2] + moved[3],
                     "tflops": 2 * 2.0 * n ** 3 * steps / dt / 1e12}
    r, c = res["row"], res["col"]
    vol = lambda d, k: d["first_iteration_bytes"] + (k - 1) * d["steady_iteration_bytes"]
    return {"metric": "2mm iterations/s", "value": r["iterations_per_s"], "unit": "iterations/s", "n_gpus": 1,
            "steps": steps, "warmup": warmup, "ms_per_step": r["ms_per_iteration"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"2mm: D=A.B, E=C.D, {n}x{n} fp32 U[-1,1), {P} partitions, GEMM clauses; "
                                   "value = ROW partitions", "n": n, "partitions": P},
            "row": r, "col": c,
            "volume_ratio_row_over_col_100_iterations": vol(r, 100) / vol(c, 100)}


def bench_conv2d(hd, rt, steps, warmup):
    """conv2d: the 3 x 3 convolution of Sec. 5.1 on 8192^2 fp32, 16 devices
    (4 x 4 blocks), use = the 3 x 3 window, def = own block.  Ping-pong
    steps (A = conv(B), B = conv(A)) exchange 48 strips and 36 corner cells
    every step; the paper's form (A = conv(B) repeated, B never redefined)
    communicates once and is timed second."""
    from workloads import CONV9_WEIGHTS, jacobi_inputs
    n = 8192
    A0, B0 = jacobi_inputs(n, 2)
    A, B = rt.create(A0), rt.create(B0)
    p = rt.partition(hd.BLOCK, (n, n), ndev=16)
    offs = [(di, dj) for di in (-1, 0, 1) for dj in (-1, 0, 1)]
    for k in ("convAB", "convBA"):
        rt.kernel(k, hd.K_CONV2D9)
        rt.set_offsets(k, 1, 0, offs)
        rt.set_offsets(k, 0, 1, [(0, 0)])
    rt.write(A, A0, p)
    rt.write(B, B0, p)
    del A0, B0
    w = [float(x) for x in CONV9_WEIGHTS]

    def pp(i):
        if i % 2 == 0:
            rt.apply("convAB", p, [A, B], w)
        else:
            rt.apply("convBA", p, [B, A], w)

    for i in range(warmup):
        pp(i)
    rt.sync()
    rt.profile(0)
    rt.profile_read()
    t0 = time.perf_counter()
    for i in range(steps):
        if i % KERNEL_SAMPLE == 0:
            rt.profile(1 << 3)
        pp(warmup + i)
        if i % KERNEL_SAMPLE == 0:
            rt.profile(0)
    rt.sync()
    dt = time.perf_counter() - t0
    kms, kcnt = rt.profile_read()["kernel"]
    st = rt.stats()
    # the paper's form: B fixed, so only the first of these calls moves data
    for _ in range(3):
        rt.apply("convAB", p, [A, B], w)
    rt.sync()
    t1 = time.perf_counter()
    for _ in range(steps):
        rt.apply("convAB", p, [A, B], w)
    rt.sync()
    dt1 = time.perf_counter() - t1
    st1 = rt.stats()
    byts = 2 * 4 * n * n
    avg_ms = kms / max(kcnt, 1)
    ach = byts / (avg_ms * 1e-3) / 1e9
    kname = stencil_kernel_name(st, "k_conv1", "k_strip", 2)
    return {"metric": "conv2d steps/s", "value": steps / dt, "unit": "steps/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": dt * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"conv2d: 3x3 convolution {n}x{n} fp32, 16 logical devices (4x4 blocks), "
                                   "use = 3x3 window, def = own block, ping-pong", "n": n, "partitions": 16,
                       "messages_per_step": st["last_messages"], "halo_bytes_per_step": st["last_bytes"]},
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "traffic": None, "kernel": kname, "bytes_per_launch": byts,
                         "avg_launch_us": avg_ms * 1e3},
            "paper_form": {"steps_per_s": steps / dt1, "ms_per_step": dt1 * 1e3 / steps,
                           "messages_last_step": st1["last_messages"]}}


def bench_batched(hd, rt, steps, warmup):
    """batched: 64 arrays (sides log-uniform in [512, 4096], 2-32 irregular
    row partitions, 5-point or lower-triangular), ping-pong; plain per-call
    steps vs one persistent graph-replayed launch per step."""
    sys.path.insert(0, ROOT)
    from workloads import programs as prog
    from workloads import batched_instance
    inst = batched_instance(seed=4)
    arrs = prog.batched_arrays(rt, inst)
    cells = 0
    for m in inst:
        H, W = m["shape"]
        cells += H * W if m["kind"] == 0 else H * (H + 1) // 2
    bytes_step = 8 * cells

    def plain(i):
        for j, (A, B, p, kind) in enumerate(arrs):
            if i % 2 == 0:
                rt.apply(f"b{j}AB", p, [A, B])
            else:
                rt.apply(f"b{j}BA", p, [B, A])

    for i in range(2):
        plain(i)
    rt.sync()
    t0 = time.perf_counter()
    for i in range(steps):
        plain(i)
    rt.sync()
    t_plain = (time.perf_counter() - t0) / steps
    ids = []
    for even in (True, False):
        rt.batch_begin()
        for j, (A, B, p, kind) in enumerate(arrs):
            if even:
                rt.apply(f"b{j}AB", p, [A, B])
            else:
                rt.apply(f"b{j}BA", p, [B, A])
        ids.append(rt.batch_end())
    cfg = rt.batch_autotune(ids, reps=2)
    for i in range(warmup):
        rt.batch_run(ids[i % 2])
    rt.sync()
    rt.profile(1 << 3)
    rt.profile_read()
    t0 = time.perf_counter()
    for i in range(steps):
        rt.batch_run(ids[i % 2])
    rt.sync()
    t_batch = (time.perf_counter() - t0) / steps
    kms, kc = rt.profile_read()["kernel"]
    rt.profile(0)
    phases = rt.batch_phase_us(ids[(steps - 1) % 2])
    ach = bytes_step / (kms / kc * 1e-3) / 1e9
    return {"metric": METRIC, "value": 1.0 / t_batch, "unit": "steps/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": t_batch * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "batched: 64 arrays, sides log-uniform [512,4096], 2-32 irregular row "
                                   "partitions, 5-point or lower-triangular stencil, ping-pong",
                       "cells": cells, "plain_steps_per_s": 1.0 / t_plain, "batched_over_plain": t_plain / t_batch,
                       # rows per wave; tile shape 0: one wave, tiles down columns first, 1: one
                       # wave, along rows, 2: four waves stacked (4 x rows per tile)
                       "autotuned_rows": (cfg >> 8) & 255, "autotuned_tile_shape": cfg & 255,
                       "autotuned_workgroups_per_cu": cfg >> 16,
                       # phases of the persistent launch up to the message table (device-clock stamps
                       # of its workgroup 0); the rest of the step (pack + unpack and GDEF update in the
                       # same launch, then the user-kernel launch) is the step's launch time minus these
                       "batch_phases_us": dict(zip(("runs", "band_flags", "band_scan", "heads", "compact_scan",
                                                    "compact_prefix", "compact_write"), phases)),
                       "pack_gdef_and_kernels_us": kms / kc * 1e3 - sum(phases[:7])},
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "traffic": None, "kernel": "k_batch + k_batch_tiles (one graph)",
                         "bytes_per_launch": bytes_step, "avg_launch_us": kms / kc * 1e3}}


def bench_stencil3d(hd, rt, steps, warmup, n=512, T=64, ckpt=8):
    """stencil3d: 7-point stencil n^3 fp32, 2x2x2 blocks; a full
    differentiable pass (T forward steps with checkpoints, then the
    checkpointed backward: recompute + adjoint steps)."""
    import torch
    from paper_1809_05657_amd import autograd as ag
    from workloads import S3D_COEFFS, stencil3d_inputs
    u0, w = stencil3d_inputs(n)
    solver = ag.Stencil3D(rt, (n, n, n), ndev=8, T=T, ckpt=ckpt)
    dev = torch.device("cuda:0")
    u0_t, w_t = torch.from_numpy(u0).to(dev), torch.from_numpy(w).to(dev)
    coef = [float(c) for c in S3D_COEFFS]
    solver.forward(u0_t, coef)
    solver.backward(w_t)
    rt.profile(0x1F)
    rt.profile_read()
    t0 = time.perf_counter()
    solver.forward(u0_t, coef)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phf = rt.profile_read()
    solver.backward(w_t)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    phb = rt.profile_read()
    rt.profile(0)
    ph = {k: (phf[k][0] + phb[k][0], phf[k][1] + phb[k][1]) for k in phf}
    # the same pass with the plan cache on (Sec. 4.2), reported beside: the
    # forward and recomputation steps repeat their calls, so their
    # derivations are skipped; the adjoint steps derive as before
    rt.set_plan_cache(True)
    solver.forward(u0_t, coef)
    solver.backward(w_t)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    solver.forward(u0_t, coef)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    solver.backward(w_t)
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    rt.set_plan_cache(False)
    cells = n ** 3
    fwd_bytes = 8 * cells   # read u once, write the next state once
    adj_bytes = 12 * cells  # read the cotangent and the state, write the cotangent
    kms, kc = phf["kernel"]
    ams, ac = phb["adjoint"]
    fwd_us = kms / max(kc, 1) * 1e3
    adj_us = ams / max(ac, 1) * 1e3
    adj_gbs = adj_bytes / (adj_us * 1e-6) / 1e9 if ac else None
    fwd_gbs = fwd_bytes / (fwd_us * 1e-6) / 1e9 if kc else None
    return {"metric": METRIC, "value": 1.0 / (t2 - t0), "unit": "passes/s", "n_gpus": 1, "steps": 1,
            "warmup": 1, "ms_per_step": (t2 - t0) * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"stencil3d: 7-point {n}^3 fp32, 8 devices (2x2x2), T={T}, checkpoint every "
                                   f"{ckpt}; forward + checkpointed adjoint", "forward_ms": (t1 - t0) * 1e3,
                       "backward_ms": (t2 - t1) * 1e3,
                       "plan_cache": {"passes_per_s": 1.0 / (t5 - t3), "forward_ms": (t4 - t3) * 1e3,
                                      "backward_ms": (t5 - t4) * 1e3}},
            "phases_us": {k: (v[0] / max(v[1], 1)) * 1e3 for k, v in ph.items()},
            "roofline": {"bound": "hbm", "achieved": adj_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": adj_gbs / HBM_PEAK_GBS if adj_gbs else None,
                         "traffic": committed_traffic("stencil3d_512", "adjoint_step", S3D_SOURCES),
                         "kernel": "adjoint step (k_s3d_adj, k_unpack_add)",
                         "bytes_per_launch": adj_bytes, "avg_launch_us": adj_us},
            "forward_kernel": {"kernel": "k_s3d", "bytes_per_launch": fwd_bytes, "avg_launch_us": fwd_us,
                               "GBps": fwd_gbs, "frac": fwd_gbs / HBM_PEAK_GBS if fwd_gbs else None,
                               "traffic": committed_traffic("stencil3d_512", "k_s3d", S3D_SOURCES)}}


def bench_copy_calib(hd, rt, steps, warmup):
    """A plain copy of known size (8192 x 8192 fp32, one logical device, no
    communication) through the built-in copy kernel: the reference for
    scaling HBM traffic counters (256 MiB read + 256 MiB written per launch)."""
    n = 8192
    X, Y = rt.create(shape=(n, n)), rt.create(shape=(n, n))
    p = rt.partition(hd.ROW, (n, n), ndev=1)
    rt.kernel("cp", hd.K_COPY)
    rt.set_offsets("cp", 1, 0, [(0, 0)])
    rt.set_offsets("cp", 0, 1, [(0, 0)])
    rt.write(X, np.ones((n, n), np.float32), p)
    rt.write(Y, np.zeros((n, n), np.float32), p)
    for _ in range(warmup):
        rt.apply("cp", p, [Y, X])
    rt.sync()
    rt.profile(1 << 3)
    rt.profile_read()
    for _ in range(steps):
        rt.apply("cp", p, [Y, X])
    rt.sync()
    kms, kc = rt.profile_read()["kernel"]
    rt.profile(0)
    b = 2 * 4 * n * n
    return {"workload": "copy_calib", "bytes_per_launch": b, "avg_launch_us": kms / kc * 1e3,
            "GBps": b / (kms / kc * 1e-3) / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--traffic", nargs=5, metavar=("NAME", "FETCH", "WRITE", "CAL_FETCH", "CAL_WRITE"),
                    help="summarise rocprofv3 FETCH_SIZE / WRITE_SIZE folders into profiles/NAME_traffic.json "
                         "(no GPU needed)")
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the jacobi_large line (no FP64-error, matmul, batched and adjoint legs)")
    ap.add_argument("--workload", default="jacobi_large",
                    choices=["jacobi_large", "matmul", "2mm", "conv2d", "batched", "stencil3d", "copy_calib"])
    args = ap.parse_args()
    if args.traffic:
        name = args.traffic[0]
        out = traffic_summary(*args.traffic)
        with open(os.path.join(ROOT, "profiles", f"{name}_traffic.json"), "w") as fh:
            json.dump(out, fh, indent=1)
        print(json.dumps({k: v.get("traffic_over_algorithmic") for k, v in out["kernels"].items()}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the runtime runs the ApplyKernel path on one GPU only (the logical devices are "
              "partitions of one MI355X); multi-GPU runs are not supported.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1809_05657_amd as hd

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    rt = hd.Runtime(stream=stream.cuda_stream)
    if args.workload != "jacobi_large":
        fn = {"matmul": bench_matmul, "2mm": bench_2mm, "conv2d": bench_conv2d, "batched": bench_batched, "stencil3d": bench_stencil3d,
              "copy_calib": bench_copy_calib}[args.workload]
        out = fn(hd, rt, args.steps, args.warmup)
        rt.close()
        print(json.dumps(out), flush=True)
        return
    n = args.n
    # tile-shape calibration: on the first calls of a box geometry the runtime
    # times its candidate stencil tile shapes (TUNE_CALLS calls), then keeps
    # the fastest for every plan with the same boxes.  Those calls run on a
    # scratch pair of arrays of the same shape and partition, so that the
    # warm-up and the timed steps below all run the chosen shape whatever W.
    S_a, S_b, s_p = setup_jacobi_large(rt, hd, n)
    for i in range(TUNE_CALLS):
        rt.apply("jacAB" if i % 2 == 0 else "jacBA", s_p, [S_a, S_b] if i % 2 == 0 else [S_b, S_a])
    rt.sync()
    A, B, p = setup_jacobi_large(rt, hd, n, declare=False)

    def step(i):
        if i % 2 == 0:
            rt.apply("jacAB", p, [A, B])
        else:
            rt.apply("jacBA", p, [B, A])

    for i in range(args.warmup):
        step(i)
    rt.sync()
    torch.cuda.synchronize()
    # timed region: the stencil launches of every KERNEL_SAMPLE-th step carry
    # an event pair on the data stream (bit 3 of the runtime's phase timing);
    # an event record costs a few microseconds of the step, so not every
    # launch is bracketed
    rt.profile(0)
    rt.profile_read()
    t0 = time.perf_counter()
    for i in range(args.steps):
        if i % KERNEL_SAMPLE == 0:
            rt.profile(1 << 3)
        step(args.warmup + i)
        if i % KERNEL_SAMPLE == 0:
            rt.profile(0)
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
    # the same steps with the plan cache on (Sec. 4.2): reported beside the
    # headline, which derives the communication sets on every step
    rt.set_plan_cache(True)
    base = args.warmup + args.steps + 20
    for i in range(10):
        step(base + i)
    rt.sync()
    h0 = rt.stats()
    t1 = time.perf_counter()
    for i in range(args.steps):
        step(base + 10 + i)
    rt.sync()
    dtc = time.perf_counter() - t1
    h1 = rt.stats()
    rt.profile(0xF)
    for i in range(20):
        step(base + 10 + args.steps + i)
    rt.sync()
    phc = rt.profile_read()
    rt.profile(0)
    rt.set_plan_cache(False)
    ms_step = dt * 1e3 / args.steps
    bytes_kernel = 2 * 4 * n * n  # read B once, write A once per step
    avg_kernel_ms = kms / max(kcnt, 1)
    achieved = bytes_kernel / (avg_kernel_ms * 1e-3) / 1e9
    # pack and unpack run as one pass (phase "pack"); algorithmic bytes are
    # those of both: read + write for the pack and again for the unpack
    pk_ms = ph["pack"][0] / max(ph["pack"][1], 1)
    moved = st["last_bytes"]
    kname = stencil_kernel_name(st, "k_jacobi1", "k_strip", 0)
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
                   "halo_bytes_per_step": moved,
                   "tile_shape_calibration": f"{TUNE_CALLS} calls on a scratch pair of arrays of the same shape "
                                             "and partition before the warm-up"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": committed_traffic("jacobi2d_8192", kname),
                     "kernel": kname, "bytes_per_launch": bytes_kernel,
                     "avg_launch_us": avg_kernel_ms * 1e3,
                     # the same kernel's average in the committed rocprofv3 summary of this workload
                     "profile_avg_us": committed_kernel_avg("jacobi2d_8192", kname)},
        "step_hbm_frac": bytes_kernel / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "phases_us": {k: (v[0] / max(v[1], 1)) * 1e3 for k, v in ph.items()},
        "pack_unpack": {"bytes": moved, "fused_pass_us": pk_ms * 1e3,
                        "GBps": 4 * moved / max(pk_ms * 1e-3, 1e-12) / 1e9},
        "plan_cache": {"steps_per_s": args.steps / dtc, "ms_per_step": dtc * 1e3 / args.steps,
                       "hits": h1["cache_hits"] - h0["cache_hits"],
                       "misses": h1["cache_misses"] - h0["cache_misses"],
                       "phases_us": {k: (v[0] / max(v[1], 1)) * 1e3 for k, v in phc.items()}},
    }
    rt.close()
    if not args.headline_only:
        sp = stream.cuda_stream
        # the metric's other legs: FP64 errors, matmul, batched vs plain, adjoint
        out["fp64_error"] = {"jacobi_8192": fp64_error_jacobi(hd, sp, n)}
        rt = hd.Runtime(stream=sp)
        m = bench_matmul(hd, rt, 10, 2)
        rt.close()
        out["fp64_error"]["matmul_4096"] = m.pop("fp64_error")
        out["matmul"] = {"steps_per_s": m["value"], "ms_per_step": m["ms_per_step"], "config": m["config"],
                         "roofline": m["roofline"], "pack_unpack_first_step": m["pack_unpack"]}
        rt = hd.Runtime(stream=sp)
        b = bench_batched(hd, rt, 20, 5)
        rt.close()
        out["batched"] = {"steps_per_s": b["value"], "ms_per_step": b["ms_per_step"],
                          "plain_steps_per_s": b["config"]["plain_steps_per_s"],
                          "batched_over_plain": b["config"]["batched_over_plain"], "roofline": b["roofline"],
                          "config": {k: v for k, v in b["config"].items() if k not in ("plain_steps_per_s",
                                                                                  "batched_over_plain")}}
        rt = hd.Runtime(stream=sp)
        a = bench_stencil3d(hd, rt, 1, 1)
        rt.close()
        out["adjoint"] = {"passes_per_s": a["value"], "ms_per_pass": a["ms_per_step"], "config": a["config"],
                          "phases_us": a["phases_us"], "roofline": a["roofline"],
                          "forward_kernel": a["forward_kernel"], "fp64_check": adjoint_error_32(hd, sp)}
    if not args.no_cpu_baseline:
        import oracle as O
        sps, secs = cpu_baseline_jacobi(n, args.cpu_steps)
        out["cpu_baseline"] = {"value": sps, "unit": "steps/s", "cores": O.threads(), "kind": "oracle",
                               "sample": f"{args.cpu_steps} ApplyKernel step(s) of jacobi_large ({n}x{n}, 16 "
                                         f"devices) after setup, C oracle with OpenMP, {secs:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
