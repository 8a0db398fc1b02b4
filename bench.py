"""Benchmark: one H-matrix-vector product per step on one MI355X.

Workload (default): 2D uniform 1024 x 1024 grid in [0,1]^2 (N = 2^20), leaf 64,
log kernel -log|x-y|/(2 pi) with unit diagonal, weak admissibility, rank-32
factors from randomized SVD (oversampling 10) computed in an untimed setup,
one RHS x ~ N(0,1). A step is one full y = K x on the GPU: V-phase, partial
reduction and z routing, U-phase plus dense near field. Inputs are resident
in HBM before timing starts.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="c2", choices=["c1", "c2"])
    ap.add_argument("--method", default=None, help="factor method override (rsvd, random, svd)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp16", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-c3", action="store_true", help="skip the multi-RHS (3D, 64 RHS) leg")
    ap.add_argument("--c3-steps", type=int, default=20)
    ap.add_argument("--no-c4", action="store_true", help="skip the batched (256 matrices) leg")
    ap.add_argument("--c4-steps", type=int, default=20)
    ap.add_argument("--c4-members", type=int, default=256)
    ap.add_argument("--c4-method", default="rsvd",
                    help="factors of the batched members: rsvd (kernel blocks, randomized SVD) or random fills")
    ap.add_argument("--no-c5", action="store_true", help="skip the large 3D (128^3, 128 RHS) storage-form leg")
    ap.add_argument("--c5-steps", type=int, default=5)
    ap.add_argument("--c3-forms", default="fp32,fp16,bf16", help="storage forms of the c3 leg")
    ap.add_argument("--c5-forms", default="fp32,fp16,fp8,fp8_f16d", help="storage forms of the c5 leg")
    ap.add_argument("--no-s2", action="store_true", help="skip the standard-admissibility 2D (1024^2, r=4) leg")
    ap.add_argument("--no-s3", action="store_true", help="skip the standard-admissibility 3D (64^3, r=4) leg")
    ap.add_argument("--s-steps", type=int, default=20)
    ap.add_argument("--no-transpose", action="store_true", help="skip the transpose-product timing on c2")
    ap.add_argument("--no-h2", action="store_true", help="skip the H^2-variant leg (2D 1024^2, rank 32)")
    ap.add_argument("--no-compress", action="store_true",
                    help="skip the timing of the GPU construction of the factors (hmat_compress) for c2 and c3")
    return ap.parse_args()


def time_matvecs(h, xd, yd, steps, warmup, stream, k=1):
    import torch

    import paper_2008_12441_amd as hm

    n = h.n
    for _ in range(warmup):
        hm.hmat_matvec(h.handle, k, 1.0, xd.data_ptr(), n, 0.0, yd.data_ptr(), n, stream.cuda_stream)
    torch.cuda.synchronize()
    hm.hmat_set_timing(h.handle, True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        hm.hmat_matvec(h.handle, k, 1.0, xd.data_ptr(), n, 0.0, yd.data_ptr(), n, stream.cuda_stream)
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    phase_ms, calls = hm.hmat_get_timing(h.handle)
    hm.hmat_set_timing(h.handle, False)
    assert calls == steps
    return total_ms / steps, [m / steps for m in phase_ms]


def probe_bandwidth(stream, nbytes=4 << 30, reps=5):
    import torch

    import paper_2008_12441_amd as hm

    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty(65536, dtype=torch.float32, device="cuda")
    hm.hmat_probe_bandwidth(src.data_ptr(), dst.data_ptr(), nbytes, 0, stream.cuda_stream)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(reps):
        hm.hmat_probe_bandwidth(src.data_ptr(), dst.data_ptr(), nbytes, 0, stream.cuda_stream)
    t1.record(stream)
    torch.cuda.synchronize()
    read_gbps = nbytes * reps / (t0.elapsed_time(t1) * 1e-3) / 1e9
    # one copy of known size: the calibration point for hardware byte counters
    half = nbytes // 2
    cpy = torch.empty(half // 4, dtype=torch.float32, device="cuda")
    t0.record(stream)
    hm.hmat_probe_bandwidth(src.data_ptr(), cpy.data_ptr(), half, 1, stream.cuda_stream)
    t1.record(stream)
    torch.cuda.synchronize()
    copy_gbps = 2 * half / (t0.elapsed_time(t1) * 1e-3) / 1e9
    del src, dst, cpy
    torch.cuda.empty_cache()
    return read_gbps, copy_gbps


SV_SOURCES = ("hmat_kernels.hip", "hmat_sv_device.h", "hmat_device_common.h", "hmat_internal.h")


MR_SOURCES = ("hmat_mr_kernels.hip", "hmat_mr_device.h", "hmat_device_common.h", "hmat_internal.h")


def kernel_source_digest(sources=SV_SOURCES):
    """First 16 hex digits of the sha256 over the sources of a set of kernels."""
    import hashlib

    h = hashlib.sha256()
    for name in sources:
        h.update(open(os.path.join(ROOT, "paper_2008_12441_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_key):
    """HBM bytes per launch from the committed counter summary, or None when the
    kernel source changed after the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "c2_fp32_hbm_traffic.json")
    try:
        prof = json.load(open(path))
        digest = kernel_source_digest()
    except (OSError, ValueError):
        return None
    if prof.get("kernel") != kernel_key or prof.get("kernel_source_sha256_16") != digest:
        return None
    return int(prof["traffic_bytes_per_launch"])


def host_cpu():
    """Model name, sockets and logical CPUs of this host (from /proc/cpuinfo)."""
    model, sockets, logical = None, set(), 0
    try:
        for line in open("/proc/cpuinfo"):
            key, _, val = line.partition(":")
            key = key.strip()
            if key == "model name" and model is None:
                model = val.strip()
            elif key == "physical id":
                sockets.add(val.strip())
            elif key == "processor":
                logical += 1
    except OSError:
        pass
    return {"model": model, "sockets": len(sockets) or None, "logical_cpus": logical or None,
            "affinity_cpus": len(os.sched_getaffinity(0))}


def mr_counters(workload):
    """HBM traffic and MFMA utilisation of the multi-RHS group kernels from the committed
    counter summary, or None once their sources changed after the counters were taken."""
    try:
        prof = json.load(open(os.path.join(ROOT, "profiles", "mr_c3_c5_counters.json")))
    except (OSError, ValueError):
        return None
    if prof.get("kernel_source_sha256_16") != kernel_source_digest(MR_SOURCES):
        return None
    return prof.get(workload)


def time_fn(fn, steps, warmup, stream):
    """Average ms of fn() over `steps` calls on `stream` (events around the loop)."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def capture_loop(fn, stream):
    """A CUDA graph of fn()'s launches on `stream` (fn issues them on the current stream)."""
    import torch

    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        fn()                                  # warm-up outside the capture
    stream.wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def run_batched(stream, steps, warmup, count=256, method="rsvd", with_oracle=True):
    """Batched workload: `count` independent H-matrices on random sub-grids (2D log
    kernel for even members, 3D 1/r kernel for odd ones, N log-uniform in [4096,
    65536], ranks uniform on {8, 16, 32}), each applied to k = 1 and then k = 16
    right-hand sides. One persistent launch over FP16 members (per-block scales)
    against per-matrix FP32 products (a host loop of hmat_matvec calls, and the
    same loop captured once in a graph and replayed, which takes the host's
    per-call cost out), with the batched FP32 and the FP16 loop beside them.
    The members' factors come from the kernels by randomized SVD (`method`
    "rsvd") or are random fills ("random", the values do not change the time).
    Errors are taken on every member and every column."""
    import ctypes

    import torch

    import paper_2008_12441_amd as hm
    from hmat_inputs import batch_problems, build_batch_member, make_rhs

    specs = batch_problems(count, seed=4)
    t0 = time.time()
    datas = []
    for i, sp in enumerate(specs):
        datas.append(build_batch_member(sp, method=method, seed=4000 + i, device="cuda", gpu_min_entries=1 << 16))
        if (i + 1) % 32 == 0:
            log(f"c4 members built ({method}): {i + 1}/{count} ({time.time() - t0:.1f} s)")
    setup_s = time.time() - t0
    descs = []
    for d in datas:
        t = d.tree
        descs.append(hm.make_descriptors(t.parent, t.begin, t.end, d.blocks.target, d.blocks.source,
                                         d.blocks.rank, d.pool, d.off_a, d.off_b))
    sum_n = int(sum(d.n for d in datas))
    elems = int(sum(d.pool.size for d in datas))
    out = {"workload": f"c4: {count} sub-grid H-matrices, 2D log / 3D 1/r kernels, N log-uniform in "
                       f"[4096, 65536] (sum {sum_n}), leaf <= 64, ranks in {{8, 16, 32}}",
           "members": count, "sum_n": sum_n, "stored_elements": elems, "factor_fill": method,
           "setup_s": round(setup_s, 1)}
    lib = hm.load_library()
    cs = stream.cuda_stream
    for k in (1, 16):
        xs_np = [make_rhs(d.n, k, 5000 + i) for i, d in enumerate(datas)]
        xs = [torch.from_numpy(np.ascontiguousarray(x.T)).cuda().T for x in xs_np]
        ys = [torch.empty((k, d.n), device="cuda").T for d in datas]
        vec_bytes = 8 * sum_n * k
        res = {"nrhs": k}
        ysave = {}
        for form in ("fp32", "fp16"):
            t1 = time.time()
            hs = [hm.HMatrix(tr, bl, storage=form, max_nrhs=k) for tr, bl, _ in descs]
            log(f"c4 k={k} {form}: {count} hmat_create in {time.time() - t1:.1f} s")
            args = [(h.handle, k, ctypes.c_float(1.0), x.data_ptr(), d.n, ctypes.c_float(0.0), y.data_ptr(), d.n)
                    for h, x, y, d in zip(hs, xs, ys, datas)]

            def loop(stream_ptr=cs):
                for a in args:
                    if lib.hmat_matvec(*a, ctypes.c_void_p(stream_ptr)) != 0:
                        raise hm.HmatError(6, hm.hmat_last_error())

            loop_ms = time_fn(loop, steps, 2, stream)
            y_loop = [y.clone() for y in ys]
            graph = capture_loop(lambda: loop(torch.cuda.current_stream().cuda_stream), stream)
            for y in ys:
                y.fill_(float("nan"))
            graph.replay()
            torch.cuda.synchronize()
            replay_ok = all(torch.equal(a, b) for a, b in zip(ys, y_loop))
            graph_ms = time_fn(graph.replay, steps, 2, stream)
            del graph, y_loop
            b = hm.HBatch(hs, [k] * len(hs))
            tuned = b.autotune(xs, ys, reps=5)
            batch_ms = time_fn(lambda: b.matvec(xs, ys), steps, warmup, stream)
            b.sync()
            info = b.info()
            ysave[form] = [y.cpu().numpy().astype(np.float64) for y in ys]
            fbytes = int(sum(h.info["factor_bytes"] for h in hs))
            dbytes = int(sum(h.info["device_factor_bytes"] for h in hs))
            res[form] = {"loop_ms": round(loop_ms, 4), "loop_graph_ms": round(graph_ms, 4),
                         "loop_graph_replay_bitwise_equal": bool(replay_ok), "batched_ms": round(batch_ms, 4),
                         "batched_GBps": round((fbytes + vec_bytes) / (batch_ms * 1e-3) / 1e9, 1),
                         "alg_bytes": fbytes + vec_bytes, "device_factor_bytes": dbytes,
                         "layout_padding": round(dbytes / fbytes, 3), "tuned": tuned,
                         "queue_items": info["num_items"], "grid": info["grid"]}
            log(f"c4 k={k} {form}: loop {loop_ms:.3f} ms, graph-captured loop {graph_ms:.3f} ms, batched "
                f"{batch_ms:.3f} ms ({res[form]['batched_GBps']} GB/s, tuned {tuned})")
            b.close()
            for h in hs:
                h.close()
            del hs, args
            torch.cuda.empty_cache()
        res["speedup_batched_fp16_vs_loop_fp32"] = round(res["fp32"]["loop_ms"] / res["fp16"]["batched_ms"], 3)
        res["speedup_batched_fp16_vs_graph_loop_fp32"] = round(res["fp32"]["loop_graph_ms"] /
                                                               res["fp16"]["batched_ms"], 3)
        res["speedup_batched_fp16_vs_batched_fp32"] = round(res["fp32"]["batched_ms"] / res["fp16"]["batched_ms"], 3)
        res["roofline_batched_fp16"] = {"bound": "hbm", "achieved": res["fp16"]["batched_GBps"],
                                        "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                        "frac": round(res["fp16"]["batched_GBps"] / HBM_PEAK_GBPS, 4)}
        if with_oracle:
            import oracle

            t1 = time.time()
            errs16, errs32 = [], []
            for i in range(count):                       # every member, every column
                ref = oracle.oracle_matvec(datas[i], xs_np[i])
                den = np.linalg.norm(ref, axis=0)
                errs16.append(float((np.linalg.norm(ysave["fp16"][i] - ref, axis=0) / den).max()))
                errs32.append(float((np.linalg.norm(ysave["fp32"][i] - ref, axis=0) / den).max()))
            res["fp16_rel_err_vs_fp64_oracle_max"] = max(errs16)
            res["fp32_rel_err_vs_fp64_oracle_max"] = max(errs32)
            res["error_sample"] = (f"all {count} members, all {k} columns: max of the relative 2-norm error, "
                                   f"FP64 oracle over the canonical FP32 factors ({method})")
            log(f"c4 k={k} oracle over {count} members: {time.time() - t1:.1f} s; fp16 err {max(errs16):.3e}, "
                f"fp32 err {max(errs32):.3e}")
        out[f"k{k}"] = res
        del xs, ys
        torch.cuda.empty_cache()
    return out


C5_ERR_COLS = list(range(0, 128, 16)) + [127]


def run_large_3d(stream, steps, warmup, with_oracle=True, forms=("fp32", "fp16", "fp8", "fp8_f16d"), method=None):
    """3D 128^3 grid (N = 2^21), 1/r kernel, rank 32, 128 RHS: the storage forms
    on the multi-RHS (MFMA) path, FP8 hi + lo U/V with BF16 dense blocks against
    FP32 on the same GPU. Errors are taken on one right-hand side of every
    16-column n-tile of the MFMA tiling (columns 0, 16, ..., 112) and on the
    last one, against the FP64 oracle over the canonical FP32 factors."""
    import torch

    import paper_2008_12441_amd as hm
    from hmat_inputs import WORKLOADS, build_workload

    w = WORKLOADS["c5"]
    t0 = time.time()
    data, x = build_workload("c5", device="cuda", method=method)
    log(f"setup c5 ({w.describe()}): {time.time() - t0:.1f} s")
    n, k = data.n, w.nrhs
    t = data.tree
    tree, blocks, keep = hm.make_descriptors(t.parent, t.begin, t.end, data.blocks.target, data.blocks.source,
                                             data.blocks.rank, data.pool, data.off_a, data.off_b)
    xd = torch.from_numpy(np.ascontiguousarray(x.T)).cuda()
    flops = 2.0 * data.pool.size * k
    vec_bytes = 2 * n * k * 4
    out = {"workload": f"c5: {w.describe()}", "nrhs": k, "alg_flops_per_step": flops,
           "stored_elements": int(data.pool.size)}
    ys = {}
    for form in forms:
        t1 = time.time()
        h = hm.HMatrix(tree, blocks, storage=form, max_nrhs=k)
        log(f"c5 {form}: hmat_create {time.time() - t1:.1f} s")
        yd = torch.empty_like(xd)
        ms, ph = time_matvecs(h, xd, yd, steps, warmup, stream, k=k)
        ys[form] = yd[C5_ERR_COLS].cpu().numpy().T.astype(np.float64)
        b = h.info["factor_bytes"] + vec_bytes
        out[form] = {"ms_per_step": round(ms, 4), "GBps": round(b / (ms * 1e-3) / 1e9, 1),
                     "TFLOPps": round(flops / (ms * 1e-3) / 1e12, 2), "alg_bytes_per_step": b,
                     "phases_ms": [round(v, 4) for v in ph]}
        log(f"c5 {form}: {ms:.3f} ms per {k}-RHS product, {out[form]['GBps']} GB/s, {out[form]['TFLOPps']} TFLOP/s")
        h.close()
        del yd
        torch.cuda.empty_cache()
    base = out["fp32"]["ms_per_step"] if "fp32" in out else None
    for form in forms:
        if base and form != "fp32":
            out[form]["speedup_vs_fp32"] = round(base / out[form]["ms_per_step"], 3)
    if "fp32" in out:
        out["roofline_fp32"] = {"bound": "mfma", "peak": 157.3, "unit": "TFLOP/s",
                                "frac": round(out["fp32"]["TFLOPps"] / 157.3, 4)}
    out["counters"] = mr_counters("c5")
    if "fp8" in out:
        out["roofline_fp8"] = {"bound": "hbm", "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                               "frac": round(out["fp8"]["GBps"] / HBM_PEAK_GBPS, 4)}
    if with_oracle:
        import oracle

        t1 = time.time()
        ref = oracle.oracle_matvec(data, x[:, C5_ERR_COLS])
        log(f"c5 oracle ({len(C5_ERR_COLS)} RHS): {time.time() - t1:.1f} s")
        for form in forms:
            e = np.linalg.norm(ys[form] - ref, axis=0) / np.linalg.norm(ref, axis=0)
            out[form]["rel_err_vs_fp64_oracle_max_col"] = float(e.max())
            out[form]["rel_err_vs_fp64_oracle_cols"] = [float(v) for v in e]
        out["error_sample"] = (f"columns {C5_ERR_COLS} (one per 16-column n-tile, and the last), FP64 oracle "
                               f"over the canonical FP32 factors")
    return out


def run_multi_rhs(stream, steps, warmup, with_oracle=True, method=None, forms=("fp32", "fp16", "bf16")):
    """3D 64^3 grid (N = 262144), 1/r kernel, rank 64, 64 RHS on MFMA: FP32 storage
    against FP16 (per-block scales) and BF16 storage, each with FP32 accumulation.
    Every result's error against the FP64 oracle over the canonical FP32 factors
    (quantisation included) and, for the 16-bit forms, over the exactly
    dequantised factors (the kernel's own arithmetic)."""
    import torch

    import paper_2008_12441_amd as hm
    from hmat_inputs import WORKLOADS, build_workload

    w = WORKLOADS["c3"]
    t0 = time.time()
    data, x = build_workload("c3", device="cuda", method=method)
    log(f"setup c3 ({w.describe()}): {time.time() - t0:.1f} s")
    n, k = data.n, w.nrhs
    t = data.tree
    tree, blocks, keep = hm.make_descriptors(t.parent, t.begin, t.end, data.blocks.target, data.blocks.source,
                                             data.blocks.rank, data.pool, data.off_a, data.off_b)
    # x and y as k contiguous columns of length n (column-major n x k)
    xd = torch.from_numpy(np.ascontiguousarray(x.T)).cuda()
    flops = 2.0 * data.pool.size * k
    vec_bytes = 2 * n * k * 4
    out = {"workload": f"c3: {w.describe()}", "nrhs": k, "alg_flops_per_step": flops}
    ys = {}
    for form in forms:
        h = hm.HMatrix(tree, blocks, storage=form, max_nrhs=k)
        yd = torch.empty_like(xd)
        ms, ph = time_matvecs(h, xd, yd, steps, warmup, stream, k=k)
        ys[form] = yd.cpu().numpy().T.astype(np.float64)
        b = h.info["factor_bytes"] + vec_bytes
        out[form] = {"ms_per_step": round(ms, 5), "GBps": round(b / (ms * 1e-3) / 1e9, 1),
                     "TFLOPps": round(flops / (ms * 1e-3) / 1e12, 2), "alg_bytes_per_step": b,
                     "phases_ms": [round(v, 5) for v in ph]}
        log(f"c3 {form}: {ms:.4f} ms per {k}-RHS product, {out[form]['GBps']} GB/s, {out[form]['TFLOPps']} TFLOP/s")
        h.close()
    out["roofline"] = {}
    if "fp32" in out:
        out["roofline"]["fp32"] = {"bound": "mfma", "peak": 157.3, "unit": "TFLOP/s",
                                   "frac": round(out["fp32"]["TFLOPps"] / 157.3, 4)}
    for form in forms:
        if form != "fp32":
            if "fp32" in out:
                out[f"{form}_speedup_vs_fp32"] = round(out["fp32"]["ms_per_step"] / out[form]["ms_per_step"], 3)
            out["roofline"][form] = {"bound": "hbm", "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                     "frac": round(out[form]["GBps"] / HBM_PEAK_GBPS, 4)}
    out["counters"] = mr_counters("c3")
    if with_oracle:
        import oracle
        from oracle.quant import dequantised

        t0 = time.time()
        ref = oracle.oracle_matvec(data, x)
        log(f"c3 oracle ({k} RHS): {time.time() - t0:.1f} s")
        for form in forms:
            e = np.linalg.norm(ys[form] - ref, axis=0) / np.linalg.norm(ref, axis=0)
            out[form]["rel_err_vs_fp64_oracle_max_col"] = float(e.max())
            if form != "fp32":
                refq = oracle.oracle_matvec(dequantised(data, form), x)
                eq = np.linalg.norm(ys[form] - refq, axis=0) / np.linalg.norm(refq, axis=0)
                out[form]["rel_err_vs_dequantised_oracle_max_col"] = float(eq.max())
        log("c3 errors: " + ", ".join(f"{f} {out[f]['rel_err_vs_fp64_oracle_max_col']:.2e}" for f in forms))
    return out


# The paper's fastest time for the same grid, rank and admissibility condition
# (Tables 1 and 2, standard-admissibility columns; distributed memory on CPU
# processes): context for the single-GPU number, not its target.
PAPER_STANDARD = {"s2": {"time_s": 6.16e-3, "processes": 512, "table": "Table 1 (2D), N = 1024^2, r = 4"},
                  "s3": {"time_s": 7.06e-3, "processes": 128, "table": "Table 2 (3D), N = 64^3, r = 4"}}


def run_standard(stream, name, steps, warmup, with_oracle=True):
    """Standard admissibility (Sec. 2) on one right-hand side: FP32 and FP16 storage.

    s2: 2D 1024^2, rank 4; s3: 3D 64^3, rank 4; random factor fills, as in the
    paper's experiments. The dominant kernel is reported with its algorithmic
    bytes per launch (U of every level and the dense near field, x, y)."""
    import torch

    import paper_2008_12441_amd as hm
    from hmat_inputs import WORKLOADS, build_workload

    w = WORKLOADS[name]
    t0 = time.time()
    data, x = build_workload(name, device="cuda")
    log(f"setup {name} ({w.describe()}): {time.time() - t0:.1f} s, {len(data.blocks)} blocks")
    n, t = data.n, data.tree
    tree, blocks, keep = hm.make_descriptors(t.parent, t.begin, t.end, data.blocks.target, data.blocks.source,
                                             data.blocks.rank, data.pool, data.off_a, data.off_b)
    sz = (t.end - t.begin).astype(np.int64)
    lr = data.blocks.rank > 0
    nlr = int(lr.sum())
    u_elems = int(np.sum(sz[data.blocks.target[lr]] * data.blocks.rank[lr]))
    v_elems = int(np.sum(sz[data.blocks.source[lr]] * data.blocks.rank[lr]))
    d_elems = int(np.sum((sz[data.blocks.target] * sz[data.blocks.source])[~lr]))
    xd = torch.from_numpy(np.ascontiguousarray(x[:, 0])).cuda()
    vec_bytes = 2 * n * 4
    out = {"workload": f"{name}: {w.describe()}", "blocks": {"low_rank": nlr, "dense": int((~lr).sum())},
           "stored_elements": int(data.pool.size), "paper": PAPER_STANDARD.get(name)}
    ys = {}
    for form in ("fp32", "fp16"):
        t1 = time.time()
        h = hm.HMatrix(tree, blocks, storage=form)
        log(f"{name} {form}: hmat_create {time.time() - t1:.1f} s")
        yd = torch.empty_like(xd)
        ms, ph = time_matvecs(h, xd, yd, steps, warmup, stream)
        ys[form] = yd.cpu().numpy().astype(np.float64)
        esz = 4 if form == "fp32" else 2
        b = h.info["factor_bytes"] + vec_bytes
        ub = esz * (u_elems + d_elems) + vec_bytes
        vb = esz * v_elems + 4 * n
        dom = "uphase_dense" if ph[2] >= ph[0] else "vphase"
        dom_b, dom_ms = (ub, ph[2]) if dom == "uphase_dense" else (vb, ph[0])
        out[form] = {"ms_per_step": round(ms, 5), "GBps": round(b / (ms * 1e-3) / 1e9, 1),
                     "pct_hbm_peak": round(100.0 * b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 2),
                     "alg_bytes_per_step": b, "phases_ms": [round(v, 5) for v in ph],
                     "roofline": {"kernel": "k_uphase" if dom == "uphase_dense" else "k_vphase", "bound": "hbm",
                                  "achieved": round(dom_b / (dom_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBPS,
                                  "unit": "GB/s", "frac": round(dom_b / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                                  "alg_bytes_per_launch": dom_b}}
        if PAPER_STANDARD.get(name):
            out[form]["vs_paper_best_time"] = round(PAPER_STANDARD[name]["time_s"] / (ms * 1e-3), 2)
        log(f"{name} {form}: {ms:.4f} ms/matvec, {out[form]['GBps']} GB/s, phases {ph}")
        h.close()
        del yd
        torch.cuda.empty_cache()
    out["fp16_speedup_vs_fp32"] = round(out["fp32"]["ms_per_step"] / out["fp16"]["ms_per_step"], 3)
    if with_oracle:
        import oracle

        t1 = time.time()
        ref = oracle.oracle_matvec(data, x)[:, 0]
        log(f"{name} oracle: {time.time() - t1:.1f} s")
        for form in ("fp32", "fp16"):
            out[form]["rel_err_vs_fp64_oracle"] = float(np.linalg.norm(ys[form] - ref) / np.linalg.norm(ref))
    return out


def run_h2(stream, steps, warmup, with_oracle=True, n_axis=1024, rank=32):
    """The H^2 variant on the c2 grid: 2D 1024^2 (N = 2^20), leaf 64, weak
    admissibility, nested bases of rank 32 with random fills (leaf bases,
    transfers, couplings, dense blocks), one right-hand side; FP32 and FP16
    storage. The dominant kernel is the leaf kernel (k_h2_leaf), whose
    algorithmic bytes per launch are the leaf U bases, the leaf and chunk E
    transfers, the chunk couplings, the dense blocks, x once and y once."""
    import torch

    import paper_2008_12441_amd as hm
    from hmat_inputs import make_rhs, uniform_tree
    from hmat_inputs.h2 import make_h2

    t0 = time.time()
    h2 = make_h2(uniform_tree(2, n_axis), method="random", rank=rank, seed=9, device="cuda")
    x = make_rhs(h2.n, 1, 1002)
    log(f"setup h2 (2D {n_axis}^2, rank {rank}, random fills): {time.time() - t0:.1f} s, {h2.pool.size} elements")
    n = h2.n
    xd = torch.from_numpy(np.ascontiguousarray(x[:, 0])).cuda()
    out = {"workload": f"H^2 variant: 2D uniform grid {n_axis}^2 (N={n}), leaf 64, weak admissibility, nested bases "
                       f"rank {rank}, random fills, 1 RHS", "stored_elements": int(h2.pool.size)}
    ys = {}
    for form in ("fp32", "fp16"):
        h = hm.H2Matrix(h2, storage=form)
        info = h.info
        yd = torch.empty_like(xd)
        for _ in range(warmup):
            h.matvec(xd, yd)
        torch.cuda.synchronize()
        hm.hmat_h2_set_timing(h.handle, True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            h.matvec(xd, yd)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        ph, calls = hm.hmat_h2_get_timing(h.handle)
        hm.hmat_h2_set_timing(h.handle, False)
        ph = [v / calls for v in ph]
        ys[form] = yd.cpu().numpy().astype(np.float64)
        b = info["factor_bytes"] + 8 * n
        lk = info["leaf_kernel_bytes"]
        out[form] = {"ms_per_step": round(ms, 5), "GBps": round(b / (ms * 1e-3) / 1e9, 1), "alg_bytes_per_step": b,
                     "phases_ms": [round(v, 5) for v in ph],
                     "roofline": {"kernel": "k_h2_leaf", "bound": "hbm",
                                  "achieved": round(lk / (ph[2] * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBPS,
                                  "unit": "GB/s", "frac": round(lk / (ph[2] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                                  "alg_bytes_per_launch": lk, "avg_ms": round(ph[2], 5)}}
        log(f"h2 {form}: {ms:.4f} ms/matvec, {out[form]['GBps']} GB/s, phases {ph}, leaf kernel "
            f"{out[form]['roofline']['achieved']} GB/s")
        h.close()
    out["fp16_speedup_vs_fp32"] = round(out["fp32"]["ms_per_step"] / out["fp16"]["ms_per_step"], 3)
    if with_oracle:
        import oracle.h2 as h2o

        t1 = time.time()
        ref = h2o.h2_oracle_matvec(h2, x)[:, 0]
        log(f"h2 oracle: {time.time() - t1:.1f} s")
        for form in ("fp32", "fp16"):
            out[form]["rel_err_vs_fp64_oracle"] = float(np.linalg.norm(ys[form] - ref) / np.linalg.norm(ref))
    return out


def run_compress(name, reps=2):
    """Wall time of hmat_compress (every block of the workload's structure: dense
    entries and randomized SVDs on the GPU, factors copied to host memory)."""
    import paper_2008_12441_amd as hm
    from hmat_inputs import WORKLOADS, enumerate_blocks, uniform_tree

    w = WORKLOADS[name]
    tree = uniform_tree(w.d, w.n_axis)
    bl = enumerate_blocks(tree, w.rank, w.admissibility)
    sz = (tree.end - tree.begin).astype(np.int64)
    lr = bl.rank > 0
    lr_entries = int(np.sum(sz[bl.target[lr]] * sz[bl.source[lr]]))
    dense_entries = int(np.sum(sz[bl.target[~lr]] * sz[bl.source[~lr]]))
    times = []
    for rep in range(reps):
        t0 = time.perf_counter()
        pool, _, _ = hm.compress_pool(tree.parent, tree.begin, tree.end, bl.target, bl.source, bl.rank, tree.points,
                                      kernel=w.kind, diag=1.0, oversample=10, seed=w.rhs_seed)
        times.append(time.perf_counter() - t0)
        assert np.isfinite(pool).all()
        del pool
    best = min(times)
    out = {"s": round(best, 3), "all_s": [round(t, 3) for t in times], "lowrank_blocks": int(lr.sum()),
           "dense_blocks": int((~lr).sum()), "rank": w.rank, "oversample": 10,
           "kernel_entries_per_s": round((2 * lr_entries + dense_entries) / best, 1),
           "note": "wall time of the synchronous call: kernel entries generated twice per low-rank block "
                   "(sample and projection), FP64 Gram/Jacobi per block, factors copied to host memory"}
    log(f"compress {name}: {best:.2f} s ({out['lowrank_blocks']} low-rank, {out['dense_blocks']} dense blocks)")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(the whole H-matrix and its product live on a single GPU)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2008_12441_amd as hm
    from hmat_inputs import WORKLOADS, build_workload
    from hmat_inputs.tree import stored_elements

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    hm.load_library()
    w = WORKLOADS[args.config]
    stream = torch.cuda.current_stream()

    read_gbps, copy_gbps = probe_bandwidth(stream)
    log(f"probe: read {read_gbps:.0f} GB/s, copy {copy_gbps:.0f} GB/s")

    t0 = time.time()
    data, x = build_workload(args.config, device="cuda", method=args.method)
    log(f"setup ({w.describe()}): {time.time() - t0:.1f} s")
    n = data.n
    t = data.tree
    tree, blocks, keep = hm.make_descriptors(t.parent, t.begin, t.end, data.blocks.target,
                                             data.blocks.source, data.blocks.rank, data.pool,
                                             data.off_a, data.off_b)
    t0 = time.time()
    h = hm.HMatrix(tree, blocks, storage="fp32")
    info = h.info
    log(f"hmat_create fp32: {time.time() - t0:.1f} s, {info}")
    xd = torch.from_numpy(np.ascontiguousarray(x[:, 0])).cuda()
    yd = torch.empty_like(xd)

    ms, phase_ms = time_matvecs(h, xd, yd, args.steps, args.warmup, stream)
    y = yd.cpu().numpy().astype(np.float64)
    vec_bytes = 2 * n * 4  # x read once, y written once
    alg_bytes = info["factor_bytes"] + vec_bytes
    gbps = alg_bytes / (ms * 1e-3) / 1e9
    log(f"fp32: {ms:.4f} ms/matvec, {gbps:.0f} GB/s algorithmic, phases(ms) {phase_ms}")

    # dominant kernel: the U-phase (U of every level + dense near field + x + y)
    sz = t.end - t.begin
    is_lr = data.blocks.rank > 0
    u_elems = int(np.sum(sz[data.blocks.target[is_lr]].astype(np.int64) * data.blocks.rank[is_lr]))
    d_elems = int(np.sum((sz[data.blocks.target] * sz[data.blocks.source])[~is_lr]))
    v_elems = int(np.sum(sz[data.blocks.source[is_lr]].astype(np.int64) * data.blocks.rank[is_lr]))
    assert u_elems + d_elems + v_elems == stored_elements(t, data.blocks)
    uphase_bytes = 4 * (u_elems + d_elems) + vec_bytes
    vphase_bytes = 4 * v_elems + 4 * n
    phases = {"vphase": {"ms": phase_ms[0], "alg_bytes": vphase_bytes},
              "zfinish": {"ms": phase_ms[1]},
              "uphase_dense": {"ms": phase_ms[2], "alg_bytes": uphase_bytes}}
    for k in ("vphase", "uphase_dense"):
        phases[k]["GBps"] = phases[k]["alg_bytes"] / (phases[k]["ms"] * 1e-3) / 1e9
    dom = max(("vphase", "uphase_dense"), key=lambda k: phases[k]["ms"])
    achieved = phases[dom]["GBps"]

    out_extra = {}
    # low-precision form on the same problem
    if not args.no_fp16:
        t0 = time.time()
        h16 = hm.HMatrix(tree, blocks, storage="fp16")
        log(f"hmat_create fp16: {time.time() - t0:.1f} s")
        y16d = torch.empty_like(xd)
        ms16, ph16 = time_matvecs(h16, xd, y16d, args.steps, args.warmup, stream)
        y16 = y16d.cpu().numpy().astype(np.float64)
        b16 = h16.info["factor_bytes"] + vec_bytes
        out_extra["fp16_scaled"] = {"ms_per_step": ms16, "GBps": b16 / (ms16 * 1e-3) / 1e9,
                                    "speedup_vs_fp32": ms / ms16, "phases_ms": ph16}
        h16.close()
        log(f"fp16: {ms16:.4f} ms/matvec, speedup {ms / ms16:.2f}x")
    else:
        y16 = None

    # the transpose product of the same matrix (a handle built for K^T, same kernels)
    if not args.no_transpose:
        t0 = time.time()
        ht = hm.HMatrix(tree, blocks, storage="fp32", transpose=True)
        log(f"hmat_create fp32 transpose: {time.time() - t0:.1f} s")
        ytd = torch.empty_like(xd)
        mst, pht = time_matvecs(ht, xd, ytd, args.steps, args.warmup, stream)
        out_extra["transpose_fp32"] = {"ms_per_step": round(mst, 5),
                                       "GBps": round(alg_bytes / (mst * 1e-3) / 1e9, 1),
                                       "phases_ms": [round(v, 5) for v in pht]}
        log(f"fp32 transpose: {mst:.4f} ms/matvec, {out_extra['transpose_fp32']['GBps']} GB/s")
        ht.close()
        del ytd

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        prep = oracle.prepare(data)
        threads = oracle.max_threads()
        oracle.oracle_matvec(prep, x)  # warm-up

        def time_oracle(nthreads, seconds):
            times, ref = [], None
            t_start = time.time()
            while True:
                t0 = time.perf_counter()
                ref = oracle.oracle_matvec(prep, x, nthreads=nthreads)[:, 0]
                times.append(time.perf_counter() - t0)
                if time.time() - t_start >= seconds:
                    break
            return float(np.median(times)), len(times), ref

        cpu_s, nrun, ref = time_oracle(threads, args.cpu_seconds)
        cpu1_s, nrun1, _ = time_oracle(1, args.cpu_seconds)
        host = host_cpu()
        cpu = {"value": round(alg_bytes / cpu_s / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
               "sample": f"{nrun} full FP64 oracle matvecs of this workload on {threads} threads (median "
                         f"{cpu_s:.4f} s each); {nrun1} on 1 thread (median {cpu1_s:.3f} s)",
               "matvecs_per_s": round(1.0 / cpu_s, 3),
               "single_core": {"value": round(alg_bytes / cpu1_s / 1e9, 3), "unit": "GB/s", "cores": 1,
                               "matvecs_per_s": round(1.0 / cpu1_s, 3)},
               "host": host, "gpu_vs_cpu_all_cores": round(cpu_s / (ms * 1e-3), 1)}
        rel = float(np.linalg.norm(y - ref) / np.linalg.norm(ref))
        out_extra["rel_err_vs_fp64_oracle"] = rel
        if y16 is not None:
            out_extra["fp16_scaled"]["rel_err_vs_fp64_oracle"] = float(np.linalg.norm(y16 - ref) / np.linalg.norm(ref))
        log(f"oracle: {cpu_s:.3f} s/matvec on {threads} threads, {cpu1_s:.3f} s on 1 thread ({host}); "
            f"fp32 rel err {rel:.3e}")

    if args.config == "c2":
        # Table 1's weak-admissibility times for the same grid (N = 1024^2), rank 4,
        # random factors, distributed memory on KNL processes: context only
        out_extra["paper_context"] = {
            "table": "Table 1 (2D), N = 1024^2, weak admissibility, r = 4, random fills",
            "one_node_s": 1.17e-2, "one_node": "1 KNL node (32 processes)",
            "fastest_s": 3.40e-3, "fastest": "16 KNL nodes (512 processes)",
            "this_gpu_over_one_node": round(1.17e-2 / (ms * 1e-3), 2),
            "this_gpu_over_fastest": round(3.40e-3 / (ms * 1e-3), 2),
            "note": "the paper's rank is 4 against 32 here (about 4.5x fewer stored elements); context, not a target"}

    result = {
        "metric": "H-matvec GB/s (% HBM peak) N=2^20 r=32; low-prec/batched speedup @1e-3 err",
        "value": round(gbps, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {w.describe()}", "n": n, "rank": w.rank, "leaf": 64,
                   "nrhs": 1, "storage": "fp32", "factor_bytes": info["factor_bytes"],
                   "alg_bytes_per_step": alg_bytes},
        "pct_hbm_peak": round(100.0 * gbps / HBM_PEAK_GBPS, 2),
        "pct_probe_read": round(100.0 * gbps / read_gbps, 2),
        "probe_GBps": {"read": round(read_gbps, 1), "copy": round(copy_gbps, 1)},
        "matvecs_per_s": round(1e3 / ms, 2),
        "roofline": {"kernel": "k_uphase (U of all levels + dense near field + y)" if dom == "uphase_dense"
                     else "k_vphase", "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic_from_profile("k_uphase<FP32>") if (dom == "uphase_dense" and args.config == "c2")
                     else None,
                     "alg_bytes_per_launch": phases[dom]["alg_bytes"], "avg_ms": round(phases[dom]["ms"], 5)},
        "phases": phases,
        "cpu_baseline": cpu,
    }
    result.update(out_extra)
    h.close()
    del h
    if not args.no_c3:
        import gc

        import torch

        del keep, tree, blocks, data
        gc.collect()
        torch.cuda.empty_cache()
        result["multi_rhs_c3"] = run_multi_rhs(stream, args.c3_steps, 3, with_oracle=not args.no_cpu_baseline,
                                               method=args.method, forms=tuple(args.c3_forms.split(",")))
    if not args.no_c5:
        import gc

        import torch

        gc.collect()
        torch.cuda.empty_cache()
        result["large_3d_c5"] = run_large_3d(stream, args.c5_steps, 2, with_oracle=not args.no_cpu_baseline,
                                             method=args.method, forms=tuple(args.c5_forms.split(",")))
    for name, skip in (("s2", args.no_s2), ("s3", args.no_s3)):
        if skip:
            continue
        import gc

        import torch

        gc.collect()
        torch.cuda.empty_cache()
        result[f"standard_{name}"] = run_standard(stream, name, args.s_steps, 5, with_oracle=not args.no_cpu_baseline)
    if not args.no_c4:
        import gc

        import torch

        gc.collect()
        torch.cuda.empty_cache()
        result["batched_c4"] = run_batched(stream, args.c4_steps, 3, count=args.c4_members, method=args.c4_method,
                                           with_oracle=not args.no_cpu_baseline)
    if not args.no_h2:
        import gc

        import torch

        gc.collect()
        torch.cuda.empty_cache()
        result["h2_c2"] = run_h2(stream, args.s_steps, 5, with_oracle=not args.no_cpu_baseline)
    if not args.no_compress:
        import gc

        import torch

        gc.collect()
        torch.cuda.empty_cache()
        result["compress"] = {name: run_compress(name) for name in ("c2", "c3")}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
