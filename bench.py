"""Benchmark: setup latency and invocations/s, shared+batched vs plain, on one
MI355X.

Workload (default): 4 functions, each an 8-layer BF16 MLP of width 4096
(256 MiB of read-only weights), with 30 % of the 64 KiB block indices holding
identical content in all four; 64 invocations per function with batch sizes
uniform on 1..32 and BF16 N(0,1) inputs.  Sources and inputs are resident in
HBM before the timed region.

One step = the whole path over one batch of 256 requests:
  shared+batched: fn_register_batch of the 4 functions (fingerprint + dedup
                  into the pool, each function's fingerprints overlapping
                  the previous one's classification), fn_setup x256, one
                  fn_invoke_batch (grouped GEMM per layer from a hipGraph),
                  fn_release x256, fn_unregister x4;
  plain:          the same registration call (code only), then per request
                  a private copy of the weights (fn_setup), one launch
                  sequence (fn_invoke), fn_release.
Setup latency of a request = its fn_setup time, plus its function's
registration time (the library's time from the previous function's
registration to its own) for the first request of each function (a cold
start).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "setup p50/p99 ms + invocations/sec, shared+batched vs plain, 1 MI355X"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
# HBM traffic of the grouped GEMM comes from rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs summarised in this file; it is reported only while the GEMM sources
# and the launch plan are the ones the counters were taken on.
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "ggemm_bf16_sharing_counters.md")
# The record is tied to the GEMM kernels' own sources (the launch plan, which
# the host planner picks, is recorded beside it).
GEMM_SOURCES = ("paper_2404_14691_amd/csrc/body_mlp.hip", "paper_2404_14691_amd/csrc/layout.h")


_T0 = time.time()


def log(msg):
    print(f"[bench {time.time() - _T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


def percentile(v, q):
    """Nearest-rank percentile."""
    s = sorted(v)
    k = max(1, int(np.ceil(q / 100.0 * len(s))))
    return s[k - 1]


class Workload:
    def __init__(self, torch, n_fns=4, layers=8, width=4096, per_fn=64, max_batch=32, seed=0):
        from paper_2404_14691_amd import synth
        self.layers, self.width, self.n_fns = layers, width, n_fns
        w = synth.shared_mlp_bf16_functions(n_fns=n_fns, layers=layers, width=width, share_frac=0.3, seed=seed)
        self.host_blobs = w.blobs
        self.dev_blobs = [torch.from_numpy(b.view(np.uint8)).cuda() for b in w.blobs]
        self.requests = []            # (fn index, batch, row offset)
        rows = 0
        for f in range(n_fns):
            for b in synth.uniform_batches(per_fn, 1, max_batch, seed=seed, stream=f):
                self.requests.append((f, int(b), rows))
                rows += int(b)
        # interleave functions the way concurrent arrivals would
        order = np.random.default_rng(seed).permutation(len(self.requests))
        self.requests = [self.requests[i] for i in order]
        self.rows = rows
        x = np.concatenate([synth.bf16_inputs(b, width, seed, 100 + i) for i, (_, b, _) in
                            enumerate(sorted(self.requests, key=lambda r: r[2]))])
        self.x_host = x
        self.x = torch.from_numpy(x).cuda()
        self.y = torch.zeros((rows, width), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        io = [self.io(r) for r in self.requests]
        self.ins = [i for i, _ in io]
        self.outs = [o for _, o in io]
        # the same, as (address, nbytes) rows and per-request arrays, built once
        self.ins_arr = np.array(self.ins, dtype=np.uint64)
        self.outs_arr = np.array(self.outs, dtype=np.uint64)
        self.fidx = np.array([f for f, _, _ in self.requests])
        self.batch_arr = np.array([b for _, b, _ in self.requests], dtype=np.uint32)
        self.first_of_fn = {}
        for i, (f, _, _) in enumerate(self.requests):
            self.first_of_fn.setdefault(f, i)

    def io(self, req):
        _, b, r = req
        xb, yb = b * self.width * 2, b * self.width * 4
        return ((self.x.data_ptr() + r * self.width * 2, xb), (self.y.data_ptr() + r * self.width * 4, yb))


def register_all(S, ctx, wl):
    """The step's functions in one fn_register_batch call (each function's
    fingerprints run while the host classifies the previous one); per
    function, the library's time since the previous one was registered."""
    desc = S.mlp_desc(S.SAGE_MLP_BF16, wl.layers, wl.width)
    srcs = [[S.make_blob(d.data_ptr(), d.numel(), where=S.SAGE_SRC_DEVICE)] for d in wl.dev_blobs]
    return S.fn_register_batch(ctx, [desc] * len(srcs), srcs)


def shared_step(S, ctx, wl, want_stats=False):
    io = S.SAGE_IO_DEVICE_IN | S.SAGE_IO_DEVICE_OUT
    fns, reg_ms = register_all(S, ctx, wl)
    # the step's requests arrive together and are admitted in one call; each
    # request's setup time is its own, measured inside the library, plus its
    # function's registration for the first request of each function
    invs, own_ms = S.fn_setup_batch(ctx, np.asarray(fns, dtype=np.uint64)[wl.fidx], wl.batch_arr, timed=True)
    for f, i in wl.first_of_fn.items():
        own_ms[i] += reg_ms[f]
    setup_ms = own_ms
    S.fn_invoke_batch(ctx, invs, wl.ins_arr, wl.outs_arr, io)
    S.fn_release_batch(ctx, invs)
    stats = S.sage_get_stats(ctx) if want_stats else None  # pool accounting: measurement, not the path
    for f in fns:
        S.fn_unregister(ctx, f)
    return setup_ms, stats


def plain_step(S, ctx, wl):
    io = S.SAGE_IO_DEVICE_IN | S.SAGE_IO_DEVICE_OUT
    fns, reg_ms = register_all(S, ctx, wl)
    setup_ms = []
    seen = set()
    for req in wl.requests:
        f = req[0]
        # the library's own per-request setup clock, as on the shared path
        invs, ms = S.fn_setup_batch(ctx, [fns[f]], [req[1]], timed=True)
        inv, dt = invs[0], ms[0]
        if f not in seen:
            dt += reg_ms[f]
            seen.add(f)
        setup_ms.append(dt)
        i, o = wl.io(req)
        S.fn_invoke(ctx, inv, i, o, io)
        S.fn_release(ctx, inv)
    for f in fns:
        S.fn_unregister(ctx, f)
    return setup_ms


# the BF16 GEMM kernels end where the FP32 layer kernel's section of the file begins
GEMM_END_MARKER = b"// ---------------------------------------------------------------- FP32 MLP"


def gemm_sources_digest():
    h = hashlib.sha256()
    for f in GEMM_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            data = fh.read()
        h.update(data.split(GEMM_END_MARKER)[0])
    return h.hexdigest()[:16]


def traffic_record(plan):
    """The committed counter record for this GEMM source and plan, or None."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    digest = gemm_sources_digest()
    for line in lines:
        if line.startswith("traffic-record: "):
            rec = json.loads(line[len("traffic-record: "):])
            if rec.get("sources") == digest and rec.get("plan") == plan:
                return rec
    return None


def timed(torch, fn, steps):
    out = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out.append(fn())
    torch.cuda.synchronize()
    return (time.perf_counter() - t0), out


def kernel_bandwidth(S, ctx, torch, nbytes=4 << 30, reps=5):
    """fp64k and blkcopy alone on `nbytes` (well above the 256 MB MALL), timed
    with HIP events on the launch stream."""
    stream = torch.cuda.current_stream().cuda_stream
    nblk = nbytes // 65536
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    fps = torch.empty(nblk, dtype=torch.int64, device="cuda")
    res = torch.empty(nblk, dtype=torch.int32, device="cuda")
    base = np.arange(nblk, dtype=np.uint64) * np.uint64(65536)
    ops = np.zeros(nblk, dtype=[("src", "<u8"), ("dst", "<u8"), ("len", "<u4"), ("op", "<u4")])
    ops["src"], ops["dst"], ops["len"], ops["op"] = base + np.uint64(src.data_ptr()), base + np.uint64(dst.data_ptr()), 65536, S.SAGE_OP_COPY
    d_copy = torch.from_numpy(ops.view(np.uint8)).cuda()
    ops["op"] = S.SAGE_OP_VERIFY
    d_verify = torch.from_numpy(ops.view(np.uint8)).cuda()
    torch.cuda.synchronize()
    out = {}
    for name, run, moved in (
            ("fp64k", lambda: S.sage_fingerprint(ctx, src.data_ptr(), nbytes, fps.data_ptr(), stream), nbytes + 8 * nblk),
            ("blkcopy", lambda: S.sage_blkcopy(ctx, d_copy.data_ptr(), nblk, res.data_ptr(), stream), 2 * nbytes),
            ("blkcopy_verify", lambda: S.sage_blkcopy(ctx, d_verify.data_ptr(), nblk, res.data_ptr(), stream), 2 * nbytes)):
        run()
        torch.cuda.synchronize()
        S.sage_timing_reset(ctx)
        S.sage_timing_enable(ctx, True)
        for _ in range(reps):
            run()
        torch.cuda.synchronize()
        S.sage_timing_enable(ctx, False)
        ms, n = S.sage_timing_get(ctx, "fp64k" if name == "fp64k" else "blkcopy")
        avg = ms / max(n, 1)
        out[name] = {"bytes": int(moved), "avg_ms": round(avg, 4), "GB/s": round(moved / (avg * 1e-3) / 1e9, 1),
                     "frac_of_8TB/s": round(moved / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if not bool((res == 0).all().item()):
        raise RuntimeError("verify after copy reported a difference")
    del src, dst, fps, res, d_copy, d_verify
    torch.cuda.empty_cache()
    return out


def host_link(S, torch, wl):
    """Registration from host memory (the path the paper parallelizes): raw
    pinned H2D peak, then 4-function registration from pinned and pageable
    sources, pipelined vs one-after-the-other setup vs no staging ring."""
    out = {}
    nbytes = 1 << 30
    h = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    d = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    d.copy_(h, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        d.copy_(h, non_blocking=True)
    torch.cuda.synchronize()
    out["pinned_h2d_GBps"] = round(3 * nbytes / (time.perf_counter() - t0) / 1e9, 2)
    del h, d
    total = sum(b.nbytes for b in wl.host_blobs)
    desc = S.mlp_desc(S.SAGE_MLP_BF16, wl.layers, wl.width)
    variants = [("pinned_pipelined", {}, True), ("pageable_pipelined", {}, False),
                ("pageable_serial_setup", {"serial_setup": 1}, False),
                ("pageable_no_ring", {"ring_slots": 1, "streams": 1}, False)]
    for name, over, pinned in variants:
        cfg = S.sage_config_default()
        cfg.pool_budget_bytes = 2 << 30
        for k, v in over.items():
            setattr(cfg, k, v)
        ctx = S.sage_open(0, cfg)
        try:
            srcs = []
            for b in wl.host_blobs:
                if pinned:
                    a = S.pinned_array(ctx, b.shape, b.dtype)
                    a[:] = b
                    srcs.append(a)
                else:
                    srcs.append(b)
            best = None
            for _ in range(2):
                t0 = time.perf_counter()
                fns = [S.fn_register(ctx, desc, [S.make_blob(a)]) for a in srcs]
                dt = time.perf_counter() - t0
                for f in fns:
                    S.fn_unregister(ctx, f)
                best = dt if best is None else min(best, dt)
            out[name] = {"register_4fn_ms": round(best * 1e3, 2), "GBps": round(total / best / 1e9, 2)}
            if pinned:
                for a in srcs:
                    S.sage_host_free(ctx, a.ctypes.data)
        finally:
            S.sage_close(ctx)
    return out


def host_sourced(S, torch, wl, shared_steps=10, naive_requests=64):
    """The metric with the host link in it: the four functions' sources in
    host memory (pinned, from sage_host_alloc, and pageable), inputs read from
    and outputs written to host memory.

    shared+batched step: fn_register_batch of the 4 functions from the host
      sources (pipelined H2D + fingerprint + dedup), fn_setup x256 (one
      call), one grouped fn_invoke_batch, fn_release x256, fn_unregister x4;
    plain step: the same registration call (code only), then per request fn_setup (a
      private copy of its function's 256 MiB through the same pipelined H2D),
      fn_invoke (one launch sequence), fn_release;
    naive plain: plain with one staging slot on one stream and the code
      branch serialised (no pipelining), on a seeded subsample of requests.

    Setup latency of a request is the library's own clock for its fn_setup
    (fn_setup_batch with per-request times) on both paths, plus its
    function's registration time (library clock) for the first request of
    each function.
    Throughput_perf follows the paper's eq. (1): the achieved invocation rate
    over the rate if each invocation cost only its computation time T_comp,
    here the mean device time of one invocation's body run alone (the plain
    path's launch sequences, HIP events on their stream)."""
    desc = S.mlp_desc(S.SAGE_MLP_BF16, wl.layers, wl.width)
    n_req = len(wl.requests)
    ro_total = sum(b.nbytes for b in wl.host_blobs)
    y = np.zeros((wl.rows, wl.width), dtype=np.float32)
    ins = [wl.x_host[r:r + b] for _, b, r in wl.requests]
    outs = [y[r:r + b] for _, b, r in wl.requests]
    io_bytes = wl.x_host.nbytes + y.nbytes
    fidx = wl.fidx
    batches = wl.batch_arr
    res = {"sources": "host memory; inputs from and outputs to host memory",
           "expected_h2d_ro_bytes_per_step": {"plain": int(sum(wl.host_blobs[f].nbytes for f, _, _ in wl.requests)),
                                              "shared": int(ro_total)}}

    def sources(ctx, pinned):
        if not pinned:
            return list(wl.host_blobs), []
        srcs = []
        for b in wl.host_blobs:
            a = S.pinned_array(ctx, b.shape, b.dtype)
            a[:] = b
            srcs.append(a)
        return srcs, srcs

    def register(ctx, srcs):
        return S.fn_register_batch(ctx, [desc] * len(srcs), [[S.make_blob(a)] for a in srcs])

    def shared_step(ctx, srcs, want_pool=False):
        fns, reg_ms = register(ctx, srcs)
        invs, own = S.fn_setup_batch(ctx, np.asarray(fns, dtype=np.uint64)[fidx], batches, timed=True)
        for f, i in wl.first_of_fn.items():
            own[i] += reg_ms[f]
        pool = S.sage_get_stats(ctx) if want_pool else None
        S.fn_invoke_batch(ctx, list(invs), ins, outs, 0)
        S.fn_release_batch(ctx, invs)
        for f in fns:
            S.fn_unregister(ctx, f)
        return list(own), pool

    def plain_step(ctx, srcs, reqs):
        fns, reg_ms = register(ctx, srcs)
        setup, seen = [], set()
        for i in reqs:
            f, b, _ = wl.requests[i]
            invs, ms = S.fn_setup_batch(ctx, [fns[f]], [b], timed=True)
            dt = ms[0]
            if f not in seen:
                dt += reg_ms[f]
                seen.add(f)
            setup.append(dt)
            S.fn_invoke(ctx, invs[0], ins[i], outs[i], 0)
            S.fn_release(ctx, invs[0])
        for f in fns:
            S.fn_unregister(ctx, f)
        return setup

    def pcts(v):
        return {"p50": round(percentile(v, 50), 4), "p99": round(percentile(v, 99), 3)}

    t_comp_ms = None
    for kind in ("pinned", "pageable"):
        pinned = kind == "pinned"
        leg = {}
        # ---- shared + batched
        cfg = S.sage_config_default()
        cfg.pool_budget_bytes = 8 << 30
        ctx = S.sage_open(0, cfg)
        try:
            srcs, owned = sources(ctx, pinned)
            pool = shared_step(ctx, srcs, want_pool=True)[1]
            shared_step(ctx, srcs)
            st0 = S.sage_get_stats(ctx)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            setup = []
            for _ in range(shared_steps):
                setup += shared_step(ctx, srcs)[0]
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            st1 = S.sage_get_stats(ctx)
            rate = n_req * shared_steps / el
            leg["shared_batched"] = {
                "invocations_per_s": round(rate, 2), "ms_per_step": round(el / shared_steps * 1e3, 3),
                "steps": shared_steps, "setup_ms": pcts(setup),
                "h2d_ro_bytes_per_step": int((st1["h2d_bytes"] - st0["h2d_bytes"]) // shared_steps),
                "h2d_io_bytes_per_step": int(io_bytes),
                "ro_GBps_per_step": round(ro_total * shared_steps / el / 1e9, 2),
                "resident_bytes": int(pool["resident_bytes"]), "unique_bytes": int(pool["unique_bytes"]),
                "live_invocations": int(pool["live_setups"])}
            for a in owned:
                S.sage_host_free(ctx, a.ctypes.data)
        finally:
            S.sage_close(ctx)
        log(f"host-sourced {kind}: shared {leg['shared_batched']}")
        # ---- plain: a private copy per invocation through the pipelined H2D
        for name, over, reqs in (("plain", {}, list(range(n_req))),
                                 ("naive_plain", {"ring_slots": 1, "streams": 1, "serial_setup": 1},
                                  sorted(np.random.default_rng(7).choice(n_req, naive_requests, replace=False)))):
            if name == "naive_plain" and pinned:
                continue  # pinned sources are copied by DMA without the ring: the naive form is the pageable one
            cfg = S.sage_config_default()
            cfg.share = 0
            cfg.pool_budget_bytes = 1 << 20
            for k, v in over.items():
                setattr(cfg, k, v)
            ctx = S.sage_open(0, cfg)
            try:
                srcs, owned = sources(ctx, pinned)
                plain_step(ctx, srcs, reqs[:8])  # warm: code object, private buffers, staging
                if t_comp_ms is None:
                    S.sage_timing_reset(ctx)
                    S.sage_timing_only(ctx, "ggemm_bf16")
                    S.sage_timing_enable(ctx, True)
                st0 = S.sage_get_stats(ctx)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                setup = plain_step(ctx, srcs, reqs)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                st1 = S.sage_get_stats(ctx)
                if t_comp_ms is None:
                    S.sage_timing_enable(ctx, False)
                    g_ms, g_n = S.sage_timing_get(ctx, "ggemm_bf16")
                    t_comp_ms = g_ms / (g_n / wl.layers)
                    res["t_comp_ms"] = {"value": round(t_comp_ms, 5), "invocations": int(g_n // wl.layers),
                                        "what": "mean device time of one invocation's 8 layers run alone"}
                rate = len(reqs) / el
                leg[name] = {"invocations_per_s": round(rate, 2), "ms_per_step": round(el * 1e3, 3),
                             "requests": len(reqs), "setup_ms": pcts(setup),
                             "h2d_ro_bytes": int(st1["h2d_bytes"] - st0["h2d_bytes"]),
                             "ro_GBps": round((st1["h2d_bytes"] - st0["h2d_bytes"]) / el / 1e9, 2)}
                if name == "naive_plain":
                    leg[name]["sample"] = f"{len(reqs)} of the {n_req} requests (seeded), in order"
                for a in owned:
                    S.sage_host_free(ctx, a.ctypes.data)
            finally:
                S.sage_close(ctx)
            log(f"host-sourced {kind}: {name} {leg[name]}")
        sb, pl = leg["shared_batched"], leg["plain"]
        sb["plain_footprint_bytes_same_concurrency"] = int(sum(wl.host_blobs[f].nbytes for f, _, _ in wl.requests))
        sb["density_vs_plain"] = round(sb["plain_footprint_bytes_same_concurrency"] / max(sb["resident_bytes"], 1), 2)
        leg["speedup_vs_plain"] = round(sb["invocations_per_s"] / pl["invocations_per_s"], 2)
        leg["setup_p50_vs_plain"] = round(pl["setup_ms"]["p50"] / max(sb["setup_ms"]["p50"], 1e-9), 2)
        res[kind] = leg
    for kind in ("pinned", "pageable"):
        for name in ("shared_batched", "plain", "naive_plain"):
            if name in res[kind]:
                res[kind][name]["throughput_perf"] = round(res[kind][name]["invocations_per_s"] * t_comp_ms * 1e-3, 4)
    return res


def cold_setup_ab(S, wl, pairs=20):
    """Parallelized setup against serialized setup on cold contexts (section
    "Effectiveness of parallelized setup mechanism"): each sample opens a new
    context, so registering a function loads its code object (hipModuleLoad)
    and allocates its block table on one thread while its 256 MiB of weights
    move from pageable host memory through the staging ring on the other; the
    serial mode runs the two branches one after the other.  Modes alternate
    (ABBA) within one process; reported: medians, interquartile ranges and
    the median of the paired differences."""
    desc = S.mlp_desc(S.SAGE_MLP_BF16, wl.layers, wl.width)
    blob = wl.host_blobs[0]
    res = {"parallel": [], "serial": []}
    code_ms = {"parallel": [], "serial": []}
    for p in range(pairs):
        order = ("parallel", "serial") if p % 2 == 0 else ("serial", "parallel")
        for mode in order:
            cfg = S.sage_config_default()
            cfg.pool_budget_bytes = 1 << 30
            cfg.serial_setup = 1 if mode == "serial" else 0
            ctx = S.sage_open(0, cfg)
            try:
                st0 = S.sage_get_stats(ctx)
                t0 = time.perf_counter()
                fn = S.fn_register(ctx, desc, [S.make_blob(blob)])
                res[mode].append((time.perf_counter() - t0) * 1e3)
                st1 = S.sage_get_stats(ctx)
                code_ms[mode].append(st1["t_module_ms"] - st0["t_module_ms"])
                S.fn_unregister(ctx, fn)
            finally:
                S.sage_close(ctx)
    diff = [s_ - p_ for s_, p_ in zip(res["serial"], res["parallel"])]

    def summ(v):
        q = np.percentile(v, [25, 50, 75])
        return {"median": round(float(q[1]), 3), "iqr": [round(float(q[0]), 3), round(float(q[2]), 3)]}
    return {"what": "cold-context fn_register of one 256 MiB BF16 MLP from pageable host memory (code object "
                    "load + block table beside the staged data), ms",
            "samples_per_mode": pairs, "parallel": summ(res["parallel"]), "serial": summ(res["serial"]),
            "serial_minus_parallel": summ(diff),
            "module_load_ms": {m: round(float(np.median(v)), 3) for m, v in code_ms.items()}}


def serving_leg(S, torch, rate=1000.0, duration=10.0):
    """Serving at the over-HBM regime of the Poisson workload, shared against
    plain on one arrival trace, at one rate (bench_workloads.ServingBench)."""
    import bench_workloads
    sb = bench_workloads.ServingBench(S, torch, log)
    try:
        return sb.rate(rate, duration)
    finally:
        sb.close()


def _host_cpu():
    """(BLAS threads, nproc, CPU model) of this host."""
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    cpu = ""
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    return int(cores), os.cpu_count(), cpu


def cpu_baseline_workload(name, min_s=3.0):
    """The oracle on the host for a secondary workload, on a bounded sample
    of it, in the workload's unit (invocations/s); None for workloads
    without one."""
    from oracle import fingerprint as OF
    from oracle import mlp as OM
    from oracle import stencil as OS
    from paper_2404_14691_amd import synth
    cores, nproc, cpu = _host_cpu()
    if name == "mlp_f32":
        # a step registers the 32 MiB of weights (fingerprints) and runs 16 invocations of 8 rows
        wl = synth.mlp_f32_workload()
        t0 = time.perf_counter()
        passes = 0
        while passes < 2 or time.perf_counter() - t0 < min_s:
            OF.fp64k_blob(wl.weights)
            W = wl.weights.astype(np.float64)
            for x in wl.inputs:
                OM.mlp_forward(x, W)
            passes += 1
        el = time.perf_counter() - t0
        value = 16 * passes / el
        sample = (f"{passes} passes of the workload's 16 invocations (2 x 2048^2 float64 layers, 8 rows), each "
                  f"pass with the fingerprints of the 32 MiB of weights; {el:.1f} s")
    elif name == "stencil":
        # one sweep of one 512^3 field; an invocation is 20 sweeps, a step
        # 32 invocations plus the fingerprints of the 512 MiB coefficient grid
        n, sweeps, n_inv = 512, 20, 32
        c = synth.stencil_coefficients(n, seed=0)
        t0 = time.perf_counter()
        OF.fp64k_blob(c)
        t_fp = time.perf_counter() - t0
        u0 = synth.stencil_field(n, 0, seed=0)
        t0 = time.perf_counter()
        OS.jacobi7(u0, c, 1)
        t_sw = time.perf_counter() - t0
        del u0, c
        step_s = t_fp + n_inv * sweeps * t_sw
        value = n_inv / step_s
        cores = 1  # numpy's elementwise array arithmetic runs on one thread
        sample = (f"one float64 sweep of one 512^3 field ({t_sw:.2f} s = {n ** 3 / t_sw / 1e6:.0f} Mcell/s) and "
                  f"the fingerprints of the 512 MiB coefficient grid ({t_fp:.2f} s); step = fingerprints + "
                  f"{n_inv} invocations x {sweeps} sweeps ({step_s:.0f} s, extrapolated)")
    elif name == "batching":
        # the 256 invocations in a seeded order, at least 16 and until min_s
        # of invocation time; extrapolated to the step when cut short
        W_, L_ = 4096, 8
        w = synth.shared_mlp_bf16_functions(n_fns=1, layers=L_, width=W_, share_frac=0.0, seed=3)
        batches = [int(b) for b in synth.lognormal_batches(256, seed=3)]
        order = np.random.default_rng(0).permutation(256)
        t0 = time.perf_counter()
        OF.fp64k_blob(w.blobs[0])
        t_fp = time.perf_counter() - t0
        Wt = OM.bf16_to_f64(w.blobs[0]).reshape(L_, W_, W_)
        t_inv, done = 0.0, []
        for i in order:
            if len(done) >= 16 and t_inv >= min_s:
                break
            x = OM.bf16_to_f64(synth.bf16_inputs(batches[i], W_, 3, int(i)))
            t0 = time.perf_counter()
            OM.mlp_forward(x, Wt)
            t_inv += time.perf_counter() - t0
            done.append(int(i))
        del Wt
        step_s = t_fp + 256 * t_inv / len(done)
        value = 256 / step_s
        sample = (f"{len(done)} of the 256 invocations in a seeded order ({sum(batches[i] for i in done)} rows, "
                  f"{t_inv:.1f} s) and the fingerprints of the 256 MiB of weights ({t_fp:.1f} s) in float64 "
                  f"numpy; step = fingerprints + 256 x mean invocation ({step_s:.1f} s"
                  f"{', extrapolated' if len(done) < 256 else ''})")
    else:
        return None
    return {"value": float(f"{value:.4g}"), "unit": "invocations/s", "cores": cores, "kind": "oracle", "nproc": nproc,
            "cpu_model": cpu, "sample": sample}


def cpu_baseline(wl, min_s=10.0, max_inv=1024):
    """The oracle on the host: fingerprints and the cross-function dedup map
    of all functions' blobs, then invocations of the workload's requests in
    order (each function's weights converted once) until at least `min_s`
    seconds of invocation time and 64 invocations; scaled to one step."""
    from oracle import dedup as OD
    from oracle import fingerprint as OF
    from oracle import mlp as OM
    t0 = time.perf_counter()
    for blob in wl.host_blobs:
        OF.fp64k_blob(blob)
    OD.partition_dict(wl.host_blobs, 65536)
    t_reg = time.perf_counter() - t0
    Ws = [OM.bf16_to_f64(b).reshape(wl.layers, wl.width, wl.width) for b in wl.host_blobs]
    t_inv, n_inv = 0.0, 0
    while n_inv < max_inv and (t_inv < min_s or n_inv < 64):
        f, b, r = wl.requests[n_inv % len(wl.requests)]
        t0 = time.perf_counter()
        OM.mlp_forward(OM.bf16_to_f64(wl.x_host[r:r + b]), Ws[f])
        t_inv += time.perf_counter() - t0
        n_inv += 1
    del Ws
    step_s = t_reg + len(wl.requests) * t_inv / n_inv
    cores, nproc, cpu = _host_cpu()
    return {"value": len(wl.requests) / step_s, "unit": "invocations/s", "cores": cores, "kind": "oracle",
            "nproc": nproc, "cpu_model": cpu, "blas_threads": cores,
            "sample": f"fingerprints + cross-function dedup map of all {wl.n_fns} functions (4 x 256 MiB, "
                      f"{t_reg:.1f} s) and {n_inv} invocations of the workload's requests in order "
                      f"({t_inv:.1f} s) in float64 numpy; step = registrations + {len(wl.requests)} x mean "
                      f"invocation ({step_s:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # one-off runtime costs (a stall of tens of ms somewhere in the first 25
    # steps of a process) belong in the warmup, not in the timed mean
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-kernels", action="store_true", help="skip the standalone 4 GiB kernel bandwidth runs")
    ap.add_argument("--no-host-link", action="store_true", help="skip the host-memory registration runs")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--only-shared", action="store_true",
                    help="time the shared+batched steps only (for counter runs); no plain path or extras")
    ap.add_argument("--workload", default="sharing",
                    help="sharing (default) | batching | stencil | mlp_f32 | serving | exit_stages | rw_only | progressive")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (this path has no "
              f"multi-GPU form: it would shard by function, each GPU with its own pool)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2404_14691_amd import sage as S

    if args.workload != "sharing":
        import bench_workloads
        line = json.loads(bench_workloads.WORKLOADS[args.workload](S, torch, log))
        if not args.no_cpu:
            cb = cpu_baseline_workload(args.workload)
            if cb is not None:
                log("cpu baseline (oracle) done")
                line["cpu_baseline"] = cb
        print(json.dumps(line), flush=True)
        return

    log("generating workload")
    wl = Workload(torch)
    log(f"workload ready: {len(wl.requests)} requests, {wl.rows} rows")
    cfg = S.sage_config_default()
    cfg.pool_budget_bytes = 8 << 30
    # autotuner cache file, if one is named; otherwise tile timings stay in memory
    if os.environ.get("SAGE_TUNE_CACHE"):
        cfg.tune_cache = os.environ["SAGE_TUNE_CACHE"].encode()
    ctx = S.sage_open(0, cfg)
    pcfg = S.sage_config_default()
    pcfg.share = 0
    pcfg.pool_budget_bytes = 1 << 20
    pctx = S.sage_open(0, pcfg)
    try:
        stats = None
        # the fingerprint and block-copy kernels are timed over the warmup
        # steps; the timed steps time only the GEMM (each timed interval costs
        # event records on the host path)
        S.sage_timing_reset(ctx)
        S.sage_timing_enable(ctx, True)
        warm_steps = 0
        for i in range(args.warmup):
            stats = shared_step(S, ctx, wl, want_stats=True)[1]
            warm_steps += 1
            log(f"warmup step {i} done")
        if stats is None:  # no warmup asked for: one untimed step for the pool accounting
            stats = shared_step(S, ctx, wl, want_stats=True)[1]
            warm_steps += 1
        S.sage_timing_enable(ctx, False)
        f_ms, f_n = S.sage_timing_get(ctx, "fp64k")
        b_ms, b_n = S.sage_timing_get(ctx, "blkcopy")
        if not args.only_shared:
            plain_step(S, pctx, wl)
            log("plain warmup done")
        # ---- timed: shared + batched, with the GEMM's device time
        S.sage_timing_reset(ctx)
        S.sage_timing_only(ctx, "ggemm_bf16")
        S.sage_timing_enable(ctx, True)
        st0 = S.sage_get_stats(ctx)
        elapsed, res = timed(torch, lambda: shared_step(S, ctx, wl), args.steps)
        st1 = S.sage_get_stats(ctx)
        S.sage_timing_enable(ctx, False)
        S.sage_timing_only(ctx, None)
        host = {k: round((st1[k] - st0[k]) / args.steps, 3) for k in st1 if k.startswith("t_")}
        log(f"shared timed: {elapsed * 1e3 / args.steps:.2f} ms/step")
        setup_shared = [x for r in res for x in r[0]]
        g_ms, g_n = S.sage_timing_get(ctx, "ggemm_bf16")
        plan = S.sage_last_launch(ctx)
        # the MFMA ceiling of the main tile shape at the clock this load sustains
        # (outside the timed region; context for the roofline, not part of a step)
        ceil_us, ceil_ghz = S.sage_mfma_ceiling(ctx, wl.width, 20)
        ceil_cus = torch.cuda.get_device_properties(0).multi_processor_count  # one workgroup per CU
        # ---- plain
        if args.only_shared:
            p_elapsed, setup_plain = None, []
        else:
            p_elapsed, p_res = timed(torch, lambda: plain_step(S, pctx, wl), args.plain_steps)
            setup_plain = [x for r in p_res for x in r]
            log(f"plain timed: {p_elapsed * 1e3 / args.plain_steps:.2f} ms/step")
        standalone = None if (args.no_kernels or args.only_shared) else kernel_bandwidth(S, ctx, torch)
        if standalone:
            log(f"standalone kernels: {standalone}")
    finally:
        S.sage_close(ctx)
        S.sage_close(pctx)

    n_req = len(wl.requests)
    ms_step = elapsed / args.steps * 1e3
    value = n_req * args.steps / elapsed
    plain_value = n_req * args.plain_steps / p_elapsed if p_elapsed else None
    flops_launch = 2.0 * wl.rows * wl.width * wl.width
    gemm_avg_ms = g_ms / max(g_n, 1)
    achieved = flops_launch / (gemm_avg_ms * 1e-3) / 1e12
    traffic = traffic_record(plan)
    ceil_flops = 2.0 * ceil_cus * 256 * 256 * wl.width
    ceil_tflops = ceil_flops / (ceil_us * 1e-6) / 1e12
    mfma_ceiling = {
        "what": "the main 256x256 tile shape without its global loads (LDS ring filled once with random BF16; "
                "same fragment reads, MFMAs, barriers), one tile per CU (sage_mfma_ceiling)",
        "us_per_launch": round(ceil_us, 2), "achieved": round(ceil_tflops, 1),
        "frac_of_peak": round(ceil_tflops / BF16_PEAK_TFLOPS, 4), "shader_ghz": round(ceil_ghz, 3),
        "layer_frac_of_ceiling": round(achieved / ceil_tflops, 4)}
    fp_bytes = (sum(b.numel() for b in wl.dev_blobs) + 8 * sum(b.numel() for b in wl.dev_blobs) // 65536)
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "invocations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {
            "workload": "sharing: 4 functions x 8-layer BF16 MLP width 4096 (256 MiB read-only each, 30% of "
                        "64 KiB blocks identical across functions), 64 invocations per function, batch U[1,32], "
                        "sources and inputs resident in HBM",
            "requests_per_step": n_req, "rows_per_step": wl.rows},
        "setup_ms": {
            "shared": {"p50": round(percentile(setup_shared, 50), 4), "p99": round(percentile(setup_shared, 99), 3)},
            "plain": {"p50": round(percentile(setup_plain, 50), 4),
                      "p99": round(percentile(setup_plain, 99), 3)} if setup_plain else None},
        "plain": {"value": round(plain_value, 2), "ms_per_step": round(p_elapsed / args.plain_steps * 1e3, 3),
                  "steps": args.plain_steps} if plain_value else None,
        "speedup_vs_plain": round(value / plain_value, 2) if plain_value else None,
        "pool": {"logical_bytes": stats["logical_bytes"], "unique_bytes": stats["unique_bytes"],
                 "shared_bytes": stats["shared_bytes"], "private_bytes": stats["private_bytes"]},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / BF16_PEAK_TFLOPS, 4),
                     "traffic": traffic["hbm_bytes_per_layer"] if traffic else None,
                     "kernel": "grouped BF16 GEMM layer: " + plan, "avg_launch_ms": round(gemm_avg_ms, 5),
                     "mfma_ceiling": mfma_ceiling,
                     "launch": "one layer (main launch + thin-tile tail launch when split)",
                     "flop_per_launch": flops_launch,
                     "traffic_source": os.path.relpath(TRAFFIC_RECORD, ROOT) if traffic else None},
        "kernels": {
            "fp64k": {"avg_ms": round(f_ms / max(f_n, 1), 5), "launches": f_n, "steps": warm_steps,
                      "GB/s": round(fp_bytes * warm_steps / max(f_ms * 1e-3, 1e-12) / 1e9, 1)},
            # every block of a registration is either COPYed into a new slot or
            # VERIFYed against its class: 2 x 64 KiB moved per block either way
            "blkcopy": {"avg_ms": round(b_ms / max(b_n, 1), 5), "launches": b_n, "steps": warm_steps,
                        "GB/s": round(2 * sum(b.numel() for b in wl.dev_blobs) * warm_steps / max(b_ms * 1e-3, 1e-12)
                                      / 1e9, 1)},
            "ggemm_bf16": {"avg_ms": round(gemm_avg_ms, 5), "launches": g_n}},
        "kernels_standalone_4GiB": standalone,
        "host_ms_per_step": host,
    }
    if not args.no_serving and not args.only_shared:
        log("serving leg ...")
        line["serving_host_sourced"] = serving_leg(S, torch)
    if not args.no_host_link and not args.only_shared:
        log("host-sourced shared vs plain ...")
        line["host_sourced"] = host_sourced(S, torch, wl)
        line["host_sourced"]["cold_setup_ab"] = cold_setup_ab(S, wl)
        log(f"cold setup A/B: {line['host_sourced']['cold_setup_ab']}")
        log("host-link registration runs ...")
        line["host_link_not_headline"] = host_link(S, torch, wl)
        log(f"host link: {line['host_link_not_headline']}")
    if not args.no_cpu and not args.only_shared:
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
