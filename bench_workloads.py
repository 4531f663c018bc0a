"""Secondary benchmark workloads, run through `bench.py --workload NAME`.

batching : 1 function, 8-layer BF16 MLP width 4096, 256 invocations with
           lognormal batch sizes (median 8, clipped 1..128) in one group.
stencil  : 7-point FP32 stencil on 512^3 with a shared 512 MiB coefficient
           grid, 32 invocations x 20 Jacobi sweeps.
mlp_f32  : 2-layer FP32 MLP 2048x2048, 16 sequential invocations of 8 rows,
           weights and inputs in host memory.
serving  : open-loop Poisson arrivals over 16 BF16 MLP functions with sizes
           lognormal in [64 MiB, 4 GiB], 20 % block overlap, pool budget
           below the unique bytes (admission + eviction), rates
           200/500/1000/2000 requests/s.
Each prints one JSON line with the same top-level fields as bench.py.
"""
from __future__ import annotations

import json
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0


def _pct(v, q):
    s = sorted(v)
    k = max(1, int(np.ceil(q / 100.0 * len(s))))
    return s[k - 1]


def _line(metric, value, unit, steps, warmup, ms, config, dtype, **extra):
    d = {"metric": metric, "value": round(value, 2), "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
         "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
         "dtype": dtype, "data": "synthetic", "config": config}
    d.update(extra)
    return json.dumps(d)


# ---------------------------------------------------------------- batching
def batching(S, torch, log, steps=10, warmup=2):
    from paper_2404_14691_amd import synth
    W, L = 4096, 8
    w = synth.shared_mlp_bf16_functions(n_fns=1, layers=L, width=W, share_frac=0.0, seed=3)
    dev = torch.from_numpy(w.blobs[0].view(np.uint8)).cuda()
    batches = [int(b) for b in synth.lognormal_batches(256, seed=3)]
    rows = sum(batches)
    x = torch.zeros((rows, W), dtype=torch.bfloat16, device="cuda").normal_()
    y = torch.zeros((rows, W), dtype=torch.float32, device="cuda")
    offs = np.concatenate([[0], np.cumsum(batches)[:-1]])
    ins = [(x.data_ptr() + int(o) * W * 2, b * W * 2) for o, b in zip(offs, batches)]
    outs = [(y.data_ptr() + int(o) * W * 4, b * W * 4) for o, b in zip(offs, batches)]
    io = S.SAGE_IO_DEVICE_IN | S.SAGE_IO_DEVICE_OUT
    desc = S.mlp_desc(S.SAGE_MLP_BF16, L, W)
    blob = [S.make_blob(dev.data_ptr(), dev.numel(), where=S.SAGE_SRC_DEVICE)]
    torch.cuda.synchronize()

    def shared(ctx):
        t0 = time.perf_counter()
        fn = S.fn_register(ctx, desc, blob)
        reg = (time.perf_counter() - t0) * 1e3
        # the requests arrive together: one admission call, each request's own time
        invs, setup = S.fn_setup_batch(ctx, [fn] * len(batches), batches, timed=True)
        setup[0] += reg
        S.fn_invoke_batch(ctx, invs, ins, outs, io)
        S.fn_release_batch(ctx, invs)
        S.fn_unregister(ctx, fn)
        return setup

    def plain(ctx):
        t0 = time.perf_counter()
        fn = S.fn_register(ctx, desc, blob)
        reg = (time.perf_counter() - t0) * 1e3
        setup = []
        for i, b in enumerate(batches):
            t0 = time.perf_counter()
            inv = S.fn_setup(ctx, fn, b)
            setup.append((time.perf_counter() - t0) * 1e3 + (reg if i == 0 else 0))
            S.fn_invoke(ctx, inv, ins[i], outs[i], io)
            S.fn_release(ctx, inv)
        S.fn_unregister(ctx, fn)
        return setup

    cfg = S.sage_config_default()
    cfg.pool_budget_bytes = 1 << 30
    ctx = S.sage_open(0, cfg)
    pcfg = S.sage_config_default()
    pcfg.share = 0
    pcfg.pool_budget_bytes = 1 << 20
    pctx = S.sage_open(0, pcfg)
    try:
        for _ in range(warmup):
            shared(ctx)
        plain(pctx)
        S.sage_timing_reset(ctx)
        S.sage_timing_only(ctx, "ggemm_bf16")  # the one kernel this line reports
        S.sage_timing_enable(ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [shared(ctx) for _ in range(steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        S.sage_timing_enable(ctx, False)
        g_ms, g_n = S.sage_timing_get(ctx, "ggemm_bf16")
        plan = S.sage_last_launch(ctx)
        t0 = time.perf_counter()
        pres = [plain(pctx)]
        torch.cuda.synchronize()
        pel = time.perf_counter() - t0
    finally:
        S.sage_close(ctx)
        S.sage_close(pctx)
    su = [v for r in res for v in r]
    ps = [v for r in pres for v in r]
    avg = g_ms / max(g_n, 1)
    ach = 2.0 * rows * W * W / (avg * 1e-3) / 1e12
    value = 256 * steps / el
    return _line("setup p50/p99 ms + invocations/sec, shared+batched vs plain, 1 MI355X", value, "invocations/s",
                 steps, warmup, el / steps * 1e3,
                 {"workload": "batching: 1 function, 8-layer BF16 MLP width 4096, 256 invocations, batch "
                              "lognormal(median 8) clipped 1..128, one grouped launch per layer", "rows": rows},
                 "bf16",
                 setup_ms={"shared": {"p50": round(_pct(su, 50), 4), "p99": round(_pct(su, 99), 3)},
                           "plain": {"p50": round(_pct(ps, 50), 4), "p99": round(_pct(ps, 99), 3)}},
                 plain={"value": round(256 / pel, 2), "ms_per_step": round(pel * 1e3, 2)},
                 speedup_vs_plain=round(value / (256 / pel), 2),
                 roofline={"bound": "mfma", "achieved": round(ach, 2), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": round(ach / BF16_PEAK_TFLOPS, 4), "traffic": None,
                           "kernel": "grouped BF16 GEMM layer: " + plan, "avg_launch_ms": round(avg, 5)})


# ---------------------------------------------------------------- stencil
def stencil(S, torch, log, steps=2, warmup=1, n=512, n_inv=32, sweeps=20):
    from paper_2404_14691_amd import synth
    c = synth.stencil_coefficients(n, seed=0)
    dc = torch.from_numpy(c).cuda()
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    fields = [torch.randn((n, n, n), generator=g, device="cuda") for _ in range(n_inv)]
    outs = [torch.empty_like(f) for f in fields]
    io = S.SAGE_IO_DEVICE_IN | S.SAGE_IO_DEVICE_OUT
    fb = n * n * n * 4
    desc = S.stencil_desc(n, n, n, sweeps)
    blob = [S.make_blob(dc.data_ptr(), dc.numel() * 4, where=S.SAGE_SRC_DEVICE)]
    ins = [(f.data_ptr(), fb) for f in fields]
    ous = [(o.data_ptr(), fb) for o in outs]
    torch.cuda.synchronize()

    def shared(ctx):
        fn = S.fn_register(ctx, desc, blob)
        invs = S.fn_setup_batch(ctx, [fn] * n_inv, [1] * n_inv)
        S.fn_invoke_batch(ctx, invs, ins, ous, io)
        S.fn_release_batch(ctx, invs)
        S.fn_unregister(ctx, fn)

    def plain(ctx):
        fn = S.fn_register(ctx, desc, blob)
        for i in range(n_inv):
            inv = S.fn_setup(ctx, fn, 1)
            S.fn_invoke(ctx, inv, ins[i], ous[i], io)
            S.fn_release(ctx, inv)
        S.fn_unregister(ctx, fn)

    cfg = S.sage_config_default()
    cfg.pool_budget_bytes = 1 << 30
    ctx = S.sage_open(0, cfg)
    pcfg = S.sage_config_default()
    pcfg.share = 0
    pcfg.pool_budget_bytes = 1 << 20
    pctx = S.sage_open(0, pcfg)
    try:
        for _ in range(warmup):
            shared(ctx)
        S.sage_timing_reset(ctx)
        S.sage_timing_only(ctx, "stencil7")  # the one kernel this line reports
        S.sage_timing_enable(ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            shared(ctx)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        S.sage_timing_enable(ctx, False)
        k_ms, k_n = S.sage_timing_get(ctx, "stencil7")
        plain(pctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain(pctx)
        torch.cuda.synchronize()
        pel = time.perf_counter() - t0
    finally:
        S.sage_close(ctx)
        S.sage_close(pctx)
    cells = n ** 3
    # the timer counts sweeps (a pass of two sweeps is two units): avg is the
    # time per sweep over all 32 fields, alg the algorithmic bytes of one sweep
    avg = k_ms / max(k_n, 1)
    alg = n_inv * cells * 8 + cells * 4           # u read + u' written per field, c once
    gbs = alg / (avg * 1e-3) / 1e9
    value = n_inv * steps / el
    return _line("invocations/sec, shared+batched vs plain, 1 MI355X", value, "invocations/s", steps, warmup,
                 el / steps * 1e3,
                 {"workload": "stencil: 7-point FP32 Jacobi on 512^3, shared 512 MiB coefficient grid, 32 "
                              "invocations x 20 sweeps, one launch per pass of two sweeps for all fields"},
                 "f32", plain={"value": round(n_inv / pel, 3), "ms_per_step": round(pel * 1e3, 2)},
                 speedup_vs_plain=round(value / (n_inv / pel), 2),
                 roofline={"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                           "kernel": "stencil7_fused2 (two sweeps per pass; per-sweep time and bytes)",
                           "avg_sweep_ms": round(avg, 4), "bytes_per_sweep": alg})


# ---------------------------------------------------------------- FP32 MLP
def mlp_f32(S, torch, log, reps=5):
    from paper_2404_14691_amd import synth
    wl = synth.mlp_f32_workload()
    blob = wl.weights.reshape(-1)
    desc = S.mlp_desc(S.SAGE_MLP_F32, 2, 2048)
    res = {}
    k_ms = k_n = 0
    for name, share in (("shared", 1), ("plain", 0)):
        cfg = S.sage_config_default()
        cfg.share = share
        cfg.pool_budget_bytes = 256 << 20
        ctx = S.sage_open(0, cfg)
        try:
            times, lat = [], []
            for r in range(reps + 1):
                if share and r == 1:  # device time of the layer launches over the timed passes
                    S.sage_timing_reset(ctx)
                    S.sage_timing_only(ctx, "mlp_f32")  # the one kernel this line reports
                    S.sage_timing_enable(ctx, True)
                y = np.zeros((8, 2048), dtype=np.float32)
                t0 = time.perf_counter()
                fn = S.fn_register(ctx, desc, [S.make_blob(blob)])
                one = []
                for x in wl.inputs:
                    t1 = time.perf_counter()
                    inv = S.fn_setup(ctx, fn, 8)
                    S.fn_invoke(ctx, inv, x, y)
                    S.fn_release(ctx, inv)
                    one.append((time.perf_counter() - t1) * 1e3)
                S.fn_unregister(ctx, fn)
                if r:
                    times.append(time.perf_counter() - t0)
                    lat += one
            res[name] = {"ms_16_invocations": round(min(times) * 1e3, 3), "invocation_ms_p50": round(_pct(lat, 50), 4),
                         "invocation_ms_p99": round(_pct(lat, 99), 4)}
            if share:
                S.sage_timing_enable(ctx, False)
                k_ms, k_n = S.sage_timing_get(ctx, "mlp_f32")
        finally:
            S.sage_close(ctx)
    value = 16 / (res["shared"]["ms_16_invocations"] * 1e-3)
    # one launch is one layer of one invocation: 2048^2 FP32 weights read,
    # 8 rows of input read and of output written
    avg = k_ms / max(k_n, 1)
    alg = 2048 * 2048 * 4 + 2 * 8 * 2048 * 4
    gbs = alg / (avg * 1e-3) / 1e9 if k_n else 0.0
    return _line("invocations/sec, shared vs plain, 1 MI355X", value, "invocations/s", reps, 1,
                 res["shared"]["ms_16_invocations"],
                 {"workload": "mlp_f32: 2-layer FP32 MLP 2048x2048 (32 MiB weights in host memory), 16 sequential "
                              "invocations of 8 rows, host inputs/outputs; includes fn_register"},
                 "f32", detail=res,
                 speedup_vs_plain=round(res["plain"]["ms_16_invocations"] / res["shared"]["ms_16_invocations"], 2),
                 roofline={"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "mlp_f32_layer (4 output columns per workgroup, K split over its waves)",
                           "avg_launch_ms": round(avg, 5), "bytes_per_launch": alg, "launches": k_n})


# ---------------------------------------------------------------- serving
class ServingBench:
    """Serving at the over-HBM regime of the Poisson workload, shared against
    plain on one arrival trace.

    16 BF16 MLP functions of width 4096 (sizes lognormal 64 MiB..4 GiB, 20 %
    of blocks from a common pool), sources in pinned host memory, so every
    reload after an eviction crosses the host link; pool budget half of the
    unique bytes (the functions' read-only data cannot all stay in HBM);
    Poisson arrivals, Zipf(1) popularity, batch U[1,64], each request with its
    own seeded input.  Shared: pool + references + eviction + continuous
    batching, reloads issued without waiting (the launch waits for them).
    Plain: the same loop with a private copy of the function's weights per
    request, on the first `plain_prefix_s` seconds of the same trace (at these
    rates its queue grows without bound).  The plain requests' outputs are
    compared bit for bit with the same requests' outputs in the shared run."""

    W = 4096

    def __init__(self, S, torch, log, budget_frac=0.5, seed=1000):
        from paper_2404_14691_amd import synth
        self.S, self.torch, self.log, self.seed = S, torch, log, seed
        self.layers = synth.serving_workload(rate=1.0, duration=1.0, seed=seed).layers
        W = self.W
        self.sizes = [l * W * W * 2 for l in self.layers]
        g = torch.Generator(device="cuda")
        g.manual_seed(0)
        self.g = g
        per = 32768
        common = (torch.randn((max(self.sizes) // 65536, per), generator=g, device="cuda") / 64.0).to(torch.bfloat16)
        self.dev_blobs = []
        for nbytes in self.sizes:
            nb = nbytes // 65536
            b = (torch.randn((nb, per), generator=g, device="cuda") / 64.0).to(torch.bfloat16)
            share = torch.rand(nb, generator=g, device="cuda") < 0.2
            b[share] = common[:nb][share]
            self.dev_blobs.append(b)
        del common
        torch.cuda.synchronize()
        cfg = S.sage_config_default()
        cfg.pool_budget_bytes = 1 << 40
        ctx = S.sage_open(0, cfg)
        try:
            for l, b in zip(self.layers, self.dev_blobs):
                S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, l, W),
                              [S.make_blob(b.data_ptr(), b.numel() * 2, where=S.SAGE_SRC_DEVICE)])
            self.unique = S.sage_get_stats(ctx)["unique_bytes"]
        finally:
            S.sage_close(ctx)
        self.budget_frac = budget_frac
        self.budget = int(self.unique * budget_frac) // 65536 * 65536
        self.logical = sum(self.sizes)

    def close(self):
        del self.dev_blobs
        self.torch.cuda.empty_cache()

    def _run(self, share, wl, reqs, x, y, row0, rows, budget):
        S, torch, W = self.S, self.torch, self.W
        cfg = S.sage_config_default()
        cfg.share = share
        cfg.pool_budget_bytes = budget
        cfg.progressive = 1 if share else 0
        io = S.SAGE_IO_DEVICE_IN | S.SAGE_IO_DEVICE_OUT
        ctx = S.sage_open(0, cfg)
        try:
            host = []
            for b in self.dev_blobs:
                a = S.pinned_array(ctx, (b.numel(),), np.uint16)
                torch.from_numpy(a.view(np.int16)).copy_(b.view(torch.int16).reshape(-1))
                host.append(a)
            fns = [S.fn_register(ctx, S.mlp_desc(S.SAGE_MLP_BF16, l, W), [S.make_blob(a)])
                   for l, a in zip(self.layers, host)]
            st0 = S.sage_get_stats(ctx)
            S.sage_serve_start(ctx)
            ids = []
            t0 = time.perf_counter()
            for i in reqs:
                while time.perf_counter() - t0 < wl.arrivals[i]:
                    pass
                r, b = int(row0[i]), int(rows[i])
                ids.append(S.sage_submit(ctx, fns[int(wl.fn[i])], b, (x.data_ptr() + r * W * 2, b * W * 2),
                                         (y.data_ptr() + r * W * 4, b * W * 4), io))
            for r in ids:
                S.sage_wait(ctx, r, 600000)
            rep = S.sage_serve_stats(ctx)
            S.sage_serve_stop(ctx)
            st1 = S.sage_get_stats(ctx)
            for f in fns:
                S.fn_unregister(ctx, f)
            for a in host:
                S.sage_host_free(ctx, a.ctypes.data)
        finally:
            S.sage_close(ctx)
        return {"requests": len(reqs), "completed": int(rep["completed"]), "failed": int(rep["failed"]),
                "throughput": round(rep["throughput"], 1),
                "setup_ms": {"p50": round(rep["setup_p50_ms"], 3), "p99": round(rep["setup_p99_ms"], 3)},
                "e2e_ms": {"p50": round(rep["e2e_p50_ms"], 3), "p99": round(rep["e2e_p99_ms"], 3)},
                "launches": int(rep["launches"]), "evictions": int(st1["evictions"] - st0["evictions"]),
                "reloads": int(st1["reloads"] - st0["reloads"]),
                "h2d_ro_bytes": int(st1["h2d_bytes"] - st0["h2d_bytes"])}

    def rate(self, rate, duration, plain_prefix_s=0.25):
        from paper_2404_14691_amd import synth
        torch, W = self.torch, self.W
        wl = synth.serving_workload(rate=rate, duration=duration, seed=self.seed)
        assert wl.layers == self.layers
        n = len(wl.arrivals)
        rows = np.asarray(wl.batch, dtype=np.int64)
        row0 = np.concatenate([[0], np.cumsum(rows)[:-1]])
        total_rows = int(rows.sum())
        x = torch.empty((total_rows, W), dtype=torch.bfloat16, device="cuda")
        for r in range(0, total_rows, 65536):  # distinct seeded inputs, generated in pieces
            k = min(65536, total_rows - r)
            x[r:r + k] = torch.randn((k, W), generator=self.g, device="cuda").to(torch.bfloat16)
        y_shared = torch.empty((total_rows, W), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        self.log(f"serving {rate:.0f}/s for {duration:.0f} s: {n} requests, shared ...")
        shared = self._run(1, wl, list(range(n)), x, y_shared, row0, rows, self.budget)
        self.log(f"serving {rate:.0f}/s shared: {shared}")
        prefix = [i for i in range(n) if wl.arrivals[i] < plain_prefix_s]
        last = int(row0[prefix[-1]] + rows[prefix[-1]]) if prefix else 0
        y_plain = torch.full((max(last, 1), W), float("nan"), dtype=torch.float32, device="cuda")
        plain = self._run(0, wl, prefix, x, y_plain, row0, rows, 1 << 20)
        self.log(f"serving {rate:.0f}/s plain: {plain}")
        same = bool(torch.equal(y_plain[:last], y_shared[:last])) if last else None
        del x, y_shared, y_plain
        torch.cuda.empty_cache()
        return {"workload": f"Poisson {rate:.0f} req/s for {duration:.0f} s over 16 BF16 MLP functions (width "
                            f"4096, {self.logical / 2**30:.2f} GiB logical, {self.unique / 2**30:.2f} GiB unique, "
                            f"20% block overlap), batch U[1,64], Zipf(1) popularity, sources in pinned host "
                            f"memory, distinct inputs",
                "pool_budget_bytes": self.budget,
                "budget_note": f"{self.budget_frac:.0%} of unique bytes: not all read-only data fits, so admission "
                               f"evicts and reloads over the host link",
                "shared_batched": shared,
                "plain": dict(plain, trace=f"the first {plain_prefix_s} s of the same trace ({len(prefix)} requests)"),
                "plain_outputs_equal_shared": same,
                "speedup_vs_plain": round(shared["throughput"] / max(plain["throughput"], 1e-9), 2)}


def serving(S, torch, log, rates=(200, 500, 1000, 2000), duration=60.0):
    """Every rate of the serving configuration for 60 s each, shared against
    plain (ServingBench)."""
    sb = ServingBench(S, torch, log)
    results = {}
    try:
        for rate in rates:
            results[str(rate)] = sb.rate(float(rate), duration)
    finally:
        sb.close()
    top = results[str(rates[-1])]
    return _line("setup/e2e p50/p99 ms + invocations/sec under Poisson load, shared vs plain, 1 MI355X",
                 top["shared_batched"]["throughput"], "invocations/s", len(rates), 0, 0.0,
                 {"workload": top["workload"].replace(f"{rates[-1]} req/s", "200-2000 req/s"),
                  "unique_bytes": int(sb.unique), "pool_budget_bytes": int(sb.budget)},
                 "bf16", rates=results)


# ---------------------------------------------------------------- exit stages
def exit_stages(S, torch, log, interval_ms=300.0, reps=3, batch=8):
    """Table 4 analogue: setup + invoke latency of one BF16 MLP (8 x 4096^2,
    256 MiB in pageable host memory) in each multi-stage exit stage and cold
    (a new context: code object, registration and all).  The stage is applied
    (sage_tick) before each timed call, as the paper's exit runs in the
    background."""
    from paper_2404_14691_amd import synth
    W, L = 4096, 8
    w = synth.shared_mlp_bf16_functions(n_fns=1, layers=L, width=W, share_frac=0.0, seed=5)
    blob = w.blobs[0]
    desc = S.mlp_desc(S.SAGE_MLP_BF16, L, W)
    x = synth.bf16_inputs(batch, W, 5, 0)
    y = np.zeros((batch, W), dtype=np.float32)
    keys = ("t_module_ms", "t_reload_ms", "t_setup_ms", "t_invoke_ms")

    def one(ctx, fn):
        st0 = S.sage_get_stats(ctx)
        t0 = time.perf_counter()
        inv = S.fn_setup(ctx, fn, batch)
        S.fn_invoke(ctx, inv, x, y)
        S.fn_release(ctx, inv)
        e2e = (time.perf_counter() - t0) * 1e3
        st1 = S.sage_get_stats(ctx)
        return e2e, {k: st1[k] - st0[k] for k in keys}, time.monotonic()

    def cfg(serial=0):
        c = S.sage_config_default()
        c.pool_budget_bytes = 2 << 30
        c.exit_stage_ms = interval_ms
        c.serial_setup = serial
        return c

    rows = {k: [] for k in ("stage1", "stage2", "stage3", "stage4", "cold", "cold_serial")}
    parts = {k: [] for k in rows}
    def cold(serial):
        t0 = time.perf_counter()
        c = S.sage_open(0, cfg(serial))
        f = S.fn_register(c, desc, [S.make_blob(blob)])
        inv = S.fn_setup(c, f, batch)
        S.fn_invoke(c, inv, x, y)
        S.fn_release(c, inv)
        return (time.perf_counter() - t0) * 1e3, c, f

    for r in range(reps):
        ms, c2, f2 = cold(1)
        rows["cold_serial"].append(ms)
        S.fn_unregister(c2, f2)
        S.sage_close(c2)
        ms, ctx, fn = cold(0)  # this context and function stay for the warm stages
        rows["cold"].append(ms)
        _, _, t_rel = one(ctx, fn)
        for k, idle in (("stage1", 0.3), ("stage2", 1.3), ("stage3", 2.3), ("stage4", 3.3)):
            dt = t_rel + idle * interval_ms / 1e3 - time.monotonic()
            if dt > 0:
                time.sleep(dt)
            S.sage_tick(ctx)
            e2e, br, t_rel = one(ctx, fn)
            rows[k].append(e2e)
            parts[k].append(br)
        S.fn_unregister(ctx, fn)
        S.sage_close(ctx)
        log(f"exit stages rep {r}: " + ", ".join(f"{k} {v[-1]:.2f} ms" for k, v in rows.items()))
    med = {k: float(np.median(v)) for k, v in rows.items()}
    breakdown = {k: {kk: round(float(np.median([p[kk] for p in parts[k]])), 3) for kk in keys}
                 for k in ("stage1", "stage2", "stage3", "stage4")}
    gain = float(np.mean([med["cold"] / med[k] for k in ("stage1", "stage2", "stage3", "stage4")]))
    return _line("setup+invoke latency per multi-stage exit stage vs cold (Table 4 analogue), 1 MI355X", gain,
                 "x mean speedup of stages 1-4 over cold", reps, 0, med["stage1"],
                 {"workload": "exit stages: 1 BF16 MLP 8 x 4096^2 (256 MiB, pageable host source), batch 8, host "
                              f"I/O, stage interval {interval_ms:.0f} ms; cold = new context + code object + "
                              "registration + first invocation"},
                 "bf16", e2e_ms={k: round(v, 3) for k, v in med.items()}, breakdown_ms=breakdown)


# ---------------------------------------------------------------- RW-only function
def rw_only(S, torch, log, reps=3, n_inv=8, nx=512, ny=512, nz=320, sweeps=20, coef=0.5):
    """A function with no read-only data (the paper's lbm: Table 2, 0 MB
    read-only, 330 MB writable; "cannot benefit" from memory sharing): the
    relaxation kind over a 512 x 512 x 320 FP32 field (335 MB) passed from
    pageable host memory, 20 sweeps, result back to host memory.  Shared and
    plain contexts do the same work; a cold run opens a new context (code
    object and all) per invocation."""
    from paper_2404_14691_amd import synth
    shape = (nz, ny, nx)
    desc = S.relax_desc(nx, ny, nz, sweeps, coef)
    u = synth.stencil_field(0, 0, seed=7, shape=shape)
    out = np.empty_like(u)
    res = {}

    def warm(share):
        cfg = S.sage_config_default()
        cfg.share = share
        ctx = S.sage_open(0, cfg)
        try:
            fn = S.fn_register(ctx, desc, [])
            inv = S.fn_setup(ctx, fn, 1)
            S.fn_invoke(ctx, inv, u, out)  # warm-up: first launch of the kind
            S.fn_release(ctx, inv)
            ms = []
            for _ in range(n_inv):
                t0 = time.perf_counter()
                inv = S.fn_setup(ctx, fn, 1)
                S.fn_invoke(ctx, inv, u, out)
                S.fn_release(ctx, inv)
                ms.append((time.perf_counter() - t0) * 1e3)
            S.fn_unregister(ctx, fn)
            return float(np.median(ms))
        finally:
            S.sage_close(ctx)

    def cold():
        t0 = time.perf_counter()
        ctx = S.sage_open(0, S.sage_config_default())
        fn = S.fn_register(ctx, desc, [])
        inv = S.fn_setup(ctx, fn, 1)
        S.fn_invoke(ctx, inv, u, out)
        S.fn_release(ctx, inv)
        ms = (time.perf_counter() - t0) * 1e3
        S.fn_unregister(ctx, fn)
        S.sage_close(ctx)
        return ms

    runs = {"shared": [], "plain": [], "cold": []}
    for r in range(reps):
        runs["shared"].append(warm(1))
        runs["plain"].append(warm(0))
        runs["cold"].append(cold())
        log(f"rw_only rep {r}: " + ", ".join(f"{k} {v[-1]:.1f} ms" for k, v in runs.items()))
    med = {k: float(np.median(v)) for k, v in runs.items()}
    value = 1e3 / med["shared"]
    return _line("invocations/sec of a function without read-only data, shared vs plain, 1 MI355X", value,
                 "invocations/s", reps, 1, med["shared"],
                 {"workload": f"rw_only: relaxation {nx}x{ny}x{nz} FP32 ({nx * ny * nz * 4 / 1e6:.0f} MB writable, no "
                              f"read-only data), {sweeps} sweeps, field from and to pageable host memory"},
                 "f32", invocation_ms=med, speedup_vs_plain=round(med["plain"] / med["shared"], 3),
                 warm_vs_cold=round(med["cold"] / med["shared"], 3))


# ---------------------------------------------------------------- progressive setup
def progressive(S, torch, log, reps=5, batches=(8, 2048), interval_ms=250.0, rounds=5):
    """Per-kernel readiness: setup + invoke latency of one BF16 MLP
    (8 x 4096^2, 256 MiB) whose blocks must all come back, with the whole
    reload inside fn_setup (off) or with layer l's launch waiting only for
    layer l's copies (on).  Sources: the function's device memory, the pinned
    host cache (second exit stage) and its pageable host memory.  Device-side
    inputs and outputs; outputs of both modes are compared bit for bit.
    Each case runs `rounds` rounds, each a fresh context per mode (the
    median of `reps` timed setups), the mode order alternating from round to
    round; reported: the median and IQR over rounds per mode and of the
    paired difference off - on."""
    from paper_2404_14691_amd import synth
    W, L = 4096, 8
    fn_bytes = L * W * W * 2
    w = synth.shared_mlp_bf16_functions(n_fns=2, layers=L, width=W, share_frac=0.0, seed=8)
    dblobs = [torch.from_numpy(b.view(np.int16)).cuda() for b in w.blobs]
    desc = S.mlp_desc(S.SAGE_MLP_BF16, L, W)
    io = S.SAGE_IO_DEVICE_IN | S.SAGE_IO_DEVICE_OUT
    maxb = max(batches)
    x = torch.from_numpy(synth.bf16_inputs(maxb, W, 8, 0).view(np.int16)).cuda()
    outs = {}

    def run(ctx, fn, b, y):
        t0 = time.perf_counter()
        inv = S.fn_setup(ctx, fn, b)
        S.fn_invoke(ctx, inv, (x.data_ptr(), b * W * 2), (y.data_ptr(), b * W * 4), io)
        S.fn_release(ctx, inv)
        return (time.perf_counter() - t0) * 1e3

    def case(source, prog, b):
        cfg = S.sage_config_default()
        cfg.progressive = prog
        if source == "host_cache":
            cfg.pool_budget_bytes = 4 * fn_bytes
            cfg.exit_stage_ms = interval_ms
        else:
            cfg.pool_budget_bytes = fn_bytes  # one function: each setup evicts the other
        ctx = S.sage_open(0, cfg)
        y = torch.zeros((b, W), dtype=torch.float32, device="cuda")
        ms = []
        try:
            if source == "device":
                blobs = [S.make_blob(d.data_ptr(), fn_bytes, where=S.SAGE_SRC_DEVICE) for d in dblobs]
            else:
                blobs = [S.make_blob(a) for a in w.blobs]
            f = S.fn_register(ctx, desc, [blobs[0]])
            g = None if source == "host_cache" else S.fn_register(ctx, desc, [blobs[1]])
            for r in range(reps + 1):
                if g is None:
                    run(ctx, f, b, y)
                    time.sleep(1.3 * interval_ms / 1e3)
                    S.sage_tick(ctx)  # second stage: f's blocks are in the host cache
                else:
                    run(ctx, g, 1, y)  # g takes the pool: f's blocks are out
                torch.cuda.synchronize()
                t = run(ctx, f, b, y)
                if r:
                    ms.append(t)
            st = S.sage_get_stats(ctx)
            if source == "host_cache":
                assert st["host_reloads"] >= reps * w.n_blocks, st["host_reloads"]
            outs[(source, prog, b)] = y.clone()
        finally:
            S.sage_close(ctx)
        return float(np.median(ms))

    def q(v):
        return {"median": round(float(np.median(v)), 3),
                "iqr": [round(float(np.percentile(v, 25)), 3), round(float(np.percentile(v, 75)), 3)]}

    res = {}
    for source in ("device", "host_cache", "pageable"):
        for b in batches:
            offs, ons = [], []
            for k in range(rounds):
                order = (0, 1) if k % 2 == 0 else (1, 0)
                for prog in order:
                    (offs if prog == 0 else ons).append(case(source, prog, b))
            same = bool(torch.equal(outs[(source, 0, b)], outs[(source, 1, b)]))
            off, on = float(np.median(offs)), float(np.median(ons))
            res[f"{source}/b{b}"] = {"off_ms": q(offs), "on_ms": q(ons),
                                     "off_minus_on_ms": q([a - c for a, c in zip(offs, ons)]),
                                     "speedup": round(off / on, 3), "outputs_identical": same}
            log(f"progressive {source} b={b}: {res[f'{source}/b{b}']}")
            if not same:
                raise RuntimeError(f"progressive outputs differ: {source} b={b}")
    gmean = float(np.exp(np.mean([np.log(v["speedup"]) for v in res.values()])))
    return _line("cold setup+invoke e2e ms, per-layer readiness vs whole-reload setup, 1 MI355X", gmean,
                 "x geometric-mean speedup", rounds * reps, 1, res[f"host_cache/b{maxb}"]["on_ms"]["median"],
                 {"workload": f"progressive setup: 1 BF16 MLP 8 x 4096^2 (256 MiB), every block reloaded (from "
                              f"device memory, the pinned host cache, pageable host memory), batch {list(batches)}, "
                              f"device I/O; {rounds} rounds per case, mode order alternating, {reps} setups each"},
                 "bf16", cases=res)


WORKLOADS = {"batching": batching, "stencil": stencil, "mlp_f32": mlp_f32, "serving": serving,
             "exit_stages": exit_stages, "rw_only": rw_only,
             "progressive": progressive}
