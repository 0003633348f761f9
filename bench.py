#!/usr/bin/env python3
"""Benchmark: twisted-mass Dslash Gflop/s + HBM GB/s on one MI355X, and mixed vs
FP64 CG time to a 1e-10 residual.

Timed step = one application of the asymmetric even-odd preconditioned operator
of the non-degenerate doublet (Eq. 2.2 with the flavour-mixing twist of
Eq. 2.1; the operator and lattice of the paper's Table 1, non-degenerate
row): two fused hop kernels, FP32 storage and arithmetic, 12-real links,
32^3 x 64 lattice, kappa = 0.1615, mu = 0.15, epsilon = 0.19, near-unit SU(3)
links, inputs resident in HBM.  Flops per even site: 5808 (1320 per hop and
flavour, twist and xpay as counted in the design notes); algorithmic bytes per
even site: 16 L + 5 S (L = 48 B per stored link, S = 192 B per doublet site).
The working set (403 MB of links, three 201 MB spinor fields) is well above
the 256 MB last-level cache.

The per-kernel durations of the roofline come from HIP events recorded on the
library's stream between the two kernels of every timed step.

Also reported: the same operator in FP64 / FP16 / BF16 and for one flavour,
the 24^3 x 48 degenerate operator (warm and with the caches flushed), the FP64
CPU oracle on the host (one thread and all threads, at 24^3 x 48 and at
32^3 x 64, and a full FP64 CG on the 4^4 lattice), the 32^3 x 64 doublet CG
comparison (FP64 CG vs mixed precision with FP64 reliable updates) to a 1e-10
true residual, batched sources, uneven lattices and the force kernel.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tm Dslash Gflop/s + HBM GB/s; mixed vs FP64 CG time to 1e-10 residual"
PEAK_HBM_GBS = 8000.0
FLOPS_PER_SITE = {"deg_asym": 2808, "deg_sym": 2832, "nd": 5808}
BYTES_PER_REAL = {0: 8, 1: 4, 2: 2, 3: 2}     # FP64, FP32, FP16, BF16
HEADLINE_DIMS = (32, 32, 32, 64)
HEADLINE = dict(kappa=0.1615, mu=0.15, eps=0.19)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hop_traffic.json")
HOP_SOURCES = ("tm_hop.inc.h", "tm_impl.h", "tm_hop_fp32.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def link_bytes(prec, recon=12):
    return recon * BYTES_PER_REAL[prec]


def site_spinor_bytes(prec, nf):
    return (24 * BYTES_PER_REAL[prec] if prec in (0, 1) else 52) * nf


def site_bytes(L, S):
    """(K1, K2) algorithmic bytes per even site: K1 = 8L + 2S, K2 = 8L + 3S."""
    return 8 * L + 2 * S, 8 * L + 3 * S


def hop_source_hash():
    import hashlib
    csrc = os.path.join(ROOT, "paper_1311_4462_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read() for f in HOP_SOURCES)
    return hashlib.sha256(src).hexdigest()[:16]


def measured_traffic(workload):
    """HBM-side bytes per launch of the roofline kernel from the committed
    FETCH_SIZE / WRITE_SIZE summary (two rocprofv3 --pmc runs of this bench),
    or None if the kernel source or the workload changed since."""
    try:
        t = json.load(open(TRAFFIC_FILE))
        if t.get("workload") != workload or hop_source_hash() != t["source_sha256_16"]:
            return None
        return int(t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def time_launches(torch, fn, reps, warm=3):
    for _ in range(warm):          # first calls may run the tuner
        fn()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3   # seconds per launch


def time_cold(torch, fn, reps, flush_bytes=512 << 20):
    """Median per-call time with the caches flushed before each call: a read
    of 512 MB (twice the last-level cache) on the same stream, outside the
    timed interval, so the operator's fields come from HBM.  The flush only
    reads, so it leaves no dirty lines whose write-back the timed call would
    pay for."""
    buf = torch.ones(flush_bytes // 4, dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    fn()
    for _ in range(3):
        buf.sum()
    for e0, e1 in evs:
        buf.sum()
        e0.record(s)
        fn()
        e1.record(s)
    torch.cuda.synchronize()
    ts = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
    del buf
    return ts[len(ts) // 2] * 1e-3


def kernel_split(torch, api, ctx, g, p, prec, x, tmp, y, reps):
    """The asymmetric operator as its two ABI hop calls, with HIP events on the
    library's stream around each kernel: returns (K1 s, K2 s, step s)."""
    s = torch.cuda.current_stream()
    k2 = -p.kappa ** 2

    def k1_call():
        api.tm_dslash(ctx, tmp, x, g, prec, 1, 0, 0, api.EPI_TWINV, None, 0.0)

    def k2_call():
        api.tm_dslash(ctx, y, tmp, g, prec, 0, 0, 0, api.EPI_RX_PLUS_KD, x, k2)

    for _ in range(3):
        k1_call()
        k2_call()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps + 1)]
    torch.cuda.synchronize()
    ev[0].record(s)
    for r in range(reps):
        k1_call()
        ev[2 * r + 1].record(s)
        k2_call()
        ev[2 * r + 2].record(s)
    ev[-1].synchronize()
    t1 = [ev[2 * r].elapsed_time(ev[2 * r + 1]) * 1e-3 for r in range(reps)]
    t2 = [ev[2 * r + 1].elapsed_time(ev[2 * r + 2]) * 1e-3 for r in range(reps)]
    return sum(t1) / reps, sum(t2) / reps, ev[0].elapsed_time(ev[-1]) * 1e-3 / reps


def headline(torch, api, ctx, g, p, a):
    """Timed region: K steps of the FP32 doublet operator, each its two hop
    kernels with events between them, after W untimed steps."""
    import numpy as np
    nf = 2
    vh = int(np.prod(HEADLINE_DIMS)) // 2
    prec = api.FP32
    from paper_1311_4462_amd import inputs
    src = torch.from_numpy(inputs.gaussian_spinor(HEADLINE_DIMS, nf, 2003)).cuda()
    x = api.tm_spinor_pack(ctx, src[None], p, prec, 0)
    del src
    y = api.new_field(p, prec)
    tmp = api.new_field(p, prec)
    k2c = -p.kappa ** 2
    s = torch.cuda.current_stream()

    def step():
        api.tm_dslash(ctx, tmp, x, g, prec, 1, 0, 0, api.EPI_TWINV, None, 0.0)
        api.tm_dslash(ctx, y, tmp, g, prec, 0, 0, 0, api.EPI_RX_PLUS_KD, x, k2c)

    for _ in range(a.warmup):
        step()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * a.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(s)
    for r in range(a.steps):
        api.tm_dslash(ctx, tmp, x, g, prec, 1, 0, 0, api.EPI_TWINV, None, 0.0)
        ev[2 * r + 1].record(s)
        api.tm_dslash(ctx, y, tmp, g, prec, 0, 0, 0, api.EPI_RX_PLUS_KD, x, k2c)
        ev[2 * r + 2].record(s)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    t_k1 = sum(ev[2 * r].elapsed_time(ev[2 * r + 1]) for r in range(a.steps)) * 1e-3 / a.steps
    t_k2 = sum(ev[2 * r + 1].elapsed_time(ev[2 * r + 2]) for r in range(a.steps)) * 1e-3 / a.steps
    # the same operator through tm_mat_pc (one ABI call), and with the caches
    # flushed before each apply
    t_mat = time_launches(torch, lambda: api.tm_mat_pc(ctx, y, x, g, prec, api.ASYM, 0), a.kernel_reps)
    t_cold = time_cold(torch, step, 20)
    del x, y, tmp
    L, S = link_bytes(prec), site_spinor_bytes(prec, nf)
    b1, b2 = site_bytes(L, S)
    return dict(dt=dt, t_k1=t_k1, t_k2=t_k2, t_mat=t_mat, t_cold=t_cold, b1=b1, b2=b2, vh=vh)


def kernel_rates(torch, api, ctx, g, p, precs, reps, flops_site, recon=12):
    """Per precision: the asymmetric operator and its two kernels on a
    resident field: us, Gflop/s, algorithmic GB/s and fraction of peak."""
    import numpy as np
    nf = 2 if p.flavor == api.NDEG else 1
    vh = int(np.prod(tuple(p.dims))) // 2
    src = torch.randn(api.canonical_shape(p), dtype=torch.complex128, device="cuda")
    out = {}
    for prec in precs:
        x = api.tm_spinor_pack(ctx, src, p, prec, 0)
        y = api.new_field(p, prec)
        tmp = api.new_field(p, prec)
        t1, t2, _ = kernel_split(torch, api, ctx, g, p, prec, x, tmp, y, reps)
        t = time_launches(torch, lambda: api.tm_mat_pc(ctx, y, x, g, prec, api.ASYM, 0), reps)
        b1, b2 = site_bytes(link_bytes(prec, recon), site_spinor_bytes(prec, nf))
        out[api.PREC_NAMES[prec]] = {
            "us": round(t * 1e6, 1), "gflops": round(flops_site * vh / t / 1e9, 1),
            "gbs": round((b1 + b2) * vh / t / 1e9, 1),
            "frac": round((b1 + b2) * vh / t / 1e9 / PEAK_HBM_GBS, 4),
            "k1_us": round(t1 * 1e6, 1), "k1_frac": round(b1 * vh / t1 / 1e9 / PEAK_HBM_GBS, 4),
            "k2_us": round(t2 * 1e6, 1), "k2_frac": round(b2 * vh / t2 / 1e9 / PEAK_HBM_GBS, 4)}
        del x, y, tmp
    del src
    return out


def operator_variants(torch, api, ctx, U, p, reps):
    """us per apply of the preconditioned operator, asym / sym, with and without
    dagger, FP64 and FP32: one flavour with 18-, 12- and 8-real links, the other
    twist sign and the doublet with 12-real links; and the asymmetric
    twisted-clover apply."""
    Ut = torch.from_numpy(U).cuda()
    out = {}
    cases = [(api.PLUS, r, "") for r in (18, 12, 8)] + [(api.MINUS, 12, "_minus"), (api.NDEG, 12, "_nd")]
    for flavor, recon, tag in cases:
        pf = api.make_params(tuple(p.dims), p.kappa, p.mu, 0.19 if flavor == api.NDEG else 0.0, flavor)
        src = torch.randn(api.canonical_shape(pf), dtype=torch.complex128, device="cuda")
        g = api.Gauge(ctx, Ut, pf, recon=recon, precs=(api.FP64, api.FP32))
        for prec in (api.FP64, api.FP32):
            x = api.tm_spinor_pack(ctx, src, pf, prec, 0)
            y = api.new_field(pf, prec)
            row = {}
            for pc, pcn in ((api.ASYM, "asym"), (api.SYM, "sym")):
                for dag in (0, 1):
                    t = time_launches(torch, lambda: api.tm_mat_pc(ctx, y, x, g, prec, pc, dag), reps)
                    row[pcn + ("_dag" if dag else "")] = round(t * 1e6, 2)
            out[f"{api.PREC_NAMES[prec]}_r{recon}{tag}"] = row
            del x, y
        g.close()
    src = torch.randn(api.canonical_shape(p), dtype=torch.complex128, device="cuda")
    import numpy as np
    vh = int(np.prod(tuple(p.dims))) // 2
    pc = api.make_params(tuple(p.dims), p.kappa, p.mu, 0.0, p.flavor, csw=1.57)
    g = api.Gauge(ctx, Ut, pc, recon=12, precs=(api.FP64, api.FP32))
    for prec in (api.FP64, api.FP32):
        x = api.tm_spinor_pack(ctx, src, pc, prec, 0)
        y = api.new_field(pc, prec)
        t = time_launches(torch, lambda: api.tm_mat_pc(ctx, y, x, g, prec, api.ASYM, 0), reps)
        rb = 8 if prec == api.FP64 else 4
        byt = (16 * 12 * rb + 5 * 24 * rb + 6 * 36 * rb) * vh
        out[f"clover_{api.PREC_NAMES[prec]}_r12"] = {
            "asym_us": round(t * 1e6, 2), "gbs": round(byt / t / 1e9, 1),
            "bytes_per_site": byt // vh}
        del x, y
    g.close()
    del Ut, src
    log(f"operator variants (us): {out}")
    return out


def section_24(torch, api, inputs, a):
    """24^3 x 48 degenerate FP32 / FP64 operator: warm (its ~223 MB FP32 working
    set largely resident in the 256 MB last-level cache) and with the caches
    flushed; the operator variants."""
    import numpy as np
    dims = (24, 24, 24, 48)
    vh = int(np.prod(dims)) // 2
    p = api.make_params(dims, 0.1615, 0.004, 0.0, api.PLUS)
    log("bench: generating 24^3x48 links")
    U = inputs.gauge_field(dims, "near_unit", 1002)
    ctx = api.Context()
    ctx.set_tuning(True)
    g = api.Gauge(ctx, torch.from_numpy(U).cuda(), p, recon=12, precs=(api.FP64, api.FP32))
    b = inputs.gaussian_spinor(dims, 1, 2002)
    out = {"rates": kernel_rates(torch, api, ctx, g, p, (api.FP32, api.FP64), a.kernel_reps,
                                 FLOPS_PER_SITE["deg_asym"])}
    x = api.tm_spinor_pack(ctx, b[None], p, api.FP32, 0)
    y = api.new_field(p, api.FP32)
    t_cold = time_cold(torch, lambda: api.tm_mat_pc(ctx, y, x, g, api.FP32, api.ASYM, 0), 20)
    mb = (16 * 48 + 5 * 96) * vh
    out["fp32_cold"] = {"us": round(t_cold * 1e6, 2), "gbs": round(mb / t_cold / 1e9, 1),
                        "frac": round(mb / t_cold / 1e9 / PEAK_HBM_GBS, 4)}
    del x, y
    if not a.no_batch:
        out["variants_us"] = operator_variants(torch, api, ctx, U, p, a.kernel_reps)
    g.close()
    ctx.close()
    log(f"24^3x48: {out.get('rates')} cold {out['fp32_cold']}")
    return out, U, b


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inputs, U3, U2, b2, with_c2_cg=False, with_c3_cg=False):
    """The FP64 oracle on this host: the asymmetric operator at 24^3 x 48
    (degenerate) and 32^3 x 64 (doublet) on one thread and on all threads,
    and a full FP64 CG (tiny 4^4 lattice; 24^3 x 48 and the 32^3 x 64 doublet
    on request)."""
    from oracle import oracle as O
    runs = []
    nthreads = O.num_threads()

    def apply_runs(tag, op, U, b, flops, reps_all):
        for th, reps in ((1, 1), (nthreads, reps_all)):
            O.set_num_threads(th)
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                O.mat_pc(op, U, b, "asym")
                ts.append(time.perf_counter() - t0)
            t = statistics.median(ts)
            runs.append({"run": tag, "threads": th, "applies": reps, "seconds": round(t, 3),
                         "gflops": round(flops / t / 1e9, 3)})
            log(f"cpu baseline {tag} threads={th}: {t:.2f} s")
        O.set_num_threads(nthreads)

    dims2 = (24, 24, 24, 48)
    op2 = O.Params(dims2, 0.1615, 0.004, 0.0, O.PLUS)
    b2e = O.project(b2, dims2, 0)
    apply_runs("mat_pc_asym_24x24x24x48_deg", op2, U2, b2e, FLOPS_PER_SITE["deg_asym"] * 331776, 3)
    op3 = O.Params(HEADLINE_DIMS, HEADLINE["kappa"], HEADLINE["mu"], HEADLINE["eps"], O.NDEG)
    b3e = O.project(inputs.gaussian_spinor(HEADLINE_DIMS, 2, 2003), HEADLINE_DIMS, 0)
    apply_runs("mat_pc_asym_32x32x32x64_nd", op3, U3, b3e, FLOPS_PER_SITE["nd"] * 1048576, 3)
    # full FP64 CG: the tiny lattice (Haar links, kappa = 0.160, mu = 0.01),
    # on request 24^3 x 48 and the 32^3 x 64 doublet of the GPU comparison
    cgs = [("4x4x4x4_deg_sym", O.Params((4, 4, 4, 4), 0.160, 0.01, 0.0, O.PLUS),
            lambda: inputs.gauge_field((4, 4, 4, 4), "haar", 1001),
            lambda: O.project(inputs.gaussian_spinor((4, 4, 4, 4), 1, 2001), (4, 4, 4, 4), 0), "sym")]
    if with_c2_cg:
        cgs.append(("24x24x24x48_deg_asym", op2, lambda: U2, lambda: b2e, "asym"))
    if with_c3_cg:
        cgs.append(("32x32x32x64_nd_asym", op3, lambda: U3, lambda: b3e, "asym"))
    for tag, op, getU, getb, pc in cgs:
        U, b = getU(), getb()
        t0 = time.perf_counter()

        def progress(it, rel, tag=tag):
            if it % 5 == 0:
                log(f"cpu baseline cg {tag}: iteration {it}, |r|/|c| = {rel:.2e}")

        _, info = O.cg(op, U, b, pc, tol=1e-10, progress=progress)
        t = time.perf_counter() - t0
        runs.append({"run": f"cg_fp64_{tag}", "threads": nthreads,
                     "seconds": round(t, 3), "iters": info["iters"],
                     "true_rel_res_normal": info["true_rel_res_normal"]})
        log(f"cpu baseline cg {tag}: {t:.2f} s, {info['iters']} iterations")
    del b3e
    head = [r for r in runs if r["run"] == "mat_pc_asym_32x32x32x64_nd" and r["threads"] == nthreads][0]
    return {"value": head["gflops"], "unit": "Gflop/s", "cores": nthreads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"median of {head['applies']} FP64 oracle applies of the headline operator "
                      f"(32^3x64 doublet, asymmetric) on {nthreads} threads, {head['seconds']} s each; "
                      f"the other runs in 'runs'",
            "runs": runs}


def cg_comparison(torch, api, ctx, g, p, inputs, reps=3):
    """32^3 x 64 doublet, mu = 0.15, eps = 0.19, kappa = 0.1615: FP64 CG vs mixed CG."""
    b = inputs.gaussian_spinor(HEADLINE_DIMS, 2, 2003)
    tb = api.tm_spinor_pack(ctx, b[None], p, api.FP64, 0)
    del b
    out = {}
    for name, inner in (("fp64", api.FP64), ("mixed_fp16", api.FP16), ("mixed_bf16", api.BF16),
                        ("mixed_fp32", api.FP32)):
        secs, res = [], None
        for _ in range(reps):
            x = api.new_field(p, api.FP64)
            torch.cuda.synchronize()
            w0 = time.monotonic_ns()
            t0 = time.perf_counter()
            res = api.tm_cg(ctx, x, tb, g, pc=api.ASYM, tol=1e-10, maxiter=20000, inner=inner)[0]
            torch.cuda.synchronize()
            secs.append(time.perf_counter() - t0)
            # CLOCK_MONOTONIC window of the solve, for attributing a kernel trace
            log(f"cg window {name} {w0} {time.monotonic_ns()}")
        out[name] = {"seconds": round(statistics.median(secs), 4), "iters": res["iters"],
                     "reliable_updates": res["reliable_updates"],
                     "true_rel_res_normal": res["true_rel_res_normal"],
                     "true_rel_res_pc": res["true_rel_res_pc"], "status": res["status"]}
        log(f"cg {name}: {out[name]}")
    out["speedup_fp16_vs_fp64"] = round(out["fp64"]["seconds"] / out["mixed_fp16"]["seconds"], 3)
    return out


def batched_section(torch, api, inputs):
    """Many sources and uneven lattices: 16 Z2 sources on 24^3 x 48 in one solve
    versus 16 single solves, and four lattices (8^4, 12^3x24, 16^3x32, 20^3x40,
    4 sources each) in one graph-captured solve versus eager launches and
    separate solves.  Mixed precision (FP16 storage) to a 1e-10 FP64 residual."""
    import numpy as np
    out = {}
    ctx = api.Context()
    ctx.set_tuning(True)
    dims = (24, 24, 24, 48)
    p = api.make_params(dims, 0.1615, 0.004, 0.0, api.PLUS)
    U = torch.from_numpy(inputs.gauge_field(dims, "near_unit", 1004)).cuda()
    g = api.Gauge(ctx, U, p, recon=12, precs=(api.FP64, api.FP16))
    del U
    z = torch.from_numpy(inputs.z2_spinor(dims, 1, 2004, nrhs=16)).cuda()
    b16 = api.tm_spinor_pack(ctx, z, p, api.FP64, 0, 16)
    bs = [api.tm_spinor_pack(ctx, z[r:r + 1], p, api.FP64, 0, 1) for r in range(16)]
    del z
    for name, inner in (("fp64", api.FP64), ("mixed_fp16", api.FP16)):
        x = api.new_field(p, api.FP64, 16)
        api.tm_cg(ctx, x, b16, g, tol=1e-10, inner=inner, nrhs=16)      # warm (tuner)
        torch.cuda.synchronize(); t0 = time.perf_counter()
        r16 = api.tm_cg(ctx, x, b16, g, tol=1e-10, inner=inner, nrhs=16)
        torch.cuda.synchronize(); t_batch = time.perf_counter() - t0
        x1 = api.new_field(p, api.FP64)
        api.tm_cg(ctx, x1, bs[0], g, tol=1e-10, inner=inner)
        torch.cuda.synchronize(); t0 = time.perf_counter()
        its = []
        for r in range(16):
            its.append(api.tm_cg(ctx, x1, bs[r], g, tol=1e-10, inner=inner)[0]["iters"])
        torch.cuda.synchronize(); t_seq = time.perf_counter() - t0
        out[f"sources16_24x24x24x48_{name}"] = {
            "batched_s": round(t_batch, 4), "sequential_s": round(t_seq, 4),
            "speedup": round(t_seq / t_batch, 3), "batched_iters": r16[0]["iters"],
            "max_res": max(r["true_rel_res_normal"] for r in r16), "sequential_iters_mean": float(np.mean(its))}
        log(f"batched {name}: {out[f'sources16_24x24x24x48_{name}']}")
    g.close()
    # uneven lattices
    dl = [(8, 8, 8, 8), (12, 12, 12, 24), (16, 16, 16, 32), (20, 20, 20, 40)]
    gs, xs, bb = [], [], []
    for i, d in enumerate(dl):
        pp = api.make_params(d, 0.1615, 0.004, 0.0, api.PLUS)
        Ui = torch.from_numpy(inputs.gauge_field(d, "near_unit", 1040 + i)).cuda()
        gs.append(api.Gauge(ctx, Ui, pp, recon=12, precs=(api.FP64, api.FP16)))
        zi = torch.from_numpy(inputs.z2_spinor(d, 1, 2040 + i, nrhs=4)).cuda()
        bb.append(api.tm_spinor_pack(ctx, zi, pp, api.FP64, 0, 4))
        xs.append(api.new_field(pp, api.FP64, 4))
    res = {}
    for name, kw in (("graph8", dict(graph_iters=8)), ("eager", dict(check_every=8))):
        api.tm_cg_batched(ctx, gs, xs, bb, [4] * 4, tol=1e-10, inner=api.FP16, **kw)   # warm
        torch.cuda.synchronize(); t0 = time.perf_counter()
        rr = api.tm_cg_batched(ctx, gs, xs, bb, [4] * 4, tol=1e-10, inner=api.FP16, **kw)
        torch.cuda.synchronize()
        res[name] = {"s": round(time.perf_counter() - t0, 4), "iters": rr[0]["iters"],
                     "max_res": max(r["true_rel_res_normal"] for r in rr)}
    for i in range(4):                                                  # warm (tuner)
        api.tm_cg(ctx, xs[i], bb[i], gs[i], tol=1e-10, inner=api.FP16, nrhs=4)
    torch.cuda.synchronize(); t0 = time.perf_counter()
    for i in range(4):
        api.tm_cg(ctx, xs[i], bb[i], gs[i], tol=1e-10, inner=api.FP16, nrhs=4)
    torch.cuda.synchronize()
    res["separate_solves_s"] = round(time.perf_counter() - t0, 4)
    out["uneven_lattices_4x4_sources"] = res
    log(f"uneven lattices: {res}")
    for gg in gs:
        gg.close()
    ctx.close()
    return out


def force_section(torch, api, inputs):
    """16^3 x 32 doublet: FP32 force kernel time and one autograd step
    (FP64 solve recomputed in backward + force)."""
    from paper_1311_4462_amd.autograd import tm_action
    dims = (16, 16, 16, 32)
    p = api.make_params(dims, 0.1615, 0.15, 0.19, api.NDEG)
    U = torch.from_numpy(inputs.gauge_field(dims, "near_unit", 1005)).cuda()
    phi = torch.from_numpy(inputs.gaussian_spinor(dims, 2, 2005)).cuda()
    ctx = api.Context()
    g = api.Gauge(ctx, U, p, recon=12, precs=(api.FP64, api.FP32))
    xb = api.tm_spinor_pack(ctx, phi[None], p, api.FP32, 0)
    F = torch.empty(U.shape, dtype=torch.complex64, device="cuda")
    t = time_launches(torch, lambda: api.tm_force(ctx, F, api.FP32, xb, g, api.FP32, api.ASYM, 1.0, False, None), 20)
    vh = (dims[0] * dims[1] * dims[2] * dims[3]) // 2
    # one action + gradient step, twice: the first call also creates the
    # autograd context and its workspaces
    t_ag = []
    for _ in range(2):
        Ur = U.clone().requires_grad_(True)
        torch.cuda.synchronize(); t0 = time.perf_counter()
        S = tm_action(Ur, phi, p)
        S.backward()
        torch.cuda.synchronize(); t_ag.append(time.perf_counter() - t0)
    g.close(); ctx.close()
    return {"force_16x16x16x32_nd": {"tm_force_fp32_us": round(t * 1e6, 1),
                                      "note": "tm_force = M X, two hops for Z and W, and the outer-product kernel",
                                      "autograd_forward_backward_s": round(t_ag[1], 4),
                                      "autograd_forward_backward_first_call_s": round(t_ag[0], 4),
                                      "links": 4 * 2 * vh}}


WORKLOAD = ("tm_mat_pc asymmetric, non-degenerate doublet (mu 0.15, eps 0.19, kappa 0.1615), "
            "32^3x64, FP32, 12-real links")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cg-24", action="store_true",
                    help="also time a full FP64 oracle CG at 24^3x48 (about a minute of CPU)")
    ap.add_argument("--cpu-cg-32", action="store_true",
                    help="also time a full FP64 oracle CG on the 32^3x64 doublet (several minutes of CPU)")
    ap.add_argument("--cpu-only", action="store_true",
                    help="only the oracle runs on the host (no GPU work), as one JSON line")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed 32^3x64 doublet section (for profiling it)")
    ap.add_argument("--cg-only", action="store_true", help="only the 32^3x64 CG comparison")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the operator-variant, batched and force sections")
    ap.add_argument("--no-24", action="store_true",
                    help="only the 32^3x64 sections: skip the 24^3x48 one and what follows it "
                         "(batched sources, force, CPU baseline)")
    ap.add_argument("--cg-reps", type=int, default=3)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (one would split "
              "the lattice in t and exchange the spin-projected faces between neighbours).",
              file=sys.stderr)
        sys.exit(2)

    if a.cpu_only:
        from paper_1311_4462_amd import inputs
        log("bench: generating links")
        U3 = inputs.gauge_field(HEADLINE_DIMS, "near_unit", 1003)
        U2 = inputs.gauge_field((24, 24, 24, 48), "near_unit", 1002)
        b2 = inputs.gaussian_spinor((24, 24, 24, 48), 1, 2002)
        print(json.dumps({"cpu_baseline": cpu_baseline(inputs, U3, U2, b2, a.cpu_cg_24, a.cpu_cg_32)}),
              flush=True)
        return

    import torch

    from paper_1311_4462_amd import api, inputs

    torch.cuda.set_device(0)
    p = api.make_params(HEADLINE_DIMS, HEADLINE["kappa"], HEADLINE["mu"], HEADLINE["eps"], api.NDEG)
    log("bench: generating 32^3x64 links")
    U3 = inputs.gauge_field(HEADLINE_DIMS, "near_unit", 1003)
    ctx = api.Context()
    ctx.set_tuning(True)      # launch shapes picked by timing, once per kernel and shape
    Ut = torch.from_numpy(U3).cuda()
    precs = (api.FP32,) if a.headline_only else (api.FP64, api.FP32, api.FP16, api.BF16)
    g = api.Gauge(ctx, Ut, p, recon=12, precs=precs)
    if a.cg_only:
        # profiling mode: the CG comparison alone, its results as one JSON line
        out = cg_comparison(torch, api, ctx, g, p, inputs, a.cg_reps)
        g.close()
        ctx.close()
        print(json.dumps({"cg_32x32x32x64_nd": out}), flush=True)
        return
    h = headline(torch, api, ctx, g, p, a)
    vh = h["vh"]
    value = FLOPS_PER_SITE["nd"] * vh / h["dt"] / 1e9
    ach = h["b2"] * vh / h["t_k2"] / 1e9
    mat_bytes = (h["b1"] + h["b2"]) * vh
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": measured_traffic(WORKLOAD),
                "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": "hop_kernel<FP32, doublet, 12-real links>, epilogue R x + k D (second "
                          "kernel of the operator)",
                "bytes_per_site": h["b2"], "sites_per_launch": vh,
                "bytes_per_launch": h["b2"] * vh, "us_per_launch": round(h["t_k2"] * 1e6, 2)}
    extra = {
        "operator": {"us": round(h["dt"] * 1e6, 2), "gbs": round(mat_bytes / h["dt"] / 1e9, 1),
                     "frac": round(mat_bytes / h["dt"] / 1e9 / PEAK_HBM_GBS, 4),
                     "us_one_call": round(h["t_mat"] * 1e6, 2)},
        "operator_caches_flushed": {"us": round(h["t_cold"] * 1e6, 2),
                                    "frac": round(mat_bytes / h["t_cold"] / 1e9 / PEAK_HBM_GBS, 4)},
        "kernels": {"k1_twinv": {"us": round(h["t_k1"] * 1e6, 2), "bytes_per_site": h["b1"],
                                 "frac": round(h["b1"] * vh / h["t_k1"] / 1e9 / PEAK_HBM_GBS, 4)},
                    "k2_rx_plus_kd": {"us": round(h["t_k2"] * 1e6, 2), "bytes_per_site": h["b2"],
                                      "frac": round(ach / PEAK_HBM_GBS, 4)}},
    }
    log(f"headline: {h['dt'] * 1e6:.1f} us/apply, {value:.1f} Gflop/s, K1 {h['t_k1'] * 1e6:.1f} us, "
        f"K2 {h['t_k2'] * 1e6:.1f} us ({ach / PEAK_HBM_GBS:.3f} of peak)")
    cpu = None
    if not a.headline_only:
        extra["rates_32x32x32x64"] = {
            "nd": kernel_rates(torch, api, ctx, g, p, (api.FP64, api.FP16, api.BF16), 20, FLOPS_PER_SITE["nd"])}
        pd = api.make_params(HEADLINE_DIMS, 0.1615, 0.004, 0.0, api.PLUS)
        gd = api.Gauge(ctx, Ut, pd, recon=12, precs=(api.FP32,))
        extra["rates_32x32x32x64"]["deg"] = kernel_rates(torch, api, ctx, gd, pd, (api.FP32,), 20,
                                                         FLOPS_PER_SITE["deg_asym"])
        gd.close()
        g8 = api.Gauge(ctx, Ut, p, recon=8, precs=(api.FP64, api.FP32, api.FP16))
        extra["rates_32x32x32x64"]["nd_recon8"] = kernel_rates(torch, api, ctx, g8, p,
                                                               (api.FP64, api.FP32, api.FP16), 20,
                                                               FLOPS_PER_SITE["nd"], recon=8)
        g8.close()
        log(f"32^3x64 rates: {extra['rates_32x32x32x64']}")
        if not a.no_cg:
            extra["cg_32x32x32x64_nd"] = cg_comparison(torch, api, ctx, g, p, inputs, a.cg_reps)
    g.close()
    ctx.close()
    del Ut
    if a.calib_copy:
        # a plain copy of known size: 256 MiB read + 256 MiB written per launch
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not a.headline_only and not a.no_24:
        extra["deg_24x24x24x48"], U2, b2 = section_24(torch, api, inputs, a)
        if not a.no_batch:
            extra["batched"] = batched_section(torch, api, inputs)
            extra.update(force_section(torch, api, inputs))
        if not a.no_cpu_baseline:
            log("cpu baseline: oracle runs")
            cpu = cpu_baseline(inputs, U3, U2, b2, a.cpu_cg_24, a.cpu_cg_32)
        del U2, b2
    del U3

    # context only (another machine): the paper's single-GPU Gflops for this
    # operator at 32^3x64 on a GTX Titan, as its abstract quotes them from
    # Table 1 (double / single / half)
    extra["paper_context_gflops_32x32x32x64"] = {
        "degenerate": {"double": 190, "single": 487, "half": 856},
        "non_degenerate": {"double": 163, "single": 516, "half": 879},
        "hardware": "NVIDIA GTX Titan (Kepler)"}
    # what the reduced-precision figures in extra compute in
    extra["dtype_notes"] = {
        "f32": "FP32 storage and arithmetic (the headline)",
        "f64": "FP64 storage and arithmetic",
        "f16": "binary16 spinors and links with an FP32 scale per site; the projected half spinor is "
               "formed in binary16 (packed adds, relative error about 3e-4 per hop), link products "
               "accumulate in FP32 through two-term dot products, epilogues in FP32",
        "bf16": "bfloat16 spinors and links with an FP32 scale per site; projection, link products and "
                "epilogues in FP32",
        "reductions": "every norm and dot product accumulates in FP64"}
    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "Gflop/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(h["dt"] * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (near-unit random SU(3) links, Gaussian two-flavour source)",
        "config": {"workload": WORKLOAD, "lattice": "32x32x32x64", "kappa": HEADLINE["kappa"],
                   "mu": HEADLINE["mu"], "epsilon": HEADLINE["eps"], "recon": 12,
                   "parallelism": "1 GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
