#!/usr/bin/env python3
"""Benchmark: twisted-mass Dslash Gflop/s + HBM GB/s on one MI355X, and mixed vs
FP64 CG time to a 1e-10 residual.

Timed step = one application of the asymmetric even-odd preconditioned operator
(Eq. 2.2, the operator Table 1 of the paper measures): two fused hop kernels,
FP32 storage and arithmetic, 12-real links, degenerate flavour, 24^3 x 48
lattice (kappa = 0.1615, mu = 0.004, near-unit SU(3) links), inputs resident in
HBM.  Flops per even site: 2808 (1320 per hop, twist and xpay as counted in
the design notes); algorithmic bytes per even site: 16 L + 5 S.

Also reported (not timed in the K steps): per-kernel durations from HIP events
with the roofline of the dominant kernel, the FP64 CPU oracle on the host as a
baseline, and the 32^3 x 64 non-degenerate doublet CG comparison (FP64 CG vs
mixed precision with FP64 reliable updates) to a 1e-10 true residual.
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def site_bytes(L, S):
    """(K1, K2) algorithmic bytes per even site: K1 = 8L + 2S, K2 = 8L + 3S."""
    return 8 * L + 2 * S, 8 * L + 3 * S


def measured_traffic():
    """HBM-side bytes per launch of the roofline kernel from the committed
    FETCH_SIZE / WRITE_SIZE summary, or None if the kernel source changed since."""
    import hashlib
    try:
        t = json.load(open(os.path.join(ROOT, "profiles", "hop_traffic.json")))
        csrc = os.path.join(ROOT, "paper_1311_4462_amd", "csrc")
        src = b"".join(open(os.path.join(csrc, f), "rb").read()
                       for f in ("tm_hop.inc.h", "tm_impl.h", "tm_hop_fp32.hip"))
        if hashlib.sha256(src).hexdigest()[:16] != t["source_sha256_16"]:
            return None
        return int(t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def time_launches(torch, fn, reps, warm=3):
    for _ in range(warm):          # first calls may run the block-size tuner
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


def cpu_baseline(U, b_e, dims, vh, budget_s=15.0):
    """The FP64 oracle's asymmetric operator apply on this host (C loop + NumPy)."""
    from oracle import oracle as O
    op = O.Params(dims, 0.1615, 0.004, 0.0, O.PLUS)
    t0 = time.perf_counter()
    O.mat_pc(op, U, b_e, "asym")
    t1 = time.perf_counter() - t0
    n = max(1, min(8, int(budget_s / max(t1, 1e-3))))
    ts = [t1]
    for _ in range(n - 1):
        t0 = time.perf_counter()
        O.mat_pc(op, U, b_e, "asym")
        ts.append(time.perf_counter() - t0)
    t = statistics.median(ts)
    return {"value": round(FLOPS_PER_SITE["deg_asym"] * vh / t / 1e9, 3), "unit": "Gflop/s",
            "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{len(ts)} FP64 applies of the asymmetric preconditioned operator at "
                      f"{'x'.join(map(str, dims))} (median {t:.2f} s each)"}


BYTES_PER_REAL = {0: 8, 1: 4, 2: 2, 3: 2}     # FP64, FP32, FP16, BF16


def mat_pc_rates(torch, api, ctx, g, p, precs, reps, flops_site, recon=12):
    """Per-precision asymmetric M apply on a resident field: us, Gflop/s, algorithmic GB/s."""
    import numpy as np
    nf = 2 if p.flavor == api.NDEG else 1
    vh = int(np.prod(tuple(p.dims))) // 2
    L = {q: recon * BYTES_PER_REAL[q] for q in (api.FP64, api.FP32, api.FP16, api.BF16)}
    S = {api.FP64: 192 * nf, api.FP32: 96 * nf, api.FP16: 52 * nf, api.BF16: 52 * nf}
    src = torch.randn(api.canonical_shape(p), dtype=torch.complex128, device="cuda")
    out = {}
    for prec in precs:
        x = api.tm_spinor_pack(ctx, src, p, prec, 0)
        y = api.new_field(p, prec)
        t = time_launches(torch, lambda: api.tm_mat_pc(ctx, y, x, g, prec, api.ASYM, 0), reps)
        out[api.PREC_NAMES[prec]] = {"us": round(t * 1e6, 1), "gflops": round(flops_site * vh / t / 1e9, 1),
                                     "gbs": round((16 * L[prec] + 5 * S[prec]) * vh / t / 1e9, 1)}
        del x, y
    del src
    return out


def operator_variants(torch, api, ctx, U, p, reps):
    """us per apply of the preconditioned operator, asym / sym, with and without
    dagger, FP64 and FP32: one flavour with 18-, 12- and 8-real links, the other
    twist sign and the doublet with 12-real links; and the asymmetric
    twisted-clover apply."""
    Ut = torch.from_numpy(U).cuda()
    out = {}
    # one flavour twisted up (PLUS) with 18/12/8-real links, then twisted down
    # (MINUS) and the doublet (eps = 0.19) with 12-real links
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
    # twisted clover (c_sw = 1.57): the same asymmetric apply, with the clover
    # blocks read by both kernels (A and B by the R^-1 kernel, A by the R kernel)
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


def cg_comparison(torch, api, inputs, reps=3):
    """32^3 x 64 doublet, mu = 0.15, eps = 0.19, kappa = 0.1615: FP64 CG vs mixed CG;
    also the operator apply rates on this lattice (doublet in all precisions, one
    flavour in FP32), whose working sets exceed the 256 MB last-level cache."""
    dims = (32, 32, 32, 64)
    p = api.make_params(dims, 0.1615, 0.15, 0.19, api.NDEG)
    log("cg: generating 32^3x64 links")
    U = inputs.gauge_field(dims, "near_unit", 1003)
    Ut = torch.from_numpy(U).cuda()
    del U
    ctx = api.Context()
    ctx.set_tuning(True)
    g = api.Gauge(ctx, Ut, p, recon=12, precs=(api.FP64, api.FP32, api.FP16, api.BF16))
    rates = {"nd": mat_pc_rates(torch, api, ctx, g, p, (api.FP64, api.FP32, api.FP16, api.BF16), 20,
                                FLOPS_PER_SITE["nd"])}
    pd = api.make_params(dims, 0.1615, 0.004, 0.0, api.PLUS)
    gd = api.Gauge(ctx, Ut, pd, recon=12, precs=(api.FP32,))
    rates["deg"] = mat_pc_rates(torch, api, ctx, gd, pd, (api.FP32,), 20, FLOPS_PER_SITE["deg_asym"])
    gd.close()
    # 8-real links: the same applies with a third fewer link bytes
    g8 = api.Gauge(ctx, Ut, p, recon=8, precs=(api.FP32, api.FP16))
    rates["nd_recon8"] = mat_pc_rates(torch, api, ctx, g8, p, (api.FP32, api.FP16), 20,
                                      FLOPS_PER_SITE["nd"], recon=8)
    g8.close()
    gd8 = api.Gauge(ctx, Ut, pd, recon=8, precs=(api.FP32,))
    rates["deg_recon8"] = mat_pc_rates(torch, api, ctx, gd8, pd, (api.FP32,), 20,
                                       FLOPS_PER_SITE["deg_asym"], recon=8)
    gd8.close()
    log(f"32^3x64 mat_pc rates: {rates}")
    del Ut
    b = inputs.gaussian_spinor(dims, 2, 2003)
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
    g.close()
    ctx.close()
    out["speedup_fp16_vs_fp64"] = round(out["fp64"]["seconds"] / out["mixed_fp16"]["seconds"], 3)
    out["mat_pc_rates"] = rates
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
    """16^3 x 32 doublet: FP32 force kernel time and bytes, and one autograd step
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
    Ur = U.clone().requires_grad_(True)
    torch.cuda.synchronize(); t0 = time.perf_counter()
    S = tm_action(Ur, phi, p)
    S.backward()
    torch.cuda.synchronize(); t_ag = time.perf_counter() - t0
    g.close(); ctx.close()
    return {"force_16x16x16x32_nd": {"tm_force_fp32_us": round(t * 1e6, 1),
                                      "note": "tm_force = M X, two hops for Z and W, and the outer-product kernel",
                                      "autograd_forward_backward_s": round(t_ag, 4),
                                      "links": 4 * 2 * vh}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--cg-only", action="store_true", help="only the CG comparison")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the operator-variant, batched and force sections")
    ap.add_argument("--cg-reps", type=int, default=3)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (one would split "
              "the lattice in t and exchange the spin-projected faces between neighbours).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1311_4462_amd import api, inputs

    torch.cuda.set_device(0)
    if a.cg_only:
        print(json.dumps({"cg_32x32x32x64_nd": cg_comparison(torch, api, inputs, a.cg_reps)}), flush=True)
        return
    dims = (24, 24, 24, 48)
    vh = int(np.prod(dims)) // 2
    p = api.make_params(dims, 0.1615, 0.004, 0.0, api.PLUS)
    log("bench: generating 24^3x48 links")
    U = inputs.gauge_field(dims, "near_unit", 1002)
    ctx = api.Context()
    ctx.set_tuning(True)      # block size and link-load policy picked by timing, once per shape
    g = api.Gauge(ctx, torch.from_numpy(U).cuda(), p, recon=12, precs=(api.FP64, api.FP32))
    b = inputs.gaussian_spinor(dims, 1, 2002)
    from oracle import oracle as O  # only for the even projection of the CPU-baseline input
    b_e = O.project(b, dims, 0) if not a.no_cpu_baseline else None
    x = api.tm_spinor_pack(ctx, b[None], p, api.FP32, 0)
    y = api.new_field(p, api.FP32)

    def step():
        api.tm_mat_pc(ctx, y, x, g, api.FP32, api.ASYM, 0)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    flops = FLOPS_PER_SITE["deg_asym"] * vh
    value = flops / dt / 1e9

    # the same apply with the caches flushed before each call (before the
    # per-kernel timing, whose launches then end the trace of this section)
    t_cold = time_cold(torch, step, 20)

    # per-kernel durations (HIP events on the stream the kernels run on)
    L, S = 48, 96
    b1, b2 = site_bytes(L, S)
    tmp = api.new_field(p, api.FP32, 1)
    kappa2 = -p.kappa ** 2
    t_k1 = time_launches(torch, lambda: api.tm_dslash(ctx, tmp, x, g, api.FP32, 1, 0, 0,
                                                      api.EPI_TWINV, None, 0.0), a.kernel_reps)
    t_k2 = time_launches(torch, lambda: api.tm_dslash(ctx, y, tmp, g, api.FP32, 0, 0, 0,
                                                      api.EPI_RX_PLUS_KD, x, kappa2), a.kernel_reps)
    ach = b2 * vh / t_k2 / 1e9
    mat_bytes = (b1 + b2) * vh
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": measured_traffic(),
                "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": "hop_kernel<FP32, 1 flavour, 1 rhs, 12-real links> with epilogue R x + k D",
                "bytes_per_launch": b2 * vh, "us_per_launch": round(t_k2 * 1e6, 2)}
    extra = {
        "hbm_gbs_mat_pc": round(mat_bytes / dt / 1e9, 1),
        "hbm_frac_mat_pc": round(mat_bytes / dt / 1e9 / PEAK_HBM_GBS, 4),
        # the same apply with the caches flushed before each call
        "mat_pc_fp32_cold": {"us": round(t_cold * 1e6, 2), "gbs": round(mat_bytes / t_cold / 1e9, 1),
                             "frac": round(mat_bytes / t_cold / 1e9 / PEAK_HBM_GBS, 4)},
        "kernel_us": {"hop_twinv": round(t_k1 * 1e6, 2), "hop_rx_plus_kd": round(t_k2 * 1e6, 2)},
        "kernel_gbs": {"hop_twinv": round(b1 * vh / t_k1 / 1e9, 1),
                       "hop_rx_plus_kd": round(ach, 1)},
    }
    log(f"mat_pc fp32: {dt * 1e6:.1f} us/apply, {value:.1f} Gflop/s, "
        f"{extra['hbm_gbs_mat_pc']} GB/s; kernels {extra['kernel_us']}; "
        f"caches flushed: {extra['mat_pc_fp32_cold']}")

    # FP64 operator on the same lattice (context figure)
    x64 = api.tm_spinor_pack(ctx, b[None], p, api.FP64, 0)
    y64 = api.new_field(p, api.FP64)
    t64 = time_launches(torch, lambda: api.tm_mat_pc(ctx, y64, x64, g, api.FP64, api.ASYM, 0),
                        a.kernel_reps)
    extra["mat_pc_fp64"] = {"us": round(t64 * 1e6, 2), "gflops": round(flops / t64 / 1e9, 1),
                            "gbs": round((16 * 96 + 5 * 192) * vh / t64 / 1e9, 1)}
    del x64, y64
    if not a.no_batch:
        extra["variants_24x24x24x48_us"] = operator_variants(torch, api, ctx, U, p, a.kernel_reps)
        v8 = extra["variants_24x24x24x48_us"]["f32_r8"]["asym"]
        extra["mat_pc_fp32_recon8"] = {"us": v8, "gflops": round(flops / (v8 * 1e-6) / 1e9, 1),
                                       "gbs": round((16 * 32 + 5 * 96) * vh / (v8 * 1e-6) / 1e9, 1)}
    g.close()
    ctx.close()
    del U

    if a.calib_copy:
        # a plain copy of known size: 256 MiB read + 256 MiB written per launch
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not a.no_cpu_baseline:
        log("cpu baseline: oracle applies")
        Uc = inputs.gauge_field(dims, "near_unit", 1002)
        cpu = cpu_baseline(Uc, b_e, dims, vh)
        del Uc
    if not a.no_cg:
        extra["cg_32x32x32x64_nd"] = cg_comparison(torch, api, inputs, a.cg_reps)
    if not a.no_batch:
        extra["batched"] = batched_section(torch, api, inputs)
        extra.update(force_section(torch, api, inputs))

    # context only (another machine): the paper's single-GPU Gflops for this
    # operator at 32^3x64 on a GTX Titan, as its abstract quotes them from
    # Table 1 (double / single / half; 8-real links for the degenerate single
    # and half figures)
    extra["paper_context_gflops_32x32x32x64"] = {
        "degenerate": {"double": 190, "single": 487, "half": 856},
        "non_degenerate": {"double": 163, "single": 516, "half": 879},
        "hardware": "NVIDIA GTX Titan (Kepler)"}
    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "Gflop/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(dt * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (near-unit random SU(3) links, Gaussian source)",
        "config": {"workload": "tm_mat_pc asymmetric, degenerate, 24^3x48, FP32, 12-real links",
                   "lattice": "24x24x24x48", "kappa": 0.1615, "mu": 0.004, "recon": 12,
                   "parallelism": "1 GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
