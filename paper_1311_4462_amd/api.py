"""Thin Python binding of the C ABI (include/tm.h).

Every function marshals torch device tensors to raw pointers and calls the
same-named entry point of libtm.so; all arithmetic runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.
"""
from __future__ import annotations

import ctypes
import warnings

import numpy as np
import torch

from ._lib import TMError, lib, tm_cg_params, tm_cg_result, tm_params, tm_solve_params

FP64, FP32, FP16, BF16 = 0, 1, 2, 3
PLUS, MINUS, NDEG = 1, -1, 2
ASYM, SYM = 0, 1
SOLUTION_MAT, SOLUTION_MATDAG_MAT = 0, 1
SOLVE_NORMOP_PC, SOLVE_DIRECT_PC = 0, 1
BASIS_INTERNAL, BASIS_CHIRAL = 0, 1
EPI_NONE, EPI_TWINV, EPI_RX_PLUS_KD, EPI_X_PLUS_K_TWINV_D, EPI_TWINV_X_PLUS_KD, EPI_X_PLUS_KD = range(6)
TM_OK, TM_NOT_CONVERGED = 0, 1
PREC_NAMES = {FP64: "f64", FP32: "f32", FP16: "f16", BF16: "bf16"}


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return t.data_ptr()
    return int(t)


def make_params(dims, kappa, mu, eps=0.0, flavor=PLUS, t_antiperiodic=True, csw=0.0) -> tm_params:
    """dims = (Lx, Ly, Lz, Lt); csw != 0 selects the twisted-clover operator."""
    p = tm_params()
    for i in range(4):
        p.dims[i] = int(dims[i])
    p.kappa, p.mu, p.epsilon = float(kappa), float(mu), float(eps)
    p.flavor = int(flavor)
    p.t_antiperiodic = 1 if t_antiperiodic else 0
    p.csw = float(csw)
    return p


class Context:
    """A library context bound to a HIP stream (torch's current stream by default)."""

    def __init__(self, stream=None):
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p()
        rc = lib().tm_ctx_create(ctypes.byref(h), ctypes.c_void_p(stream or 0))
        if rc != TM_OK:
            raise TMError(rc, lib().tm_error_string(rc).decode())
        self.h = h

    def check(self, rc: int, what: str = "") -> int:
        if rc < 0:
            msg = lib().tm_last_error(self.h).decode()
            raise TMError(rc, f"{what}: {msg}" if what else msg)
        if rc > 0:
            warnings.warn(f"{what}: {lib().tm_error_string(rc).decode()}")
        return rc

    def set_stream(self, stream):
        self.check(lib().tm_ctx_set_stream(self.h, ctypes.c_void_p(stream or 0)), "set_stream")

    def set_tuning(self, enable: bool):
        self.check(lib().tm_set_tuning(self.h, int(enable)), "set_tuning")

    def close(self):
        if getattr(self, "h", None):
            lib().tm_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Gauge:
    """Packed gauge field + operator parameters (tm_gauge)."""

    def __init__(self, ctx: Context, links, params: tm_params, recon: int = 12,
                 precs=(FP64, FP32)):
        if isinstance(links, np.ndarray):
            links = torch.from_numpy(np.ascontiguousarray(links))
        if links.device.type != "cuda":
            links = links.to("cuda")
        assert links.dtype == torch.complex128 and links.is_contiguous()
        self.ctx = ctx
        self.params = params
        self.recon = recon
        self.nf = 2 if params.flavor == NDEG else 1
        self.dims = tuple(params.dims)
        self.vh = int(np.prod(self.dims)) // 2
        mask = 0
        for p in precs:
            mask |= 1 << p
        h = ctypes.c_void_p()
        ctx.check(lib().tm_gauge_create(ctx.h, ctypes.byref(h), ctypes.c_void_p(links.data_ptr()),
                                        ctypes.byref(params), recon, mask), "tm_gauge_create")
        self.h = h

    def bytes(self, prec: int) -> int:
        return int(lib().tm_gauge_bytes(self.h, prec))

    def close(self):
        if getattr(self, "h", None):
            lib().tm_gauge_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tm_spinor_bytes(params: tm_params, prec: int, nrhs: int = 1) -> int:
    return int(lib().tm_spinor_bytes(ctypes.byref(params), prec, nrhs))


def new_field(params: tm_params, prec: int, nrhs: int = 1, zero: bool = False) -> torch.Tensor:
    n = tm_spinor_bytes(params, prec, nrhs)
    if n == 0:
        raise ValueError("invalid parameters for a spinor field")
    f = torch.empty(n, dtype=torch.uint8, device="cuda")
    if zero:
        f.zero_()
    return f


def canonical_shape(params: tm_params, nrhs: int = 1):
    lx, ly, lz, lt = params.dims
    nf = 2 if params.flavor == NDEG else 1
    return (nrhs, lt, lz, ly, lx, nf, 4, 3)


def tm_spinor_pack(ctx: Context, canonical, params: tm_params, prec: int, parity: int,
                   nrhs: int = 1, out=None, basis: int = BASIS_INTERNAL) -> torch.Tensor:
    if isinstance(canonical, np.ndarray):
        canonical = torch.from_numpy(np.ascontiguousarray(canonical))
    canonical = canonical.to("cuda").contiguous()
    assert canonical.dtype == torch.complex128
    assert canonical.numel() == int(np.prod(canonical_shape(params, nrhs)))
    out = new_field(params, prec, nrhs) if out is None else out
    ctx.check(lib().tm_spinor_pack(ctx.h, _ptr(out), _ptr(canonical), ctypes.byref(params), prec,
                                   parity, nrhs, basis), "tm_spinor_pack")
    return out


def tm_spinor_unpack(ctx: Context, native, params: tm_params, prec: int, parity: int,
                     nrhs: int = 1, out=None, basis: int = BASIS_INTERNAL) -> torch.Tensor:
    if out is None:
        out = torch.zeros(canonical_shape(params, nrhs), dtype=torch.complex128, device="cuda")
    ctx.check(lib().tm_spinor_unpack(ctx.h, _ptr(out), _ptr(native), ctypes.byref(params), prec,
                                     parity, nrhs, basis), "tm_spinor_unpack")
    return out


def tm_dslash(ctx, out, inp, gauge: Gauge, prec, out_parity, dagger=0, twist_on_load=0,
              epi=EPI_NONE, x=None, k=0.0, nrhs=1):
    return ctx.check(lib().tm_dslash(ctx.h, _ptr(out), _ptr(inp), gauge.h, prec, out_parity,
                                     int(dagger), int(twist_on_load), int(epi), _ptr(x), float(k),
                                     nrhs), "tm_dslash")


def tm_mat_pc(ctx, out, inp, gauge: Gauge, prec, pc=ASYM, dagger=0, nrhs=1):
    return ctx.check(lib().tm_mat_pc(ctx.h, _ptr(out), _ptr(inp), gauge.h, prec, pc, int(dagger),
                                     nrhs), "tm_mat_pc")


def tm_mat_pc_noalloc(ctx, out, inp, gauge: Gauge, prec, pc=ASYM, dagger=0, nrhs=1):
    return ctx.check(lib().tm_mat_pc_noalloc(ctx.h, _ptr(out), _ptr(inp), gauge.h, prec, pc, int(dagger),
                                             nrhs), "tm_mat_pc_noalloc")


def tm_twist(ctx, out, inp, gauge: Gauge, prec, parity, dagger=0, inverse=1, nrhs=1):
    return ctx.check(lib().tm_twist(ctx.h, _ptr(out), _ptr(inp), gauge.h, prec, parity,
                                    int(dagger), int(inverse), nrhs), "tm_twist")


def tm_twist_inv(ctx, out, inp, gauge: Gauge, prec, parity, dagger=0, nrhs=1):
    return ctx.check(lib().tm_twist_inv(ctx.h, _ptr(out), _ptr(inp), gauge.h, prec, parity,
                                        int(dagger), nrhs), "tm_twist_inv")


def tm_prepare(ctx, bhat_e, b_e, b_o, gauge: Gauge, prec, pc=ASYM, nrhs=1):
    return ctx.check(lib().tm_prepare(ctx.h, _ptr(bhat_e), _ptr(b_e), _ptr(b_o), gauge.h, prec, pc,
                                      nrhs), "tm_prepare")


def tm_reconstruct_odd(ctx, x_o, x_e, b_o, gauge: Gauge, prec, nrhs=1):
    return ctx.check(lib().tm_reconstruct_odd(ctx.h, _ptr(x_o), _ptr(x_e), _ptr(b_o), gauge.h, prec,
                                              nrhs), "tm_reconstruct_odd")


def _cg_params(pc, tol, maxiter, inner, delta, use_x0, nrhs, graph_iters, check_every,
               solution=0, stall_factor=0.0, max_stalls=0):
    p = tm_cg_params()
    p.solution = solution
    p.pc, p.tol, p.maxiter, p.outer, p.inner = pc, tol, maxiter, FP64, inner
    p.delta, p.use_x0, p.nrhs, p.graph_iters, p.check_every = (delta, int(use_x0), nrhs,
                                                               graph_iters, check_every)
    p.stall_factor, p.max_stalls = stall_factor, max_stalls
    return p


def _results(res, n):
    return [dict(iters=res[i].iters, reliable_updates=res[i].reliable_updates,
                 true_rel_res_normal=res[i].true_rel_res_normal,
                 true_rel_res_pc=res[i].true_rel_res_pc, seconds=res[i].seconds,
                 true_rel_res_full=res[i].true_rel_res_full,
                 precision_fallbacks=res[i].precision_fallbacks,
                 res_history=list(res[i].res_history[:res[i].history_len])) for i in range(n)]


def tm_cg(ctx, x_e, b_e, gauge: Gauge, pc=ASYM, tol=1e-10, maxiter=5000, inner=FP64, delta=0.0,
          use_x0=False, nrhs=1, graph_iters=0, check_every=0, solution=SOLUTION_MAT,
          stall_factor=0.0, max_stalls=0):
    """CG on the normal equations of the preconditioned operator; x_e, b_e FP64 native."""
    p = _cg_params(pc, tol, maxiter, inner, delta, use_x0, nrhs, graph_iters, check_every, solution,
                   stall_factor, max_stalls)
    res = (tm_cg_result * nrhs)()
    rc = ctx.check(lib().tm_cg(ctx.h, _ptr(x_e), _ptr(b_e), gauge.h, ctypes.byref(p), res), "tm_cg")
    out = _results(res, nrhs)
    for o in out:
        o["status"] = rc
    return out


def tm_cg_batched(ctx, gauges, xs, bs, nrhs, pc=ASYM, tol=1e-10, maxiter=5000, inner=FP64,
                  delta=0.0, graph_iters=0, check_every=0, solution=SOLUTION_MAT):
    n = len(gauges)
    p = _cg_params(pc, tol, maxiter, inner, delta, False, nrhs[0], graph_iters, check_every, solution)
    ga = (ctypes.c_void_p * n)(*[g.h.value for g in gauges])
    xa = (ctypes.c_void_p * n)(*[_ptr(x) for x in xs])
    ba = (ctypes.c_void_p * n)(*[_ptr(b) for b in bs])
    na = (ctypes.c_int * n)(*nrhs)
    total = sum(nrhs)
    res = (tm_cg_result * total)()
    rc = ctx.check(lib().tm_cg_batched(ctx.h, n, ga, xa, ba, na, ctypes.byref(p), res),
                   "tm_cg_batched")
    out = _results(res, total)
    for o in out:
        o["status"] = rc
    return out


def tm_solve(ctx, x_e, x_o, b_e, b_o, gauge: Gauge, solution=SOLUTION_MAT,
             solve_type=SOLVE_NORMOP_PC, pc=ASYM, tol=1e-10, maxiter=5000, inner=FP64, delta=0.0,
             nrhs=1, graph_iters=0, check_every=0):
    """Full-system solve M x = b or M^+ M x = b; all four fields FP64 native."""
    p = tm_solve_params()
    p.cg = _cg_params(pc, tol, maxiter, inner, delta, False, nrhs, graph_iters, check_every)
    p.solve_type, p.solution = solve_type, solution
    res = (tm_cg_result * nrhs)()
    rc = ctx.check(lib().tm_solve(ctx.h, _ptr(x_e), _ptr(x_o), _ptr(b_e), _ptr(b_o), gauge.h,
                                  ctypes.byref(p), res), "tm_solve")
    out = _results(res, nrhs)
    for o in out:
        o["status"] = rc
    return out


def tm_norm2(ctx, x, params: tm_params, prec, nrhs=1) -> np.ndarray:
    out = (ctypes.c_double * nrhs)()
    ctx.check(lib().tm_norm2(ctx.h, out, _ptr(x), ctypes.byref(params), prec, nrhs), "tm_norm2")
    return np.array(out[:])


def tm_dot(ctx, x, y, params: tm_params, prec, nrhs=1) -> np.ndarray:
    out = (ctypes.c_double * (2 * nrhs))()
    ctx.check(lib().tm_dot(ctx.h, out, _ptr(x), _ptr(y), ctypes.byref(params), prec, nrhs), "tm_dot")
    a = np.array(out[:])
    return a[0::2] + 1j * a[1::2]


def tm_convert(ctx, dst, dst_prec, src, src_prec, params: tm_params, nrhs=1):
    return ctx.check(lib().tm_convert(ctx.h, _ptr(dst), dst_prec, _ptr(src), src_prec,
                                      ctypes.byref(params), nrhs), "tm_convert")


def tm_scale(ctx, dst, dst_prec, src, src_prec, a, params: tm_params, nrhs=1):
    return ctx.check(lib().tm_scale(ctx.h, _ptr(dst), dst_prec, _ptr(src), src_prec, float(a),
                                    ctypes.byref(params), nrhs), "tm_scale")


def tm_force(ctx, F, force_prec, X_e, gauge: Gauge, prec, pc=ASYM, coeff=1.0, accumulate=False,
             G=None):
    return ctx.check(lib().tm_force(ctx.h, _ptr(F), force_prec, _ptr(X_e), gauge.h, prec, pc,
                                    float(coeff), int(accumulate), _ptr(G)), "tm_force")
