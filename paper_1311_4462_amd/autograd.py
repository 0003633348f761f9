"""torch.autograd.Function for S(U, phi) = phi^+ (M^+ M)^-1 phi.

M is the even-odd preconditioned twisted-mass operator (Eq. 2.2 asym or 2.3
sym) built from the links U (complex128, canonical [4, Lt, Lz, Ly, Lx, 3, 3],
on the GPU) and phi a canonical source whose even sites are used.  Forward runs
the library's FP64 CG; backward recomputes the solve (nothing but U and phi is
stored) and calls the hand-written force kernel (tm_force), which returns the
unconstrained gradient G with dS = Re tr(G^+ dU) -- torch's convention for a
real function of complex inputs -- and grad_phi = 2 X.  The incoming gradient
enters as the force kernel's coefficient and as the factor of tm_scale, so the
binding only moves data (packing, dtype of the returned tensors).
"""
from __future__ import annotations

import torch

from . import api

_CTX = {}


def _context():
    dev = torch.cuda.current_device()
    c = _CTX.get(dev)
    if c is None:
        c = _CTX[dev] = api.Context()
    c.set_stream(torch.cuda.current_stream().cuda_stream)
    return c


def _solve(ctx, U, phi, params, pc, tol, recon, precs):
    g = api.Gauge(ctx, U.detach().contiguous(), params, recon=recon, precs=precs)
    phi_n = api.tm_spinor_pack(ctx, phi.detach().reshape((1,) + tuple(phi.shape)).contiguous(),
                               params, api.FP64, 0)
    x = api.new_field(params, api.FP64)
    res = api.tm_cg(ctx, x, phi_n, g, pc=pc, tol=tol, maxiter=100000,
                    solution=api.SOLUTION_MATDAG_MAT)[0]
    if res["status"] != 0:
        raise RuntimeError(f"TMAction: solve did not converge: {res}")
    return g, phi_n, x, res


class TMAction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, U, phi, params, pc=api.ASYM, tol=1e-12, force_prec=api.FP32, recon=12):
        ctx = _context()
        g, phi_n, x, _ = _solve(ctx, U, phi, params, pc, tol, recon, (api.FP64,))
        S = api.tm_dot(ctx, phi_n, x, params, api.FP64)[0].real
        g.close()
        fctx.save_for_backward(U, phi)
        fctx.cfg = (params, pc, tol, force_prec, recon)
        return torch.tensor(S, dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(fctx, gS):
        U, phi = fctx.saved_tensors
        params, pc, tol, force_prec, recon = fctx.cfg
        ctx = _context()
        precs = (api.FP64,) if force_prec == api.FP64 else (api.FP64, api.FP32)
        g, phi_n, x, _ = _solve(ctx, U, phi, params, pc, tol, recon, precs)   # recomputed
        if force_prec == api.FP64:
            xf, fdt = x, torch.complex128
        else:
            xf = api.new_field(params, api.FP32)
            api.tm_convert(ctx, xf, api.FP32, x, api.FP64, params)
            fdt = torch.complex64
        F = torch.empty(U.shape, dtype=fdt, device=U.device)
        G = torch.empty(U.shape, dtype=fdt, device=U.device)
        gs = float(gS)
        api.tm_force(ctx, F, force_prec, xf, g, force_prec, pc, gs, False, G)
        gU = G.to(torch.complex128)
        gphi = None
        if fctx.needs_input_grad[1]:
            api.tm_scale(ctx, x, api.FP64, x, api.FP64, 2.0 * gs, params)
            X = api.tm_spinor_unpack(ctx, x, params, api.FP64, 0)[0]
            gphi = X.reshape(phi.shape).to(phi.dtype)
        g.close()
        return gU, gphi, None, None, None, None, None


def tm_action(U, phi, params, pc=api.ASYM, tol=1e-12, force_prec=api.FP32, recon=12):
    return TMAction.apply(U, phi, params, pc, tol, force_prec, recon)


def tm_force(U, X_even, params, pc=api.ASYM, force_prec=api.FP32, recon=12, with_G=False):
    """Force F (traceless anti-Hermitian, [4, Lt, Lz, Ly, Lx, 3, 3]) for a given
    canonical X = (M^+ M)^-1 phi (even sites)."""
    ctx = _context()
    precs = (api.FP64,) if force_prec == api.FP64 else (api.FP64, api.FP32)
    g = api.Gauge(ctx, U.contiguous(), params, recon=recon, precs=precs)
    xn = api.tm_spinor_pack(ctx, X_even.reshape((1,) + tuple(X_even.shape)).contiguous(), params,
                            force_prec, 0)
    fdt = torch.complex128 if force_prec == api.FP64 else torch.complex64
    F = torch.empty(U.shape, dtype=fdt, device=U.device)
    G = torch.empty(U.shape, dtype=fdt, device=U.device) if with_G else None
    api.tm_force(ctx, F, force_prec, xn, g, force_prec, pc, 1.0, False, G)
    g.close()
    return (F, G) if with_G else F
