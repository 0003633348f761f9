"""Helpers shared by the GPU parity tests: move canonical fields through the C ABI
and build the oracle's version of every fused-kernel call."""
import numpy as np

from oracle import oracle as O

TOL = {0: 1e-12, 1: 1e-5, 2: 5e-3, 3: 5e-3}      # FP64, FP32, FP16, BF16 (norm-wise relative)
RES_TOL = 1e-10                                   # true FP64 residual of every solve


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def oparams(api_p):
    flavor = api_p.flavor
    return O.Params(tuple(api_p.dims), api_p.kappa, api_p.mu,
                    api_p.epsilon if flavor == O.NDEG else 0.0, flavor,
                    -1.0 if api_p.t_antiperiodic else 1.0)


def with_rhs(a):
    return a if a.ndim == 8 else a[None]


def to_native(api, ctx, a, p, prec, parity, nrhs=1):
    return api.tm_spinor_pack(ctx, with_rhs(a), p, prec, parity, nrhs)


def from_native(api, ctx, t, p, prec, parity, nrhs=1):
    out = api.tm_spinor_unpack(ctx, t, p, prec, parity, nrhs)
    return out.cpu().numpy()


def oracle_dslash(p, U, inp, out_parity, dagger, twl, epi, x, k):
    """The oracle's composition for tm_dslash's fused epilogues."""
    v = O.twist(p, inp, inverse=True, dagger=dagger, parity=1 - out_parity) if twl else inp
    A = O.hop(p, U, v, out_parity, dagger=dagger)

    def Rinv(z):
        return O.twist(p, z, inverse=True, dagger=dagger, parity=out_parity)

    def R(z):
        return O.twist(p, z, dagger=dagger, parity=out_parity)

    if epi == 0:
        return A
    if epi == 1:
        return Rinv(A)
    if epi == 2:
        return R(x) + k * A
    if epi == 3:
        return x + k * Rinv(A)
    if epi == 4:
        return Rinv(x + k * A)
    if epi == 5:
        return x + k * A
    raise ValueError(epi)


def oracle_normal_residual(op, U, x_e, b_e, pc, solution="mat"):
    """|c - M^+ M x| / |c| with c = M^+ b (solution "mat") or c = b, all by the oracle."""
    c = O.mat_pc(op, U, b_e, pc, dagger=True) if solution == "mat" else b_e
    return np.linalg.norm(c - O.normal_op(op, U, x_e, pc)) / np.linalg.norm(c)


def check_solve(op, U, x_e, b_e, pc, reported, solution="mat"):
    """A GPU solution's normal residual recomputed by the oracle is at most the
    solve tolerance and equals the residual the library reported (1e-3
    relative: both are FP64, only the summation order differs)."""
    r = oracle_normal_residual(op, U, x_e, b_e, pc, solution)
    assert r <= RES_TOL, r
    assert abs(r - reported) <= 1e-3 * r, (r, reported)
    return r
