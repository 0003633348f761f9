"""FP64 CPU oracle for the even-odd preconditioned Wilson twisted-mass operator.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark; never by the library's product path.
It shares no code with the HIP implementation: the Wilson hop is the plain C
loop in ``tm_oracle.c`` (built into ``liboracle.so``), everything else here is
NumPy on canonical full-lattice arrays

    spinor  complex128 [(nrhs,) Lt, Lz, Ly, Lx, nf, 4, 3]
    links   complex128 [4, Lt, Lz, Ly, Lx, 3, 3]

A field "of parity p" is a full-lattice array that is zero on the other
parity.

Conventions (the paper leaves them open; the readings are the ones written in
the design notes):
  * M = R - kappa * D, i.e. Eq. (2.1) multiplied by 2*kappa with
    kappa = 1 / (2 m0 + 8), Wilson r = 1.
  * R = 1 + i a g5 t3 + b t1 with a = 2 kappa mu, b = 2 kappa eps (Eq. 2.1);
    single flavour: R = 1 +- i a g5 (twist_flavor PLUS / MINUS, Sec. 2.2).
    Flavour 0 has t3 = +1; t1 swaps the flavours.
  * g5 = g1 g2 g3 g4 = [[0, 1], [1, 0]] in 2x2 blocks of the basis of Sec. 2.
  * Preconditioned operators (Eqs. 2.2, 2.3):
        asym:  R_ee - kappa^2 D_eo R_oo^-1 D_oe
        sym :  1    - kappa^2 R_ee^-1 D_eo R_oo^-1 D_oe
  * Right-hand side: b_e + kappa D_eo R_oo^-1 b_o (asym), R_ee^-1 times that
    (sym).  The printed Eqs. (2.2)/(2.3) omit the kappa, which the kappa^2 of
    their left-hand side requires once M = R - kappa D.
  * Odd reconstruction: psi_o = R_oo^-1 (b_o + kappa D_oe psi_e).  The printed
    Eq. (2.4) has R_ee^-1 psi_e in place of psi_e, which holds only for the
    right-preconditioned variable R_ee psi_e.
  * CG: conjugate gradient on the normal equations M^+ M x = M^+ b (the
    NORMOP solve of Sec. 2.2) in FP64, stopped on the true residual.
  * Twisted clover (the future work of Sec. 4): R(x) = A(x) + i a g5 t3 + b t1
    with A = 1 + i kappa c_sw sum_{mu<nu} sigma_munu F_munu, F from the
    four-leaf clover (with_clover); every operator above then uses it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_oracle(force: bool = False) -> str:
    """Compile tm_oracle.c with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build_oracle()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_hop.argtypes = [dp, dp, dp, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                              ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int]
        L.orc_hop.restype = ctypes.c_int
        L.orc_gammas.argtypes = [dp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_set_num_threads.restype = None
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.complex128 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the C hop's parallel loops from now on (timing only)."""
    lib().orc_set_num_threads(int(n))


def gammas() -> np.ndarray:
    """gamma_mu, mu = x, y, z, t, as complex [4, 4, 4] (from the C oracle)."""
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    lib().orc_gammas(_dp(g))
    return g


# --- site-local algebra -----------------------------------------------------

I2 = np.eye(2, dtype=np.complex128)
GAMMA5 = np.block([[np.zeros((2, 2)), I2], [I2, np.zeros((2, 2))]]).astype(np.complex128)
TAU1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
TAU3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)

PLUS, MINUS, NDEG = 1, -1, 2


@dataclass
class Params:
    """Operator parameters.  dims = (Lx, Ly, Lz, Lt); flavor in {PLUS, MINUS, NDEG}."""
    dims: tuple
    kappa: float
    mu: float
    eps: float = 0.0
    flavor: int = PLUS
    tsign: float = -1.0   # -1: antiperiodic in t
    # twisted clover (see with_clover): c_sw and the per-site R, R^-1 on
    # (flavour, spin, colour), shape [Lt, Lz, Ly, Lx, 12 nf, 12 nf]
    csw: float = 0.0
    clover_R: object = None
    clover_Rinv: object = None

    @property
    def nf(self) -> int:
        return 2 if self.flavor == NDEG else 1

    @property
    def a(self) -> float:
        return 2.0 * self.kappa * self.mu

    @property
    def b(self) -> float:
        return 2.0 * self.kappa * self.eps if self.flavor == NDEG else 0.0


def twist_matrix(p: Params, inverse: bool = False, dagger: bool = False) -> np.ndarray:
    """R or R^-1 (optionally daggered) as a (4 nf) x (4 nf) matrix on (flavour, spin)."""
    if p.nf == 1:
        s = 1.0 if p.flavor == PLUS else -1.0
        if not inverse:
            m = np.eye(4) + 1j * s * p.a * GAMMA5
        else:
            m = (np.eye(4) - 1j * s * p.a * GAMMA5) / (1.0 + p.a ** 2)
    else:
        if not inverse:
            m = np.eye(8) + 1j * p.a * np.kron(TAU3, GAMMA5) + p.b * np.kron(TAU1, np.eye(4))
        else:
            d = 1.0 + p.a ** 2 - p.b ** 2
            m = (np.eye(8) - 1j * p.a * np.kron(TAU3, GAMMA5) - p.b * np.kron(TAU1, np.eye(4))) / d
    m = m.astype(np.complex128)
    return m.conj().T.copy() if dagger else m


def _site_apply(m: np.ndarray, psi: np.ndarray) -> np.ndarray:
    nf = psi.shape[-3]
    sh = psi.shape
    v = psi.reshape(sh[:-3] + (nf * 4, 3))
    return np.einsum("ij,...jc->...ic", m, v).reshape(sh)


def parity_mask(dims, parity: int) -> np.ndarray:
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    return ((x + y + z + t) & 1) == parity


def project(psi: np.ndarray, dims, parity: int) -> np.ndarray:
    """Zero the sites of the other parity (psi canonical, optionally with a rhs axis)."""
    m = parity_mask(dims, parity)[..., None, None, None]
    return psi * m


def twist(p: Params, psi: np.ndarray, inverse=False, dagger=False, parity: int = -1):
    """R psi, R^-1 psi, R^+ psi or R^-+ psi on every site (parity -1) or one parity.
    With a clover term attached (with_clover) R is the per-site matrix."""
    if p.clover_R is not None:
        m = p.clover_Rinv if inverse else p.clover_R
        if dagger:
            m = np.conj(np.swapaxes(m, -1, -2))
        sh = psi.shape
        v = psi.reshape(sh[:-3] + (sh[-3] * 12,))
        out = np.einsum("...ij,...j->...i", m, v).reshape(sh)
    else:
        out = _site_apply(twist_matrix(p, inverse, dagger), psi)
    return out if parity < 0 else project(out, p.dims, parity)


def hop(p: Params, U: np.ndarray, psi: np.ndarray, out_parity: int = -1, dagger=False):
    """Wilson hop D psi (or D^+ psi) through the C loop; see tm_oracle.c."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    U = np.ascontiguousarray(U, dtype=np.complex128)
    nrhs = 1 if psi.ndim == 7 else psi.shape[0]
    assert psi.shape[-3] == p.nf
    out = np.empty_like(psi)
    dims = (ctypes.c_int * 4)(*p.dims)
    lib().orc_hop(_dp(out), _dp(psi), _dp(U), dims, p.nf, nrhs, int(bool(dagger)),
                  float(p.tsign), int(out_parity))
    return out


# --- full and preconditioned operators ---------------------------------------

EVEN, ODD = 0, 1


def full_M(p: Params, U, psi, dagger=False):
    """M psi = R psi - kappa D psi (Eq. 2.1 times 2 kappa); M^+ = R^+ - kappa D^+."""
    return twist(p, psi, dagger=dagger) - p.kappa * hop(p, U, psi, dagger=dagger)


def mat_pc(p: Params, U, x_e, pc: str = "asym", dagger=False):
    """Preconditioned even-even operator of Eq. (2.2) (asym) or Eq. (2.3) (sym)."""
    k2 = p.kappa ** 2
    if pc == "asym":
        if not dagger:
            t = twist(p, hop(p, U, x_e, ODD), inverse=True, parity=ODD)
            return twist(p, x_e, parity=EVEN) - k2 * hop(p, U, t, EVEN)
        # (R_ee - k^2 D_eo R_oo^-1 D_oe)^+ = R_ee^+ - k^2 (D_oe)^+ R_oo^-+ (D_eo)^+
        t = twist(p, hop(p, U, x_e, ODD, dagger=True), inverse=True, dagger=True, parity=ODD)
        return twist(p, x_e, dagger=True, parity=EVEN) - k2 * hop(p, U, t, EVEN, dagger=True)
    if pc == "sym":
        if not dagger:
            t = twist(p, hop(p, U, x_e, ODD), inverse=True, parity=ODD)
            return x_e - k2 * twist(p, hop(p, U, t, EVEN), inverse=True, parity=EVEN)
        # (1 - k^2 R_ee^-1 D_eo R_oo^-1 D_oe)^+ = 1 - k^2 (D_oe)^+ R_oo^-+ (D_eo)^+ R_ee^-+
        y = twist(p, x_e, inverse=True, dagger=True, parity=EVEN)
        t = twist(p, hop(p, U, y, ODD, dagger=True), inverse=True, dagger=True, parity=ODD)
        return x_e - k2 * hop(p, U, t, EVEN, dagger=True)
    raise ValueError(pc)


def normal_op(p: Params, U, x_e, pc="asym"):
    return mat_pc(p, U, mat_pc(p, U, x_e, pc), pc, dagger=True)


def prepare(p: Params, U, b, pc="asym"):
    """Even right-hand side of the Schur system from a full source b."""
    b_e = project(b, p.dims, EVEN)
    b_o = project(b, p.dims, ODD)
    rhs = b_e + p.kappa * hop(p, U, twist(p, b_o, inverse=True, parity=ODD), EVEN)
    if pc == "sym":
        rhs = twist(p, rhs, inverse=True, parity=EVEN)
    return rhs


def reconstruct(p: Params, U, x_e, b):
    """Odd half of the solution: R_oo^-1 (b_o + kappa D_oe x_e)."""
    b_o = project(b, p.dims, ODD)
    return twist(p, b_o + p.kappa * hop(p, U, x_e, ODD), inverse=True, parity=ODD)


def _dot(a, b):
    return complex(np.vdot(a, b))


def _nrm2(a):
    return float(np.vdot(a, a).real)


def cg(p: Params, U, b_e, pc="asym", tol=1e-10, maxiter=10000, x0=None, progress=None):
    """CG on M^+ M x = M^+ b in FP64 (normal equations, even sites).

    Stops when the true residual |M^+ b - M^+ M x| <= tol |M^+ b|.  Returns
    (x, info) with info = dict(iters, true_rel_res_normal, true_rel_res_pc).
    progress: optional callable(iteration, |r| / |M^+ b|) after each iteration
    (output for long runs; it takes no part in the arithmetic).
    """
    c = mat_pc(p, U, b_e, pc, dagger=True)
    x = np.zeros_like(b_e) if x0 is None else x0.copy()
    r = c - normal_op(p, U, x, pc) if x0 is not None else c.copy()
    cc = _nrm2(c)
    pdir = r.copy()
    rr = _nrm2(r)
    it = 0
    while it < maxiter:
        if rr <= tol * tol * cc:
            rtrue = c - normal_op(p, U, x, pc)
            if _nrm2(rtrue) <= tol * tol * cc:
                break
            r = rtrue                       # restart from the true residual
            rr = _nrm2(r)
            pdir = r.copy()
        mp = mat_pc(p, U, pdir, pc)
        ap = mat_pc(p, U, mp, pc, dagger=True)
        alpha = rr / _nrm2(mp)
        x = x + alpha * pdir
        r = r - alpha * ap
        rr_new = _nrm2(r)
        pdir = r + (rr_new / rr) * pdir
        rr = rr_new
        it += 1
        if progress is not None:
            progress(it, np.sqrt(rr / cc))
    rn = np.sqrt(_nrm2(c - normal_op(p, U, x, pc)) / cc)
    rp = np.sqrt(_nrm2(b_e - mat_pc(p, U, x, pc)) / _nrm2(b_e))
    return x, dict(iters=it, true_rel_res_normal=rn, true_rel_res_pc=rp)


def solve(p: Params, U, b, pc="asym", tol=1e-12, maxiter=10000):
    """Full solution of M psi = b by the Schur route: prepare, CG, reconstruct."""
    rhs = prepare(p, U, b, pc)
    x_e, info = cg(p, U, rhs, pc, tol, maxiter)
    return x_e + reconstruct(p, U, x_e, b), info


# --- twisted clover (the paper's stated future work, Sec. 4) ------------------
#
# M = R - kappa D with R(x) = A(x) + i a g5 t3 + b t1 and the clover term
#     A(x) = 1 + i kappa c_sw sum_{mu<nu} sigma_munu F_munu(x),
#     sigma_munu = (i/2)[g_mu, g_nu],  F_munu = (Q_munu - Q_munu^+) / 8,
# Q_munu(x) the sum of the four plaquettes of the mu-nu plane that start and
# end at x (counter-clockwise).  c_sw = 0 gives back the twisted-mass R.

def _nbr(f, mu, d):
    """f(x + d mu^) for a field [Lt, Lz, Ly, Lx, ...]."""
    return np.roll(f, -d, axis=3 - mu)


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def clover_leaves(U, mu, nu):
    """Q_munu(x): the four plaquette leaves of the mu-nu plane at every site."""
    Um, Un = U[mu], U[nu]
    mm = lambda *ms: ms[0] if len(ms) == 1 else ms[0] @ mm(*ms[1:])
    l1 = mm(Um, _nbr(Un, mu, 1), _dag(_nbr(Um, nu, 1)), _dag(Un))
    Um_b = _nbr(Um, mu, -1)                       # U_mu(x - mu)
    l2 = mm(Un, _dag(_nbr(Um_b, nu, 1)), _dag(_nbr(Un, mu, -1)), Um_b)
    Un_b = _nbr(Un, nu, -1)                       # U_nu(x - nu)
    l3 = mm(_dag(Um_b), _dag(_nbr(Un_b, mu, -1)), _nbr(Um_b, nu, -1), Un_b)
    l4 = mm(_dag(Un_b), _nbr(Um, nu, -1), _nbr(Un_b, mu, 1), _dag(Um))
    return l1 + l2 + l3 + l4


def clover_term(p: Params, U, csw):
    """A(x) on (spin, colour), shape [Lt, Lz, Ly, Lx, 12, 12]."""
    g = gammas()
    sh = U.shape[1:5]
    A = np.zeros(sh + (12, 12), dtype=np.complex128)
    A[...] = np.eye(12)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            sig = 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])
            Q = clover_leaves(U, mu, nu)
            F = (Q - _dag(Q)) / 8.0
            # kron(sigma, F) per site
            A += 1j * p.kappa * csw * np.einsum("ab,...cd->...acbd", sig, F).reshape(sh + (12, 12))
    return A


def with_clover(p: Params, U, csw):
    """A copy of p whose twist is the twisted-clover R(x) (and R^-1 by inversion)."""
    from dataclasses import replace
    A = clover_term(p, U, csw)
    nf = p.nf
    sh = A.shape[:4]
    R = np.zeros(sh + (12 * nf, 12 * nf), dtype=np.complex128)
    tw = twist_matrix(p)                      # 1 + i a g5 t3 + b t1 on (flavour, spin)
    for f in range(nf):
        for h in range(nf):
            blk = np.kron(tw[4 * f:4 * f + 4, 4 * h:4 * h + 4], np.eye(3))
            if f == h:
                blk = blk - np.eye(12) + A    # the clover term replaces the 1
            R[..., 12 * f:12 * f + 12, 12 * h:12 * h + 12] = blk
    return replace(p, csw=csw, clover_R=R, clover_Rinv=np.linalg.inv(R))


# --- full-system solves (Sec. 2.2: solution types) ---------------------------

def cg_full_normal(p: Params, U, b, tol=1e-12, maxiter=100000):
    """CG on M^+ M x = b over the whole lattice with no preconditioning: the
    plain definition of the MATDAG_MAT solution of Sec. 2.2.  Stops on the true
    residual |b - M^+ M x| <= tol |b|."""
    def A(v):
        return full_M(p, U, full_M(p, U, v), dagger=True)

    x = np.zeros_like(b)
    r = b.copy()
    bb = _nrm2(b)
    pdir = r.copy()
    rr = _nrm2(r)
    it = 0
    while it < maxiter:
        if rr <= tol * tol * bb:
            rtrue = b - A(x)
            if _nrm2(rtrue) <= tol * tol * bb:
                break
            r = rtrue
            rr = _nrm2(r)
            pdir = r.copy()
        ap = A(pdir)
        alpha = rr / _dot(pdir, ap).real
        x = x + alpha * pdir
        r = r - alpha * ap
        rr_new = _nrm2(r)
        pdir = r + (rr_new / rr) * pdir
        rr = rr_new
        it += 1
    return x, dict(iters=it, true_rel_res=np.sqrt(_nrm2(b - A(x)) / bb))


def solve_full(p: Params, U, b, solution="mat", pc="asym", tol=1e-12):
    """Solution of the full system: M psi = b ("mat", by the Schur route of
    Eqs. 2.2-2.4) or M^+ M psi = b ("matdag_mat", plain CG on the full lattice)."""
    if solution == "mat":
        return solve(p, U, b, pc, tol)
    if solution == "matdag_mat":
        return cg_full_normal(p, U, b, tol)
    raise ValueError(solution)


# --- chiral basis (Sec. 2: conversion into the internal basis) ---------------
#
# The internal basis is the non-relativistic one of Sec. 2 (g4 diagonal).  The
# chiral basis has g5 diagonal; the two are related by the real orthogonal
# S = H (x) 1_2 on the spin index, H = [[1, 1], [1, -1]] / sqrt 2 acting on the
# upper / lower pairs of spin components:
#     psi_chiral = S psi_internal,   g_chiral = S g_internal S^T.
# S is symmetric and its own inverse.

CHIRAL_S = np.kron(np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0), np.eye(2)).astype(np.complex128)


def _spin_apply(m, psi):
    return np.einsum("ij,...jc->...ic", m, psi)


def to_chiral(psi):
    """Internal-basis spinor (canonical, spin axis -2) -> chiral basis."""
    return _spin_apply(CHIRAL_S, psi)


def from_chiral(psi):
    """Chiral-basis spinor -> internal basis."""
    return _spin_apply(CHIRAL_S.conj().T, psi)


def chiral_gammas():
    """g_mu (x, y, z, t) in the chiral basis, S g S^T of the internal ones."""
    g = gammas()
    return np.einsum("ij,mjk,lk->mil", CHIRAL_S, g, CHIRAL_S.conj())


# --- gauge force -------------------------------------------------------------
#
# S = phi^+ (M^+ M)^-1 phi with M the preconditioned operator on even sites.
# A link variation U -> exp(w^a T^a) U, T^a = i lambda_a / 2, changes S by
# dS/dw^a = f^a; the force is F = sum_a f^a T^a (traceless anti-Hermitian),
# i.e. f^a = -2 tr(F T^a).  The unconstrained complex gradient G (the one
# torch returns for a real function of complex U) obeys dS = Re tr(G^+ dU).

def _gell_mann():
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return lam


SU3_GENERATORS = 0.5j * _gell_mann()      # T^a, tr(T^a T^b) = -delta_ab / 2


def action(p: Params, U, phi_e, pc="asym", tol=1e-14):
    """S = <phi, (M^+ M)^-1 phi> (real) and X = (M^+ M)^-1 phi by FP64 CG."""
    X = _cg_normal(p, U, phi_e, pc, tol)
    return float(np.vdot(phi_e, X).real), X


def _cg_normal(p, U, c, pc, tol, maxiter=100000):
    """Plain CG on M^+ M X = c (c given directly)."""
    x = np.zeros_like(c)
    r = c.copy()
    d = r.copy()
    rr = _nrm2(r)
    cc = _nrm2(c)
    for _ in range(maxiter):
        if rr <= tol * tol * cc:
            break
        mp = mat_pc(p, U, d, pc)
        alpha = rr / _nrm2(mp)
        x = x + alpha * d
        r = r - alpha * mat_pc(p, U, mp, pc, dagger=True)
        rr_new = _nrm2(r)
        d = r + (rr_new / rr) * d
        rr = rr_new
    return x


def force_product_rule(p: Params, U, X_e, links, pc="asym"):
    """dS/dw^a for the listed links (mu, t, z, y, x) from the product rule
    dM = -k^2 (dD_eo R_oo^-1 D_oe + D_eo R_oo^-1 dD_oe) (times R_ee^-1 for sym),
    dS = -2 Re <M X, dM X>, with dD the hop built from the varied link alone
    (D is linear in the links).  Returns F per listed link as [n, 3, 3]."""
    Y = mat_pc(p, U, X_e, pc)
    Z = twist(p, hop(p, U, X_e, ODD), inverse=True, parity=ODD)
    out = []
    for (mu, t, z, y, x) in links:
        F = np.zeros((3, 3), dtype=np.complex128)
        for a in range(8):
            dU = np.zeros_like(U)
            dU[mu, t, z, y, x] = SU3_GENERATORS[a] @ U[mu, t, z, y, x]
            dmx = hop(p, dU, Z, EVEN) + hop(p, U, twist(p, hop(p, dU, X_e, ODD), inverse=True,
                                                        parity=ODD), EVEN)
            if pc == "sym":
                dmx = twist(p, dmx, inverse=True, parity=EVEN)
            dmx = -p.kappa ** 2 * dmx
            f = -2.0 * np.vdot(Y, dmx).real
            F += f * SU3_GENERATORS[a]
        out.append(F)
    return np.array(out)


def _traceless_antiherm(m):
    a = 0.5 * (m - np.swapaxes(m.conj(), -1, -2))
    tr = np.trace(a, axis1=-2, axis2=-1)[..., None, None]
    return a - tr / 3.0 * np.eye(3)


def force(p: Params, U, X_e, pc="asym"):
    """Force on every link from outer products of spinor fields:
    with Y = M X, A = (Y or R_ee^-+ Y for sym) on even sites and
    R_oo^-+ (D^+)_oe of that on odd sites, B = X on even and R_oo^-1 D_oe X on
    odd sites, dS = 2 k^2 Re <A, dD B>, so for the link U_mu(x) with boundary
    factor s
      G = 2 k^2 s sum_{flavour, spin} [ (1 - g_mu) A(x) B(x+mu)^+ + B(x) ((1 + g_mu) A(x+mu))^+ ],
      F = -1/2 T_A(U G^+).
    Returns (F, G), complex [4, Lt, Lz, Ly, Lx, 3, 3]."""
    Y = mat_pc(p, U, X_e, pc)
    Ae = twist(p, Y, inverse=True, dagger=True, parity=EVEN) if pc == "sym" else Y
    Wo = twist(p, hop(p, U, Ae, ODD, dagger=True), inverse=True, dagger=True, parity=ODD)
    Zo = twist(p, hop(p, U, X_e, ODD), inverse=True, parity=ODD)
    A = Ae + Wo
    B = X_e + Zo
    g = gammas()
    lt = p.dims[3]
    G = np.zeros_like(U)
    for mu in range(4):
        ax = 3 - mu                          # array axis of direction mu in [t, z, y, x]
        Af = np.roll(A, -1, axis=ax)
        Bf = np.roll(B, -1, axis=ax)
        Pm = np.eye(4) - g[mu]
        Pp = np.eye(4) + g[mu]
        PmA = np.einsum("st,...ftc->...fsc", Pm, A)
        PpAf = np.einsum("st,...ftc->...fsc", Pp, Af)
        term = (np.einsum("...fsa,...fsb->...ab", PmA, Bf.conj())
                + np.einsum("...fsa,...fsb->...ab", B, PpAf.conj()))
        if mu == 3:
            sb = np.ones(term.shape[:4])
            sb[lt - 1] = p.tsign
            term = term * sb[..., None, None]
        G[mu] = 2.0 * p.kappa ** 2 * term
    F = -0.5 * _traceless_antiherm(U @ np.swapaxes(G.conj(), -1, -2))
    return F, G
