"""Pins of the oracle's gauge force (S = phi^+ (M^+ M)^-1 phi) against central
finite differences of S along random su(3) directions (step 1e-5), against the
product-rule derivative of the operator built from the varied link alone, and
against its invariants (traceless anti-Hermitian, gauge covariant)."""
import numpy as np
import pytest

from paper_1311_4462_amd import inputs

DIMS = (4, 4, 4, 4)
LINKS = [(0, 0, 0, 0, 0), (3, 3, 1, 2, 1), (1, 2, 3, 0, 1), (2, 1, 0, 3, 2), (3, 0, 2, 2, 3),
         (3, 3, 3, 3, 3)]


def _setup(orc, flavor, pc, seed=1005):
    p = orc.Params(DIMS, 0.1615, 0.15, 0.19 if flavor == orc.NDEG else 0.0, flavor)
    U = inputs.gauge_field(DIMS, "near_unit", seed)
    phi = orc.project(inputs.gaussian_spinor(DIMS, p.nf, seed + 1000), DIMS, 0)
    S, X = orc.action(p, U, phi, pc)
    return p, U, phi, S, X


def _exp_step(orc, H, h):
    ev, V = np.linalg.eigh((-1j * h * H).reshape(-1, 3, 3))
    return np.einsum("nij,nj,nkj->nik", V, np.exp(1j * ev), V.conj()).reshape(H.shape)


@pytest.mark.parametrize("flavor,pc", [(2, "asym"), (1, "asym"), (2, "sym"), (-1, "sym")])
def test_force_matches_central_differences(orc, flavor, pc):
    p, U, phi, S, X = _setup(orc, flavor, pc)
    F, G = orc.force(p, U, X, pc)
    rng = np.random.default_rng(17)
    w = rng.standard_normal((4,) + DIMS[::-1] + (8,))
    H = np.einsum("...a,aij->...ij", w, orc.SU3_GENERATORS)
    h = 1e-5
    Sp, _ = orc.action(p, _exp_step(orc, H, h) @ U, phi, pc)
    Sm, _ = orc.action(p, _exp_step(orc, H, -h) @ U, phi, pc)
    fd = (Sp - Sm) / (2 * h)
    fa = -2.0 * np.einsum("...ij,aji->...a", F, orc.SU3_GENERATORS).real
    an = float(np.sum(w * fa))
    assert abs(fd - an) <= 1e-7 * abs(an)
    # the unconstrained gradient: dS = Re tr(G^+ dU) for arbitrary complex dU
    dU = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
    Sp, _ = orc.action(p, U + h * dU, phi, pc)
    Sm, _ = orc.action(p, U - h * dU, phi, pc)
    fd = (Sp - Sm) / (2 * h)
    an = float(np.sum(G.conj() * dU).real)
    assert abs(fd - an) <= 1e-7 * abs(an)


@pytest.mark.parametrize("flavor,pc", [(2, "asym"), (1, "sym")])
def test_force_formula_matches_product_rule(orc, flavor, pc):
    p, U, phi, S, X = _setup(orc, flavor, pc)
    F, _ = orc.force(p, U, X, pc)
    Fp = orc.force_product_rule(p, U, X, LINKS, pc)
    Fa = np.array([F[l] for l in LINKS])
    assert np.abs(Fp - Fa).max() <= 1e-12 * np.abs(Fa).max()


def test_force_invariants(orc):
    p, U, phi, S, X = _setup(orc, orc.NDEG, "asym")
    F, G = orc.force(p, U, X, "asym")
    assert np.abs(F + np.swapaxes(F.conj(), -1, -2)).max() < 1e-13 * np.abs(F).max()
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() < 1e-13 * np.abs(F).max()
    # F = -1/2 T_A(U G^+) is what the formula returns; also the generator components
    # of F reproduce it (F = sum_a f^a T^a with f^a = -2 tr(F T^a))
    fa = -2.0 * np.einsum("...ij,aji->...a", F, orc.SU3_GENERATORS)
    assert np.abs(fa.imag).max() < 1e-12 * np.abs(fa).max()
    assert np.abs(np.einsum("...a,aij->...ij", fa.real, orc.SU3_GENERATORS) - F).max() < 1e-12
    # gauge covariance: U_mu(x) -> g(x) U g(x+mu)^+, phi -> g phi: F_mu(x) -> g(x) F g(x)^+
    g = inputs.random_gauge_transform(DIMS, 77)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[mu] = g @ U[mu] @ np.roll(g, -1, axis=3 - mu).conj().swapaxes(-1, -2)
    phig = np.einsum("tzyxab,tzyxfsb->tzyxfsa", g, phi)
    Sg, Xg = orc.action(p, Ug, phig, "asym")
    assert abs(Sg - S) < 1e-10 * abs(S)
    Fg, _ = orc.force(p, Ug, Xg, "asym")
    assert np.abs(Fg - g[None] @ F @ g[None].conj().swapaxes(-1, -2)).max() < 1e-9 * np.abs(F).max()
