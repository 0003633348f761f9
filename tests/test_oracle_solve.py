"""Pins of the oracle's full-system solution types and of its chiral basis
(Sec. 2 and Sec. 2.2) against brute force and written-out definitions."""
import numpy as np
import pytest

from paper_1311_4462_amd import inputs
from tests import dense_ref

PLUS, MINUS, NDEG = 1, -1, 2


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _params(orc, dims, flavor, kappa=0.16, mu=0.13, eps=0.17):
    return orc.Params(tuple(dims), kappa, mu, eps if flavor == NDEG else 0.0, flavor)


def test_chiral_gammas_are_the_written_out_chiral_set(orc):
    g = orc.chiral_gammas()
    ref = dense_ref.chiral_gammas()
    for mu in range(4):
        assert np.allclose(g[mu], ref[mu], atol=1e-15)
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    assert np.allclose(g5, np.diag([1, 1, -1, -1]), atol=1e-15)
    # Clifford algebra survives the change of basis
    for a in range(4):
        for b in range(4):
            assert np.allclose(g[a] @ g[b] + g[b] @ g[a], 2 * (a == b) * np.eye(4), atol=1e-14)


def test_chiral_conversion_is_unitary_and_invertible(orc):
    psi = inputs.gaussian_spinor((2, 2, 2, 2), 2, 5)
    ch = orc.to_chiral(psi)
    assert np.allclose(orc.from_chiral(ch), psi, atol=1e-14)
    assert abs(np.linalg.norm(ch) - np.linalg.norm(psi)) < 1e-12 * np.linalg.norm(psi)


def test_chiral_components_are_g5_eigenvectors(orc):
    """A chiral-basis spinor with only its first two spin components is a +1
    eigenvector of g5 in the internal basis; the last two give -1."""
    rng = np.random.default_rng(3)
    up = np.zeros((4, 3), complex)
    up[:2] = rng.normal(size=(2, 3)) + 1j * rng.normal(size=(2, 3))
    dn = np.zeros((4, 3), complex)
    dn[2:] = rng.normal(size=(2, 3)) + 1j * rng.normal(size=(2, 3))
    g = dense_ref.gammas()
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    for v, s in ((up, 1), (dn, -1)):
        w = orc.from_chiral(v)
        assert np.allclose(g5 @ w, s * w, atol=1e-14)


@pytest.mark.parametrize("flavor", [PLUS, NDEG])
def test_operator_in_chiral_basis_matches_dense_chiral_builder(orc, flavor):
    """Converting to the internal basis, applying M there and converting back
    equals M assembled directly from the chiral gamma matrices."""
    dims = (2, 2, 2, 4)
    p = _params(orc, dims, flavor)
    U = inputs.gauge_field(dims, "haar", 31)
    psi_ch = inputs.gaussian_spinor(dims, p.nf, 32)
    M_ch = dense_ref.dense_M(dims, U, p.kappa, p.mu, p.eps, p.nf, 1, gam=dense_ref.chiral_gammas())
    want = (M_ch @ psi_ch.reshape(-1)).reshape(psi_ch.shape)
    got = orc.to_chiral(orc.full_M(p, U, orc.from_chiral(psi_ch)))
    assert _rel(got, want) < 1e-13


@pytest.mark.parametrize("flavor", [PLUS, MINUS, NDEG])
def test_matdag_mat_solution_matches_dense(orc, flavor):
    dims = (2, 2, 2, 4)
    p = _params(orc, dims, flavor)
    U = inputs.gauge_field(dims, "haar", 33)
    b = inputs.gaussian_spinor(dims, p.nf, 34)
    M = dense_ref.dense_M(dims, U, p.kappa, p.mu, p.eps, p.nf, -1 if flavor == MINUS else 1)
    want = np.linalg.solve(M.conj().T @ M, b.reshape(-1)).reshape(b.shape)
    x, info = orc.solve_full(p, U, b, "matdag_mat", tol=1e-13)
    assert info["true_rel_res"] <= 1e-13
    assert _rel(x, want) < 1e-10
    xm, _ = orc.solve_full(p, U, b, "mat", "sym", tol=1e-13)
    assert _rel(xm, np.linalg.solve(M, b.reshape(-1)).reshape(b.shape)) < 1e-10
