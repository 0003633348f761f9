"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the twisted-mass method: it only draws
gauge links, gauge transformations and source fields from fixed seeds, in the
canonical layout

    links   : complex128 [4, Lt, Lz, Ly, Lx, 3, 3]   (direction mu = x, y, z, t)
    spinors : complex128 [(nrhs,) Lt, Lz, Ly, Lx, nf, 4, 3]

Both sides of every parity check receive the very same arrays.

Distributions (stand-ins for the paper's gauge ensembles, which are not
available; the paper's single-GPU lattice is 32^3 x 64, Sec. 3):
  * ``haar_su3``       complex Gaussian 3x3, Gram-Schmidt by rows with the
                       diagonal phases of the triangular factor made positive,
                       then multiplied by exp(-i arg(det)/3) (principal branch)
                       so that det = 1.
  * ``near_unit_su3``  exp(i * eps * H), H = sum_a h_a lambda_a / 2 with
                       h_a ~ N(0, 1) and lambda_a the Gell-Mann matrices;
                       computed through the eigen-decomposition of H.
  * ``gaussian_spinor`` real and imaginary parts i.i.d. N(0, 1).
  * ``z2_spinor``      every complex entry (+-1 +- i)/sqrt(2), signs uniform.
"""
from __future__ import annotations

import concurrent.futures as _cf
import os

import numpy as np

__all__ = [
    "haar_su3", "near_unit_su3", "gauge_field", "gaussian_spinor", "z2_spinor",
    "random_gauge_transform", "unit_gauge", "GELL_MANN",
]


def _gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


GELL_MANN = _gell_mann()


def _nthreads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def haar_su3(rng: np.random.Generator, n: int) -> np.ndarray:
    """n random SU(3) matrices from Gram-Schmidt of complex Gaussian matrices."""
    g = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    # Gram-Schmidt on rows == QR of the transpose; fix the phases so that the
    # triangular factor has a positive real diagonal.
    q, r = np.linalg.qr(np.swapaxes(g, 1, 2))
    d = np.diagonal(r, axis1=1, axis2=2)
    ph = d / np.abs(d)
    q = q * ph[:, None, :]
    u = np.swapaxes(q, 1, 2).copy()
    det = np.linalg.det(u)
    u *= np.exp(-1j * np.angle(det) / 3.0)[:, None, None]
    return u


def _expm_herm(h: np.ndarray, eps: float) -> np.ndarray:
    w, v = np.linalg.eigh(h)
    return np.einsum("nij,nj,nkj->nik", v, np.exp(1j * eps * w), v.conj())


def near_unit_su3(rng: np.random.Generator, n: int, eps: float = 0.3) -> np.ndarray:
    """n matrices exp(i*eps*H), H = sum_a h_a lambda_a / 2, h_a ~ N(0,1)."""
    coef = rng.standard_normal((n, 8))
    h = np.einsum("na,aij->nij", coef, GELL_MANN / 2.0)
    chunks = np.array_split(np.arange(n), _nthreads())
    out = np.empty((n, 3, 3), dtype=np.complex128)
    with _cf.ThreadPoolExecutor(len(chunks)) as ex:
        futs = {ex.submit(_expm_herm, h[c[0]:c[-1] + 1], eps): c for c in chunks if len(c)}
        for f, c in futs.items():
            out[c[0]:c[-1] + 1] = f.result()
    return out


def gauge_field(dims, kind: str, seed: int) -> np.ndarray:
    """Links U_mu(x), complex128 [4, Lt, Lz, Ly, Lx, 3, 3]; dims = (Lx, Ly, Lz, Lt)."""
    lx, ly, lz, lt = dims
    n = 4 * lx * ly * lz * lt
    rng = np.random.default_rng(seed)
    if kind == "haar":
        u = haar_su3(rng, n)
    elif kind == "near_unit":
        u = near_unit_su3(rng, n)
    else:
        raise ValueError(f"unknown gauge kind {kind!r}")
    return u.reshape(4, lt, lz, ly, lx, 3, 3)


def unit_gauge(dims) -> np.ndarray:
    lx, ly, lz, lt = dims
    u = np.zeros((4, lt, lz, ly, lx, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1
    return u


def random_gauge_transform(dims, seed: int) -> np.ndarray:
    """One Haar SU(3) matrix per site, complex128 [Lt, Lz, Ly, Lx, 3, 3]."""
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(seed)
    return haar_su3(rng, lx * ly * lz * lt).reshape(lt, lz, ly, lx, 3, 3)


def _shape(dims, nf, nrhs):
    lx, ly, lz, lt = dims
    s = (lt, lz, ly, lx, nf, 4, 3)
    return s if nrhs is None else (nrhs,) + s


def gaussian_spinor(dims, nf: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    rng = np.random.default_rng(seed)
    s = _shape(dims, nf, nrhs)
    return rng.standard_normal(s) + 1j * rng.standard_normal(s)


def z2_spinor(dims, nf: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    rng = np.random.default_rng(seed)
    s = _shape(dims, nf, nrhs)
    re = rng.integers(0, 2, size=s) * 2 - 1
    im = rng.integers(0, 2, size=s) * 2 - 1
    return (re + 1j * im) / np.sqrt(2.0)


def parity_mask(dims) -> np.ndarray:
    """(x+y+z+t) & 1 as int array [Lt, Lz, Ly, Lx] (site bookkeeping only)."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    return (x + y + z + t) & 1


def parity_project(psi: np.ndarray, dims, parity: int) -> np.ndarray:
    """Copy of a canonical field with the sites of the other parity set to zero."""
    m = (parity_mask(dims) == parity)
    out = psi.copy()
    bshape = m.shape + (1,) * 3
    if psi.ndim == 8:
        out *= m.reshape((1,) + bshape)
    else:
        out *= m.reshape(bshape)
    return out
