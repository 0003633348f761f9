"""Full-system solves (Sec. 2.2 solution and solver types) and the chiral-basis
conversion of the pack/unpack routines, through the C ABI, against the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1311_4462_amd import inputs
from tests.gpu_util import from_native, oparams, rel, to_native

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1311_4462_amd import api as A
    return A


@pytest.fixture(scope="module")
def ctx(api):
    c = api.Context()
    yield c
    c.close()


def _setup(api, ctx, dims, flavor, seed, nrhs=1, precs=(0, 1)):
    p = api.make_params(dims, 0.16, 0.13, 0.17 if flavor == api.NDEG else 0.0, flavor)
    op = oparams(p)
    U = inputs.gauge_field(dims, "haar", seed)
    g = api.Gauge(ctx, U, p, precs=precs)
    b = inputs.gaussian_spinor(dims, op.nf, seed + 1, nrhs=nrhs) if nrhs > 1 else \
        inputs.gaussian_spinor(dims, op.nf, seed + 1)
    return p, op, U, g, b


def _full(api, ctx, xe, xo, p, nrhs=1):
    return from_native(api, ctx, xe, p, 0, 0, nrhs) + from_native(api, ctx, xo, p, 0, 1, nrhs)


def _native_halves(api, ctx, b, p, nrhs=1):
    return to_native(api, ctx, b, p, 0, 0, nrhs), to_native(api, ctx, b, p, 0, 1, nrhs)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("flavor", [1, 2])
def test_chiral_pack_unpack(api, ctx, prec, flavor):
    dims = (4, 2, 4, 6)
    p = api.make_params(dims, 0.16, 0.1, 0.2 if flavor == 2 else 0.0, flavor)
    nf = 2 if flavor == 2 else 1
    psi_ch = inputs.gaussian_spinor(dims, nf, 41)
    tol = 1e-14 if prec == 0 else 1e-6
    for par in (0, 1):
        t = api.tm_spinor_pack(ctx, psi_ch[None], p, prec, par, basis=api.BASIS_CHIRAL)
        internal = api.tm_spinor_unpack(ctx, t, p, prec, par).cpu().numpy()[0]
        assert rel(internal, O.project(O.from_chiral(psi_ch), dims, par)) < tol
        back = api.tm_spinor_unpack(ctx, t, p, prec, par, basis=api.BASIS_CHIRAL).cpu().numpy()[0]
        assert rel(back, O.project(psi_ch, dims, par)) < tol


@pytest.mark.parametrize("flavor", [1, -1, 2])
@pytest.mark.parametrize("pc", [0, 1])
@pytest.mark.parametrize("solution", [0, 1])
def test_solve_full_system(api, ctx, flavor, pc, solution):
    dims = (4, 4, 4, 6)
    p, op, U, g, b = _setup(api, ctx, dims, flavor, 50)
    be, bo = _native_halves(api, ctx, b, p)
    xe, xo = api.new_field(p, 0), api.new_field(p, 0)
    r = api.tm_solve(ctx, xe, xo, be, bo, g, solution=solution, pc=pc, tol=1e-12)[0]
    assert r["status"] == 0
    x = _full(api, ctx, xe, xo, p)
    if solution == 0:
        want, _ = O.solve_full(op, U, b, "mat", "asym" if pc == 0 else "sym", tol=1e-13)
        full_res = rel(O.full_M(op, U, x), b)
    else:
        want, _ = O.solve_full(op, U, b, "matdag_mat", tol=1e-13)
        full_res = rel(O.full_M(op, U, O.full_M(op, U, x), dagger=True), b)
    assert rel(x, want) < 1e-8
    # the reported residual of the full system is the one the oracle recomputes
    assert abs(r["true_rel_res_full"] - full_res) <= 1e-3 * full_res + 1e-15
    assert full_res < 1e-9
    g.close()


@pytest.mark.parametrize("pc", [0, 1])
def test_direct_pc_bounds_the_system_residual(api, ctx, pc):
    dims = (4, 4, 4, 6)
    p, op, U, g, b = _setup(api, ctx, dims, 2, 60)
    be, bo = _native_halves(api, ctx, b, p)
    xe, xo = api.new_field(p, 0), api.new_field(p, 0)
    tol = 1e-9
    r = api.tm_solve(ctx, xe, xo, be, bo, g, solve_type=api.SOLVE_DIRECT_PC, pc=pc, tol=tol)[0]
    assert r["status"] == 0 and r["true_rel_res_pc"] <= tol
    pcs = "asym" if pc == 0 else "sym"
    bh = O.prepare(op, U, b, pcs)
    x_e = from_native(api, ctx, xe, p, 0, 0)[0]
    assert rel(O.mat_pc(op, U, x_e, pcs), bh) <= tol * 1.0001
    g.close()


def test_solve_mixed_multi_rhs_chiral(api, ctx):
    """Four sources given in the chiral basis, FP32-inner mixed CG, MATDAG_MAT:
    the chiral-basis solution equals the oracle's solution converted back."""
    dims = (4, 4, 4, 8)
    nrhs = 4
    p, op, U, g, _ = _setup(api, ctx, dims, 1, 70)
    b_ch = inputs.gaussian_spinor(dims, 1, 71, nrhs=nrhs)
    be = api.tm_spinor_pack(ctx, b_ch, p, 0, 0, nrhs, basis=api.BASIS_CHIRAL)
    bo = api.tm_spinor_pack(ctx, b_ch, p, 0, 1, nrhs, basis=api.BASIS_CHIRAL)
    xe, xo = api.new_field(p, 0, nrhs), api.new_field(p, 0, nrhs)
    res = api.tm_solve(ctx, xe, xo, be, bo, g, solution=api.SOLUTION_MATDAG_MAT, inner=api.FP32,
                       tol=1e-11, nrhs=nrhs)
    assert all(r["status"] == 0 for r in res)
    x_ch = (api.tm_spinor_unpack(ctx, xe, p, 0, 0, nrhs, basis=api.BASIS_CHIRAL).cpu().numpy() +
            api.tm_spinor_unpack(ctx, xo, p, 0, 1, nrhs, basis=api.BASIS_CHIRAL).cpu().numpy())
    for k in (0, 3):
        want, _ = O.solve_full(op, U, O.from_chiral(b_ch[k]), "matdag_mat", tol=1e-13)
        assert rel(x_ch[k], O.to_chiral(want)) < 1e-7
    g.close()


def test_solve_errors(api, ctx):
    from paper_1311_4462_amd._lib import TMError
    dims = (4, 4, 4, 4)
    p, op, U, g, b = _setup(api, ctx, dims, 1, 80, precs=(0,))
    be, bo = _native_halves(api, ctx, b, p)
    xe, xo = api.new_field(p, 0), api.new_field(p, 0)
    for kw, code in ((dict(solve_type=5), -1), (dict(solution=3), -1), (dict(inner=1), -4),
                     (dict(tol=0.0), -1)):
        with pytest.raises(TMError) as e:
            api.tm_solve(ctx, xe, xo, be, bo, g, **kw)
        assert e.value.code == code
    with pytest.raises(TMError):
        api.tm_solve(ctx, xe, xe, be, bo, g)
    with pytest.raises(TMError):
        api.tm_spinor_pack(ctx, b[None], p, 0, 0, basis=2)
    g.close()
