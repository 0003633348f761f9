"""8-real link storage (a2, a3, b1 and the phases of a1, c1; the rest rebuilt
from unitarity and det U = 1) in every precision, against the FP64 oracle that
uses the full links.  Tolerances as for 12-real links: 1e-12 FP64, 1e-5 FP32,
5e-3 FP16 / BF16 (norm-wise relative)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1311_4462_amd import inputs
from tests.gpu_util import TOL, check_solve, from_native, oparams, oracle_dslash, rel, to_native

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


@pytest.mark.parametrize("kind", ["haar", "near_unit"])
@pytest.mark.parametrize("flavor", [1, -1, 2])
@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_mat_pc_recon8(api, ctx, kind, flavor, prec):
    dims = (8, 6, 4, 10)
    p = api.make_params(dims, 0.16, 0.13, 0.17 if flavor == 2 else 0.0, flavor)
    op = oparams(p)
    U = inputs.gauge_field(dims, kind, 81)
    g = api.Gauge(ctx, U, p, recon=8, precs=(prec,))
    x = O.project(inputs.gaussian_spinor(dims, op.nf, 82), dims, 0)
    t = to_native(api, ctx, x, p, prec, 0)
    out = api.new_field(p, prec)
    for pc in (0, 1):
        for dag in (0, 1):
            api.tm_mat_pc(ctx, out, t, g, prec, pc, dag)
            ref = O.mat_pc(op, U, x, "asym" if pc == 0 else "sym", bool(dag))
            got = from_native(api, ctx, out, p, prec, 0)[0]
            assert rel(got, ref) < TOL[prec], (pc, dag, rel(got, ref))
    g.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_dslash_epilogues_recon8(api, ctx, prec):
    dims = (6, 4, 4, 6)
    p = api.make_params(dims, 0.16, 0.13, 0.0, 1)
    op = oparams(p)
    U = inputs.gauge_field(dims, "haar", 83)
    g = api.Gauge(ctx, U, p, recon=8, precs=(prec,))
    for outp in (0, 1):
        inp = O.project(inputs.gaussian_spinor(dims, 1, 84), dims, 1 - outp)
        xv = O.project(inputs.gaussian_spinor(dims, 1, 85), dims, outp)
        ti, tx = to_native(api, ctx, inp, p, prec, 1 - outp), to_native(api, ctx, xv, p, prec, outp)
        out = api.new_field(p, prec)
        for epi in range(6):
            for dag in (0, 1):
                api.tm_dslash(ctx, out, ti, g, prec, outp, dag, 0, epi, tx, -0.37)
                ref = oracle_dslash(op, U, inp, outp, dag, 0, epi, xv, -0.37)
                assert rel(from_native(api, ctx, out, p, prec, outp)[0], ref) < TOL[prec]
    g.close()


def test_recon8_storage_and_cg(api, ctx):
    """Links take 8 reals (FP32: 32 bytes per link) and a mixed solve on 8-real
    links reaches the FP64 residual."""
    dims = (8, 8, 8, 8)
    p = api.make_params(dims, 0.1615, 0.15, 0.19, api.NDEG)
    op = oparams(p)
    U = inputs.gauge_field(dims, "near_unit", 86)
    g = api.Gauge(ctx, U, p, recon=8, precs=(0, 1, 2))
    vh = int(np.prod(dims)) // 2
    assert g.bytes(1) == 2 * 4 * vh * 32
    assert g.bytes(2) == 2 * 4 * vh * 16
    b = O.project(inputs.gaussian_spinor(dims, 2, 87), dims, 0)
    tb = to_native(api, ctx, b, p, 0, 0)
    tx = api.new_field(p, 0)
    r = api.tm_cg(ctx, tx, tb, g, tol=1e-10, inner=2)[0]
    assert r["status"] == 0 and r["true_rel_res_normal"] <= 1e-10
    x = from_native(api, ctx, tx, p, 0, 0)[0]
    check_solve(op, U, x, b, "asym", r["true_rel_res_normal"])
    g.close()


def test_recon8_rejects_unrepresentable_links(api, ctx):
    """A link whose first row is (a1, 0, 0) cannot be stored in 8 reals: the
    unit gauge field is refused, and the force kernel asks for 12 or 18."""
    from paper_1311_4462_amd._lib import TMError
    dims = (4, 4, 4, 4)
    p = api.make_params(dims, 0.16, 0.1)
    with pytest.raises(TMError) as e:
        api.Gauge(ctx, inputs.unit_gauge(dims), p, recon=8, precs=(0,))
    assert e.value.code == -1
    U = inputs.gauge_field(dims, "haar", 88)
    g = api.Gauge(ctx, U, p, recon=8, precs=(1,))
    x = api.new_field(p, 1)
    F = __import__("torch").empty((4,) + dims[::-1] + (3, 3), dtype=__import__("torch").complex64,
                                  device="cuda")
    with pytest.raises(TMError) as e:
        api.tm_force(ctx, F, 1, x, g, 1)
    assert e.value.code == -1
    g.close()
