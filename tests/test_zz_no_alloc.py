"""tm_mat_pc_noalloc (the allocation-free operator call: its temporaries in a
device scratch array) against tm_mat_pc, the entry point with the same kernels
whose temporary the context allocates: bit-identical outputs on two calls in
a row, the second on a smaller lattice (the scratch keeps the first call's
contents), in every form, precision and flavour content, for twisted clover's
sym^+ (two temporaries), and against the oracle on the smaller lattice.  A
fresh context's call allocates no device memory of the temporary's size, and
a request beyond the scratch is refused before any launch."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1311_4462_amd import inputs
from tests.gpu_util import TOL, from_native, oparams, rel, to_native

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1311_4462_amd import api as A
    return A


def _fields(api, ctx, dims, flavor, csw=0.0):
    p = api.make_params(dims, 0.1615, 0.15, 0.19 if flavor == 2 else 0.0, flavor, csw=csw)
    op = oparams(p)
    U = inputs.gauge_field(dims, "near_unit", 401)
    precs = (0, 1) if csw else (0, 1, 2)
    g = api.Gauge(ctx, U, p, precs=precs)
    x = O.project(inputs.gaussian_spinor(dims, op.nf, 402), dims, 0)
    return p, op, U, g, x, precs


@pytest.mark.parametrize("flavor", [1, 2])
def test_noalloc_matches_tm_mat_pc_two_calls(api, flavor):
    import torch
    c = api.Context()
    # first call on the larger lattice, second on the smaller one
    for dims in ((16, 16, 16, 32), (8, 4, 6, 10)):
        p, op, U, g, x, precs = _fields(api, c, dims, flavor)
        for prec in precs:
            t = to_native(api, c, x, p, prec, 0)
            xq = from_native(api, c, t, p, prec, 0)[0]
            a = api.new_field(p, prec)
            b = api.new_field(p, prec)
            for pc in (0, 1):
                for dag in (0, 1):
                    api.tm_mat_pc_noalloc(c, a, t, g, prec, pc, dag)
                    api.tm_mat_pc(c, b, t, g, prec, pc, dag)
                    torch.cuda.synchronize()
                    assert torch.equal(a, b), (dims, prec, pc, dag)
                    if dims[0] == 8:
                        ref = O.mat_pc(op, U, xq, "asym" if pc == 0 else "sym", bool(dag))
                        got = from_native(api, c, a, p, prec, 0)[0]
                        assert rel(got, ref) < TOL[prec], (dims, prec, pc, dag)
        g.close()
    c.close()


def test_noalloc_clover_sym_dagger(api):
    """Twisted clover sym^+ takes both temporaries from the scratch."""
    import torch
    c = api.Context()
    for dims in ((8, 8, 8, 16), (4, 4, 6, 8)):
        p, op, U, g, x, precs = _fields(api, c, dims, 1, csw=1.57)
        for prec in precs:
            t = to_native(api, c, x, p, prec, 0)
            a = api.new_field(p, prec)
            b = api.new_field(p, prec)
            for pc in (0, 1):
                for dag in (0, 1):
                    api.tm_mat_pc_noalloc(c, a, t, g, prec, pc, dag)
                    api.tm_mat_pc(c, b, t, g, prec, pc, dag)
                    torch.cuda.synchronize()
                    assert torch.equal(a, b), (dims, prec, pc, dag)
        g.close()
    c.close()


def test_noalloc_allocates_nothing_and_refuses_oversize(api):
    import torch
    from paper_1311_4462_amd._lib import TMError
    dims = (16, 16, 16, 32)
    warm = api.Context()
    p, op, U, g, x, precs = _fields(api, warm, dims, 2)
    t = to_native(api, warm, x, p, 1, 0)
    a = api.new_field(p, 1)
    b = api.new_field(p, 1)
    api.tm_mat_pc(warm, b, t, g, 1, 0, 0)          # loads the kernels' code
    torch.cuda.synchronize()
    fresh = api.Context()                          # no workspace yet
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        api.tm_mat_pc_noalloc(fresh, a, t, g, 1, 0, 0)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    odd_bytes = api.tm_spinor_bytes(p, 1)
    assert free0 - free1 < odd_bytes // 2, (free0, free1, odd_bytes)
    assert torch.equal(a, b)
    # beyond the 256 MiB scratch (FP64 doublet, 16^3 x 32: 25 MB per rhs)
    nbig = (256 << 20) // api.tm_spinor_bytes(p, 0) + 1
    with pytest.raises(TMError) as e:
        api.tm_mat_pc_noalloc(fresh, a, b, g, 0, 0, 0, nbig)
    assert e.value.code == -9
    g.close()
    fresh.close()
    warm.close()
