"""GPU path (through the C ABI) against the FP64 oracle, element by element on
the same seeded inputs.  Tolerances (norm-wise relative): 1e-12 FP64 apply,
1e-5 FP32, 5e-3 FP16 / BF16; solves to a 1e-10 true FP64 residual."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1311_4462_amd import inputs
from tests.gpu_util import TOL, check_solve, from_native, oparams, oracle_dslash, rel, to_native

pytestmark = pytest.mark.gpu

SMALL_DIMS = [(2, 2, 2, 2), (4, 4, 4, 4), (6, 4, 4, 6), (8, 6, 4, 10)]


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


def _setup(api, ctx, dims, flavor, recon=12, precs=(0, 1, 2, 3), kind="haar", seed=3,
           kappa=0.16, mu=0.13, eps=0.17):
    p = api.make_params(dims, kappa, mu, eps if flavor == api.NDEG else 0.0, flavor)
    U = inputs.gauge_field(dims, kind, seed)
    g = api.Gauge(ctx, U, p, recon=recon, precs=precs)
    return p, U, g


# ------------------------------------------------------------------ layout

@pytest.mark.parametrize("prec", [0, 1, 2, 3])
@pytest.mark.parametrize("flavor", [1, 2])
def test_pack_unpack_roundtrip(api, ctx, prec, flavor):
    dims = (6, 4, 4, 6)
    p = api.make_params(dims, 0.16, 0.1, 0.1 if flavor == 2 else 0.0, flavor)
    nf = 2 if flavor == 2 else 1
    a = inputs.gaussian_spinor(dims, nf, 5, nrhs=2)
    for par in (0, 1):
        t = to_native(api, ctx, a, p, prec, par, 2)
        back = from_native(api, ctx, t, p, prec, par, 2)
        ref = O.project(a, dims, par)
        if prec == 0:
            assert np.array_equal(back, ref)
        else:
            assert rel(back, ref) < {1: 1e-7, 2: 1e-3, 3: 5e-3}[prec]
            assert np.all(back[O.project(np.ones_like(a), dims, 1 - par) != 0] == 0)


# ------------------------------------------------------------------ hop + epilogues

@pytest.mark.parametrize("dims", SMALL_DIMS)
@pytest.mark.parametrize("flavor", [1, -1, 2])
@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_dslash_all_epilogues(api, ctx, dims, flavor, prec):
    p, U, g = _setup(api, ctx, dims, flavor)
    op = oparams(p)
    nf = op.nf
    rng_in = inputs.gaussian_spinor(dims, nf, 11)
    rng_x = inputs.gaussian_spinor(dims, nf, 12)
    for out_par in (0, 1):
        inp = O.project(rng_in, dims, 1 - out_par)
        x = O.project(rng_x, dims, out_par)
        tin = to_native(api, ctx, inp, p, prec, 1 - out_par)
        tx = to_native(api, ctx, x, p, prec, out_par)
        # the oracle sees exactly the values the GPU stored (for half precision)
        inp_q = from_native(api, ctx, tin, p, prec, 1 - out_par)[0]
        x_q = from_native(api, ctx, tx, p, prec, out_par)[0]
        for dagger in (0, 1):
            for twl in (0, 1):
                for epi in range(6):
                    if twl and epi not in (0, 4, 5):
                        continue
                    out = api.new_field(p, prec)
                    api.tm_dslash(ctx, out, tin, g, prec, out_par, dagger, twl, epi,
                                  tx if epi >= 2 else None, -0.37)
                    got = from_native(api, ctx, out, p, prec, out_par)[0]
                    ref = oracle_dslash(op, U, inp_q, out_par, dagger, twl, epi, x_q, -0.37)
                    e = rel(got, ref)
                    assert e < TOL[prec], (out_par, dagger, twl, epi, e)


@pytest.mark.parametrize("recon", [12, 18])
@pytest.mark.parametrize("flavor", [1, 2])
def test_recon18_matches_recon12(api, ctx, recon, flavor):
    dims = (6, 4, 4, 6)
    p, U, g = _setup(api, ctx, dims, flavor, recon=recon, precs=(0, 1))
    op = oparams(p)
    inp = O.project(inputs.gaussian_spinor(dims, op.nf, 21), dims, 0)
    for prec in (0, 1):
        t = to_native(api, ctx, inp, p, prec, 0)
        out = api.new_field(p, prec)
        for pc in (0, 1):
            for dag in (0, 1):
                api.tm_mat_pc(ctx, out, t, g, prec, pc, dag)
                got = from_native(api, ctx, out, p, prec, 0)[0]
                ref = O.mat_pc(op, U, inp, "asym" if pc == 0 else "sym", bool(dag))
                assert rel(got, ref) < TOL[prec]


# ------------------------------------------------------------------ preconditioned operator

@pytest.mark.parametrize("dims", SMALL_DIMS[1:])
@pytest.mark.parametrize("flavor", [1, -1, 2])
@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_mat_pc_variants(api, ctx, dims, flavor, prec):
    p, U, g = _setup(api, ctx, dims, flavor)
    op = oparams(p)
    inp = O.project(inputs.gaussian_spinor(dims, op.nf, 31), dims, 0)
    t = to_native(api, ctx, inp, p, prec, 0)
    inq = from_native(api, ctx, t, p, prec, 0)[0]
    out = api.new_field(p, prec)
    for pc in (0, 1):
        for dag in (0, 1):
            api.tm_mat_pc(ctx, out, t, g, prec, pc, dag)
            got = from_native(api, ctx, out, p, prec, 0)[0]
            ref = O.mat_pc(op, U, inq, "asym" if pc == 0 else "sym", bool(dag))
            assert rel(got, ref) < TOL[prec], (pc, dag, rel(got, ref))


@pytest.mark.parametrize("flavor", [1, 2])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_twist_and_inverse(api, ctx, flavor, prec):
    dims = (6, 4, 4, 6)
    p, U, g = _setup(api, ctx, dims, flavor)
    op = oparams(p)
    a = O.project(inputs.gaussian_spinor(dims, op.nf, 41), dims, 1)
    t = to_native(api, ctx, a, p, prec, 1)
    aq = from_native(api, ctx, t, p, prec, 1)[0]
    out = api.new_field(p, prec)
    for dag in (0, 1):
        for inv in (0, 1):
            api.tm_twist(ctx, out, t, g, prec, 1, dag, inv)
            got = from_native(api, ctx, out, p, prec, 1)[0]
            ref = O.twist(op, aq, inverse=bool(inv), dagger=bool(dag), parity=1)
            assert rel(got, ref) < TOL[prec]
    # R^-1 R = 1 through the library
    if prec == 0:
        out2 = api.new_field(p, prec)
        api.tm_twist(ctx, out, t, g, prec, 1, 0, 0)
        api.tm_twist_inv(ctx, out2, out, g, prec, 1, 0)
        assert rel(from_native(api, ctx, out2, p, prec, 1)[0], aq) < 1e-14


@pytest.mark.parametrize("flavor", [1, 2])
@pytest.mark.parametrize("pc", [0, 1])
def test_prepare_and_reconstruct(api, ctx, flavor, pc):
    dims = (6, 4, 4, 6)
    p, U, g = _setup(api, ctx, dims, flavor, precs=(0,))
    op = oparams(p)
    b = inputs.gaussian_spinor(dims, op.nf, 51)
    be, bo = O.project(b, dims, 0), O.project(b, dims, 1)
    tbe, tbo = to_native(api, ctx, be, p, 0, 0), to_native(api, ctx, bo, p, 0, 1)
    bh = api.new_field(p, 0)
    api.tm_prepare(ctx, bh, tbe, tbo, g, 0, pc)
    ref = O.prepare(op, U, b, "asym" if pc == 0 else "sym")
    assert rel(from_native(api, ctx, bh, p, 0, 0)[0], ref) < 1e-12
    xe = O.project(inputs.gaussian_spinor(dims, op.nf, 52), dims, 0)
    txe = to_native(api, ctx, xe, p, 0, 0)
    xo = api.new_field(p, 0)
    api.tm_reconstruct_odd(ctx, xo, txe, tbo, g, 0)
    ref = O.reconstruct(op, U, xe, b)
    assert rel(from_native(api, ctx, xo, p, 0, 1)[0], ref) < 1e-12


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_multi_rhs_apply_equals_single(api, ctx, prec):
    """Four rhs in one launch (links loaded once per site for all) equal four
    single-rhs applies (to rounding: the two kernels may contract differently)."""
    dims = (8, 6, 4, 10)
    p, U, g = _setup(api, ctx, dims, 1)
    a = O.project(inputs.gaussian_spinor(dims, 1, 61, nrhs=4), dims, 0)
    t4 = to_native(api, ctx, a, p, prec, 0, 4)
    o4 = api.new_field(p, prec, 4)
    for pc in (0, 1):
        for dag in (0, 1):
            api.tm_mat_pc(ctx, o4, t4, g, prec, pc, dag, nrhs=4)
            got4 = from_native(api, ctx, o4, p, prec, 0, 4)
            for r in range(4):
                t1 = to_native(api, ctx, a[r], p, prec, 0, 1)
                o1 = api.new_field(p, prec, 1)
                api.tm_mat_pc(ctx, o1, t1, g, prec, pc, dag, nrhs=1)
                got1 = from_native(api, ctx, o1, p, prec, 0, 1)[0]
                assert rel(got4[r], got1) < {0: 1e-14, 1: 1e-6, 2: TOL[2], 3: TOL[3]}[prec]


def test_blas_norm_dot(api, ctx):
    dims = (8, 6, 4, 10)
    p = api.make_params(dims, 0.16, 0.1, 0.2, 2)
    a = O.project(inputs.gaussian_spinor(dims, 2, 71, nrhs=3), dims, 1)
    b = O.project(inputs.gaussian_spinor(dims, 2, 72, nrhs=3), dims, 1)
    ta, tb = to_native(api, ctx, a, p, 0, 1, 3), to_native(api, ctx, b, p, 0, 1, 3)
    n = api.tm_norm2(ctx, ta, p, 0, 3)
    d = api.tm_dot(ctx, ta, tb, p, 0, 3)
    for r in range(3):
        assert abs(n[r] - np.vdot(a[r], a[r]).real) < 1e-12 * n[r]
        assert abs(d[r] - np.vdot(a[r], b[r])) < 1e-12 * np.sqrt(n[r] * np.vdot(b[r], b[r]).real)
    # deterministic: the same bits twice
    assert np.array_equal(api.tm_norm2(ctx, ta, p, 0, 3), n)
    for prec in (1, 2, 3):
        t = api.new_field(p, prec, 3)
        api.tm_convert(ctx, t, prec, ta, 0, p, 3)
        back = api.new_field(p, 0, 3)
        api.tm_convert(ctx, back, 0, t, prec, p, 3)
        assert rel(from_native(api, ctx, back, p, 0, 1, 3), a) < {1: 1e-7, 2: 1e-3, 3: 5e-3}[prec]
    # dst = a src: in place in FP64 (exact scaling by a power of two, then a
    # general factor), and converted into every precision
    t = to_native(api, ctx, a, p, 0, 1, 3)
    api.tm_scale(ctx, t, 0, t, 0, -0.5, p, 3)
    assert np.array_equal(from_native(api, ctx, t, p, 0, 1, 3), -0.5 * a)
    api.tm_scale(ctx, t, 0, t, 0, 2.37, p, 3)
    assert rel(from_native(api, ctx, t, p, 0, 1, 3), -1.185 * a) < 1e-15
    for prec in (1, 2, 3):
        t = api.new_field(p, prec, 3)
        api.tm_scale(ctx, t, prec, ta, 0, -1.7, p, 3)
        assert rel(from_native(api, ctx, t, p, prec, 1, 3), -1.7 * a) < {1: 1e-7, 2: 1e-3, 3: 5e-3}[prec]


# ------------------------------------------------------------------ solvers

@pytest.mark.parametrize("pc", [0, 1])
def test_cg_fp64_tiny_config(api, ctx, pc):
    """4^4, Haar links, kappa = 0.160, mu = 0.01, one flavour: GPU FP64 CG to
    1e-10 plus reconstruction against the oracle's solve."""
    dims = (4, 4, 4, 4)
    p = api.make_params(dims, 0.160, 0.01, 0.0, api.PLUS)
    U = inputs.gauge_field(dims, "haar", 1001)
    g = api.Gauge(ctx, U, p, precs=(0,))
    op = oparams(p)
    b = inputs.gaussian_spinor(dims, 1, 2001)
    pcs = "asym" if pc == 0 else "sym"
    bh = O.prepare(op, U, b, pcs)
    tb = to_native(api, ctx, bh, p, 0, 0)
    tx = api.new_field(p, 0)
    res = api.tm_cg(ctx, tx, tb, g, pc=pc, tol=1e-10)[0]
    assert res["status"] == 0 and res["true_rel_res_normal"] <= 1e-10
    xe = from_native(api, ctx, tx, p, 0, 0)[0]
    check_solve(op, U, xe, bh, pcs, res["true_rel_res_normal"])
    xref, info = O.cg(op, U, bh, pcs, tol=1e-12)
    assert rel(xe, xref) < 1e-8
    # reconstruct the odd half and check the full system M psi = b
    tbo = to_native(api, ctx, O.project(b, dims, 1), p, 0, 1)
    txo = api.new_field(p, 0)
    api.tm_reconstruct_odd(ctx, txo, tx, tbo, g, 0)
    psi = xe + from_native(api, ctx, txo, p, 0, 1)[0]
    assert rel(O.full_M(op, U, psi), b) < 1e-8


@pytest.mark.parametrize("inner", [1, 2, 3])
@pytest.mark.parametrize("flavor", [1, 2])
def test_cg_mixed_reaches_fp64_residual(api, ctx, inner, flavor):
    dims = (8, 8, 8, 8)
    p = api.make_params(dims, 0.1615, 0.15 if flavor == 2 else 0.004, 0.19, flavor)
    U = inputs.gauge_field(dims, "near_unit", 1003)
    g = api.Gauge(ctx, U, p, precs=(0, inner))
    op = oparams(p)
    b = O.project(inputs.gaussian_spinor(dims, op.nf, 2003), dims, 0)
    tb = to_native(api, ctx, b, p, 0, 0)
    tx = api.new_field(p, 0)
    res = api.tm_cg(ctx, tx, tb, g, pc=0, tol=1e-10, inner=inner)[0]
    assert res["status"] == 0, res
    assert res["true_rel_res_normal"] <= 1e-10 and res["reliable_updates"] >= 1
    xe = from_native(api, ctx, tx, p, 0, 0)[0]
    check_solve(op, U, xe, b, "asym", res["true_rel_res_normal"])


def test_cg_multi_rhs_and_graph(api, ctx):
    """A 4-rhs solve equals four single solves (solutions agree to the solve
    tolerance), and k captured iterations replayed from a hipGraph give the
    eager result."""
    dims = (8, 8, 8, 8)
    p = api.make_params(dims, 0.1615, 0.004, 0.0, api.PLUS)
    U = inputs.gauge_field(dims, "near_unit", 1004)
    g = api.Gauge(ctx, U, p, precs=(0, 1))
    op = oparams(p)
    b = O.project(inputs.z2_spinor(dims, 1, 2004, nrhs=4), dims, 0)
    tb = to_native(api, ctx, b, p, 0, 0, 4)
    tx = api.new_field(p, 0, 4)
    res = api.tm_cg(ctx, tx, tb, g, tol=1e-10, nrhs=4)
    x4 = from_native(api, ctx, tx, p, 0, 0, 4)
    for r in range(4):
        assert res[r]["true_rel_res_normal"] <= 1e-10
        t1 = to_native(api, ctx, b[r], p, 0, 0)
        x1 = api.new_field(p, 0)
        api.tm_cg(ctx, x1, t1, g, tol=1e-10)
        assert rel(x4[r], from_native(api, ctx, x1, p, 0, 0)[0]) < 1e-8
        check_solve(op, U, x4[r], b[r], "asym", res[r]["true_rel_res_normal"])
    # graph replay vs eager, same iteration schedule (check every 5)
    xg = api.new_field(p, 0, 4)
    xe_ = api.new_field(p, 0, 4)
    rg = api.tm_cg(ctx, xg, tb, g, tol=1e-10, nrhs=4, graph_iters=5)
    re_ = api.tm_cg(ctx, xe_, tb, g, tol=1e-10, nrhs=4, check_every=5)
    assert rg[0]["iters"] == re_[0]["iters"]
    assert np.array_equal(from_native(api, ctx, xg, p, 0, 0, 4), from_native(api, ctx, xe_, p, 0, 0, 4))
    # and once more, after other eager work, the same bits
    api.tm_cg(ctx, xe_, tb, g, tol=1e-10, nrhs=4)
    xg2 = api.new_field(p, 0, 4)
    api.tm_cg(ctx, xg2, tb, g, tol=1e-10, nrhs=4, graph_iters=5)
    assert np.array_equal(from_native(api, ctx, xg2, p, 0, 0, 4), from_native(api, ctx, xg, p, 0, 0, 4))


@pytest.mark.parametrize("inner", [1, 2])
def test_cg_mixed_graph_device_updates(api, ctx, inner):
    """Mixed CG with captured iterations: reliable updates decided and gated on
    the device every iteration; same tolerance as the host-driven solver."""
    dims = (8, 8, 8, 8)
    p = api.make_params(dims, 0.1615, 0.15, 0.19, api.NDEG)
    U = inputs.gauge_field(dims, "near_unit", 1007)
    g = api.Gauge(ctx, U, p, precs=(0, inner))
    op = oparams(p)
    b = O.project(inputs.gaussian_spinor(dims, 2, 2007, nrhs=2), dims, 0)
    tb = to_native(api, ctx, b, p, 0, 0, 2)
    xg = api.new_field(p, 0, 2)
    rg = api.tm_cg(ctx, xg, tb, g, tol=1e-10, inner=inner, nrhs=2, graph_iters=6)
    xh = api.new_field(p, 0, 2)
    rh = api.tm_cg(ctx, xh, tb, g, tol=1e-10, inner=inner, nrhs=2)
    x = from_native(api, ctx, xg, p, 0, 0, 2)
    for r in range(2):
        assert rg[r]["status"] == 0 and rg[r]["true_rel_res_normal"] <= 1e-10
        assert rg[r]["reliable_updates"] >= 1
        check_solve(op, U, x[r], b[r], "asym", rg[r]["true_rel_res_normal"])
    # the device-decided schedule does not cost more than one graph of extra iterations
    assert rg[0]["iters"] <= rh[0]["iters"] + 6
    # two replays in a row give the same bits
    xg2 = api.new_field(p, 0, 2)
    api.tm_cg(ctx, xg2, tb, g, tol=1e-10, inner=inner, nrhs=2, graph_iters=6)
    assert np.array_equal(from_native(api, ctx, xg2, p, 0, 0, 2), x)


def test_cg_batched_uneven_lattices(api, ctx):
    """Several lattices of different size in one batched solve (each stage one
    launch over all problems) equal separate solves."""
    dims_list = [(4, 4, 4, 4), (6, 6, 6, 8), (8, 8, 8, 8)]
    gs, xs, bs, ps, Us, bnp = [], [], [], [], [], []
    for i, dims in enumerate(dims_list):
        p = api.make_params(dims, 0.1615, 0.004, 0.0, api.PLUS)
        U = inputs.gauge_field(dims, "near_unit", 1100 + i)
        g = api.Gauge(ctx, U, p, precs=(0, 1))
        b = O.project(inputs.z2_spinor(dims, 1, 2100 + i, nrhs=4), dims, 0)
        gs.append(g); ps.append(p); Us.append(U); bnp.append(b)
        bs.append(to_native(api, ctx, b, p, 0, 0, 4))
        xs.append(api.new_field(p, 0, 4))
    for inner, graph in ((0, 0), (1, 4)):
        res = api.tm_cg_batched(ctx, gs, xs, bs, [4, 4, 4], tol=1e-10, inner=inner, graph_iters=graph)
        k = 0
        for i, dims in enumerate(dims_list):
            x = from_native(api, ctx, xs[i], ps[i], 0, 0, 4)
            for r in range(4):
                assert res[k]["true_rel_res_normal"] <= 1e-10
                check_solve(oparams(ps[i]), Us[i], x[r], bnp[i][r], "asym", res[k]["true_rel_res_normal"])
                k += 1
