"""GPU: serving loop, batched series, autotuner and the stencil timing hook.

The serving determinism test is the one the continuous-batching design is
held to: a request gives bitwise the same solution alone and in a mix with
other requests that overlap it on the device (per-solve reductions run in a
fixed order and a solve's iterations do not depend on its neighbours in the
batch).
"""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

ddml = pytest.importorskip("paper_1601_04587_amd.ddml")
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    L = (16, 8, 8, 8)
    U = inputs.quenched_field(L, 1601002)
    ctx = ddml.Context(L, ddml.BC_ANTIPERIODIC)
    gid = ctx.set_gauge(U, 0.1340, 1.769)
    doms = {"G0": ((6, 0, 0, 0), (10, 8, 8, 8)), "G1": ((4, 0, 0, 0), (12, 8, 8, 8)), "G2": ((0, 0, 0, 0), L)}
    ids = {k: ctx.set_domain(*v) for k, v in doms.items()}
    yield L, U, ctx, gid, doms, ids
    ctx.close()


def test_serving_alone_equals_mixed_bitwise(setup):
    L, U, ctx, gid, doms, ids = setup
    dev = torch.device("cuda:0")
    V = int(np.prod(L))
    srcs = [torch.from_numpy(inputs.point_source(L, (7, k, 0, 1))).to(dev) for k in range(4)]
    outs = [torch.zeros((12, V, 4, 3), dtype=torch.complex128, device=dev) for _ in range(4)]
    torch.cuda.synchronize()
    ctx.server_start(ddml.solver_params(tol=1e-10))
    try:
        t = ctx.submit(gid, ids["G1"], srcs[0], outs[0], 12)
        r = ctx.wait(t, 120.0)
        assert r is not None and r.status == ddml.OK
        alone = outs[0].clone()
        outs[0].zero_()
        torch.cuda.synchronize()
        # the same request in a mix: others arrive before and after it
        tk = [ctx.submit(gid, ids["G2"], srcs[1], outs[1], 12),
              ctx.submit(gid, ids["G1"], srcs[0], outs[0], 12),
              ctx.submit(gid, ids["G0"], srcs[2], outs[2], 12),
              ctx.submit(gid, ids["G2"], srcs[3], outs[3], 12)]
        res = [ctx.wait(x, 120.0) for x in tk]
        assert all(r is not None and r.status == ddml.OK for r in res)
        st = ctx.stats()
        assert st.completed == 5 and st.p99_latency >= st.p50_latency > 0
    finally:
        ctx.server_stop()
    torch.cuda.synchronize()
    assert torch.equal(alone, outs[0])
    # and the mixed results are right: oracle residual on the full-lattice request
    C = oracle.clover_term(U, L, 1.769)
    b = srcs[3].cpu().numpy()
    res = oracle.residual(U, L, 0.1340, b, outs[3].cpu().numpy(), C=C)
    assert res.max() <= 1e-10 * (1 + 1e-3)


def test_submit_rejects_host_and_short_buffers(setup):
    """Host memory is refused by the binding and by ddml_submit itself before
    anything is queued; a device buffer too small for nrhs canonical fields
    finishes with EINVAL at admission, before any kernel reads it."""
    import ctypes
    L, U, ctx, gid, doms, ids = setup
    dev = torch.device("cuda:0")
    V = int(np.prod(L))
    src = torch.from_numpy(inputs.point_source(L, (7, 0, 0, 0))).to(dev)
    out = torch.zeros((12, V, 4, 3), dtype=torch.complex128, device=dev)
    host = np.zeros((12, V, 4, 3), dtype=np.complex128)
    torch.cuda.synchronize()
    ctx.server_start(ddml.solver_params(tol=1e-10))
    try:
        with pytest.raises(ValueError):
            ctx.submit(gid, ids["G0"], src, host, 12)
        with pytest.raises(ValueError):
            ctx.submit(gid, ids["G0"], src.cpu(), out, 12)
        # the C entry point on its own (no binding check in front of it)
        ticket = ctypes.c_uint64()
        for ps, pd in ((host.ctypes.data, out.data_ptr()), (src.data_ptr(), host.ctypes.data)):
            req = ddml.Request(gid, ids["G0"], ps, pd, 12, ddml.now())
            assert ctx.lib.ddml_submit(ctx.h, ctypes.byref(req), ctypes.byref(ticket)) == ddml.EINVAL
        # one element in a small-block segment cannot hold 12 fields of 16 x 8^3 sites
        tiny = torch.zeros(1, dtype=torch.complex128, device=dev)
        torch.cuda.synchronize()
        r = ctx.wait(ctx.submit(gid, ids["G0"], src, tiny, 12), 60.0)
        assert r is not None and r.status == ddml.EINVAL
        assert tiny.item() == 0
        # the loop keeps serving good requests
        r = ctx.wait(ctx.submit(gid, ids["G0"], src, out, 12), 120.0)
        assert r is not None and r.status == ddml.OK
    finally:
        ctx.server_stop()


def test_series_batch_matches_single_series(setup):
    L, U, ctx, gid, doms, ids = setup
    V = int(np.prod(L))
    order = [ids["G0"], ids["G1"], ids["G2"]]
    b1 = inputs.point_source(L, (7, 0, 0, 0))
    b2 = inputs.point_source(L, (8, 1, 2, 3))
    t1 = np.zeros((3, 12, V, 4, 3), dtype=np.complex128)
    t2 = np.zeros_like(t1)
    rc, infos = ctx.propagator_series_batch([(gid, order, b1, t1, None), (gid, order, b2, t2, None)], 12)
    assert rc == ddml.OK
    s1 = np.zeros_like(t1)
    rc, _ = ctx.propagator_series(gid, order, b1, 12, s1)
    assert rc == ddml.OK
    assert np.array_equal(s1, t1)
    C = oracle.clover_term(U, L, 1.769)
    cum = np.cumsum(t2, axis=0)
    for i, k in enumerate(["G0", "G1", "G2"]):
        lo, hi = doms[k]
        assert oracle.residual(U, L, 0.1340, b2, cum[i], C=C, lo=lo, hi=hi).max() <= 1e-10 * (1 + 1e-3)


def test_series_requests_match_series_call_bitwise(setup):
    """Propagator series submitted to the request loop (one solve per nested
    domain, differences on completion) give the bits of ddml_propagator_series,
    also when several series and single solves overlap on the device; a series
    naming an unknown domain finishes with EINVAL and leaves its buffers alone."""
    L, U, ctx, gid, doms, ids = setup
    dev = torch.device("cuda:0")
    V = int(np.prod(L))
    order = [ids["G0"], ids["G1"], ids["G2"]]
    b = [inputs.point_source(L, (7, k, 1, 0)) for k in range(3)]
    ref = []
    for k in range(3):
        t = np.zeros((3, 12, V, 4, 3), dtype=np.complex128)
        sm = np.zeros((12, V, 4, 3), dtype=np.complex128)
        rc, _ = ctx.propagator_series(gid, order, b[k], 12, t, sm)
        assert rc == ddml.OK
        ref.append((t, sm))
    srcs = [torch.from_numpy(x).to(dev) for x in b]
    terms = [torch.zeros((3, 12, V, 4, 3), dtype=torch.complex128, device=dev) for _ in range(3)]
    sums = [torch.zeros((12, V, 4, 3), dtype=torch.complex128, device=dev) for _ in range(3)]
    single = torch.zeros((12, V, 4, 3), dtype=torch.complex128, device=dev)
    bad = torch.full((3, 12, V, 4, 3), 7.0, dtype=torch.complex128, device=dev)
    infos = [(ddml.RhsInfo * 36)() for _ in range(3)]
    torch.cuda.synchronize()
    ctx.server_start(ddml.solver_params(tol=1e-10))
    try:
        tk = [ctx.submit_series(gid, order, srcs[0], terms[0], 12, sum=sums[0], info=infos[0]),
              ctx.submit(gid, ids["G2"], srcs[2], single, 12),
              ctx.submit_series(gid, order, srcs[1], terms[1], 12, sum=sums[1], info=infos[1]),
              ctx.submit_series(gid, [ids["G0"], 999], srcs[1], bad, 12),
              ctx.submit_series(gid, order, srcs[2], terms[2], 12, sum=sums[2], info=infos[2])]
        # the solver graphs hold the loop's slots: no relaunch while it runs
        with pytest.raises(ddml.DDMLError):
            ctx.set_launch(ddml.MIXED_FP32, 1, 0, 1024, 1, 1)
        with pytest.raises(ddml.DDMLError):
            ctx.autotune(gid, ids["G0"], 12)
        res = [ctx.wait(x, 300.0) for x in tk]
    finally:
        ctx.server_stop()
    torch.cuda.synchronize()
    assert [r is not None for r in res] == [True] * 5
    assert [r.status for r in res] == [ddml.OK, ddml.OK, ddml.OK, ddml.EINVAL, ddml.OK]
    for k, j in ((0, 0), (1, 2), (2, 4)):
        assert np.array_equal(terms[k].cpu().numpy(), ref[k][0]), k
        assert np.array_equal(sums[k].cpu().numpy(), ref[k][1]), k
        assert res[j].max_outer == max(i.outer_iters for i in infos[k]) >= 1
        assert res[j].worst_rel_residual == max(i.true_rel_residual for i in infos[k]) <= 1e-10
    assert bool(torch.all(bad == 7.0))


@pytest.mark.parametrize("solver", [0, 1])
def test_mixed_solver_iterations_close_to_fp64(setup, solver):
    """Mixed precision (restarted or with reliable updates) converges in about
    as many BiCGstab iterations as the FP64 solver, to the FP64 residual."""
    L, U, ctx, gid, doms, ids = setup
    b = inputs.point_source(L, (7, 0, 0, 0))
    x = np.zeros_like(b)
    rc, info32 = ctx.solve_domain(gid, ids["G2"], b, x, 12, ddml.solver_params(tol=1e-10, solver=solver))
    assert rc == ddml.OK
    C = oracle.clover_term(U, L, 1.769)
    assert oracle.residual(U, L, 0.1340, b, x, C=C).max() <= 1e-10 * (1 + 1e-3)
    rc, info64 = ctx.solve_domain(gid, ids["G2"], b, x, 12, ddml.solver_params(tol=1e-10, prec=ddml.FP64))
    assert rc == ddml.OK
    it32 = max(i.inner_iters for i in info32)
    it64 = max(i.inner_iters for i in info64)
    # restarted: within 25% of FP64; with reliable updates the Krylov space built
    # against the FP32 recursive residual is kept across each FP64 replacement,
    # which costs more iterations on small volumes (measured 1.2-1.35x here)
    factor = 1.25 if solver == 0 else 1.5
    assert it32 <= factor * it64 + 5, (it32, it64)
    assert max(i.outer_iters for i in info32) >= 2


def test_autotune_and_stencil_timing(setup):
    L, U, ctx, gid, doms, ids = setup
    R, order, grid, splits, stage, ms = ctx.autotune(gid, ids["G2"], 12, ddml.MIXED_FP32)
    assert 1 <= R <= 3 and order in (0, 1, 2, 3, 4, 5) and grid in (512, 1024, 2048) and 1 <= splits <= 3 and ms > 0
    assert stage in (0, 1)
    ms_odd, ms_even, b_odd, b_even = ctx.time_stencil(gid, ids["G2"], 12, ddml.MIXED_FP32, 5)
    Vh = int(np.prod(L)) // 2
    # two-row links in FP32: 8 links x 12 reals + 72 of A^-1 per output site
    assert b_odd == Vh * (48 * 12 + 96 + 72) * 4 and b_even == Vh * (72 * 12 + 96 + 72) * 4
    assert ms_odd > 0 and ms_even > 0
    # a solve after retuning still matches the oracle
    lo, hi = doms["G0"]
    b = inputs.point_source(L, (7, 0, 0, 0))
    x = np.zeros_like(b)
    rc, _ = ctx.solve_domain(gid, ids["G0"], b, x, 12)
    assert rc == ddml.OK
    C = oracle.clover_term(U, L, 1.769)
    assert oracle.residual(U, L, 0.1340, b, x, C=C, lo=lo, hi=hi).max() <= 1e-10 * (1 + 1e-3)


def test_fp16_storage_solve_and_iterations(setup):
    """16-bit storage of the inner solver: FP64 defect correction still reaches
    1e-10, at a bounded cost in BiCGstab iterations over FP32 storage."""
    L, U, ctx, gid, doms, ids = setup
    b = inputs.point_source(L, (7, 0, 0, 0))
    C = oracle.clover_term(U, L, 1.769)
    x16 = np.zeros_like(b)
    rc, info16 = ctx.solve_domain(gid, ids["G2"], b, x16, 12, ddml.solver_params(tol=1e-10, prec=ddml.MIXED_FP16))
    assert rc == ddml.OK
    assert oracle.residual(U, L, 0.1340, b, x16, C=C).max() <= 1e-10 * (1 + 1e-3)
    x32 = np.zeros_like(b)
    rc, info32 = ctx.solve_domain(gid, ids["G2"], b, x32, 12, ddml.solver_params(tol=1e-10))
    assert rc == ddml.OK
    it16 = max(i.inner_iters for i in info16)
    it32 = max(i.inner_iters for i in info32)
    assert it16 <= 2 * it32 + 10, (it16, it32)
    # 16-bit runs take at least as many FP64 corrections (each inner solve stops at 3e-4)
    assert max(i.outer_iters for i in info16) >= max(i.outer_iters for i in info32)


def test_every_launch_variant_computes_the_same_bits():
    """The stencil launch (columns per thread, tile order, grid, column splits,
    LDS staging, which FP32 and 16-bit need for their two-row links) changes only the schedule: every site and column is computed
    and reduced the same way, so solves agree bit for bit.  A 16^4 box gives
    planar tile walks (sub-banded orders); a 6^4 box has time slices that are
    not whole tiles (banded fallback walks, a padded last tile)."""
    L = (16, 16, 16, 16)
    U = inputs.random_links(L, 1601077, 0.3)
    ctx = ddml.Context(L, ddml.BC_ANTIPERIODIC)
    try:
        gid = ctx.set_gauge(U, 0.1200, 1.0)
        dom = ctx.set_domain((4, 0, 0, 0), (10, 16, 16, 16))
        b = inputs.point_source(L, (6, 3, 5, 7))
        # a box whose time slice (6^3 sites) is not a whole number of 64-site tiles
        dom2 = ctx.set_domain((2, 2, 2, 2), (8, 8, 8, 8))
        b2 = inputs.point_source(L, (4, 4, 4, 4))
        variants = {
            ddml.MIXED_FP32: [(1, 1, 1024, 1, 1), (1, 3, 512, 1, 1), (1, 2, 1024, 2, 1), (2, 0, 512, 2, 1),
                              (3, 1, 2048, 1, 1), (1, 0, 1024, 3, 1), (1, 4, 1024, 1, 1)],
            ddml.FP64: [(1, 1, 1024, 1, 0), (1, 3, 1024, 1, 1), (3, 2, 512, 2, 1)],
            ddml.MIXED_FP16: [(1, 1, 1024, 1, 1), (1, 3, 512, 2, 1), (2, 2, 1024, 1, 1), (1, 4, 2048, 1, 1)],
        }
        for prec, vs in variants.items():
            ref = None
            for v in vs:
                ctx.set_launch(prec, *v)
                xs = []
                for d, src in ((dom, b), (dom2, b2)):
                    x = np.zeros_like(src)
                    rc, info = ctx.solve_domain(gid, d, src, x, 12, ddml.solver_params(tol=1e-10, prec=prec))
                    assert rc == ddml.OK, (prec, v)
                    xs.append(x)
                if ref is None:
                    ref = xs
                else:
                    assert all(np.array_equal(x, r) for x, r in zip(xs, ref)), (prec, v)
        with pytest.raises(ddml.DDMLError):
            ctx.set_launch(ddml.MIXED_FP16, 1, 1, 1024, 1, 0)      # 16-bit needs the LDS staging
        with pytest.raises(ddml.DDMLError):
            ctx.set_launch(ddml.MIXED_FP32, 1, 1, 1024, 1, 0)      # so does FP32 (two-row links)
        with pytest.raises(ddml.DDMLError):
            ctx.set_launch(ddml.MIXED_FP32, 1, 1, 1024, 1, 2)      # no such stage
    finally:
        ctx.close()


def test_quadrant_walk_computes_the_same_bits():
    """Tile order 5 (each XCD owns half of the x1 rows and a quarter of the
    tiles of a plane, 4 sub-bands along x1) needs a box whose x1 extent splits
    into 2 x 4 rows and whose (x2, x3) planes hold a multiple of 4 tiles: on
    8^3 x 32 boxes of an 8 x 8 x 16 x 32 lattice (a 4-slice slab and the
    whole antiperiodic lattice) it walks its own table, and solves agree bit
    for bit with the banded order in all three precisions, alone and as two
    series in one batch (slots of both boxes in every launch)."""
    L = (8, 8, 16, 32)
    U = inputs.random_links(L, 1601078, 0.3)
    ctx = ddml.Context(L, ddml.BC_ANTIPERIODIC)
    try:
        gid = ctx.set_gauge(U, 0.1200, 1.0)
        doms = [(ctx.set_domain((2, 0, 0, 0), (6,) + L[1:]), inputs.point_source(L, (3, 1, 5, 7))),
                (ctx.set_domain((0, 0, 0, 0), L), inputs.point_source(L, (7, 6, 2, 30)))]
        variants = {
            ddml.MIXED_FP32: [(1, 1, 1024, 1, 1), (1, 5, 512, 1, 1), (1, 5, 1024, 1, 1), (2, 5, 512, 2, 1)],
            ddml.FP64: [(1, 1, 1024, 1, 0), (1, 5, 1024, 1, 1), (1, 5, 512, 1, 0)],
            ddml.MIXED_FP16: [(1, 1, 1024, 1, 1), (1, 5, 2048, 1, 1)],
        }
        for prec, vs in variants.items():
            ref = None
            for v in vs:
                ctx.set_launch(prec, *v)
                xs = []
                for d, src in doms:
                    x = np.zeros_like(src)
                    rc, info = ctx.solve_domain(gid, d, src, x, 12, ddml.solver_params(tol=1e-10, prec=prec))
                    assert rc == ddml.OK, (prec, v)
                    xs.append(x)
                if ref is None:
                    ref = xs
                else:
                    assert all(np.array_equal(x, r) for x, r in zip(xs, ref)), (prec, v)
        # two series in one batch: slots of both boxes share every launch
        ids = [d for d, _ in doms]
        srcs = [doms[0][1], inputs.point_source(L, (4, 6, 2, 30))]   # both inside the inner level
        for prec, vs in ((ddml.MIXED_FP32, [(1, 1, 1024, 1, 1), (1, 4, 1024, 1, 1), (1, 5, 512, 1, 1)]),
                         (ddml.MIXED_FP16, [(1, 1, 1024, 1, 1), (1, 5, 1024, 1, 1)])):
            ref = None
            for v in vs:
                ctx.set_launch(prec, *v)
                terms = [np.zeros((2,) + b.shape, complex) for b in srcs]
                rc, _ = ctx.propagator_series_batch([(gid, ids, b, t, None) for b, t in zip(srcs, terms)], 12,
                                                    ddml.solver_params(tol=1e-10, prec=prec, solver=1))
                assert rc == ddml.OK, (prec, v)
                if ref is None:
                    ref = terms
                else:
                    assert all(np.array_equal(t, r) for t, r in zip(terms, ref)), (prec, v)
    finally:
        ctx.close()
