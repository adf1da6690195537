"""GPU: serving domain solves on host fields of several lattice sizes.

The request mix of the serving workload: Dirichlet time slabs (periodic
space) of 8^4 in an 8^3x16 field, 16^3x8 in 16^3x16, 24^3x16 in 24^3x48 and
32^3x16 in 32^3x64, each a point source at the slab centre x 12 columns,
kappa = 0.1340, c_sw = 1.769, mixed precision to 1e-10.  One context holds the
four fields (ddml_set_gauge_lattice) and one serving loop batches their
requests together.  Each result is checked against the oracle's FP64 residual
on its own host lattice, and one request gives the same bits alone and in the
mix.
"""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

ddml = pytest.importorskip("paper_1601_04587_amd.ddml")
torch = pytest.importorskip("torch")

KAPPA, CSW = 0.1340, 1.769
# (host lattice, slab [t0, t1), seed)
MIX = [((16, 8, 8, 8), (4, 12), 1601051), ((16, 16, 16, 16), (4, 12), 1601052),
       ((48, 24, 24, 24), (16, 32), 1601053), ((64, 32, 32, 32), (24, 40), 1601054)]


@pytest.fixture(scope="module")
def served():
    dev = torch.device("cuda:0")
    ctx = ddml.Context(MIX[0][0], ddml.BC_ANTIPERIODIC)
    fields, reqs = [], []
    for L, (t0, t1), seed in MIX:
        U = inputs.quenched_field(L, seed)
        gid = ctx.set_gauge_lattice(L, torch.from_numpy(U).to(dev), KAPPA, CSW)
        lo, hi = (t0, 0, 0, 0), (t1,) + tuple(L[1:])
        dom = ctx.set_domain(lo, hi)
        src = ((t0 + t1) // 2, L[1] // 2, L[2] // 2, L[3] // 2)
        b = torch.from_numpy(inputs.point_source(L, src)).to(dev)
        fields.append((L, U, lo, hi))
        reqs.append((gid, dom, b))
    yield ctx, dev, fields, reqs
    ctx.close()


def test_mixed_lattice_serving_matches_oracle_and_alone(served):
    ctx, dev, fields, reqs = served
    outs = [torch.zeros_like(b) for (_, _, b) in reqs]
    torch.cuda.synchronize()
    ctx.server_start(ddml.solver_params(tol=1e-10))
    try:
        # the 24^3x16 request alone
        gid, dom, b = reqs[2]
        alone = torch.zeros_like(b)
        r = ctx.wait(ctx.submit(gid, dom, b, alone, 12), 300.0)
        assert r is not None and r.status == ddml.OK
        # the whole mix, twice over, arriving together
        tickets = []
        outs2 = [torch.zeros_like(b) for (_, _, b) in reqs]   # kept alive until the results are in
        for rep in range(2):
            for k, (gid, dom, b) in enumerate(reqs):
                tickets.append((k, ctx.submit(gid, dom, b, outs[k] if rep == 0 else outs2[k], 12)))
        res = [(k, ctx.wait(t, 300.0)) for k, t in tickets]
        assert all(r is not None and r.status == ddml.OK for _, r in res)
        st = ctx.stats()
        assert st.completed == 1 + 2 * len(reqs) and st.p99_latency >= st.p50_latency > 0
    finally:
        ctx.server_stop()
    torch.cuda.synchronize()
    assert torch.equal(alone, outs[2]) and torch.equal(outs2[2], outs[2])
    for (L, U, lo, hi), (gid, dom, b), x in zip(fields, reqs, outs):
        C = oracle.clover_term(U, L, CSW)
        res = oracle.residual(U, L, KAPPA, b.cpu().numpy(), x.cpu().numpy(), C=C, lo=lo, hi=hi)
        assert res.max() <= 1e-10 * (1 + 1e-3), (L, res.max())
        m = oracle.domain_mask(L, lo, hi)
        assert x.cpu().numpy()[:, ~m].size == 0 or np.abs(x.cpu().numpy()[:, ~m]).max() == 0.0


def test_domain_outside_a_smaller_lattice_is_rejected(served):
    ctx, dev, fields, reqs = served
    gid_small = reqs[0][0]
    big_dom = reqs[3][1]      # a 32^3x16 slab does not fit the 8^3x16 field
    b = torch.zeros((12,) + (int(np.prod(fields[0][0])), 4, 3), dtype=torch.complex128, device=dev)
    x = torch.zeros_like(b)
    with pytest.raises(ddml.DDMLError) as e:
        ctx.solve_domain(gid_small, big_dom, b, x, 12)
    assert e.value.code == ddml.EINVAL
