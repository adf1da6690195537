"""GPU: one step of the benchmark's batched multi-level workload at its full
size, in the launch configuration the benchmark times, against the oracle on
sampled outputs.

32^3x64, quenched beta = 6.0 field, kappa = 0.1340, c_sw = 1.769,
antiperiodic time; the stencil launch picked by the autotuner; each of the 4
slabs of 16 slices updated by one level-1 sweep on the device; the nested
domains Gamma0/1/2 = 4/8/16 slices around the source (slab start + 7) solved
for 12 point-source columns to 1e-10, submitted as the benchmark does: one
series request per slab to the library's request loop.  Checked:
* the slab links of one update against the oracle's level-1 sweep;
* for two slabs, every level's residual on the updated field at 4096 random
  sites of its domain and at the source (|r(x)| <= 1e-10 ||b|| per column
  must hold at every site);
* the telescoping sum of the terms equals the returned total to rounding;
* the nucleon contraction on three sampled sink slices and the disconnected
  pieces of a slab pair against the oracle's, from the GPU terms (1e-11);
* the series of two slabs through the request loop equal the same series
  solved by ddml_propagator_series_batch, bit for bit.
"""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

ddml = pytest.importorskip("paper_1601_04587_amd.ddml")
torch = pytest.importorskip("torch")

L = (64, 32, 32, 32)
KAPPA, CSW, BETA, SEED = 0.1340, 1.769, 6.0, 1601004
TOL = 1e-10


def test_one_headline_step_on_sampled_sites():
    V = int(np.prod(L))
    V3 = V // L[0]
    nslab = L[0] // 16
    dev = torch.device("cuda:0")
    U0 = inputs.quenched_field(L, SEED)
    ctx = ddml.Context(L, ddml.BC_ANTIPERIODIC, device=0)
    try:
        gid0 = ctx.set_gauge(torch.from_numpy(U0).to(dev), KAPPA, CSW)
        doms, xs, srcs, terms = [], [], [], []
        for s in range(nslab):
            a = 16 * s
            doms.append([ctx.set_domain((a + 6, 0, 0, 0), (a + 10,) + L[1:]),
                         ctx.set_domain((a + 4, 0, 0, 0), (a + 12,) + L[1:]),
                         ctx.set_domain((a, 0, 0, 0), (a + 16,) + L[1:])])
            xs.append((a + 7, 0, 0, 0))
            srcs.append(torch.from_numpy(inputs.point_source(L, xs[-1])).to(dev))
            terms.append(torch.zeros((3, 12, V, 4, 3), dtype=torch.complex128, device=dev))
        ctx.autotune(gid0, doms[0][2], 12, ddml.MIXED_FP32)
        gids = [ctx.level1_update(gid0, 16 * s, 16 * s + 16, BETA, SEED, 3 + 1000 + s, 1, 0) for s in range(nslab)]
        totals = [torch.zeros((12, V, 4, 3), dtype=torch.complex128, device=dev) for _ in range(nslab)]
        torch.cuda.synchronize()
        prm = ddml.solver_params(tol=TOL, solver=1)   # the benchmark's solver
        arrays = [(ddml.RhsInfo * 36)() for _ in range(nslab)]
        ctx.server_start(prm)
        try:
            tickets = [ctx.submit_series(gids[s], doms[s], srcs[s], terms[s], 12, sum=totals[s], info=arrays[s])
                       for s in range(nslab)]
            res = [ctx.wait(t, 600.0) for t in tickets]
        finally:
            ctx.server_stop()
        torch.cuda.synchronize()
        assert all(r is not None and r.status == ddml.OK for r in res), ctx.last_error()
        infos = [[list(a[12 * lev:12 * (lev + 1)]) for lev in range(3)] for a in arrays]
        nuc = [ctx.contract_nucleon(terms[s], 3) for s in (0, 2)]
        pp = ctx.contract_pp_disconnected(terms[0], terms[2], 3, xs[0], xs[2])
        Ug = np.zeros((V, 4, 3, 3), complex)
        ctx.get_gauge(gids[1], Ug)
        # the device update of slab 1 against the oracle's sweep
        ref_u = oracle.level1_update(U0, L, BETA, SEED, 1000 + 1, 16, 32, 1, 0)
        assert np.abs(Ug - ref_u).max() < 1e-11
        del ref_u
        rng = np.random.default_rng(1601901)
        e = np.zeros((12, 4, 3))
        for k in range(12):
            e[k, k // 3, k % 3] = 1.0
        for s in (0, 2):
            ctx.get_gauge(gids[s], Ug)
            cum = torch.cumsum(terms[s], dim=0)
            assert (cum[-1] - totals[s]).abs().max().item() <= 1e-15 * totals[s].abs().max().item()
            sx = inputs.site_index(L, xs[s])
            for lev, (t0, t1) in enumerate([(16 * s + 6, 16 * s + 10), (16 * s + 4, 16 * s + 12),
                                            (16 * s, 16 * s + 16)]):
                psi = cum[lev].cpu().numpy()
                sites = np.unique(np.concatenate([rng.integers(t0 * V3, t1 * V3, 4096), [sx]]))
                r = oracle.apply_D_sites(Ug, L, KAPPA, psi, sites, csw=CSW, antiperiodic=True,
                                         lo=(t0, 0, 0, 0), hi=(t1,) + L[1:])
                r[:, sites == sx] -= e[:, None]
                assert np.abs(r).max() <= TOL * (1 + 1e-3), (s, lev, np.abs(r).max())
                assert all(i.status == ddml.OK for i in infos[s][lev])
                # nucleon on sampled sink slices from the same cumulative propagator
                lv, _ = nuc[0 if s == 0 else 1]
                for t in (t0, 16 * s + 7, t1 - 1):
                    ref = oracle.nucleon(psi[:, t * V3:(t + 1) * V3], (1,) + L[1:])[0]
                    assert abs(lv[lev, t] - ref) <= 1e-11 * abs(ref), (s, lev, t)
                del psi
        # the same two series through the batch call
        again = [torch.zeros_like(terms[0]) for _ in range(2)]
        rc, _ = ctx.propagator_series_batch([(gids[s], doms[s], srcs[s], again[k], None)
                                             for k, s in enumerate((0, 2))], 12, prm)
        torch.cuda.synchronize()
        assert rc == ddml.OK
        assert torch.equal(again[0], terms[0]) and torch.equal(again[1], terms[2])
        del again
        # disconnected pieces from the terms at the two source points
        tx = terms[0][:, :, inputs.site_index(L, xs[0])].cpu().numpy()[:, :, None]
        ty = terms[2][:, :, inputs.site_index(L, xs[2])].cpu().numpy()[:, :, None]
        ref = oracle.contract_pp_disconnected(tx, ty, 0, 0, V3)
        assert np.abs(pp - ref).max() <= 1e-11 * np.abs(ref).max()
        print("headline step: inner iterations", [[max(i.inner_iters for i in lev) for lev in per] for per in infos])
    finally:
        ctx.close()
