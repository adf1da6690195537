#!/usr/bin/env python3
"""Benchmark of the batched multi-level domain-solve path on one MI355X.

Workload (one "step" = one level-1 update round of the two-level scheme):
  32^3 x 64 lattice, quenched beta = 6.0 field, kappa = 0.1340, c_sw = 1.769,
  antiperiodic time; 4 time slabs of 16 slices, each updated independently by
  one heatbath sweep with its first-slice spatial links frozen (Section 3.1),
  on the device, each slab's chain starting from its previous update;
  for every slab update: the new gauge version's clover term is
  built, then the nested Dirichlet domains Gamma0 (4 slices), Gamma1 (8) and
  Gamma2 (the 16-slice slab) are solved for 12 point-source columns to a
  relative residual of 1e-10 (FP32 inner BiCGstab with reliable updates,
  FP64 defect correction on the device); the telescoping series and the nucleon and disconnected
  pseudoscalar contractions follow.  The default 16 steps are the n1 = 16
  updates of every slab, run as one continuous queue: each update's series
  (three solves) enters the library's request loop as soon as its gauge
  version exists, so the next round's solves join the slot table while the
  previous round's largest domains still run; a round is contracted when its
  output buffers are needed again (two rounds in flight).
Reported: domain solves/s (a solve = one domain x 12 columns to 1e-10), the
stencil roofline (HIP events inside the library), the plain FP64 solver one
solve at a time, serving latency percentiles, and the FP64 CPU oracle on a
bounded sample.  Inputs are resident on the GPU before timing starts.
A second workload (Section 5.2): the two-domain factorized propagator and
connected pion series on the same field with open time boundaries, x0cut = 24,
Delta = 8, 12, 16, source on t = 4 (eqs. approxlong, W0pc, seriespi), plus the
whole-lattice solve for the rest; reported beside the headline figure.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12  # MI355X HBM3E, bytes/s
# reals per domain site of the links of both stencil halves and the clover
# inverse in one M-hat application: 4 links per site and half, stored as their
# first two rows (12 reals; the stencil rebuilds the third), 72 for A^-1
LINK_REALS = 168


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def counter_traffic(mode_key):
    """HBM bytes per launch of a stencil kernel from the committed rocprofv3
    counter summary, or None if the kernel source changed since it was taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "stencil_k_hop_batch_fp32_32x32x32x16_12rhs.md")
    src = os.path.join(ROOT, "paper_1601_04587_amd", "csrc", "dirac.hip")
    if not (os.path.exists(prof) and os.path.exists(src)):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    vals = {}
    for line in open(prof):
        if line.startswith("machine-readable: "):
            k, v = line[len("machine-readable: "):].strip().rsplit("=", 1)
            vals[k] = v
    if vals.get("dirac_hip_sha256") != sha:
        return None
    v = vals.get("traffic_bytes[%s]" % mode_key)
    return float(v) if v else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16, help="level-1 update rounds (16 = n1 updates of every slab)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dims", default="64,32,32,32", help="T,L1,L2,L3 (T a multiple of 16)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-fp16", action="store_true", help="skip the 16-bit storage leg")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-factorized", action="store_true", help="skip the factorized pion leg")
    ap.add_argument("--no-hpe", action="store_true", help="skip the stochastic trace leg")
    ap.add_argument("--no-projected", action="store_true", help="skip the projector-cut pion leg")
    ap.add_argument("--proj-vectors", type=int, default=24, help="basis vectors of the projector-cut leg")
    ap.add_argument("--proj-iters", type=int, default=4, help="inverse iterations of the projector-cut leg")
    ap.add_argument("--hpe-sources", type=int, default=24, help="Gaussian sources per domain (stochastic traces)")
    ap.add_argument("--factorized-only", action="store_true",
                    help="only the factorized pion leg (profiling runs)")
    ap.add_argument("--projected-only", action="store_true",
                    help="only the projector-cut pion and nucleon leg (profiling runs)")
    ap.add_argument("--serve-requests", type=int, default=256,
                    help="requests per serving stream (at least a few hundred, so that p99 is not the maximum)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="configured Poisson rate, req/s")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--stencil-iters", type=int, default=20)
    ap.add_argument("--sweep-iters", type=int, default=2, help="timed pairs per launch variant (--stencil-only)")
    ap.add_argument("--decorrelate", type=int, default=50,
                    help="full-volume sweeps (1 heatbath + 4 over-relaxation) of the base field after replicating "
                         "a thermalised 16x8^3 field")
    ap.add_argument("--stencil-only", action="store_true",
                    help="only time the stencil kernels on the 32^3x16 slab domain (profiling runs); "
                         "also runs one plain 1 GiB device copy as the reference for HBM counters")
    ap.add_argument("--stencil-prec", choices=("fp32", "fp16"), default="fp32",
                    help="storage of the --stencil-only kernels: FP32 or 16-bit fixed point")
    ap.add_argument("--stencil-launch", default=None,
                    help="R,order,grid,splits,stage: time this launch only (--stencil-only, no sweep)")
    return ap.parse_args()


def launch_variants(nrhs=12):
    """Every stencil launch the autotuner considers, in its order:
    (R, tile_order, grid, splits, stage)."""
    out = []
    for stage in (1,):   # FP32 fields are read through the LDS staging (two-row links)
        for R in (1, 2, 3):
            for splits in (1, 2, 3):
                if splits > (nrhs + R - 1) // R:
                    continue
                for order in (0, 1, 2, 3, 4, 5):
                    for grid in (512, 1024, 2048):
                        out.append((R, order, grid, splits, stage))
    return out


def stencil_only(args):
    """Stencil kernels alone on the Gamma2 slab domain, for rocprofv3 runs: every
    launch variant (3 untimed + `--sweep-iters` timed pairs each, in the order
    printed), then the fastest one for `--stencil-iters` pairs; with
    `--stencil-launch` only that launch (3 untimed + `--stencil-iters` pairs)."""
    import torch

    import inputs
    from paper_1601_04587_amd import ddml

    L = tuple(int(v) for v in args.dims.split(","))
    U = inputs.random_links(L, 1601004, 0.3)   # bandwidth does not depend on the link values
    ctx = ddml.Context(L, ddml.BC_ANTIPERIODIC, device=0)
    gid = ctx.set_gauge(U, 0.1340, 1.769)
    dom = ctx.set_domain((0, 0, 0, 0), (16,) + L[1:])
    prec, name = (ddml.MIXED_FP32, "fp32") if args.stencil_prec == "fp32" else (ddml.MIXED_FP16, "fp16")
    sweep = []
    if args.stencil_launch:
        tune = tuple(int(v) for v in args.stencil_launch.split(","))
        if len(tune) != 5:
            raise SystemExit("--stencil-launch takes R,order,grid,splits,stage")
    else:
        for v in launch_variants():
            o = ctx.time_stencil(gid, dom, 12, prec, args.sweep_iters, *v)
            sweep.append(list(v) + [o[0], o[1]])
        best = min(sweep, key=lambda r: r[5] + r[6])
        tune = tuple(best[:5])
        log("fastest %s launch: R=%d order=%d grid=%d splits=%d stage=%d" % ((name,) + tune))
    s32 = ctx.time_stencil(gid, dom, 12, prec, args.stencil_iters, *tune)
    log("stencil-only %s: odd %.4f ms (%.3e B), even %.4f ms (%.3e B) -> even %.0f GB/s, odd %.0f GB/s"
        % (name, s32[0], s32[2], s32[1], s32[3], s32[3] / s32[1] * 1e-6, s32[2] / s32[0] * 1e-6))
    # plain copy of known size: the reference reading of the HBM byte counters
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0")   # 1 GiB
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps({"stencil_" + name: {"ms_odd": s32[0], "ms_even": s32[1], "bytes_odd": s32[2],
                                       "bytes_even": s32[3], "R": tune[0], "tile_order": tune[1], "grid": tune[2],
                                       "splits": tune[3], "stage": tune[4]},
                      "sweep_iters": args.sweep_iters, "stencil_iters": args.stencil_iters,
                      "sweep": sweep, "copy_bytes_each_way": 1 << 30}), flush=True)
    return 0


def main():
    args = parse()
    if args.stencil_only:
        return stencil_only(args)
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs every domain solve on a single "
              "MI355X (no collectives); --gpus %d is not supported." % args.gpus, file=sys.stderr)
        return 2
    import torch

    import inputs
    from paper_1601_04587_amd import ddml

    assert torch.cuda.is_available(), "needs a GPU"
    dev = torch.device("cuda:0")
    L = tuple(int(v) for v in args.dims.split(","))
    T = L[0]
    nslab = T // 16
    V = int(np.prod(L))
    V3 = V // T
    kappa, csw, beta = 0.1340, 1.769, 6.0
    seed = 1601004
    nsteps = args.warmup + args.steps

    # ------------------------------------------------------------ inputs
    t = time.time()
    U0 = inputs.quenched_field(L, seed, beta=beta, decorrelate=args.decorrelate)
    plaq0 = inputs.plaquette(U0, L)
    log("base field %s plaquette %.5f after %d full sweeps (%.1fs)" % (L, plaq0, args.decorrelate, time.time() - t))
    if args.factorized_only or args.projected_only:
        ctx = ddml.Context(L, ddml.BC_ANTIPERIODIC, device=0)
        U0_dev = torch.from_numpy(U0).to(dev)
        g = ctx.set_gauge(U0_dev, kappa, csw)
        tune = ctx.autotune(g, ctx.set_domain((0, 0, 0, 0), (16,) + L[1:]), 12, ddml.MIXED_FP32)
        log("autotune fp32 R=%d order=%d grid=%d splits=%d stage=%d (%.3f ms/pair)" % tune)
        if args.factorized_only:
            out = {"factorized_pion": run_factorized(ctx, ddml, torch, dev, U0_dev, L, kappa, csw, args)}
        else:
            out = {"projected_pion": run_projected(ctx, ddml, torch, dev, U0_dev, L, kappa, csw, args)}
        ctx.close()
        print(json.dumps(out), flush=True)
        return 0
    U0_dev = torch.from_numpy(U0).to(dev)
    srcs, terms = [], []
    xs = []
    for s in range(nslab):
        x = (16 * s + 7, 0, 0, 0)
        xs.append(x)
        b = torch.zeros((12, V, 4, 3), dtype=torch.complex128, device=dev)
        idx = inputs.site_index(L, x)
        for r in range(12):
            b[r, idx, r // 3, r % 3] = 1.0
        srcs.append(b)
        # two rounds in flight: ring of two series outputs per slab
        terms.append([torch.zeros((3, 12, V, 4, 3), dtype=torch.complex128, device=dev) for _ in range(2)])
    torch.cuda.synchronize()

    ctx = ddml.Context(L, ddml.BC_ANTIPERIODIC, device=0)
    gid0 = ctx.set_gauge(U0_dev, kappa, csw)
    doms = []
    for s in range(nslab):
        a = 16 * s
        doms.append([ctx.set_domain((a + 6, 0, 0, 0), (a + 10,) + L[1:]),
                     ctx.set_domain((a + 4, 0, 0, 0), (a + 12,) + L[1:]),
                     ctx.set_domain((a, 0, 0, 0), (a + 16,) + L[1:])])
    # BiCGstab with reliable updates: on these volumes keeping the Krylov space
    # across FP64 corrections saves a correction on Gamma2 (restarted BiCGstab,
    # the library default, does better on small lattices)
    params = ddml.solver_params(tol=1e-10, prec=ddml.MIXED_FP32, solver=1)
    # the project's autotuner picks the stencil launch (rhs per thread, tile order, grid)
    tune32 = ctx.autotune(gid0, doms[0][2], 12, ddml.MIXED_FP32)
    tune64 = ctx.autotune(gid0, doms[0][2], 12, ddml.FP64)
    log("autotune fp32 R=%d order=%d grid=%d splits=%d stage=%d (%.3f ms/pair); "
        "fp64 R=%d order=%d grid=%d splits=%d stage=%d (%.3f ms/pair)" % (tune32 + tune64))

    def advance(prev, j):
        """The level-1 update round j: every slab's chain moves on by one sweep
        (heatbath, first-slice spatial links frozen) on the device."""
        return [ctx.level1_update(prev[s], 16 * s, 16 * s + 16, beta, seed, 3 + 1000 + j * nslab + s, 1, 0)
                for s in range(nslab)]

    def release(gids):
        for g in gids:
            if g != gid0:
                ctx.release_gauge(g)

    def step(prev, j, prm=params, batched=True, update=True):
        gids = advance(prev, j) if update else prev
        if update:
            release(prev)   # the previous round's versions and their operator data
        buf = [terms[s][0] for s in range(nslab)]
        if batched:
            rc, infos = ctx.propagator_series_batch(
                [(gids[s], doms[s], srcs[s], buf[s], None) for s in range(nslab)], 12, prm)
        else:
            infos = []
            rc = ddml.OK
            for s in range(nslab):
                per = []
                for lev in range(3):
                    r, inf = ctx.solve_domain(gids[s], doms[s][lev], srcs[s], buf[s][lev], 12, prm)
                    rc = rc or r
                    per.append(inf)
                infos.append(per)
        nuc, pp = contract(buf)
        return gids, rc, infos, nuc, pp

    def contract(buf):
        nuc = [ctx.contract_nucleon(buf[s], 3) for s in range(nslab)]
        pp = [ctx.contract_pp_disconnected(buf[s], buf[(s + 2) % nslab], 3, xs[s], xs[(s + 2) % nslab])
              for s in range(nslab // 2)]
        tr = [ctx.trace_g5(buf[s], 3, xs[s]) for s in range(nslab)]   # factors of the two-level estimator
        return nuc, (pp, tr)

    def queue_rounds(chain, j0, n, prm):
        """Rounds j0 .. j0+n-1 as one continuous queue through the request loop.
        Round j draws the 4 slab updates on the device and submits their 4
        series (12 solves) into ring position j % 2; before that, round j - 2
        (the previous user of the position) is waited for, contracted and its
        gauge versions released.  Returns the last round's gauge versions, the
        per-round [slab][level][column] solve details and the contractions."""
        live = {}
        infos, meas, nucs = [], [], []

        def finish(r):
            gids, tks, inf = live.pop(r)
            for t in tks:
                res = ctx.wait(t, 1200.0)
                assert res is not None and res.status == ddml.OK, "series failed: %s" % (
                    None if res is None else ddml.STATUS_NAMES.get(res.status, res.status))
            nuc, pp = contract([terms[s][r % 2] for s in range(nslab)])
            nucs.append(nuc)
            meas.append(pp)
            infos.append([[list(inf[s][12 * lev:12 * (lev + 1)]) for lev in range(3)] for s in range(nslab)])
            return gids

        ctx.server_start(prm, max_queue=1000)
        try:
            older = []
            for j in range(j0, j0 + n):
                if j - 2 in live:
                    older.append(finish(j - 2))
                gids = advance(chain, j)
                tks, inf = [], []
                for s in range(nslab):
                    ia = (ddml.RhsInfo * 36)()
                    tks.append(ctx.submit_series(gids[s], doms[s], srcs[s], terms[s][j % 2], 12, info=ia))
                    inf.append(ia)
                live[j] = (gids, tks, inf)
                if j == j0:
                    older.append(chain)   # the chain heads this call started from
                chain = gids
                for g in older:
                    release(g)   # versions of finished rounds that no chain continues from
                older = []
            for r in sorted(live):
                g = finish(r)
                if g is not chain:
                    release(g)
        finally:
            ctx.server_stop()
        return chain, infos, nucs, meas

    # device level-1 generator on its own: one round of the 4 slab updates
    chain = [gid0] * nslab
    torch.cuda.synchronize()
    a = time.perf_counter()
    trial = advance(chain, 0)
    torch.cuda.synchronize()
    l1_ms = 1e3 * (time.perf_counter() - a) / nslab
    release(trial)
    nlinks = 16 * V3 * 4 - V3 * 3
    level1 = {"ms_per_slab_update": l1_ms, "links_per_s": nlinks / (l1_ms * 1e-3),
              "slab": "16 x %d^3, 1 heatbath sweep, spatial links of the first slice frozen" % L[1]}
    log("level-1 update: %.2f ms per 16-slice slab (%.3g links/s)" % (l1_ms, level1["links_per_s"]))

    # ------------------------------------------------------------ timed
    if args.warmup:
        chain, _, _, _ = queue_rounds(chain, 0, args.warmup, params)   # graph capture, allocator warm-up
        log("warmup: %d rounds" % args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chain, rinfos, _, meas = queue_rounds(chain, args.warmup, args.steps, params)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    iters, outers, worst = [], [], 0.0
    for per_round in rinfos:
        for per_slab in per_round:
            for per_level in per_slab:
                iters.append(max(i.inner_iters for i in per_level))
                outers.append(max(i.outer_iters for i in per_level))
                worst = max(worst, max(i.true_rel_residual for i in per_level))
    nsolves = 3 * nslab * args.steps
    solves_per_s = nsolves / (t1 - t0)
    ms_per_step = 1e3 * (t1 - t0) / args.steps
    log("mixed batched: %d solves in %.2fs -> %.3f solves/s, worst residual %.2e, inner iters %s"
        % (nsolves, t1 - t0, solves_per_s, worst, iters[:6]))

    two_level = two_level_pp(ddml, meas, nslab, L)
    log("two-level disconnected PP (n0 = 1, n1 = %d): f %s" % (args.steps, two_level["f"]))

    # ------------------------------------ 16-bit storage of the inner solve
    fp16 = None
    if not args.no_fp16:
        tune16 = ctx.autotune(gid0, doms[0][2], 12, ddml.MIXED_FP16)
        # restarted BiCGstab: with 16-bit storage each correction rebuilds the
        # Krylov space from the FP64 residual, which reaches 1e-10 in three
        prm16 = ddml.solver_params(tol=1e-10, prec=ddml.MIXED_FP16, solver=0)
        chain16 = [gid0] * nslab   # the same chains again, solved with 16-bit storage
        if args.warmup:
            chain16, _, _, _ = queue_rounds(chain16, 0, args.warmup, prm16)   # warm-up (graph capture)
        torch.cuda.synchronize()
        a = time.perf_counter()
        chain16, rinf16, _, _ = queue_rounds(chain16, args.warmup, args.steps, prm16)
        torch.cuda.synchronize()
        b = time.perf_counter()
        it16, outer16, worst16 = [], [], 0.0
        for per_round in rinf16:
            for per_slab in per_round:
                for per_level in per_slab:
                    it16.append(max(i.inner_iters for i in per_level))
                    outer16.append(max(i.outer_iters for i in per_level))
                    worst16 = max(worst16, max(i.true_rel_residual for i in per_level))
        release(chain16)
        s16 = ctx.time_stencil(gid0, doms[0][2], 12, ddml.MIXED_FP16, args.stencil_iters)
        fp16 = {"solves_per_s": nsolves / (b - a), "ms_per_step": 1e3 * (b - a) / args.steps,
                "inner_iters_per_solve": it16, "outer_iters_per_solve": outer16,
                "worst_true_rel_residual": worst16,
                "autotune": dict(zip(("R", "tile_order", "grid", "splits", "stage", "ms_pair"), tune16)),
                "stencil_even_half": {"ms": s16[1], "bytes": s16[3], "GB/s": s16[3] / s16[1] * 1e-6},
                "stencil_odd_half": {"ms": s16[0], "bytes": s16[2], "GB/s": s16[2] / s16[0] * 1e-6}}
        log("16-bit storage: %.3f solves/s, worst residual %.2e, inner iters %s, outer %s; stencil even %.3f ms "
            "%.0f GB/s (algorithmic, 16-bit)" % (fp16["solves_per_s"], worst16, it16[:6], outer16[:6], s16[1],
                                                 s16[3] / s16[1] * 1e-6))

    # --------------------------------------------------- stencil roofline
    # One application of the Schur operator M-hat (odd half, then even half) on
    # the 16-slice slab domain, 12 columns: (60 nrhs + LINK_REALS) reals per
    # site of the domain (input, intermediate and output spinors; links of
    # both halves and the clover inverse), HIP events around each launch.
    sten32 = ctx.time_stencil(gid0, doms[0][2], 12, ddml.MIXED_FP32, args.stencil_iters)
    sten64 = ctx.time_stencil(gid0, doms[0][2], 12, ddml.FP64, max(4, args.stencil_iters // 2))
    VG = 16 * V3
    bytes_pair = VG * (60 * 12 + LINK_REALS) * 4
    ms_pair = sten32[0] + sten32[1]
    ach = bytes_pair / (ms_pair * 1e-3)
    ach64 = VG * (60 * 12 + 216) * 8 / ((sten64[0] + sten64[1]) * 1e-3)
    t_odd = counter_traffic("odd,R=%d,order=%d,grid=%d,splits=%d,stage=%d" % tune32[:5])
    t_even = counter_traffic("even,R=%d,order=%d,grid=%d,splits=%d,stage=%d" % tune32[:5])
    traffic = (t_odd + t_even) if (t_odd is not None and t_even is not None) else None
    log("stencil fp32 M-hat: odd %.3f ms + even %.3f ms -> %.0f GB/s (%.3f of peak); fp64 M-hat %.0f GB/s"
        % (sten32[0], sten32[1], ach / 1e9, ach / PEAK_HBM, ach64 / 1e9))

    # ------------------------------------------------ plain FP64 baseline
    fp64 = None
    if not args.no_fp64:
        prm64 = ddml.solver_params(tol=1e-10, prec=ddml.FP64)
        torch.cuda.synchronize()
        a = time.perf_counter()
        _, rc, infos, _, _ = step(chain, nsteps - 1, prm64, batched=False, update=False)   # the last round's fields
        torch.cuda.synchronize()
        b = time.perf_counter()
        fp64 = {"solves_per_s": 3 * nslab / (b - a), "mode": "FP64 inner and outer, one solve at a time",
                "status": ddml.STATUS_NAMES[rc]}
        log("plain FP64 one-at-a-time: %.3f solves/s" % fp64["solves_per_s"])

    # ------------------------------------------------- factorized pion series
    # the series buffers of the multi-level workload are not needed any more
    terms.clear()
    srcs.clear()
    release(chain)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    fact = None
    if not args.no_factorized:
        fact = run_factorized(ctx, ddml, torch, dev, U0_dev, L, kappa, csw, args)
    hpe = None
    if not args.no_hpe:
        hpe = run_hpe(ctx, ddml, torch, dev, gid0, L, args)
    proj = None
    if not args.no_projected:
        proj = run_projected(ctx, ddml, torch, dev, U0_dev, L, kappa, csw, args)

    # ------------------------------------------------------------ serving
    serve = None
    if not args.no_serve:
        serve = run_serving(ctx, ddml, torch, dev, gid0, L, args)

    # ------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu:
        lev_iters = [float(np.mean(iters[k::3])) for k in range(3)]
        cpu = cpu_baseline(U0, L, kappa, csw, args.cpu_seconds, lev_iters)
        level1["cpu_oracle"] = cpu_level1(U0, L, beta, seed)

    ctx.close()
    out = {
        "metric": "domain solves/s & stencil HBM GB/s, mixed vs FP64 @1e-10; p50/p99 solve latency",
        "value": solves_per_s,
        "unit": "domain solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 inner / fp64 outer",
        "data": "synthetic: seeded beta=6.0 quenched heatbath fields and level-1 slab updates",
        "base_field": {"plaquette": plaq0, "full_volume_sweeps": args.decorrelate},
        "config": {"workload": "batched multi-level, %s lattice, %d slabs x %d updates as one continuous queue "
                               "(device-side outer loop), Gamma0/1/2 = 4/8/16 slices x 12 rhs, tol 1e-10"
                               % ("x".join(map(str, L)), nslab, args.steps),
                   "lattice": list(L), "kappa": kappa, "csw": csw, "solves_per_step": 3 * nslab, "nrhs": 12,
                   "solver": "FP32 BiCGstab with reliable updates, FP64 defect correction to 1e-10",
                   "solves": nsolves},
        "roofline": {"bound": "hbm", "achieved": ach / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                     "frac": ach / PEAK_HBM, "traffic": traffic,
                     "kernel": "k_hop_batch<float2> M-hat pair (odd half A^-1 H, then even half Schur + fused "
                               "shadow dot), 32^3x16 domain, 12 rhs",
                     "ms_per_launch": ms_pair, "bytes_per_launch": bytes_pair,
                     "bytes_per_site": (60 * 12 + LINK_REALS) * 4,
                     "odd_half": {"ms": sten32[0], "bytes": sten32[2], "GB/s": sten32[2] / sten32[0] * 1e-6},
                     "even_half": {"ms": sten32[1], "bytes": sten32[3], "GB/s": sten32[3] / sten32[1] * 1e-6},
                     "fp64_mhat_GBps": ach64 / 1e9},
        "autotune": {"fp32": dict(zip(("R", "tile_order", "grid", "splits", "stage", "ms_pair"), tune32)),
                     "fp64": dict(zip(("R", "tile_order", "grid", "splits", "stage", "ms_pair"), tune64))},
        "fp64_one_at_a_time": fp64,
        "fp16_storage": fp16,
        "mixed_over_fp64": (solves_per_s / fp64["solves_per_s"]) if fp64 else None,
        "serving": serve,
        "factorized_pion": fact,
        "stochastic_traces": hpe,
        "projected_pion": proj,
        "inner_iters_per_solve": iters,
        "outer_iters_per_solve": outers,
        "worst_true_rel_residual": worst,
        "level1_update": level1,
        "two_level_pp": two_level,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


def two_level_pp(ddml, meas, nslab, L):
    """Two-level estimate (Section 3.1) of the disconnected pseudoscalar pieces
    for the slab pairs (s, s + 2): the factorized part f = [t_x][t_y] / L^3 from
    the level-1 means of the two traces, each over its own slab's updates, and
    r1, r2 binned over the updates.  One level-0 field here (n0 = 1), so no
    error estimate; the rounds of the timed loop are the level-1 updates."""
    L3 = float(np.prod(L[1:]))
    n1 = len(meas)
    out = {"n0": 1, "n1": n1, "pairs": [], "f": [], "r1": [], "r2": []}
    for s in range(nslab // 2):
        y = (s + 2) % nslab
        tx = np.array([m[1][s] for m in meas])    # [n1, levels] complex
        ty = np.array([m[1][y] for m in meas])
        a = np.stack([tx.real, tx.imag], axis=1)[None]            # [1, n1, 2, levels]
        b = np.stack([ty.real, -ty.imag], axis=1)[None]           # Re(t_x t_y) = sum_c a_c b_c
        rest = np.array([np.concatenate([m[0][s][:, 1].real, m[0][s][:, 2].real]) for m in meas])[None]
        est, _, est_r, _ = ddml.two_level_average(a, b, rest)
        nl = tx.shape[1]
        out["pairs"].append([s, y])
        out["f"].append([est[i, i] / L3 for i in range(nl)])
        out["r1"].append(list(est_r[:nl]))
        out["r2"].append(list(est_r[nl:]))
    return out


SERVE_MIX = [((16, 8, 8, 8), (4, 12), 1601051), ((16, 16, 16, 16), (4, 12), 1601052),
             ((48, 24, 24, 24), (16, 32), 1601053), (None, (24, 40), None)]   # None: the base 32^3x64 field


def run_serving(ctx, ddml, torch, dev, gid0, L, args):
    """Serving workload: Poisson streams of domain-solve requests whose domain is
    drawn uniformly from the 8^4, 16^3x8, 24^3x16 and 32^3x16 Dirichlet time slabs
    of 8^3x16, 16^3x16, 24^3x48 and 32^3x64 fields (12 rhs, point source at the
    slab centre, mixed precision to 1e-10), at the configured rate and at 0.7x
    the measured capacity."""
    import inputs

    kinds = []
    for Lh, (t0, t1), seed in SERVE_MIX:
        if Lh is None:
            Lh, gid = L, gid0
        else:
            U = inputs.quenched_field(Lh, seed)
            gid = ctx.set_gauge_lattice(Lh, torch.from_numpy(U).to(dev), 0.1340, 1.769)
        dom = ctx.set_domain((t0, 0, 0, 0), (t1,) + tuple(Lh[1:]))
        src = ((t0 + t1) // 2, Lh[1] // 2, Lh[2] // 2, Lh[3] // 2)
        b = torch.from_numpy(inputs.point_source(Lh, src)).to(dev)
        sols = [torch.zeros_like(b) for _ in range(4)]   # reused round-robin (outputs not inspected here)
        kinds.append({"gid": gid, "dom": dom, "src": b, "sols": sols,
                      "name": "%d^3x%d" % (Lh[1], t1 - t0)})
    params = ddml.solver_params(tol=1e-10)
    # capacity: the mix (4 of each) as one batch; FP64 one at a time: one of each
    items = [(k["gid"], k["dom"], k["src"], k["sols"][j], 12) for j in range(4) for k in kinds]
    ctx.solve_batch(items[:4], params)   # warm-up
    torch.cuda.synchronize()
    a = time.perf_counter()
    rc, _ = ctx.solve_batch(items, params)
    torch.cuda.synchronize()
    capacity = len(items) / (time.perf_counter() - a)
    a = time.perf_counter()
    for k in kinds:
        ctx.solve_domain(k["gid"], k["dom"], k["src"], k["sols"][0], 12, ddml.solver_params(tol=1e-10, prec=ddml.FP64))
    torch.cuda.synchronize()
    fp64 = len(kinds) / (time.perf_counter() - a)

    def stream(rate, n, seed):
        rng = np.random.default_rng(seed)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n))
        pick = rng.integers(0, len(kinds), size=n)
        ctx.server_start(params, max_queue=100000)
        t0 = ddml.now()
        tickets = []
        for j in range(n):
            while ddml.now() - t0 < arrivals[j]:
                time.sleep(0.0005)
            k = kinds[int(pick[j])]
            tickets.append(ctx.submit(k["gid"], k["dom"], k["src"], k["sols"][j % 4], 12,
                                      arrival_time=t0 + arrivals[j]))
            if (j + 1) % 250 == 0:
                log("serving stream at %.3g req/s: %d of %d submitted" % (rate, j + 1, n))
        res = []
        for j, tk in enumerate(tickets):
            res.append(ctx.wait(tk, 600.0))
            if (j + 1) % 250 == 0:
                log("serving stream at %.3g req/s: %d of %d finished" % (rate, j + 1, n))
        st = ctx.stats()
        ctx.server_stop()
        ok = sum(1 for r in res if r is not None and r.status == ddml.OK)
        failed = {}
        for r in res:
            if r is None or r.status != ddml.OK:
                name = "timeout" if r is None else ddml.STATUS_NAMES.get(r.status, str(r.status))
                failed[name] = failed.get(name, 0) + 1
        return {"requests": n, "rate_req_per_s": rate, "ok": ok, "failed": failed, "p50_latency_s": st.p50_latency,
                "p99_latency_s": st.p99_latency, "mean_latency_s": st.mean_latency,
                "solves_per_s": st.solves_per_s}

    out = {"domains": "uniform over %s slabs (12 rhs, mixed 1e-10)" % ", ".join(k["name"] for k in kinds),
           "capacity_solves_per_s": capacity, "fp64_one_at_a_time_solves_per_s": fp64,
           "configured": stream(args.serve_rate, args.serve_requests, 1601005),
           "sub_saturation_0.7x": stream(0.7 * capacity, args.serve_requests, 1601006)}
    log("serving: %s" % out)
    return out


def run_factorized(ctx, ddml, torch, dev, U0_dev, L, kappa, csw, args):
    """Section 5.2 workload: S^(f) = -D_{Gamma*}^{-1} D_{dGamma*} D_{Gammabar_i}^{-1}
    with Gammabar_i = [0, x0cut + Delta_i), Gamma* = [x0cut, T), open time
    boundaries, then C^(i)_Pc, the series differences and the rest against the
    whole-lattice propagator.  Timed: the 2 x 3 domain solves (one batch per
    stage), the boundary blocks, the whole-lattice solve and the contraction."""
    T = L[0]
    xcut = 24 if T >= 48 else T // 2
    deltas = [d for d in (8, 12, 16) if xcut + d <= T] or [T - xcut]
    xsrc = (4 if xcut > 4 else 0, 0, 0, 0)
    V = int(np.prod(L))
    gid = ctx.set_gauge_lattice(L, U0_dev, kappa, csw, bc_time=ddml.BC_OPEN)
    bars = [ctx.set_domain((0, 0, 0, 0), (xcut + d,) + tuple(L[1:])) for d in deltas]
    star = ctx.set_domain((xcut, 0, 0, 0), tuple(L))
    b = torch.zeros((12, V, 4, 3), dtype=torch.complex128, device=dev)
    idx = ((xsrc[0] * L[1] + xsrc[1]) * L[2] + xsrc[2]) * L[3] + xsrc[3]
    for r in range(12):
        b[r, idx, r // 3, r % 3] = 1.0
    levels = torch.zeros((len(deltas), 12, V, 4, 3), dtype=torch.complex128, device=dev)
    full = torch.zeros((12, V, 4, 3), dtype=torch.complex128, device=dev)
    prm = ddml.solver_params(tol=1e-10)

    def once():
        t0 = time.perf_counter()
        rc, infos = ctx.factorized_series(gid, bars, star, b, 12, levels, None, prm)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rc2, info_full = ctx.solve_domain(gid, -1, b, full, 12, prm)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        C, diffs, rest = ctx.contract_pion(levels, len(deltas), full)
        t3 = time.perf_counter()
        return rc or rc2, infos, info_full, (C, diffs, rest), (t1 - t0, t2 - t1, t3 - t2)

    once()    # warm-up
    rc, infos, info_full, (C, diffs, rest), (ts, tf, tc) = once()
    assert rc == ddml.OK, "factorized series failed: %s" % ctx.last_error()
    chain = run_chain(ctx, ddml, torch, gid, L, b, full, xsrc, prm) if T >= 48 else None
    ctx.release_gauge(gid)
    worst = max(x.true_rel_residual for per in infos for stage in per for x in stage)
    ys = [y for y in (xcut, xcut + 8, xcut + 16, xcut + 24, T - 1) if y < T]
    out = {"lattice": list(L), "bc_time": "open", "x0cut": xcut, "deltas": deltas, "source": list(xsrc),
           "nrhs": 12, "tol": 1e-10, "prec": "fp32 inner / fp64 outer",
           "s_series": ts, "solves_per_s": 2 * len(deltas) / ts, "s_whole_lattice_solve": tf,
           "s_contraction": tc,
           "inner_iters": [[max(x.inner_iters for x in stage) for stage in per] for per in infos],
           "whole_lattice_inner_iters": max(x.inner_iters for x in info_full),
           "worst_true_rel_residual": worst,
           "C_levels": {str(y): [float(C[i, y]) for i in range(len(deltas))] for y in ys},
           "C_rest": {str(y): float(rest[y]) for y in ys},
           "multi_slab_chain": chain}
    log("factorized pion: %s" % out)
    return out


def run_chain(ctx, ddml, torch, gid, L, b, full, xsrc, prm, delta=8):
    """Section 4 workload (eq. fctpr): the lattice cut in thick slices of
    Delta = 8, the source in Lambda_0, sinks in Lambda_6 = [48, 56): the chain
    Omega_2 = [0, 16) (open boundary: no Lambda_{-1}), then Omega*_i =
    Lambda_i u Lambda_{i+1} for i = 1 .. 6, seven solves one after the other.
    Reported: the time, and C_Pc on the sink slices against the whole-lattice
    propagator (eq. errorfact)."""
    T = L[0]
    m, l = xsrc[0] // delta, 6
    blocks = [(max(0, (m - 1) * delta), (m + 2) * delta)] + \
             [(i * delta, min((i + 2) * delta, T)) for i in range(m + 1, l + 1)]
    doms = [ctx.set_domain((t0, 0, 0, 0), (t1,) + tuple(L[1:])) for t0, t1 in blocks]
    out = torch.zeros_like(full)
    torch.cuda.synchronize()
    a = time.perf_counter()
    rc, infos = ctx.factorized_chain(gid, doms, b, 12, out, None, prm)
    torch.cuda.synchronize()
    t = time.perf_counter() - a
    assert rc == ddml.OK, "chain failed: %s" % ctx.last_error()
    C, _, rest = ctx.contract_pion(out[None], 1, full)
    ys = [l * delta, l * delta + delta // 2, (l + 1) * delta - 1]
    res = {"delta": delta, "domains": [list(x) for x in blocks], "source": list(xsrc), "s": t,
           "solves_per_s": len(doms) / t,
           "inner_iters": [max(x.inner_iters for x in inf) for inf in infos],
           "C_chain": {str(y): float(C[0, y]) for y in ys},
           "C_exact": {str(y): float(C[0, y] + rest[y]) for y in ys},
           "rel_error": {str(y): float(abs(rest[y] / (C[0, y] + rest[y]))) for y in ys}}
    log("multi-slab chain: %s" % res)
    return res


def run_hpe(ctx, ddml, torch, dev, gid, L, args):
    """Section 6 workload: the disconnected traces on the two halves
    Gamma_A = [0, T/2), Gamma_B = [T/2, T) of the base field (clover, so the
    hopping parameter expansion goes to p = 2), from Gaussian sources over the
    volume drawn on the device with a seeded generator; 12 sources per solve.
    Timed: the solves, the 2 x p FP64 operator applications and the
    contractions of both domains."""
    T = L[0]
    V = int(np.prod(L))
    n = args.hpe_sources
    gen = torch.Generator(device=dev)
    gen.manual_seed(1601601)
    eta = torch.complex(torch.randn((n, V, 4, 3), generator=gen, device=dev, dtype=torch.float64),
                        torch.randn((n, V, 4, 3), generator=gen, device=dev, dtype=torch.float64)) / np.sqrt(2.0)
    doms = [ctx.set_domain((0, 0, 0, 0), (T // 2,) + tuple(L[1:])), ctx.set_domain((T // 2, 0, 0, 0), tuple(L))]
    prm = ddml.solver_params(tol=1e-10)
    ctx.hpe_trace(gid, doms[0], eta[:12].contiguous(), 12, 2, prm)   # warm-up
    torch.cuda.synchronize()
    a = time.perf_counter()
    outs, iters = [], []
    for d in doms:
        rc, out, info = ctx.hpe_trace(gid, d, eta, n, 2, prm)
        assert rc == ddml.OK, "stochastic trace failed: %s" % ctx.last_error()
        outs.append(out)
        iters.append(max(x.inner_iters for x in info))
    torch.cuda.synchronize()
    el = time.perf_counter() - a
    ys = [1, T // 4, T // 2 - 2, T // 2 + 1, 3 * T // 4, T - 2]
    res = {"lattice": list(L), "domains": "t in [0, %d) and [%d, %d)" % (T // 2, T // 2, T), "sources": n, "p": 2,
           "nrhs_per_solve": 12, "tol": 1e-10, "s": el, "sources_per_s": 2 * n / el,
           "domain_solves_per_s": 2 * ((n + 11) // 12) / el, "max_inner_iters": iters,
           "trace_p0": {str(y): [outs[y >= T // 2][0][y].real, outs[y >= T // 2][0][y].imag] for y in ys},
           "trace_hpe": {str(y): [outs[y >= T // 2][1][y].real, outs[y >= T // 2][1][y].imag] for y in ys}}
    log("stochastic traces: %s" % res)
    return res


def run_projected(ctx, ddml, torch, dev, U0_dev, L, kappa, csw, args):
    """Section 5.2 projector-cut workload on the base field with open time
    boundaries: n basis vectors from inverse iterations on
    Omega* = [x0cut - 8, x0cut + 8) (Gaussian start from a seeded device
    generator), then chi = D_Gammabar^{-1} gamma5 phi, eta = D_Gamma*^{-1} D_d phi,
    the per-slice Gram matrices (rocBLAS ZGEMM, batched over slices) and
    C(y0, x0) = -(1/L^3) Tr(Gt(y0) G(x0)), and from the same solves the
    nucleon of eq. W0tbary (slice sums of the colourless spinors of xi and
    eta, one ZGEMM per slice); x0cut = 24, Gammabar = [0, 32), Gamma* = [24, 64)."""
    T = L[0]
    xcut = 24 if T >= 48 else T // 2
    d = 8 if T >= 48 else max(2, T // 8)
    V = int(np.prod(L))
    n = args.proj_vectors
    gid = ctx.set_gauge_lattice(L, U0_dev, kappa, csw, bc_time=ddml.BC_OPEN)
    om = ctx.set_domain((xcut - d, 0, 0, 0), (xcut + d,) + tuple(L[1:]))
    bar = ctx.set_domain((0, 0, 0, 0), (xcut + d,) + tuple(L[1:]))
    star = ctx.set_domain((xcut, 0, 0, 0), tuple(L))
    gen = torch.Generator(device=dev)
    gen.manual_seed(1601901)
    start = torch.complex(torch.randn((n, V, 4, 3), generator=gen, device=dev, dtype=torch.float64),
                          torch.randn((n, V, 4, 3), generator=gen, device=dev, dtype=torch.float64))
    phi = torch.zeros_like(start)
    prm = ddml.solver_params(tol=1e-10)
    torch.cuda.synchronize()
    a = time.perf_counter()
    rc, info = ctx.inverse_iteration(gid, om, start, n, args.proj_iters, phi, prm)
    assert rc == ddml.OK, "inverse iteration failed: %s" % ctx.last_error()
    torch.cuda.synchronize()
    b = time.perf_counter()
    rc, CN, Cm, info2 = ctx.projected_nucleon(gid, bar, star, phi, n, prm, pion=True)
    assert rc == ddml.OK, "projected pion/nucleon failed: %s" % ctx.last_error()
    torch.cuda.synchronize()
    c = time.perf_counter()
    ctx.release_gauge(gid)
    x0 = 4 if xcut > 4 else 0
    ys = [y for y in (xcut, xcut + 8, xcut + 16, xcut + 24, T - 1) if y < T]
    res = {"lattice": list(L), "bc_time": "open", "vectors": n, "inverse_iterations": args.proj_iters,
           "omega": [xcut - d, xcut + d], "gammabar": [0, xcut + d], "gamma_star": [xcut, T],
           "s_inverse_iteration": b - a, "s_projected_pion_and_nucleon": c - b,
           "vector_solves_per_s": (args.proj_iters * n + 2 * n) / (c - a),
           "max_inner_iters": {"inverse_iteration_last": max(x.inner_iters for x in info),
                               "projected": max(x.inner_iters for x in info2)},
           "C_y0_x0=%d" % x0: {str(y): float(Cm[y, x0]) for y in ys},
           "nucleon_C_y0_x0=%d" % x0: {str(y): [float(CN[y, x0].real), float(CN[y, x0].imag)] for y in ys}}
    log("projected pion and nucleon: %s" % res)
    return res


def cpu_level1(U0, L, beta, seed):
    """The FP64 CPU oracle's level-1 sweep of one 16-slice slab (the same update
    the device makes first), timed on the host cores."""
    import oracle

    V3 = int(np.prod(L[1:]))
    t = time.time()
    oracle.level1_update(U0, L, beta, seed, 1000, 0, 16, 1, 0)
    dt = time.time() - t
    nlinks = 16 * V3 * 4 - V3 * 3
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
    return {"s_per_slab_update": dt, "links_per_s": nlinks / dt, "cores": cores, "kind": "oracle"}


def cpu_baseline(U0, L, kappa, csw, seconds, lev_iters):
    """FP64 CPU oracle on a bounded sample: one column of a Gamma0 (4 x 32^3)
    solve to 1e-10, scaled to the step's mix of Gamma0/1/2 solves (volumes
    1:2:4) with the GPU's measured inner iterations per level as the ratio of
    iteration counts (the oracle's unpreconditioned BiCGstab needs more
    iterations than the even-odd solve, by about the same factor on every
    level).  Also the single-thread rate from a few iterations on one thread."""
    import ctypes

    import inputs
    import oracle

    V3 = int(np.prod(L[1:]))
    Ls = (16,) + tuple(L[1:])
    Us = np.ascontiguousarray(U0[:16 * V3])          # slab 0 as its own 16 x 32^3 lattice
    C = oracle.clover_term(Us, Ls, csw)
    lo, hi = (6, 0, 0, 0), (10,) + tuple(L[1:])
    b = inputs.point_source(Ls, (7, 0, 0, 0))[:1]
    # calibrate the iteration time, then run a bounded solve
    t = time.time()
    oracle.solve(Us, Ls, kappa, b, C=C, lo=lo, hi=hi, tol=1e-30, maxiter=3)
    per_it = (time.time() - t) / 3
    maxit = max(5, int(seconds / per_it))
    t = time.time()
    x, it, res = oracle.solve(Us, Ls, kappa, b, C=C, lo=lo, hi=hi, tol=1e-10, maxiter=maxit)
    el = time.time() - t
    it = int(it[0])
    r = float(res[0])
    if r <= 1e-10:
        need = it
    else:  # linear in log residual
        need = int(np.ceil(it * np.log(1e-10) / np.log(max(r, 1e-300))))
    t_col = el / max(it, 1) * need
    vol = (1.0, 2.0, 4.0)
    ratio = [lev_iters[k] / lev_iters[0] for k in range(3)]
    t_step_cols = 12 * t_col * sum(vol[k] * ratio[k] for k in range(3))   # one Gamma0/1/2 triple
    solves_per_s = 3.0 / t_step_cols
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
    # one thread: a few iterations of the same column
    single = None
    try:
        omp = ctypes.CDLL("libgomp.so.1")
        omp.omp_set_num_threads(1)
        t = time.time()
        oracle.solve(Us, Ls, kappa, b, C=C, lo=lo, hi=hi, tol=1e-30, maxiter=3)
        per_it1 = (time.time() - t) / 3
        omp.omp_set_num_threads(cores)
        single = solves_per_s * per_it / per_it1
    except OSError:
        pass
    out = {"value": solves_per_s, "unit": "domain solves/s", "cores": cores, "kind": "oracle",
           "single_thread_value": single,
           "sample": "1 of 12 columns of a Gamma0 (4x32^3) solve, %d BiCGstab iterations in %.1fs, residual %.1e%s; "
                     "scaled to 12 columns and to the step's Gamma0/1/2 mix by volume (1:2:4) times the GPU's "
                     "measured inner-iteration ratio per level (%.2f : %.2f : %.2f)"
                     % (it, el, r, "" if r <= 1e-10 else " (iterations to 1e-10 extrapolated: %d)" % need,
                        ratio[0], ratio[1], ratio[2])}
    log("cpu baseline: %s" % out)
    return out


if __name__ == "__main__":
    sys.exit(main())
