"""GPU: the allocation-free nucleon contraction against the allocating one.

ddml_contract_nucleon_noalloc keeps its scratch (per-workgroup partial sums of
W_N1 - W_N2) in a static device array instead of allocating it.  Both entry
points contract the same terms; the slice sums are taken in a different order
(eight sites first), so the two agree to FP64 rounding: the tolerance is
64 ulp of the largest slice sum, far above the ~log2(V) ulp such a reordering
can move a sum of V/T site values of comparable size, and far below any
change of a term.  Two calls in a row, the second on a smaller lattice with
fewer levels, show that nothing of the first call's scratch leaks into the
second.  Host pointers and a request beyond the 16 MiB scratch are refused
on the host before any kernel is queued.
"""
import ctypes

import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu

ddml = pytest.importorskip("paper_1601_04587_amd.ddml")
torch = pytest.importorskip("torch")


def _terms(L, nlevels, seed):
    return inputs.gaussian(seed, 7, (nlevels, 12, int(np.prod(L)), 4, 3))


def _compare(L, nlevels, seed):
    dev = torch.device("cuda:0")
    T = L[0]
    ctx = ddml.Context(L, ddml.BC_ANTIPERIODIC, device=0)
    try:
        terms = torch.from_numpy(np.ascontiguousarray(_terms(L, nlevels, seed))).to(dev)
        ref_levels, ref_diffs = ctx.contract_nucleon(terms, nlevels)
        levels = torch.full((nlevels, T), complex(7.0, -7.0), dtype=torch.complex128, device=dev)
        diffs = torch.full((nlevels, T), complex(-3.0, 3.0), dtype=torch.complex128, device=dev)
        torch.cuda.synchronize()
        ctx.contract_nucleon_noalloc(terms, nlevels, levels, diffs)
        torch.cuda.synchronize()
        lv, df = levels.cpu().numpy(), diffs.cpu().numpy()
        scale = np.abs(ref_levels).max()
        assert scale > 0
        tol = 64 * np.finfo(np.float64).eps * scale
        assert np.abs(lv - ref_levels).max() <= tol
        assert np.abs(df - ref_diffs).max() <= 2 * tol
        # the differences telescope back to the levels
        assert np.abs(np.cumsum(df, axis=0) - lv).max() <= 4 * tol
    finally:
        ctx.close()


def test_noalloc_nucleon_matches_allocating_entry_point_twice():
    _compare((16, 8, 8, 8), 3, 1601091)
    _compare((8, 4, 4, 4), 2, 1601092)     # smaller lattice, fewer levels, same scratch


def test_noalloc_nucleon_rejects_host_memory_and_oversize():
    dev = torch.device("cuda:0")
    L = (8, 4, 4, 4)
    ctx = ddml.Context(L, ddml.BC_ANTIPERIODIC, device=0)
    try:
        host = np.zeros((2, 12, int(np.prod(L)), 4, 3), dtype=np.complex128)
        out = torch.zeros((2, L[0]), dtype=torch.complex128, device=dev)
        rc = ctx.lib.ddml_contract_nucleon_noalloc(ctx.h, host.ctypes.data, 2, out.data_ptr(), None, None)
        assert rc == ddml.EINVAL
        with pytest.raises(ValueError):
            ctx.contract_nucleon_noalloc(torch.from_numpy(host), 2, out)
    finally:
        ctx.close()
    # 64 x 32^3: 4 MiB of partial sums per level, so 5 levels exceed 16 MiB;
    # refused before the (too small) buffers are looked at
    big = ddml.Context((64, 32, 32, 32), ddml.BC_ANTIPERIODIC, device=0)
    try:
        t = torch.zeros(16, dtype=torch.complex128, device=dev)
        rc = big.lib.ddml_contract_nucleon_noalloc(big.h, t.data_ptr(), 5, t.data_ptr(), None, None)
        assert rc == ddml.EINVAL
        assert "16777216" in big.last_error()
    finally:
        big.close()
