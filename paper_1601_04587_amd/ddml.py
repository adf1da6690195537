"""Python binding of libddml (argument marshalling only).

Every entry point has the name and meaning of its C counterpart in
include/ddml.h.  Arrays are either numpy complex128 arrays (host, on_device=0)
or torch complex128 / float64 tensors on the GPU (on_device=1); torch is used
for device memory and the current stream only.  All arithmetic happens in the
HIP library; if libddml.so is missing, loading fails with an error.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddml.so")

OK, EINVAL, ENOMEM, EAGAIN, ENOTCONVERGED, ENUMERIC, EDEVICE = 0, -1, -2, -3, -4, -5, -6
BC_PERIODIC, BC_ANTIPERIODIC, BC_OPEN = 0, 1, 2
FP64, MIXED_FP32, MIXED_FP16 = 0, 1, 2
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EAGAIN", -4: "ENOTCONVERGED", -5: "ENUMERIC",
                -6: "EDEVICE"}


class Lattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("bc_time", ctypes.c_int)]


class SolverParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_outer", ctypes.c_int), ("max_inner", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("prec", ctypes.c_int), ("solver", ctypes.c_int),
                ("gcr_m", ctypes.c_int)]


class RhsInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("outer_iters", ctypes.c_int), ("inner_iters", ctypes.c_int),
                ("true_rel_residual", ctypes.c_double)]


class SolveDesc(ctypes.Structure):
    _fields_ = [("gauge_id", ctypes.c_int), ("dom_id", ctypes.c_int), ("src", ctypes.c_void_p),
                ("sol", ctypes.c_void_p), ("nrhs", ctypes.c_int), ("info", ctypes.POINTER(RhsInfo))]


class SeriesDesc(ctypes.Structure):
    _fields_ = [("gauge_id", ctypes.c_int), ("dom_ids", ctypes.POINTER(ctypes.c_int)), ("nlevels", ctypes.c_int),
                ("src", ctypes.c_void_p), ("terms", ctypes.c_void_p), ("sum", ctypes.c_void_p),
                ("info", ctypes.POINTER(RhsInfo))]


class Request(ctypes.Structure):
    _fields_ = [("gauge_id", ctypes.c_int), ("dom_id", ctypes.c_int), ("src", ctypes.c_void_p),
                ("sol", ctypes.c_void_p), ("nrhs", ctypes.c_int), ("arrival_time", ctypes.c_double)]


class SeriesRequest(ctypes.Structure):
    _fields_ = [("gauge_id", ctypes.c_int), ("dom_ids", ctypes.POINTER(ctypes.c_int)), ("nlevels", ctypes.c_int),
                ("src", ctypes.c_void_p), ("terms", ctypes.c_void_p), ("sum", ctypes.c_void_p),
                ("nrhs", ctypes.c_int), ("arrival_time", ctypes.c_double), ("info", ctypes.POINTER(RhsInfo))]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("max_outer", ctypes.c_int), ("max_inner_iters", ctypes.c_int),
                ("worst_rel_residual", ctypes.c_double), ("arrival_time", ctypes.c_double),
                ("admit_time", ctypes.c_double), ("finish_time", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_long), ("completed", ctypes.c_long), ("queued", ctypes.c_long),
                ("in_flight", ctypes.c_long), ("p50_latency", ctypes.c_double), ("p99_latency", ctypes.c_double),
                ("mean_latency", ctypes.c_double), ("solves_per_s", ctypes.c_double),
                ("hbm_in_use", ctypes.c_size_t), ("hbm_budget", ctypes.c_size_t)]


EXPORTS = ["ddml_create", "ddml_destroy", "ddml_last_error", "ddml_set_gauge", "ddml_set_gauge_lattice",
           "ddml_set_gauge_region", "ddml_level1_update", "ddml_get_gauge",
           "ddml_release_gauge", "ddml_set_domain", "ddml_apply_Dw", "ddml_apply_eo", "ddml_solve_domain",
           "ddml_solve_batch", "ddml_propagator_series", "ddml_propagator_series_batch", "ddml_time_stencil", "ddml_autotune", "ddml_set_launch", "ddml_contract_pp_disconnected", "ddml_contract_nucleon",
           "ddml_contract_nucleon_noalloc",
           "ddml_apply_boundary", "ddml_factorized_series", "ddml_factorized_chain", "ddml_contract_pion", "ddml_hpe_trace",
           "ddml_inverse_iteration", "ddml_projected_pion", "ddml_projected_nucleon", "ddml_two_level_average", "ddml_trace_g5",
           "ddml_server_start", "ddml_submit", "ddml_submit_series", "ddml_poll", "ddml_wait", "ddml_stats", "ddml_server_stop",
           "ddml_now"]

_lib = None


def load():
    """Load libddml.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libddml.so is not built; run `python -m paper_1601_04587_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    IP = ctypes.POINTER(ctypes.c_int)
    lib.ddml_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(Lattice), I, ctypes.c_size_t]
    lib.ddml_destroy.argtypes = [P]
    lib.ddml_last_error.argtypes = [P]
    lib.ddml_last_error.restype = ctypes.c_char_p
    lib.ddml_set_gauge.argtypes = [P, P, I, D, D, IP]
    lib.ddml_set_gauge_lattice.argtypes = [P, ctypes.POINTER(Lattice), P, I, D, D, IP]
    lib.ddml_set_gauge_region.argtypes = [P, I, I, I, P, I, IP]
    lib.ddml_level1_update.argtypes = [P, I, I, I, D, ctypes.c_uint64, ctypes.c_uint32, I, I, IP]
    lib.ddml_get_gauge.argtypes = [P, I, P, I]
    lib.ddml_projected_nucleon.argtypes = [P, I, I, I, P, I, ctypes.POINTER(SolverParams), P, P, P, I, P]
    lib.ddml_trace_g5.argtypes = [P, P, I, IP, P, I, P]
    lib.ddml_two_level_average.argtypes = [I, I, I, I, I, P, P, I, P, P, P, P, P]
    lib.ddml_release_gauge.argtypes = [P, I]
    lib.ddml_set_domain.argtypes = [P, IP, IP, IP]
    lib.ddml_apply_Dw.argtypes = [P, I, I, P, P, I, I, I, P]
    lib.ddml_apply_eo.argtypes = [P, I, I, P, P, I, I, I, P]
    lib.ddml_solve_domain.argtypes = [P, I, I, P, P, I, ctypes.POINTER(SolverParams), ctypes.POINTER(RhsInfo), I, P]
    lib.ddml_solve_batch.argtypes = [P, I, ctypes.POINTER(SolveDesc), ctypes.POINTER(SolverParams), I, P]
    lib.ddml_propagator_series.argtypes = [P, I, IP, I, P, I, ctypes.POINTER(SolverParams), P, P,
                                           ctypes.POINTER(RhsInfo), I, P]
    lib.ddml_propagator_series_batch.argtypes = [P, I, ctypes.POINTER(SeriesDesc), I, ctypes.POINTER(SolverParams),
                                                 I, P]
    lib.ddml_time_stencil.argtypes = [P, I, I, I, I, I, I, I, I, I, I, ctypes.POINTER(ctypes.c_double)]
    lib.ddml_autotune.argtypes = [P, I, I, I, I, ctypes.POINTER(ctypes.c_double)]
    lib.ddml_set_launch.argtypes = [P, I, I, I, I, I, I]
    lib.ddml_contract_pp_disconnected.argtypes = [P, P, P, I, IP, IP, P, I, P]
    lib.ddml_contract_nucleon.argtypes = [P, P, I, P, P, I, P]
    lib.ddml_contract_nucleon_noalloc.argtypes = [P, P, I, P, P, P]
    lib.ddml_apply_boundary.argtypes = [P, I, I, P, P, I, D, I, P]
    lib.ddml_factorized_chain.argtypes = [P, I, IP, I, P, I, ctypes.POINTER(SolverParams), P, P, P, I, P]
    lib.ddml_factorized_series.argtypes = [P, I, IP, I, I, P, I, ctypes.POINTER(SolverParams), P, P,
                                           ctypes.POINTER(RhsInfo), I, P]
    lib.ddml_contract_pion.argtypes = [P, P, I, P, P, P, P, I, P]
    lib.ddml_inverse_iteration.argtypes = [P, I, I, P, I, I, ctypes.POINTER(SolverParams), P,
                                           ctypes.POINTER(RhsInfo), I, P]
    lib.ddml_projected_pion.argtypes = [P, I, I, I, P, I, ctypes.POINTER(SolverParams), P, P, P,
                                        ctypes.POINTER(RhsInfo), I, P]
    lib.ddml_hpe_trace.argtypes = [P, I, I, P, I, I, ctypes.POINTER(SolverParams), P, P, P,
                                   ctypes.POINTER(RhsInfo), I, P]
    lib.ddml_server_start.argtypes = [P, ctypes.POINTER(SolverParams), I]
    lib.ddml_submit.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    lib.ddml_submit_series.argtypes = [P, ctypes.POINTER(SeriesRequest), ctypes.POINTER(ctypes.c_uint64)]
    lib.ddml_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(Result)]
    lib.ddml_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(Result), D]
    lib.ddml_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
    lib.ddml_server_stop.argtypes = [P]
    lib.ddml_now.argtypes = []
    lib.ddml_now.restype = D
    _lib = lib
    return lib


class DDMLError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(code, "?"), code, msg))
        self.code = code


def solver_params(tol=1e-10, max_outer=12, max_inner=4000, inner_tol=1e-5, prec=MIXED_FP32, solver=0, gcr_m=0):
    """solver 0: BiCGstab restarted at each FP64 correction; 1: BiCGstab with
    reliable updates; 2: GCR(gcr_m) (gcr_m 0 = 8)."""
    return SolverParams(tol, max_outer, max_inner, inner_tol, prec, solver, gcr_m)


def two_level_average(a, b, rest=None):
    """ddml_two_level_average: a [n0, n1, nc, ma], b [n0, n1, nc, mb], rest
    [n0, n1, k] or None (host float64).  Returns (est_f, err_f) [ma, mb] and,
    with rest, (est_r, err_r) [k]."""
    lib = load()
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    if a.ndim != 4 or b.ndim != 4 or a.shape[:3] != b.shape[:3]:
        raise ValueError("a and b must be [n0, n1, nc, m] with the same n0, n1, nc")
    n0, n1, nc, ma = a.shape
    mb = b.shape[3]
    est, err = np.zeros((ma, mb)), np.zeros((ma, mb))
    k = 0
    if rest is not None:
        rest = np.ascontiguousarray(rest, dtype=np.float64)
        if rest.ndim != 3 or rest.shape[:2] != (n0, n1):
            raise ValueError("rest must be [n0, n1, k]")
        k = rest.shape[2]
    est_r, err_r = np.zeros(k), np.zeros(k)
    rc = lib.ddml_two_level_average(n0, n1, nc, ma, mb, a.ctypes.data, b.ctypes.data, k,
                                    rest.ctypes.data if k else None, est.ctypes.data, err.ctypes.data,
                                    est_r.ctypes.data, err_r.ctypes.data)
    if rc != OK:
        raise DDMLError(rc, "ddml_two_level_average: bad sizes")
    return (est, err, est_r, err_r) if rest is not None else (est, err)


def _ptr(a):
    """(pointer, on_device) of a numpy array or a torch tensor."""
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data, 0
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr(), 1 if a.is_cuda else 0
    raise TypeError("expected numpy array or torch tensor")


def _stream(a):
    if hasattr(a, "is_cuda") and a.is_cuda:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream(a.device).cuda_stream)
    return ctypes.c_void_p(0)


def now():
    return load().ddml_now()


class Context:
    """One libddml context (ddml_create ... ddml_destroy)."""

    def __init__(self, dims, bc_time=BC_ANTIPERIODIC, device=0, hbm_budget=0):
        self.lib = load()
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.gauge_dims = {}   # host lattice of fields set with set_gauge_lattice
        lat = Lattice((ctypes.c_int * 4)(*self.dims), bc_time)
        h = ctypes.c_void_p()
        rc = self.lib.ddml_create(ctypes.byref(h), ctypes.byref(lat), device, hbm_budget)
        if rc != OK:
            raise DDMLError(rc, "ddml_create failed")
        self.h = h
        self.device = int(device)

    def close(self):
        if self.h:
            self.lib.ddml_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != OK and rc not in allow:
            raise DDMLError(rc, self.lib.ddml_last_error(self.h).decode())
        return rc

    def last_error(self):
        return self.lib.ddml_last_error(self.h).decode()

    # ------------------------------------------------------------ set-up
    def set_gauge(self, U, kappa, csw):
        p, dev = _ptr(U)
        gid = ctypes.c_int()
        self._check(self.lib.ddml_set_gauge(self.h, p, dev, kappa, csw, ctypes.byref(gid)))
        return gid.value

    def set_gauge_lattice(self, dims, U, kappa, csw, bc_time=BC_ANTIPERIODIC):
        """A gauge field on its own host lattice `dims` (T, L1, L2, L3)."""
        p, dev = _ptr(U)
        gid = ctypes.c_int()
        lat = Lattice((ctypes.c_int * 4)(*[int(v) for v in dims]), bc_time)
        self._check(self.lib.ddml_set_gauge_lattice(self.h, ctypes.byref(lat), p, dev, kappa, csw, ctypes.byref(gid)))
        self.gauge_dims[gid.value] = tuple(int(v) for v in dims)
        return gid.value

    def set_gauge_region(self, base, t0, t1, U_region):
        p, dev = _ptr(U_region)
        gid = ctypes.c_int()
        self._check(self.lib.ddml_set_gauge_region(self.h, base, t0, t1, p, dev, ctypes.byref(gid)))
        if base in self.gauge_dims:
            self.gauge_dims[gid.value] = self.gauge_dims[base]
        return gid.value

    def level1_update(self, base, t0, t1, beta, seed, stream, nsweeps=1, n_or=0):
        gid = ctypes.c_int()
        self._check(self.lib.ddml_level1_update(self.h, base, t0, t1, float(beta), int(seed) & (2**64 - 1),
                                                int(stream) & 0xFFFFFFFF, nsweeps, n_or, ctypes.byref(gid)))
        if base in self.gauge_dims:
            self.gauge_dims[gid.value] = self.gauge_dims[base]
        return gid.value

    def get_gauge(self, gid, out):
        p, dev = _ptr(out)
        self._check(self.lib.ddml_get_gauge(self.h, gid, p, dev))
        return out

    def release_gauge(self, gid):
        self._check(self.lib.ddml_release_gauge(self.h, gid))

    def set_domain(self, lo, hi):
        did = ctypes.c_int()
        self._check(self.lib.ddml_set_domain(self.h, (ctypes.c_int * 4)(*lo), (ctypes.c_int * 4)(*hi),
                                             ctypes.byref(did)))
        return did.value

    # ---------------------------------------------------------- operators
    def apply_Dw(self, gid, dom, inp, out, nrhs, prec=FP64):
        pi, dev = _ptr(inp)
        po, _ = _ptr(out)
        self._check(self.lib.ddml_apply_Dw(self.h, gid, dom, pi, po, nrhs, prec, dev, _stream(inp)))
        return out

    def apply_eo(self, gid, dom, inp, out, nrhs, prec=FP64):
        pi, dev = _ptr(inp)
        po, _ = _ptr(out)
        self._check(self.lib.ddml_apply_eo(self.h, gid, dom, pi, po, nrhs, prec, dev, _stream(inp)))
        return out

    def apply_boundary(self, gid, dom, inp, out, nrhs, scale=1.0):
        """out = scale * D_{dGamma} inp (couplings of D from outside the domain into it)."""
        pi, dev = _ptr(inp)
        po, _ = _ptr(out)
        self._check(self.lib.ddml_apply_boundary(self.h, gid, dom, pi, po, nrhs, float(scale), dev, _stream(inp)))
        return out

    # ------------------------------------------------------------- solves
    def solve_domain(self, gid, dom, src, sol, nrhs, params=None):
        params = params or solver_params()
        info = (RhsInfo * nrhs)()
        ps, dev = _ptr(src)
        pd, _ = _ptr(sol)
        rc = self.lib.ddml_solve_domain(self.h, gid, dom, ps, pd, nrhs, ctypes.byref(params), info, dev,
                                        _stream(src))
        self._check(rc, allow=(ENOTCONVERGED, ENUMERIC))
        return rc, list(info)

    def solve_batch(self, items, params=None):
        """items: list of (gauge_id, dom_id, src, sol, nrhs)."""
        params = params or solver_params()
        n = len(items)
        descs = (SolveDesc * n)()
        infos = []
        dev = 0
        for k, (gid, dom, src, sol, nrhs) in enumerate(items):
            info = (RhsInfo * nrhs)()
            infos.append(info)
            ps, dev = _ptr(src)
            pd, _ = _ptr(sol)
            descs[k] = SolveDesc(gid, dom, ps, pd, nrhs, ctypes.cast(info, ctypes.POINTER(RhsInfo)))
        rc = self.lib.ddml_solve_batch(self.h, n, descs, ctypes.byref(params), dev, _stream(items[0][2]))
        self._check(rc, allow=(ENOTCONVERGED, ENUMERIC))
        return rc, [list(i) for i in infos]

    def propagator_series(self, gid, doms, src, nrhs, terms, total=None, params=None):
        params = params or solver_params()
        n = len(doms)
        info = (RhsInfo * (n * nrhs))()
        ps, dev = _ptr(src)
        pt, _ = _ptr(terms)
        psum = _ptr(total)[0] if total is not None else None
        rc = self.lib.ddml_propagator_series(self.h, gid, (ctypes.c_int * n)(*doms), n, ps, nrhs,
                                             ctypes.byref(params), pt, psum, info, dev, _stream(src))
        self._check(rc, allow=(ENOTCONVERGED, ENUMERIC))
        return rc, [list(info[i * nrhs:(i + 1) * nrhs]) for i in range(n)]

    def propagator_series_batch(self, items, nrhs, params=None):
        """items: list of (gauge_id, dom_ids, src, terms, total_or_None); returns (rc, infos)."""
        params = params or solver_params()
        n = len(items)
        descs = (SeriesDesc * n)()
        keep = []
        dev = 0
        for k, (gid, doms, src, terms, total) in enumerate(items):
            nl = len(doms)
            d = (ctypes.c_int * nl)(*doms)
            info = (RhsInfo * (nl * nrhs))()
            keep.append((d, info))
            ps, dev = _ptr(src)
            pt, _ = _ptr(terms)
            psum = _ptr(total)[0] if total is not None else None
            descs[k] = SeriesDesc(gid, ctypes.cast(d, ctypes.POINTER(ctypes.c_int)), nl, ps, pt, psum,
                                  ctypes.cast(info, ctypes.POINTER(RhsInfo)))
        rc = self.lib.ddml_propagator_series_batch(self.h, n, descs, nrhs, ctypes.byref(params), dev,
                                                   _stream(items[0][2]))
        self._check(rc, allow=(ENOTCONVERGED, ENUMERIC))
        return rc, [[list(info[i * nrhs:(i + 1) * nrhs]) for i in range(len(d))] for d, info in keep]

    def factorized_series(self, gid, bar_doms, star_dom, src, nrhs, levels, bar=None, params=None):
        """S^(f)_i src = -D_{Gamma*}^{-1} D_{dGamma*} D_{Gammabar_i}^{-1} src for each Gammabar_i.

        Returns (rc, infos) with infos[i] = (Gammabar_i solve infos, Gamma* solve infos)."""
        params = params or solver_params()
        n = len(bar_doms)
        info = (RhsInfo * (2 * n * nrhs))()
        ps, dev = _ptr(src)
        pl, _ = _ptr(levels)
        pb = _ptr(bar)[0] if bar is not None else None
        rc = self.lib.ddml_factorized_series(self.h, gid, (ctypes.c_int * n)(*bar_doms), n, star_dom, ps, nrhs,
                                             ctypes.byref(params), pl, pb, info, dev, _stream(src))
        self._check(rc, allow=(ENOTCONVERGED, ENUMERIC))
        return rc, [(list(info[(2 * i) * nrhs:(2 * i + 1) * nrhs]), list(info[(2 * i + 1) * nrhs:(2 * i + 2) * nrhs]))
                    for i in range(n)]

    def factorized_chain(self, gid, doms, src, nrhs, out, steps=None, params=None):
        """psi_0 = D_{doms[0]}^{-1} src, psi_k = -D_{doms[k]}^{-1} D_{d doms[k]} psi_{k-1};
        out = the last psi.  Returns (rc, infos) with infos[k] the solve infos of step k."""
        params = params or solver_params()
        n = len(doms)
        info = (RhsInfo * (n * nrhs))()
        ps, dev = _ptr(src)
        po, _ = _ptr(out)
        pst = _ptr(steps)[0] if steps is not None else None
        rc = self.lib.ddml_factorized_chain(self.h, gid, (ctypes.c_int * n)(*doms), n, ps, nrhs,
                                            ctypes.byref(params), po, pst, info, dev, _stream(src))
        self._check(rc, allow=(ENOTCONVERGED, ENUMERIC))
        return rc, [list(info[k * nrhs:(k + 1) * nrhs]) for k in range(n)]

    def hpe_trace(self, gid, dom, eta, nsrc, p, params=None, psi_out=None, phi_out=None):
        """Stochastic trace estimates per time slice without and with the hopping
        parameter expansion; returns (rc, out [2, T] complex, infos)."""
        params = params or solver_params()
        T = self.gauge_dims.get(gid, self.dims)[0]
        out = np.zeros((2, T), dtype=np.complex128)
        info = (RhsInfo * nsrc)()
        pe, dev = _ptr(eta)
        pp = _ptr(psi_out)[0] if psi_out is not None else None
        pf = _ptr(phi_out)[0] if phi_out is not None else None
        rc = self.lib.ddml_hpe_trace(self.h, gid, dom, pe, nsrc, p, ctypes.byref(params), out.ctypes.data, pp, pf,
                                     info, dev, _stream(eta))
        self._check(rc, allow=(ENOTCONVERGED, ENUMERIC))
        return rc, out, list(info)

    def inverse_iteration(self, gid, dom, start, nvec, niter, out, params=None):
        """nvec orthonormal vectors on the domain from niter inverse iterations; returns (rc, infos)."""
        params = params or solver_params()
        info = (RhsInfo * nvec)()
        ps, dev = _ptr(start)
        po, _ = _ptr(out)
        rc = self.lib.ddml_inverse_iteration(self.h, gid, dom, ps, nvec, niter, ctypes.byref(params), po, info, dev,
                                             _stream(start))
        self._check(rc, allow=(ENOTCONVERGED, ENUMERIC))
        return rc, list(info)

    def projected_pion(self, gid, bar, star, phi, nvec, params=None, grams=False):
        """Projector-cut connected pion C(y0, x0) [T, T]; with grams=True also the
        per-slice Gram matrices (G, Gt) as [T, nvec, nvec] arrays (row-major i, j)."""
        params = params or solver_params()
        T = self.gauge_dims.get(gid, self.dims)[0]
        out = np.zeros((T, T))
        info = (RhsInfo * (2 * nvec))()
        gb = np.zeros((T, nvec, nvec), dtype=np.complex128) if grams else None
        gs = np.zeros((T, nvec, nvec), dtype=np.complex128) if grams else None
        pp, dev = _ptr(phi)
        rc = self.lib.ddml_projected_pion(self.h, gid, bar, star, pp, nvec, ctypes.byref(params), out.ctypes.data,
                                          gb.ctypes.data if grams else None, gs.ctypes.data if grams else None,
                                          info, dev, _stream(phi))
        self._check(rc, allow=(ENOTCONVERGED, ENUMERIC))
        if grams:   # stored column-major: transpose to [t][i][j]
            gb = np.ascontiguousarray(gb.transpose(0, 2, 1))
            gs = np.ascontiguousarray(gs.transpose(0, 2, 1))
        return rc, out, (gb, gs), list(info)

    def projected_nucleon(self, gid, bar, star, phi, nvec, params=None, pion=False):
        """Projector-cut nucleon C_N(y0, x0) [T, T] complex; with pion=True also the
        projected pion [T, T] from the same solves.  Returns (rc, C_N, C_pi or None, infos)."""
        params = params or solver_params()
        T = self.gauge_dims.get(gid, self.dims)[0]
        out = np.zeros((T, T), dtype=np.complex128)
        pout = np.zeros((T, T)) if pion else None
        info = (RhsInfo * (2 * nvec))()
        pp, dev = _ptr(phi)
        rc = self.lib.ddml_projected_nucleon(self.h, gid, bar, star, pp, nvec, ctypes.byref(params), out.ctypes.data,
                                             pout.ctypes.data if pion else None, info, dev, _stream(phi))
        self._check(rc, allow=(ENOTCONVERGED, ENUMERIC))
        return rc, out, pout, list(info)

    def time_stencil(self, gid, dom, nrhs, prec=MIXED_FP32, iters=20, R=0, order=-1, grid=0, splits=0, stage=-1):
        """(ms_odd_half, ms_even_half, bytes_odd_half, bytes_even_half) per launch."""
        out = (ctypes.c_double * 4)()
        self._check(self.lib.ddml_time_stencil(self.h, gid, dom, nrhs, prec, iters, R, order, grid, splits, stage,
                                               out))
        return tuple(out)

    def autotune(self, gid, dom, nrhs, prec=MIXED_FP32):
        """Pick the fastest stencil launch; returns (R, order, grid, splits, stage, ms per odd+even pair)."""
        out = (ctypes.c_double * 6)()
        self._check(self.lib.ddml_autotune(self.h, gid, dom, nrhs, prec, out))
        return int(out[0]), int(out[1]), int(out[2]), int(out[3]), int(out[4]), out[5]

    def set_launch(self, prec, R, order, grid, splits, stage):
        """Set the stencil launch of a precision by hand (see time_stencil)."""
        self._check(self.lib.ddml_set_launch(self.h, prec, R, order, grid, splits, stage))

    # ------------------------------------------------------- contractions
    def contract_pp_disconnected(self, terms_x, terms_y, nlevels, xsrc, ysrc):
        out = np.zeros((nlevels, 4), dtype=np.complex128)
        px, dev = _ptr(terms_x)
        py, _ = _ptr(terms_y)
        self._check(self.lib.ddml_contract_pp_disconnected(self.h, px, py, nlevels, (ctypes.c_int * 4)(*xsrc),
                                                           (ctypes.c_int * 4)(*ysrc), out.ctypes.data, dev,
                                                           _stream(terms_x)))
        return out

    def trace_g5(self, terms, nlevels, xsrc):
        out = np.zeros(nlevels, dtype=np.complex128)
        pt, dev = _ptr(terms)
        self._check(self.lib.ddml_trace_g5(self.h, pt, nlevels, (ctypes.c_int * 4)(*xsrc), out.ctypes.data, dev,
                                           _stream(terms)))
        return out

    def contract_nucleon(self, terms, nlevels):
        T = self.dims[0]
        levels = np.zeros((nlevels, T), dtype=np.complex128)
        diffs = np.zeros((nlevels, T), dtype=np.complex128)
        pt, dev = _ptr(terms)
        self._check(self.lib.ddml_contract_nucleon(self.h, pt, nlevels, levels.ctypes.data, diffs.ctypes.data, dev,
                                                   _stream(terms)))
        return levels, diffs

    def contract_nucleon_noalloc(self, terms, nlevels, levels_out, diffs_out=None):
        """ddml_contract_nucleon_noalloc: terms, levels_out [nlevels, T] and diffs_out
        (or None) complex128 device tensors; queued on terms' current stream."""
        for a in (terms, levels_out) + ((diffs_out,) if diffs_out is not None else ()):
            if not (hasattr(a, "is_cuda") and a.is_cuda):
                raise ValueError("contract_nucleon_noalloc takes device tensors")
        pt, _ = _ptr(terms)
        pl, _ = _ptr(levels_out)
        pd = _ptr(diffs_out)[0] if diffs_out is not None else None
        self._check(self.lib.ddml_contract_nucleon_noalloc(self.h, pt, nlevels, pl, pd, _stream(terms)))

    def contract_pion(self, levels, nlevels, full=None):
        """Connected pion correlator per level, its series differences and (with the full
        propagator) the rest; returns (levels [n, T], diffs [n, T], rest [T] or None)."""
        T = self.dims[0]
        lv = np.zeros((nlevels, T))
        df = np.zeros((nlevels, T))
        rest = np.zeros(T) if full is not None else None
        pl, dev = _ptr(levels)
        pf = _ptr(full)[0] if full is not None else None
        self._check(self.lib.ddml_contract_pion(self.h, pl, nlevels, pf, lv.ctypes.data, df.ctypes.data,
                                                rest.ctypes.data if rest is not None else None, dev,
                                                _stream(levels)))
        return lv, df, rest

    # ------------------------------------------------------------ serving
    def server_start(self, params=None, max_queue=100000):
        params = params or solver_params()
        self._check(self.lib.ddml_server_start(self.h, ctypes.byref(params), max_queue))

    def submit(self, gid, dom, src, sol, nrhs, arrival_time=None):
        """Queue one request; src and sol must be contiguous device tensors on
        the context's device (the request loop reads and writes them later)."""
        for name, a in (("src", src), ("sol", sol)):
            if not (hasattr(a, "is_cuda") and a.is_cuda and a.is_contiguous()):
                raise ValueError("%s must be a contiguous device tensor" % name)
            if a.device.index != self.device:
                raise ValueError("%s is on device %s, the context on %d" % (name, a.device, self.device))
        ps, _ = _ptr(src)
        pd, _ = _ptr(sol)
        t = now() if arrival_time is None else arrival_time
        req = Request(gid, dom, ps, pd, nrhs, t)
        ticket = ctypes.c_uint64()
        rc = self.lib.ddml_submit(self.h, ctypes.byref(req), ctypes.byref(ticket))
        self._check(rc)
        return ticket.value

    def submit_series(self, gid, doms, src, terms, nrhs, sum=None, info=None, arrival_time=None):
        """Queue a propagator series over the nested domains `doms` (eq. Dseries);
        src, terms ([levels][nrhs][V][4][3]) and sum are contiguous device tensors
        on the context's device, info an optional (RhsInfo * levels*nrhs) array
        filled before completion."""
        for name, a in (("src", src), ("terms", terms), ("sum", sum)):
            if a is None and name == "sum":
                continue
            if not (hasattr(a, "is_cuda") and a.is_cuda and a.is_contiguous()):
                raise ValueError("%s must be a contiguous device tensor" % name)
            if a.device.index != self.device:
                raise ValueError("%s is on device %s, the context on %d" % (name, a.device, self.device))
        ids = (ctypes.c_int * len(doms))(*doms)
        ps, _ = _ptr(src)
        pt, _ = _ptr(terms)
        pm = _ptr(sum)[0] if sum is not None else None
        t = now() if arrival_time is None else arrival_time
        inf = ctypes.cast(info, ctypes.POINTER(RhsInfo)) if info is not None else None
        req = SeriesRequest(gid, ids, len(doms), ps, pt, pm, nrhs, t, inf)
        ticket = ctypes.c_uint64()
        rc = self.lib.ddml_submit_series(self.h, ctypes.byref(req), ctypes.byref(ticket))
        self._check(rc)
        return ticket.value

    def poll(self, ticket):
        r = Result()
        rc = self.lib.ddml_poll(self.h, ticket, ctypes.byref(r))
        if rc == EAGAIN:
            return None
        self._check(rc)
        return r

    def wait(self, ticket, timeout=-1.0):
        r = Result()
        rc = self.lib.ddml_wait(self.h, ticket, ctypes.byref(r), timeout)
        if rc == EAGAIN:
            return None
        self._check(rc)
        return r

    def stats(self):
        s = ServerStats()
        self._check(self.lib.ddml_stats(self.h, ctypes.byref(s)))
        return s

    def server_stop(self):
        self._check(self.lib.ddml_server_stop(self.h))
