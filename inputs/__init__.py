"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

Holds none of the method's arithmetic: only the Philox random generator, the
quenched SU(3) gauge-field generator (Cabibbo-Marinari heatbath plus
over-relaxation at coupling beta), level-1 slab updates with frozen boundary
links, Gaussian sources and unit point sources.  The paper's own ensembles are
HMC-generated 24^3x64 quenched fields at beta=6.0 that do not ship with it; the
fields here stand in for them (same action, same coupling).

Array conventions (numpy, complex128):
  links   U[site, mu, 3, 3], U_mu(x) joins x and x+mu, site = ((t*L1+x1)*L2+x2)*L3+x3
  spinors psi[rhs, site, 4, 3]
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libgen.so")
_lib = None


def build(force=False):
    """Compile gen.c into libgen.so next to it (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", "-O3", "-fcx-limited-range", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_DEFAULT_SOURCE", "-o", _LIB + ".tmp", _SRC, "-lm"])
        os.replace(_LIB + ".tmp", _LIB)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i4 = ctypes.POINTER(ctypes.c_int)
        lib.gen_philox4x32_10.argtypes = [P, P, P]
        lib.gen_random_links.argtypes = [i4, ctypes.c_uint64, ctypes.c_double, P]
        lib.gen_heatbath.argtypes = [i4, ctypes.c_double, ctypes.c_uint64, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, P]
        lib.gen_level1_update.argtypes = [i4, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
        lib.gen_tile.argtypes = [i4, P, i4, P]
        lib.gen_plaquette.argtypes = [i4, P]
        lib.gen_plaquette.restype = ctypes.c_double
        lib.gen_gaussian.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_long, P]
        lib.gen_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_long, P]
        _lib = lib
    return _lib


def _dims(L):
    L = tuple(int(v) for v in L)
    assert len(L) == 4 and all(v > 0 for v in L)
    return (ctypes.c_int * 4)(*L), L


def volume(L):
    return int(np.prod(L))


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: 4 counter words, 2 key words -> 4 output words."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    _load().gen_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def random_links(L, seed, eps=0.3):
    """U_mu(x) = exp(i eps H), H = sum_a h_a lambda_a/2, h_a ~ N(0,1) (Gell-Mann lambda_a)."""
    cL, L = _dims(L)
    U = np.empty((volume(L), 4, 3, 3), dtype=np.complex128)
    _load().gen_random_links(cL, seed, eps, U.ctypes.data)
    return U


def unit_links(L):
    U = np.zeros((volume(L), 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    return U


def heatbath(L, beta, seed, nsweeps, n_or=4, hot_start=True, U=None):
    """Quenched field: hot start then nsweeps x (1 heatbath + n_or over-relaxation)."""
    cL, L = _dims(L)
    if U is None:
        U = np.empty((volume(L), 4, 3, 3), dtype=np.complex128)
    else:
        U = np.ascontiguousarray(U, dtype=np.complex128).copy()
    _load().gen_heatbath(cL, beta, seed, nsweeps, n_or, 1 if hot_start else 0, U.ctypes.data)
    return U


def tile(Usmall, Ls, L):
    """Periodic replication of a small field into a larger lattice."""
    cLs, Ls = _dims(Ls)
    cL, L = _dims(L)
    assert all(a % b == 0 for a, b in zip(L, Ls))
    U = np.empty((volume(L), 4, 3, 3), dtype=np.complex128)
    _load().gen_tile(cLs, np.ascontiguousarray(Usmall).ctypes.data, cL, U.ctypes.data)
    return U


def level1_update(U, L, beta, seed, update_id, t0, t1, nsweeps=1, n_or=4):
    """New field: U with the slab [t0,t1) updated, spatial links of slice t0 frozen."""
    cL, L = _dims(L)
    U2 = np.ascontiguousarray(U, dtype=np.complex128).copy()
    _load().gen_level1_update(cL, beta, seed, update_id, t0, t1, nsweeps, n_or, U2.ctypes.data)
    return U2


def level1_update_inplace(U, L, beta, seed, update_id, t0, t1, nsweeps=1, n_or=4):
    """In-place version of level1_update (U must be C-contiguous complex128).

    Updates of different slabs touch disjoint links and read only their own
    slab and frozen links, so several slab chains can share one array."""
    cL, L = _dims(L)
    assert U.dtype == np.complex128 and U.flags["C_CONTIGUOUS"]
    _load().gen_level1_update(cL, beta, seed, update_id, t0, t1, nsweeps, n_or, U.ctypes.data)
    return U


def plaquette(U, L):
    cL, L = _dims(L)
    return _load().gen_plaquette(cL, np.ascontiguousarray(U).ctypes.data)


def gaussian(seed, stream, shape):
    """Complex Gaussian array with E|z|^2 = 1."""
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.complex128)
    _load().gen_gaussian(seed, stream, n, out.ctypes.data)
    return out.reshape(shape)


def uniform(seed, stream, n):
    out = np.empty(int(n), dtype=np.float64)
    _load().gen_uniform(seed, stream, int(n), out.ctypes.data)
    return out


def point_source(L, x):
    """12 right-hand sides: a unit spin-colour vector at site x (rhs = 3*beta + b)."""
    L = tuple(L)
    V = volume(L)
    idx = ((x[0] * L[1] + x[1]) * L[2] + x[2]) * L[3] + x[3]
    b = np.zeros((12, V, 4, 3), dtype=np.complex128)
    for r in range(12):
        b[r, idx, r // 3, r % 3] = 1.0
    return b


def site_index(L, x):
    return ((x[0] * L[1] + x[1]) * L[2] + x[2]) * L[3] + x[3]


# ------------------------------------------------------------------ recipes
_CACHE_DIR = os.environ.get("DDML_INPUT_CACHE", os.path.join(os.path.dirname(_HERE), ".inputs_cache"))
_mem_cache = {}


def _cached(name, fn):
    if name in _mem_cache:
        return _mem_cache[name]
    path = os.path.join(_CACHE_DIR, name + ".npy")
    if os.path.exists(path):
        arr = np.load(path)
    else:
        arr = fn()
        try:
            os.makedirs(_CACHE_DIR, exist_ok=True)
            np.save(path + ".tmp.npy", arr)
            os.replace(path + ".tmp.npy", path)
        except OSError:
            pass
    _mem_cache[name] = arr
    return arr


def quenched_field(L, seed, beta=6.0, therm_sweeps=200, base=(16, 8, 8, 8), decorrelate=4):
    """A beta=6.0 quenched field of dims L.

    Lattices no larger than `base` are thermalised directly from a hot start
    with `therm_sweeps` sweeps (1 heatbath + 4 over-relaxation each).  Larger
    lattices replicate a thermalised `base` field periodically and then run
    `decorrelate` full sweeps on the large lattice, which restores local
    equilibrium fluctuations at a small fraction of the cost of thermalising
    the large lattice from scratch.
    """
    L = tuple(int(v) for v in L)
    name = "q_%s_%d_b%g_t%d_d%d_base%s" % ("x".join(map(str, L)), seed, beta, therm_sweeps,
                                           decorrelate, "x".join(map(str, base)))
    if volume(L) <= volume(base) or any(a % b for a, b in zip(L, base)):
        return _cached(name, lambda: heatbath(L, beta, seed, therm_sweeps))

    def make():
        Ub = quenched_field(base, seed, beta, therm_sweeps, base, decorrelate)
        U = tile(Ub, base, L)
        return heatbath(L, beta, seed + 17, decorrelate, hot_start=False, U=U)
    return _cached(name, make)
