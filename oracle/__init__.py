"""CPU oracle for the conservative CCD pipeline (test infrastructure only).

Plain, slow, independent reference implementation in C (ccd_oracle.c),
loaded through ctypes.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product package never imports it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ccd_oracle.c")
_LIB = os.path.join(_HERE, "libccd_oracle.so")
_lib = None

KIND_VF, KIND_EE = 0, 1


def build(force=True):
    """Compile the oracle with contraction off (every fma is explicit)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-pthread", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.oracle_rd32.restype = ctypes.c_float
    lib.oracle_rd32.argtypes = [ctypes.c_double]
    lib.oracle_ru32.restype = ctypes.c_float
    lib.oracle_ru32.argtypes = [ctypes.c_double]
    lib.oracle_boxes.argtypes = [P, P, i64, P, i64, P, i64, P, P]
    lib.oracle_broad.argtypes = [P, P, i64, P, i64, P, i64, ctypes.c_int,
                                 ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)), ctypes.POINTER(i64),
                                 ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)), ctypes.POINTER(i64)]
    lib.oracle_broad_sample.argtypes = [P, P, i64, P, i64, P, i64, ctypes.c_int, i64, ctypes.POINTER(i64),
                                        ctypes.POINTER(i64), P]
    lib.oracle_free.argtypes = [P]
    lib.oracle_query.argtypes = [ctypes.c_int, P, ctypes.c_double, i64, P, P, P, P]
    lib.oracle_query_levels.argtypes = [ctypes.c_int, P, ctypes.c_double, i64, P, P, P, P]
    lib.oracle_eval_F.argtypes = [ctypes.c_int, P, ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
    lib.oracle_eps.argtypes = [ctypes.c_int, P, P]
    lib.oracle_levels_needed.argtypes = [ctypes.c_int, P, ctypes.c_double, P]
    lib.oracle_narrow.argtypes = [P, P, P, P, P, i64, P, i64, ctypes.c_double, i64, ctypes.c_int,
                                  P, P, P, P, P, P]
    lib.oracle_narrow_ex.argtypes = [P, P, P, P, P, i64, P, i64, ctypes.c_double, i64, P, ctypes.c_int,
                                     ctypes.c_int, P, P, P, P, P, P]
    lib.oracle_narrow_global.argtypes = [P, P, P, P, P, i64, P, i64, ctypes.c_double, i64, P, ctypes.c_int,
                                         P, P, P]
    lib.oracle_initial_distance.argtypes = [P, P, P, P, i64, P, i64, P]
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def default_threads():
    return max(1, min(16, os.cpu_count() or 1))


def rd32(x):
    return np.float32(_load().oracle_rd32(float(x)))


def ru32(x):
    return np.float32(_load().oracle_ru32(float(x)))


def boxes(V0, V1, E, F):
    """Per-primitive boxes, vertices then edges then faces: (lo, hi), each nb x 3 float32."""
    lib = _load()
    V0, V1 = _c(V0, np.float64), _c(V1, np.float64)
    E, F = _c(E, np.int32).reshape(-1, 2), _c(F, np.int32).reshape(-1, 3)
    nb = len(V0) + len(E) + len(F)
    lo = np.zeros((nb, 3), np.float32)
    hi = np.zeros((nb, 3), np.float32)
    lib.oracle_boxes(_ptr(V0), _ptr(V1), len(V0), _ptr(E), len(E), _ptr(F), len(F), _ptr(lo), _ptr(hi))
    return lo, hi


def broad(V0, V1, E, F, nthreads=None):
    """All overlapping VF and EE pairs by brute force, sorted: (vf (n,2), ee (m,2)) int32."""
    lib = _load()
    V0, V1 = _c(V0, np.float64), _c(V1, np.float64)
    E, F = _c(E, np.int32).reshape(-1, 2), _c(F, np.int32).reshape(-1, 3)
    pvf = ctypes.POINTER(ctypes.c_int32)()
    pee = ctypes.POINTER(ctypes.c_int32)()
    nvf = ctypes.c_int64()
    nee = ctypes.c_int64()
    lib.oracle_broad(_ptr(V0), _ptr(V1), len(V0), _ptr(E), len(E), _ptr(F), len(F),
                     nthreads or default_threads(), ctypes.byref(pvf), ctypes.byref(nvf),
                     ctypes.byref(pee), ctypes.byref(nee))
    vf = np.ctypeslib.as_array(pvf, shape=(max(nvf.value, 1) * 2,))[:nvf.value * 2].reshape(-1, 2).copy()
    ee = np.ctypeslib.as_array(pee, shape=(max(nee.value, 1) * 2,))[:nee.value * 2].reshape(-1, 2).copy()
    lib.oracle_free(ctypes.cast(pvf, ctypes.c_void_p))
    lib.oracle_free(ctypes.cast(pee, ctypes.c_void_p))
    return vf, ee


def broad_sample(V0, V1, E, F, stride, nthreads=None):
    """Timing sample of `broad`: the brute force over 1 / stride of its rows.  Returns
    (VF pairs found, EE pairs found, VF box tests, EE box tests)."""
    lib = _load()
    V0, V1 = _c(V0, np.float64), _c(V1, np.float64)
    E, F = _c(E, np.int32).reshape(-1, 2), _c(F, np.int32).reshape(-1, 3)
    nvf, nee = ctypes.c_int64(), ctypes.c_int64()
    tests = np.zeros(2, np.float64)
    lib.oracle_broad_sample(_ptr(V0), _ptr(V1), len(V0), _ptr(E), len(E), _ptr(F), len(F),
                            nthreads or default_threads(), int(stride), ctypes.byref(nvf), ctypes.byref(nee),
                            _ptr(tests))
    return nvf.value, nee.value, float(tests[0]), float(tests[1])


def query(kind, q24, delta=1e-6, max_iter=10**6):
    """One query (24 doubles: 4 points at t=0 then at t=1). Returns (hit, toi, n_enq, n_eval)."""
    lib = _load()
    q = _c(q24, np.float64).reshape(24)
    hit = np.zeros(1, np.uint8)
    toi = np.zeros(1, np.float64)
    ne = np.zeros(1, np.int64)
    nv = np.zeros(1, np.int64)
    lib.oracle_query(int(kind), _ptr(q), float(delta), int(max_iter), _ptr(hit), _ptr(toi), _ptr(ne), _ptr(nv))
    return bool(hit[0]), float(toi[0]), int(ne[0]), int(nv[0])


def query_levels(kind, q24, delta=1e-6, max_iter=10**6):
    """One query; returns (hit, toi, n_enq, levels): levels = (l_t, l_u, l_v) of the last frontier built."""
    lib = _load()
    q = _c(q24, np.float64).reshape(24)
    hit = np.zeros(1, np.uint8)
    toi = np.zeros(1, np.float64)
    ne = np.zeros(1, np.int64)
    lv = np.zeros(3, np.int32)
    lib.oracle_query_levels(int(kind), _ptr(q), float(delta), int(max_iter), _ptr(hit), _ptr(toi), _ptr(ne),
                            _ptr(lv))
    return bool(hit[0]), float(toi[0]), int(ne[0]), tuple(int(x) for x in lv)


def eval_F(kind, q24, t, u, v):
    lib = _load()
    q = _c(q24, np.float64).reshape(24)
    out = np.zeros(3, np.float64)
    lib.oracle_eval_F(int(kind), _ptr(q), float(t), float(u), float(v), _ptr(out))
    return out


def eps(kind, q24):
    lib = _load()
    q = _c(q24, np.float64).reshape(24)
    out = np.zeros(3, np.float64)
    lib.oracle_eps(int(kind), _ptr(q), _ptr(out))
    return out


def levels_needed(kind, q24, delta):
    lib = _load()
    q = _c(q24, np.float64).reshape(24)
    out = np.zeros(3, np.int32)
    lib.oracle_levels_needed(int(kind), _ptr(q), float(delta), _ptr(out))
    return out


def _min_sep(ms, n):
    if ms is None:
        return None
    ms = _c(ms, np.float64).reshape(-1)
    if len(ms) != n or not np.all(np.isfinite(ms)) or np.any(ms < 0):
        raise ValueError("ms must hold one finite, non-negative separation per pair")
    return ms


def narrow_with_work(V0, V1, E, F, vf, ee, delta=1e-6, max_iter=10**6, nthreads=None, ms=None, no_zero=False):
    """Per-pair (hit, toi, n_enq, n_eval, n_axis) and the global minimum TOI.

    n_axis counts the per-axis inclusion boxes the solver computed (its
    arithmetic work).  ms: per-pair minimum separation (Sec. 7) or None;
    no_zero: the no-zero-TOI strategy (App. B)."""
    lib = _load()
    V0, V1 = _c(V0, np.float64), _c(V1, np.float64)
    E, F = _c(E, np.int32).reshape(-1, 2), _c(F, np.int32).reshape(-1, 3)
    vf = _c(vf, np.int32).reshape(-1, 2)
    ee = _c(ee, np.int32).reshape(-1, 2)
    n = len(vf) + len(ee)
    hit = np.zeros(n, np.uint8)
    toi = np.zeros(n, np.float64)
    n_enq = np.zeros(n, np.int64)
    n_eval = np.zeros(n, np.int64)
    n_axis = np.zeros(n, np.int64)
    tmin = np.zeros(1, np.float64)
    ms = _min_sep(ms, n)
    lib.oracle_narrow_ex(_ptr(V0), _ptr(V1), _ptr(E), _ptr(F), _ptr(vf), len(vf), _ptr(ee), len(ee),
                         float(delta), int(max_iter), _ptr(ms), int(bool(no_zero)), nthreads or default_threads(),
                         _ptr(hit), _ptr(toi), _ptr(n_enq), _ptr(n_eval), _ptr(n_axis), _ptr(tmin))
    return hit, toi, n_enq, n_eval, n_axis, float(tmin[0])


def narrow(V0, V1, E, F, vf, ee, delta=1e-6, max_iter=10**6, nthreads=None, ms=None, no_zero=False):
    """Per-pair (hit uint8, toi float64, n_enq int64, n_eval int64) and the global minimum TOI."""
    hit, toi, n_enq, n_eval, _, tmin = narrow_with_work(V0, V1, E, F, vf, ee, delta, max_iter, nthreads, ms,
                                                        no_zero)
    return hit, toi, n_enq, n_eval, tmin


def narrow_global(V0, V1, E, F, vf, ee, delta=1e-6, max_iter=10**6, order=None, ms=None, no_zero=False):
    """Alg. 3 with one t* shared by all pairs, pairs taken one after another in `order` (default: index order).
    Returns (t*, number of pairs whose search started)."""
    lib = _load()
    V0, V1 = _c(V0, np.float64), _c(V1, np.float64)
    E, F = _c(E, np.int32).reshape(-1, 2), _c(F, np.int32).reshape(-1, 3)
    vf = _c(vf, np.int32).reshape(-1, 2)
    ee = _c(ee, np.int32).reshape(-1, 2)
    n = len(vf) + len(ee)
    if order is not None:
        order = _c(order, np.int64).reshape(-1)
        if len(order) != n or not np.array_equal(np.sort(order), np.arange(n)):
            raise ValueError("order must be a permutation of the pair indices")
    ms = _min_sep(ms, n)
    tmin = np.zeros(1, np.float64)
    nsr = np.zeros(1, np.int64)
    lib.oracle_narrow_global(_ptr(V0), _ptr(V1), _ptr(E), _ptr(F), _ptr(vf), len(vf), _ptr(ee), len(ee),
                             float(delta), int(max_iter), _ptr(ms), int(bool(no_zero)), _ptr(order), _ptr(tmin),
                             _ptr(nsr))
    return float(tmin[0]), int(nsr[0])


def initial_distance(V0, E, F, vf, ee):
    """Distance between the primitives of every pair at t = 0 (VF pairs first)."""
    lib = _load()
    V0 = _c(V0, np.float64)
    E, F = _c(E, np.int32).reshape(-1, 2), _c(F, np.int32).reshape(-1, 3)
    vf = _c(vf, np.int32).reshape(-1, 2)
    ee = _c(ee, np.int32).reshape(-1, 2)
    d0 = np.zeros(len(vf) + len(ee), np.float64)
    lib.oracle_initial_distance(_ptr(V0), _ptr(E), _ptr(F), _ptr(vf), len(vf), _ptr(ee), len(ee), _ptr(d0))
    return d0


def all_pairs(E, F, nv):
    """Every VF pair with v not in f and every EE pair e < g sharing no endpoint."""
    E = np.asarray(E, np.int64).reshape(-1, 2)
    F = np.asarray(F, np.int64).reshape(-1, 3)
    v = np.repeat(np.arange(nv), len(F))
    f = np.tile(np.arange(len(F)), nv)
    keep = (F[f, 0] != v) & (F[f, 1] != v) & (F[f, 2] != v)
    vf = np.stack([v[keep], f[keep]], 1).astype(np.int32)
    i, j = np.triu_indices(len(E), 1)
    share = ((E[i, 0] == E[j, 0]) | (E[i, 0] == E[j, 1]) | (E[i, 1] == E[j, 0]) | (E[i, 1] == E[j, 1]))
    ee = np.stack([i[~share], j[~share]], 1).astype(np.int32)
    return vf, ee
