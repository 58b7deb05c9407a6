"""Python binding of the MI355X (gfx950) conservative CCD library.

Argument marshalling only: every step of the broad and narrow phases runs in
the HIP kernels of libccd.so, reached through its C ABI (include/ccd.h).
PyTorch supplies device memory and the current HIP stream.  There is no CPU
fallback: importing works without the library, but every call raises if
libccd.so is missing or no GPU is present.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccd.so")

CCD_OK = 0
CCD_ERR_INVALID_ARG = -1
CCD_ERR_CAPACITY = -2
CCD_ERR_DEVICE = -3
CCD_ERR_OOM = -4
CCD_ERR_NONFINITE = -5

_STATUS_NAMES = {
    CCD_ERR_INVALID_ARG: "CCD_ERR_INVALID_ARG",
    CCD_ERR_CAPACITY: "CCD_ERR_CAPACITY",
    CCD_ERR_DEVICE: "CCD_ERR_DEVICE",
    CCD_ERR_OOM: "CCD_ERR_OOM",
    CCD_ERR_NONFINITE: "CCD_ERR_NONFINITE",
}

# Every symbol include/ccd.h declares.
EXPORTED = ["ccd_create", "ccd_destroy", "ccd_last_error", "ccd_version", "ccd_broad", "ccd_narrow",
            "ccd_narrow_sched", "ccd_detect", "ccd_features", "ccd_mlp_predict", "ccd_mlp_grad", "ccd_adam_step",
            "ccd_get_stats", "ccd_set_tuning", "ccd_get_tuning", "ccd_batch_create", "ccd_batch_destroy",
            "ccd_batch_run", "ccd_batch_autotune", "ccd_narrow_ex", "ccd_detect_ex", "ccd_initial_distance",
            "ccd_toi_step", "ccd_narrow_noalloc", "ccd_narrow_noalloc_max_pairs", "ccd_detect_budget"]

NUM_FEATURES = 16
HIDDEN = 64
MODEL_PARAMS = NUM_FEATURES * HIDDEN + HIDDEN + HIDDEN * HIDDEN + HIDDEN + HIDDEN + 1
SCHED_PLAIN, SCHED_LEARNED, SCHED_ORDER, SCHED_COST = 0, 1, 2, 3


class CCDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [("broad_ms", ctypes.c_double), ("box_ms", ctypes.c_double), ("sort_ms", ctypes.c_double),
                ("gather_ms", ctypes.c_double), ("sweep_ms", ctypes.c_double), ("narrow_ms", ctypes.c_double),
                ("narrow_prep_ms", ctypes.c_double), ("narrow_sched_ms", ctypes.c_double),
                ("narrow_pool_ms", ctypes.c_double),
                ("narrow_heavy_ms", ctypes.c_double),
                ("sort_axis", ctypes.c_int64), ("heavy_pairs", ctypes.c_int64),
                ("heavy_reruns", ctypes.c_int64), ("sched_heavy_pairs", ctypes.c_int64),
                ("batch_ms", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("sweep_tile_group", ctypes.c_int32), ("pool_blocks_per_cu", ctypes.c_int32),
                ("heavy_slots", ctypes.c_int32), ("heavy_cap_log2", ctypes.c_int32), ("heavy_lds", ctypes.c_int32),
                ("heavy_block", ctypes.c_int32), ("pool_wait", ctypes.c_int32), ("resume_block", ctypes.c_int32),
                ("resume_slots_per_cu", ctypes.c_int32), ("sweep_classes", ctypes.c_int32),
                ("pool_root_limit", ctypes.c_int32)]


class Schedule(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("params", ctypes.c_void_p), ("norm", ctypes.c_void_p),
                ("order", ctypes.c_void_p), ("heavy_threshold", ctypes.c_float), ("max_heavy", ctypes.c_int32),
                ("cost", ctypes.c_void_p)]


class NarrowOptions(ctypes.Structure):
    _fields_ = [("earliest_only", ctypes.c_int32), ("no_zero_toi", ctypes.c_int32), ("min_sep", ctypes.c_void_p),
                ("min_sep_d0_factor", ctypes.c_double)]


class BudgetResult(ctypes.Structure):
    _fields_ = [("n_vf", ctypes.c_int64), ("n_ee", ctypes.c_int64), ("n_hits", ctypes.c_int64),
                ("broad_batches", ctypes.c_int64), ("broad_splits", ctypes.c_int64),
                ("narrow_splits", ctypes.c_int64), ("pair_capacity", ctypes.c_int64),
                ("vf", ctypes.c_void_p), ("vf_cap", ctypes.c_int64), ("ee", ctypes.c_void_p),
                ("ee_cap", ctypes.c_int64), ("vf_hit", ctypes.c_void_p), ("ee_hit", ctypes.c_void_p),
                ("vf_toi", ctypes.c_void_p), ("ee_toi", ctypes.c_void_p)]


# Learned schedule defaults: predictions of log2(1 + n_enq) from which a pair starts in the wide stage, and
# the most such pairs (measured best on the cloth workload; the perturbed torus prefers 14 and 40,000).
HEAVY_THRESHOLD = 7.0
MAX_HEAVY = 256
TORUS_HEAVY_THRESHOLD = 14.0
TORUS_MAX_HEAVY = 40000


_lib = None


def load_library(path=LIB_PATH):
    """Load libccd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2112_06300_amd/build.py "
                           "(the CCD path has no CPU fallback)")
    # PyTorch ships its own HIP runtime under the same soname as the system's: whichever is loaded first
    # serves the whole process.  Loading torch first binds the library to the runtime its tensors and
    # streams belong to (loaded the other way round, torch finds no GPU).
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.ccd_create.argtypes = [ctypes.c_int, ctypes.POINTER(P)]
    lib.ccd_create.restype = ctypes.c_int
    lib.ccd_destroy.argtypes = [P]
    lib.ccd_destroy.restype = None
    lib.ccd_last_error.argtypes = []
    lib.ccd_last_error.restype = ctypes.c_char_p
    lib.ccd_version.argtypes = []
    lib.ccd_version.restype = ctypes.c_char_p
    lib.ccd_broad.argtypes = [P, P, P, i64, P, i64, P, i64, P, i64, ctypes.POINTER(i64), P, i64,
                              ctypes.POINTER(i64), P]
    lib.ccd_broad.restype = ctypes.c_int
    lib.ccd_narrow.argtypes = [P, P, P, i64, P, i64, P, i64, P, i64, P, i64, ctypes.c_double, i64,
                               P, P, P, P, P]
    lib.ccd_narrow.restype = ctypes.c_int
    lib.ccd_narrow_sched.argtypes = [P, P, P, i64, P, i64, P, i64, P, i64, P, i64, ctypes.c_double, i64,
                                     P, P, P, P, ctypes.POINTER(Schedule), P]
    lib.ccd_narrow_sched.restype = ctypes.c_int
    lib.ccd_detect.argtypes = [P, P, P, i64, P, i64, P, i64, P, i64, ctypes.POINTER(i64), P, i64, ctypes.POINTER(i64),
                               ctypes.c_double, i64, P, P, P, P, ctypes.POINTER(Schedule), P]
    lib.ccd_detect.restype = ctypes.c_int
    lib.ccd_features.argtypes = [P, P, P, i64, P, i64, P, i64, P, i64, P, i64, ctypes.c_double, P, P]
    lib.ccd_features.restype = ctypes.c_int
    lib.ccd_mlp_predict.argtypes = [P, P, P, P, i64, P, P]
    lib.ccd_mlp_predict.restype = ctypes.c_int
    lib.ccd_mlp_grad.argtypes = [P, P, P, P, P, i64, P, P, P]
    lib.ccd_mlp_grad.restype = ctypes.c_int
    f32 = ctypes.c_float
    lib.ccd_adam_step.argtypes = [P, P, P, P, P, i64, f32, f32, f32, f32, P]
    lib.ccd_adam_step.restype = ctypes.c_int
    lib.ccd_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    lib.ccd_set_tuning.restype = ctypes.c_int
    lib.ccd_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    lib.ccd_get_tuning.restype = ctypes.c_int
    lib.ccd_batch_create.argtypes = [P, i64, P, P, P, i64, i64, ctypes.POINTER(P)]
    lib.ccd_batch_create.restype = ctypes.c_int
    lib.ccd_batch_destroy.argtypes = [P]
    lib.ccd_batch_destroy.restype = None
    lib.ccd_batch_run.argtypes = [P, P, P, P, P, ctypes.c_double, i64, P, P, ctypes.POINTER(i64),
                                  ctypes.POINTER(i64), P, P, P, P, ctypes.c_int, P]
    lib.ccd_batch_run.restype = ctypes.c_int
    lib.ccd_batch_autotune.argtypes = [P, P, P, P, P, ctypes.c_double, i64, P, P, P, P, P, ctypes.c_char_p,
                                       ctypes.POINTER(Tuning), P]
    lib.ccd_batch_autotune.restype = ctypes.c_int
    lib.ccd_narrow_ex.argtypes = [P, P, P, i64, P, i64, P, i64, P, i64, P, i64, ctypes.c_double, i64,
                                  P, P, P, P, ctypes.POINTER(Schedule), ctypes.POINTER(NarrowOptions), P]
    lib.ccd_narrow_ex.restype = ctypes.c_int
    lib.ccd_detect_ex.argtypes = [P, P, P, i64, P, i64, P, i64, P, i64, ctypes.POINTER(i64), P, i64,
                                  ctypes.POINTER(i64), ctypes.c_double, i64, P, P, P, P, ctypes.POINTER(Schedule),
                                  ctypes.POINTER(NarrowOptions), P]
    lib.ccd_detect_ex.restype = ctypes.c_int
    lib.ccd_initial_distance.argtypes = [P, P, i64, P, i64, P, i64, P, i64, P, i64, P, P]
    lib.ccd_initial_distance.restype = ctypes.c_int
    lib.ccd_toi_step.argtypes = [P, P, P, i64, P, i64, P, i64, P, i64, ctypes.POINTER(i64), P, i64,
                                 ctypes.POINTER(i64), ctypes.c_double, i64, ctypes.c_double, ctypes.c_double,
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32), P]
    lib.ccd_toi_step.restype = ctypes.c_int
    lib.ccd_narrow_noalloc.argtypes = [P, P, P, i64, P, i64, P, i64, P, i64, P, i64, ctypes.c_double, i64,
                                       P, P, P, P, P]
    lib.ccd_narrow_noalloc.restype = ctypes.c_int
    lib.ccd_narrow_noalloc_max_pairs.argtypes = [P]
    lib.ccd_narrow_noalloc_max_pairs.restype = i64
    lib.ccd_detect_budget.argtypes = [P, P, P, i64, P, i64, P, i64, i64, ctypes.c_double, i64,
                                      ctypes.POINTER(NarrowOptions), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(BudgetResult), P]
    lib.ccd_detect_budget.restype = ctypes.c_int
    lib.ccd_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
    lib.ccd_get_stats.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status):
    if status != CCD_OK:
        raise CCDError(status, load_library().ccd_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _require(t, name, dtype, device, cols=None, rows=None, min_numel=None):
    """Check a tensor handed to the library as a raw pointer: a contiguous CUDA tensor of `dtype` on the
    context's device, with `cols` columns (2-D) and `rows` rows, or at least `min_numel` elements.  Raises
    ValueError instead of letting a kernel read or write outside it."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: expected dtype {dtype}, got {t.dtype}")
    if not t.is_cuda or t.device.index != device:
        raise ValueError(f"{name}: expected a tensor on cuda:{device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
        raise ValueError(f"{name}: expected shape (n, {cols}), got {tuple(t.shape)}")
    if rows is not None and t.shape[0] != rows:
        raise ValueError(f"{name}: expected {rows} rows, got {t.shape[0]}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name}: expected at least {min_numel} elements, got {t.numel()}")
    return t


def _require_scene(V0, V1, E, F, device):
    import torch
    _require(V0, "V0", torch.float64, device, cols=3)
    _require(V1, "V1", torch.float64, device, cols=3, rows=V0.shape[0])
    _require(E, "E", torch.int32, device, cols=2)
    _require(F, "F", torch.int32, device, cols=3)


def _dev(t, dtype, cols):
    import torch
    t = torch.as_tensor(t)
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        t = t.to(device="cuda", dtype=dtype).contiguous()
    return t.reshape(-1, cols)


class Context:
    """A library context on one GPU: owns the device scratch pool."""

    def __init__(self, device=0):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.ccd_create(int(device), ctypes.byref(h)))
        self._h = h
        self.device = int(device)

    def close(self):
        if getattr(self, "_h", None):
            load_library().ccd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_tuning(self, tuning=None):
        """Set launch-shape tuning from a dict (missing keys keep their current value); None restores defaults."""
        lib = load_library()
        if tuning is None:
            _check(lib.ccd_set_tuning(self._h, None))
            return
        t = Tuning()
        _check(lib.ccd_get_tuning(self._h, ctypes.byref(t)))
        for k, v in dict(tuning).items():
            setattr(t, k, int(v))
        _check(lib.ccd_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self):
        t = Tuning()
        _check(load_library().ccd_get_tuning(self._h, ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    def stats(self):
        st = Stats()
        _check(load_library().ccd_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in Stats._fields_}

    def broad(self, V0, V1, E, F, vf_cap=None, ee_cap=None, stream=None):
        """Candidate pairs (vf (n,2) int32, ee (m,2) int32) as CUDA tensors; order unspecified."""
        import torch
        lib = load_library()
        V0 = _dev(V0, torch.float64, 3)
        V1 = _dev(V1, torch.float64, 3)
        E = _dev(E, torch.int32, 2)
        F = _dev(F, torch.int32, 3)
        nb = V0.shape[0] + E.shape[0] + F.shape[0]
        vf_cap = int(vf_cap if vf_cap is not None else max(1024, 4 * nb))
        ee_cap = int(ee_cap if ee_cap is not None else max(1024, 4 * nb))
        for _ in range(2):
            vf = torch.empty((vf_cap, 2), dtype=torch.int32, device=V0.device)
            ee = torch.empty((ee_cap, 2), dtype=torch.int32, device=V0.device)
            n_vf = ctypes.c_int64()
            n_ee = ctypes.c_int64()
            st = lib.ccd_broad(self._h, _ptr(V0), _ptr(V1), V0.shape[0], _ptr(E), E.shape[0], _ptr(F), F.shape[0],
                               _ptr(vf), vf_cap, ctypes.byref(n_vf), _ptr(ee), ee_cap, ctypes.byref(n_ee),
                               _stream(stream))
            if st == CCD_ERR_CAPACITY:
                vf_cap = max(vf_cap, n_vf.value)
                ee_cap = max(ee_cap, n_ee.value)
                continue
            _check(st)
            return vf[:n_vf.value], ee[:n_ee.value]
        raise CCDError(CCD_ERR_CAPACITY, "broad phase output did not fit after resizing")

    def broad_into(self, V0, V1, E, F, vf, ee, stream=None):
        """Broad phase into preallocated outputs; returns (n_vf, n_ee) or raises CCDError."""
        import torch
        lib = load_library()
        _require_scene(V0, V1, E, F, self.device)
        _require(vf, "vf", torch.int32, self.device, cols=2)
        _require(ee, "ee", torch.int32, self.device, cols=2)
        n_vf = ctypes.c_int64()
        n_ee = ctypes.c_int64()
        st = lib.ccd_broad(self._h, _ptr(V0), _ptr(V1), V0.shape[0], _ptr(E), E.shape[0], _ptr(F), F.shape[0],
                           _ptr(vf), vf.shape[0], ctypes.byref(n_vf), _ptr(ee), ee.shape[0], ctypes.byref(n_ee),
                           _stream(stream))
        _check(st)
        return n_vf.value, n_ee.value

    def narrow(self, V0, V1, E, F, vf, ee, delta=1e-6, max_iter=10**6, with_costs=False, out=None, stream=None,
               schedule=None, options=None):
        """Per-pair (hit uint8, toi float64, toi_min (1,) float64, n_enq int64 or None), VF pairs first.

        schedule: None (plain: pairs in index order), ("learned", params, norm[, heavy_threshold, max_heavy]),
        ("cost", per-pair costs[, heavy_threshold, max_heavy]) or ("order", perm) -- where and in which order
        pairs are searched; the results are the same for every schedule.  options: None or a dict with earliest_only, no_zero_toi, min_sep (a CUDA float64 tensor,
        one per pair) and min_sep_d0_factor (see ccd_narrow_options)."""
        import torch
        lib = load_library()
        V0 = _dev(V0, torch.float64, 3)
        V1 = _dev(V1, torch.float64, 3)
        E = _dev(E, torch.int32, 2)
        F = _dev(F, torch.int32, 3)
        vf = _dev(vf, torch.int32, 2)
        ee = _dev(ee, torch.int32, 2)
        n = vf.shape[0] + ee.shape[0]
        if out is None:
            hit = torch.empty(n, dtype=torch.uint8, device=V0.device)
            toi = torch.empty(n, dtype=torch.float64, device=V0.device)
            tmin = torch.empty(1, dtype=torch.float64, device=V0.device)
            nenq = torch.empty(n, dtype=torch.int64, device=V0.device) if with_costs else None
        else:
            hit, toi, tmin, nenq = out
            _require(hit, "hit", torch.uint8, self.device, min_numel=n)
            _require(toi, "toi", torch.float64, self.device, min_numel=n)
            _require(tmin, "toi_min", torch.float64, self.device, min_numel=1)
            if nenq is not None:
                _require(nenq, "n_enq", torch.int64, self.device, min_numel=n)
        if options is not None:
            opt, okeep = _options(options, self.device, n)
            sch, keep = _schedule(schedule) if schedule is not None else (None, None)
            _check_schedule_len(sch, keep, n)
            _check(lib.ccd_narrow_ex(self._h, _ptr(V0), _ptr(V1), V0.shape[0], _ptr(E), E.shape[0], _ptr(F),
                                     F.shape[0], _ptr(vf), vf.shape[0], _ptr(ee), ee.shape[0], float(delta),
                                     int(max_iter), _ptr(hit), _ptr(toi), _ptr(tmin), _ptr(nenq),
                                     ctypes.byref(sch) if sch is not None else None, ctypes.byref(opt),
                                     _stream(stream)))
            del keep, okeep
            return hit, toi, tmin, nenq
        if schedule is None:
            _check(lib.ccd_narrow(self._h, _ptr(V0), _ptr(V1), V0.shape[0], _ptr(E), E.shape[0], _ptr(F),
                                  F.shape[0], _ptr(vf), vf.shape[0], _ptr(ee), ee.shape[0], float(delta),
                                  int(max_iter), _ptr(hit), _ptr(toi), _ptr(tmin), _ptr(nenq), _stream(stream)))
            return hit, toi, tmin, nenq
        sch, keep = _schedule(schedule)
        _check_schedule_len(sch, keep, n)
        _check(lib.ccd_narrow_sched(self._h, _ptr(V0), _ptr(V1), V0.shape[0], _ptr(E), E.shape[0], _ptr(F),
                                    F.shape[0], _ptr(vf), vf.shape[0], _ptr(ee), ee.shape[0], float(delta),
                                    int(max_iter), _ptr(hit), _ptr(toi), _ptr(tmin), _ptr(nenq),
                                    ctypes.byref(sch), _stream(stream)))
        del keep
        return hit, toi, tmin, nenq

    def narrow_noalloc(self, V0, V1, E, F, vf, ee, hit, toi, tmin, nenq=None, delta=1e-6, max_iter=10**6,
                       stream=None):
        """ccd_narrow into preallocated outputs without any device allocation by the library (its workspace is
        a fixed per-GPU array): for callers that cannot allocate.  Raises CCDError (CCD_ERR_CAPACITY above
        noalloc_max_pairs())."""
        import torch
        lib = load_library()
        _require_scene(V0, V1, E, F, self.device)
        _require(vf, "vf", torch.int32, self.device, cols=2)
        _require(ee, "ee", torch.int32, self.device, cols=2)
        n = vf.shape[0] + ee.shape[0]
        _require(hit, "hit", torch.uint8, self.device, min_numel=n)
        _require(toi, "toi", torch.float64, self.device, min_numel=n)
        _require(tmin, "toi_min", torch.float64, self.device, min_numel=1)
        if nenq is not None:
            _require(nenq, "n_enq", torch.int64, self.device, min_numel=n)
        _check(lib.ccd_narrow_noalloc(self._h, _ptr(V0), _ptr(V1), V0.shape[0], _ptr(E), E.shape[0], _ptr(F),
                                      F.shape[0], _ptr(vf), vf.shape[0], _ptr(ee), ee.shape[0], float(delta),
                                      int(max_iter), _ptr(hit), _ptr(toi), _ptr(tmin), _ptr(nenq), _stream(stream)))

    def noalloc_max_pairs(self):
        return int(load_library().ccd_narrow_noalloc_max_pairs(self._h))

    def detect_into(self, V0, V1, E, F, vf, ee, hit, toi, tmin, nenq=None, delta=1e-6, max_iter=10**6,
                    schedule=None, stream=None, options=None):
        """Broad and narrow phase in one call (one wait for the device, at the end).

        Pairs go into the preallocated vf (cap, 2) and ee (cap, 2); hit, toi and nenq (optional) hold
        vf.shape[0] + ee.shape[0] entries, of which the first n_vf + n_ee are written, VF pairs first.
        schedule: None (plain) or ("learned", params, norm[, heavy_threshold, max_heavy]).  Returns
        (n_vf, n_ee) or raises CCDError (CCD_ERR_CAPACITY when the pairs do not fit)."""
        import torch
        lib = load_library()
        _require_scene(V0, V1, E, F, self.device)
        _require(vf, "vf", torch.int32, self.device, cols=2)
        _require(ee, "ee", torch.int32, self.device, cols=2)
        n = vf.shape[0] + ee.shape[0]
        _require(hit, "hit", torch.uint8, self.device, min_numel=n)
        _require(toi, "toi", torch.float64, self.device, min_numel=n)
        _require(tmin, "toi_min", torch.float64, self.device, min_numel=1)
        if nenq is not None:
            _require(nenq, "n_enq", torch.int64, self.device, min_numel=n)
        n_vf = ctypes.c_int64()
        n_ee = ctypes.c_int64()
        sch, keep = _schedule(schedule) if schedule is not None else (None, None)
        if options is not None:
            if isinstance(options, dict) and options.get("min_sep") is not None:
                raise ValueError("detect takes min_sep_d0_factor, not per-pair min_sep (pairs are not known yet)")
            opt, okeep = _options(options, self.device, 0)
            _check(lib.ccd_detect_ex(self._h, _ptr(V0), _ptr(V1), V0.shape[0], _ptr(E), E.shape[0], _ptr(F),
                                     F.shape[0], _ptr(vf), vf.shape[0], ctypes.byref(n_vf), _ptr(ee), ee.shape[0],
                                     ctypes.byref(n_ee), float(delta), int(max_iter), _ptr(hit), _ptr(toi),
                                     _ptr(tmin), _ptr(nenq), ctypes.byref(sch) if sch is not None else None,
                                     ctypes.byref(opt), _stream(stream)))
            del okeep
        else:
            _check(lib.ccd_detect(self._h, _ptr(V0), _ptr(V1), V0.shape[0], _ptr(E), E.shape[0], _ptr(F),
                                  F.shape[0], _ptr(vf), vf.shape[0], ctypes.byref(n_vf), _ptr(ee), ee.shape[0],
                                  ctypes.byref(n_ee), float(delta), int(max_iter), _ptr(hit), _ptr(toi), _ptr(tmin),
                                  _ptr(nenq), ctypes.byref(sch) if sch is not None else None, _stream(stream)))
        del keep
        return n_vf.value, n_ee.value

    def detect_budget(self, V0, V1, E, F, budget_bytes, delta=1e-6, max_iter=10**6, options=None, vf_cap=0,
                      ee_cap=0, stream=None):
        """Broad + narrow phase within a device-memory budget (ccd_detect_budget).  Returns (toi_min, info) with
        info the counts and, when vf_cap / ee_cap > 0, host numpy arrays vf, ee, vf_hit, ee_hit, vf_toi, ee_toi
        of the first stored pairs (batch order)."""
        import numpy as np
        import torch
        lib = load_library()
        _require_scene(V0, V1, E, F, self.device)
        r = BudgetResult()
        keep = {}
        if vf_cap > 0:
            keep["vf"] = np.zeros((vf_cap, 2), np.int32)
            keep["vf_hit"] = np.zeros(vf_cap, np.uint8)
            keep["vf_toi"] = np.zeros(vf_cap, np.float64)
        if ee_cap > 0:
            keep["ee"] = np.zeros((ee_cap, 2), np.int32)
            keep["ee_hit"] = np.zeros(ee_cap, np.uint8)
            keep["ee_toi"] = np.zeros(ee_cap, np.float64)
        for k, a in keep.items():
            setattr(r, k, a.ctypes.data)
        r.vf_cap, r.ee_cap = int(vf_cap), int(ee_cap)
        opt, okeep = _options(options, self.device, 0) if options is not None else (None, None)
        t = ctypes.c_double()
        _check(lib.ccd_detect_budget(self._h, _ptr(V0), _ptr(V1), V0.shape[0], _ptr(E), E.shape[0], _ptr(F),
                                     F.shape[0], int(budget_bytes), float(delta), int(max_iter),
                                     ctypes.byref(opt) if opt is not None else None, ctypes.byref(t),
                                     ctypes.byref(r), _stream(stream)))
        info = {k: getattr(r, k) for k in ("n_vf", "n_ee", "n_hits", "broad_batches", "broad_splits",
                                           "narrow_splits", "pair_capacity")}
        kv, ke = min(r.n_vf, vf_cap), min(r.n_ee, ee_cap)
        for k, a in keep.items():
            info[k] = a[:kv] if k.startswith("vf") else a[:ke]
        return t.value, info

    def initial_distance(self, V0, E, F, vf, ee, stream=None):
        """d0 of every pair (distance of its primitives at t = 0), float64 on the device, VF pairs first."""
        import torch
        lib = load_library()
        V0 = _dev(V0, torch.float64, 3)
        E = _dev(E, torch.int32, 2)
        F = _dev(F, torch.int32, 3)
        vf = _dev(vf, torch.int32, 2)
        ee = _dev(ee, torch.int32, 2)
        d0 = torch.empty(vf.shape[0] + ee.shape[0], dtype=torch.float64, device=V0.device)
        _check(lib.ccd_initial_distance(self._h, _ptr(V0), V0.shape[0], _ptr(E), E.shape[0], _ptr(F), F.shape[0],
                                        _ptr(vf), vf.shape[0], _ptr(ee), ee.shape[0], _ptr(d0), _stream(stream)))
        return d0

    def toi_step(self, V0, V1, E, F, vf, ee, delta=1e-6, max_iter=10**6, ms_factor=0.2, scale=0.8, stream=None):
        """App. B's step size: (toi, rerun, n_vf, n_ee).  vf / ee are preallocated (cap, 2) int32 outputs."""
        import torch
        lib = load_library()
        _require(V0, "V0", torch.float64, self.device, cols=3)
        _require(V1, "V1", torch.float64, self.device, cols=3, rows=V0.shape[0])
        _require(E, "E", torch.int32, self.device, cols=2)
        _require(F, "F", torch.int32, self.device, cols=3)
        _require(vf, "vf", torch.int32, self.device, cols=2)
        _require(ee, "ee", torch.int32, self.device, cols=2)
        n_vf, n_ee = ctypes.c_int64(), ctypes.c_int64()
        t, rr = ctypes.c_double(), ctypes.c_int32()
        _check(lib.ccd_toi_step(self._h, _ptr(V0), _ptr(V1), V0.shape[0], _ptr(E), E.shape[0], _ptr(F), F.shape[0],
                                _ptr(vf), vf.shape[0], ctypes.byref(n_vf), _ptr(ee), ee.shape[0], ctypes.byref(n_ee),
                                float(delta), int(max_iter), float(ms_factor), float(scale), ctypes.byref(t),
                                ctypes.byref(rr), _stream(stream)))
        return t.value, bool(rr.value), n_vf.value, n_ee.value

    def features(self, V0, V1, E, F, vf, ee, delta=1e-6, stream=None):
        """Scheduling features, (n_vf + n_ee) x 16 float32 on the device, VF pairs first."""
        import torch
        lib = load_library()
        V0 = _dev(V0, torch.float64, 3)
        V1 = _dev(V1, torch.float64, 3)
        E = _dev(E, torch.int32, 2)
        F = _dev(F, torch.int32, 3)
        vf = _dev(vf, torch.int32, 2)
        ee = _dev(ee, torch.int32, 2)
        n = vf.shape[0] + ee.shape[0]
        feat = torch.empty((n, NUM_FEATURES), dtype=torch.float32, device=V0.device)
        _check(lib.ccd_features(self._h, _ptr(V0), _ptr(V1), V0.shape[0], _ptr(E), E.shape[0], _ptr(F), F.shape[0],
                                _ptr(vf), vf.shape[0], _ptr(ee), ee.shape[0], float(delta), _ptr(feat),
                                _stream(stream)))
        return feat

    def mlp_predict(self, params, norm, feat, out=None, stream=None):
        """Predicted log2(1 + n_enq) of every row of feat (float32 on the device)."""
        import torch
        lib = load_library()
        params, norm, feat = _f32(params, MODEL_PARAMS), _f32(norm, 2 * NUM_FEATURES), _dev(feat, torch.float32,
                                                                                          NUM_FEATURES)
        n = feat.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=feat.device)
        _check(lib.ccd_mlp_predict(self._h, _ptr(params), _ptr(norm), _ptr(feat), n, _ptr(out), _stream(stream)))
        return out

    def mlp_grad(self, params, norm, feat, label, grad=None, loss=None, stream=None):
        """(gradient of the mean squared error w.r.t. params, sum of squared errors (1,)), on the device."""
        import torch
        lib = load_library()
        params, norm = _f32(params, MODEL_PARAMS), _f32(norm, 2 * NUM_FEATURES)
        feat = _dev(feat, torch.float32, NUM_FEATURES)
        label = _dev(label, torch.float32, 1).reshape(-1)
        n = feat.shape[0]
        if label.shape[0] != n:
            raise ValueError("label and feat have different lengths")
        if grad is None:
            grad = torch.empty(MODEL_PARAMS, dtype=torch.float32, device=feat.device)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=feat.device)
        _check(lib.ccd_mlp_grad(self._h, _ptr(params), _ptr(norm), _ptr(feat), _ptr(label), n, _ptr(grad),
                                _ptr(loss), _stream(stream)))
        return grad, loss

    def adam_step(self, params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        """One in-place Adam step on params (device float32, MODEL_PARAMS values)."""
        for t in (params, grad, m, v):
            _require_f32(t, MODEL_PARAMS)
        _check(load_library().ccd_adam_step(self._h, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step),
                                            float(lr), float(beta1), float(beta2), float(eps), _stream(stream)))


class Batch:
    """Several scenes in CSR layout through one broad + narrow pass (see ccd_batch_run).

    v_off, e_off, f_off: S + 1 offsets each; V0/V1/E/F passed to run() are the concatenated scenes with
    global vertex ids.  The batch owns its pair and result buffers (sized by vf_cap / ee_cap), so repeated
    graph runs reuse one captured graph."""

    def __init__(self, ctx, v_off, e_off, f_off, vf_cap, ee_cap):
        import numpy as np
        import torch
        lib = load_library()
        self.ctx = ctx
        offs = [np.ascontiguousarray(np.asarray(o, dtype=np.int64)) for o in (v_off, e_off, f_off)]
        self.n_scenes = len(offs[0]) - 1
        if any(len(o) != self.n_scenes + 1 for o in offs):
            raise ValueError("offset arrays must have the same length")
        self.vf_cap, self.ee_cap = int(vf_cap), int(ee_cap)
        self.sizes = (int(offs[0][-1]), int(offs[1][-1]), int(offs[2][-1]))
        h = ctypes.c_void_p()
        _check(lib.ccd_batch_create(ctx.handle, self.n_scenes, offs[0].ctypes.data, offs[1].ctypes.data,
                                    offs[2].ctypes.data, self.vf_cap, self.ee_cap, ctypes.byref(h)))
        self._h = h
        dev = torch.device("cuda", ctx.device)
        cap = self.vf_cap + self.ee_cap
        self.vf = torch.empty((self.vf_cap, 2), dtype=torch.int32, device=dev)
        self.ee = torch.empty((self.ee_cap, 2), dtype=torch.int32, device=dev)
        self.hit = torch.empty(cap, dtype=torch.uint8, device=dev)
        self.toi = torch.empty(cap, dtype=torch.float64, device=dev)
        self.n_enq = torch.empty(cap, dtype=torch.int64, device=dev)
        self.toi_min = torch.empty(self.n_scenes, dtype=torch.float64, device=dev)

    def _check_inputs(self, V0, V1, E, F):
        _require_scene(V0, V1, E, F, self.ctx.device)
        if (V0.shape[0], E.shape[0], F.shape[0]) != self.sizes:
            raise ValueError(f"scene sizes {(V0.shape[0], E.shape[0], F.shape[0])} differ from the batch's "
                             f"offsets {self.sizes}")

    def close(self):
        if getattr(self, "_h", None):
            load_library().ccd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, V0, V1, E, F, delta=1e-6, max_iter=10**6, use_graph=True, with_costs=False, stream=None):
        """(vf, ee, hit, toi, toi_min, n_enq or None): views of the batch's buffers, valid until the next run."""
        lib = load_library()
        self._check_inputs(V0, V1, E, F)
        n_vf, n_ee = ctypes.c_int64(), ctypes.c_int64()
        st = lib.ccd_batch_run(self._h, _ptr(V0), _ptr(V1), _ptr(E), _ptr(F), float(delta), int(max_iter),
                               _ptr(self.vf), _ptr(self.ee), ctypes.byref(n_vf), ctypes.byref(n_ee), _ptr(self.hit),
                               _ptr(self.toi), _ptr(self.toi_min), _ptr(self.n_enq) if with_costs else None,
                               int(bool(use_graph)), _stream(stream))
        self.n_vf, self.n_ee = n_vf.value, n_ee.value
        _check(st)
        n = self.n_vf + self.n_ee
        return (self.vf[:self.n_vf], self.ee[:self.n_ee], self.hit[:n], self.toi[:n], self.toi_min,
                self.n_enq[:n] if with_costs else None)

    def autotune(self, V0, V1, E, F, delta=1e-6, max_iter=10**6, cache_path=None, stream=None):
        """Time candidate tunings, set the best on the context and return it (dict)."""
        lib = load_library()
        self._check_inputs(V0, V1, E, F)
        t = Tuning()
        _check(lib.ccd_batch_autotune(self._h, _ptr(V0), _ptr(V1), _ptr(E), _ptr(F), float(delta), int(max_iter),
                                      _ptr(self.vf), _ptr(self.ee), _ptr(self.hit), _ptr(self.toi),
                                      _ptr(self.toi_min), cache_path.encode() if cache_path else None,
                                      ctypes.byref(t), _stream(stream)))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}


def _f32(t, size):
    import torch
    t = torch.as_tensor(t)
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        t = t.to(device="cuda", dtype=torch.float32).contiguous()
    t = t.reshape(-1)
    if t.numel() != size:
        raise ValueError(f"expected {size} float32 values, got {t.numel()}")
    return t


def _require_f32(t, size):
    import torch
    if not (isinstance(t, torch.Tensor) and t.dtype == torch.float32 and t.is_cuda and t.is_contiguous()
            and t.numel() == size):
        raise ValueError(f"expected a contiguous CUDA float32 tensor of {size} values")


class PreparedSchedule:
    """A schedule converted once (ctypes struct and the device tensors it points into), for calls in a loop."""

    def __init__(self, schedule):
        self.sch, self.keep = _schedule(schedule)


def prepare_schedule(schedule):
    """Convert a schedule tuple once; pass the result wherever a schedule is taken."""
    return PreparedSchedule(schedule)


def _schedule(schedule):
    """ctypes Schedule for ("learned", params, norm) or ("order", perm); also the tensors it points into."""
    import torch
    if isinstance(schedule, PreparedSchedule):
        return schedule.sch, schedule.keep
    kind = schedule[0]
    if kind == "plain":
        return Schedule(SCHED_PLAIN, None, None, None, 0.0, 0, None), ()
    if kind == "learned":
        params, norm = _f32(schedule[1], MODEL_PARAMS), _f32(schedule[2], 2 * NUM_FEATURES)
        thr = float(schedule[3]) if len(schedule) > 3 else HEAVY_THRESHOLD
        mh = int(schedule[4]) if len(schedule) > 4 else MAX_HEAVY
        return Schedule(SCHED_LEARNED, params.data_ptr(), norm.data_ptr(), None, thr, mh, None), (params, norm)
    if kind == "order":
        perm = _dev(schedule[1], torch.int32, 1).reshape(-1)
        return Schedule(SCHED_ORDER, None, None, perm.data_ptr() if perm.numel() else None, 0.0, 0, None), (perm,)
    if kind == "cost":
        cost = _dev(schedule[1], torch.float32, 1).reshape(-1)
        thr = float(schedule[2]) if len(schedule) > 2 else HEAVY_THRESHOLD
        mh = int(schedule[3]) if len(schedule) > 3 else MAX_HEAVY
        return Schedule(SCHED_COST, None, None, None, thr, mh, cost.data_ptr() if cost.numel() else None), (cost,)
    raise ValueError(f"unknown schedule {kind!r}")


def _check_schedule_len(sch, keep, n):
    """An order or cost schedule holds exactly one entry per pair (the kernels read n of them)."""
    if sch is not None and sch.kind in (SCHED_ORDER, SCHED_COST) and keep[0].numel() != n:
        raise ValueError(f"schedule: expected {n} entries, one per pair, got {keep[0].numel()}")


def _options(options, device, n):
    """ctypes NarrowOptions from a dict (earliest_only, no_zero_toi, min_sep, min_sep_d0_factor)."""
    import torch
    o = dict(options)
    unknown = set(o) - {"earliest_only", "no_zero_toi", "min_sep", "min_sep_d0_factor"}
    if unknown:
        raise ValueError(f"unknown narrow-phase options {sorted(unknown)}")
    ms = o.get("min_sep")
    keep = ()
    ptr = None
    if ms is not None:
        _require(ms, "min_sep", torch.float64, device, min_numel=n)
        if ms.dim() != 1 or ms.numel() != n:
            raise ValueError(f"min_sep: expected {n} values, one per pair")
        ptr = ms.data_ptr() if n else None
        keep = (ms,)
    return NarrowOptions(int(bool(o.get("earliest_only", 0))), int(bool(o.get("no_zero_toi", 0))), ptr,
                         float(o.get("min_sep_d0_factor", 0.0))), keep


def version():
    return load_library().ccd_version().decode()
