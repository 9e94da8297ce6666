"""Python binding of libmase.so (include/mase.h): argument marshalling only.

Every computation runs in the HIP library; this module converts numpy arrays
and device pointers (ints or torch tensors) into C arguments and raises
MaseError on a non-zero return code.  There is no fallback: if the library
has not been built, loading it raises immediately.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmase.so")

MASE_VM, MASE_PINJ, MASE_QINJ, MASE_PF, MASE_QF, MASE_PT, MASE_QT = range(7)
MASE_OK, MASE_NOT_CONVERGED = 0, 1
MASE_ERR_ARG, MASE_ERR_STATE, MASE_ERR_NOT_POSDEF = -1, -2, -3
MASE_ERR_HIP, MASE_ERR_OOM, MASE_ERR_NO_DEVICE = -4, -5, -6
MASE_GAMMA_SPARSE, MASE_GAMMA_DENSE = 0, 1

INFO = {"n_gamma": 0, "n_boundary_bus": 1, "gamma_tail": 2, "nnz_factor": 3, "max_levels": 4,
        "flops_local": 5, "flops_gamma": 6, "bytes_assembly": 7, "n_snap": 8, "n_area": 9,
        "bytes_condense": 10, "flops_dense": 11, "bytes_backsolve": 12, "flops_gamma_sparse": 13,
        "gamma_levels": 14, "gamma_supernodes": 15, "gamma_supernodal": 16, "pipeline_groups": 17,
        "gamma_subtree_groups": 18, "gamma_dense_panel": 19, "area_lds": 20,
        "elim_threads": 21}
STAGES = ("assemble", "condense", "gamma_gather", "gamma_sparse", "gamma_dense", "gamma_back",
          "backsolve", "update", "local")
MAPS = {"boundary_flag": 0, "meas_area": 1, "gamma_vars": 2, "local_vars": 3,
        "n_internal": 4, "E": 5}

# Every symbol include/mase.h declares (checked by the CPU test suite).
SYMBOLS = (
    "mase_default_options", "mase_create", "mase_destroy", "mase_last_error", "mase_strerror",
    "mase_set_measurements", "mase_set_measurements_dev", "mase_set_state", "mase_set_state_dev",
    "mase_gn_iter", "mase_solve", "mase_solve_stream", "mase_solve_stream_host", "mase_stream_host_work",
    "mase_solve_stream_noalloc", "mase_stream_noalloc_max",
    "mase_state", "mase_state_dev", "mase_objective",
    "mase_eval_h_dev", "mase_info", "mase_export_map", "mase_export_pattern",
    "mase_stage_assemble", "mase_stage_condense", "mase_stage_gamma_assemble",
    "mase_stage_gamma_solve", "mase_stage_update", "mase_read_local_system", "mase_read_schur",
    "mase_read_gamma_system", "mase_read_step", "mase_profile", "mase_profile_read",
    "mase_mlp_create", "mase_mlp_destroy", "mase_mlp_info", "mase_mlp_io_map", "mase_mlp_set_params",
    "mase_mlp_get_params", "mase_mlp_set_norm", "mase_mlp_fit_norm", "mase_mlp_get_norm", "mase_mlp_loss_grad", "mase_mlp_train_step",
    "mase_mlp_predict_dev", "mase_warm_start", "mase_mlp_set_accept_cap", "mase_warm_start_objectives",
)


class MaseError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("batched", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("gamma_mode", ctypes.c_int32),
                ("host_only", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p), ("local_steps", ctypes.c_int32),
                ("pipeline_groups", ctypes.c_int32)]


_lib = None


def load():
    """Load libmase.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32p = ctypes.POINTER(ctypes.c_int32)
    f64p = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "mase_default_options": (None, [ctypes.POINTER(Options)]),
        "mase_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, i32p, i32p, f64p, f64p, f64p,
                                       ctypes.c_int32, ctypes.c_int32, i32p, ctypes.c_int32, i32p, i32p,
                                       f64p, ctypes.c_int32, ctypes.POINTER(Options),
                                       ctypes.POINTER(P)]),
        "mase_destroy": (None, [P]),
        "mase_last_error": (ctypes.c_char_p, []),
        "mase_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "mase_set_measurements": (ctypes.c_int, [P, f64p, f64p]),
        "mase_set_measurements_dev": (ctypes.c_int, [P, P, P]),
        "mase_set_state": (ctypes.c_int, [P, f64p, f64p]),
        "mase_set_state_dev": (ctypes.c_int, [P, P, P]),
        "mase_gn_iter": (ctypes.c_int, [P, f64p]),
        "mase_solve": (ctypes.c_int, [P, ctypes.c_double, ctypes.c_int32, i32p, i32p]),
        "mase_solve_stream": (ctypes.c_int, [P, P, P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                             P, P, i32p, i32p]),
        "mase_solve_stream_host": (ctypes.c_int, [P, P, P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                                  P, P, i32p, i32p, P, ctypes.c_int64]),
        "mase_stream_host_work": (ctypes.c_int64, [P, ctypes.c_int64, ctypes.c_int32]),
        "mase_solve_stream_noalloc": (ctypes.c_int, [P, P, P, P, ctypes.c_int64, ctypes.c_double,
                                                     ctypes.c_int32, P, P, i32p, i32p]),
        "mase_stream_noalloc_max": (ctypes.c_int64, [P]),
        "mase_state": (ctypes.c_int, [P, f64p, f64p]),
        "mase_state_dev": (ctypes.c_int, [P, P, P]),
        "mase_objective": (ctypes.c_int, [P, f64p]),
        "mase_eval_h_dev": (ctypes.c_int, [P, P, P, P]),
        "mase_info": (ctypes.c_int, [P, ctypes.c_int32, i64p]),
        "mase_export_map": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int32, i32p, ctypes.c_int64, i64p]),
        "mase_export_pattern": (ctypes.c_int, [P, ctypes.c_int32, i32p, i32p, ctypes.c_int64, i64p]),
        "mase_stage_assemble": (ctypes.c_int, [P]),
        "mase_stage_condense": (ctypes.c_int, [P]),
        "mase_stage_gamma_assemble": (ctypes.c_int, [P]),
        "mase_stage_gamma_solve": (ctypes.c_int, [P]),
        "mase_stage_update": (ctypes.c_int, [P, f64p]),
        "mase_read_local_system": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int32, f64p, f64p]),
        "mase_read_schur": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int32, f64p, f64p]),
        "mase_read_gamma_system": (ctypes.c_int, [P, ctypes.c_int32, f64p, f64p]),
        "mase_read_step": (ctypes.c_int, [P, ctypes.c_int32, f64p]),
        "mase_profile": (ctypes.c_int, [P, ctypes.c_int32]),
        "mase_profile_read": (ctypes.c_int, [P, f64p, i64p, i64p]),
        "mase_mlp_create": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(P)]),
        "mase_mlp_destroy": (None, [P]),
        "mase_mlp_info": (ctypes.c_int, [P, ctypes.c_int32, i32p, i32p, i64p]),
        "mase_mlp_io_map": (ctypes.c_int, [P, ctypes.c_int32, i32p, i32p]),
        "mase_mlp_set_params": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_float)]),
        "mase_mlp_get_params": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_float)]),
        "mase_mlp_set_norm": (ctypes.c_int, [P, f64p, f64p, f64p]),
        "mase_mlp_fit_norm": (ctypes.c_int, [P, P, P, P, ctypes.c_int32, f64p]),
        "mase_mlp_get_norm": (ctypes.c_int, [P, f64p, f64p, f64p]),
        "mase_mlp_loss_grad": (ctypes.c_int, [P, P, P, P, ctypes.c_int32, f64p, ctypes.POINTER(ctypes.c_float)]),
        "mase_mlp_train_step": (ctypes.c_int, [P, P, P, P, ctypes.c_int32, ctypes.c_float, f64p]),
        "mase_mlp_predict_dev": (ctypes.c_int, [P, P, ctypes.c_int32, P, P]),
        "mase_warm_start": (ctypes.c_int, [P, P, i32p]),
        "mase_mlp_set_accept_cap": (ctypes.c_int, [P, ctypes.c_double]),
        "mase_warm_start_objectives": (ctypes.c_int, [P, f64p, f64p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dptr(x):
    """Device pointer of a torch tensor (or an int)."""
    if x is None:
        return None
    if isinstance(x, int):
        return ctypes.c_void_p(x)
    return ctypes.c_void_p(x.data_ptr())


def _dev(x, shape, name, dtype="float64", min_rows=None):
    """Device pointer of a torch tensor after checking what the C call
    assumes: a contiguous tensor on a GPU with the given dtype and shape (-1
    matches any length; min_rows: at least that many rows).  A raw int
    pointer is passed unchecked; None stays None."""
    if x is None or isinstance(x, int):
        return _dptr(x)
    if not getattr(x, "is_cuda", False):
        raise ValueError(f"{name}: expected a GPU tensor")
    if str(x.dtype) != "torch." + dtype:
        raise ValueError(f"{name}: expected dtype {dtype}, got {x.dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    want = tuple(shape)
    got = tuple(x.shape)
    ok = len(got) == len(want) and all(w == -1 or w == g for w, g in zip(want, got))
    if ok and min_rows is not None:
        ok = got[0] >= min_rows
    if not ok:
        raise ValueError(f"{name}: expected shape {want}" + (f" with >= {min_rows} rows" if min_rows else "")
                         + f", got {got}")
    return _dptr(x)


def _check(rc, allow=(MASE_OK,)):
    if rc in allow:
        return rc
    msg = load().mase_last_error().decode()
    raise MaseError(rc, msg)


def mase_default_options():
    o = Options()
    load().mase_default_options(ctypes.byref(o))
    return o


def mase_create(n_bus, br_from, br_to, br_r, br_x, br_b, slack_bus, n_area, bus_area,
                meas_type, meas_at, meas_sigma, n_snap, opt=None):
    lib = load()
    f, fp = _i32(br_from)
    t, tp = _i32(br_to)
    r, rp = _f64(br_r)
    x, xp = _f64(br_x)
    b, bp = _f64(br_b)
    a, ap = _i32(bus_area)
    mt, mtp = _i32(meas_type)
    ma, map_ = _i32(meas_at)
    ms, msp = _f64(meas_sigma)
    out = ctypes.c_void_p()
    o = opt if opt is not None else mase_default_options()
    rc = lib.mase_create(int(n_bus), int(f.size), fp, tp, rp, xp, bp, int(slack_bus), int(n_area), ap,
                         int(mt.size), mtp, map_, msp, int(n_snap), ctypes.byref(o), ctypes.byref(out))
    _check(rc)
    return out


class Mase:
    """One context (mase_ctx*) with the C calls as methods of the same names."""

    def __init__(self, n_bus, br_from, br_to, br_r, br_x, br_b, slack_bus, n_area, bus_area,
                 meas_type, meas_at, meas_sigma, n_snap, batched=True, use_graph=True,
                 gamma_mode=MASE_GAMMA_SPARSE, host_only=False, stream=None, pipeline_groups=0,
                 autotune=False, tune_cache=None, local_steps=0):
        self.lib = load()
        o = mase_default_options()
        o.batched = int(bool(batched))
        o.use_graph = int(bool(use_graph))
        o.gamma_mode = int(gamma_mode)
        o.host_only = int(bool(host_only))
        o.pipeline_groups = int(pipeline_groups)
        o.local_steps = int(local_steps)
        o.autotune = int(bool(autotune))
        self._tune_cache = None if tune_cache is None else str(tune_cache).encode()
        o.tune_cache = self._tune_cache
        o.stream = stream
        self.n_bus = int(n_bus)
        self.n_meas = int(np.asarray(meas_type).size)
        self.n_snap = int(n_snap)
        self.n_area = int(n_area)
        self.slack = int(slack_bus)
        self.ctx = mase_create(n_bus, br_from, br_to, br_r, br_x, br_b, slack_bus, n_area, bus_area,
                               meas_type, meas_at, meas_sigma, n_snap, o)

    @classmethod
    def from_grid(cls, grid, meas_type, meas_at, meas_sigma, n_snap, slack=None, **kw):
        return cls(grid.n_bus, grid.br_from, grid.br_to, grid.br_r, grid.br_x, grid.br_b,
                   grid.slack if slack is None else slack, grid.n_area, grid.bus_area,
                   meas_type, meas_at, meas_sigma, n_snap, **kw)

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.lib.mase_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- measurements and state ----
    def mase_set_measurements(self, z, w=None):
        z, zp = _f64(z)
        assert z.size == self.n_snap * self.n_meas
        if w is not None:
            w, wp = _f64(w)
        else:
            wp = None
        _check(self.lib.mase_set_measurements(self.ctx, zp, wp))

    def mase_set_measurements_dev(self, z_dev, w_dev=None):
        _check(self.lib.mase_set_measurements_dev(self.ctx, _dev(z_dev, (self.n_snap, self.n_meas), "z_dev"),
                                                  _dev(w_dev, (self.n_meas,), "w_dev")))

    def mase_set_state(self, vm=None, va=None):
        if vm is None:
            _check(self.lib.mase_set_state(self.ctx, None, None))
            return
        vm, vp = _f64(vm)
        va, ap = _f64(va)
        assert vm.size == va.size == self.n_snap * self.n_bus
        _check(self.lib.mase_set_state(self.ctx, vp, ap))

    def mase_set_state_dev(self, vm_dev=None, va_dev=None):
        shp = (self.n_snap, self.n_bus)
        _check(self.lib.mase_set_state_dev(self.ctx, _dev(vm_dev, shp, "vm_dev"), _dev(va_dev, shp, "va_dev")))

    def mase_gn_iter(self):
        out = np.zeros(self.n_snap)
        _check(self.lib.mase_gn_iter(self.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def mase_solve(self, tol=1e-6, max_iter=10):
        iters = np.zeros(self.n_snap, dtype=np.int32)
        conv = np.zeros(self.n_snap, dtype=np.int32)
        rc = self.lib.mase_solve(self.ctx, float(tol), int(max_iter),
                                 iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 conv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        _check(rc, allow=(MASE_OK, MASE_NOT_CONVERGED))
        return iters, conv.astype(bool)

    def mase_solve_stream(self, z_dev, vm_out, va_out, vm0_dev=None, va0_dev=None, tol=1e-6, max_iter=10):
        """Solves the n_total snapshots of z_dev [n_total][n_meas] through the
        context's slots (continuous batching); states into vm_out / va_out
        [n_total][n_bus] (device).  Returns per-snapshot iterations and flags."""
        n_total = int(z_dev.shape[0])
        iters = np.zeros(n_total, dtype=np.int32)
        conv = np.zeros(n_total, dtype=np.int32)
        sb = (n_total, self.n_bus)
        zp = _dev(z_dev, (n_total, self.n_meas), "z_dev")
        v0, a0 = _dev(vm0_dev, sb, "vm0_dev"), _dev(va0_dev, sb, "va0_dev")
        vo, ao = _dev(vm_out, sb, "vm_out"), _dev(va_out, sb, "va_out")
        rc = self.lib.mase_solve_stream(self.ctx, zp, v0, a0, n_total,
                                        float(tol), int(max_iter), vo, ao,
                                        iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                        conv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        _check(rc, allow=(MASE_OK, MASE_NOT_CONVERGED))
        return iters, conv.astype(bool)

    def mase_solve_stream_noalloc(self, z_dev, vm_out, va_out, vm0_dev=None, va0_dev=None, tol=1e-6,
                                  max_iter=10):
        """mase_solve_stream that allocates no device memory (the stream's
        bookkeeping lives in the library's fixed scratch array); same
        arguments and results."""
        n_total = int(z_dev.shape[0])
        iters = np.zeros(n_total, dtype=np.int32)
        conv = np.zeros(n_total, dtype=np.int32)
        sb = (n_total, self.n_bus)
        zp = _dev(z_dev, (n_total, self.n_meas), "z_dev")
        v0, a0 = _dev(vm0_dev, sb, "vm0_dev"), _dev(va0_dev, sb, "va0_dev")
        vo, ao = _dev(vm_out, sb, "vm_out"), _dev(va_out, sb, "va_out")
        rc = self.lib.mase_solve_stream_noalloc(self.ctx, zp, v0, a0, n_total,
                                                float(tol), int(max_iter), vo, ao,
                                                iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                                conv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        _check(rc, allow=(MASE_OK, MASE_NOT_CONVERGED))
        return iters, conv.astype(bool)

    def mase_stream_noalloc_max(self):
        return int(self.lib.mase_stream_noalloc_max(self.ctx))

    def mase_stream_host_work(self, n_total, with_start=False):
        return int(self.lib.mase_stream_host_work(self.ctx, int(n_total), int(bool(with_start))))

    def mase_solve_stream_host(self, z_host, vm_out, va_out, work_dev, vm0_host=None, va0_host=None, tol=1e-6,
                               max_iter=10):
        """As mase_solve_stream with host buffers (torch CPU tensors, pinned
        for overlapped copies): z_host [n_total][n_meas] in, vm_out / va_out
        [n_total][n_bus] out; work_dev a float64 GPU tensor of at least
        mase_stream_host_work(n_total, ...) elements."""
        n_total = int(z_host.shape[0])
        sb = (n_total, self.n_bus)

        def host(x, shape, name):
            if x is None:
                return None
            if getattr(x, "is_cuda", False) or str(x.dtype) != "torch.float64" or not x.is_contiguous() \
                    or tuple(x.shape) != tuple(shape):
                raise ValueError(f"{name}: expected a contiguous float64 CPU tensor of shape {shape}")
            return ctypes.c_void_p(x.data_ptr())
        zp = host(z_host, (n_total, self.n_meas), "z_host")
        v0, a0 = host(vm0_host, sb, "vm0_host"), host(va0_host, sb, "va0_host")
        vo, ao = host(vm_out, sb, "vm_out"), host(va_out, sb, "va_out")
        need = self.mase_stream_host_work(n_total, vm0_host is not None)
        wp = _dev(work_dev, (-1,), "work_dev", min_rows=need)
        iters = np.zeros(n_total, dtype=np.int32)
        conv = np.zeros(n_total, dtype=np.int32)
        rc = self.lib.mase_solve_stream_host(self.ctx, zp, v0, a0, n_total, float(tol), int(max_iter), vo, ao,
                                             iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                             conv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                             wp, int(work_dev.numel()) if work_dev is not None else 0)
        _check(rc, allow=(MASE_OK, MASE_NOT_CONVERGED))
        return iters, conv.astype(bool)

    def mase_state(self):
        vm = np.zeros((self.n_snap, self.n_bus))
        va = np.zeros((self.n_snap, self.n_bus))
        _check(self.lib.mase_state(self.ctx, vm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   va.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return vm, va

    def mase_state_dev(self, vm_dev, va_dev):
        shp = (self.n_snap, self.n_bus)
        _check(self.lib.mase_state_dev(self.ctx, _dev(vm_dev, shp, "vm_dev"), _dev(va_dev, shp, "va_dev")))

    def mase_objective(self):
        J = np.zeros(self.n_snap)
        _check(self.lib.mase_objective(self.ctx, J.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return J

    def mase_eval_h_dev(self, vm_dev, va_dev, h_dev):
        shp = (self.n_snap, self.n_bus)
        _check(self.lib.mase_eval_h_dev(self.ctx, _dev(vm_dev, shp, "vm_dev"), _dev(va_dev, shp, "va_dev"),
                                        _dev(h_dev, (self.n_snap, self.n_meas), "h_dev")))

    # ---- per-stage timing ----
    def mase_profile(self, enable=True):
        _check(self.lib.mase_profile(self.ctx, int(bool(enable))))

    def mase_profile_read(self):
        n = len(STAGES)
        ms = np.zeros(n)
        la = np.zeros(n, dtype=np.int64)
        un = np.zeros(n, dtype=np.int64)
        _check(self.lib.mase_profile_read(self.ctx, ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          la.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                          un.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return {STAGES[i]: {"ms": float(ms[i]), "launches": int(la[i]), "units": int(un[i])}
                for i in range(n)}

    # ---- structure ----
    def mase_info(self, key):
        v = ctypes.c_int64()
        _check(self.lib.mase_info(self.ctx, INFO[key] if isinstance(key, str) else int(key),
                                  ctypes.byref(v)))
        return int(v.value)

    def mase_export_map(self, kind, area=0):
        k = MAPS[kind] if isinstance(kind, str) else int(kind)
        n = ctypes.c_int64()
        self.lib.mase_export_map(self.ctx, k, int(area), None, 0, ctypes.byref(n))
        buf = np.zeros(max(1, n.value), dtype=np.int32)
        _check(self.lib.mase_export_map(self.ctx, k, int(area),
                                        buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                        buf.size, ctypes.byref(n)))
        return buf[:n.value]

    def mase_export_pattern(self, area):
        n = ctypes.c_int64()
        nloc = self.mase_export_map("local_vars", area).size
        self.lib.mase_export_pattern(self.ctx, int(area), None, None, 0, ctypes.byref(n))
        rp = np.zeros(nloc + 1, dtype=np.int32)
        ci = np.zeros(max(1, n.value), dtype=np.int32)
        _check(self.lib.mase_export_pattern(self.ctx, int(area),
                                            rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            ci.size, ctypes.byref(n)))
        return rp, ci[:n.value]

    # ---- stages and debug reads ----
    def mase_stage_assemble(self):
        _check(self.lib.mase_stage_assemble(self.ctx))

    def mase_stage_condense(self):
        _check(self.lib.mase_stage_condense(self.ctx))

    def mase_stage_gamma_assemble(self):
        _check(self.lib.mase_stage_gamma_assemble(self.ctx))

    def mase_stage_gamma_solve(self):
        _check(self.lib.mase_stage_gamma_solve(self.ctx))

    def mase_stage_update(self):
        out = np.zeros(self.n_snap)
        _check(self.lib.mase_stage_update(self.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def mase_read_local_system(self, snap, area):
        n = self.mase_export_map("local_vars", area).size
        G = np.zeros((n, n))
        b = np.zeros(n)
        _check(self.lib.mase_read_local_system(self.ctx, int(snap), int(area),
                                               G.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                               b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return G, b

    def mase_read_schur(self, snap, area):
        n = self.mase_export_map("E", area).size
        S = np.zeros((n, n))
        b = np.zeros(n)
        _check(self.lib.mase_read_schur(self.ctx, int(snap), int(area),
                                        S.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return S, b

    def mase_read_gamma_system(self, snap):
        n = self.mase_info("n_gamma")
        S = np.zeros((max(n, 1), max(n, 1)))
        b = np.zeros(max(n, 1))
        _check(self.lib.mase_read_gamma_system(self.ctx, int(snap),
                                               S.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                               b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return S[:n, :n], b[:n]

    def mase_read_step(self, snap):
        dx = np.zeros(2 * self.n_bus)
        _check(self.lib.mase_read_step(self.ctx, int(snap), dx.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return dx


class Mlp:
    """Per-area warm-start networks of one context (mase_mlp*)."""

    def __init__(self, ctx: "Mase", hidden=256, max_batch=256):
        self.lib = load()
        self.owner = ctx
        self.hidden = int(hidden)
        self.h = ctypes.c_void_p()
        _check(self.lib.mase_mlp_create(ctx.ctx, int(hidden), int(max_batch), ctypes.byref(self.h)))
        n_in, n_out, n_param = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(self.lib.mase_mlp_info(self.h, -1, ctypes.byref(n_in), ctypes.byref(n_out), ctypes.byref(n_param)))
        self.n_param = int(n_param.value)
        self.n_out = int(n_out.value)
        self.shapes, self.in_meas, self.out_var = [], [], []
        for k in range(ctx.n_area):
            _check(self.lib.mase_mlp_info(self.h, k, ctypes.byref(n_in), ctypes.byref(n_out), None))
            mi = np.zeros(n_in.value, dtype=np.int32)
            ov = np.zeros(n_out.value, dtype=np.int32)
            _check(self.lib.mase_mlp_io_map(self.h, k, mi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            ov.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
            self.in_meas.append(mi)
            self.out_var.append(ov)
            self.shapes.append((int(n_in.value), self.hidden, int(n_out.value)))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.mase_mlp_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _io(self, z_dev, vm_dev, va_dev, batch):
        o = self.owner
        return (_dev(z_dev, (-1, o.n_meas), "z_dev", min_rows=int(batch)),
                _dev(vm_dev, (-1, o.n_bus), "vm_dev", min_rows=int(batch)),
                _dev(va_dev, (-1, o.n_bus), "va_dev", min_rows=int(batch)))

    def mase_mlp_set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == self.n_param
        _check(self.lib.mase_mlp_set_params(self.h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def mase_mlp_get_params(self):
        p = np.zeros(self.n_param, dtype=np.float32)
        _check(self.lib.mase_mlp_get_params(self.h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return p

    def mase_mlp_set_norm(self, z_mean, y_mean, y_std):
        zm, zp = _f64(z_mean)
        ym, yp = _f64(y_mean)
        ys, sp = _f64(y_std)
        _check(self.lib.mase_mlp_set_norm(self.h, zp, yp, sp))

    def mase_mlp_fit_norm(self, z_dev, vm_dev, va_dev):
        """Normalisation statistics of the training set (device tensors z
        [n][n_meas], vm / va [n][n_bus]) computed and set by the library;
        returns the per-area RMS of the normalised inputs."""
        n = int(z_dev.shape[0])
        zp = _dev(z_dev, (n, self.owner.n_meas), "z_dev")
        vp = _dev(vm_dev, (n, self.owner.n_bus), "vm_dev")
        ap = _dev(va_dev, (n, self.owner.n_bus), "va_dev")
        rms = np.zeros(self.owner.n_area)
        _check(self.lib.mase_mlp_fit_norm(self.h, zp, vp, ap, n, rms.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return rms

    def mase_mlp_get_norm(self):
        z_mean = np.zeros(self.owner.n_meas)
        y_mean = np.zeros(2 * self.owner.n_bus)
        y_std = np.zeros(2 * self.owner.n_bus)
        f = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
        _check(self.lib.mase_mlp_get_norm(self.h, f(z_mean), f(y_mean), f(y_std)))
        return z_mean, y_mean, y_std

    def mase_mlp_loss_grad(self, z_dev, vm_dev, va_dev, batch, want_grad=True):
        loss = ctypes.c_double()
        g = np.zeros(self.n_param, dtype=np.float32) if want_grad else None
        zp, vp, ap = self._io(z_dev, vm_dev, va_dev, batch)
        _check(self.lib.mase_mlp_loss_grad(self.h, zp, vp, ap, int(batch),
                                           ctypes.byref(loss),
                                           g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if want_grad else None))
        return float(loss.value), g

    def mase_mlp_train_step(self, z_dev, vm_dev, va_dev, batch, lr, want_loss=False):
        loss = ctypes.c_double()
        zp, vp, ap = self._io(z_dev, vm_dev, va_dev, batch)
        _check(self.lib.mase_mlp_train_step(self.h, zp, vp, ap, int(batch),
                                            float(lr), ctypes.byref(loss) if want_loss else None))
        return float(loss.value) if want_loss else None

    def mase_mlp_predict_dev(self, z_dev, batch, vm_dev, va_dev):
        zp, vp, ap = self._io(z_dev, vm_dev, va_dev, batch)
        _check(self.lib.mase_mlp_predict_dev(self.h, zp, int(batch), vp, ap))

    def mase_mlp_set_accept_cap(self, j_cap):
        _check(self.lib.mase_mlp_set_accept_cap(self.h, float(j_cap)))

    def mase_warm_start_objectives(self):
        n = self.owner.n_snap
        jp, jf = np.zeros(n), np.zeros(n)
        _check(self.lib.mase_warm_start_objectives(self.h, jp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                   jf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return jp, jf


def mase_warm_start(ctx: Mase, mlp: Mlp):
    """Warm start of ctx's snapshots from mlp; returns the accepted flags."""
    acc = np.zeros(ctx.n_snap, dtype=np.int32)
    _check(load().mase_warm_start(ctx.ctx, mlp.h, acc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return acc.astype(bool)
