"""ctypes binding of libstm.so (include/stm.h).  Argument marshalling only:
every step of the matching runs in the library's HIP kernels.

Point sets are any objects with `xy` [n,2] float32, `t` [n] int32, `desc`
[n,dim] float32 and (scenes) `n_frames`.  numpy arrays give a synchronous
host-pointer call; torch CUDA tensors (see `DevicePoints`) give a call on the
current torch stream with device outputs.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libstm.so")

STM_OK, STM_EINVAL, STM_ENOMEM, STM_EHIP, STM_EUNSUPPORTED = 0, -1, -2, -3, -4
STM_K_LIMIT = 64
STM_DEVICE_PTRS = 0x1
STM_UNARY_BF16 = 0x2
STM_K_DENSITY = 0x4
STM_DUMMY = 0x8
STM_CLOSENESS_SPAN = 0x10
STM_TRELLIS_STEPWISE = 0x20  # trellis: one launch per step even where the band fits LDS
STM_ANGLE_UNSIGNED = 0x40  # triangle angles read as magnitudes (params.angle_unsigned)
STM_CAUSAL_NODE = 0x80  # causality as increasing scene node ids (params.causal_node)
STM_DUMMY_NODE = -2  # assignment value of a dummy (unmatched model point)
STM_UNCHAINED_NODE = -3  # assignment value of a point in no kept chain (stm_match_chains)
STM_NOALLOC_SCRATCH_BYTES = 256 << 20  # fixed device array of stm_match_noalloc

EXPORTS = ("stm_create", "stm_destroy", "stm_last_error", "stm_offsets", "stm_match",
           "stm_candidates", "stm_unary", "stm_count_work", "stm_set_dp_waves",
           "stm_profile_enable", "stm_profile_read", "stm_plan_create", "stm_plan_destroy",
           "stm_plan_rows", "stm_plan_run", "stm_plan_set_tuning", "stm_plan_set_shape",
           "stm_plan_get_shape", "stm_plan_autotune",
           "stm_match_batch", "stm_pruner_num_params", "stm_pruner_create", "stm_pruner_destroy",
           "stm_pruner_set_params", "stm_pruner_get_params", "stm_pruner_save", "stm_pruner_load",
           "stm_pruner_features", "stm_pruner_gradient", "stm_pruner_train_step", "stm_pruner_infer",
           "stm_match_pruned", "stm_match_lists", "stm_pruner_set_rule", "stm_plan_run_pruned",
           "stm_match_chains", "stm_plan_run_lists", "stm_match_noalloc", "stm_trellis_create",
           "stm_trellis_destroy", "stm_trellis_run", "stm_trellis_info", "stm_match_trellis")


class StmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"stm error {code}: {msg}")
        self.code = code


class _Points(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("dim", ctypes.c_int32), ("n_frames", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("xy", ctypes.c_void_p), ("t", ctypes.c_void_p),
                ("desc", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("lambda1", ctypes.c_double), ("lambda2", ctypes.c_double),
                ("lambda3", ctypes.c_double), ("T", ctypes.c_int32), ("window", ctypes.c_int32),
                ("k_max", ctypes.c_int32), ("flags", ctypes.c_uint32), ("w_dummy", ctypes.c_double)]


_lib = None


def load() -> ctypes.CDLL:
    """Loads libstm.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1505_00581_amd.build` (no CPU fallback exists)")
        # torch first: its HIP runtime (soname libamdhip64.so.7) is then the one
        # libstm.so binds to, so the process holds a single runtime whichever
        # module touches the GPU first
        import torch  # noqa: F401
        lib = ctypes.CDLL(LIB_PATH)
        P, i32 = ctypes.c_void_p, ctypes.c_int32
        lib.stm_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
        lib.stm_destroy.argtypes = [P]
        lib.stm_destroy.restype = None
        lib.stm_last_error.restype = ctypes.c_char_p
        lib.stm_offsets.argtypes = [P, ctypes.POINTER(_Points), ctypes.POINTER(_Points),
                                    ctypes.c_uint32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        lib.stm_match.argtypes = [P, ctypes.POINTER(_Points), ctypes.POINTER(_Points),
                                  ctypes.POINTER(_Params), i32, i32, P, P, P, P, P]
        lib.stm_candidates.argtypes = [P, ctypes.POINTER(_Points), ctypes.POINTER(_Points),
                                       ctypes.POINTER(_Params), i32, i32, P, P, P]
        lib.stm_unary.argtypes = [P, ctypes.POINTER(_Points), ctypes.POINTER(_Points),
                                  ctypes.POINTER(_Params), P, P]
        lib.stm_count_work.argtypes = [P, ctypes.POINTER(_Points), ctypes.POINTER(_Points),
                                       ctypes.POINTER(_Params), i32, i32, P, P]
        lib.stm_set_dp_waves.argtypes = [P, ctypes.c_int]
        lib.stm_plan_create.argtypes = [P, P, i32, P, i32, P, i32, ctypes.POINTER(_Params),
                                        ctypes.POINTER(P)]
        lib.stm_plan_destroy.argtypes = [P]
        lib.stm_plan_destroy.restype = None
        lib.stm_plan_rows.argtypes = [P, P, P, P, P]
        lib.stm_plan_run.argtypes = [P, P, P, P, P, P]
        lib.stm_plan_set_tuning.argtypes = [P, i32, i32]
        lib.stm_plan_set_shape.argtypes = [P, P]
        lib.stm_plan_get_shape.argtypes = [P, P]
        lib.stm_plan_autotune.argtypes = [P, ctypes.c_char_p, i32, P]
        lib.stm_match_batch.argtypes = [P, P, i32, P, i32, P, i32, ctypes.POINTER(_Params), P, P, P,
                                        P, P]
        lib.stm_profile_enable.argtypes = [P, ctypes.c_int]
        lib.stm_profile_read.argtypes = [P, P, P, P]
        PP, PS = ctypes.POINTER(_Points), ctypes.POINTER(_Params)
        lib.stm_pruner_num_params.argtypes = [i32]
        lib.stm_pruner_num_params.restype = ctypes.c_int64
        lib.stm_pruner_create.argtypes = [P, i32, ctypes.POINTER(P)]
        lib.stm_pruner_destroy.argtypes = [P]
        lib.stm_pruner_destroy.restype = None
        lib.stm_pruner_set_params.argtypes = [P, P, ctypes.c_int64]
        lib.stm_pruner_get_params.argtypes = [P, P, ctypes.c_int64]
        lib.stm_pruner_save.argtypes = [P, ctypes.c_char_p]
        lib.stm_pruner_load.argtypes = [P, ctypes.c_char_p]
        lib.stm_pruner_features.argtypes = [P, PP, PP, PS, P, i32, P, P, P, P]
        lib.stm_pruner_gradient.argtypes = [P, PP, PP, PS, P, P, i32, P, P, P, P]
        lib.stm_pruner_train_step.argtypes = [P, PP, PP, PS, P, P, i32, ctypes.c_float, P, P]
        lib.stm_pruner_infer.argtypes = [P, PP, PP, PS, P, i32, i32, P, P, P, P]
        lib.stm_match_pruned.argtypes = [P, P, PP, PP, PS, i32, i32, i32, P, P, P, P, P, P]
        lib.stm_match_lists.argtypes = [P, PP, PP, PS, i32, i32, P, P, i32, P, P, P, P, P]
        lib.stm_pruner_set_rule.argtypes = [P, i32]
        lib.stm_plan_run_pruned.argtypes = [P, P, i32, P, P, P, P, P, P]
        lib.stm_match_chains.argtypes = [P, PP, P, i32, PP, PS, i32, i32, P, P, P, P, P, P]
        lib.stm_plan_run_lists.argtypes = [P, P, P, i32, P, P, P, P, P]
        lib.stm_match_noalloc.argtypes = [P, PP, PP, PS, i32, i32, P, P, P, P, P]
        lib.stm_trellis_create.argtypes = [P, P, i32, PP, i32, i32, PS, ctypes.POINTER(P)]
        lib.stm_trellis_destroy.argtypes = [P]
        lib.stm_trellis_destroy.restype = None
        lib.stm_trellis_run.argtypes = [P, P, P, P, P, P]
        lib.stm_trellis_info.argtypes = [P, P]
        lib.stm_match_trellis.argtypes = [P, P, i32, PP, i32, i32, PS, P, P, P, P, P]
        for name in ("stm_create", "stm_offsets", "stm_match", "stm_candidates", "stm_unary",
                     "stm_count_work", "stm_set_dp_waves", "stm_profile_enable",
                     "stm_profile_read", "stm_plan_create", "stm_plan_rows", "stm_plan_run",
                     "stm_plan_set_tuning", "stm_plan_set_shape", "stm_plan_get_shape", "stm_plan_autotune", "stm_match_batch",
                     "stm_pruner_create", "stm_pruner_set_params", "stm_pruner_get_params",
                     "stm_pruner_save", "stm_pruner_load", "stm_pruner_features",
                     "stm_pruner_gradient", "stm_pruner_train_step", "stm_pruner_infer",
                     "stm_match_pruned", "stm_match_lists", "stm_pruner_set_rule", "stm_plan_run_pruned",
                     "stm_match_chains", "stm_plan_run_lists", "stm_match_noalloc", "stm_trellis_create",
                     "stm_trellis_run", "stm_trellis_info", "stm_match_trellis"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != STM_OK:
        raise StmError(rc, load().stm_last_error().decode())


@dataclasses.dataclass
class DevicePoints:
    """A point set resident in device memory (torch CUDA tensors)."""

    xy: "object"
    t: "object"
    desc: "object"
    n_frames: int = 0

    @staticmethod
    def from_host(p, device="cuda"):
        import torch
        return DevicePoints(torch.as_tensor(np.ascontiguousarray(p.xy, np.float32), device=device),
                            torch.as_tensor(np.ascontiguousarray(p.t, np.int32), device=device),
                            torch.as_tensor(np.ascontiguousarray(p.desc, np.float32), device=device),
                            int(getattr(p, "n_frames", 0)))


def _is_device(p) -> bool:
    return isinstance(p, DevicePoints)


def _ptr(a) -> int:
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _points(p, keep: list) -> _Points:
    if _is_device(p):
        xy, t, d = p.xy.contiguous(), p.t.contiguous(), p.desc.contiguous()
        assert str(xy.dtype) == "torch.float32" and str(t.dtype) == "torch.int32"
    else:
        xy = np.ascontiguousarray(p.xy, np.float32)
        t = np.ascontiguousarray(p.t, np.int32)
        d = np.ascontiguousarray(p.desc, np.float32)
    keep += [xy, t, d]
    n, dim = int(t.shape[0]), int(d.shape[1])
    return _Points(n, dim, int(getattr(p, "n_frames", 0)), 0, _ptr(xy), _ptr(t), _ptr(d))


def _params(params, device: bool) -> _Params:
    wd = getattr(params, "w_dummy", None)
    flags = ((STM_DEVICE_PTRS if device else 0) | (STM_K_DENSITY if params.k_density else 0)
             | (STM_UNARY_BF16 if getattr(params, "unary_bf16", False) else 0)
             | (STM_DUMMY if wd is not None else 0)
             | (STM_CLOSENESS_SPAN if getattr(params, "closeness_span", False) else 0)
             | (STM_ANGLE_UNSIGNED if getattr(params, "angle_unsigned", False) else 0)
             | (STM_CAUSAL_NODE if getattr(params, "causal_node", False) else 0))
    return _Params(params.lambda1, params.lambda2, params.lambda3, params.T, params.window,
                   params.k_max, flags, 0.0 if wd is None else float(wd))


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


class Context:
    """Owns a libstm context (device scratch).  Device calls are queued on the
    current torch stream."""

    def __init__(self, device: int = 0):
        self._lib = load()
        h = ctypes.c_void_p()
        _check(self._lib.stm_create(ctypes.byref(h), device))
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            self._lib.stm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- offsets ----------------------------------------------------------------
    def offsets(self, model, scene) -> tuple:
        keep = []
        pm, ps = _points(model, keep), _points(scene, keep)
        b, e = ctypes.c_int32(), ctypes.c_int32()
        flags = STM_DEVICE_PTRS if _is_device(model) else 0
        _check(self._lib.stm_offsets(self.handle, ctypes.byref(pm), ctypes.byref(ps), flags,
                                     ctypes.byref(b), ctypes.byref(e)))
        return b.value, e.value

    def _range(self, model, scene, tau_begin, tau_end):
        if tau_begin is None or tau_end is None:
            b, e = self.offsets(model, scene)
            tau_begin = b if tau_begin is None else tau_begin
            tau_end = e if tau_end is None else tau_end
        return int(tau_begin), int(tau_end)

    # -- the exact matching -------------------------------------------------------
    def match(self, model, scene, params, tau_begin=None, tau_end=None, out=None):
        """Exact optimum at every offset in [tau_begin, tau_end) (default: all).

        Returns dict(energy32, energy64, energy_u64, assign, tau_begin, tau_end);
        numpy arrays for host inputs, torch tensors for DevicePoints (then the
        work is queued on the current torch stream and this returns after the
        input validation)."""
        b, e = self._range(model, scene, tau_begin, tau_end)
        n, M = e - b, int(model.t.shape[0])
        keep = []
        pm, ps = _points(model, keep), _points(scene, keep)
        dev = _is_device(model)
        if dev:
            import torch
            d = model.xy.device
            if out is None:
                out = dict(energy32=torch.empty(n, dtype=torch.float32, device=d),
                           energy64=torch.empty(n, dtype=torch.float64, device=d),
                           energy_u64=torch.empty(n, dtype=torch.float64, device=d),
                           assign=torch.empty((n, M), dtype=torch.int32, device=d))
            stream = _stream()
        else:
            out = dict(energy32=np.empty(n, np.float32), energy64=np.empty(n, np.float64),
                       energy_u64=np.empty(n, np.float64), assign=np.empty((n, M), np.int32))
            stream = None
        pp = _params(params, dev)
        _check(self._lib.stm_match(self.handle, ctypes.byref(pm), ctypes.byref(ps),
                                   ctypes.byref(pp), b, e, _ptr(out["energy32"]),
                                   _ptr(out["energy64"]), _ptr(out["energy_u64"]),
                                   _ptr(out["assign"]), stream))
        out["tau_begin"], out["tau_end"] = b, e
        return out

    def match_noalloc(self, model, scene, params, tau_begin=None, tau_end=None, out=None):
        """stm_match_noalloc: the exact matching on the library's fixed device
        array (no device allocation by the library).  DevicePoints only; the
        outputs are torch tensors (`out`, or new ones)."""
        if not _is_device(model) or not _is_device(scene):
            raise TypeError("match_noalloc takes DevicePoints (device pointers only)")
        import torch
        b, e = self._range(model, scene, tau_begin, tau_end)
        n, M = e - b, int(model.t.shape[0])
        keep = []
        pm, ps = _points(model, keep), _points(scene, keep)
        d = model.xy.device
        if out is None:
            out = dict(energy32=torch.empty(n, dtype=torch.float32, device=d),
                       energy64=torch.empty(n, dtype=torch.float64, device=d),
                       energy_u64=torch.empty(n, dtype=torch.float64, device=d),
                       assign=torch.empty((n, M), dtype=torch.int32, device=d))
        pp = _params(params, True)
        _check(self._lib.stm_match_noalloc(self.handle, ctypes.byref(pm), ctypes.byref(ps),
                                           ctypes.byref(pp), b, e, _ptr(out["energy32"]),
                                           _ptr(out["energy64"]), _ptr(out["energy_u64"]),
                                           _ptr(out["assign"]), _stream()))
        out["tau_begin"], out["tau_end"] = b, e
        return out

    def match_lists(self, model, scene, params, cand, count, tau_begin=None, tau_end=None):
        """The exact recursion on given lists cand [n, M, kc] / count [n, M]
        (numpy for host Points, torch tensors for DevicePoints)."""
        b, e = self._range(model, scene, tau_begin, tau_end)
        n, M = e - b, int(model.t.shape[0])
        keep = []
        pm, ps = _points(model, keep), _points(scene, keep)
        dev = _is_device(model)
        if dev:
            import torch
            d = model.xy.device
            cand = torch.as_tensor(cand, device=d).to(torch.int32).contiguous()
            count = torch.as_tensor(count, device=d).to(torch.int32).contiguous()
            out = dict(energy32=torch.empty(n, dtype=torch.float32, device=d),
                       energy64=torch.empty(n, dtype=torch.float64, device=d),
                       energy_u64=torch.empty(n, dtype=torch.float64, device=d),
                       assign=torch.empty((n, M), dtype=torch.int32, device=d))
            stream = _stream()
        else:
            cand = np.ascontiguousarray(cand, np.int32)
            count = np.ascontiguousarray(count, np.int32)
            out = dict(energy32=np.empty(n, np.float32), energy64=np.empty(n, np.float64),
                       energy_u64=np.empty(n, np.float64), assign=np.empty((n, M), np.int32))
            stream = None
        assert tuple(cand.shape[:2]) == (n, M) and tuple(count.shape) == (n, M)
        pp = _params(params, dev)
        _check(self._lib.stm_match_lists(self.handle, ctypes.byref(pm), ctypes.byref(ps),
                                         ctypes.byref(pp), b, e, _ptr(cand), _ptr(count),
                                         int(cand.shape[2]), _ptr(out["energy32"]),
                                         _ptr(out["energy64"]), _ptr(out["energy_u64"]),
                                         _ptr(out["assign"]), stream))
        out["tau_begin"], out["tau_end"] = b, e
        return out

    def match_chains(self, model, scene, params, saliency=None, n_chains: int = 3, tau_begin=None,
                     tau_end=None):
        """The multiple-points variant 2 (stm_match_chains): the mean energy of
        the model's single-point chains at every offset of the whole model.
        Returns the stm_match outputs (assign [n, M] in model point order) plus
        chains_used."""
        b, e = self._range(model, scene, tau_begin, tau_end)
        n, M = e - b, int(model.t.shape[0])
        keep = []
        pm, ps = _points(model, keep), _points(scene, keep)
        dev = _is_device(model)
        if dev:
            import torch
            d = model.xy.device
            sal = None if saliency is None else torch.as_tensor(saliency, device=d).to(torch.float32).contiguous()
            out = dict(energy32=torch.empty(n, dtype=torch.float32, device=d),
                       energy64=torch.empty(n, dtype=torch.float64, device=d),
                       energy_u64=torch.empty(n, dtype=torch.float64, device=d),
                       assign=torch.empty((n, M), dtype=torch.int32, device=d))
            stream = _stream()
        else:
            sal = None if saliency is None else np.ascontiguousarray(saliency, np.float32)
            out = dict(energy32=np.empty(n, np.float32), energy64=np.empty(n, np.float64),
                       energy_u64=np.empty(n, np.float64), assign=np.empty((n, M), np.int32))
            stream = None
        used = ctypes.c_int32(0)
        pp = _params(params, dev)
        _check(self._lib.stm_match_chains(self.handle, ctypes.byref(pm), None if sal is None else _ptr(sal),
                                          int(n_chains), ctypes.byref(ps), ctypes.byref(pp), b, e,
                                          _ptr(out["energy32"]), _ptr(out["energy64"]),
                                          _ptr(out["energy_u64"]), _ptr(out["assign"]), ctypes.byref(used),
                                          stream))
        out["tau_begin"], out["tau_end"], out["chains_used"] = b, e, used.value
        return out

    def candidates(self, model, scene, params, tau_begin=None, tau_end=None):
        b, e = self._range(model, scene, tau_begin, tau_end)
        n, M = e - b, int(model.t.shape[0])
        keep = []
        pm, ps = _points(model, keep), _points(scene, keep)
        dev = _is_device(model)
        if dev:
            import torch
            d = model.xy.device
            cand = torch.empty((n, M, params.k_max), dtype=torch.int32, device=d)
            cnt = torch.empty((n, M), dtype=torch.int32, device=d)
            stream = _stream()
        else:
            cand = np.empty((n, M, params.k_max), np.int32)
            cnt = np.empty((n, M), np.int32)
            stream = None
        pp = _params(params, dev)
        _check(self._lib.stm_candidates(self.handle, ctypes.byref(pm), ctypes.byref(ps),
                                        ctypes.byref(pp), b, e, _ptr(cand), _ptr(cnt), stream))
        return cand, cnt

    def unary(self, model, scene, params):
        keep = []
        pm, ps = _points(model, keep), _points(scene, keep)
        dev = _is_device(model)
        M, S = int(model.t.shape[0]), int(scene.t.shape[0])
        if dev:
            import torch
            U = torch.empty((M, S), dtype=torch.float32, device=model.xy.device)
            stream = _stream()
        else:
            U = np.empty((M, S), np.float32)
            stream = None
        pp = _params(params, dev)
        _check(self._lib.stm_unary(self.handle, ctypes.byref(pm), ctypes.byref(ps),
                                   ctypes.byref(pp), _ptr(U), stream))
        return U

    def count_work(self, model, scene, params, tau_begin=None, tau_end=None) -> dict:
        b, e = self._range(model, scene, tau_begin, tau_end)
        keep = []
        pm, ps = _points(model, keep), _points(scene, keep)
        dev = _is_device(model)
        c = np.zeros(4, np.int64)
        pp = _params(params, dev)
        _check(self._lib.stm_count_work(self.handle, ctypes.byref(pm), ctypes.byref(ps),
                                        ctypes.byref(pp), b, e, c.ctypes.data,
                                        _stream() if dev else None))
        return dict(dense_cells=int(c[0]), feasible_cells=int(c[1]), dense_relax=int(c[2]),
                    feasible_relax=int(c[3]))

    # -- tuning -------------------------------------------------------------------
    def set_dp_waves(self, waves: int):
        _check(self._lib.stm_set_dp_waves(self.handle, int(waves)))

    # -- kernel timing ------------------------------------------------------------
    def profile_enable(self, enable: bool = True):
        _check(self._lib.stm_profile_enable(self.handle, int(bool(enable))))

    def profile_read(self) -> dict:
        ms = ctypes.c_double()
        nl, nm = ctypes.c_int64(), ctypes.c_int64()
        _check(self._lib.stm_profile_read(self.handle, ctypes.addressof(ms), ctypes.addressof(nl),
                                          ctypes.addressof(nm)))
        return dict(dp_ms=ms.value, dp_launches=nl.value, dp_matchings=nm.value)


class Trellis:
    """The trellis over a scene block (stm_trellis_*): every model against every
    node of scene nodes [node_begin, node_end), the paper's own problem.
    Device point sets (DevicePoints) are referenced and must outlive it."""

    def __init__(self, ctx: Context, models, scene, params, node_begin: int = 0, node_end=None,
                 stepwise: bool = False):
        self._lib = ctx._lib
        self.ctx = ctx
        self.device = _is_device(scene)
        self._keep = []
        self._models = (_Points * len(models))(*[_points(m, self._keep) for m in models])
        self._scene = _points(scene, self._keep)
        self.msizes = [int(m.t.shape[0]) for m in models]
        self.assign_offsets = np.concatenate([[0], np.cumsum(self.msizes)]).astype(np.int64)
        e = int(scene.t.shape[0]) if node_end is None else int(node_end)
        pp = _params(params, self.device)
        if stepwise:
            pp.flags |= STM_TRELLIS_STEPWISE
        h = ctypes.c_void_p()
        _check(self._lib.stm_trellis_create(ctx.handle, ctypes.addressof(self._models), len(models),
                                            ctypes.byref(self._scene), int(node_begin), e, ctypes.byref(pp),
                                            ctypes.byref(h)))
        self.handle = h

    def info(self) -> dict:
        v = np.zeros(10, np.int64)
        _check(self._lib.stm_trellis_info(self.handle, v.ctypes.data))
        return dict(cells_per_step=int(v[0]), pairs=int(v[1]), tiles=int(v[2]), degenerate=bool(v[3]),
                    dense_cells=int(v[4]), feasible_cells=int(v[5]), dense_relax=int(v[6]),
                    feasible_relax=int(v[7]), points=int(v[8]), fused=bool(v[9]))

    def run(self, out=None):
        """Solves every model.  Returns dict(energy32, energy64, energy_u64
        [n_models], assign [sum of model sizes]); torch tensors on the current
        stream for device point sets (`out` reused when given), numpy otherwise."""
        n, na = len(self.msizes), int(self.assign_offsets[-1])
        if self.device:
            import torch
            if out is None:
                out = dict(energy32=torch.empty(n, dtype=torch.float32, device="cuda"),
                           energy64=torch.empty(n, dtype=torch.float64, device="cuda"),
                           energy_u64=torch.empty(n, dtype=torch.float64, device="cuda"),
                           assign=torch.empty(na, dtype=torch.int32, device="cuda"))
            stream = _stream()
        else:
            out = dict(energy32=np.empty(n, np.float32), energy64=np.empty(n, np.float64),
                       energy_u64=np.empty(n, np.float64), assign=np.empty(na, np.int32))
            stream = None
        _check(self._lib.stm_trellis_run(self.handle, _ptr(out["energy32"]), _ptr(out["energy64"]),
                                         _ptr(out["energy_u64"]), _ptr(out["assign"]), stream))
        return out

    def model_rows(self, out, q):
        """Assignment of model q from a run's output."""
        return out["assign"][self.assign_offsets[q]:self.assign_offsets[q + 1]]

    def close(self):
        if getattr(self, "handle", None):
            self._lib.stm_trellis_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Every offset of every (model, scene) pair in one persistent, graph-replayed
    launch (stm_plan_*).  `pairs` is [n_pairs, 2] (model index, scene index).
    Device point sets (DevicePoints) are referenced and must outlive the plan."""

    def __init__(self, ctx: Context, models, scenes, pairs, params):
        self._lib = ctx._lib
        self.ctx = ctx
        self.device = _is_device(models[0])
        self._keep = []
        self._models = (_Points * len(models))(*[_points(m, self._keep) for m in models])
        self._scenes = (_Points * len(scenes))(*[_points(s_, self._keep) for s_ in scenes])
        self.pairs = np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
        self.msizes = [int(m.t.shape[0]) for m in models]
        pp = _params(params, self.device)
        h = ctypes.c_void_p()
        _check(self._lib.stm_plan_create(ctx.handle, ctypes.addressof(self._models), len(models),
                                         ctypes.addressof(self._scenes), len(scenes),
                                         self.pairs.ctypes.data, self.pairs.shape[0], ctypes.byref(pp),
                                         ctypes.byref(h)))
        self.handle = h
        n = self.pairs.shape[0]
        self.row_offsets = np.zeros(n + 1, np.int64)
        self.assign_offsets = np.zeros(n + 1, np.int64)
        nr, na = ctypes.c_int64(), ctypes.c_int64()
        _check(self._lib.stm_plan_rows(self.handle, self.row_offsets.ctypes.data,
                                       self.assign_offsets.ctypes.data, ctypes.addressof(nr),
                                       ctypes.addressof(na)))
        self.n_rows, self.n_assign = nr.value, na.value

    def close(self):
        if getattr(self, "handle", None):
            self._lib.stm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def outputs(self):
        if self.device:
            import torch
            return dict(energy32=torch.empty(self.n_rows, dtype=torch.float32, device="cuda"),
                        energy64=torch.empty(self.n_rows, dtype=torch.float64, device="cuda"),
                        energy_u64=torch.empty(self.n_rows, dtype=torch.float64, device="cuda"),
                        assign=torch.empty(max(self.n_assign, 1), dtype=torch.int32, device="cuda"))
        return dict(energy32=np.empty(self.n_rows, np.float32), energy64=np.empty(self.n_rows, np.float64),
                    energy_u64=np.empty(self.n_rows, np.float64),
                    assign=np.empty(max(self.n_assign, 1), np.int32))

    def run(self, out=None):
        out = out if out is not None else self.outputs()
        _check(self._lib.stm_plan_run(self.handle, _ptr(out["energy32"]), _ptr(out["energy64"]),
                                      _ptr(out["energy_u64"]), _ptr(out["assign"]),
                                      _stream() if self.device else None))
        return out

    def run_lists(self, cands, counts, kc: int, out=None):
        """A run on given candidate lists (stm_plan_run_lists): cands[q] [n_q, M_q,
        kc] and counts[q] [n_q, M_q] int32 CUDA tensors for every pair q."""
        assert len(cands) == len(counts) == self.pairs.shape[0]
        out = out if out is not None else self.outputs()
        P = ctypes.c_void_p
        cp = (P * len(cands))(*[c.data_ptr() for c in cands])
        np_ = (P * len(counts))(*[c.data_ptr() for c in counts])
        _check(self._lib.stm_plan_run_lists(self.handle, ctypes.addressof(cp), ctypes.addressof(np_), int(kc),
                                            _ptr(out["energy32"]), _ptr(out["energy64"]),
                                            _ptr(out["energy_u64"]), _ptr(out["assign"]),
                                            _stream() if self.device else None))
        return out

    def run_pruned(self, pruner, topk: int = 48, out=None):
        """A run on the pruner's top-k lists with the exact fallback on the
        device; adds fell_back [rows] to the outputs."""
        out = out if out is not None else self.outputs()
        if "fell_back" not in out:
            if self.device:
                import torch
                out["fell_back"] = torch.empty(self.n_rows, dtype=torch.int32, device="cuda")
            else:
                out["fell_back"] = np.empty(self.n_rows, np.int32)
        _check(self._lib.stm_plan_run_pruned(self.handle, pruner.handle, int(topk), _ptr(out["energy32"]),
                                             _ptr(out["energy64"]), _ptr(out["energy_u64"]),
                                             _ptr(out["assign"]), _ptr(out["fell_back"]),
                                             _stream() if self.device else None))
        return out

    def pair_rows(self, out, q):
        """(energy32, energy64, assign [n_tau, M]) slices of pair q."""
        r0, r1 = self.row_offsets[q], self.row_offsets[q + 1]
        a0, a1 = self.assign_offsets[q], self.assign_offsets[q + 1]
        M = self.msizes[self.pairs[q, 0]]
        return (out["energy32"][r0:r1], out["energy64"][r0:r1], out["energy_u64"][r0:r1],
                out["assign"][a0:a1].reshape(-1, M))

    def set_tuning(self, waves: int, wgs_per_cu: int):
        _check(self._lib.stm_plan_set_tuning(self.handle, waves, wgs_per_cu))

    def set_shape(self, waves: int, wgs_per_cu: int, batch: int = 0, sched: int = -1):
        sh = (ctypes.c_int32 * 4)(waves, wgs_per_cu, batch, sched)
        _check(self._lib.stm_plan_set_shape(self.handle, ctypes.addressof(sh)))

    def shape(self) -> dict:
        sh = (ctypes.c_int32 * 4)()
        _check(self._lib.stm_plan_get_shape(self.handle, ctypes.addressof(sh)))
        return dict(waves=sh[0], wgs_per_cu=sh[1], batch=sh[2], packed=sh[3])

    def autotune(self, cache_path=None, n_sample: int = 0):
        ch = (ctypes.c_int32 * 5)()
        _check(self._lib.stm_plan_autotune(self.handle, cache_path.encode() if cache_path else None,
                                           n_sample, ctypes.addressof(ch)))
        return dict(waves=ch[0], wgs_per_cu=ch[1], cached=bool(ch[2]), batch=ch[3], packed=ch[4])


def pruner_num_params(dim: int) -> int:
    """Packed parameter count of the candidate pruner for descriptor dim."""
    return int(load().stm_pruner_num_params(int(dim)))


class Pruner:
    """The learned candidate pruner of a context (device parameters).

    groups: int32 [G, 2] of (tau, i); labels: int32 [G] node ids.  Model and
    scene are host Points or DevicePoints as for Context.match."""

    def __init__(self, ctx: Context, dim: int):
        self._lib = load()
        self.ctx = ctx
        self.dim = int(dim)
        self.n_params = pruner_num_params(dim)
        h = ctypes.c_void_p()
        _check(self._lib.stm_pruner_create(ctx.handle, self.dim, ctypes.byref(h)))
        self.handle = h
        self.rule = Pruner.TIME_NEAREST

    def close(self):
        if getattr(self, "handle", None):
            self._lib.stm_pruner_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    SCORE, FRAMES_FIRST, TIME_NEAREST = 0, 1, 2

    def set_rule(self, rule: int):
        """Selection rule: Pruner.SCORE, Pruner.FRAMES_FIRST or
        Pruner.TIME_NEAREST (the default: the windowed rule's first topk, no
        network evaluation in match_pruned / plan runs)."""
        _check(self._lib.stm_pruner_set_rule(self.handle, int(rule)))
        self.rule = int(rule)

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, np.float32).reshape(-1)
        _check(self._lib.stm_pruner_set_params(self.handle, _ptr(th), th.size))

    def get_params(self) -> np.ndarray:
        th = np.empty(self.n_params, np.float32)
        _check(self._lib.stm_pruner_get_params(self.handle, _ptr(th), th.size))
        return th

    def save(self, path: str):
        _check(self._lib.stm_pruner_save(self.handle, str(path).encode()))

    def load(self, path: str):
        _check(self._lib.stm_pruner_load(self.handle, str(path).encode()))

    def _pair(self, model, scene, params, keep):
        pm, ps = _points(model, keep), _points(scene, keep)
        dev = _is_device(model)
        return pm, ps, _params(params, dev), (_stream() if dev else None)

    @staticmethod
    def _groups(groups):
        g = np.ascontiguousarray(groups, np.int32).reshape(-1, 2)
        return g, int(g.shape[0])

    def features(self, model, scene, params, groups):
        """node [G, 64], phi [G, 64, 8], q [G, 2] (host arrays)."""
        keep = []
        pm, ps, pp, st = self._pair(model, scene, params, keep)
        g, G = self._groups(groups)
        node = np.empty((G, 64), np.int32)
        phi = np.empty((G, 64, 8), np.float32)
        q = np.empty((G, 2), np.int32)
        _check(self._lib.stm_pruner_features(self.handle, ctypes.byref(pm), ctypes.byref(ps),
                                             ctypes.byref(pp), _ptr(g), G, _ptr(node), _ptr(phi),
                                             _ptr(q), st))
        return node, phi, q

    def gradient(self, model, scene, params, groups, labels):
        """(mean loss, gradient [n_params], scores [G, 64]); no update."""
        keep = []
        pm, ps, pp, st = self._pair(model, scene, params, keep)
        g, G = self._groups(groups)
        lab = np.ascontiguousarray(labels, np.int32)
        loss = np.zeros(1, np.float32)
        grad = np.empty(self.n_params, np.float32)
        scores = np.empty((G, 64), np.float32)
        _check(self._lib.stm_pruner_gradient(self.handle, ctypes.byref(pm), ctypes.byref(ps),
                                             ctypes.byref(pp), _ptr(g), _ptr(lab), G, _ptr(loss),
                                             _ptr(grad), _ptr(scores), st))
        return float(loss[0]), grad, scores

    def train_step(self, model, scene, params, groups, labels, lr: float) -> float:
        keep = []
        pm, ps, pp, st = self._pair(model, scene, params, keep)
        g, G = self._groups(groups)
        lab = np.ascontiguousarray(labels, np.int32)
        loss = np.zeros(1, np.float32)
        _check(self._lib.stm_pruner_train_step(self.handle, ctypes.byref(pm), ctypes.byref(ps),
                                               ctypes.byref(pp), _ptr(g), _ptr(lab), G,
                                               float(lr), _ptr(loss), st))
        return float(loss[0])

    def infer(self, model, scene, params, groups, topk: int):
        """BF16 scores [G, 64], kept nodes cand [G, topk] and count [G]."""
        keep = []
        pm, ps, pp, st = self._pair(model, scene, params, keep)
        g, G = self._groups(groups)
        scores = np.empty((G, 64), np.float32)
        cand = np.empty((G, topk), np.int32)
        count = np.empty(G, np.int32)
        _check(self._lib.stm_pruner_infer(self.handle, ctypes.byref(pm), ctypes.byref(ps),
                                          ctypes.byref(pp), _ptr(g), G, int(topk), _ptr(scores),
                                          _ptr(cand), _ptr(count), st))
        return scores, cand, count

    def match(self, model, scene, params, topk: int = 16, tau_begin=None, tau_end=None, out=None):
        """stm_match on the pruned lists; adds fell_back [n] to the outputs."""
        b, e = self.ctx._range(model, scene, tau_begin, tau_end)
        n, M = e - b, int(model.t.shape[0])
        keep = []
        pm, ps, pp, st = self._pair(model, scene, params, keep)
        if _is_device(model):
            import torch
            d = model.xy.device
            if out is None:
                out = dict(energy32=torch.empty(n, dtype=torch.float32, device=d),
                           energy64=torch.empty(n, dtype=torch.float64, device=d),
                           energy_u64=torch.empty(n, dtype=torch.float64, device=d),
                           assign=torch.empty((n, M), dtype=torch.int32, device=d),
                           fell_back=torch.empty(n, dtype=torch.int32, device=d))
        else:
            out = dict(energy32=np.empty(n, np.float32), energy64=np.empty(n, np.float64),
                       energy_u64=np.empty(n, np.float64), assign=np.empty((n, M), np.int32),
                       fell_back=np.empty(n, np.int32))
        _check(self._lib.stm_match_pruned(self.ctx.handle, self.handle, ctypes.byref(pm),
                                          ctypes.byref(ps), ctypes.byref(pp), int(topk), b, e,
                                          _ptr(out["energy32"]), _ptr(out["energy64"]),
                                          _ptr(out["energy_u64"]), _ptr(out["assign"]),
                                          _ptr(out["fell_back"]), st))
        out["tau_begin"], out["tau_end"] = b, e
        return out
