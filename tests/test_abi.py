"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/stm.h declares, and rejects invalid arguments and
invalid host data before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1505_00581_amd as stm
from paper_1505_00581_amd import _binding as B
from paper_1505_00581_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "stm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(stm_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = stm.load()
    names = _declared()
    assert len(names) >= 8
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(stm.EXPORTS)


def test_last_error_starts_empty_or_is_a_string():
    assert isinstance(stm.load().stm_last_error(), bytes)


def _call_match(model, scene, params, ctx=None, taus=(0, 1)):
    lib = stm.load()
    keep = []
    pm, ps = B._points(model, keep), B._points(scene, keep)
    pp = B._params(params, False)
    n = taus[1] - taus[0]
    e = np.zeros(max(n, 1), np.float32)
    a = np.zeros((max(n, 1), model.t.shape[0]), np.int32)
    rc = lib.stm_match(ctx, ctypes.byref(pm), ctypes.byref(ps), ctypes.byref(pp), taus[0], taus[1],
                       e.ctypes.data, None, None, a.ctypes.data, None)
    return rc, lib.stm_last_error().decode()


def _good():
    w = synth.config1(0)
    return w.models[0], w.scenes[0], w.params


def test_null_context_is_einval_after_argument_checks():
    m, s, p = _good()
    rc, msg = _call_match(m, s, p)
    assert rc == stm.STM_EINVAL and "context" in msg


@pytest.mark.parametrize("mutate,needle", [
    (lambda m, s, p: setattr(p, "k_max", 0), "k_max"),
    (lambda m, s, p: setattr(p, "window", -1), "window"),
    (lambda m, s, p: setattr(p, "lambda2", -0.1), "lambda"),
    (lambda m, s, p: setattr(p, "lambda3", float("nan")), "lambda"),
    (lambda m, s, p: m.t.__setitem__(3, m.t[2]), "model frames"),
    (lambda m, s, p: s.t.__setitem__(5, s.t[4] - 1), "sorted"),
    (lambda m, s, p: s.t.__setitem__(s.t.shape[0] - 1, s.n_frames), "outside"),
    (lambda m, s, p: m.desc.__setitem__((0, 0), np.nan), "non-finite model"),
    (lambda m, s, p: s.xy.__setitem__((7, 1), np.inf), "non-finite scene"),
    (lambda m, s, p: setattr(p, "w_dummy", -0.5), "w_dummy"),
    (lambda m, s, p: setattr(p, "w_dummy", float("inf")), "w_dummy"),
])
def test_invalid_inputs_rejected_on_host(mutate, needle):
    m, s, p = _good()
    m = synth.Points(m.xy.copy(), m.t.copy(), m.desc.copy())
    s = synth.Points(s.xy.copy(), s.t.copy(), s.desc.copy(), s.n_frames)
    mutate(m, s, p)
    rc, msg = _call_match(m, s, p)
    assert rc == stm.STM_EINVAL, msg
    assert needle in msg


def test_k_max_above_64_unsupported():
    m, s, p = _good()
    p.k_max = 65
    rc, msg = _call_match(m, s, p)
    assert rc == stm.STM_EUNSUPPORTED and "k_max" in msg and "trellis" in msg


def test_span_with_dummies_unsupported():
    m, s, p = _good()
    p.w_dummy, p.closeness_span = 0.5, True
    rc, msg = _call_match(m, s, p)
    assert rc == stm.STM_EUNSUPPORTED and "span" in msg


def test_short_model_and_dim_mismatch_rejected():
    m, s, p = _good()
    m2 = synth.Points(m.xy[:2].copy(), m.t[:2].copy(), m.desc[:2].copy())
    assert _call_match(m2, s, p)[0] == stm.STM_EINVAL
    m3 = synth.Points(m.xy.copy(), m.t.copy(), np.ascontiguousarray(m.desc[:, :100]))
    rc, msg = _call_match(m3, s, p)
    assert rc == stm.STM_EINVAL and "dim" in msg


def test_offsets_host_pointers():
    lib = stm.load()
    m, s, p = _good()
    keep = []
    pm, ps = B._points(m, keep), B._points(s, keep)
    b, e = ctypes.c_int32(-1), ctypes.c_int32(-1)
    assert lib.stm_offsets(None, ctypes.byref(pm), ctypes.byref(ps), 0, ctypes.byref(b),
                           ctypes.byref(e)) == 0
    assert b.value == 0 and e.value == s.n_frames - int(m.t[-1] - m.t[0])
    # a model longer than the scene has no offsets
    s2 = synth.Points(s.xy, np.minimum(s.t, 5).astype(np.int32), s.desc, 6)
    ps2 = B._points(s2, keep)
    assert lib.stm_offsets(None, ctypes.byref(pm), ctypes.byref(ps2), 0, ctypes.byref(b),
                           ctypes.byref(e)) == 0
    assert (b.value, e.value) == (0, 0)


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = stm.load()
    h = ctypes.c_void_p()
    rc = lib.stm_create(ctypes.byref(h), 0)
    assert rc in (stm.STM_EHIP, stm.STM_EINVAL)
    assert not h.value
    lib.stm_destroy(None)  # no-op


def test_pruner_parameter_count_and_null_arguments():
    lib = stm.load()
    assert lib.stm_pruner_num_params(162) == 128 * 332 + 128 + 128 * 128 + 128 + 128 + 1
    assert stm.pruner_num_params(4) == 128 * 16 + 128 + 128 * 128 + 257
    assert lib.stm_pruner_num_params(0) == -1
    h = ctypes.c_void_p()
    assert lib.stm_pruner_create(None, 162, ctypes.byref(h)) == stm.STM_EINVAL
    assert "context" in lib.stm_last_error().decode()
    assert lib.stm_pruner_set_params(None, None, 0) == stm.STM_EINVAL
    lib.stm_pruner_destroy(None)   # a no-op


def test_match_lists_checks_arguments_before_the_device():
    m, s, p = _good()
    lib = stm.load()
    keep = []
    pm, ps = B._points(m, keep), B._points(s, keep)
    pp = B._params(p, False)
    e = np.zeros(1, np.float32)
    a = np.zeros((1, m.n), np.int32)
    cand = np.zeros((1, m.n, 4), np.int32)
    cnt = np.zeros((1, m.n), np.int32)
    rc = lib.stm_match_lists(None, ctypes.byref(pm), ctypes.byref(ps), ctypes.byref(pp), 0, 1,
                             cand.ctypes.data, cnt.ctypes.data, 4, e.ctypes.data, None, None,
                             a.ctypes.data, None)
    assert rc == stm.STM_EINVAL and "context" in lib.stm_last_error().decode()


def test_one_hip_runtime_per_process():
    """Loading the library binds it to torch's HIP runtime: a process that
    touches libstm.so before torch must not end up with two runtimes."""
    import subprocess
    import sys
    code = ("import paper_1505_00581_amd as s; s.load(); "
            "print(sorted(set(l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l)))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         check=True).stdout.strip().splitlines()[-1]
    assert out.count("libamdhip64") == 1, out


def test_plan_run_pruned_rejects_null_arguments():
    lib = stm.load()
    assert lib.stm_plan_run_pruned(None, None, 16, None, None, None, None, None, None) == stm.STM_EINVAL
    assert "null" in lib.stm_last_error().decode()


def test_params_struct_and_dummy_constants_match_the_header():
    src = open(os.path.join(ROOT, "include", "stm.h")).read()
    body = dict((n, b) for b, n in re.findall(r"typedef struct \{(.*?)\} (\w+);", src, flags=re.S))["stm_params"]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b(\w+)\s*;", body)
    assert fields == [f[0] for f in B._Params._fields_]
    assert ctypes.sizeof(B._Params) == 48
    assert int(re.search(r"#define STM_DUMMY\s+(0x[0-9a-f]+)u", src).group(1), 16) == B.STM_DUMMY
    assert int(re.search(r"#define STM_DUMMY_NODE \((-?\d+)\)", src).group(1)) == B.STM_DUMMY_NODE


def test_dummy_params_pass_the_argument_checks():
    m, s, p = _good()
    p.w_dummy = 0.4
    rc, msg = _call_match(m, s, p)
    assert rc == stm.STM_EINVAL and "context" in msg


def test_plan_run_lists_rejects_null_arguments():
    lib = stm.load()
    assert lib.stm_plan_run_lists(None, None, None, 8, None, None, None, None, None) == stm.STM_EINVAL
