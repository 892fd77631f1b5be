"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every function include/bf.h declares, and
reject every invalid description on the host before any device call.
"""
import ctypes
import math
import os
import re
import threading

import numpy as np
import pytest

import paper_2512_11086_amd as bfm
from paper_2512_11086_amd import _lib
from synth import configs, hadamard_sylvester

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions(header="bf.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(bf_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_function():
    L = _lib.lib()
    names = _declared_functions()
    assert len(names) >= 15, names
    for name in names:
        assert hasattr(L, name), f"{name} declared in bf.h but not exported"
    assert set(names) == set(_lib.EXPORTED)
    hooks = _declared_functions("bf_test.h")
    assert set(hooks) == set(_lib.TEST_HOOKS)
    for name in hooks:
        assert hasattr(L, name), f"{name} declared in bf_test.h but not exported"
    # the binding, the header and the library agree on the ABI version
    with open(os.path.join(ROOT, "include", "bf.h")) as fp:
        text = fp.read()
    m = re.search(r"#define BF_ABI_VERSION (\d+)", text)
    assert m and int(m.group(1)) == _lib.ABI_VERSION == L.bf_abi_version()
    m = re.search(r"#define BF_MAX_FRAMES (\d+)", text)
    assert m and int(m.group(1)) == _lib.MAX_FRAMES


def _good(k=0):
    d = configs.workload(k)
    return d, hadamard_sylvester(d["n_tx"])


def _status(desc, H, **kw):
    m = bfm.params_from_desc(desc, H, **kw)
    return _lib.lib().bf_validate(ctypes.byref(m.p))


def test_validate_accepts_workloads():
    for k in (0, 1, 3):
        d, H = _good(k)
        assert _status(d, H) == 0, _lib.lib().bf_last_error()
    plan = configs.frames_4_plan(np.random.default_rng(0), 4)
    for kind, cols in plan:
        d = configs.frame_4(kind, cols)
        assert _status(d, hadamard_sylvester(d["n_tx"])) == 0


def test_validate_null_and_hadamard_errors():
    L = _lib.lib()
    assert L.bf_validate(None) == -1
    d, H = _good()
    assert _status(d, None) == 0          # NULL: unencoded acquisition, identity decode
    bad = H.copy()
    bad[3, 5] = 0
    assert _status(d, bad) == -3
    bad = H.copy()
    bad[3, :] = bad[4, :]            # +-1 entries but rows not orthogonal
    assert _status(d, bad) == -3
    assert b"H H^T" in L.bf_last_error()
    # any Hadamard matrix is accepted, e.g. rows permuted and a column negated
    P = H[np.random.default_rng(1).permutation(32)].copy()
    P[:, 7] *= -1
    assert _status(d, P) == 0


@pytest.mark.parametrize("field,value,code", [
    ("n_tx", 0, -2), ("n_tx", 257, -2), ("n_ch", 0, -2), ("n_samples", 0, -2),
    ("dims", (0, 1, 128), -2), ("pitch", (0.0, 2e-4), -4), ("pitch", (math.nan, 2e-4), -4),
    ("fs", 0.0, -4), ("fs", math.inf, -4), ("c", -1540.0, -4), ("t0", math.nan, -4),
    ("f_number", -1.0, -4), ("gmin", (math.nan, 0, 0), -4), ("mode", "bogus", None),
])
def test_validate_field_errors(field, value, code):
    d, H = _good()
    d = dict(d)
    if field == "mode":
        m = bfm.params_from_desc(d, H)
        m.p.mode = 7
        assert _lib.lib().bf_validate(ctypes.byref(m.p)) == -5
        return
    if field == "n_tx":
        d[field] = value
        d["tx_elements"] = None
        H = np.ones((max(value, 1), max(value, 1)), dtype=np.int8)
    else:
        d[field] = value
    assert _status(d, H) == code


def test_validate_transform_and_indices():
    d, H = _good()
    M = np.array(d["xdc"], dtype=float)
    M[3, 2] = 1.0
    assert _status(dict(d, xdc=M), H) == -4
    tx = np.arange(32, dtype=np.int32)
    tx[5] = 32                                    # column outside a 32-column array
    assert _status(dict(d, tx_elements=tx), H) == -2
    ch = np.arange(32, dtype=np.int32)
    ch[0] = -1
    assert _status(dict(d, channel_map=ch), H) == -2


def test_validate_size_limits_and_unsupported():
    d, H = _good(1)
    assert _status(dict(d, dims=(2048, 1024, 1024)), H) == -6     # 2^31 output points
    d2 = dict(d, n_samples=65536, n_ch=256, channel_map=None)    # 128*256*65536 = 2^31
    assert _status(d2, H) == -6
    assert _status(dict(d, focal_depth=0.03), H) == -5           # diverging wave not built
    m = bfm.params_from_desc(d, H)
    m.p.interp = 9
    assert _lib.lib().bf_validate(ctypes.byref(m.p)) == -5


def test_error_message_is_thread_local():
    L = _lib.lib()
    d, H = _good()
    bad = H.copy()
    bad[0, 0] = 3
    assert _status(d, bad) == -3
    seen = {}

    def other():
        seen["before"] = L.bf_last_error()
        assert _status(d, H) == 0
        seen["after"] = L.bf_last_error()

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert seen["before"] == b"" and seen["after"] == b""
    assert b"not +-1" in L.bf_last_error()


def test_device_calls_fail_cleanly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = _lib.lib()
    d, H = _good()
    m = bfm.params_from_desc(d, H)
    h = ctypes.c_void_p(123)
    st = L.bf_plan_create(ctypes.byref(m.p), ctypes.byref(h))
    assert st == -8 and h.value is None
    assert L.bf_plan_destroy(None) == 0
    assert L.bf_decode(None, None, None, None) == -1
    assert L.bf_das(None, None, None, ctypes.c_double(1540.0), None) == -1
    assert L.bf_das_frames(None, None, 2, None, 1540.0, None) == -1
    assert L.bf_das_adjoint_frames(None, None, None, 2, 1540.0, None, None, None) == -1
    assert L.bf_sharpness(None, 1, 1, None, None, None) == -1
    assert L.bf_batch_get_frame_info(None, 0, None) == -1
    assert L.bf_das_noalloc(None, None, None, ctypes.c_double(1540.0), None) == -1
    assert L.bf_test_set_stack_cap(None, 1) == -1


def test_hann_polynomial_matches_window():
    # The library's polynomial in u^2 (test hook) against Eq. 3 evaluated directly.
    poly = _lib.lib().bf_test_hann_poly
    u = np.linspace(0.0, 0.5, 2001)[:-1]
    want = np.cos(np.pi * u) ** 2
    got = np.array([poly(v * v) for v in u])
    assert np.max(np.abs(got - want)) < 3e-7
    assert poly(0.0) == 1.0
    assert abs(poly(0.25)) < 1e-6


def test_validate_iq_descriptions():
    d, H = _good(1)
    iq = dict(d, iq=True)
    assert _status(iq, H) == 0, _lib.lib().bf_last_error()
    assert _status(iq, H, e_type="bf16") == -5          # IQ decodes to FP32 only
    m = bfm.params_from_desc(d, H)
    m.p.iq = 2
    assert _lib.lib().bf_validate(ctypes.byref(m.p)) == -5


def _demod_status(**kw):
    taps = np.ascontiguousarray(kw.pop("taps", np.ones(4)), dtype=np.float64)
    p = _lib.DemodParams()
    p.n_traces, p.n_samples, p.decimation = kw.get("n_traces", 4), kw.get("S", 100), kw.get("D", 2)
    p.n_taps = kw.get("n_taps", taps.size)
    p.taps_re = taps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if kw.get("re", True) else None
    p.taps_im = None
    p.fs, p.fd = kw.get("fs", 20e6), kw.get("fd", 5e6)
    p.out_type = kw.get("out_type", 0)
    h = ctypes.c_void_p()
    st = _lib.lib().bf_demod_create(ctypes.byref(p), ctypes.byref(h))
    if st == 0:
        _lib.lib().bf_demod_destroy(h)
    return st


@pytest.mark.parametrize("kw,code", [
    (dict(n_traces=0), -2), (dict(S=0), -2), (dict(S=65537), -2), (dict(D=0), -2),
    (dict(D=17), -2), (dict(n_taps=0), -2), (dict(taps=np.ones(1025)), -2),
    (dict(out_type=7), -5), (dict(fs=0.0), -4), (dict(fd=math.inf), -4),
    (dict(taps=np.array([1.0, math.nan])), -4), (dict(re=False), -1),
    (dict(n_traces=40000, S=65536), -6),
])
def test_demod_validation_errors(kw, code):
    assert _demod_status(**kw) == code


def test_demod_null_arguments_and_no_device():
    L = _lib.lib()
    assert L.bf_demod_create(None, None) == -1
    assert L.bf_demod_destroy(None) == 0
    assert L.bf_demodulate(None, None, None, None) == -1
    n = ctypes.c_int32()
    assert L.bf_demod_out_samples(None, ctypes.byref(n)) == -1
    import torch
    if not torch.cuda.is_available():
        assert _demod_status() == -8                     # valid, but no gfx950 here


def test_envelope_validation_on_host():
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.bf_env_create(4, 16, 0, None) == -1
    assert L.bf_env_create(0, 16, 0, ctypes.byref(h)) == -2
    assert L.bf_env_create(4, 0, 0, ctypes.byref(h)) == -2
    assert L.bf_env_create(4, 4097, 0, ctypes.byref(h)) == -2
    assert L.bf_env_create(4, 16, 2, ctypes.byref(h)) == -5
    assert L.bf_env_create(1 << 20, 4096, 0, ctypes.byref(h)) == -6
    assert L.bf_env_destroy(None) == 0
    assert L.bf_envelope(None, None, None, 0, 0.0, 1.0, None) == -1
    import torch
    if not torch.cuda.is_available():
        assert L.bf_env_create(4, 16, 0, ctypes.byref(h)) == -8


def test_validate_transmit_models():
    MM = 1e-3
    d, H = _good(1)
    ok = dict(d, focal_depth=-20 * MM)                       # diverging HERCULES
    assert _status(ok, H) == 0, _lib.lib().bf_last_error()
    assert _status(dict(d, focal_depth=20 * MM), H) == -5    # focused HERCULES: not a model here
    tpw = dict(d, mode="tpw", tx_angles=np.linspace(-0.2, 0.2, d["n_tx"]))
    assert _status(tpw, None) == 0, _lib.lib().bf_last_error()
    assert _status(dict(tpw, tx_angles=None), None) == -1
    bad = np.zeros(d["n_tx"])
    bad[3] = math.pi / 2
    assert _status(dict(tpw, tx_angles=bad), None) == -4
    bad[3] = math.nan
    assert _status(dict(tpw, tx_angles=bad), None) == -4
    vls = dict(d, mode="vls", focal_depth=-5 * MM)
    assert _status(vls, None) == 0
    assert _status(dict(vls, focal_depth=math.inf), None) == -4
    m = bfm.params_from_desc(d, H)
    m.p.mode = 4
    assert _lib.lib().bf_validate(ctypes.byref(m.p)) == -5
