"""bf_das_noalloc: DAS with its partial images in the library's static
scratch array instead of plan memory (GPU).

Called through the C ABI on two plans in a row, the second with a smaller
input, both split over channel groups (so the scratch is used), then on a
volume plan (no split): each output must equal bf_das's on the same plan and
data bit for bit, and the first output must stay intact after the second
call reused the scratch.
"""
import ctypes

import numpy as np
import pytest

import paper_2512_11086_amd as bfm
import synth
from paper_2512_11086_amd import _lib
from synth.configs import MM, describe

pytestmark = pytest.mark.gpu


def _noalloc(plan, e, out, c, torch):
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(_lib.lib().bf_das_noalloc(plan._h, ctypes.c_void_p(e.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), float(c), s))


def _case(k):
    if k == 3:
        desc, H, rfs, info = synth.make_inputs(3, frame=0)
        return desc, H, rfs[0]
    if k == 0:
        desc, H, rf, _ = synth.make_inputs(0)
        return desc, H, rf
    desc = describe("hercules", (32, 16), (0.2 * MM, 0.2 * MM), 16, 16, 700, 20e6, 5e6,
                    (128, 64, 64), (-3 * MM, -1.5 * MM, 3 * MM), (3 * MM, 1.5 * MM, 10 * MM))
    H = synth.hadamard_sylvester(16)
    rng = np.random.default_rng(3)
    pts = rng.uniform([-2 * MM, -1 * MM, 4 * MM], [2 * MM, 1 * MM, 9 * MM], size=(5, 3))
    return desc, H, synth.acquire(desc, pts, np.ones(5), rng, H=H)


def test_das_noalloc_matches_das():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    results = []
    for k in (3, 0, "volume"):            # a large plane, a smaller plane, a volume
        desc, H, rf = _case(k)
        plan = bfm.Plan(desc, H)
        groups = plan.info()["channel_groups"]
        assert (groups > 1) == (k != "volume"), (k, groups)
        e = plan.decode(torch.from_numpy(rf).cuda())
        ref = plan.das(e)
        got = torch.full(plan.out_shape, float("nan"), device="cuda")
        for c in (desc["c"] * 1.01, desc["c"]):      # ends at the plan's own c
            _noalloc(plan, e, got, c, torch)
            torch.cuda.synchronize()
            want = ref if c == desc["c"] else plan.das(e, c=c)
            assert torch.equal(got, want), (k, c)
        results.append((got, ref))
        torch.cuda.synchronize()
    for got, ref in results:            # outputs are the caller's: later calls left them intact
        assert torch.equal(got, ref)


def test_das_noalloc_errors():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L = _lib.lib()
    assert L.bf_das_noalloc(None, None, None, 1540.0, None) == -1
    desc, H, rf = _case(0)
    plan = bfm.Plan(desc, H)
    e = torch.zeros(plan.e_shape, device="cuda")
    assert L.bf_das_noalloc(plan._h, ctypes.c_void_p(e.data_ptr()), None, 1540.0, None) == -1
    out = torch.zeros(plan.out_shape, device="cuda")
    assert L.bf_das_noalloc(plan._h, ctypes.c_void_p(e.data_ptr()),
                            ctypes.c_void_p(out.data_ptr()), -1.0, None) == -4
