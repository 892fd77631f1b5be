"""Host-side argument checks of the Python binding (no GPU needed).

A host tensor handed to a kernel would be read as a device address, and a
short frame list would make the library read past the pointer arrays.  The
binding must reject both, and wrong dtypes and shapes, with ValueError
before it calls the library.  The objects are built without a device plan
(the checks run before the plan handle is used); the library is replaced by
a stub that fails the test if any call reaches it.
"""
import numpy as np
import pytest
import torch

import paper_2512_11086_amd as bfm
from synth import configs


class _NoCalls:
    def __getattr__(self, name):
        raise AssertionError(f"library call {name} reached despite invalid arguments")


@pytest.fixture
def no_lib(monkeypatch):
    monkeypatch.setattr(bfm, "lib", lambda: _NoCalls())


def _plan(k=0):
    d = configs.workload(k)
    p = object.__new__(bfm.Plan)
    p.desc, p.e_type, p._h = d, "f32", None
    p.n_tx, p.n_ch, p.n_samples = d["n_tx"], d["n_ch"], d["n_samples"]
    nx, ny, nz = d["dims"]
    p.out_shape = (ny, nx, nz)
    p.iq = False
    p.rf_shape = p.e_shape = (p.n_tx, p.n_ch, p.n_samples)
    p.c = d["c"]
    return p


def test_plan_rejects_host_tensors(no_lib):
    p = _plan()
    rf = torch.zeros(p.rf_shape, dtype=torch.int16)
    e = torch.zeros(p.e_shape, dtype=torch.float32)
    g = torch.zeros(p.out_shape, dtype=torch.float32)
    with pytest.raises(ValueError, match="CUDA"):
        p.decode(rf)
    with pytest.raises(ValueError, match="CUDA"):
        p.das_fused(rf)
    with pytest.raises(ValueError, match="CUDA"):
        p.das(e)
    with pytest.raises(ValueError, match="CUDA"):
        p.das_adjoint(e, g)
    with pytest.raises(ValueError, match="CUDA"):
        p.das_adjoint(None, g, want_c=False)
    with pytest.raises(ValueError, match="CUDA"):
        bfm.sharpness(g.reshape(1, -1))


def test_plan_rejects_wrong_dtype_and_shape(no_lib):
    p = _plan()
    with pytest.raises(ValueError):
        p._check_rf(torch.zeros(p.rf_shape, dtype=torch.int32))
    with pytest.raises(ValueError):
        p._check_e(torch.zeros((3, 3), dtype=torch.float32))


def _batch(n=3):
    rng = np.random.default_rng(5)
    descs = [configs.frame_4(kind, cols) for kind, cols in configs.frames_4_plan(rng, n)]
    b = object.__new__(bfm.BatchPlan)
    b.descs, b._h = descs, None
    b.out_shapes = [(d["dims"][1], d["dims"][0], d["dims"][2]) for d in descs]
    return b


def test_batch_rejects_short_lists_and_host_tensors(no_lib):
    b = _batch(3)
    rfs = [torch.zeros((d["n_tx"], d["n_ch"], d["n_samples"]), dtype=torch.int16) for d in b.descs]
    outs = [torch.zeros(s, dtype=torch.float32) for s in b.out_shapes]
    with pytest.raises(ValueError, match="need 3"):
        b.run(rfs[:2], outs)
    with pytest.raises(ValueError, match="need 3"):
        b.graph_launch(rfs, outs[:1])
    with pytest.raises(ValueError, match="CUDA"):
        b.run(rfs, outs)
    with pytest.raises(ValueError, match="CUDA"):
        b.graph_launch(rfs, outs)


def test_stage_objects_reject_host_tensors(no_lib):
    env = object.__new__(bfm.Envelope)
    env.shape, env.iq, env._h = (4, 64), False, None
    with pytest.raises(ValueError, match="CUDA"):
        env(torch.zeros((4, 64)))
    dm = object.__new__(bfm.Demod)
    dm.n_traces, dm.n_samples, dm.n_out, dm.out, dm._h = 2, 16, 8, "i16", None
    with pytest.raises(ValueError, match="CUDA"):
        dm(torch.zeros((2, 16), dtype=torch.int16))
