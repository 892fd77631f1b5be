"""dL/dc on the LDS-staged kernel (bf_das_adjoint without the RF gradient,
FP32 data, linear or cubic reads) against the FP64 oracle and the gather
adjoint.

dL/dc = sum_p G(p) d(image)(p)/dc; the oracle's per-point derivative is
summed against a random G.  Same bound as the gather adjoint's test:
relative 1e-4 (a sum of signed terms whose magnitude is set by the delays,
~1e3 samples, times FP32 sums of weighted derivatives).
"""
import numpy as np
import pytest

import oracle
import paper_2512_11086_amd as bfm
import synth
from synth import configs
from synth.configs import MM, describe
from tests.helpers import hadamard

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _desc(mode, interp, rotate=False, **kw):
    M = None
    if rotate:
        a = 0.3
        R = np.array([[np.cos(a), 0, np.sin(a)], [0, 1, 0], [-np.sin(a), 0, np.cos(a)]])
        M = configs.centered_xdc((12, 10), (0.25 * MM, 0.3 * MM))
        M[:3, :3] = R
        M[:3, 3] += [0.2 * MM, -0.1 * MM, 0.5 * MM]
    n_ch = 10 if mode in ("hercules", "tpw", "vls") else 12
    dims = (37, 1, 53) if mode == "forces" else (13, 9, 29)
    if mode == "tpw":
        kw.setdefault("tx_angles", np.deg2rad(np.linspace(-10, 10, 8)))
    return describe(mode, (12, 10), (0.25 * MM, 0.3 * MM), 8, n_ch, 600, 25e6, 6e6, dims,
                    (-2 * MM, -1.5 * MM, 1.0 * MM), (2.2 * MM, 1.2 * MM, 9 * MM), t0=0.3e-6,
                    f_number=1.0, interp=interp, tx_elements=[0, 3, 4, 6, 7, 8, 10, 11],
                    channel_map=np.random.default_rng(2).permutation(n_ch), xdc=M, **kw)


def _data(desc, seed, encoded=True):
    rng = np.random.default_rng(seed)
    pts = rng.uniform([-2 * MM, -1 * MM, 1.5 * MM], [2 * MM, 1 * MM, 8 * MM], size=(6, 3))
    if desc["mode"] == "forces":
        pts[:, 1] = 0
    H = hadamard(desc["n_tx"], "scrambled", seed=seed) if encoded else None
    rf = synth.acquire(desc, pts, np.ones(6), rng, H=H, encoded=encoded)
    return H, oracle.decode(np.eye(desc["n_tx"], dtype=np.int8) if H is None else H, rf)


CASES = [("forces", {}, False), ("hercules", {}, False), ("hercules", {}, True),
         ("hercules", dict(focal_depth=-6 * MM), False), ("tpw", {}, False),
         ("vls", dict(focal_depth=-4 * MM), False), ("vls", dict(focal_depth=5.1 * MM), False)]


@pytest.mark.parametrize("mode, kw, rotate", CASES)
@pytest.mark.parametrize("interp", ["linear", "cubic"])
def test_dc_lds_matches_oracle_and_gather(torch_mod, mode, kw, rotate, interp):
    torch = torch_mod
    d = _desc(mode, interp, rotate, **kw)
    encoded = mode in ("forces", "hercules")
    H, e = _data(d, 7, encoded)
    G = np.random.default_rng(5).normal(size=oracle.Geometry(d).shape)
    plan = bfm.Plan(d, H)
    et = torch.from_numpy(e.astype(np.float32)).cuda()
    Gt = torch.from_numpy(G.astype(np.float32)).cuda()
    _, gc_lds = plan.das_adjoint(et, Gt, want_e=False)          # LDS path
    _, gc_gat = plan.das_adjoint(et, Gt, want_e=True)           # gather path
    torch.cuda.synchronize()
    ref = float(np.sum(G * oracle.das_dc(d, e)))
    assert abs(gc_lds.item() - ref) <= 1e-4 * abs(ref), (gc_lds.item(), ref)
    assert abs(gc_gat.item() - ref) <= 1e-4 * abs(ref)
    # repeated calls are bit-identical (fixed-order sums)
    _, again = plan.das_adjoint(et, Gt, want_e=False)
    assert again.item() == gc_lds.item()


def test_dc_lds_workload3_frames(torch_mod):
    torch = torch_mod
    desc, H, rfs, info = synth.make_inputs(3)
    plan = bfm.Plan(desc, H)
    rng = np.random.default_rng(9)
    for f in range(2):
        e = oracle.decode(H, rfs[f])
        G = rng.normal(size=oracle.Geometry(desc).shape)
        _, gc = plan.das_adjoint(torch.from_numpy(e.astype(np.float32)).cuda(),
                                 torch.from_numpy(G.astype(np.float32)).cuda(), c=1520.0,
                                 want_e=False)
        ref = float(np.sum(G * oracle.das_dc(desc, e, c=1520.0)))
        assert abs(gc.item() - ref) <= 1e-4 * abs(ref), (f, gc.item(), ref)
