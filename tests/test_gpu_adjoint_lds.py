"""The adjoint on the LDS-staged kernel (bf_das_adjoint, linear or cubic
reads) against the FP64 oracle and the gather adjoint.

dL/dc = sum_p G(p) d(image)(p)/dc; the oracle's per-point derivative is
summed against a random G.  Same bound as the gather adjoint's test:
relative 1e-4 (a sum of signed terms whose magnitude is set by the delays,
~1e3 samples, times FP32 sums of weighted derivatives).

dL/de (the RF gradient, scattered through LDS windows): relative L2 1e-5
against oracle.das_adjoint_e, as for the gather adjoint, and the
dot-product identity <DAS(e), G> = <e, dL/de> on the GPU's own outputs.
"""
import numpy as np
import pytest

import oracle
import paper_2512_11086_amd as bfm
import synth
from synth import configs
from synth.configs import MM, describe
from tests.helpers import hadamard, rel_l2

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


def _ge_cases():
    out = []
    for mode, kw, rotate in CASES:
        for interp in ("linear", "cubic"):
            out.append((mode, kw, rotate, interp))
    return out


@pytest.mark.parametrize("mode, kw, rotate, interp", _ge_cases())
def test_de_lds_matches_oracle_and_gather(torch_mod, mode, kw, rotate, interp):
    torch = torch_mod
    d = _desc(mode, interp, rotate, **kw)
    encoded = mode in ("forces", "hercules")
    H, e = _data(d, 11, encoded)
    G = np.random.default_rng(6).normal(size=oracle.Geometry(d).shape)
    ref_e = oracle.das_adjoint_e(d, G)
    ref_c = float(np.sum(G * oracle.das_dc(d, e)))
    plan = bfm.Plan(d, H)
    et = torch.from_numpy(e.astype(np.float32)).cuda()
    Gt = torch.from_numpy(G.astype(np.float32)).cuda()
    ge_only, none = plan.das_adjoint(None, Gt, want_c=False)      # no data read
    ge_both, gc = plan.das_adjoint(et, Gt)
    torch.cuda.synchronize()
    assert none is None
    assert rel_l2(ge_only.cpu().numpy(), ref_e) <= 1e-5
    assert rel_l2(ge_both.cpu().numpy(), ref_e) <= 1e-5
    assert abs(gc.item() - ref_c) <= 1e-4 * abs(ref_c)
    # the gather adjoint on the same plan
    gat = bfm.Plan(d, H)
    gat.set_das_config("gather", (4, 1, 4) if mode == "forces" else (4, 4, 1), 16)
    ge_g, _ = gat.das_adjoint(et, Gt, want_c=False)
    assert rel_l2(ge_only.cpu().numpy(), ge_g.cpu().numpy()) <= 1e-5
    # adjoint identity on the GPU's forward and adjoint
    img = plan.das(et).cpu().numpy().astype(np.float64)
    lhs = float(np.sum(img * G))
    rhs = float(np.sum(e * ge_only.cpu().numpy().astype(np.float64)))
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(img) * np.linalg.norm(G)


@pytest.mark.parametrize("variant, block, nb", [
    ("lds2", (2, 2, 3), 40), ("lds2", (1, 1, 1), 4), ("lds", (4, 2, 1), 32),
    ("lds", (1, 1, 2), 8), ("lds2", (2, 2, 2), 16),
])
def test_de_lds_configurations(torch_mod, variant, block, nb):
    torch = torch_mod
    d = _desc("hercules", "cubic")
    H, e = _data(d, 13)
    G = np.random.default_rng(8).normal(size=oracle.Geometry(d).shape)
    ref = oracle.das_adjoint_e(d, G)
    plan = bfm.Plan(d, H)
    plan.set_das_config(variant, block, nb)
    ge, _ = plan.das_adjoint(None, torch.from_numpy(G.astype(np.float32)).cuda(), want_c=False)
    assert rel_l2(ge.cpu().numpy(), ref) <= 1e-5, (variant, block, nb)


@pytest.mark.parametrize("mode", ["hercules", "forces", "tpw"])
def test_de_grid_through_the_array_plane_and_short_record(torch_mod, mode):
    # depth from -0.6 mm (points at z <= 0 form no image, so G there must not
    # reach grad_e) to 9 mm with a record of 280 samples: the deep points'
    # windows run past the record's end (those taps read 0 and get no gradient)
    torch = torch_mod
    n_ch = 12 if mode == "forces" else 10
    dims = (37, 1, 41) if mode == "forces" else (13, 9, 33)
    kw = dict(tx_angles=np.deg2rad(np.linspace(-10, 10, 8))) if mode == "tpw" else {}
    d = describe(mode, (12, 10), (0.25 * MM, 0.3 * MM), 8, n_ch, 280, 25e6, 6e6, dims,
                 (-2 * MM, -1.5 * MM, -0.6 * MM), (2.2 * MM, 1.2 * MM, 9 * MM), t0=0.3e-6,
                 f_number=1.0, interp="cubic", tx_elements=[0, 3, 4, 6, 7, 8, 10, 11],
                 channel_map=np.random.default_rng(2).permutation(n_ch), **kw)
    G = np.random.default_rng(9).normal(size=oracle.Geometry(d).shape)
    ref = oracle.das_adjoint_e(d, G)
    assert np.abs(ref[..., -3:]).sum() > 0      # gradient reaches the record's end
    plan = bfm.Plan(d, hadamard(8, "scrambled", seed=1) if mode != "tpw" else None)
    ge, _ = plan.das_adjoint(None, torch.from_numpy(G.astype(np.float32)).cuda(), want_c=False)
    assert rel_l2(ge.cpu().numpy(), ref) <= 1e-5


def test_de_repeated_calls_and_workload3(torch_mod):
    # grad_e is cleared by every call (FP32 atomics: equal to rounding)
    torch = torch_mod
    desc, H, rfs, info = synth.make_inputs(3)
    plan = bfm.Plan(desc, H)
    rng = np.random.default_rng(4)
    G = rng.normal(size=oracle.Geometry(desc).shape)
    Gt = torch.from_numpy(G.astype(np.float32)).cuda()
    e = plan.decode(torch.from_numpy(rfs[0]).cuda())
    a, gc = plan.das_adjoint(e, Gt, c=1520.0)
    b, _ = plan.das_adjoint(None, Gt, c=1520.0, want_c=False)
    torch.cuda.synchronize()
    ref = oracle.das_adjoint_e(desc, G, c=1520.0)
    assert rel_l2(a.cpu().numpy(), ref) <= 1e-5
    assert rel_l2(b.cpu().numpy(), a.cpu().numpy()) <= 1e-6
    ref_c = float(np.sum(G * oracle.das_dc(desc, oracle.decode(H, rfs[0]), c=1520.0)))
    assert abs(gc.item() - ref_c) <= 1e-4 * abs(ref_c)


def test_de_fixed_point_range(torch_mod):
    # the LDS windows hold 64-bit fixed point scaled by each workgroup's
    # largest |G|: an all-zero G gives exactly zero, one nonzero point gives
    # that point's own adjoint, and G spanning 12 orders of magnitude keeps
    # the small terms' relative accuracy
    torch = torch_mod
    d = _desc("hercules", "cubic")
    plan = bfm.Plan(d, hadamard(8, "scrambled", seed=3))
    shape = oracle.Geometry(d).shape
    zero, _ = plan.das_adjoint(None, torch.zeros(shape, device="cuda"), want_c=False)
    assert torch.count_nonzero(zero).item() == 0
    G1 = np.zeros(shape)
    G1[6, 4, 20] = -3.5
    g1, _ = plan.das_adjoint(None, torch.from_numpy(G1.astype(np.float32)).cuda(), want_c=False)
    ref1 = oracle.das_adjoint_e(d, G1)
    assert np.count_nonzero(ref1) > 0
    assert rel_l2(g1.cpu().numpy(), ref1) <= 1e-6
    rng = np.random.default_rng(12)
    Gw = rng.normal(size=shape) * 10.0 ** rng.uniform(-6, 6, size=shape)
    gw, _ = plan.das_adjoint(None, torch.from_numpy(Gw.astype(np.float32)).cuda(), want_c=False)
    refw = oracle.das_adjoint_e(d, Gw.astype(np.float32).astype(np.float64))
    assert rel_l2(gw.cpu().numpy(), refw) <= 1e-5
    # the small-G part alone (G below 1e-3 of the largest) is still accurate
    small = np.where(np.abs(Gw) < 1e-3 * np.abs(Gw).max(), Gw, 0.0)
    gs, _ = plan.das_adjoint(None, torch.from_numpy(small.astype(np.float32)).cuda(), want_c=False)
    refs = oracle.das_adjoint_e(d, small.astype(np.float32).astype(np.float64))
    assert rel_l2(gs.cpu().numpy(), refs) <= 1e-5


@pytest.mark.parametrize("k", [1, 6, 7])
def test_de_full_size_adjoint_identity(torch_mod, k):
    # full-size volumes (HERCULES, TPW-32, VLS-128, default configuration):
    # <DAS(e), G> = <e, dL/de> holds at any size
    torch = torch_mod
    desc, H, rf, _ = synth.make_inputs(k)
    plan = bfm.Plan(desc, H)
    e = plan.decode(torch.from_numpy(rf).cuda())
    img = plan.das(e)
    gen = torch.Generator(device="cuda").manual_seed(100 + k)
    G = torch.randn(img.shape, device="cuda", generator=gen)
    ge, _ = plan.das_adjoint(None, G, want_c=False)
    lhs = (img.double() * G.double()).sum().item()
    rhs = (e.double() * ge.double()).sum().item()
    bound = 1e-5 * img.double().norm().item() * G.double().norm().item()
    assert abs(lhs - rhs) <= bound, (lhs, rhs, bound)


@pytest.mark.parametrize("e_type", ["bf16", "i32"])
def test_adjoint_for_other_storage_types(torch_mod, e_type):
    # dL/de reads no data: the LDS kernel serves every storage type; dL/dc of
    # BF16 / INT32 data runs the gather adjoint in the same call
    torch = torch_mod
    d = _desc("hercules", "cubic")
    H, e = _data(d, 14)
    G = np.random.default_rng(15).normal(size=oracle.Geometry(d).shape)
    plan = bfm.Plan(d, H, e_type=e_type)
    dt = {"bf16": torch.bfloat16, "i32": torch.int32}[e_type]
    et = torch.from_numpy(np.rint(e).astype(np.float32)).to(dt).cuda()
    e_ref = et.float().cpu().numpy().astype(np.float64)
    ge, gc = plan.das_adjoint(et, torch.from_numpy(G.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    assert rel_l2(ge.cpu().numpy(), oracle.das_adjoint_e(d, G)) <= 1e-5
    ref_c = float(np.sum(G * oracle.das_dc(d, e_ref)))
    assert abs(gc.item() - ref_c) <= 1e-4 * abs(ref_c)
