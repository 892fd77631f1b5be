"""The LDS DAS kernel with two adjacent depth points per lane (variant "lds2",
the default for HERCULES plans with real data) against the FP64 oracle.

Same tolerances as the other DAS kernels (relative L2 1e-5; nearest reads
1e-4).  Covers odd depth counts (the second point of the last lane row falls
outside the grid), depth counts of 1 and 2, several lane tiles, workgroup
shapes and batch sizes (one to three staging rounds), BF16 / INT32 storage,
the full-size workload (sampled points, default configuration), agreement
with the one-point kernel, and the persistent batched path and its graph.
"""
import numpy as np
import pytest

import oracle
import paper_2512_11086_amd as bfm
import synth
from synth.configs import MM, describe
from tests.helpers import hadamard, rel_l2, sample_voxels

pytestmark = pytest.mark.gpu

TOL_L2 = 1e-5
TOL_NEAREST = 1e-4


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _desc(interp="cubic", nz=29, f_number=0.8, rotate=False, **kw):
    M = None
    if rotate:
        a = 0.25
        R = np.array([[np.cos(a), 0, np.sin(a)], [0, 1, 0], [-np.sin(a), 0, np.cos(a)]])
        M = synth.configs.centered_xdc((12, 10), (0.25 * MM, 0.3 * MM))
        M[:3, :3] = R
        M[:3, 3] += [0.2 * MM, -0.1 * MM, 0.5 * MM]
    return describe("hercules", (12, 10), (0.25 * MM, 0.3 * MM), 8, 10, 600, 25e6, 6e6,
                    (13, 9, nz), (-2 * MM, -1.5 * MM, 1.0 * MM), (2.2 * MM, 1.2 * MM, 9 * MM),
                    t0=0.3e-6, f_number=f_number, interp=interp,
                    tx_elements=[0, 3, 4, 6, 7, 8, 10, 11],
                    channel_map=np.random.default_rng(2).permutation(10), xdc=M, **kw)


def _data(desc, seed):
    rng = np.random.default_rng(seed)
    pts = rng.uniform([-2 * MM, -1 * MM, 1.5 * MM], [2 * MM, 1 * MM, 8 * MM], size=(6, 3))
    H = hadamard(desc["n_tx"], "scrambled", seed=seed)
    rf = synth.acquire(desc, pts, np.ones(6), rng, H=H)
    return H, oracle.decode(H, rf)


def _run(torch, desc, H, e, variant="lds2", tile=None, block=(2, 2, 3), nb=40, e_type="f32"):
    plan = bfm.Plan(desc, H, e_type=e_type, tile=tile)
    plan.set_das_config(variant, block, nb)
    dt = {"f32": torch.float32, "bf16": torch.bfloat16, "i32": torch.int32}[e_type]
    x = torch.from_numpy(np.ascontiguousarray(e)).to(dt).cuda()
    img = plan.das(x)
    torch.cuda.synchronize()
    return plan, img.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("interp", ["nearest", "linear", "cubic"])
@pytest.mark.parametrize("rotate", [False, True])
def test_small_volume_matches_oracle(torch_mod, interp, rotate):
    desc = _desc(interp, rotate=rotate)
    H, e = _data(desc, 5)
    ref = oracle.das(desc, e)
    plan, got = _run(torch_mod, desc, H, e.astype(np.float32))
    # a depth axis tilted in the array frame runs one point per lane
    assert plan.info()["variant"] == (0 if rotate else 2)
    err = rel_l2(got, ref)
    assert err <= (TOL_NEAREST if interp == "nearest" else TOL_L2), err


@pytest.mark.parametrize("nz", [1, 2, 3, 8, 31])
def test_depth_counts(torch_mod, nz):
    desc = _desc(nz=nz)
    H, e = _data(desc, 6)
    ref = oracle.das(desc, e)
    _, got = _run(torch_mod, desc, H, e.astype(np.float32), block=(1, 1, 2), nb=8)
    assert rel_l2(got, ref) <= TOL_L2


@pytest.mark.parametrize("tile, block, nb", [
    ((3, 3, 0), (2, 2, 3), 40), ((3, 3, 0), (1, 1, 1), 4), ((2, 2, 2), (2, 2, 2), 16),
    ((1, 1, 4), (1, 1, 4), 24), ((3, 3, 0), (4, 2, 1), 32), ((0, 0, 6), (1, 1, 2), 64),
    ((2, 3, 1), (2, 2, 4), 40),
])
def test_configurations_agree(torch_mod, tile, block, nb):
    desc = _desc(f_number=1.0)
    H, e = _data(desc, 8)
    ref = oracle.das(desc, e)
    _, got = _run(torch_mod, desc, H, e.astype(np.float32), tile=tile, block=block, nb=nb)
    assert rel_l2(got, ref) <= TOL_L2, (tile, block, nb)
    # one point per lane on the same tile: terms at the very edge of the
    # aperture (weight ~1e-7) may be visited differently, and the read
    # positions are rounded in FP32 around each box's reference sample, so
    # two tilings round a point's positions differently (each stays within
    # TOL_L2 of the oracle; tests/test_fold_precision.py bounds the rounding)
    _, one = _run(torch_mod, desc, H, e.astype(np.float32), variant="lds", tile=tile,
                  block=(4, 4, 1), nb=16)
    assert rel_l2(one, ref) <= TOL_L2
    assert rel_l2(got, one) <= 4e-6


@pytest.mark.parametrize("e_type", ["bf16", "i32"])
def test_storage_types(torch_mod, e_type):
    torch = torch_mod
    desc = _desc()
    H, e = _data(desc, 9)
    if e_type == "bf16":
        e_in = torch.from_numpy(e.astype(np.float32)).to(torch.bfloat16)
        e_ref = e_in.float().numpy().astype(np.float64)
        x = e_in.float().numpy()
    else:
        e_ref = e
        x = e.astype(np.int32)
    _, got = _run(torch, desc, H, x, e_type=e_type)
    assert rel_l2(got, oracle.das(desc, e_ref)) <= TOL_L2


@pytest.mark.parametrize("variant", ["lds2", "lds"])
def test_grid_through_the_array_plane(torch_mod, variant):
    # depth step 0.3 mm from z = -0.15 mm: a lane's first point lies behind the
    # array (output exactly 0) and its second point in front of it
    desc = describe("hercules", (12, 10), (0.25 * MM, 0.3 * MM), 8, 10, 600, 25e6, 6e6,
                    (13, 9, 29), (-2 * MM, -1.5 * MM, -0.15 * MM), (2.2 * MM, 1.2 * MM, 8.25 * MM),
                    t0=0.3e-6, f_number=0.8, tx_elements=[0, 3, 4, 6, 7, 8, 10, 11],
                    channel_map=np.random.default_rng(2).permutation(10))
    H, e = _data(desc, 12)
    ref = oracle.das(desc, e)
    assert np.all(ref[..., 0] == 0)
    _, got = _run(torch_mod, desc, H, e.astype(np.float32), variant=variant, block=(2, 2, 2),
                  nb=16)
    assert np.all(got[..., 0] == 0)
    assert rel_l2(got, ref) <= TOL_L2


def test_diverging_transmit(torch_mod):
    desc = _desc(focal_depth=-6 * MM)
    H, e = _data(desc, 10)
    _, got = _run(torch_mod, desc, H, e.astype(np.float32), block=(2, 2, 1), nb=16)
    assert rel_l2(got, oracle.das(desc, e)) <= TOL_L2


def test_rejected_where_unsupported(torch_mod):
    # two depth points per lane: HERCULES and FORCES with real data only
    tpw = describe("tpw", (12, 10), (0.25 * MM, 0.3 * MM), 8, 10, 600, 25e6, 6e6,
                   (13, 9, 29), (-2 * MM, -1.5 * MM, 1 * MM), (2.2 * MM, 1.2 * MM, 9 * MM),
                   tx_angles=np.deg2rad(np.linspace(-10, 10, 8)))
    p = bfm.Plan(tpw, None)
    with pytest.raises(bfm.BfError):
        p.set_das_config("lds2", (2, 2, 2), 8)
    _, _, iq = synth.configs.iq_frontend(synth.configs.workload(0))
    p = bfm.Plan(iq, synth.hadamard_sylvester(32))
    assert p.info()["variant"] != 2
    with pytest.raises(bfm.BfError):
        p.set_das_config("lds2", (2, 1, 4), 16)
    _, _, iq = synth.configs.iq_frontend(_desc())
    p = bfm.Plan(iq, synth.hadamard_sylvester(8))
    assert p.info()["variant"] != 2
    with pytest.raises(bfm.BfError):
        p.set_das_config("lds2", (2, 2, 3), 16)


def test_workload1_default_sampled(torch_mod):
    torch = torch_mod
    desc, H, rf, _ = synth.make_inputs(1)
    plan = bfm.Plan(desc, H)
    info = plan.info()
    assert info["variant"] == 2 and info["block"] == (2, 2, 3)
    img = plan.das(plan.decode(torch.from_numpy(rf).cuda())).cpu().numpy().reshape(-1)
    vox = sample_voxels(img.size, 3000, seed=21)
    ref = oracle.das_points(desc, oracle.decode(H, rf), vox)
    assert rel_l2(img[vox], ref) <= TOL_L2


def _herc_frames(seed, n=4):
    rng = np.random.default_rng(seed)
    out = []
    for f in range(n):
        n_tx = int(rng.choice([8, 16, 32]))
        cols = np.sort(rng.choice(32, size=n_tx, replace=False))
        d = describe("hercules", (32, 16), (0.2 * MM, 0.2 * MM), n_tx, 16, 700, 20e6, 5e6,
                     (19, 13 + f, 27 + 2 * f), (-2.5 * MM, -1.5 * MM, 3 * MM),
                     (2.5 * MM, 1.5 * MM, 9 * MM), tx_elements=cols)
        H = synth.hadamard_sylvester(n_tx)
        pts = rng.uniform([-2 * MM, -1 * MM, 5 * MM], [2 * MM, 1 * MM, 8 * MM], size=(5, 3))
        out.append((d, H, synth.acquire(d, pts, np.ones(5), rng, H=H)))
    return out


def test_batched_two_points_and_graph(torch_mod):
    torch = torch_mod
    frames = _herc_frames(4)
    descs, Hs = [f[0] for f in frames], [f[1] for f in frames]
    rfs = [torch.from_numpy(f[2]).cuda() for f in frames]
    results = {}
    for variant in ("lds2", "lds"):
        bp = bfm.BatchPlan(descs, Hs)
        bp.set_das_config(variant, (2, 2, 3), 40)
        outs = [torch.empty(s, device="cuda") for s in bp.out_shapes]
        bp.run(rfs, outs)
        torch.cuda.synchronize()
        results[variant] = [o.cpu().numpy() for o in outs]
        if variant == "lds2":
            for rep in range(2):
                outs2 = [torch.full(s, float("nan"), device="cuda") for s in bp.out_shapes]
                bp.graph_launch(rfs, outs2)
                junk = torch.randn(1000, device="cuda").sum()
                torch.cuda.synchronize()
                assert torch.isfinite(junk)
                for o, r in zip(outs2, results["lds2"]):
                    assert np.array_equal(o.cpu().numpy(), r), rep
            with pytest.raises(bfm.BfError):     # configuration is fixed once launched
                bp.set_das_config("lds", (2, 2, 3), 40)
    for (d, H, rf), a, b in zip(frames, results["lds2"], results["lds"]):
        ref = oracle.das(d, oracle.decode(H, rf))
        assert rel_l2(a, ref) <= TOL_L2
        assert rel_l2(a, b) <= 1e-6


def _plane(interp="cubic", nz=53, f_number=1.0, along_y=False):
    """A small FORCES plane (x-z, or y-z through a frame rotated about z)."""
    M = None
    if along_y:
        M = synth.configs.centered_xdc((12, 10), (0.25 * MM, 0.25 * MM))
        M[:3, :3] = [[0, 1, 0], [-1, 0, 0], [0, 0, 1]]
        dims, g0, g1 = (1, 37, nz), (0, -2 * MM, 1 * MM), (0, 2.2 * MM, 9 * MM)
    else:
        dims, g0, g1 = (37, 1, nz), (-2 * MM, 0, 1 * MM), (2.2 * MM, 0, 9 * MM)
    return describe("forces", (12, 10), (0.25 * MM, 0.25 * MM), 8, 12, 600, 25e6, 6e6, dims,
                    g0, g1, t0=0.3e-6, f_number=f_number, interp=interp,
                    tx_elements=[0, 3, 4, 6, 7, 8, 10, 11],
                    channel_map=np.random.default_rng(2).permutation(12), xdc=M)


@pytest.mark.parametrize("interp, nz, tile, block, nb, kw", [
    ("cubic", 53, (5, 0, 1), (2, 1, 4), 16, {}),
    ("cubic", 2, (5, 0, 1), (2, 1, 4), 16, {}),
    ("cubic", 1, (3, 0, 3), (2, 1, 2), 8, {}),
    ("linear", 41, (5, 0, 1), (2, 1, 4), 4, dict(f_number=0.0)),
    ("nearest", 53, (4, 0, 2), (4, 1, 4), 24, {}),
    ("cubic", 53, (0, 5, 1), (1, 2, 4), 16, dict(along_y=True)),
])
def test_forces_plane_two_points_matches_oracle(torch_mod, interp, nz, tile, block, nb, kw):
    """FORCES planes with two depth points per lane (variant lds2):
    odd and tiny depth counts, several tiles, workgroups and batches, linear
    and nearest reads, F# 0, the y-z plane of a frame rotated about z; and
    the one-point kernel gives the same image to FP32 rounding (of the
    window positions, which depend on the box)."""
    torch = torch_mod
    d = _plane(interp, nz, **kw)
    H, e = _data(d, 11)
    plan = bfm.Plan(d, H, tile=tile)
    block = (block[0], 1, block[2]) if not kw.get("along_y") else (1, block[1], block[2])
    plan.set_das_config("lds2", block, nb)
    # (a depth count of 2 spaces the points 8 mm apart: the boxes' windows
    # exceed LDS and the gather kernel runs, as bf_plan_get_info reports)
    assert plan.info()["variant"] == (1 if nz == 2 else 2)
    et = torch.from_numpy(e.astype(np.float32)).cuda()
    got = plan.das(et).cpu().numpy()
    ref = oracle.das(d, e)
    tol = TOL_NEAREST if interp == "nearest" else TOL_L2
    assert rel_l2(got, ref) <= tol
    p1 = bfm.Plan(d, H, tile=tile)
    p1.set_das_config("lds", block, nb)
    one = p1.das(et).cpu().numpy()
    # (cubic and linear reads: the two kernels' boxes differ, and with them
    # the window-start parts folded into the FP32 positions; the agreement
    # bound is the one of the plane kernel's tilings, test_das_tiles_agree)
    assert rel_l2(got, one) <= (tol if interp == "nearest" else 4e-6)


@pytest.mark.parametrize("e_type", ["bf16", "i32"])
def test_forces_plane_two_points_storage_types(torch_mod, e_type):
    torch = torch_mod
    d = _plane()
    H, e = _data(d, 13)
    plan = bfm.Plan(d, H, e_type=e_type)
    plan.set_das_config("lds2", (2, 1, 4), 16)
    assert plan.info()["variant"] == 2
    if e_type == "bf16":
        et = torch.from_numpy(e.astype(np.float32)).to(torch.bfloat16).cuda()
        ref = oracle.das(d, et.float().cpu().numpy().astype(np.float64))
    else:
        et = torch.from_numpy(np.rint(e).astype(np.int32)).cuda()
        ref = oracle.das(d, e)
    assert rel_l2(plan.das(et).cpu().numpy(), ref) <= TOL_L2


def test_forces_plane_two_points_adjoint(torch_mod):
    """Both adjoint gradients of a plane with two depth points per lane
    against the oracle (dL/dc: the FP64 analytic derivative; dL/de: the
    transpose of the FP64 beamforming map)."""
    torch = torch_mod
    d = _plane()
    H, e = _data(d, 17)
    plan = bfm.Plan(d, H)
    plan.set_das_config("lds2", (2, 1, 4), 16)
    et = torch.from_numpy(e.astype(np.float32)).cuda()
    G = np.random.default_rng(5).normal(size=plan.out_shape).astype(np.float32).astype(np.float64)
    ge, gc = plan.das_adjoint(et, torch.from_numpy(G.astype(np.float32)).cuda())
    ref_c = float(np.sum(G * oracle.das_dc(d, e)))
    assert abs(float(gc) - ref_c) <= 1e-4 * abs(ref_c)
    assert rel_l2(ge.cpu().numpy(), oracle.das_adjoint_e(d, G)) <= TOL_L2
