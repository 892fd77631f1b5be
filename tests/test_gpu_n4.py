"""Additional transmit models on the GPU against the FP64 oracle: tilted plane
waves (TPW) and virtual line sources (VLS) on row-column volumes, the
diverging-wave HERCULES transmit, unencoded acquisitions, their adjoints, the
full-size workloads (sampled points) and a cross-plane parameter-set batch
(two FORCES planes with different orientations plus a volume, in one batched
launch and one captured graph).  Tolerances as for the RF path (relative L2
1e-5; nearest reads 1e-4)."""
import numpy as np
import pytest

import oracle
import paper_2512_11086_amd as bfm
import synth
from synth.configs import MM, describe
from tests.helpers import rel_l2, sample_voxels

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _small(mode, interp="cubic", **kw):
    n = 16
    extra = {}
    if mode == "tpw":
        extra["tx_angles"] = np.deg2rad(np.linspace(-12, 12, n))
    return describe(mode, (n, n), (0.3 * MM, 0.3 * MM), n, n, 700, 20e6, 5e6, (21, 19, 37),
                    (-2 * MM, -1.5 * MM, 2 * MM), (2 * MM, 1.5 * MM, 9 * MM), interp=interp,
                    t0=0.5e-6, **extra, **kw)


def _data(desc, seed, encoded):
    rng = np.random.default_rng(seed)
    pts = rng.uniform([-1.5 * MM, -1 * MM, 4 * MM], [1.5 * MM, 1 * MM, 8 * MM], size=(6, 3))
    H = synth.hadamard_sylvester(desc["n_tx"]) if encoded else None
    rf = synth.acquire(desc, pts, np.ones(6), rng, H=H, encoded=encoded)
    return H, rf


def _decode_oracle(H, rf):
    return oracle.decode(np.eye(rf.shape[0], dtype=np.int8) if H is None else H, rf)


CASES = [("tpw", {}), ("vls", dict(focal_depth=-4 * MM)), ("vls", dict(focal_depth=6 * MM)),
         ("hercules", dict(focal_depth=-10 * MM))]


@pytest.mark.parametrize("mode, kw", CASES)
@pytest.mark.parametrize("interp", ["nearest", "linear", "cubic"])
def test_small_volumes_match_oracle(torch_mod, mode, kw, interp):
    torch = torch_mod
    d = _small(mode, interp, **kw)
    H, rf = _data(d, 3, encoded=mode == "hercules")
    ref = oracle.das(d, _decode_oracle(H, rf))
    plan = bfm.Plan(d, H)
    for v in ("gather", "lds"):
        if v == "lds":
            plan.set_das_config("lds", (2, 2, 1), 8)
            assert plan.info()["variant"] == 0
        else:
            plan.set_das_config("gather", (1, 1, 1), 4)
        got = plan.das(plan.decode(torch.from_numpy(rf).cuda())).cpu().numpy()
        err = rel_l2(got, ref)
        assert err <= (1e-4 if interp == "nearest" else 1e-5), (v, err)


@pytest.mark.parametrize("mode, kw", CASES[:3])
@pytest.mark.parametrize("tile, block, nb", [
    ((3, 3, 0), (2, 2, 3), 48), ((2, 2, 2), (1, 1, 1), 4), ((1, 1, 4), (2, 2, 2), 16),
    ((0, 0, 6), (1, 1, 2), 64), ((3, 3, 0), (4, 2, 1), 32),
])
def test_separable_lds_configurations(torch_mod, mode, kw, tile, block, nb):
    # row-column volumes on the LDS kernel: window bounds per transmit model
    # (tilted plane, virtual line behind or in front of the volume), batches
    # of 4 rows x nb/4 transmits, several lane tiles and workgroup shapes
    torch = torch_mod
    d = _small(mode, **kw)
    H, rf = _data(d, 11, encoded=False)
    ref = oracle.das(d, _decode_oracle(H, rf))
    plan = bfm.Plan(d, H, tile=tile)
    plan.set_das_config("lds", block, nb)
    got = plan.das(plan.decode(torch.from_numpy(rf).cuda())).cpu().numpy()
    assert rel_l2(got, ref) <= 1e-5, (tile, block, nb, plan.info())


@pytest.mark.parametrize("mode, kw", [("tpw", {}), ("vls", dict(focal_depth=5.1 * MM)),
                                      ("vls", dict(focal_depth=2.6 * MM))])
def test_separable_lds_volume_through_the_focus_and_array_plane(torch_mod, mode, kw):
    # depths from -0.5 mm (behind the array: zero output) past a virtual line
    # inside the volume (VLS: converging above, diverging below it; the
    # transmit path jumps at the line's depth, which no LDS box may straddle)
    torch = torch_mod
    n = 16
    extra = dict(tx_angles=np.deg2rad(np.linspace(-12, 12, n))) if mode == "tpw" else {}
    d = describe(mode, (n, n), (0.3 * MM, 0.3 * MM), n, n, 700, 20e6, 5e6, (17, 15, 41),
                 (-2 * MM, -1.5 * MM, -0.5 * MM), (2 * MM, 1.5 * MM, 9.5 * MM), t0=0.5e-6,
                 **extra, **kw)
    H, rf = _data(d, 12, encoded=False)
    ref = oracle.das(d, _decode_oracle(H, rf))
    plan = bfm.Plan(d, H)
    plan.set_das_config("lds", (2, 2, 2), 16)
    got = plan.das(plan.decode(torch.from_numpy(rf).cuda())).cpu().numpy()
    assert np.all(got[..., :3] == 0)
    assert rel_l2(got, ref) <= 1e-5


def test_unencoded_decode_is_exact_copy(torch_mod):
    torch = torch_mod
    d = _small("tpw")
    rng = np.random.default_rng(1)
    rf = rng.integers(-32768, 32767, size=(16, 16, 700)).astype(np.int16)
    for algo in ("mfma", "fma"):
        plan = bfm.Plan(d, None, decode_algo=algo)
        e = plan.decode(torch.from_numpy(rf).cuda()).cpu().numpy()
        np.testing.assert_array_equal(e, rf.astype(np.float32))


@pytest.mark.parametrize("mode, kw", CASES)
def test_adjoint_matches_oracle(torch_mod, mode, kw):
    torch = torch_mod
    d = _small(mode, **kw)
    H, rf = _data(d, 5, encoded=mode == "hercules")
    e64 = _decode_oracle(H, rf)
    plan = bfm.Plan(d, H)
    e = torch.from_numpy(e64.astype(np.float32)).cuda()
    G = np.random.default_rng(2).normal(size=plan.out_shape)
    ge, gc = plan.das_adjoint(e, torch.from_numpy(G.astype(np.float32)).cuda())
    assert rel_l2(ge.cpu().numpy(), oracle.das_adjoint_e(d, G)) <= 1e-5
    ref_c = float(np.sum(G * oracle.das_dc(d, e64)))
    assert abs(gc.item() - ref_c) <= 1e-4 * abs(ref_c) + 1e-6 * np.abs(G).sum()


@pytest.mark.parametrize("k", [5, 6, 7])
def test_full_size_workloads_sampled(torch_mod, k):
    torch = torch_mod
    desc, H, rf, _ = synth.make_inputs(k)
    plan = bfm.Plan(desc, H)
    img = plan.das(plan.decode(torch.from_numpy(rf).cuda())).cpu().numpy().reshape(-1)
    vox = sample_voxels(img.size, 256, k)
    ref = oracle.das_points(desc, _decode_oracle(H, rf), vox)
    assert rel_l2(img[vox], ref) <= 1e-5, rel_l2(img[vox], ref)


def test_row_column_batch_and_graph(torch_mod):
    # TPW and VLS frames (LDS kernel, persistent path) with a FORCES plane in
    # one batch: oracle parity per frame, graph replays equal the eager run
    torch = torch_mod
    frames = []
    for k, (mode, kw) in enumerate([("tpw", {}), ("vls", dict(focal_depth=-4 * MM)),
                                    ("vls", dict(focal_depth=6.1 * MM))]):
        d = _small(mode, **kw)
        frames.append((d,) + _data(d, 20 + k, encoded=False))
    descs = [f[0] for f in frames]
    bp = bfm.BatchPlan(descs, [f[1] for f in frames])      # unencoded: no Hadamard matrix
    rf_d = [torch.from_numpy(f[2]).cuda() for f in frames]
    outs = [torch.empty(s, device="cuda") for s in bp.out_shapes]
    bp.run(rf_d, outs)
    torch.cuda.synchronize()
    for (d, H, rf), o in zip(frames, outs):
        ref = oracle.das(d, _decode_oracle(H, rf))
        assert rel_l2(o.cpu().numpy(), ref) <= 1e-5, d["mode"]
    eager = [o.clone() for o in outs]
    for rep in range(2):
        outs2 = [torch.full(s, float("nan"), device="cuda") for s in bp.out_shapes]
        bp.graph_launch(rf_d, outs2)
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for o, r in zip(outs2, eager):
            assert torch.equal(o, r), rep


def test_cross_plane_batch_and_graph(torch_mod):
    # two orthogonal FORCES planes (rows as the second plane's elements via a
    # rotated transform) and a diverging HERCULES volume in one batched plan
    torch = torch_mod
    descs, Hs, rfs, _ = synth.make_inputs(8)
    vol = _small("hercules", focal_depth=-10 * MM)
    Hv, rfv = _data(vol, 9, encoded=True)
    descs, Hs, rfs = descs + [vol], Hs + [Hv], rfs + [rfv]
    bp = bfm.BatchPlan(descs, Hs)
    rf_d = [torch.from_numpy(r).cuda() for r in rfs]
    outs = [torch.empty(s, device="cuda") for s in bp.out_shapes]
    bp.run(rf_d, outs)
    torch.cuda.synchronize()
    # each 256 x 256 plane (64 boxes x 8 channel groups) fills the GPU with its
    # own LDS launch; the small volume takes the persistent launch
    paths = [bp.frame_info(f)["das_path"] for f in range(len(descs))]
    assert paths[:2] == ["frame_lds", "frame_lds"] and paths[2] != "gather", paths
    eager = [o.clone() for o in outs]
    for f, (d, H, rf) in enumerate(zip(descs, Hs, rfs)):
        e64 = oracle.decode(H, rf)
        got = outs[f].cpu().numpy().reshape(-1)
        vox = sample_voxels(got.size, 300, f)
        ref = oracle.das_points(d, e64, vox)
        assert rel_l2(got[vox], ref) <= 1e-5, (f, rel_l2(got[vox], ref))
    for rep in range(3):
        outs2 = [torch.full(s, float("nan"), device="cuda") for s in bp.out_shapes]
        bp.graph_launch(rf_d, outs2)
        junk = torch.randn(4096, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for o, r in zip(outs2, eager):
            assert torch.equal(o, r), rep
