"""Batched persistent path, hipGraph replay and autotuner (GPU).

A batch of frames with different modes, transmit subsets and grids goes
through bf_batch_run (persistent kernels) and bf_graph_launch (the same
kernels captured once, replayed with new buffers).  Every frame is checked
against the FP64 oracle, the batch against the per-frame plans, and every
graph replay against an eager run on the same inputs, with the program's own
eager work and synchronisations between replays.
"""
import numpy as np
import pytest

import oracle
import paper_2512_11086_amd as bfm
import synth
from synth.configs import MM, describe
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _frames(seed=0, n=6):
    rng = np.random.default_rng(seed)
    out = []
    for f in range(n):
        n_tx = int(rng.choice([4, 8, 16, 32]))
        cols = np.sort(rng.choice(32, size=n_tx, replace=False))
        if f % 2 == 0:
            d = describe("forces", (32, 16), (0.2 * MM, 0.2 * MM), n_tx, 32, 700, 20e6, 5e6,
                         (40 + 3 * f, 1, 57), (-3 * MM, 0, 4 * MM), (3 * MM, 0, 14 * MM),
                         tx_elements=cols)
        else:
            d = describe("hercules", (32, 16), (0.2 * MM, 0.2 * MM), n_tx, 16, 700, 20e6, 5e6,
                         (19, 13 + f, 27), (-2.5 * MM, -1.5 * MM, 3 * MM), (2.5 * MM, 1.5 * MM, 9 * MM),
                         tx_elements=cols)
        H = synth.hadamard_sylvester(n_tx)
        pts = rng.uniform([-2 * MM, -1 * MM, 5 * MM], [2 * MM, 1 * MM, 8 * MM], size=(5, 3))
        if d["mode"] == "forces":
            pts[:, 1] = 0
        rf = synth.acquire(d, pts, np.ones(5), rng, H=H)
        out.append((d, H, rf))
    return out


def test_batch_matches_oracle_and_per_frame(torch_mod):
    torch = torch_mod
    frames = _frames()
    bp = bfm.BatchPlan([f[0] for f in frames], [f[1] for f in frames])
    rfs = [torch.from_numpy(f[2]).cuda() for f in frames]
    outs = [torch.empty(s, device="cuda") for s in bp.out_shapes]
    bp.run(rfs, outs)
    torch.cuda.synchronize()
    for (d, H, rf), o in zip(frames, outs):
        ref = oracle.das(d, oracle.decode(H, rf))
        assert rel_l2(o.cpu().numpy(), ref) <= 1e-5
        p = bfm.Plan(d, H)
        single = p.das(p.decode(torch.from_numpy(rf).cuda()))
        assert rel_l2(o.cpu().numpy(), single.cpu().numpy()) <= 1e-6


def test_graph_replays_match_eager(torch_mod):
    torch = torch_mod
    frames = _frames(seed=3)
    bp = bfm.BatchPlan([f[0] for f in frames], [f[1] for f in frames])
    sets = []
    for k in range(3):     # three input sets: the frames' data scaled and shifted
        rfs = [torch.from_numpy(np.roll(f[2], 7 * k, axis=2) // (k + 1)).cuda() for f in frames]
        sets.append(rfs)
    eager = []
    for rfs in sets:
        outs = [torch.empty(s, device="cuda") for s in bp.out_shapes]
        bp.run(rfs, outs)
        torch.cuda.synchronize()
        eager.append([o.clone() for o in outs])
    for rep in range(2):
        for k, rfs in enumerate(sets):
            outs = [torch.full(s, float("nan"), device="cuda") for s in bp.out_shapes]
            bp.graph_launch(rfs, outs)
            junk = torch.randn(1000, device="cuda").sum()      # eager work between replays
            torch.cuda.synchronize()
            assert torch.isfinite(junk)
            for o, ref in zip(outs, eager[k]):
                assert torch.equal(o, ref), (rep, k)


def test_batch_rejects_bad_arguments(torch_mod):
    torch = torch_mod
    frames = _frames(n=2)
    bp = bfm.BatchPlan([f[0] for f in frames], [f[1] for f in frames])
    rfs = [torch.from_numpy(f[2]).cuda() for f in frames]
    with pytest.raises(bfm.BfError):
        bfm._lib.check(bfm._lib.lib().bf_batch_run(bp._h, None, None, None))
    outs = [torch.empty(s, device="cuda") for s in bp.out_shapes]
    bp.run(rfs, outs)
    torch.cuda.synchronize()


def test_autotune_choice_is_valid_and_cached(torch_mod, tmp_path):
    torch = torch_mod
    (d, H, rf) = _frames(seed=5, n=2)[1]
    p = bfm.Plan(d, H)
    cache = str(tmp_path / "tune.txt")
    info = p.autotune(cache)
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and lines[0].split()[0].startswith("gfx950")
    e = p.decode(torch.from_numpy(rf).cuda())
    ref = oracle.das(d, oracle.decode(H, rf))
    assert rel_l2(p.das(e).cpu().numpy(), ref) <= 1e-5
    p2 = bfm.Plan(d, H)
    info2 = p2.autotune(cache)      # served from the cache
    assert info2["tile"] == info["tile"] and info2["block"] == info["block"]
    assert len(open(cache).read().strip().splitlines()) == 1


def _big_frames(seed):
    # enough LDS boxes per kernel class (>= 2 per CU) for the persistent path:
    # four FORCES planes of 512 x 256 points and four HERCULES volumes of
    # 64 x 64 x 60 points (two depth points per lane)
    rng = np.random.default_rng(seed)
    out = []
    for f in range(8):
        n_tx = 32
        cols = np.arange(32)
        if f % 2 == 0:
            d = describe("forces", (32, 16), (0.2 * MM, 0.2 * MM), n_tx, 32, 800, 20e6, 5e6,
                         (512, 1, 256), (-3.2 * MM, 0, 3 * MM), (3.2 * MM, 0, 14 * MM),
                         tx_elements=cols)
        else:
            d = describe("hercules", (32, 16), (0.2 * MM, 0.2 * MM), n_tx, 16, 800, 20e6, 5e6,
                         (64, 64, 60), (-3 * MM, -1.5 * MM, 3 * MM), (3 * MM, 1.5 * MM, 10 * MM),
                         tx_elements=cols)
        H = synth.hadamard_sylvester(n_tx)
        pts = rng.uniform([-2 * MM, -1 * MM, 4 * MM], [2 * MM, 1 * MM, 9 * MM], size=(5, 3))
        if d["mode"] == "forces":
            pts[:, 1] = 0
        rf = synth.acquire(d, pts, np.ones(5), rng, H=H)
        out.append((d, H, rf))
    return out


def test_persistent_lds_classes_and_graph(torch_mod):
    torch = torch_mod
    frames = _big_frames(7)
    bp = bfm.BatchPlan([f[0] for f in frames], [f[1] for f in frames])
    rfs = [torch.from_numpy(f[2]).cuda() for f in frames]
    outs = [torch.empty(s, device="cuda") for s in bp.out_shapes]
    bp.run(rfs, outs)
    torch.cuda.synchronize()
    for f, ((d, H, rf), o) in enumerate(zip(frames, outs)):
        # the four volumes (80 boxes each) share a persistent launch with
        # channel-group items; each plane's own launch (128 boxes x 4 channel
        # groups) fills the GPU, so the planes run their own LDS launches
        want = "frame_lds" if d["mode"] == "forces" else "persistent_lds"
        assert bp.frame_info(f)["das_path"] == want, (f, bp.frame_info(f))
        ref = oracle.das(d, oracle.decode(H, rf))
        assert rel_l2(o.cpu().numpy(), ref) <= 1e-5, d["mode"]
    eager = [o.clone() for o in outs]
    for rep in range(2):
        outs2 = [torch.full(s, float("nan"), device="cuda") for s in bp.out_shapes]
        bp.graph_launch(rfs, outs2)
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for o, r in zip(outs2, eager):
            assert torch.equal(o, r), rep


def test_graph_reuses_staged_pointers(torch_mod):
    """A call with the same buffers on the same stream as the last pointer
    copy stages nothing; buffers that change (and change back) are staged
    again, whichever entry point made the last copy."""
    torch = torch_mod
    frames = _frames(seed=11, n=2)
    bp = bfm.BatchPlan([f[0] for f in frames], [f[1] for f in frames])
    rfs = [torch.from_numpy(f[2]).cuda() for f in frames]
    eager = [torch.empty(s, device="cuda") for s in bp.out_shapes]
    bp.run(rfs, eager)
    a = [torch.empty(s, device="cuda") for s in bp.out_shapes]
    b = [torch.empty(s, device="cuda") for s in bp.out_shapes]
    calls = [(bp.graph_launch, a), (bp.graph_launch, a), (bp.graph_launch, b),
             (bp.run, b), (bp.graph_launch, a), (bp.run, a), (bp.graph_launch, a)]
    for fn, outs in calls:
        for o in outs:
            o.fill_(float("nan"))
        fn(rfs, outs)
        torch.cuda.synchronize()
        for o, r in zip(outs, eager):
            assert torch.equal(o, r)


def test_batch_autotune_keeps_persistent_classes(torch_mod, tmp_path):
    """Tuning a batch plan keeps every kernel class on one persistent launch
    (same workgroup size and kernel, so no class splits) and every frame on
    an LDS path, caches its choice under batch keys, and the tuned plan still
    matches the oracle."""
    torch = torch_mod
    frames = _big_frames(9)
    rfs = [torch.from_numpy(f[2]).cuda() for f in frames]
    untuned = bfm.BatchPlan([f[0] for f in frames], [f[1] for f in frames])
    untuned.run(rfs, [torch.empty(s, device="cuda") for s in untuned.out_shapes])
    torch.cuda.synchronize()
    before = [untuned.frame_info(f) for f in range(len(frames))]
    bp = bfm.BatchPlan([f[0] for f in frames], [f[1] for f in frames])
    cache = str(tmp_path / "tune.txt")
    bp.autotune(cache)
    keys = [ln.split()[0] for ln in open(cache).read().strip().splitlines()]
    assert len(keys) == 2 and all(k.endswith("|batch") for k in keys), keys
    outs = [torch.empty(s, device="cuda") for s in bp.out_shapes]
    bp.run(rfs, outs)
    torch.cuda.synchronize()
    for f, ((d, H, rf), o) in enumerate(zip(frames, outs)):
        fi = bp.frame_info(f)
        # (a tuned tile can change a frame's box count and with it whether its
        # own launch fills the GPU: persistent <-> own LDS launch)
        assert fi["das_path"] != "gather", (f, fi)
        if fi["das_path"] == before[f]["das_path"] == "persistent_lds":
            assert fi["das_class"] == before[f]["das_class"], (f, fi, before[f])
        ref = oracle.das(d, oracle.decode(H, rf))
        assert rel_l2(o.cpu().numpy(), ref) <= 1e-5, d["mode"]


def test_workload4_all_frames_match_oracle():
    """Full size, the whole batched stream: all 64 frames (planes and volumes,
    every 16-, 32-, 64- and 128-transmit subset) through one batch plan and
    its captured graph, against the FP64 oracle on 400 sampled points per
    frame (relative L2 1e-5).  The persistent run and the graph replay must
    agree bit for bit, and every frame must take the persistent LDS path."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    descs, Hs, rfs, info = synth.make_inputs(4)
    kinds = [k for k, _ in info["plan"]]
    assert len(descs) == 64 and {d["n_tx"] for d in descs} == {16, 32, 64, 128}
    bp = bfm.BatchPlan(descs, Hs)
    rf_d = [torch.from_numpy(r).cuda() for r in rfs]
    outs = [torch.empty(s, device="cuda") for s in bp.out_shapes]
    bp.run(rf_d, outs)
    outs_g = [torch.full(s, float("nan"), device="cuda") for s in bp.out_shapes]
    bp.graph_launch(rf_d, outs_g)
    torch.cuda.synchronize()
    rng = np.random.default_rng(44)
    worst = 0.0
    for i, d in enumerate(descs):
        fi = bp.frame_info(i)
        assert fi["das_path"] == "persistent_lds", (i, fi)
        assert torch.equal(outs_g[i], outs[i]), i
        got = outs_g[i].cpu().numpy().reshape(-1).astype(np.float64)
        vox = np.sort(rng.choice(got.size, 400, replace=False))
        ref = oracle.das_points(d, oracle.decode(Hs[i], rfs[i]), vox)
        err = rel_l2(got[vox], ref)
        worst = max(worst, err)
        print(f"workload 4 frame {i:2d} ({kinds[i]}, {d['n_tx']:3d} tx, {fi['channel_groups']} "
              f"channel groups): rel L2 {err:.2e}", flush=True)
        assert err <= 1e-5, i
    print(f"workload 4: worst rel L2 over 64 frames {worst:.2e}")
