"""Stacks of frames (bf_das_frames, bf_das_adjoint_frames).

A stack of F frames of one plan is beamformed one launch per frame, and its
LDS adjoint takes the whole stack in one launch per gradient (grid z =
frame).  Per frame the kernel body, the channel groups and the order of
every sum are those of the single-frame call, so:
  * out[f] equals bf_das on frame f alone bit for bit, and the stack matches
    the FP64 oracle at the single-frame bound (relative L2 1e-5);
  * grad_c[f] equals bf_das_adjoint's grad_c on frame f bit for bit (FP64
    workgroup partials, summed per frame in a fixed order);
  * grad_e[f] equals it up to the order of FP32 atomics across workgroups
    (relative L2 1e-6), and matches oracle.das_adjoint_e at 1e-5.
Kernels that run frame by frame (gather variant, nearest reads) must give the
same results.  The full-size case is the differentiable FORCES workload
(8 frames, 256 x 256 plane, 64 transmits x 64 channels x 2048 samples) in the
configuration the benchmark times.
"""
import numpy as np
import pytest

import oracle
import paper_2512_11086_amd as bfm
import synth
from paper_2512_11086_amd import _lib
from paper_2512_11086_amd.autofocus import focus_loss
from synth.configs import MM, describe
from tests.helpers import hadamard, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _desc(mode, interp, **kw):
    n_ch = 12 if mode == "forces" else 10
    dims = (37, 1, 53) if mode == "forces" else (13, 9, 29)
    if mode == "tpw":
        kw.setdefault("tx_angles", np.deg2rad(np.linspace(-10, 10, 8)))
    return describe(mode, (12, 10), (0.25 * MM, 0.3 * MM), 8, n_ch, 600, 25e6, 6e6, dims,
                    (-2 * MM, -1.5 * MM, 1.0 * MM), (2.2 * MM, 1.2 * MM, 9 * MM), t0=0.3e-6,
                    f_number=1.0, interp=interp, tx_elements=[0, 3, 4, 6, 7, 8, 10, 11],
                    channel_map=np.random.default_rng(2).permutation(n_ch), **kw)


def _frames(desc, n, seed):
    """n decoded frames of different scatterers, (H, [n, n_tx, n_ch, S] FP64);
    the row-column models (TPW, VLS) are acquired unencoded (H None)."""
    encoded = desc["mode"] in ("forces", "hercules")
    H = hadamard(desc["n_tx"], "scrambled", seed=seed) if encoded else None
    es = []
    for f in range(n):
        rng = np.random.default_rng(seed + 17 * f)
        pts = rng.uniform([-2 * MM, -1 * MM, 1.5 * MM], [2 * MM, 1 * MM, 8 * MM], size=(6, 3))
        if desc["mode"] == "forces":
            pts[:, 1] = 0
        rf = synth.acquire(desc, pts, rng.uniform(0.5, 1.5, 6), rng, H=H, encoded=encoded)
        es.append(oracle.decode(np.eye(desc["n_tx"], dtype=np.int8) if H is None else H, rf))
    return H, np.stack(es)


CASES = [("forces", "cubic", "lds"), ("forces", "linear", "lds"), ("hercules", "cubic", "lds"),
         ("hercules", "cubic", "lds2"), ("hercules", "linear", "lds"),
         ("forces", "cubic", "gather"), ("hercules", "nearest", "lds")]


@pytest.mark.parametrize("mode, interp, variant", CASES)
def test_das_frames_matches_single_frames_and_oracle(torch_mod, mode, interp, variant):
    torch = torch_mod
    d = _desc(mode, interp)
    H, e = _frames(d, 3, 31)
    plan = bfm.Plan(d, H)
    if variant == "gather":
        plan.set_das_config("gather", (1, 1, 1), 4)
    elif variant == "lds2":
        plan.set_das_config("lds2", (2, 2, 1), 16)
    et = torch.from_numpy(e.astype(np.float32)).cuda()
    stack = plan.das(et).cpu().numpy()
    assert stack.shape == (3,) + plan.out_shape
    for f in range(3):
        one = plan.das(et[f]).cpu().numpy()
        assert np.array_equal(stack[f], one), f"frame {f} differs from its single-frame image"
    bound = 1e-4 if interp == "nearest" else 1e-5
    ref = oracle.das(d, e[2])        # the last frame: offsets of every array
    assert rel_l2(stack[2], ref) < bound


def test_das_frames_partial_images(torch_mod):
    """A small grid splits the channel sum into groups (partial images);
    stacks of every size, larger and smaller than the one before, give each
    frame's own image."""
    torch = torch_mod
    d = _desc("forces", "cubic")
    H, e = _frames(d, 5, 41)
    plan = bfm.Plan(d, H)
    et = torch.from_numpy(e.astype(np.float32)).cuda()
    singles = [plan.das(et[f]).cpu().numpy() for f in range(5)]
    for n in (2, 5, 3, 1):
        stack = plan.das(et[:n].contiguous()).cpu().numpy()
        for f in range(n):
            assert np.array_equal(stack[f], singles[f]), (n, f)


@pytest.mark.parametrize("mode, interp, kw", [
    ("forces", "cubic", {}), ("hercules", "cubic", {}), ("hercules", "linear", {}),
    ("forces", "nearest", {}), ("hercules", "cubic", dict(focal_depth=-6 * MM)),
    ("tpw", "cubic", {}), ("vls", "cubic", dict(focal_depth=-4 * MM)),
    ("vls", "linear", dict(focal_depth=5.1 * MM))])
def test_adjoint_frames_matches_single_frames(torch_mod, mode, interp, kw):
    torch = torch_mod
    d = _desc(mode, interp, **kw)
    H, e = _frames(d, 3, 51)
    plan = bfm.Plan(d, H)
    et = torch.from_numpy(e.astype(np.float32)).cuda()
    G = np.random.default_rng(9).normal(size=(3,) + plan.out_shape).astype(np.float32)
    Gt = torch.from_numpy(G).cuda()
    ge, gc = plan.das_adjoint(et, Gt)
    assert tuple(gc.shape) == (3,) and tuple(ge.shape) == (3,) + tuple(et.shape[1:])
    ge_n, gc_n = ge.cpu().numpy(), gc.cpu().numpy()
    for f in range(3):
        ge1, gc1 = plan.das_adjoint(et[f], Gt[f])
        assert gc_n[f] == float(gc1), f"grad_c of frame {f}"
        assert rel_l2(ge_n[f], ge1.cpu().numpy()) < 1e-6, f"grad_e of frame {f}"
    if interp != "nearest":          # nearest reads: frame-by-frame gather, compared above
        ref_e = oracle.das_adjoint_e(d, G[2].astype(np.float64))
        assert rel_l2(ge_n[2], ref_e) < 1e-5
        ref_c = float(np.sum(G[2].astype(np.float64) * oracle.das_dc(d, e[2])))
        assert abs(gc_n[2] - ref_c) <= 1e-4 * abs(ref_c)


def test_adjoint_frames_e_only_and_c_only(torch_mod):
    torch = torch_mod
    d = _desc("hercules", "cubic")
    H, e = _frames(d, 2, 61)
    plan = bfm.Plan(d, H)
    et = torch.from_numpy(e.astype(np.float32)).cuda()
    Gt = torch.from_numpy(np.random.default_rng(3).normal(
        size=(2,) + plan.out_shape).astype(np.float32)).cuda()
    ge_both, gc_both = plan.das_adjoint(et, Gt)
    ge, none_c = plan.das_adjoint(None, Gt, want_c=False)
    none_e, gc = plan.das_adjoint(et, Gt, want_e=False)
    assert none_c is None and none_e is None
    assert torch.equal(gc, gc_both)
    assert rel_l2(ge.cpu().numpy(), ge_both.cpu().numpy()) < 1e-6


def test_frames_argument_errors(torch_mod):
    torch = torch_mod
    d = _desc("forces", "cubic")
    H, e = _frames(d, 2, 71)
    plan = bfm.Plan(d, H)
    et = torch.from_numpy(e.astype(np.float32)).cuda()
    out = torch.empty((2,) + plan.out_shape, device="cuda")
    L = _lib.lib()
    for n in (0, -1, _lib.MAX_FRAMES + 1):
        st = L.bf_das_frames(plan._h, et.data_ptr(), n, out.data_ptr(), 1540.0, None)
        assert st == _lib.BF_ERR_SHAPE
        st = L.bf_das_adjoint_frames(plan._h, et.data_ptr(), out.data_ptr(), n, 1540.0, None,
                                     None, None)
        assert st == _lib.BF_ERR_SHAPE
    assert L.bf_das_frames(plan._h, None, 2, out.data_ptr(), 1540.0, None) == _lib.BF_ERR_NULL
    with pytest.raises(ValueError):
        plan.das(et, out=torch.empty(plan.out_shape, device="cuda"))
    with pytest.raises(ValueError):
        plan.das_adjoint(et, out[:1].contiguous())       # 2 frames of data, 1 of grad_out


def test_focus_loss_stacked_matches_list(torch_mod):
    """The autofocus loss and dL/dc of a stacked batch equal the per-frame
    (checkpointed) path: same images, per-frame dL/dc terms summed."""
    torch = torch_mod
    d = _desc("forces", "cubic")
    H, e = _frames(d, 4, 81)
    plan = bfm.Plan(d, H)
    et = torch.from_numpy(e.astype(np.float32)).cuda()
    res = []
    for frames in (et, [et[f] for f in range(4)]):
        c = torch.tensor(1530.0, dtype=torch.float64, requires_grad=True)
        loss = focus_loss(frames, c, plan)
        loss.backward()
        res.append((float(loss), float(c.grad)))
    (l_s, g_s), (l_l, g_l) = res
    assert abs(l_s - l_l) <= 1e-6 * abs(l_l)
    assert abs(g_s - g_l) <= 1e-6 * abs(g_l) + 1e-12


def test_differentiable_forces_workload_stack(torch_mod):
    """Full size: the 8 frames of the differentiable FORCES workload as one
    stack, bit-identical to the per-frame calls (images and grad_c), as the
    benchmark's batched autofocus step runs them."""
    torch = torch_mod
    desc, H, rfs, info = synth.make_inputs(3)
    plan = bfm.Plan(desc, H)
    c = float(info["c_true"])
    es = torch.stack([plan.decode(torch.from_numpy(r).cuda()) for r in rfs]).contiguous()
    imgs = plan.das(es, c=c)
    loss, g = bfm.sharpness(imgs.reshape(len(rfs), -1))
    _, gc = plan.das_adjoint(es, g.reshape(imgs.shape), c=c, want_e=False)
    for f in range(len(rfs)):
        one = plan.das(es[f], c=c)
        assert torch.equal(imgs[f], one), f
        _, gc1 = plan.das_adjoint(es[f], g.reshape(imgs.shape)[f], c=c, want_e=False)
        assert float(gc[f]) == float(gc1), f


@pytest.mark.parametrize("mode", ["forces", "hercules"])
def test_iq_das_frames_matches_single_frames(torch_mod, mode):
    """Complex (IQ) stacks: frame offsets count complex samples."""
    torch = torch_mod
    d = dict(_desc(mode, "cubic"))
    d["iq"] = True
    rng = np.random.default_rng(91)
    n_ch = d["n_ch"]
    e = (rng.normal(size=(3, 8, n_ch, 600)) + 1j * rng.normal(size=(3, 8, n_ch, 600)))
    plan = bfm.Plan(d, hadamard(8, "scrambled", seed=91))
    et = torch.from_numpy(e.astype(np.complex64).view(np.float32).reshape(3, 8, n_ch, 600, 2)).cuda()
    stack = plan.das(et).cpu()
    for f in range(3):
        assert torch.equal(stack[f], plan.das(et[f]).cpu()), f
    ref = oracle.das_iq(d, e[1])
    assert rel_l2(stack[1].numpy(), ref) < 1e-5


def test_large_stack(torch_mod):
    """150 frames of the 256 x 256 FORCES plane: every frame's image and
    dL/dc (one stacked adjoint launch) equal its own calls, at the first,
    last and some middle frames."""
    torch = torch_mod
    desc, H, _, info = synth.make_inputs(3)
    plan = bfm.Plan(desc, H)
    c = float(info["c_true"])
    gen = torch.Generator(device="cuda").manual_seed(123)
    nf = 150
    es = torch.randn((nf,) + plan.e_shape, generator=gen, device="cuda") * 100.0
    imgs = plan.das(es, c=c)
    G = torch.randn(imgs.shape, generator=gen, device="cuda")
    _, gc = plan.das_adjoint(es, G, c=c, want_e=False)
    for f in (0, 127, 128, 143, 144, nf - 1):
        assert torch.equal(imgs[f], plan.das(es[f], c=c)), f
        _, gc1 = plan.das_adjoint(es[f], G[f], c=c, want_e=False)
        assert float(gc[f]) == float(gc1), f


@pytest.mark.parametrize("cap", [1, 2])
def test_stack_split_over_launches(torch_mod, cap):
    """A stack taken in several launches per gradient (the frame cap, which
    production sizes reach only with very long stacks, forced through the
    test hook): 5 frames in launches of `cap` frames give grad_c bit for bit
    and grad_e up to the order of FP32 atomics of the single-frame calls, and
    the same as the uncapped stack."""
    torch = torch_mod
    d = _desc("forces", "cubic")
    H, e = _frames(d, 5, 71)
    plan = bfm.Plan(d, H)
    et = torch.from_numpy(e.astype(np.float32)).cuda()
    Gt = torch.from_numpy(np.random.default_rng(8).normal(
        size=(5,) + plan.out_shape).astype(np.float32)).cuda()
    ge_all, gc_all = plan.das_adjoint(et, Gt)
    _lib.check(_lib.lib().bf_test_set_stack_cap(plan._h, cap))
    ge, gc = plan.das_adjoint(et, Gt)
    _lib.check(_lib.lib().bf_test_set_stack_cap(plan._h, 0))
    assert torch.equal(gc, gc_all)
    assert rel_l2(ge.cpu().numpy(), ge_all.cpu().numpy()) < 1e-6
    for f in range(5):
        ge1, gc1 = plan.das_adjoint(et[f], Gt[f])
        assert float(gc[f]) == float(gc1), (cap, f)
        assert rel_l2(ge[f].cpu().numpy(), ge1.cpu().numpy()) < 1e-6, (cap, f)


@pytest.mark.parametrize("e_type", ["bf16", "i32"])
def test_frames_storage_types(torch_mod, e_type):
    """Stacks of BF16 / int32 decoded data: frame offsets in their element
    size; the adjoint's dL/dc (gather kernel for these types) and dL/de
    (LDS kernel, which reads no data) per frame as in single calls."""
    torch = torch_mod
    d = _desc("hercules", "cubic")
    H, e = _frames(d, 3, 101)
    plan = bfm.Plan(d, H, e_type=e_type)
    dt = torch.bfloat16 if e_type == "bf16" else torch.int32
    et = (torch.from_numpy(e.astype(np.float32)).to(dt) if e_type == "bf16"
          else torch.from_numpy(np.rint(e).astype(np.int32))).cuda()
    stack = plan.das(et)
    G = torch.from_numpy(np.random.default_rng(4).normal(
        size=(3,) + plan.out_shape).astype(np.float32)).cuda()
    ge, gc = plan.das_adjoint(et, G)
    for f in range(3):
        assert torch.equal(stack[f], plan.das(et[f])), f
        ge1, gc1 = plan.das_adjoint(et[f], G[f])
        assert rel_l2(gc[f:f + 1].cpu().numpy(), gc1.reshape(1).cpu().numpy()) <= 1e-6, f
        assert rel_l2(ge[f].cpu().numpy(), ge1.cpu().numpy()) <= 1e-6, f
