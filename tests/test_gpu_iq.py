"""Demodulation (Eq. 4) and IQ beamforming on the GPU against the FP64 oracle.

Demodulation computes in FP32.  Its error is bounded by
    delta = 2 (N_f + 8) 2^-24 sum_k |h_k| |x[qD - k]|
(FP32 rounding of the folded taps, the products, the N_f-term sum and the
final rotation, with a factor 2 of margin).  int16 output must equal the
oracle's rounding wherever the exact value lies farther than delta from a
rounding boundary (x.5); within delta of one, either neighbour is correct.
FP32 output must lie within delta of the oracle.

IQ beamforming is compared like RF beamforming (relative L2 <= 1e-5 on the
complex image; the per-term rotation adds an FP32 phase error of the same size
as the delay error).  The whole chain -- demodulate, decode the complex int16,
beamform -- is compared with the oracle's chain on the same RF.
"""
import numpy as np
import pytest
import scipy.signal

import oracle
import paper_2512_11086_amd as bfm
import synth
from synth.configs import MM, describe, iq_frontend
from tests.helpers import rel_l2, sample_voxels

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _bound(x, taps, D):
    ax = np.abs(x.astype(np.float64))
    s = scipy.signal.lfilter(np.abs(np.asarray(taps)), [1.0], ax, axis=-1)[..., ::D]
    return 2.0 * (len(taps) + 8) * 2.0 ** -24 * s


def _check_i16(got, x, taps, fd, fs, D):
    """got: int16 (..., n_out, 2); returns how many values differ from the
    oracle's rounding (each one within delta of a rounding boundary)."""
    y = oracle.demod(x, taps, fd, fs, D)
    q = oracle.quantise_iq(y)
    delta = _bound(x, taps, D)
    amb = 0
    for part in (0, 1):
        v = y.real if part == 0 else y.imag
        g = got[..., part].astype(np.int64)
        ref = q[..., part].astype(np.int64)
        dist = np.abs(v - np.floor(v) - 0.5)
        safe = dist > delta
        bad = safe & (g != ref)
        assert not bad.any(), (np.argwhere(bad)[:5], v[bad][:5], g[bad][:5], ref[bad][:5])
        lo = np.clip(np.floor(v), -32768, 32767)
        hi = np.clip(np.ceil(v), -32768, 32767)
        ok = (g == lo) | (g == hi)
        assert ok[~safe].all()
        amb += int((g != ref).sum())
    return amb


CASES = [
    # (n_traces, S, D, n_taps, complex taps, fd/fs)
    (3, 1, 1, 1, False, 0.25),
    (2, 255, 2, 36, False, 0.25),
    (4, 257, 3, 7, True, 0.1234),
    (3, 1000, 4, 166, True, 0.3),
    (2, 2048, 16, 36, False, 0.25),
    (5, 600, 1, 64, True, 0.0),
    (2, 300, 5, 1024, False, 0.07),
]


@pytest.mark.parametrize("n_tr, S, D, n_taps, cplx, r", CASES)
def test_demod_matches_oracle(torch_mod, n_tr, S, D, n_taps, cplx, r):
    torch = torch_mod
    rng = np.random.default_rng(S + 7 * D + n_taps)
    x = rng.integers(-30000, 30000, size=(n_tr, S)).astype(np.int16)
    h = rng.normal(size=n_taps) / n_taps
    if cplx:
        h = h + 1j * rng.normal(size=n_taps) / n_taps
    fs = 20e6
    fd = r * fs
    dm = bfm.Demod(n_tr, S, h, fd, fs, D, out="i16")
    got = dm(torch.from_numpy(x).cuda()).cpu().numpy()
    assert got.shape == (n_tr, (S + D - 1) // D, 2)
    amb = _check_i16(got, x, h, fd, fs, D)
    assert amb <= max(2, got.size // 1000)
    dm32 = bfm.Demod(n_tr, S, h, fd, fs, D, out="f32")
    g32 = dm32(torch.from_numpy(x).cuda()).cpu().numpy()
    y = oracle.demod(x, h, fd, fs, D)
    delta = _bound(x, h, D)
    assert np.all(np.abs(g32[..., 0] - y.real) <= delta + 1e-30)
    assert np.all(np.abs(g32[..., 1] - y.imag) <= delta + 1e-30)


def test_demod_saturates_and_is_repeatable(torch_mod):
    torch = torch_mod
    # gain 4 on full-scale input: large outputs saturate exactly like the oracle
    rng = np.random.default_rng(2)
    x = rng.integers(-32768, 32767, size=(4, 513)).astype(np.int16)
    h = np.full(4, 1.0)
    dm = bfm.Demod(4, 513, h, 0.0, 1.0, 1)
    a = dm(torch.from_numpy(x).cuda())
    b = dm(torch.from_numpy(x).cuda())
    assert torch.equal(a, b)
    got = a.cpu().numpy()
    _check_i16(got, x, h, 0.0, 1.0, 1)
    assert (got[..., 0] == 32767).any() and (got[..., 0] == -32768).any()


def test_demod_full_size_workload_sampled_traces(torch_mod):
    torch = torch_mod
    desc, H, rf, _ = synth.make_inputs(1)
    taps, D, _ = iq_frontend(desc)
    n_tr = desc["n_tx"] * desc["n_ch"]
    dm = bfm.Demod(n_tr, desc["n_samples"], taps, desc["fc"], desc["fs"], D)
    got = dm(torch.from_numpy(rf).cuda()).cpu().numpy().reshape(n_tr, -1, 2)
    idx = np.random.default_rng(0).choice(n_tr, size=48, replace=False)
    x = rf.reshape(n_tr, -1)[idx]
    _check_i16(got[idx], x, taps, desc["fc"], desc["fs"], D)


def test_demod_rejects_bad_arguments(torch_mod):
    with pytest.raises(bfm.BfError):
        bfm.Demod(1, 100, [1.0], 0.0, 1.0, decimation=0)
    with pytest.raises(bfm.BfError):
        bfm.Demod(1, 100, np.ones(1025), 0.0, 1.0)
    with pytest.raises(bfm.BfError):
        bfm.Demod(1, 100, [np.nan], 0.0, 1.0)
    with pytest.raises(bfm.BfError):
        bfm.Demod(1, 100, [1.0], 0.0, 0.0)


# ---------------------------------------------------------------------------
# IQ beamforming
# ---------------------------------------------------------------------------
def _small(mode, S=160, interp="cubic", **kw):
    if mode == "forces":
        return describe("forces", (16, 16), (0.3 * MM, 0.3 * MM), 16, 16, S, 10e6, 2.7e6,
                        (37, 1, 45), (-2 * MM, 0, 2 * MM), (2 * MM, 0, 9 * MM), interp=interp,
                        t0=0.8e-6, **kw)
    return describe("hercules", (16, 16), (0.3 * MM, 0.3 * MM), 16, 16, S, 10e6, 2.7e6,
                    (21, 19, 45), (-2 * MM, -1.5 * MM, 2 * MM), (2 * MM, 1.5 * MM, 9 * MM),
                    interp=interp, t0=0.8e-6, **kw)


def _iq(desc):
    d = dict(desc)
    d["iq"] = True
    return d


@pytest.mark.parametrize("mode", ["forces", "hercules"])
@pytest.mark.parametrize("variant", ["lds", "gather"])
@pytest.mark.parametrize("interp", ["nearest", "linear", "cubic"])
def test_iq_das_matches_oracle(torch_mod, mode, variant, interp):
    torch = torch_mod
    d = _iq(_small(mode, interp=interp))
    seed = 100 * ["forces", "hercules"].index(mode) + 10 * ["lds", "gather"].index(variant)
    rng = np.random.default_rng(seed + ["nearest", "linear", "cubic"].index(interp))
    e = (rng.normal(size=(16, 16, 160)) + 1j * rng.normal(size=(16, 16, 160))).astype(np.complex64)
    plan = bfm.Plan(d, synth.hadamard_sylvester(16))
    if variant == "gather":
        plan.set_das_config("gather", (1, 1, 1), 4)
    else:
        plan.set_das_config("lds", (2, 1, 2) if mode == "forces" else (2, 2, 1), 8)
    et = torch.from_numpy(e.view(np.float32).reshape(16, 16, 160, 2)).cuda()
    img = plan.das(et).cpu().numpy()
    ref = oracle.das_iq(d, e.astype(np.complex128))
    if variant == "lds":
        assert plan.info()["variant"] == 0
    tol = 1e-5 if interp != "nearest" else 1e-4
    assert rel_l2(img, ref) <= tol, rel_l2(img, ref)


def test_iq_das_single_trace_phase(torch_mod):
    # One element under the points and a constant trace: the output is
    # exp(j 2 pi fd (2 z / c - t0)) exactly (oracle pin), so this checks the
    # kernel's phase path (hardware sine / cosine) directly.
    torch = torch_mod
    fd, fs, c, t0, S = 2.7e6, 10e6, 1540.0, 1.3e-6, 512
    d = _iq(describe("hercules", (1, 1), (0.3 * MM, 0.3 * MM), 1, 1, S, fs, fd, (1, 1, 64),
                     (0, 0, 4 * MM), (0, 0, 16 * MM), c=c, t0=t0, f_number=0.0))
    plan = bfm.Plan(d, np.ones((1, 1), dtype=np.int8))
    e = torch.zeros((1, 1, S, 2), dtype=torch.float32, device="cuda")
    e[..., 0] = 1.0
    for variant in ("lds", "gather"):
        plan.set_das_config(variant, (1, 1, 1), 4)
        img = plan.das(e).cpu().numpy().reshape(-1)
        z = np.linspace(4 * MM, 16 * MM, 64)
        ref = np.exp(2j * np.pi * fd * (2 * z / c - t0))
        err = np.abs(img - ref).max()
        assert err < 3e-6, (variant, err)


def test_iq_decode_is_exact(torch_mod):
    torch = torch_mod
    d = _iq(_small("hercules", S=333))
    H = synth.hadamard_sylvester(16)
    rng = np.random.default_rng(4)
    rf = rng.integers(-32768, 32767, size=(16, 16, 333, 2)).astype(np.int16)
    plan = bfm.Plan(d, H)
    e = plan.decode(torch.from_numpy(rf).cuda())
    assert e.shape == (16, 16, 333, 2)
    ref = oracle.decode(H, rf.reshape(16, 16, 666)).reshape(16, 16, 333, 2)
    np.testing.assert_array_equal(e.cpu().numpy().astype(np.int64), ref)


def _chain_oracle(desc, H, rf, taps, D, desc_iq, vox=None):
    n_tx, n_ch, S = rf.shape
    y = oracle.demod(rf.reshape(n_tx * n_ch, S), taps, desc["fc"], desc["fs"], D)
    q = oracle.quantise_iq(y).reshape(n_tx, n_ch, -1, 2)
    e = oracle.decode(H, q.reshape(n_tx, n_ch, -1)).reshape(n_tx, n_ch, -1, 2)
    ec = e[..., 0] + 1j * e[..., 1]
    if vox is None:
        return oracle.das_iq(desc_iq, ec)
    return oracle.das_iq_points(desc_iq, ec, vox)


def _chain_gpu(torch, desc, H, rf, taps, D, desc_iq):
    n_tx, n_ch, S = rf.shape
    dm = bfm.Demod(n_tx * n_ch, S, taps, desc["fc"], desc["fs"], D)
    plan = bfm.Plan(desc_iq, H)
    iq = dm(torch.from_numpy(rf).cuda())
    return plan.das(plan.decode(iq)), plan


def test_iq_chain_workload0_matches_oracle(torch_mod):
    torch = torch_mod
    desc, H, rf, _ = synth.make_inputs(0)
    taps, D, desc_iq = iq_frontend(desc)
    img, _ = _chain_gpu(torch, desc, H, rf, taps, D, desc_iq)
    ref = _chain_oracle(desc, H, rf, taps, D, desc_iq)
    assert rel_l2(img.cpu().numpy(), ref) <= 1e-5


def test_iq_chain_workload1_sampled(torch_mod):
    torch = torch_mod
    desc, H, rf, _ = synth.make_inputs(1)
    taps, D, desc_iq = iq_frontend(desc)
    img, plan = _chain_gpu(torch, desc, H, rf, taps, D, desc_iq)
    assert plan.info()["variant"] == 0
    vox = sample_voxels(int(np.prod(desc_iq["dims"])), 384, 1)
    ref = _chain_oracle(desc, H, rf, taps, D, desc_iq, vox=vox)
    got = img.cpu().numpy().reshape(-1)[vox]
    assert rel_l2(got, ref) <= 1e-5, rel_l2(got, ref)


def test_iq_plans_reject_adjoint_and_batch(torch_mod):
    torch = torch_mod
    d = _iq(_small("hercules"))
    H = synth.hadamard_sylvester(16)
    plan = bfm.Plan(d, H)
    e = torch.zeros(plan.e_shape, dtype=torch.float32, device="cuda")
    g = torch.zeros(plan.out_shape, dtype=torch.float32, device="cuda")
    with pytest.raises(bfm.BfError) as ei:
        plan.das_adjoint(e, g)
    assert ei.value.status == -5
    bp = bfm.BatchPlan([d, d], [H, H])
    rf = [torch.zeros((16, 16, 160, 2), dtype=torch.int16, device="cuda")] * 2
    out = [torch.zeros(plan.out_shape, dtype=torch.complex64, device="cuda")] * 2
    with pytest.raises(bfm.BfError) as ei:
        bp.run(rf, out)
    assert ei.value.status == -5
