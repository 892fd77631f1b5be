"""Envelope (analytic signal along depth) and display compression on the GPU
against the FP64 oracle.

The FP32 FFT (power-of-two depths) and the direct circular sum (other depths)
carry a rounding error of order log2(N) or N times 2^-24 of the column's
energy; envelopes must be within relative L2 1e-5 of the oracle's and within
1e-5 of the image maximum everywhere.  Log-compressed values are compared
where the envelope is above the clip level (in dB the envelope error is scaled
by 20 / ln 10 / env) and must equal -DR where the oracle's value lies well
below the clip.
"""
import numpy as np
import pytest

import oracle
import paper_2512_11086_amd as bfm
import synth
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _env_gpu(torch, img, compress="none", ref=0.0, param=60.0, iq=False):
    env = bfm.Envelope(img.shape, iq=iq)
    x = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    return env(x, compress, ref, param).cpu().numpy()


def _check_env(got, ref):
    assert rel_l2(got, ref) <= 1e-5, rel_l2(got, ref)
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()


@pytest.mark.parametrize("N", [2, 4, 64, 128, 256, 512, 1024, 2048, 4096])
def test_envelope_fft_path_matches_oracle(torch_mod, N):
    img = np.random.default_rng(N).normal(size=(5, 3, N)).astype(np.float32)
    got = _env_gpu(torch_mod, img)
    _check_env(got, oracle.envelope(img.astype(np.float64)))


def test_envelope_pairs_of_unequal_columns(torch_mod):
    # power-of-two depths up to 1024 pack two columns into one complex FFT; a
    # weak column next to a 1000x stronger one keeps the image-level bound
    # and stays within 1e-5 of its partner's maximum
    rng = np.random.default_rng(7)
    img = rng.normal(size=(7, 256)).astype(np.float32)
    img[0::2] *= 1000.0
    got = _env_gpu(torch_mod, img)
    ref = oracle.envelope(img.astype(np.float64))
    _check_env(got, ref)
    for c in range(1, 7, 2):
        assert np.abs(got[c] - ref[c]).max() <= 1e-5 * np.abs(ref[c - 1]).max(), c


@pytest.mark.parametrize("N", [1, 3, 37, 100, 255, 1000])
def test_envelope_direct_path_matches_oracle(torch_mod, N):
    img = np.random.default_rng(N).normal(size=(7, N)).astype(np.float32)
    got = _env_gpu(torch_mod, img)
    _check_env(got, oracle.envelope(img.astype(np.float64)))


def test_envelope_of_iq_image_is_modulus(torch_mod):
    rng = np.random.default_rng(3)
    z = (rng.normal(size=(4, 6, 50)) + 1j * rng.normal(size=(4, 6, 50))).astype(np.complex64)
    got = _env_gpu(torch_mod, z, iq=True)
    np.testing.assert_allclose(got, np.abs(z.astype(np.complex128)), rtol=2e-7, atol=0)


def _check_log(got, env_ref, ref_level, dr):
    y_ref = oracle.compress(env_ref, "log", ref_level, dr)
    above = env_ref > ref_level * 10 ** (-(dr - 1) / 20)
    # dB error of an envelope error of 1e-5 max|env| at this envelope
    tol = 20 / np.log(10) * 1e-5 * env_ref.max() / np.maximum(env_ref, 1e-30) + 1e-4
    assert np.all(np.abs(got - y_ref)[above] <= tol[above])
    well_below = env_ref < ref_level * 10 ** (-(dr + 1) / 20)
    assert np.all(got[well_below] == -dr)
    assert got.max() <= 20 * np.log10(env_ref.max() / ref_level) + 1e-3


@pytest.mark.parametrize("N", [256, 100])
def test_log_compression_given_and_image_maximum(torch_mod, N):
    rng = np.random.default_rng(10 + N)
    img = (rng.normal(size=(6, N)) * np.exp(-np.linspace(0, 8, N))).astype(np.float32)
    env_ref = oracle.envelope(img.astype(np.float64))
    got = _env_gpu(torch_mod, img, "log", ref=0.0, param=50.0)
    _check_log(got, env_ref, env_ref.max(), 50.0)
    got = _env_gpu(torch_mod, img, "log", ref=0.5, param=40.0)
    _check_log(got, env_ref, 0.5, 40.0)


def test_power_compression_and_zero_image(torch_mod):
    rng = np.random.default_rng(4)
    img = rng.normal(size=(3, 64)).astype(np.float32)
    env_ref = oracle.envelope(img.astype(np.float64))
    got = _env_gpu(torch_mod, img, "power", ref=1.2, param=0.5)
    ref = oracle.compress(env_ref, "power", 1.2, 0.5)
    assert np.abs(got - ref).max() <= 1e-5
    got = _env_gpu(torch_mod, img, "power", ref=0.0, param=2.0)
    assert np.abs(got - oracle.compress(env_ref, "power", 0.0, 2.0)).max() <= 1e-5
    z = np.zeros((2, 64), dtype=np.float32)
    assert np.all(_env_gpu(torch_mod, z, "log", 0.0, 45.0) == -45.0)
    assert np.all(_env_gpu(torch_mod, z, "power", 0.0, 1.0) == 0.0)


def test_envelope_rejects_bad_arguments(torch_mod):
    torch = torch_mod
    with pytest.raises(bfm.BfError):
        bfm.Envelope((4, 4097))
    with pytest.raises(bfm.BfError):
        bfm.Envelope((0, 16))
    env = bfm.Envelope((2, 16))
    x = torch.zeros((2, 16), device="cuda")
    with pytest.raises(bfm.BfError):
        env(x, "log", 0.0, -3.0)
    with pytest.raises(bfm.BfError):
        env(x, "log", float("nan"), 60.0)


def test_chain_workload0_das_envelope_log(torch_mod):
    torch = torch_mod
    desc, H, rf, _ = synth.make_inputs(0)
    plan = bfm.Plan(desc, H)
    img = plan.das(plan.decode(torch.from_numpy(rf).cuda()))
    env = bfm.Envelope(img.shape)
    got = env(img, "log", 0.0, 60.0).cpu().numpy()
    ref_img = oracle.das(desc, oracle.decode(H, rf))
    env_ref = oracle.envelope(ref_img)
    _check_log(got, env_ref, env_ref.max(), 60.0)
    raw = env(img).cpu().numpy()
    assert rel_l2(raw, env_ref) <= 1e-5


def test_full_volume_sampled_columns(torch_mod):
    # workload-1 volume: the GPU envelope of the GPU image against the oracle
    # envelope of the same image's columns (DAS parity is tested elsewhere)
    torch = torch_mod
    desc, H, rf, _ = synth.make_inputs(1)
    plan = bfm.Plan(desc, H)
    img = plan.das(plan.decode(torch.from_numpy(rf).cuda()))
    got = bfm.Envelope(img.shape)(img).cpu().numpy().reshape(-1, img.shape[-1])
    cols = np.random.default_rng(0).choice(got.shape[0], size=64, replace=False)
    src = img.cpu().numpy().reshape(-1, img.shape[-1])[cols].astype(np.float64)
    _check_env(got[cols], oracle.envelope(src))
