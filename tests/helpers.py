"""Shared helpers of the test suite (matrices, error measures, seeded data)."""
import numpy as np

import synth


def _as64(a):
    a = np.asarray(a)
    return a.astype(np.complex128) if np.iscomplexobj(a) else a.astype(np.float64)


def rel_l2(got, ref):
    got, ref = _as64(got), _as64(ref)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / den) if den > 0 else float(np.linalg.norm(got))


def max_rel(got, ref):
    got, ref = _as64(got), _as64(ref)
    m = np.abs(ref).max()
    return float(np.abs(got - ref).max() / m) if m > 0 else float(np.abs(got).max())


def _is_prime(q):
    return q > 1 and all(q % d for d in range(2, int(q ** 0.5) + 1))


def paley_hadamard(n):
    """Order-n Hadamard matrix by Paley's first construction (n - 1 prime, = 3 mod 4)."""
    q = n - 1
    assert _is_prime(q) and q % 4 == 3, n
    squares = {(x * x) % q for x in range(1, q)}
    chi = lambda a: 0 if a % q == 0 else (1 if a % q in squares else -1)
    Q = np.array([[chi(j - i) for j in range(q)] for i in range(q)], dtype=np.int64)
    S = np.zeros((n, n), dtype=np.int64)
    S[0, 1:] = 1
    S[1:, 0] = -1
    S[1:, 1:] = Q
    H = S + np.eye(n, dtype=np.int64)
    assert np.array_equal(H @ H.T, n * np.eye(n, dtype=np.int64))
    return H.astype(np.int8)


def hadamard(n, kind="sylvester", seed=0):
    if kind == "paley":
        return paley_hadamard(n)
    H = synth.hadamard_sylvester(n).astype(np.int64)
    if kind == "scrambled":
        rng = np.random.default_rng(seed)
        H = H[rng.permutation(n)] * rng.choice([-1, 1], size=(n, 1)) * rng.choice([-1, 1], size=(1, n))
    return H.astype(np.int8)


def random_rf(shape, seed, full_range=True):
    rng = np.random.default_rng(seed)
    r = rng.integers(-32768, 32768, size=shape).astype(np.int16)
    if full_range and r.size >= 4:
        flat = r.reshape(-1)
        flat[:4] = [-32768, 32767, -32768, -1]
    return r


def sample_voxels(n_vox, count, seed):
    rng = np.random.default_rng(seed)
    v = rng.choice(n_vox, size=min(count, n_vox), replace=False)
    return np.unique(np.concatenate([v, [0, n_vox - 1]])).astype(np.int64)
