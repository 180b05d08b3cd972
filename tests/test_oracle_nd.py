"""Pins of the multi-dimensional oracle (oracle.fftn: the 1-D result oracle
along each axis) against facts fixed by the mathematics: the O(N^2)
definition of the multi-dimensional DFT summed directly over all index
pairs, the separable closed forms, Parseval, the adjoint identity, and a
library routine (numpy's fftn) for the textbook case."""
import itertools

import numpy as np
import pytest

import oracle


def brute_nd(x, sign):
    """X[k] = sum_j x[j] exp(sign 2 pi i sum_a j_a k_a / n_a), summed over every
    pair (j, k) with the phase reduced exactly in integers (common
    denominator prod n_a)."""
    shape = x.shape
    N = int(np.prod(shape))
    M = N  # common denominator: sum_a j_a k_a N / n_a is an integer
    idx = list(itertools.product(*[range(n) for n in shape]))
    out = np.zeros(N, complex)
    xv = x.ravel()
    for kk, k in enumerate(idx):
        acc = 0j
        for jj, j in enumerate(idx):
            e = sum(ja * ka * (M // na) for ja, ka, na in zip(j, k, shape)) % M
            acc += xv[jj] * complex(np.cos(2 * np.pi * e / M), sign * np.sin(2 * np.pi * e / M))
        out[kk] = acc
    return out.reshape(shape)


SHAPES = [(2, 4), (4, 4), (8, 2), (2, 2, 4), (4, 2, 8), (1, 8), (16, 1, 2), (2, 2, 2, 2)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("sign", [-1, 1])
def test_fftn_matches_brute_force(shape, sign):
    rng = np.random.default_rng(sum(shape) + sign)
    x = rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape)
    got = oracle.fftn(x, len(shape), sign)
    want = brute_nd(x, sign)
    assert np.abs(got - want).max() < 1e-12 * x.size


def test_fftn_transforms_only_the_trailing_axes():
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, (3, 4, 8)) + 1j * rng.uniform(-1, 1, (3, 4, 8))
    got = oracle.fftn(x, 2)
    for b in range(3):
        assert np.abs(got[b] - brute_nd(x[b], -1)).max() < 1e-12 * 32


def test_fftn_against_numpy():
    rng = np.random.default_rng(6)
    for shape in [(64, 32), (16, 8, 32), (2, 128, 4), (4, 4, 4, 4)]:
        x = rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape)
        want = np.fft.fftn(x)
        assert np.linalg.norm(oracle.fftn(x, len(shape)) - want) <= 1e-14 * np.linalg.norm(want)
        inv = np.fft.ifftn(x) * x.size
        assert np.linalg.norm(oracle.fftn(x, len(shape), +1) - inv) <= 1e-14 * np.linalg.norm(inv)


def test_fftn_closed_forms():
    shape = (8, 16, 4)
    N = int(np.prod(shape))
    delta = np.zeros(shape, complex)
    delta[0, 0, 0] = 1
    assert np.abs(oracle.fftn(delta, 3) - 1).max() < 1e-15
    assert np.abs(oracle.fftn(np.ones(shape, complex), 3) - N * delta).max() < 1e-12 * N
    # plane wave exp(+2 pi i sum_a j_a k0_a / n_a) -> N delta_{k0}
    k0 = (3, 11, 1)
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    phase = sum(g * k / n for g, k, n in zip(grids, k0, shape))
    wave = np.exp(2j * np.pi * phase)
    want = np.zeros(shape, complex)
    want[k0] = N
    assert np.abs(oracle.fftn(wave, 3) - want).max() < 1e-11 * N
    # a shifted delta -> the conjugate plane wave
    d2 = np.zeros(shape, complex)
    d2[k0] = 1
    assert np.abs(oracle.fftn(d2, 3) - np.conj(wave)).max() < 1e-13


def test_fftn_parseval_and_adjoint():
    rng = np.random.default_rng(7)
    shape = (32, 64)
    x = rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape)
    y = rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape)
    X = oracle.fftn(x, 2)
    assert abs(np.sum(np.abs(X) ** 2) - x.size * np.sum(np.abs(x) ** 2)) < 1e-12 * x.size * np.sum(np.abs(x) ** 2)
    lhs = np.vdot(y, X)
    rhs = np.vdot(oracle.fftn(y, 2, +1), x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    assert np.abs(oracle.fftn(X, 2, +1) - x.size * x).max() < 1e-12 * x.size
