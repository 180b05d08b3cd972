"""Pins of the FP64 result oracle (the DFT of Ch. 3's problem statement, by the
recursive even/odd split of its definition)
against facts fixed by the mathematics: the O(n^2) definition, closed forms,
linearity, Parseval, the adjoint identity, shift/modulation and the real-input
symmetry, plus a library routine (numpy's pocketfft) for the textbook case.
"""
import numpy as np
import pytest

import oracle

POW2 = [1, 2, 4, 8, 16, 32, 64, 128, 256]
PI_LD = np.longdouble("3.141592653589793238462643383279502884")


def rand_c(rng, n):
    return rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("n", POW2)
def test_matches_brute_force_dft(n):
    rng = np.random.default_rng(n)
    x = rand_c(rng, n)
    for sign in (-1, +1):
        assert rel(oracle.fft(x, sign), oracle.dft_brute(x, sign)) < 1e-14


@pytest.mark.parametrize("n", [1, 3, 5, 6, 7, 12])
def test_brute_force_closed_form_any_n(n):
    # delta_0 -> ones, and exp(+2 pi i k0 j / n) -> n delta_k0 (forward sign -1)
    d = np.zeros(n, complex)
    d[0] = 1
    assert np.allclose(oracle.dft_brute(d), np.ones(n), atol=1e-15)
    for k0 in range(n):
        j = np.arange(n)
        x = np.exp(2j * np.pi * k0 * j / n)
        want = np.zeros(n, complex)
        want[k0] = n
        assert np.abs(oracle.dft_brute(x) - want).max() < 1e-12 * n


def test_brute_force_matches_library_dft():
    rng = np.random.default_rng(7)
    for n in (2, 3, 8, 10, 64, 100, 256):
        x = rand_c(rng, n)
        assert rel(oracle.dft_brute(x), np.fft.fft(x)) < 1e-14
        assert rel(oracle.dft_brute(x, +1), np.fft.ifft(x) * n) < 1e-14


@pytest.mark.parametrize("n", [2 ** k for k in range(0, 15)])
def test_closed_forms(n):
    j = np.arange(n)
    d = np.zeros(n, complex)
    d[0] = 1
    assert np.abs(oracle.fft(d) - 1).max() < 1e-15
    const = np.full(n, 0.75 - 0.5j)
    want = np.zeros(n, complex)
    want[0] = n * (0.75 - 0.5j)
    assert np.abs(oracle.fft(const) - want).max() < 1e-12 * n
    for k0 in sorted({0, 1, n // 3, n // 2, n - 1} & set(range(n))):
        # exact integer phase so the input itself carries no rounding of j*k0
        x = np.array([oracle.root(jj * k0, n, +1) for jj in j]) if n <= 4096 else None
        if x is None:
            continue
        want = np.zeros(n, complex)
        want[k0] = n
        assert np.abs(oracle.fft(x) - want).max() < 5e-15 * n * max(1, np.log2(n))
    if n >= 2:
        alt = (-1.0) ** j
        want = np.zeros(n, complex)
        want[n // 2] = n
        assert np.abs(oracle.fft(alt) - want).max() < 1e-15 * n


@pytest.mark.parametrize("n", [16, 1024, 1 << 14])
def test_linearity_parseval_adjoint(n):
    rng = np.random.default_rng(n + 1)
    x, y = rand_c(rng, n), rand_c(rng, n)
    a, b = 0.3 - 1.1j, -2.0 + 0.25j
    Fx, Fy = oracle.fft(x), oracle.fft(y)
    assert rel(oracle.fft(a * x + b * y), a * Fx + b * Fy) < 1e-14
    # Parseval: sum |X|^2 = n sum |x|^2
    assert abs(np.sum(abs(Fx) ** 2) - n * np.sum(abs(x) ** 2)) / (n * np.sum(abs(x) ** 2)) < 1e-14
    # adjoint identity <F x, y> = <x, F^H y> and F^H F = n I
    lhs = np.vdot(y, Fx)
    rhs = np.vdot(oracle.fft(y, +1), x)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13
    assert rel(oracle.fft(Fx, +1), n * x) < 1e-14


@pytest.mark.parametrize("n", [8, 256, 4096])
def test_shift_modulation_and_real_symmetry(n):
    rng = np.random.default_rng(3 * n)
    x = rand_c(rng, n)
    s = 5 % n
    X = oracle.fft(x)
    k = np.arange(n)
    mod = np.array([oracle.root(kk * s, n, -1) for kk in k])
    assert rel(oracle.fft(np.roll(x, s)), X * mod) < 1e-13
    xr = rng.uniform(-1, 1, n).astype(complex)
    Xr = oracle.fft(xr)
    assert np.abs(Xr[(n - k) % n] - np.conj(Xr)).max() < 1e-12


@pytest.mark.parametrize("n", [2 ** k for k in range(0, 21, 2)])
def test_matches_library_fft(n):
    rng = np.random.default_rng(11 + n)
    x = rand_c(rng, n)
    assert rel(oracle.fft(x), np.fft.fft(x)) < 2e-15 * max(1, np.log2(n))


def test_roots_of_unity():
    s = np.sqrt(0.5)
    assert oracle.root(1, 4, -1) == -1j
    assert oracle.root(1, 4, +1) == 1j
    assert oracle.root(2, 4, -1) == -1
    assert oracle.root(0, 1, -1) == 1
    assert abs(oracle.root(1, 8, -1) - (s - 1j * s)) < 2e-16
    assert oracle.root(5, 4, -1) == oracle.root(1, 4, -1)
    assert oracle.root(-1, 4, -1) == oracle.root(3, 4, -1)
    rng = np.random.default_rng(0)
    for _ in range(2000):
        L = 1 << int(rng.integers(0, 31))
        e = int(rng.integers(0, L)) if L > 1 else 0
        w = oracle.root(e, L, -1)
        a = 2 * PI_LD * np.longdouble(e) / np.longdouble(L)
        assert abs(w.real - float(np.cos(a))) <= 1.2e-16
        assert abs(w.imag + float(np.sin(a))) <= 1.2e-16


def test_batch_and_packed_agree_with_single():
    rng = np.random.default_rng(5)
    sizes = [64, 8, 1, 256, 2, 64]
    x = rand_c(rng, sum(sizes))
    got = oracle.fft_packed(x, sizes, threads=2)
    off = 0
    for s in sizes:
        assert rel(got[off:off + s], oracle.fft(x[off:off + s])) == 0.0
        off += s
    xb = rand_c(rng, 4 * 128).reshape(4, 128)
    assert np.array_equal(oracle.fft_batch(xb, threads=3), np.stack([oracle.fft(r) for r in xb]))
    buf = np.array(x, dtype=np.complex128)
    assert oracle.fft_packed_inplace(buf, sizes, threads=2) is buf
    assert np.array_equal(buf, got)
    with pytest.raises(ValueError):
        oracle.fft_packed_inplace(x.astype(np.complex64), sizes)
    with pytest.raises(ValueError):
        oracle.fft_packed_inplace(np.array(x, dtype=np.complex128)[::-1], sizes)


def test_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        oracle.fft(np.zeros(12, complex))
