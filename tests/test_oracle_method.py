"""Pins of the method oracle (the cache-optimized FFT of Ch. 3): its index
moves against the paper's printed examples, its transformed weights against
an independent derivation (the weight vector xi transformed like the data,
"Transforming the Weights") and the printed N^(1), N^(2), N^(3) patterns, the
weight-count formulas, and its result against the result oracle.
"""
import numpy as np
import pytest

import oracle
from tests.conftest import golden


def iota(n):
    return np.arange(n, dtype=np.float64).astype(np.complex128)


def as_int(a):
    return np.real(a).astype(np.int64)


def test_reshape_transpose_printed_example():
    g = golden("reshape_transpose_iota32.json")
    n, c = g["n"], g["c"]
    xa = iota(n)
    assert as_int(xa).reshape(n // c, c).tolist() == g["x_a"]
    xc = oracle.trans_rshp(xa, c)
    assert as_int(xc).reshape(n // c, c).tolist() == g["x_c"]
    # the two-stage view: transpose, then reshape the c x r result to r x c
    assert as_int(xa).reshape(n // c, c).T.tolist() == g["x_b"]
    xd = oracle.trans_rshp(xc, c)
    assert as_int(xd).reshape(n // c, c).tolist() == g["x_d"]


def test_printed_trans_rshp_bound_is_an_erratum():
    # The printed outer bound max(0, n/c^2 - 1) visits only n^2/c^3 elements
    # (16 of 32 for n = 32, c = 4); the full range reproduces Eq. reshape3.
    n, c = 32, 4
    printed_count = (max(0, n // (c * c) - 1) + 1) * (n // c)
    assert printed_count == 16
    assert len(set(as_int(oracle.trans_rshp(iota(n), c)).tolist())) == n


@pytest.mark.parametrize("n,c", [(32, 4), (64, 4), (1024, 8), (4096, 16), (512, 8), (16, 4), (8, 2)])
def test_final_transpose_restores_order(n, c):
    l_max, p_max = oracle.lift_levels(n, c)
    x = iota(n)
    for _ in range(l_max):
        x = oracle.trans_rshp(x, c)
    assert np.array_equal(as_int(oracle.final_trans(x, l_max, c)), np.arange(n))


def test_lift_levels_reading():
    # n = 2^p_max c^l_max with 1 <= p_max <= log2 c ("Number of Different Weight Matrices")
    assert oracle.lift_levels(32, 4) == (2, 1)
    assert oracle.lift_levels(16, 4) == (1, 2)    # the "integer part" reading would give 2
    assert oracle.lift_levels(1 << 24, 4096) == (1, 12)
    assert oracle.lift_levels(1 << 20, 4096) == (1, 8)
    assert oracle.lift_levels(64, 64) == (0, 6)
    assert oracle.lift_levels(64, 128) == (0, 6)
    for d in range(1, 21):
        for lam in range(1, 13):
            lm, pm = oracle.lift_levels(1 << d, 1 << lam)
            assert lm * lam + pm == d
            assert 1 <= pm <= lam or (lm == 0 and pm == d)


def test_printed_weight_patterns():
    g = golden("weights_n32_c4.json")
    for case in g["cases"]:
        e, L = oracle.lifted_exponents(g["n"], g["c"], case["l"], case["p"])
        assert L == case["L"], case["name"]
        assert e.tolist() == case["exponents"], case["name"]


def xi_exponents(n, q):
    """Weight vector xi of M^(q) (stage q, L = 2^q): per block of L, L/2 unit
    entries (marked -1) followed by the exponents 0..L/2-1 of Omega_{L/2}."""
    L = 1 << q
    i = np.arange(n)
    r = i % L
    return np.where(r < L // 2, -1, r - L // 2)


@pytest.mark.parametrize("n,c", [(32, 4), (256, 4), (1024, 8), (4096, 8), (2048, 16), (512, 2)])
def test_weights_transform_like_the_data(n, c):
    lam = c.bit_length() - 1
    l_max, p_max = oracle.lift_levels(n, c)
    for l in range(0, l_max + 1):
        for p in range(1, (lam if l < l_max else p_max) + 1):
            q = l * lam + p
            xi = xi_exponents(n, q).astype(np.complex128)
            for _ in range(l):
                xi = oracle.trans_rshp(xi, c)
            xi = as_int(xi)
            half = 1 << (p - 1)
            upper = [P for P in range(n) if not P & half]
            assert all(xi[P] == -1 for P in upper)
            e, L = oracle.lifted_exponents(n, c, l, p)
            assert L == 1 << q
            assert np.array_equal(e, xi[np.array(upper) + half])


@pytest.mark.parametrize("n,c", [(1024, 4), (4096, 16), (1 << 15, 32)])
def test_weight_count_formulas(n, c):
    lam = c.bit_length() - 1
    l_max, p_max = oracle.lift_levels(n, c)
    for l in range(l_max + 1):
        for p in range(1, (lam if l < l_max else p_max) + 1):
            e, L = oracle.lifted_exponents(n, c, l, p)
            assert L == (1 << p) * c ** l
            sigma = e % (c ** l) if l else np.zeros_like(e)
            assert len(set(sigma.tolist())) == c ** l            # d_v = c^l types
            counts = np.bincount(e, minlength=L // 2)
            assert counts.size == L // 2
            assert np.all(counts == n // L)                      # S_v = n / L copies each


@pytest.mark.parametrize("n", [2 ** k for k in range(1, 13)])
def test_method_equals_result_oracle(n):
    rng = np.random.default_rng(n)
    x = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    want = oracle.fft(x)
    for c in [2 ** k for k in range(1, 14)]:
        for sign in (-1, 1):
            got = oracle.fft_lifted(x, c, sign)
            ref = want if sign < 0 else oracle.fft(x, 1)
            assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13, (n, c, sign)


def test_method_large_lift():
    n, c = 1 << 16, 256
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    got = oracle.fft_lifted(x, c)
    assert np.linalg.norm(got - oracle.fft(x)) / np.linalg.norm(got) < 1e-13


def test_level0_intermediate_is_row_ffts_of_columns():
    # After level 0 and its reshape-transpose, row m of <r c> holds, at
    # position rho, frequency m of the length-c DFT of input column
    # bitrev(rho) (stride r), i.e. the paper's in-row stages are column FFTs.
    n, c = 256, 16
    r = n // c
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    mid = oracle.fft_lifted(x, c, -1, stop_level=0).reshape(c, r)
    cols = x.reshape(c, r)  # cols[:, rho'] is column rho' (stride r)
    br = [int(format(i, f"0{r.bit_length() - 1}b")[::-1], 2) for i in range(r)]
    for rho in range(r):
        want = oracle.dft_brute(cols[:, br[rho]])
        assert np.abs(mid[:, rho] - want).max() < 1e-12
