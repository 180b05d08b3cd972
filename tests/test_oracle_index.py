"""Pins of the index-algebra oracle (oracle/moa.py) against the paper's
printed MoA examples (Ch. 2 and Ch. 4) and against brute-force enumeration."""
import itertools

import numpy as np
import pytest

from oracle import moa
from tests.conftest import golden


def A345():
    return moa.MArray([3, 5, 4], list(range(60)))


def test_psi_printed_examples():
    g = golden("psi_examples.json")
    A = A345()
    sub = moa.psi(g["psi_1"]["index"], A)
    assert sub.shape == g["psi_1"]["shape"] and sub.ravel == g["psi_1"]["ravel"]
    assert moa.psi(g["psi_2_1"]["index"], A).ravel == g["psi_2_1"]["ravel"]
    assert moa.psi(g["psi_2_1_3"]["index"], A) == g["psi_2_1_3"]["value"]
    assert moa.psi([], A).ravel == A.ravel


def test_psi_reduction_example():
    g = golden("psi_examples.json")["reverse_take_example"]
    A = A345()
    lhs = moa.psi(g["index"], moa.take_array(g["take"], moa.reverse(A)))
    rhs = moa.psi(g["equals_index_of_A"], A)
    assert lhs.shape == g["shape"] and lhs.ravel == rhs.ravel


def test_reverse_definition_on_visible_rows():
    # Ch. 2, Def. reverse: rho(Phi A) = rho A and <i> psi (Phi A) = <s_0 - i - 1> psi A.
    # Four rows (no fixed middle row) and a 3-D case, so an identity, a
    # rotation or a reversal of the wrong axis all fail.
    A = moa.MArray([4, 2], list(range(8)))
    R = moa.reverse(A)
    assert R.shape == [4, 2]
    assert R.ravel == [6, 7, 4, 5, 2, 3, 0, 1]
    B = moa.MArray([2, 3, 2], list(range(12)))
    RB = moa.reverse(B)
    assert RB.ravel == [6, 7, 8, 9, 10, 11, 0, 1, 2, 3, 4, 5]
    for X, RX in ((A, R), (B, RB), (A345(), moa.reverse(A345()))):
        s0 = X.shape[0]
        for i in range(s0):
            assert moa.psi([i], RX).ravel == moa.psi([s0 - 1 - i], X).ravel
        assert moa.reverse(RX).ravel == X.ravel
    # the printed psi-reduction example on a 4-row array: <1 2> psi (2 take (Phi A))
    # is <2 2> psi A (row s_0 - 1 - 1 of A), which an identity reverse gets wrong
    C = moa.MArray([4, 5, 4], list(range(80)))
    assert moa.psi([1, 2], moa.take_array(2, moa.reverse(C))).ravel == moa.psi([2, 2], C).ravel
    assert moa.psi([1, 2], moa.take_array(2, C)).ravel != moa.psi([2, 2], C).ravel


def test_omega_rotate_example():
    g = golden("psi_examples.json")["omega_rotate"]
    rows = [moa.rotate(k, row) for k, row in zip(g["amounts"], g["matrix"])]
    assert rows == g["result"]


def test_psi_composition_theorem():
    A = A345()
    for p in itertools.product(range(3), range(5)):
        q, r = list(p[:1]), list(p[1:])
        assert moa.psi(list(p), A).ravel == moa.psi(r, moa.psi(q, A)).ravel


def test_gamma_inverse_and_column_major():
    shape = [3, 5, 4, 2]
    for off in range(moa.pi(shape)):
        idx = moa.gamma_inv(shape, off)
        assert moa.gamma(shape, idx) == off
    # column-major: first index fastest
    assert moa.gamma_col([3, 5], [1, 0]) == 1
    assert moa.gamma_col([3, 5], [0, 1]) == 3
    assert moa.pi([]) == 1 and moa.gamma([], []) == 0


def test_take_drop_rotate_vectors():
    v = [0, 1, 2, 3, 4]
    assert moa.take(2, v) == [0, 1] and moa.take(-2, v) == [3, 4]
    assert moa.drop(2, v) == [2, 3, 4] and moa.drop(-2, v) == [0, 1, 2]
    assert moa.rotate(2, v) == [2, 3, 4, 0, 1]
    assert moa.rotate(-2, v) == [3, 4, 0, 1, 2]


def test_reshape_wraps_cyclically():
    A = moa.MArray([4], [0, 1, 2, 3])
    assert moa.reshape([2, 3], A).ravel == [0, 1, 2, 3, 0, 1]
    assert moa.reshape([3], A).ravel == [0, 1, 2]


@pytest.mark.parametrize("shape", [[4, 6, 7], [2, 3], [5], [2, 2, 2, 2]])
def test_pct_against_enumeration(shape):
    A = moa.MArray(shape, list(range(moa.pi(shape))))
    for k in range(len(shape)):
        for j in itertools.product(*[range(s) for s in shape[:k]]):
            start, length = moa.pct(shape, list(j))
            sub = moa.psi(list(j), A)
            assert sub.ravel == A.ravel[start:start + length]


def test_four_by_four_hypercube_rule():
    g = golden("hypercube_rules.json")
    A = moa.reshape([4, 4], moa.MArray([16], list(range(16))))
    B = moa.reshape([4, 4], moa.transpose(A))
    assert B.ravel == [0, 4, 8, 12, 1, 5, 9, 13, 2, 6, 10, 14, 3, 7, 11, 15]
    Ah, Bh = moa.hyper(A), moa.hyper(B)
    for case in g["four_by_four"]:
        assert moa.psi(case["p_B"], Bh) == case["value"]
        assert moa.psi(case["q_A"], Ah) == case["value"]
    for p in itertools.product(range(2), repeat=4):
        i, j, k, l = p
        assert moa.psi([i, j, k, l], Bh) == moa.psi([k, l, i, j], Ah)


def test_d5_rotation_rule():
    g = golden("hypercube_rules.json")["d5"]
    n, r, c = g["n"], g["r"], g["c"]
    A = moa.reshape([r, c], moa.MArray([n], list(range(n))))
    B = moa.reshape_transpose(A, r, c)
    Ah, Bh = moa.hyper(A), moa.hyper(B)
    assert moa.transpose(Ah, g["B_from_A_perm"]).ravel == Bh.ravel
    assert moa.transpose(Bh, g["A_from_B_perm"]).ravel == Ah.ravel
    for p in itertools.product(range(2), repeat=5):
        assert moa.psi(list(p), Bh) == moa.psi(moa.rotate(g["rotate"], list(p)), Ah)
    assert moa.rotate(g["rotate"], list(range(5))) == g["B_from_A_perm"]
    assert moa.rotate(-g["rotate"], list(range(5))) == g["A_from_B_perm"]


def test_reshape_transpose_matches_c_oracle():
    import oracle
    for n, c in [(32, 4), (64, 8), (128, 4)]:
        A = moa.MArray([n], list(range(n)))
        want = moa.reshape_transpose(A, n // c, c).ravel
        got = np.real(oracle.trans_rshp(np.arange(n, dtype=complex), c)).astype(int).tolist()
        assert got == want
