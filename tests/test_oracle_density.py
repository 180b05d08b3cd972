"""Pins of the Ch. 6 oracles: the transpose vector (oracle/moa.py,
gate_transpose_vector), the hyper-cube transpose and its normal form, and the
density-matrix gate (oracle/density.py) -- against the paper's printed
permutation vectors, the block-diagonal form the paper states, textbook
identities (Kronecker products, Pauli X, SWAP, phase gates) and the
invariants of a unitary transformation."""
import itertools

import numpy as np
import pytest

from oracle import density, moa
from tests.conftest import golden


def rand_unitary(k, rng):
    z = rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))
    qm, r = np.linalg.qr(z)
    return qm * (np.diag(r) / np.abs(np.diag(r)))


def rand_density(n, rng):
    N = 1 << n
    a = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    rho = a @ a.conj().T
    return rho / np.trace(rho)


def test_printed_permutation_vectors():
    g = golden("density_permutations.json")
    for case in g["cases"]:
        assert moa.gate_transpose_vector(g["n"], case["gated_bits"]) == case["t"], case["pattern"]
        # the order in which the gated bits are named does not matter
        assert moa.gate_transpose_vector(g["n"], case["gated_bits"][::-1]) == case["t"]


def test_transpose_vector_moves_gated_bits_to_the_diagonal_blocks():
    """t transpose (hyper-cube of G) is block diagonal with U on every
    diagonal block: the paper's statement that the gated sub-matrices land on
    the diagonal in 2^q x 2^q blocks.  A wrong order of the gated or free
    axes breaks it."""
    rng = np.random.default_rng(1)
    for n, gated in [(4, [0, 2]), (4, [1, 2]), (5, [0, 4]), (5, [3]), (5, [1, 2, 4]), (3, [0, 1, 2])]:
        q = len(gated)
        U = rand_unitary(1 << q, rng)
        G = density.gate_matrix(n, U, gated)
        Gb = np.array(moa.block_diagonal_view(list(G.reshape(-1)), n, gated)).reshape(1 << n, 1 << n)
        want = np.kron(np.eye(1 << (n - q)), U)
        assert np.array_equal(Gb, want), (n, gated)


def test_reading_of_the_printed_vectors():
    """The printed xabx vector <0 3 1 2 4 7 5 6> is not an involution.  Read
    as 'axis k of the view is axis t[k] of D_h' (the order the paper's swaps
    build), the view (inverse t) transpose D_h is block diagonal; read as
    t transpose D_h in the sense of Ch. 2, it puts bits 0 and 2 on the
    diagonal instead of the gated 1 and 2.  For xaxb both readings agree."""
    rng = np.random.default_rng(7)
    n = 4
    U = rand_unitary(4, rng)
    for gated, t, involutive in (([0, 2], [0, 2, 1, 3, 4, 6, 5, 7], True), ([1, 2], [0, 3, 1, 2, 4, 7, 5, 6], False)):
        G = list(density.gate_matrix(n, U, gated).reshape(-1))
        want = np.kron(np.eye(4), U)
        view = np.array(moa.hypercube_transpose(G, moa.inverse_permutation(t))).reshape(16, 16)
        assert np.array_equal(view, want)
        other = np.array(moa.hypercube_transpose(G, t)).reshape(16, 16)
        assert np.array_equal(other, want) == involutive


def test_hypercube_transpose_definition_and_inverse():
    rng = np.random.default_rng(2)
    for m in (1, 2, 3, 5, 7):
        t = list(rng.permutation(m))
        vals = list(range(1 << m))
        out = moa.hypercube_transpose(vals, t)
        # the normal form gives the same elements
        assert out == moa.hypercube_source_offsets(m, t)
        assert list(density.moa_source_offsets_fast(m, t)) == out
        # the inverse permutation undoes it
        inv = [0] * m
        for k, v in enumerate(t):
            inv[v] = k
        assert moa.hypercube_transpose(out, inv) == vals
    # <1 0> on <2 2> is the 2 x 2 matrix transpose; reversing all axes of
    # a <2 2 2> cube reverses the bits of every offset
    assert moa.hypercube_transpose([0, 1, 2, 3], [1, 0]) == [0, 2, 1, 3]
    assert moa.hypercube_transpose(list(range(8)), [2, 1, 0]) == [0, 4, 2, 6, 1, 5, 3, 7]


@pytest.mark.parametrize("n,gated", [(1, [0]), (2, [0]), (2, [1]), (3, [0, 2]), (4, [0, 2]), (4, [1, 2]),
                                     (4, [3, 0]), (5, [2, 3, 4]), (5, [0, 1, 2, 3]), (6, [5, 0])])
def test_gate_two_routes_agree(n, gated):
    rng = np.random.default_rng(n * 31 + len(gated))
    rho = rand_density(n, rng)
    U = rand_unitary(1 << len(gated), rng)
    a = density.apply_gate(rho, U, gated)
    b = density.apply_gate_blocks(rho, U, gated)
    assert np.allclose(a, b, atol=1e-13)


def test_gate_adjacent_qubits_is_a_kronecker_product():
    """Gating qubits b+1 and b (adjacent) is I (x) U (x) I with U's most
    significant index bit on qubit b+1: the bit-order convention."""
    rng = np.random.default_rng(3)
    n = 5
    for b in range(n - 1):
        U = rand_unitary(4, rng)
        G = np.kron(np.kron(np.eye(1 << (n - b - 2)), U), np.eye(1 << b))
        assert np.allclose(density.gate_matrix(n, U, [b, b + 1]), G, atol=0)
        rho = rand_density(n, rng)
        assert np.allclose(density.apply_gate(rho, U, [b + 1, b]), G @ rho @ G.conj().T, atol=1e-14)


def test_gate_closed_forms():
    rng = np.random.default_rng(4)
    n = 4
    N = 1 << n
    rho = rand_density(n, rng)
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    # Pauli X on qubit k flips bit k of both indices
    X = np.array([[0, 1], [1, 0]], complex)
    for k in range(n):
        out = density.apply_gate_blocks(rho, X, [k])
        assert np.array_equal(out, rho[i ^ (1 << k), j ^ (1 << k)])
    # SWAP of qubits a and b exchanges those bits of both indices
    SW = np.eye(4)[[0, 2, 1, 3]]
    for a_, b_ in [(0, 1), (0, 3), (1, 2)]:
        def swapbits(v):
            ba, bb = (v >> a_) & 1, (v >> b_) & 1
            return v ^ ((ba ^ bb) << a_) ^ ((ba ^ bb) << b_)
        out = density.apply_gate_blocks(rho, SW, [a_, b_])
        assert np.array_equal(out, rho[swapbits(i), swapbits(j)])
    # a diagonal phase gate multiplies element (i, j) by e^{i(phi(g(i)) - phi(g(j)))}
    phi = rng.uniform(0, 2 * np.pi, 4)
    P = np.diag(np.exp(1j * phi))
    gated = [3, 1]
    gi = np.vectorize(lambda v: density.gated_index(v, gated))
    out = density.apply_gate_blocks(rho, P, gated)
    assert np.allclose(out, rho * np.exp(1j * (phi[gi(i)] - phi[gi(j)])), atol=1e-15)
    # the identity gate changes nothing
    assert np.array_equal(density.apply_gate_blocks(rho, np.eye(4), [0, 2]), rho)


def test_gate_invariants():
    """A unitary transformation keeps the trace, Hermiticity and the spectrum;
    two gates on disjoint qubits commute and compose to their Kronecker
    product."""
    rng = np.random.default_rng(5)
    n = 5
    rho = rand_density(n, rng)
    U = rand_unitary(8, rng)
    out = density.apply_gate(rho, U, [4, 2, 0])
    assert abs(np.trace(out) - 1) < 1e-13
    assert np.allclose(out, out.conj().T, atol=1e-14)
    assert np.allclose(np.linalg.eigvalsh(out), np.linalg.eigvalsh(rho), atol=1e-13)
    A, B = rand_unitary(2, rng), rand_unitary(2, rng)
    ab = density.apply_gate(density.apply_gate(rho, A, [3]), B, [1])
    ba = density.apply_gate(density.apply_gate(rho, B, [1]), A, [3])
    both = density.apply_gate(rho, np.kron(A, B), [3, 1])
    assert np.allclose(ab, ba, atol=1e-14) and np.allclose(ab, both, atol=1e-14)


def test_invalid_gated_bits():
    for bad in ([0, 0], [4], [-1]):
        with pytest.raises(ValueError):
            moa.gate_transpose_vector(4, bad)


def test_source_of_subset_matches_full_table():
    rng = np.random.default_rng(9)
    for m in (3, 9, 14):
        t = list(rng.permutation(m))
        full = density.moa_source_offsets_fast(m, t)
        idx = rng.integers(0, 1 << m, 50)
        assert np.array_equal(density.hypercube_source_of(m, t, idx), full[idx])
