"""GPU parity of the hyper-cube kernels (include/moa_hypercube.h, through the
C ABI) against the Ch. 6 oracles.

Transpose: bit-exact against the MoA transpose of the index oracle
(i psi (t transpose A) = i[t] psi A; vectorised as the source offsets of the
normal form for large arrays).  Gate: against the oracle's G rho G^H (dense
definition for n <= 7, the block route beyond), relative L2 per matrix
<= 2^(q+1) u, u = 2^-23 (complex64) or 2^-52 (complex128): every output is
two complex sums of 2^q products, each rounded; permutation gates (X,
SWAP) bit-exact.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import density, moa  # noqa: E402
from paper_0803_2386_amd import capi  # noqa: E402
from paper_0803_2386_amd import hypercube as hc  # noqa: E402

pytestmark = pytest.mark.gpu


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gate_tol(q, dtype):
    return 2.0 ** (q + 1) * (2.0 ** -23 if dtype == torch.complex64 else 2.0 ** -52)


def rand_unitary(k, rng):
    z = rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))
    qm, r = np.linalg.qr(z)
    return qm * (np.diag(r) / np.abs(np.diag(r)))


def rand_density(n, rng):
    N = 1 << n
    a = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    rho = a @ a.conj().T
    return rho / np.trace(rho).real


@pytest.mark.parametrize("dtype", [torch.float32, torch.complex64, torch.complex128])
def test_transpose_small_ranks_bit_exact(dtype):
    need_gpu()
    rng = np.random.default_rng(11)
    for m in list(range(1, 15)) + [16, 19]:
        for rep in range(4):
            t = list(range(m)) if rep == 0 else (list(range(m))[::-1] if rep == 1 else list(rng.permutation(m)))
            x = torch.arange(1 << m, dtype=torch.float64).to(dtype).cuda() if dtype != torch.complex128 else \
                torch.complex(torch.arange(1 << m, dtype=torch.float64), -torch.arange(1 << m, dtype=torch.float64)).cuda()
            y = hc.hypercube_transpose(x, t)
            torch.cuda.synchronize()
            src = density.moa_source_offsets_fast(m, t)
            want = x.cpu().numpy()[src]
            assert np.array_equal(y.cpu().numpy(), want), (m, t)
            if m <= 8:
                assert list(src) == moa.hypercube_source_offsets(m, t)


def test_transpose_printed_vectors_and_large_array():
    """The paper's two 8-axis vectors, then a 2^26-element complex64 array
    (512 MiB each way) through the block-diagonal view of a 13-qubit matrix."""
    need_gpu()
    for t in ([0, 2, 1, 3, 4, 6, 5, 7], [0, 3, 1, 2, 4, 7, 5, 6]):
        x = torch.arange(256, dtype=torch.float32).cuda()
        y = hc.hypercube_transpose(x, t).cpu().numpy()
        assert list(y.astype(int)) == moa.hypercube_transpose(list(range(256)), t)
    n = 13
    t = hc.block_diagonal_transpose_vector(n, [0, 2])
    m = 2 * n
    x = torch.randn(1 << m, dtype=torch.complex64, device="cuda")
    y = hc.hypercube_transpose(x, t)
    torch.cuda.synchronize()
    src = density.moa_source_offsets_fast(m, t)
    assert np.array_equal(y.cpu().numpy(), x.cpu().numpy()[src])


def test_block_diagonal_view_of_a_gate_matrix():
    """Transposing the gate matrix G with the block-diagonal vector gives
    I (x) U on the GPU as in the oracle."""
    need_gpu()
    rng = np.random.default_rng(3)
    for n, gated in [(4, [0, 2]), (4, [1, 2]), (5, [4, 1, 0])]:
        U = rand_unitary(1 << len(gated), rng)
        G = density.gate_matrix(n, U, gated)
        t = hc.block_diagonal_transpose_vector(n, gated)
        Gb = hc.hypercube_transpose(torch.from_numpy(G.reshape(-1)).cuda(), t).cpu().numpy()
        assert np.array_equal(Gb.reshape(G.shape), np.kron(np.eye(1 << (n - len(gated))), U))
        assert np.array_equal(Gb, np.array(moa.block_diagonal_view(list(G.reshape(-1)), n, gated)))


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_gate_matches_oracle(dtype):
    need_gpu()
    rng = np.random.default_rng(21)
    npd = np.complex64 if dtype == torch.complex64 else np.complex128
    cases = [(1, [0]), (2, [1]), (3, [0, 2]), (4, [0, 2]), (4, [1, 2]), (4, [3, 2, 1, 0]), (5, [4, 0]),
             (6, [2, 3, 5]), (7, [6, 0, 3, 1]), (7, [0]), (9, [8, 7]), (10, [0, 5, 9]), (12, [0, 2]),
             (12, [11, 10, 1, 0]), (12, [6])]
    for n, gated in cases:
        q = len(gated)
        rho = rand_density(n, rng).astype(npd)
        U = rand_unitary(1 << q, rng).astype(npd)
        r = torch.from_numpy(rho).cuda()
        hc.density_gate(r, torch.from_numpy(U).cuda(), gated)
        got = r.cpu().numpy().astype(np.complex128)
        if n <= 7:
            want = density.apply_gate(rho.astype(np.complex128), U.astype(np.complex128), gated)
        else:
            want = density.apply_gate_blocks(rho.astype(np.complex128), U.astype(np.complex128), gated)
        err = np.linalg.norm(got - want) / np.linalg.norm(want)
        print(f"gate n={n} gated={gated} {dtype}: rel err {err:.3e} (bound {gate_tol(q, dtype):.1e})", flush=True)
        assert err <= gate_tol(q, dtype), (n, gated)


def test_permutation_gates_are_exact():
    need_gpu()
    rng = np.random.default_rng(5)
    n = 6
    N = 1 << n
    rho = rand_density(n, rng).astype(np.complex64)
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    X = np.array([[0, 1], [1, 0]], np.complex64)
    for k in (0, 3, 5):
        r = torch.from_numpy(rho).cuda()
        hc.density_gate(r, torch.from_numpy(X).cuda(), [k])
        assert np.array_equal(r.cpu().numpy(), rho[i ^ (1 << k), j ^ (1 << k)])
    SW = np.eye(4, dtype=np.complex64)[[0, 2, 1, 3]]
    a_, b_ = 1, 4
    r = torch.from_numpy(rho).cuda()
    hc.density_gate(r, torch.from_numpy(SW).cuda(), [a_, b_])

    def swapbits(v):
        ba, bb = (v >> a_) & 1, (v >> b_) & 1
        return v ^ ((ba ^ bb) << a_) ^ ((ba ^ bb) << b_)
    assert np.array_equal(r.cpu().numpy(), rho[swapbits(i), swapbits(j)])


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_four_qubit_permutation_gates_are_exact(dtype):
    """A 16 x 16 permutation gate moves elements without arithmetic error (on
    complex64 the four-qubit gate runs on the matrix cores: products by 0 and
    1 and sums with zeros are exact there too)."""
    need_gpu()
    rng = np.random.default_rng(17)
    npd = np.complex64 if dtype == torch.complex64 else np.complex128
    for n, gated in ((6, [0, 2, 3, 5]), (9, [8, 1, 4, 6]), (11, [10, 9, 0, 1])):
        rho = rand_density(n, rng).astype(npd)
        P = np.eye(16, dtype=npd)[rng.permutation(16)]
        r = torch.from_numpy(rho).cuda()
        hc.density_gate(r, torch.from_numpy(P).cuda(), gated)
        want = density.apply_gate_blocks(rho.astype(np.complex128), P.astype(np.complex128), gated).astype(npd)
        assert np.array_equal(r.cpu().numpy(), want), (n, gated)


@pytest.mark.parametrize("n,dtype,gated", [(13, torch.complex64, [0, 1, 2, 3]), (13, torch.complex64, [11, 12, 0, 5]),
                                            (12, torch.complex128, [0, 1, 2, 3]), (12, torch.complex128, [11, 10, 0, 5])])
def test_large_four_qubit_gate(n, dtype, gated):
    """2^26 complex64 or 2^24 complex128 elements, four qubits gated (the
    matrix-core kernel, f32 or f64 instruction): every element against the
    oracle's block route on the host."""
    need_gpu()
    rng = np.random.default_rng(9)
    N = 1 << n
    npd = np.complex64 if dtype == torch.complex64 else np.complex128
    rho = torch.randn(N, N, dtype=dtype, device="cuda")
    U = rand_unitary(16, rng).astype(npd)
    before = rho.cpu().numpy().astype(np.complex128)
    hc.density_gate(rho, torch.from_numpy(U).cuda(), gated)
    got = rho.cpu().numpy().astype(np.complex128)
    want = density.apply_gate_blocks(before, U.astype(np.complex128), gated)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"four-qubit gate n={n} {dtype} gated={gated} rel err {err:.3e}", flush=True)
    assert err <= gate_tol(4, dtype)


def test_large_gate_sampled_blocks():
    """13 qubits (2^26 complex64 elements, 512 MiB), two qubits gated: every
    element checked against the oracle's block route on the host."""
    need_gpu()
    n, gated = 13, [0, 2]
    rng = np.random.default_rng(8)
    N = 1 << n
    rho = torch.randn(N, N, dtype=torch.complex64, device="cuda")
    U = rand_unitary(4, rng).astype(np.complex64)
    before = rho.cpu().numpy().astype(np.complex128)
    hc.density_gate(rho, torch.from_numpy(U).cuda(), gated)
    got = rho.cpu().numpy().astype(np.complex128)
    want = density.apply_gate_blocks(before, U.astype(np.complex128), gated)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"gate n=13 rel err {err:.3e}", flush=True)
    assert err <= gate_tol(2, torch.complex64)


def test_transpose_largest_arrays():
    """Rank 30 with 8-byte elements (8 GiB each way) and rank 31 with 4-byte
    elements (every element distinct): the inverse permutation restores the input exactly, and 4096
    seeded output positions hold the input element the normal form names."""
    need_gpu()
    rng = np.random.default_rng(30)
    for m, dtype in ((30, torch.complex64), (31, torch.int32)):
        t = [int(v) for v in rng.permutation(m)]
        inv = moa.inverse_permutation(t)
        if dtype == torch.int32:
            x = torch.arange(1 << m, dtype=torch.int32, device="cuda")   # every value distinct
        else:
            i = torch.arange(1 << m, dtype=torch.int64, device="cuda")
            x = torch.complex((i >> 15).to(torch.float32), (i & 32767).to(torch.float32))  # distinct, exact
            del i
        y = hc.hypercube_transpose(x, t)
        idx = rng.integers(0, 1 << m, 4096)
        src = density.hypercube_source_of(m, t, idx)
        got = y[torch.from_numpy(idx).cuda()].cpu().numpy()
        want = x[torch.from_numpy(src).cuda()].cpu().numpy()
        assert np.array_equal(got, want), (m, dtype)
        z = hc.hypercube_transpose(y, inv)
        torch.cuda.synchronize()
        assert torch.equal(z, x), (m, dtype)
        print(f"transpose rank {m} {dtype}: round trip exact, 4096 positions exact", flush=True)
        del x, y, z
        torch.cuda.empty_cache()


def test_gate_largest_matrix_sampled_blocks():
    """15 qubits (2^30 complex64 elements, 8 GiB), gated qubits 0 and 14:
    256 seeded blocks of the block-diagonal view read back before and after
    the gate, each checked against U B U^H in FP64."""
    need_gpu()
    n, gated = 15, [0, 14]
    N = 1 << n
    rng = np.random.default_rng(15)
    U = rand_unitary(4, rng).astype(np.complex64)
    rho = torch.randn(N * N, dtype=torch.complex64, device="cuda")
    # element addresses of 256 blocks: free bits random, gated bits enumerated
    free_mask = (N - 1) & ~((1 << 0) | (1 << 14))
    rows = rng.integers(0, N, 256) & free_mask
    cols = rng.integers(0, N, 256) & free_mask
    ab = np.array([(a >> 1) << 14 | (a & 1) for a in range(4)])   # U index bit 1 = qubit 14, bit 0 = qubit 0
    addr = (rows[:, None, None] | ab[None, :, None]) * N + (cols[:, None, None] | ab[None, None, :])
    at = torch.from_numpy(addr.reshape(-1)).cuda()
    before = rho[at].cpu().numpy().astype(np.complex128).reshape(256, 4, 4)
    hc.density_gate(rho.view(N, N), torch.from_numpy(U).cuda(), gated)
    after = rho[at].cpu().numpy().astype(np.complex128).reshape(256, 4, 4)
    Ud = U.astype(np.complex128)
    want = np.einsum("ak,rkl,bl->rab", Ud, before, Ud.conj())
    err = np.linalg.norm(after - want) / np.linalg.norm(want)
    print(f"gate 15 qubits, 256 blocks: rel err {err:.3e}", flush=True)
    assert err <= gate_tol(2, torch.complex64)
