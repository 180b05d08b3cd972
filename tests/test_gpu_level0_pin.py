"""GPU pin of a lift's intermediate array: the output of level 0 alone.

For a two-level lift <r c> of n = r c points (Ch. 3, "The General Algorithm";
"Restructuring the Data: the Reshape-Transpose Operation"), the method
oracle stopped after level 0 holds, at position k r + rho, frequency k of
the length-c DFT of the stride-r column bitrev(rho) (the column index stays
bit-reversed for the next level's in-row stages).  The GPU's level 0 writes
the same length-c DFTs, column a at its natural index, multiplied by the
inter-level factor omega_n^(a k) (the transformed weights of level 1 taken
out as one factor, the four-step identity), in the plan's workspace layout
(moa_fft_describe: the digit strides and, for the paired-column lift
<4096 4096>, the blocked layout).  The test re-lays the oracle's
intermediate to that layout, applies the factor, and compares element by
element.  Tolerance: relative L2 <= 2e-6 (log2 c + 1) (complex64: the c-point
DFT plus one twiddle product), 1e-13 (complex128).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_0803_2386_amd import inputs  # noqa: E402
from paper_0803_2386_amd import fft as mfft  # noqa: E402

pytestmark = pytest.mark.gpu


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def bitrev(v, bits):
    v = np.asarray(v, np.int64)
    out = np.zeros_like(v)
    for b in range(bits):
        out |= ((v >> b) & 1) << (bits - 1 - b)
    return out


def level0_positions(desc, r, c):
    """Workspace position of (frequency k, column a) for every k < c, a < r
    (array [k, a]), from pass 0's output descriptor."""
    p0 = desc["passes"][0]
    lay = p0["out_layout"]
    s0 = p0["batch_axes"][0]["out_stride"]
    W = p0["tile_width"]
    a = np.arange(r, dtype=np.int64)
    t, w = a // W, a % W
    col = t * lay["tile_stride"] + (w // 2) * lay["pair_stride"] + (w % 2) * s0
    k = np.arange(c, dtype=np.int64)
    lgb = lay["block_lg"]
    if lgb >= 30:
        row = k * p0["dft_axis"]["out_stride"]
    else:
        row = (k & ((1 << lgb) - 1)) * p0["dft_axis"]["out_stride"] + (k >> lgb) * lay["stride_hi"]
    return row[:, None] + col[None, :]


def factor(r, c, n, sign):
    k = np.arange(c, dtype=np.int64)[:, None]
    a = np.arange(r, dtype=np.int64)[None, :]
    return np.exp(sign * 2j * np.pi * ((k * a) % n) / n)


def check_level0(r, c, batch, dtype, use_method_oracle):
    n = r * c
    npd = np.complex64 if dtype == torch.complex64 else np.complex128
    x = inputs.uniform_complex((batch, n), seed=r + 3 * c + batch, dtype=npd)
    plan = mfft.Plan(n, batch, [r, c], dtype=dtype)
    desc = plan.describe()
    assert plan.num_levels == 2
    pos = level0_positions(desc, r, c)
    assert np.array_equal(np.sort(pos.ravel()), np.arange(n)), "level 0 must write every position once"
    xd = torch.from_numpy(x).cuda()
    y = torch.empty_like(xd)
    lam = int(np.log2(c))
    tol = 1e-13 if dtype == torch.complex128 else 2e-6 * (lam + 1)
    for direction, sign in ((0, -1), (1, 1)):
        plan.run_level(0, xd, y, direction=direction)
        torch.cuda.synchronize()
        got = y.cpu().numpy().astype(np.complex128).reshape(batch, n)
        for b in range(batch):
            xb = x[b].astype(np.complex128)
            if use_method_oracle:
                z = oracle.fft_lifted(xb, c, sign=sign, stop_level=0)   # [k r + rho]
                Y = z.reshape(c, r)[:, bitrev(np.arange(r), int(np.log2(r)))]  # [k, a]
            else:
                # the same array from its definition: the c-point DFT of
                # column a (elements x[i r + a])
                Y = oracle.fft(xb.reshape(c, r).T, sign=sign).T  # [k, a]
            want = np.empty(n, np.complex128)
            want[pos] = Y * factor(r, c, n, sign)
            err = np.linalg.norm(got[b] - want) / np.linalg.norm(want)
            print(f"level0 <{r} {c}> batch {b} dir {direction} err {err:.3e}", flush=True)
            assert err <= tol, (err, desc["passes"][0])
    plan.close()


@pytest.mark.parametrize("r,c,batch", [(64, 64, 1), (16, 256, 3), (256, 256, 2), (64, 4096, 1),
                                       (1024, 1024, 1), (4, 8192, 1)])
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_level0_matches_method_oracle(r, c, batch, dtype):
    need_gpu()
    if dtype == torch.complex128 and c > 1 << 13:
        pytest.skip("level longer than the complex128 block limit")
    check_level0(r, c, batch, dtype, use_method_oracle=True)


def test_level0_blocked_workspace_headline():
    """<4096 4096>: the paired-column levels with the blocked workspace, on
    the full 2^24-point vector (the column DFTs from the result oracle; the
    smaller lifts above tie that route to the method oracle)."""
    need_gpu()
    plan = mfft.Plan(1 << 24, 1, [4096, 4096], host_only=True)
    assert plan.describe()["passes"][0]["out_layout"]["block_lg"] < 30
    plan.close()
    check_level0(4096, 4096, 1, torch.complex64, use_method_oracle=False)


def test_level0_two_routes_agree_small():
    need_gpu()
    check_level0(256, 256, 1, torch.complex64, use_method_oracle=False)
