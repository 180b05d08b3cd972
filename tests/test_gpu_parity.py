"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances (relative L2 per transform, max over the batch):
  complex64  : 2e-6 * log2 n  (FP32 butterflies, FP64-generated twiddles)
  complex128 : 1e-13
Inputs are seeded U[-1, 1) re/im (paper_0803_2386_amd.inputs); the oracle
consumes exactly the values the GPU sees, upcast to float64.
"""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_0803_2386_amd import capi, inputs  # noqa: E402
from paper_0803_2386_amd import fft as mfft  # noqa: E402

pytestmark = pytest.mark.gpu


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def tol(n, dtype):
    if dtype == torch.complex128:
        return 1e-13
    return 2e-6 * max(1, int(np.log2(n)))


def rel_err_rows(got, want):
    got = np.asarray(got, np.complex128).reshape(want.shape)
    num = np.linalg.norm(got - want, axis=-1)
    den = np.maximum(np.linalg.norm(want, axis=-1), 1e-300)
    return float((num / den).max())


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def run_plan(n, batch, lift, dtype, x_np, direction="forward", **kw):
    plan = mfft.Plan(n, batch, lift, dtype=dtype, **kw)
    x = to_dev(x_np, dtype)
    y = plan.forward(x) if direction == "forward" else plan.adjoint(x)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.complex128), plan


CASES = [
    # (n, batch, lift)
    (1, 3, None), (2, 1, None), (4, 5, None), (8, 2, None), (16, 1, None), (32, 3, None), (64, 7, None),
    (128, 1, None), (256, 9, None), (512, 2, None), (1024, 3, None), (2048, 1, None), (4096, 2, None),
    (8192, 1, None), (16384, 2, None),
    (64, 2, [8, 8]), (256, 3, [16, 16]), (1024, 1, [32, 32]), (4096, 2, [64, 64]), (4096, 1, [16, 256]),
    (4096, 1, [256, 16]), (1 << 15, 1, None), (1 << 16, 2, [256, 256]), (1 << 16, 1, [16, 16, 256]),
    (2048, 2, [2, 4, 2, 8, 16]), (1 << 18, 1, [64, 4096]), (1 << 20, 1, [1024, 1024]),
]


@pytest.mark.parametrize("n,batch,lift", CASES)
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_forward_and_adjoint_match_oracle(n, batch, lift, dtype):
    need_gpu()
    if dtype == torch.complex128 and lift and max(lift) > 1 << 13:
        pytest.skip("level longer than the complex128 block limit")
    np_dtype = np.complex64 if dtype == torch.complex64 else np.complex128
    x = inputs.uniform_complex((batch, n), seed=n + batch, dtype=np_dtype).astype(np.complex128)
    for direction, sign in (("forward", -1), ("adjoint", +1)):
        got, plan = run_plan(n, batch, lift, dtype, x, direction)
        want = oracle.fft(x, sign)
        err = rel_err_rows(got, want)
        print(f"n={n} batch={batch} lift={lift} {dtype} {direction} err={err:.3e}", flush=True)
        assert err <= tol(n, dtype), plan.describe()


def test_c128_n1024_vs_oracle_and_brute_force():
    need_gpu()
    n = 1 << 10
    x = inputs.uniform_complex(n, seed=0, dtype=np.complex128)
    got, _ = run_plan(n, 1, None, torch.complex128, x)
    assert rel_err_rows(got, oracle.fft(x)) <= 1e-13
    assert rel_err_rows(got, oracle.dft_brute(x)) <= 1e-13


def test_n2p24_lift_4096x4096_full_vector():
    need_gpu()
    n = 1 << 24
    x = inputs.uniform_complex(n, seed=0, dtype=np.complex64)
    got, plan = run_plan(n, 1, [4096, 4096], torch.complex64, x)
    d = plan.describe()
    assert d["lift"] == [4096, 4096] and len(d["passes"]) == 2
    want = oracle.fft(x.astype(np.complex128))
    err = rel_err_rows(got, want)
    print(f"2^24 <4096 4096> err={err:.3e}", flush=True)
    assert err <= 2e-6 * 24


def test_closed_forms_on_gpu():
    need_gpu()
    for n, lift in [(1 << 12, None), (1 << 16, [256, 256]), (1 << 20, [1024, 1024])]:
        d = np.zeros(n, np.complex64)
        d[0] = 1
        got, _ = run_plan(n, 1, lift, torch.complex64, d)
        assert np.abs(got - 1).max() < 1e-6
        k0 = 3
        j = np.arange(n)
        x = np.exp(2j * np.pi * ((k0 * j) % n) / n).astype(np.complex64)
        got, _ = run_plan(n, 1, lift, torch.complex64, x)
        want = np.zeros(n)
        want[k0] = n
        assert np.abs(got - want).max() < 2e-6 * np.log2(n) * np.sqrt(n) * 4


@pytest.mark.parametrize("n,batch,lift", [(1 << 20, 64, [1024, 1024]), (1 << 18, 256, [512, 512])])
def test_complex128_write_side_tiles_beyond_the_infinity_cache(n, batch, lift):
    """Complex128, 1 GiB: the last level writes along 8-column tiles (128-byte
    runs) with its rows 8 or 16 KB apart; three seeded rows of each direction
    against the oracle."""
    need_gpu()
    dev = torch.device("cuda", 0)
    x = inputs.device_uniform_complex(n * batch, 27, torch.complex128, dev)
    plan = mfft.Plan(n, batch, lift, dtype=torch.complex128)
    assert plan.describe()["passes"][-1]["tile_width"] == 8
    rows = torch.from_numpy(np.random.default_rng(n).choice(batch, 3, replace=False)).to(dev)
    xr = x.view(batch, n)[rows].cpu().numpy()
    for name, sign, fn in (("forward", -1, plan.forward), ("adjoint", 1, plan.adjoint)):
        got = fn(x).view(batch, n)[rows].cpu().numpy()
        err = rel_err_rows(got, oracle.fft_batch(xr, sign, threads=8))
        print(f"c128 {batch} x {n} {lift} {name}: rel err {err:.3e}", flush=True)
        assert err <= tol(n, torch.complex128)
    plan.close()
    del x
    torch.cuda.empty_cache()


def test_wide_read_tiles_beyond_the_infinity_cache():
    """1024 transforms of 2^16 points (2^26 points): the first 256-point
    level reads 64-column tiles (rows 2 KB apart); four seeded rows of each
    direction against the oracle."""
    need_gpu()
    n, batch = 1 << 16, 1024
    dev = torch.device("cuda", 0)
    x = inputs.device_uniform_complex(n * batch, 26, torch.complex64, dev)
    plan = mfft.Plan(n, batch, None)
    assert [p["tile_width"] for p in plan.describe()["passes"]] == [64, 16]
    rows = torch.from_numpy(np.random.default_rng(26).choice(batch, 4, replace=False)).to(dev)
    xr = x.view(batch, n)[rows].cpu().numpy().astype(np.complex128)
    for name, sign, fn in (("forward", -1, plan.forward), ("adjoint", 1, plan.adjoint)):
        got = fn(x).view(batch, n)[rows].cpu().numpy().astype(np.complex128)
        err = rel_err_rows(got, oracle.fft_batch(xr, sign, threads=8))
        print(f"1024 x 2^16 {name}: rel err {err:.3e}", flush=True)
        assert err <= tol(n, torch.complex64)
    plan.close()


@pytest.mark.parametrize("n,batch,dtype,lift", [(1 << 20, 16, torch.complex64, [256, 4096]),
                                                (1 << 23, 2, torch.complex64, [256, 128, 256]),
                                                (1 << 25, 1, torch.complex64, [256, 4096, 32]),
                                                (1 << 23, 1, torch.complex128, [256, 256, 128])])
def test_default_lifts_on_the_full_vector(n, batch, dtype, lift):
    """The measured default lifts (a 4096-point level for complex64 at 2^19
    .. 2^23 points in batches of 2^24 points or more, <256 128 256> for 2^23
    points in batches of up to 2^25 points, <256 4096 n/2^20> from
    2^25, <256 256 n/2^16> for complex128 at 2^23 .. 2^26) on every element,
    both directions, against the oracle."""
    need_gpu()
    dev = torch.device("cuda", 0)
    x = inputs.device_uniform_complex(n * batch, 19, dtype, dev)
    plan = mfft.Plan(n, batch, None, dtype=dtype)
    assert plan.describe()["lift"] == lift
    xr = x.cpu().numpy().astype(np.complex128).reshape(batch, n)
    for name, sign, fn in (("forward", -1, plan.forward), ("adjoint", 1, plan.adjoint)):
        got = fn(x).cpu().numpy().astype(np.complex128).reshape(batch, n)
        err = rel_err_rows(got, oracle.fft_batch(xr, sign, threads=8))
        print(f"default lift {lift} {dtype} {name}: rel err {err:.3e}", flush=True)
        assert err <= tol(n, dtype)
    plan.close()


@pytest.mark.parametrize("n,batch,lift,w1,dtype", [
    (1 << 20, 256, [256, 4096], 32, torch.complex64), (1 << 21, 128, [512, 4096], 16, torch.complex64),
    (1 << 22, 64, [1024, 4096], 16, torch.complex64), (1 << 23, 32, [2048, 4096], 8, torch.complex64),
    (1 << 22, 8, [1024, 4096], 16, torch.complex64), (1 << 22, 4, [1024, 4096], 8, torch.complex128),
    (1 << 21, 16, [512, 4096], 8, torch.complex128)])
def test_far_writing_last_levels_beyond_the_infinity_cache(n, batch, lift, w1, dtype):
    """256 MiB to 2 GiB whose last level writes rows 32 KB apart, on the
    wide default tiles such levels take once a buffer outgrows the Infinity
    Cache (complex64: 32 columns at 256 points, 16 at 512 and 1024, 8 at
    2048; complex128: 8 columns): three seeded rows of each direction
    against the oracle."""
    need_gpu()
    dev = torch.device("cuda", 0)
    x = inputs.device_uniform_complex(n * batch, 28, dtype, dev)
    plan = mfft.Plan(n, batch, lift, dtype=dtype)
    assert plan.describe()["passes"][-1]["tile_width"] == w1
    rows = np.random.default_rng(n).choice(batch, 3, replace=False)
    ridx = torch.from_numpy(rows).to(dev)
    xr = x.view(batch, n)[ridx].cpu().numpy().astype(np.complex128)
    for name, sign, fn in (("forward", -1, plan.forward), ("adjoint", 1, plan.adjoint)):
        y = fn(x)
        got = y.view(batch, n)[ridx].cpu().numpy().astype(np.complex128)
        del y
        err = rel_err_rows(got, oracle.fft_batch(xr, sign, threads=8))
        print(f"{batch} x {n} {lift} {dtype} {name}: rel err {err:.3e}", flush=True)
        assert err <= tol(n, dtype)
    plan.close()
    del x
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_maximum_size_sparse_spectrum(dtype):
    """n = 2^30, the largest size the library plans (default lift).  The input
    is a sum of seeded complex exponentials generated on the device in FP64
    (phases from the exact integer product j k mod n), so the exact transform
    is n a_t at bin k_t (forward) or -k_t mod n (adjoint) and 0 elsewhere.
    The whole output is compared with that by relative L2, summed in FP64 in
    chunks on the device, to the same tolerance as the oracle comparisons."""
    need_gpu()
    n, C = 1 << 30, 1 << 24
    rng = np.random.default_rng(30)
    ks = sorted({0, 1, n // 2, n - 1, *(int(k) for k in rng.integers(0, n, 4))})
    amps = rng.uniform(-1, 1, len(ks)) + 1j * rng.uniform(-1, 1, len(ks))
    dev = torch.device("cuda", 0)
    kt = torch.tensor(ks, dtype=torch.int64, device=dev)
    at = torch.tensor(amps, dtype=torch.complex128, device=dev)
    x = torch.empty(n, dtype=dtype, device=dev)
    for s in range(0, n, C):
        j = torch.arange(s, s + C, dtype=torch.int64, device=dev)
        ph = ((j[:, None] * kt[None, :]) % n).to(torch.float64) * (2 * np.pi / n)
        x[s:s + C] = (torch.polar(torch.ones_like(ph), ph) * at[None, :]).sum(1).to(dtype)
        del j, ph
    plan = mfft.Plan(n, 1, None, dtype=dtype)
    den = n * float(np.sqrt(np.sum(np.abs(amps) ** 2)))
    for direction, bins in (("forward", ks), ("adjoint", [(-k) % n for k in ks])):
        y = plan.forward(x) if direction == "forward" else plan.adjoint(x)
        # Error at the tone bins, then the energy everywhere else (the bins
        # zeroed first: no difference of two sums of size n^2 |a|^2).
        idx = torch.tensor(bins, device=dev)
        yt = y[idx].to(torch.complex128).cpu().numpy()
        num2 = float(np.sum(np.abs(yt - n * amps) ** 2))
        y[idx] = 0
        for s in range(0, n, C):
            num2 += float((y[s:s + C].to(torch.complex128).abs() ** 2).sum())
        err = np.sqrt(num2) / den
        print(f"n=2^30 {dtype} {direction}: rel L2 {err:.3e} (lift {plan.describe()['lift']})", flush=True)
        assert err <= tol(n, dtype), (direction, err)
        del y
    plan.close()
    del x
    torch.cuda.empty_cache()


def test_misaligned_unit_stride_buffers_are_rejected():
    """Paired-column levels move column pairs with 16-byte accesses on their
    unit-stride side: a buffer 8 bytes off that alignment is refused before
    any launch (MOA_ERR_ARG), on the input of a first level and on the output
    of a last level, and the aligned calls still match the oracle."""
    need_gpu()
    n = 1 << 16
    x_np = inputs.uniform_complex(n, seed=9, dtype=np.complex64)
    want = oracle.fft(x_np.astype(np.complex128))
    x = to_dev(x_np, torch.complex64)
    buf = torch.zeros(n + 1, dtype=torch.complex64, device="cuda")
    mis = buf[1:]
    assert mis.data_ptr() % 16 == 8
    for lift, call in (([16, 4096], lambda p: p.forward(mis)),              # level 0 reads in pairs
                       ([4096, 16], lambda p: p.forward(x, out=mis))):      # last level writes in pairs
        p = mfft.Plan(n, 1, lift)
        with pytest.raises(capi.MoaError) as e:
            call(p)
        assert e.value.status == capi.MOA_ERR_ARG
        y = p.forward(x)
        torch.cuda.synchronize()
        assert rel_err_rows(y.cpu().numpy(), want) <= tol(n, torch.complex64)
        p.close()


def test_streaming_and_plain_input_loads_agree_bitwise():
    """The first level's loads of the caller's input run as streaming or as
    plain loads (tuning stream 1 / -1): same arithmetic, so the outputs
    are equal bit for bit, on the paired-column, the persistent and the
    uneven-batch kernels, and match the oracle."""
    need_gpu()
    for n, batch, lift in ((1 << 16, 1, [16, 4096]), (1 << 16, 2, [256, 256]), (1 << 12, 3, None)):
        x_np = inputs.uniform_complex((batch, n), seed=11, dtype=np.complex64)
        x = to_dev(x_np, torch.complex64)
        outs = []
        for mode in (1, -1):
            p = mfft.Plan(n, batch, lift, tuning={"stream": mode})
            assert p.describe()["stream"] == (mode == 1)
            outs.append(p.forward(x))
            p.close()
        torch.cuda.synchronize()
        assert torch.equal(outs[0], outs[1])
        want = oracle.fft(x_np.astype(np.complex128))
        assert rel_err_rows(outs[0].cpu().numpy(), want) <= tol(n, torch.complex64)
    sizes = [64, 16384, 1, 8192, 128, 4096]
    xb = to_dev(inputs.uniform_complex(sum(sizes), seed=12, dtype=np.complex64), torch.complex64)
    outs = []
    for mode in (1, -1):
        p = mfft.BatchedPlan(sizes, tuning={"stream": mode})
        outs.append(p.forward(xb))
        p.close()
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])


def test_in_place_and_determinism():
    need_gpu()
    n, batch = 1 << 16, 4
    x = inputs.uniform_complex((batch, n), seed=5, dtype=np.complex64)
    plan = mfft.Plan(n, batch, [256, 256])
    a = to_dev(x, torch.complex64)
    b = plan.forward(a)
    c = plan.forward(a)
    torch.cuda.synchronize()
    assert torch.equal(b, c)
    a2 = a.clone()
    plan.forward(a2, out=a2)
    torch.cuda.synchronize()
    assert torch.equal(a2, b)


def test_roundtrip_is_n_times_identity():
    need_gpu()
    n, batch = 1 << 14, 3
    x = inputs.uniform_complex((batch, n), seed=9, dtype=np.complex64)
    plan = mfft.Plan(n, batch, [128, 128])
    t = to_dev(x, torch.complex64)
    back = plan.adjoint(plan.forward(t)).cpu().numpy() / n
    assert rel_err_rows(back, x.astype(np.complex128)) <= 2 * tol(n, torch.complex64)


@pytest.mark.parametrize("cols", [1, 2, 4, 8])
def test_tuned_tile_widths(cols):
    need_gpu()
    n = 1 << 16
    x = inputs.uniform_complex((2, n), seed=cols, dtype=np.complex64).astype(np.complex128)
    got, plan = run_plan(n, 2, [256, 256], torch.complex64, x, tuning=dict(cols_per_block=[cols, cols]))
    assert plan.describe()["passes"][0]["tile_width"] == cols
    assert rel_err_rows(got, oracle.fft(x)) <= tol(n, torch.complex64)


def test_graph_replays_match_eager():
    need_gpu()
    n, batch = 1 << 16, 2
    x = inputs.uniform_complex((batch, n), seed=3, dtype=np.complex64)
    eager = mfft.Plan(n, batch, [256, 256])
    graph = mfft.Plan(n, batch, [256, 256], graph=True)
    t = to_dev(x, torch.complex64)
    ref = eager.forward(t)
    out = torch.empty_like(t)
    for _ in range(4):
        out.zero_()
        graph.forward(t, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        _ = eager.adjoint(ref)  # unrelated eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("n,batch,lift,dtype", [(1 << 10, 1, None, torch.complex128),
                                                (1 << 16, 2, [256, 256], torch.complex64)])
def test_launches_recorded_in_a_caller_graph(n, batch, lift, dtype):
    """The caller may record exec into its own HIP graph (torch capture on the
    capture stream): several back-to-back transforms, replayed with eager work
    and synchronisations between the replays, match the eager result bit for
    bit on every replay, and the eager result matches the oracle."""
    need_gpu()
    x_np = inputs.uniform_complex((batch, n), seed=11, dtype=np.complex64 if dtype == torch.complex64
                                  else np.complex128)
    plan = mfft.Plan(n, batch, lift, dtype=dtype)
    x = to_dev(x_np, dtype)
    ref = plan.forward(x)
    torch.cuda.synchronize()
    want = oracle.fft(np.asarray(x.cpu().numpy(), np.complex128))
    assert rel_err_rows(ref.cpu().numpy(), want) <= tol(n, dtype)
    outs = [torch.empty_like(x) for _ in range(3)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.forward(x, out=outs[0])
        plan.adjoint(outs[0], out=outs[1])
        plan.forward(x, out=outs[2])
    for _ in range(4):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(outs[0], ref) and torch.equal(outs[2], ref)
        assert torch.equal(outs[1], plan.adjoint(ref))
        _ = plan.adjoint(x)  # unrelated eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_short_transform_kernel_every_size(dtype):
    """The latency kernel (2^4..2^12 points; 2^11 for complex128): forward
    and adjoint against the oracle at every size it serves, in place equal to
    out of place, within tolerance of the level kernel the planner uses when a
    tile width is given, and in batches (one workgroup a transform)."""
    need_gpu()
    top = 12 if dtype == torch.complex64 else 11
    for lg in range(4, top + 1):
        n = 1 << lg
        x_np = inputs.uniform_complex(n, seed=100 + lg, dtype=np.complex64 if dtype == torch.complex64
                                      else np.complex128)
        plan = mfft.Plan(n, 1, None, dtype=dtype)
        assert plan.describe()["passes"][0]["kernel_mode"] == 4
        x = to_dev(x_np, dtype)
        xd = np.asarray(x.cpu().numpy(), np.complex128)
        for sign, run in ((-1, plan.forward), (1, plan.adjoint)):
            y = run(x)
            z = x.clone()
            run(z, out=z)
            torch.cuda.synchronize()
            assert torch.equal(y, z), (lg, sign)
            assert rel_err_rows(y.cpu().numpy(), oracle.fft(xd, sign)) <= tol(n, dtype), (lg, sign)
        level = mfft.Plan(n, 1, None, dtype=dtype, tuning={"cols_per_block": [1]})
        assert level.describe()["passes"][0]["kernel_mode"] != 4
        ref = level.forward(x).cpu().numpy()
        assert rel_err_rows(plan.forward(x).cpu().numpy(), ref.astype(np.complex128)) <= 2 * tol(n, dtype)
        plan.close()
        level.close()
    # a batch: one workgroup per transform
    for lg, B in ((4, 2048), (9, 5), (top, 3)):
        n = 1 << lg
        x_np = inputs.uniform_complex((B, n), seed=200 + lg, dtype=np.complex64 if dtype == torch.complex64
                                      else np.complex128)
        plan = mfft.Plan(n, B, None, dtype=dtype)
        assert plan.describe()["passes"][0]["kernel_mode"] == 4 and plan.describe()["passes"][0]["grid"] == B
        x = to_dev(x_np, dtype)
        xd = np.asarray(x.cpu().numpy(), np.complex128)
        assert rel_err_rows(plan.forward(x).cpu().numpy(), oracle.fft(xd)) <= tol(n, dtype), (lg, B)
        assert rel_err_rows(plan.adjoint(x).cpu().numpy(), oracle.fft(xd, 1)) <= tol(n, dtype), (lg, B)
        plan.close()
