"""GPU parity of the split-precision matrix-core path (every radix-16 stage a
dense 16-point DFT on v_mfma_f32_16x16x32_{bf16,f16}) against the FP64 oracle.

Error bounds (relative L2 per transform):
  split fp16 (11 + 11 significant bits, dropped lo*lo term ~2^-22): the FP32
    bound 2e-6 * log2 n.
  split bf16 (8 + 8 bits, dropped lo*lo ~2^-16 per operand): S stages of
    relative error at most 2 * 2^-16 each, i.e. 2 * S * 2^-16, S = number of
    radix-16 stages on the matrix cores.
The measured errors are printed for the record.
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


def bound(prec, n, stages):
    if prec == "split_fp16":
        return 2e-6 * np.log2(n)
    return 2.0 * stages * 2.0 ** -16


def rows_err(got, want):
    return float((np.linalg.norm(got - want, axis=-1) / np.linalg.norm(want, axis=-1)).max())


@pytest.mark.parametrize("prec", ["split_fp16", "split_bf16"])
@pytest.mark.parametrize("n,batch,lift", [(256, 64, None), (4096, 4, None), (1 << 16, 2, [16, 4096]),
                                          (1 << 16, 2, [256, 256]), (1 << 20, 2, [256, 4096]),
                                          (1 << 12, 3, [16, 256]), (1 << 20, 2, [4096, 256]),
                                          (1 << 20, 16, None), (1 << 19, 16, None), (1 << 25, 1, None)])
def test_split_matches_oracle(prec, n, batch, lift):
    need_gpu()
    x = inputs.uniform_complex((batch, n), seed=n + batch, dtype=np.complex64)
    plan = mfft.Plan(n, batch, lift, prec=prec)
    d = plan.describe()
    stages = sum(int(np.log2(p["N"])) // 4 for p in d["passes"] if p["mfma"] != "none")
    assert stages >= 1
    t = torch.from_numpy(x).cuda()
    for name, sign, fn in (("forward", -1, plan.forward), ("adjoint", 1, plan.adjoint)):
        got = fn(t).cpu().numpy().astype(np.complex128).reshape(batch, n)
        want = oracle.fft(x.astype(np.complex128), sign)
        err = rows_err(got, want)
        print(f"{prec} n={n} batch={batch} lift={lift} {name}: rel err {err:.3e} "
              f"(bound {bound(prec, n, stages):.2e}, {stages} MFMA stages)", flush=True)
        assert err <= bound(prec, n, stages)


@pytest.mark.parametrize("prec", ["split_fp16", "split_bf16"])
@pytest.mark.parametrize("n,batch,lift", [(16, 64, None), (256, 4, None), (256, 2, [16, 16])])
def test_split_levels_with_too_few_transforms_run_fp32(prec, n, batch, lift):
    """A matrix-core tile gathers 2^11 points; a level with fewer transforms
    runs in FP32 under a split plan and meets the FP32 bound."""
    need_gpu()
    plan = mfft.Plan(n, batch, lift, prec=prec)
    assert any(p["mfma"] == "none" and p["N"] in (16, 256) for p in plan.describe()["passes"])
    x = inputs.uniform_complex((batch, n), seed=n + batch + 1, dtype=np.complex64)
    t = torch.from_numpy(x).cuda()
    for sign, fn in ((-1, plan.forward), (1, plan.adjoint)):
        got = fn(t).cpu().numpy().astype(np.complex128).reshape(batch, n)
        err = rows_err(got, oracle.fft(x.astype(np.complex128), sign))
        stages = sum(int(np.log2(p["N"])) // 4 for p in plan.describe()["passes"] if p["mfma"] != "none")
        print(f"{prec} n={n} batch={batch} lift={lift}: rel err {err:.3e}, {stages} MFMA stages", flush=True)
        assert err <= max(2e-6 * np.log2(n), bound(prec, n, stages))


@pytest.mark.parametrize("lift", [[256, 4096], [4096, 256]])
def test_b256_n2p20_sampled_rows(lift):
    """256 transforms of 2^20 points through either two-level lift; the
    oracle checks 8 seeded rows of each precision."""
    need_gpu()
    n, B = 1 << 20, 256
    dev = torch.device("cuda", 0)
    x = inputs.device_uniform_complex(n * B, 5, torch.complex64, dev)
    rows = np.random.default_rng(5).choice(B, 8, replace=False)
    xr = x.view(B, n)[torch.from_numpy(rows).to(dev)].cpu().numpy().astype(np.complex128)
    want = oracle.fft_batch(xr, -1, threads=8)
    errs = {}
    for prec in ("native", "split_fp16", "split_bf16"):
        plan = mfft.Plan(n, B, lift, prec=prec)
        y = plan.forward(x).view(B, n)
        got = y[torch.from_numpy(rows).to(dev)].cpu().numpy().astype(np.complex128)
        errs[prec] = rows_err(got, want)
        plan.close()
        del y
    print(f"256 x 2^20 lift {lift} errors: {errs}", flush=True)
    assert errs["native"] <= 2e-6 * 20
    assert errs["split_fp16"] <= 2e-6 * 20
    assert errs["split_bf16"] <= 2.0 * 5 * 2.0 ** -16


@pytest.mark.parametrize("prec", ["split_fp16", "split_bf16"])
@pytest.mark.parametrize("scale,kind", [(1e-4, "uniform"), (1e3, "uniform"), (1e3, "dc"), (1e-4, "dc"),
                                        (3e4, "dc"), (1.0, "mixed")])
@pytest.mark.parametrize("n,lift", [(1 << 20, [256, 4096]), (4096, None), (1 << 12, [16, 256])])
def test_split_input_range(prec, scale, kind, n, lift):
    """The split levels scale every tile by a power of two from its own data,
    so their error does not depend on the input's range: tiny inputs keep
    their low parts out of fp16's subnormal range, large or coherent (DC)
    inputs do not overflow it.  'dc' is a constant signal plus 1e-3 noise
    (all energy in one bin, the worst-case growth of every stage); 'mixed'
    has transforms of amplitude 1e-3 and 1e3 side by side in one batch."""
    need_gpu()
    batch = 2
    x = inputs.uniform_complex((batch, n), seed=n + 7, dtype=np.complex128)
    if kind == "dc":
        x = 1.0 + 1e-3 * x
    if kind == "mixed":
        x = x * np.array([[1e-3], [1e3]])
    x = (scale * x).astype(np.complex64)
    plan = mfft.Plan(n, batch, lift, prec=prec)
    d = plan.describe()
    stages = sum(int(np.log2(p["N"])) // 4 for p in d["passes"] if p["mfma"] != "none")
    t = torch.from_numpy(x).cuda()
    for name, sign, fn in (("forward", -1, plan.forward), ("adjoint", 1, plan.adjoint)):
        got = fn(t).cpu().numpy().astype(np.complex128).reshape(batch, n)
        assert np.isfinite(got).all()
        want = oracle.fft(x.astype(np.complex128), sign)
        err = rows_err(got, want)
        print(f"{prec} {kind} scale {scale:g} n={n} lift={lift} {name}: rel err {err:.3e}", flush=True)
        assert err <= bound(prec, n, stages)
    plan.close()
