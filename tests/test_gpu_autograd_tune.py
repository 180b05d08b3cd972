"""GPU: the differentiable workload (forward + hand-written adjoint through
torch.autograd) against the FP64 oracle's analytic gradient, and the
autotuner's chosen plan against the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_0803_2386_amd import inputs, tune  # noqa: E402
from paper_0803_2386_amd import fft as mfft  # noqa: E402

pytestmark = pytest.mark.gpu


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_b256_n2p16_weighted_power_loss_gradient():
    """loss = sum_k w_k |FFT(x)_k|^2 over 256 x 2^16 (lift <256 256>); the
    gradient is the adjoint kernel applied to 2 w . X.  Eight seeded rows are
    checked against the FP64 analytic gradient 2 F^H (w . F x) of the oracle,
    and 12 coordinates of one row against FP64 central differences
    (h = 1e-6) of the oracle's loss at the same input."""
    need_gpu()
    n, B = 1 << 16, 256
    dev = torch.device("cuda", 0)
    x = inputs.device_uniform_complex(n * B, 11, torch.complex64, dev).view(B, n).requires_grad_(True)
    w_np = inputs.loss_weights(n, seed=11)
    w = torch.from_numpy(w_np).to(dev, torch.float32)
    y = mfft.FFTFunction.apply(x, [256, 256])
    loss = (w * (y.real ** 2 + y.imag ** 2)).sum()
    loss.backward()
    torch.cuda.synchronize()
    rows = np.random.default_rng(11).choice(B, 8, replace=False)
    xr = x.detach()[torch.from_numpy(rows).to(dev)].cpu().numpy().astype(np.complex128)
    L_ref, g_ref = oracle.weighted_power_loss(xr, w_np, threads=8)
    g = x.grad[torch.from_numpy(rows).to(dev)].cpu().numpy().astype(np.complex128)
    err = float((np.linalg.norm(g - g_ref, axis=1) / np.linalg.norm(g_ref, axis=1)).max())
    yr = y.detach()[torch.from_numpy(rows).to(dev)].cpu().numpy().astype(np.complex128)
    L_rows = float((w_np * np.abs(yr) ** 2).sum())
    print(f"256 x 2^16 grad rel err {err:.3e}; loss(rows) {L_rows:.6e} vs {L_ref:.6e}", flush=True)
    # FP32 bound of one transform of n = 2^16 points: 2e-6 log2 n.
    tol = 2e-6 * 16
    assert err <= tol
    assert abs(L_rows - L_ref) / L_ref <= tol
    # FP64 central differences (h = 1e-6) of the loss of one row at the
    # values the GPU saw, at 12 seeded coordinates, real and imaginary
    # parts: torch's gradient of a real loss is dL/dRe + i dL/dIm.
    h = 1e-6
    x0 = xr[0]
    coords = np.random.default_rng(12).choice(n, 12, replace=False)
    scale = float(np.sqrt(np.mean(np.abs(g_ref[0]) ** 2)))

    def loss_diff(xp, xm):
        # L(xp) - L(xm), the two sums subtracted term by term (the loss is
        # about 1e9 here: subtracting the two totals would lose the digits
        # a step of 1e-6 changes)
        Xp, Xm = oracle.fft(xp), oracle.fft(xm)
        return float(np.sum(w_np * ((Xp.real ** 2 + Xp.imag ** 2) - (Xm.real ** 2 + Xm.imag ** 2))))

    worst = 0.0
    for j in coords:
        parts = []
        for step in (h, 1j * h):
            xp, xm = x0.copy(), x0.copy()
            xp[j] += step
            xm[j] -= step
            parts.append(loss_diff(xp, xm) / (2 * h))
        g_fd = parts[0] + 1j * parts[1]
        worst = max(worst, abs(g[0, j] - g_fd) / scale)
    print(f"256 x 2^16 GPU gradient vs FP64 central differences: max |diff| / rms(grad) = {worst:.3e}", flush=True)
    assert worst <= tol


def test_adjoint_identity_on_gpu():
    need_gpu()
    n, B = 1 << 14, 4
    x = inputs.uniform_complex((B, n), 3, np.complex64)
    yv = inputs.uniform_complex((B, n), 4, np.complex64)
    plan = mfft.Plan(n, B, [128, 128])
    tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(yv).cuda()
    Fx = plan.forward(tx).cpu().numpy().astype(np.complex128)
    FHy = plan.adjoint(ty).cpu().numpy().astype(np.complex128)
    lhs = np.vdot(yv.astype(np.complex128), Fx)
    rhs = np.vdot(FHy, x.astype(np.complex128))
    assert abs(lhs - rhs) / abs(lhs) < 1e-5


def test_tuner_picks_a_correct_plan(tmp_path, monkeypatch):
    need_gpu()
    monkeypatch.setenv("MOA_FFT_TUNE_CACHE", str(tmp_path / "tune.json"))
    n, B = 1 << 16, 8
    best = tune.tune(n, B, reps=2, candidates_limit=12, verbose=True)
    assert best["tried"] >= 2 and best["ms"] > 0
    again = tune.tune(n, B, reps=2, candidates_limit=12)   # served from the cache
    assert again["lift"] == best["lift"]
    plan = tune.tuned_plan(n, B, reps=2, candidates_limit=12)
    x = inputs.uniform_complex((B, n), 5, np.complex64)
    got = plan.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.complex128)
    want = oracle.fft(x.astype(np.complex128))
    err = float((np.linalg.norm(got - want, axis=1) / np.linalg.norm(want, axis=1)).max())
    assert err <= 2e-6 * 16
    g = tune.tune_batched([64, 4096, 16384, 512] * 20, grids=(0, 64), reps=2)
    assert g["ms"] > 0


def test_tuner_radix_round_picks_a_correct_plan(tmp_path, monkeypatch):
    """The radix round of the tuner (register radix 4 / 8 / 32 per level)
    on 64 transforms of 2^14 points; whatever it picks matches the oracle."""
    need_gpu()
    monkeypatch.setenv("MOA_FFT_TUNE_CACHE", str(tmp_path / "tune.json"))
    n, B = 1 << 14, 64
    best = tune.tune(n, B, max_levels=1, reps=3, refine=1, verbose=True)
    assert best["tried"] >= 4
    plan = mfft.Plan(n, B, best["lift"], tuning=best["tuning"])
    x = inputs.uniform_complex((B, n), 6, np.complex64)
    got = plan.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.complex128)
    want = oracle.fft(x.astype(np.complex128))
    err = float((np.linalg.norm(got - want, axis=1) / np.linalg.norm(want, axis=1)).max())
    print(f"tuned 64 x 2^14: {best['tuning']} {best['ms']:.4f} ms, err {err:.3e}", flush=True)
    assert err <= 2e-6 * 14


def test_tuner_split_precision_keeps_the_matrix_cores(tmp_path, monkeypatch):
    """Tuning a split-precision plan of 16 x 2^16 picks a lift with a
    matrix-core level, and that plan meets the split-bf16 bound."""
    need_gpu()
    monkeypatch.setenv("MOA_FFT_TUNE_CACHE", str(tmp_path / "tune.json"))
    n, B = 1 << 16, 16
    best = tune.tune(n, B, prec="split_bf16", reps=2, refine=2, radix=False, verbose=True)
    plan = mfft.Plan(n, B, best["lift"], prec="split_bf16", tuning=best["tuning"])
    stages = sum(int(np.log2(p["N"])) // 4 for p in plan.describe()["passes"] if p["mfma"] != "none")
    assert stages >= 1
    x = inputs.uniform_complex((B, n), 8, np.complex64)
    got = plan.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.complex128)
    want = oracle.fft(x.astype(np.complex128))
    err = float((np.linalg.norm(got - want, axis=1) / np.linalg.norm(want, axis=1)).max())
    print(f"tuned split bf16 16 x 2^16: {best['lift']} {best['tuning']} {best['ms']:.4f} ms, err {err:.3e}, "
          f"{stages} MFMA stages", flush=True)
    assert err <= 2.0 * stages * 2.0 ** -16
