"""GPU parity of the level kernel with register stages of radix 4, 8 and 32
(the general-radix block of Ch. 1, selected per level through the tuning
block) against the FP64 oracle, for every kernel variant those schedules
instantiate (points per thread, workgroup shape, unit-stride sides), both
directions.  Tolerance: relative L2 per transform <= 2e-6 log2 n.
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


def rel_err_rows(got, want):
    got = np.asarray(got, np.complex128).reshape(want.shape)
    return float((np.linalg.norm(got - want, axis=-1) / np.linalg.norm(want, axis=-1)).max())


CASES = [
    # (n, batch, lift, lg_radix per level)
    (1 << 5, 64, None, [2]), (1 << 5, 64, None, [3]), (1 << 5, 64, None, [5]),
    (1 << 7, 16, None, [2]), (1 << 7, 16, None, [3]), (1 << 7, 16, None, [5]),
    (1 << 10, 8, None, [2]), (1 << 10, 8, None, [3]), (1 << 10, 8, None, [5]),
    (1 << 13, 3, None, [2]), (1 << 13, 3, None, [3]), (1 << 13, 3, None, [5]),
    (1 << 14, 2, None, [2]), (1 << 14, 2, None, [3]), (1 << 14, 2, None, [5]),
    (1 << 16, 2, [256, 256], [3, 2]), (1 << 16, 2, [256, 256], [5, 3]), (1 << 16, 2, [256, 256], [2, 5]),
    (1 << 18, 1, [64, 4096], [5, 2]), (1 << 18, 1, [64, 4096], [3, 3]), (1 << 18, 1, [64, 4096], [2, 0]),
    (1 << 20, 1, [1024, 1024], [5, 5]), (1 << 20, 1, [1024, 1024], [3, 0]),
    (1 << 19, 1, [32, 16384], [0, 5]), (1 << 19, 1, [32, 16384], [2, 3]),
    (1 << 21, 1, [128, 128, 128], [5, 3, 2]), (1 << 18, 1, [64, 64, 64], [2, 5, 3]),
    (1 << 24, 1, [4096, 4096], [5, 3]),
    (1 << 17, 2, [4096, 32], [2, 2]), (1 << 17, 1, [4096, 32], [3, 3]),   # the last level on 1024 threads
]


@pytest.mark.parametrize("n,batch,lift,lg_radix", CASES)
def test_radix_schedules_match_oracle(n, batch, lift, lg_radix):
    need_gpu()
    try:
        plan = mfft.Plan(n, batch, lift, tuning={"lg_radix": lg_radix})
    except capi.MoaError as e:
        pytest.fail(f"schedule {lg_radix} of {lift} did not plan: {e}")
    d = plan.describe()
    x = inputs.uniform_complex((batch, n), seed=n + sum(lg_radix), dtype=np.complex64)
    xd = torch.from_numpy(x).cuda()
    want_f = oracle.fft_batch(x.astype(np.complex128), -1, threads=8)
    want_a = oracle.fft_batch(x.astype(np.complex128), 1, threads=8)
    tol = 2e-6 * np.log2(n)
    for fn, want, name in ((plan.forward, want_f, "forward"), (plan.adjoint, want_a, "adjoint")):
        got = fn(xd)
        torch.cuda.synchronize()
        err = rel_err_rows(got.cpu().numpy(), want)
        print(f"radix n={n} b={batch} lift={lift} lg_radix={lg_radix} {name}: err {err:.3e} "
              f"{[(p['kernel_mode'], p['lg_radix'], p['in_tile_fast'], p['out_tile_fast']) for p in d['passes']]}",
              flush=True)
        assert err <= tol, d["passes"]
    plan.close()


def test_every_radix_kernel_variant_is_covered():
    """The cases above reach every (radix, points per thread, unit-stride
    sides) variant of the other-radix level kernel that the planner emits for
    any lift of up to three levels (swept on the host)."""
    import itertools

    def variants(n, batch, lift, lg):
        try:
            h = capi.moa_fft_plan(n, batch, lift, flags=capi.MOA_FFT_FLAG_HOST_ONLY, tuning={"lg_radix": lg})
        except capi.MoaError:
            return set()
        out = {(p["lg_radix"], p["kernel_mode"], p["in_tile_fast"], p["out_tile_fast"])
               for p in json.loads(capi.moa_fft_describe(h))["passes"] if p["lg_radix"] != 4 and p["kernel_mode"] != 4}
        capi.moa_fft_destroy(h)
        return out
    seen = set()
    for n, batch, lift, lg in CASES:
        seen |= variants(n, batch, lift, lg)
    emitted = set()
    for L in (1, 2, 3):
        for parts in itertools.product(range(1, 15), repeat=L):
            if sum(parts) > 24:
                continue
            lift = [1 << q for q in parts]
            n = int(np.prod(lift))
            for g in (2, 3, 5):
                for batch in (1, 3):
                    emitted |= variants(n, batch, lift, [g] * L)
    print("emitted", sorted(emitted), "covered", sorted(seen), flush=True)
    assert emitted <= seen, sorted(emitted - seen)
