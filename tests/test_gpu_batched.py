"""GPU parity of the uneven batch (one fused launch with one workgroup per
task or a smaller persistent grid, per-size launches, graph replay) against
the FP64 oracle, per transform."""
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


def per_transform_errors(got, want, sizes):
    errs = []
    off = 0
    for s in sizes:
        g, w = got[off:off + s], want[off:off + s]
        errs.append(np.linalg.norm(g - w) / max(np.linalg.norm(w), 1e-300))
        off += s
    return np.array(errs)


def check(sizes, seed, threads, **kw):
    sizes = [int(s) for s in sizes]
    x = inputs.uniform_complex(sum(sizes), seed=seed, dtype=np.complex64)
    plan = mfft.BatchedPlan(sizes, **kw)
    t = torch.from_numpy(x).cuda()
    results = {}
    for name, sign, fn in (("forward", -1, plan.forward), ("adjoint", 1, plan.adjoint)):
        got = fn(t).cpu().numpy().astype(np.complex128)
        want = oracle.fft_packed(x.astype(np.complex128), sizes, sign, threads=threads)
        errs = per_transform_errors(got, want, sizes)
        bound = 2e-6 * np.maximum(1, np.log2(np.array(sizes)))
        print(f"batched {kw} {name}: max err/bound = {(errs / bound).max():.3f}", flush=True)
        assert np.all(errs <= bound)
        results[name] = got
    return results


@pytest.mark.parametrize("per_size", [False, True])
def test_small_uneven_batch(per_size):
    need_gpu()
    sizes = [64, 1, 2, 16384, 8, 8192, 128, 64, 4096, 16, 1024, 32, 2048, 512, 256, 4]
    check(sizes * 5, seed=1, threads=4, per_size=per_size)


def test_uneven_8192_transforms_2p6_to_2p14():
    need_gpu()
    sizes = inputs.uneven_sizes(8192, 6, 14, seed=0)
    import os
    r1 = check(sizes, seed=0, threads=min(16, os.cpu_count() or 1))
    # the per-size launches and the graph replay give the identical bits
    x = inputs.uniform_complex(int(sizes.sum()), seed=0, dtype=np.complex64)
    t = torch.from_numpy(x).cuda()
    per = mfft.BatchedPlan(list(sizes), per_size=True).forward(t)
    gp = mfft.BatchedPlan(list(sizes), graph=True)
    out = torch.empty_like(t)
    for _ in range(3):
        out.zero_()
        gp.forward(t, out=out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().astype(np.complex128), r1["forward"])
    assert np.array_equal(per.cpu().numpy().astype(np.complex128), r1["forward"])


@pytest.mark.parametrize("task_lg", [11, 12])
def test_tuned_task_packing(task_lg):
    """Smaller tasks (at most 2^11 or 2^12 points packed a workgroup) match
    the oracle, and give the same bits as the default packing: a transform's
    arithmetic does not depend on which task carries it."""
    need_gpu()
    sizes = [int(s) for s in inputs.uneven_sizes(600, 0, 14, seed=9)]
    r = check(sizes, seed=9, threads=4, tuning=dict(batch_task_lg=task_lg, persistent_blocks=97))
    x = torch.from_numpy(inputs.uniform_complex(sum(sizes), seed=9, dtype=np.complex64)).cuda()
    default = mfft.BatchedPlan(sizes).forward(x).cpu().numpy().astype(np.complex128)
    assert np.array_equal(default, r["forward"])


def test_persistent_grid_smaller_than_tasks():
    need_gpu()
    sizes = [1 << (6 + (i % 9)) for i in range(300)]
    check(sizes, seed=4, threads=4, tuning=dict(persistent_blocks=7))


def test_per_size_levels_compose_to_the_batch():
    """Running the size groups of a per-size plan one by one (exec_level)
    writes every transform once and equals the whole execution."""
    need_gpu()
    sizes = [int(s) for s in inputs.uneven_sizes(300, 0, 14, seed=5)]
    x = torch.from_numpy(inputs.uniform_complex(sum(sizes), seed=6, dtype=np.complex64)).cuda()
    plan = mfft.BatchedPlan(sizes, per_size=True)
    want = plan.forward(x)
    got = torch.zeros_like(x)
    assert plan.num_levels == len(set(sizes))
    for g in range(plan.num_levels):
        plan.run_level(g, x, got)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    whole = mfft.BatchedPlan(sizes)
    assert whole.num_levels == 1
    got2 = torch.zeros_like(x)
    whole.run_level(0, x, got2)
    torch.cuda.synchronize()
    assert torch.equal(got2, whole.forward(x))
