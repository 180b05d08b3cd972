"""Host-side tests of the autotuner's candidate space (no GPU)."""
import numpy as np

from paper_0803_2386_amd import capi, tune


def test_lift_candidates_cover_paper_blockings():
    n = 1 << 24
    cands = tune.lift_candidates(n)
    assert [4096, 4096] in cands
    # the paper's uniform blocking n = 2^p_max c^l_max for c = 256: <256 256 256>
    assert [256, 256, 256] in cands
    # c = 2^12 with d = 24 gives p_max = 12: <4096 4096>; c = 2^13: <2^11 2^13>
    assert [2048, 8192] in cands
    for c in cands:
        assert int(np.prod(c)) == n
        assert all(f <= capi.moa_fft_max_block(capi.MOA_C64) for f in c)
        assert len(c) <= 3


def test_single_level_when_it_fits():
    assert [1 << 12] in tune.lift_candidates(1 << 12)
    assert all(len(c) >= 2 for c in tune.lift_candidates(1 << 14, capi.MOA_C128))


def test_candidates_plan_on_host():
    cands = tune.candidates(1 << 16, 4)
    assert len(cands) > 5
    lifts = {tuple(l) for l, _ in cands}
    assert (256, 256) in lifts and (1 << 16,) not in lifts


def test_cache_key_names_the_search_and_the_library():
    k_full = tune._key("dev", capi.MOA_C64, 1 << 16, 8, 0, 3, None, 5)
    k_cut = tune._key("dev", capi.MOA_C64, 1 << 16, 8, 0, 3, 12, 5)
    k_deep = tune._key("dev", capi.MOA_C64, 1 << 16, 8, 0, 4, None, 5)
    assert len({k_full, k_cut, k_deep}) == 3
    assert tune.library_digest() in k_full


def test_radix_candidates_change_one_level_and_plan():
    cands = tune.radix_candidates(1 << 16, 4, [256, 256], None, capi.MOA_C64, 0)
    assert cands, "no radix candidates"
    for t in cands:
        lr = t["lg_radix"]
        assert sum(1 for v in lr if v) == 1 and set(lr) <= {0, 2, 3, 5}
    # complex128 levels keep radix 16: no candidates
    assert tune.radix_candidates(1 << 16, 4, [256, 256], None, capi.MOA_C128, 0) == []
    k = tune._key("dev", capi.MOA_C64, 1 << 16, 8, 0, 3, None, 5, radix=False)
    assert k != tune._key("dev", capi.MOA_C64, 1 << 16, 8, 0, 3, None, 5, radix=True)


def test_split_precision_tunes_matrix_core_lifts_only():
    """A split-precision request is tuned over lifts with a level on the
    matrix cores (16, 256 or 4096 points); FP32 tunes over every lift."""
    n, B = 1 << 20, 256
    native = tune.first_round_lifts(n, B)
    assert [1024, 1024] in native and [4096, 256] in native
    for prec in (capi.MOA_FFT_PREC_SPLIT_BF16, capi.MOA_FFT_PREC_SPLIT_FP16):
        split = tune.first_round_lifts(n, B, prec=prec)
        assert [4096, 256] in split and [256, 4096] in split and [16, 256, 256] in split
        assert [1024, 1024] not in split and [512, 2048] not in split
        assert all(any(f in (16, 256, 4096) for f in lift) for lift in split)
        assert set(map(tuple, split)) < set(map(tuple, native))
    # no lift of 2^2 points has a matrix-core level: split tunes over all of them
    assert tune.first_round_lifts(4, 64, prec=capi.MOA_FFT_PREC_SPLIT_BF16) == tune.first_round_lifts(4, 64)
