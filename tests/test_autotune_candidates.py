"""Host logic of the autotuner's candidate set (no GPU): every candidate is a
launch shape the library has a kernel for, and for mixed-precision DOPRI5
both policies of placing the FP64 work are timed."""
import paper_1706_07062_amd as K
from paper_1706_07062_amd import autotune


def _cands(**kw):
    return list(autotune.candidates(K.kh_default_params(**kw)))


def test_fp64_and_fp32_candidates_keep_the_policy_off():
    for prec, waves in ((K.P64, {1, 3, 4}), (K.P32, {1, 4, 5})):
        c = _cands(precision=prec)
        assert {d["mixed_split"] for d in c} == {0}
        assert {d["waves_per_eu"] for d in c} == waves
        assert len(c) == 3 * len(waves) * 4


def test_mixed_dopri5_times_both_policies():
    c = _cands(precision=K.PMIXED)
    per_wave = [d for d in c if d["mixed_split"] == 0]
    split = [d for d in c if d["mixed_split"] == 1]
    assert {d["waves_per_eu"] for d in per_wave} == {1, 3, 4}
    # the first pass of the split is built for two register budgets only
    assert {d["waves_per_eu"] for d in split} == {1, 3}
    assert len(per_wave) == 36 and len(split) == 24
    assert all(d["block_size"] in (64, 128, 256) and d["refill_min"] in (4, 8, 12, 16) for d in c)


def test_other_methods_keep_the_callers_policy():
    for method in (K.RK4, K.DOPRI5_T):
        c = _cands(method=method, precision=K.PMIXED)
        assert {d["mixed_split"] for d in c} == {0}
        assert {d["waves_per_eu"] for d in c} == {1}
    applied = autotune.apply(K.kh_default_params(precision=K.PMIXED), {"mixed_split": 1, "waves_per_eu": 3})
    assert applied.mixed_split == 1 and applied.waves_per_eu == 3 and applied.precision == K.PMIXED
