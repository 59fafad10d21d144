"""Host logic of the schedule autotuner: the candidate set it measures."""
import itertools

from paper_2606_05687_amd import autotune


def test_candidate_grid_short_horizons():
    cands = list(autotune.candidates(20))
    assert len(cands) == 5 * 2 * 3 * 3
    assert {c["form"] for c in cands} == {1}              # fused form up to 40 stages
    assert {c["iters"] for c in cands} == {3, 5, 10, 20, 50}
    assert {c["rho"] for c in cands} == {10.0, 30.0}
    assert {c["refine_passes"] for c in cands} == {8, 12, 16}
    assert {c["first_passes"] for c in cands} == {0, 2, 4}
    assert {c["precision"] for c in cands} == {0}
    # every combination exactly once
    keys = {tuple(sorted(c.items())) for c in cands}
    assert len(keys) == len(cands)
    # at least three ADMM sweeps before the refinement
    assert min(c["iters"] for c in cands) >= 3


def test_candidate_grid_long_horizons_and_bf16():
    cands = list(autotune.candidates(60, allow_bf16=True))
    assert {c["form"] for c in cands} == {-1}             # packed by horizon class beyond 40
    assert {c["precision"] for c in cands} == {0, 1}
    assert len(cands) == 2 * 5 * 2 * 3 * 3
    for a, b in itertools.combinations(cands[:6], 2):
        assert a != b
