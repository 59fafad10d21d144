"""Host logic of the schedule autotuner: the candidate sets it measures."""
from paper_2606_05687_amd import autotune


def test_first_stage_grid_short_horizons():
    cands = list(autotune.stage_a(20))
    assert len(cands) == 4 * 9
    assert {c["form"] for c in cands} == {1}              # fused form up to 40 stages
    assert {c["iters"] for c in cands} == {1, 2, 3, 5, 10, 20, 50, 100, 200}
    assert {c["rho"] for c in cands} == {1.0, 3.0, 10.0, 30.0}
    assert {c["refine_passes"] for c in cands} == {12}
    assert {c["first_passes"] for c in cands} == {0}
    assert {c["precision"] for c in cands} == {0}
    keys = {tuple(sorted(c.items())) for c in cands}
    assert len(keys) == len(cands)
    # a single ADMM sweep is a candidate: the refinement may not need more
    assert min(c["iters"] for c in cands) == 1


def test_second_stage_varies_only_the_refinement_budget():
    best = dict(form=1, iters=3, rho=10.0, refine_passes=12, first_passes=0, precision=0,
                group=1)
    cands = list(autotune.stage_b(best, 20))
    assert len(cands) == 5 * 3 * 2 - 1                  # the base point is not re-measured
    for c in cands:
        assert {k: c[k] for k in ("form", "iters", "rho", "precision")} == \
            {k: best[k] for k in ("form", "iters", "rho", "precision")}
    assert {(c["refine_passes"], c["first_passes"], c["group"]) for c in cands} | {(12, 0, 1)} \
        == {(a, b, g) for a in (2, 4, 8, 12, 16) for b in (0, 2, 4) for g in (1, 2)}
    # problems per workgroup that fit 1024 threads: 512 per problem at 20 stages,
    # 256 at 10, 1024 at 40
    assert autotune.groups_for(20) == (1, 2) and autotune.groups_for(10) == (1, 2, 4)
    assert autotune.groups_for(40) == (1,)
    assert autotune.groups_for(60) == (1, 2)             # packed: the 20-stage class


def test_long_horizons_and_bf16():
    cands = list(autotune.stage_a(60, allow_bf16=True))
    assert {c["form"] for c in cands} == {-1}             # packed by horizon class beyond 40
    assert {c["precision"] for c in cands} == {0, 1}
    assert len(cands) == 2 * 4 * 9
    full = list(autotune.candidates(60, allow_bf16=True))
    assert len({tuple(sorted(c.items())) for c in full}) == len(full)


def test_third_stage_chooses_the_backward_recursion():
    best = dict(form=1, iters=2, rho=1.0, refine_passes=12, first_passes=0, precision=0,
                group=1, scan=0)
    cands = list(autotune.stage_c(best, 20))
    assert [c["scan"] for c in cands] == [2, 4, 8]
    for c in cands:
        assert {k: v for k, v in c.items() if k != "scan"} == \
            {k: v for k, v in best.items() if k != "scan"}
    assert list(autotune.stage_c(best, 7)) == []          # too short to cut: sequential only
    assert {c["scan"] for c in autotune.stage_a(20)} == {0}
