"""Host logic of the training driver (no GPU): the evaluation workloads by
grid and the per-seed markdown record."""
from paper_2502_04217_amd import learn
from paper_2502_04217_amd import workload as wl


def test_eval_families_and_seeds():
    assert learn.eval_seeds(128, 3) == [10000, 10001, 10002]      # held out of training seeds 0-199
    assert learn.eval_seeds(256, 3) == [1, 2, 3]
    assert learn.eval_seeds(512, 2) == [1, 2]
    assert learn.EVAL_FAMILIES[128][0] is wl.grid128_family
    assert learn.EVAL_FAMILIES[256][0] is wl.grid256
    assert learn.EVAL_FAMILIES[512][0] is wl.grid512
    assert not set(learn.eval_seeds(128, 50)) & set(learn.TRAIN_SEEDS)


def test_markdown_record():
    row = {"seed": 1, "name": "grid256-s1", "missing": 0.03}
    for k in ("fp64_plain", "fp64_learned", "fp32_plain", "fp32_learned"):
        row[k] = {"cg": 17, "ipm": 9, "s": 0.019, "fallbacks": 0, "rel_kkt": 6e-7, "status": 0}
    summ = learn.summarize([row])
    assert summ["cg_ratio_fp32"] == 1.0 and summ["time_ratio_fp64"] == 1.0
    md = learn.markdown([row], summ, "python -m paper_2502_04217_amd.learn --eval-only --eval-grid 256", "p", grid=256)
    assert md.startswith("# Learned preconditioner correction on held-out 256^3 problems")
    assert "the 256^3 recipe" in md and "| 1 | 0.0300 |" in md
