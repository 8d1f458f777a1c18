"""What the learned step-time model gains over the FLOP-count model.

Step timings are measured live on the GPU for seeded circuits of the
cost-model corpus (grid circuits with 16 open qubits; here the ones of at
most 40 qubits, so that planning stays quick), each planned four ways
(one-shot and dynamic slicing, with and without branch merging).  The MLP is
trained by the library's own kernels on the training circuits and evaluated
on held-out circuits:

* prediction: held-out RMSE of log step time against the FLOP-count model
  fitted to the same samples (a least-squares line of log time on log
  multiply-adds per kernel class);
* decisions: each held-out circuit is planned with the FLOP-count model (the
  candidate with the fewest multiply-adds, branch merging judged by the
  roofline estimate) and with the learned model (finalized plan variants
  ranked by predicted job time), and both jobs are timed.
"""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N_TRAIN, N_HELD = 8, 4


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def trained():
    import torch
    assert torch.cuda.is_available()
    from paper_2103_03074_amd import costmodel, tn
    circs = [c for c in costmodel.corpus_circuits(60) if c["n"] <= 40][:N_TRAIN + N_HELD]
    assert len(circs) == N_TRAIN + N_HELD
    _say("cost model: timing", N_TRAIN, "training circuits, 4 plans each")
    X, Y, F, K, _ = costmodel.collect(circs[:N_TRAIN], groups=1, restarts=2, max_log2_size=22)
    _say("cost model: timing", N_HELD, "held-out circuits")
    Xt, Yt, Ft, Kt, _ = costmodel.collect(circs[N_TRAIN:], groups=1, restarts=2, max_log2_size=22)
    assert len(X) > 200 and len(Xt) > 50
    model = tn.Mlp(tn.STEP_FEATURES, 128, seed=0)
    losses = costmodel.train(model, X, Y, epochs=150)
    model.set_support(X.min(axis=0), X.max(axis=0), margin=0.05)
    return {"model": model, "losses": losses, "X": X, "Y": Y, "F": F, "K": K, "Xt": Xt, "Yt": Yt, "Ft": Ft,
            "Kt": Kt, "held": circs[N_TRAIN:]}


def test_learned_model_predicts_heldout_step_times_better_than_flop_count(trained):
    from paper_2103_03074_amd import costmodel
    t = trained
    assert t["losses"][-1] < 0.25 * t["losses"][0]
    coef = costmodel.fit_flop_model(t["F"], t["K"], t["Y"])
    rmse_mlp = float(np.sqrt(np.mean((costmodel.predict(t["model"], t["Xt"]) - t["Yt"]) ** 2)))
    rmse_flop = float(np.sqrt(np.mean((costmodel.flop_predict(coef, t["Ft"], t["Kt"]) - t["Yt"]) ** 2)))
    _say("held-out RMSE of log(ms): MLP", rmse_mlp, "FLOP model", rmse_flop)
    assert rmse_mlp < 0.6 * rmse_flop


def test_learned_model_plans_are_no_slower_than_flop_count_plans(trained):
    """Held-out circuits: the learned model's plan choices, timed, take no
    longer in total than the FLOP-count choices (5 % allowance for run-to-run
    noise of the timings); how many choices differ is reported."""
    from paper_2103_03074_amd import costmodel
    rows = costmodel.compare_choices(trained["held"], trained["model"], restarts=2, max_log2_size=22, groups=2)
    j0 = sum(r["flop_job_s"] for r in rows)
    j1 = sum(r["mlp_job_s"] for r in rows)
    differ = sum(not r["same_plan"] for r in rows)
    used = sum(r["mlp_used"] == 1 for r in rows)
    _say("plan choice: FLOP-chosen jobs", f"{j0:.4g}s", "MLP-chosen jobs", f"{j1:.4g}s",
         "choices differing", differ, "of", len(rows), "model used on", used)
    for r in rows:
        _say("  ", r)
    assert used >= 1
    assert j1 <= 1.05 * j0
