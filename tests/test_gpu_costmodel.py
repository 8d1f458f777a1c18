"""What the learned step-time model gains over the FLOP-count model.

Step timings are measured live on the GPU for a few seeded circuits of the
cost-model corpus (36-53 qubits, 12-20 cycles); the MLP is trained on some
circuits by the library's own kernels and evaluated on the others, against
the FLOP-count model fitted to the same training samples (a least-squares
line of log time on log multiply-adds per kernel class).
"""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def test_learned_model_predicts_heldout_step_times_better_than_flop_count():
    import torch
    assert torch.cuda.is_available()
    from paper_2103_03074_amd import costmodel, tn
    circs = costmodel.corpus_circuits(12)
    _say("cost model: timing 9 training circuits")
    X, Y, F, K, _ = costmodel.collect(circs[:9], groups=1, restarts=2, max_log2_size=22)
    _say("cost model: timing 3 held-out circuits")
    Xt, Yt, Ft, Kt, _ = costmodel.collect(circs[9:], groups=1, restarts=2, max_log2_size=22)
    assert len(X) > 200 and len(Xt) > 50
    model = tn.Mlp(tn.STEP_FEATURES, 128, seed=0)
    losses = costmodel.train(model, X, Y, epochs=150)
    assert losses[-1] < 0.25 * losses[0]
    coef = costmodel.fit_flop_model(F, K, Y)
    rmse_mlp = float(np.sqrt(np.mean((costmodel.predict(model, Xt) - Yt) ** 2)))
    rmse_flop = float(np.sqrt(np.mean((costmodel.flop_predict(coef, Ft, Kt) - Yt) ** 2)))
    _say("held-out RMSE of log(ms): MLP", rmse_mlp, "FLOP model", rmse_flop)
    assert rmse_mlp < 0.6 * rmse_flop
