"""Learned step-time model: timing corpus, training and evaluation.

The corpus is built from seeded random grid circuits of 36-53 qubits and
12-20 cycles with 16 open qubits.  Each circuit is planned four ways
(one-shot and dynamic slicing, with and without branch merging), a few launch
groups of each plan are contracted with the library's per-step HIP-event
timing on, and every slice-dependent step contributes one sample: (features
of its shape, log of its mean milliseconds per launch).  Training
runs the library's own MLP kernels (forward, backward, Adam).  Evaluation on
held-out circuits compares

* prediction error (log ms) of the MLP with the FLOP-count model (a
  least-squares fit of log time on log complex multiply-adds per kernel
  class, the paper's cost 2^(nA+nB+nAB) made into a time), and
* the measured time of the plan each picks: the FLOP-count model takes the
  candidate with the fewest multiply-adds (branch merging judged by the
  roofline estimate), the learned model ranks finalized plan variants (the
  four cheapest candidates, each unmerged and merged) by predicted job time.

Everything numeric (contraction, timing, training, inference) happens in the
library; this module only moves data between calls.

    python -m paper_2103_03074_amd.costmodel --circuits 200 --out result.json
"""

import argparse
import json
import math
import sys
import time

import numpy as np

from . import tn, runtime


def log(*a):
    print("[costmodel]", *a, file=sys.stderr, flush=True)


def corpus_circuits(count, seed0=0):
    import rqc
    from rqc.generate import cost_model_corpus
    return cost_model_corpus(count=count, seed0=seed0, n_open=16)


def time_groups(plan, groups, profile):
    """Contract `groups` launch groups; returns (seconds per group, profile)."""
    import torch
    s = plan.stats()
    ws = runtime.workspace(plan)
    acc = runtime.accumulator(plan)
    per = 2 ** s["batch_log2"]
    n = min(s["n_slices"], per * groups)
    plan.contract_slices(ws, acc, 0, per)          # warm-up (also computes invariant tensors)
    torch.cuda.synchronize()
    if profile:
        plan.set_profiling(True)
    t0 = time.perf_counter()
    plan.contract_slices(ws, acc, 0, n)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(1, n // per)
    prof = plan.step_profile() if profile else None
    if profile:
        plan.set_profiling(False)
    return dt, prof


# Plan variants timed per training circuit, so that the samples cover the
# steps of every kind of plan the learned model later ranks: one-shot and
# dynamic slicing, with and without branch merging.
VARIANTS = [dict(branch_merge=0, slicing=1), dict(branch_merge=1, slicing=0),
            dict(branch_merge=0, slicing=2), dict(branch_merge=1, slicing=1)]


def collect(circs, groups=2, restarts=6, max_log2_size=24, variants=None):
    X, Y, F, K, owner = [], [], [], [], []
    variants = VARIANTS if variants is None else variants
    for i, c in enumerate(circs):
        t0 = time.perf_counter()
        n_steps = 0
        for v in variants:
            p = tn.Plan(c["circuit"], c["open_q"], c["fixed_q"], c["bits"], restarts=restarts,
                        max_log2_size=max_log2_size, seed=0, **v)
            feats = tn.plan_step_features(p)
            _, prof = time_groups(p, groups, True)
            for f, st in zip(feats, prof[:len(feats)]):
                if st["launches"] == 0 or st["total_ms"] <= 0:
                    continue
                X.append(f)
                Y.append(math.log(st["total_ms"] / st["launches"]))
                F.append(math.log(max(st["cmacs"], 1.0)))
                K.append(st["kernel"])
                owner.append(i)
            n_steps += len(feats)
            p.close()
        log(f"circuit {i}: n={c['n']} m={c['cycles']} steps={n_steps} over {len(variants)} plans "
            f"({time.perf_counter() - t0:.1f}s)")
    return (np.array(X, dtype=np.float32), np.array(Y, dtype=np.float32), np.array(F), np.array(K),
            np.array(owner))


def job_seconds(plan, groups):
    """Steady-state seconds per launch group (graph replays) times the number
    of launch groups of the job."""
    s = plan.stats()
    g, _ = time_groups(plan, groups, False)
    return g * 2 ** (s["n_sliced"] - s["batch_log2"])


def same_plan(a, b):
    return (a["cmacs_per_batch"] == b["cmacs_per_batch"] and a["n_sliced"] == b["n_sliced"]
            and a["batch_log2"] == b["batch_log2"] and a["bytes_per_batch"] == b["bytes_per_batch"])


def compare_choices(circs, model, restarts, max_log2_size, groups=2):
    """Plan each circuit with the FLOP-count model (branch merging judged by
    the roofline estimate) and with the learned model (ranking finalized plan
    variants by predicted job time); time both jobs."""
    rows = []
    for i, c in enumerate(circs):
        p0 = tn.Plan(c["circuit"], c["open_q"], c["fixed_q"], c["bits"], restarts=restarts,
                     max_log2_size=max_log2_size, seed=0, branch_merge=1, cost_model=0)
        p1 = tn.Plan(c["circuit"], c["open_q"], c["fixed_q"], c["bits"], restarts=restarts,
                     max_log2_size=max_log2_size, seed=0, branch_merge=1, cost_model=1, model=model)
        s0, s1 = p0.stats(), p1.stats()
        j0 = job_seconds(p0, groups)
        j1 = job_seconds(p1, groups)
        rows.append({"n": c["n"], "cycles": c["cycles"], "flop_job_s": j0, "mlp_job_s": j1,
                     "mlp_used": s1["cost_model_used"], "variants_ranked": s1["n_candidates"],
                     "same_plan": same_plan(s0, s1),
                     "flop_cmacs_per_slice": s0["cmacs_per_slice"], "mlp_cmacs_per_slice": s1["cmacs_per_slice"]})
        log(f"held-out {i}: FLOP-chosen job {j0:.4g}s, MLP-chosen job {j1:.4g}s, model used {s1['cost_model_used']}, "
            f"same plan {rows[-1]['same_plan']}")
        p0.close()
        p1.close()
    return rows


def fit_flop_model(F, K, Y):
    """log ms = a_k + b_k * log(cmacs), one line per kernel class."""
    coef = {}
    for k in np.unique(K):
        sel = K == k
        A = np.stack([np.ones(sel.sum()), F[sel]], axis=1)
        coef[int(k)] = np.linalg.lstsq(A, Y[sel], rcond=None)[0]
    return coef


def flop_predict(coef, F, K):
    return np.array([coef.get(int(k), coef[next(iter(coef))])[0] + coef.get(int(k), coef[next(iter(coef))])[1] * f
                     for f, k in zip(F, K)])


def train(model, X, Y, epochs=300, lr=2e-3, batch=512, seed=0):
    import torch
    rng = np.random.default_rng(seed)
    n = len(X)
    losses = []
    for ep in range(epochs):
        perm = rng.permutation(n)
        tot = 0.0
        for s in range(0, n, batch):
            idx = perm[s:s + batch]
            dx = torch.from_numpy(np.ascontiguousarray(X[idx])).cuda()
            dt = torch.from_numpy(np.ascontiguousarray(Y[idx])).cuda()
            tot += model.train_step(dx, dt, lr) * len(idx)
        losses.append(tot / n)
    return losses


def predict(model, X):
    import torch
    dx = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    y = torch.empty(len(X), dtype=torch.float32, device="cuda")
    model.forward(dx, y)
    return y.cpu().numpy()


def run(n_circuits=200, n_train=None, groups=2, epochs=300, restarts=6, max_log2_size=24, eval_groups=2,
        max_qubits=64):
    """n_circuits circuits of the corpus with at most max_qubits qubits (the
    corpus is drawn in seed order and filtered), 80 % for training."""
    n_train = n_train if n_train is not None else int(round(0.8 * n_circuits))
    circs = []
    pool = 0
    while len(circs) < n_circuits:
        pool += 4 * n_circuits
        circs = [c for c in corpus_circuits(pool) if c["n"] <= max_qubits][:n_circuits]
    tr, te = circs[:n_train], circs[n_train:]
    log(f"collecting timings on {len(tr)} training circuits")
    X, Y, F, K, _ = collect(tr, groups, restarts, max_log2_size)
    log(f"collecting timings on {len(te)} held-out circuits")
    Xt, Yt, Ft, Kt, _ = collect(te, groups, restarts, max_log2_size)
    model = tn.Mlp(tn.STEP_FEATURES, 128, seed=0)
    t0 = time.perf_counter()
    losses = train(model, X, Y, epochs=epochs)
    t_train = time.perf_counter() - t0
    model.set_support(X.min(axis=0), X.max(axis=0), margin=0.05)
    coef = fit_flop_model(F, K, Y)
    rmse = lambda a, b: float(np.sqrt(np.mean((a - b) ** 2)))
    res = {
        "train_samples": int(len(X)), "heldout_samples": int(len(Xt)),
        "train_seconds_gpu": t_train, "final_train_mse": losses[-1],
        "heldout_rmse_log_ms_mlp": rmse(predict(model, Xt), Yt),
        "heldout_rmse_log_ms_flop": rmse(flop_predict(coef, Ft, Kt), Yt),
        "train_rmse_log_ms_flop": rmse(flop_predict(coef, F, K), Y),
    }
    log("prediction:", res)
    # plan choice on held-out circuits: FLOP-count planning against the
    # learned model's ranking of finalized plan variants
    rows = compare_choices(te, model, restarts, max_log2_size, eval_groups)
    j0 = np.array([r["flop_job_s"] for r in rows])
    j1 = np.array([r["mlp_job_s"] for r in rows])
    res.update({"heldout_circuits": len(rows), "heldout_plans": rows,
                "geomean_speedup_mlp_vs_flop": float(np.exp(np.mean(np.log(j0 / j1)))),
                "total_job_s_flop": float(j0.sum()), "total_job_s_mlp": float(j1.sum()),
                "choices_differing": int(sum(not r["same_plan"] for r in rows)),
                "mlp_fallbacks": int(sum(r["mlp_used"] == 2 for r in rows))})
    return res, model


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--circuits", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--restarts", type=int, default=6)
    ap.add_argument("--max-log2-size", type=int, default=24)
    ap.add_argument("--max-qubits", type=int, default=64, help="use only corpus circuits with at most this many qubits")
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available()
    res, _ = run(args.circuits, epochs=args.epochs, restarts=args.restarts, max_log2_size=args.max_log2_size,
                 max_qubits=args.max_qubits)
    text = json.dumps(res)
    print(text, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text + "\n")


if __name__ == "__main__":
    main()
