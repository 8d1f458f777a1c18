"""CPU-only checks of the C-ABI library: it loads, exports every symbol the
header declares, plans on the host, rejects bad input, and its planner's
network and cost accounting agree with the oracle's independent build."""

import math
import os
import re

import numpy as np
import pytest

import rqc
from oracle import network as nw
from paper_2103_03074_amd import tn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names.update(re.findall(r"\b(tn_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    import ctypes
    lib = ctypes.CDLL(tn.LIB_PATH)
    names = _declared_symbols()
    assert "tn_plan" in names and "tn_contract_slices" in names and "tn_xeb" in names
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(tn._SIGS) == names, "binding and header disagree"


def _plan(name, **kw):
    w = rqc.workload(name)
    return w, tn.Plan(w["circuit"], w["open_q"], w["fixed_q"], w["bits"], **kw)


def test_planner_network_matches_oracle_naming():
    for name in ("c1_tiny_3x4_m8", "c2_5x5_m16"):
        w, p = _plan(name, n_slice_edges=2, restarts=1)
        ex = p.export()
        net = nw.build_network(w["circuit"], w["open_q"], w["fixed_q"], w["bits"])
        assert len(ex["leaves"]) == len(net.labels)
        for mine, ref in zip(ex["leaves"], net.labels):
            assert sorted(tuple(e) for e in mine) == sorted(ref)
        assert [tuple(e) for e in ex["open"]] == net.open_labels


def test_planner_cost_accounting_matches_oracle():
    w, p = _plan("c2_5x5_m16", n_slice_edges=8, restarts=2)
    ex = p.export()
    s = p.stats()
    net = nw.build_network(w["circuit"], w["open_q"], w["fixed_q"], w["bits"])
    sliced = [tuple(e) for e in ex["sliced"]]
    sub = nw.slice_network(net, sliced, [0] * len(sliced))
    order = list(zip(ex["lhs"], ex["rhs"]))
    mx, macs = nw.log2_sizes(sub.labels, order)
    assert macs == pytest.approx(s["cmacs_per_slice_unmerged"] + s["cmacs_invariant"], rel=1e-12)
    assert s["max_log2_size"] == mx
    assert s["n_sliced"] == len(sliced) == 8
    assert s["n_slices"] == 256


def test_planner_meets_memory_target():
    for target in (12, 16, 20):
        _, p = _plan("c2_5x5_m16", max_log2_size=target, restarts=2)
        s = p.stats()
        assert s["max_log2_size"] <= target


def test_planner_respects_given_slicing_and_tree():
    w, p = _plan("c1_tiny_3x4_m8", n_slice_edges=3, restarts=1)
    ex = p.export()
    tree = list(zip(ex["lhs"], ex["rhs"]))
    sliced = [tuple(e) for e in ex["sliced"]]
    p2 = tn.Plan(w["circuit"], w["open_q"], w["fixed_q"], w["bits"], tree=tree, sliced=sliced)
    assert p2.sliced_edges() == sliced
    ex2 = p2.export()
    assert ex2["lhs"] == ex["lhs"] and ex2["rhs"] == ex["rhs"]


@pytest.mark.parametrize("case", ["overlap", "missing", "bad_bit", "open_slice", "not_edge", "bad_tree"])
def test_planner_rejects_bad_input(case):
    w = rqc.workload("c1_tiny_3x4_m8")
    c, o, f, b = w["circuit"], list(w["open_q"]), list(w["fixed_q"]), list(w["bits"])
    kw = {}
    if case == "overlap":
        f[0] = o[0]
    elif case == "missing":
        f, b = f[1:], b[1:]
    elif case == "bad_bit":
        b[0] = 2
    elif case == "open_slice":
        net = nw.build_network(c, w["open_q"], w["fixed_q"], w["bits"])
        kw["sliced"] = [net.open_labels[0]]
    elif case == "not_edge":
        kw["sliced"] = [(0, 999)]
    elif case == "bad_tree":
        kw["tree"] = [(0, 0)] * 33
    with pytest.raises(tn.TnError) as ei:
        tn.Plan(c, o, f, b, **kw)
    assert ei.value.status == -1


@pytest.mark.parametrize("name,n_open", [("c1_tiny_3x4_m8", None), ("c2_5x5_m16", None), ("c1_tiny_3x4_m8", 0)])
def test_bighead_split_plans(name, n_open):
    """Head/tail split: the accumulator is the head's vector over the n_c cut
    legs; the tail is contracted by tn_amplitudes."""
    w = rqc.workload(name)
    o, f, b = list(w["open_q"]), list(w["fixed_q"]), list(w["bits"])
    if n_open == 0:
        f, b = sorted(o + f), [1] * (len(o) + len(f))
        o = []
    p = tn.Plan(w["circuit"], o, f, b, bighead=1)
    s = p.stats()
    assert s["n_open"] == len(o)
    assert s["acc_log2"] == s["n_c"] and 0 <= s["n_c"] <= 28
    assert (s["n_c"] > 0) == (len(o) > 0)
    assert s["tail_workspace_bytes"] >= 256 and (s["cmacs_tail"] > 0) == (len(o) > 0)
    # sliced edges are edges of the full network, never open legs
    net = nw.build_network(w["circuit"], o, f, b)
    for e in p.sliced_edges():
        assert tuple(e) in net.edges() and tuple(e) not in set(map(tuple, net.open_labels))


def test_bighead_refuses_user_tree_or_slicing():
    w = rqc.workload("c1_tiny_3x4_m8")
    net = nw.build_network(w["circuit"], w["open_q"], w["fixed_q"], w["bits"])
    closed = [e for e in net.edges() if e not in set(map(tuple, net.open_labels))]
    with pytest.raises(tn.TnError) as ei:
        tn.Plan(w["circuit"], w["open_q"], w["fixed_q"], w["bits"], bighead=1, sliced=[closed[0]])
    assert ei.value.status == -1 and "bighead" in str(ei.value)


def test_planner_degenerate_networks():
    # one qubit pair, one gate; and a qubit with no two-qubit gate
    c = rqc.random_circuit(rqc.rect_layout(1, 3), 1, seed=1)
    for open_q in ([0, 1, 2], [], [2]):
        fixed_q = [q for q in range(3) if q not in open_q]
        p = tn.Plan(c, open_q, fixed_q, [1] * len(fixed_q), n_slice_edges=0)
        s = p.stats()
        assert s["n_open"] == len(open_q) and s["n_slices"] == 1


def test_sample_workspace_sizes():
    """cdf (2^n doubles) plus one double per block of 1024 at every scan level."""
    assert tn.sample_workspace_bytes(0) == 8 * (1 + 1)
    assert tn.sample_workspace_bytes(10) == 8 * (1024 + 1)
    assert tn.sample_workspace_bytes(21) == 8 * (2 ** 21 + 2048 + 2 + 1)
    assert tn.sample_workspace_bytes(-1) == 0 and tn.sample_workspace_bytes(35) == 0


def test_branch_merging_decided_per_launch_group():
    """Branch merging is kept only if the executed steps of one whole job get
    faster.  On the 25-qubit workload all 2^8 slices share one launch group;
    the per-slice estimate alone once merged its tree to 100x the
    multiply-adds (37 ms per job against 4.9 ms unmerged on MI355X)."""
    w = rqc.workload("c2_5x5_m16")
    kw = dict(restarts=16, n_slice_edges=8, seed=0)
    plain = tn.Plan(w["circuit"], w["open_q"], w["fixed_q"], w["bits"], branch_merge=0, **kw).stats()
    merged = tn.Plan(w["circuit"], w["open_q"], w["fixed_q"], w["bits"], branch_merge=1, **kw).stats()
    assert merged["batch_log2"] == 8
    # merging may trade multiply-adds for bytes, within bounds far from the
    # 100x blow-up of the per-slice estimate
    assert merged["cmacs_per_batch"] <= 4 * plain["cmacs_per_batch"]
    if merged["cmacs_per_batch"] != plain["cmacs_per_batch"]:
        assert merged["bytes_per_batch"] < plain["bytes_per_batch"]
    # the 40-qubit bench plan does merge: more multiply-adds, fewer bytes
    w3 = rqc.workload("c3_5x8_m16")
    kw3 = dict(restarts=16, n_slice_edges=16, seed=0)
    p0 = tn.Plan(w3["circuit"], w3["open_q"], w3["fixed_q"], w3["bits"], branch_merge=0, **kw3).stats()
    p1 = tn.Plan(w3["circuit"], w3["open_q"], w3["fixed_q"], w3["bits"], branch_merge=1, **kw3).stats()
    g0 = p0["n_slices"] >> p0["batch_log2"]
    g1 = p1["n_slices"] >> p1["batch_log2"]
    assert p1["bytes_per_batch"] * g1 < p0["bytes_per_batch"] * g0


def test_step_candidates_and_forcing():
    w = rqc.workload("c3_5x8_m16")
    p = tn.Plan(w["circuit"], w["open_q"], w["fixed_q"], w["bits"], prec="split_fp16", n_slice_edges=16, restarts=4,
                seed=0, branch_merge=1)
    ex = p.export()
    i = next(k for k, st in enumerate(ex["steps"]) if st["kernel"] == 5)
    cands = p.step_candidates(i)
    assert (ex["steps"][i]["kernel"], ex["steps"][i]["tile"]) in cands
    # mixed panels: pre-split, FP32, FP32 non-temporal, register-split (and non-temporal) per base tile
    tiles = {t for k, t in cands if k == 5}
    assert {0, 4, 20, 8, 24} <= tiles
    k, t = cands[-1]
    p.set_step_kernel(i, k, t)
    assert (p.export()["steps"][i]["kernel"], p.export()["steps"][i]["tile"]) == (k, t)
    with pytest.raises(tn.TnError) as ei:
        p.set_step_kernel(i, 5, 999)
    assert ei.value.status == -1
    with pytest.raises(tn.TnError):
        p.set_step_kernel(len(ex["steps"]), 0, 0)


def test_sample_argument_errors_before_any_launch():
    """tn_sample validates its arguments on the host: no device is touched."""
    import ctypes
    lib = tn.library()
    fake = ctypes.c_void_p(16)   # never dereferenced: every case fails validation first
    assert lib.tn_sample(None, 4, fake, 1, fake, fake, 1 << 20, None) == -1            # NULL amplitudes
    assert lib.tn_sample(fake, 4, None, 1, fake, fake, 1 << 20, None) == -1            # NULL uniforms
    assert lib.tn_sample(fake, 35, fake, 1, fake, fake, 1 << 40, None) == -1           # n_open too large
    assert lib.tn_sample(fake, 10, fake, 1, fake, fake, tn.sample_workspace_bytes(10) - 8, None) == -1
    assert "workspace" in lib.tn_last_error().decode()


def test_open_qubits_read_off_the_order():
    # two halves that never interact: a half is a subtree with no legs to the rest
    lay = rqc.rect_layout(2, 3)
    c = rqc.random_circuit(lay, 6, seed=3)
    half = {0, 1, 2}
    c.gates = [g for g in c.gates if len(g.qubits) == 1 or (set(g.qubits) <= half or not set(g.qubits) & half)]
    oq, cut = tn.choose_open_qubits(c, 3, restarts=4, seed=0)
    assert cut == 0 and set(oq) in ({0, 1, 2}, {3, 4, 5})
    # the 40-qubit circuit: distinct, sorted, in range; the big-head split of
    # the chosen set plans and its cut is no larger than the node's leg count
    w = rqc.workload("c3_5x8_m16")
    oq, cut = tn.choose_open_qubits(w["circuit"], 16, restarts=8, seed=0)
    assert oq == sorted(set(oq)) and len(oq) == 16 and 0 <= oq[0] and oq[-1] < 40 and cut > 0
    f = [q for q in range(40) if q not in set(oq)]
    s = tn.Plan(w["circuit"], oq, f, [0] * len(f), bighead=1, restarts=8, seed=0).stats()
    assert s["n_open"] == 16 and 0 < s["n_c"] <= cut
    for bad in (0, 41):
        with pytest.raises(tn.TnError) as ei:
            tn.choose_open_qubits(w["circuit"], bad)
        assert ei.value.status == -1


def test_lanes_setting_and_workspace_size():
    """tn_plan_set_lanes: range checks and the workspace the lanes need
    (lane i at i * stride, stride = workspace_bytes rounded up to 256)."""
    _, p = _plan("c1_tiny_3x4_m8", n_slice_edges=2)
    s = p.stats()
    assert s["lanes"] == 1 and s["lanes_workspace_bytes"] == s["workspace_bytes"]
    stride = (s["workspace_bytes"] + 255) // 256 * 256
    for n in (2, 3, 8):
        p.set_lanes(n)
        s = p.stats()
        assert s["lanes"] == n
        assert s["lanes_workspace_bytes"] == (n - 1) * stride + s["workspace_bytes"]
    for bad in (0, -1, 9):
        with pytest.raises(tn.TnError) as ei:
            p.set_lanes(bad)
        assert ei.value.status == -1
    assert p.stats()["lanes"] == 8
    p.set_lanes(1)
    assert p.stats()["lanes_workspace_bytes"] == p.stats()["workspace_bytes"]


def test_profile_overlap_summary(tmp_path):
    """profile_summary's concurrency figures on a hand-made kernel trace: two
    bracketing copies, then kernels a [0, 10), b [5, 20), c [30, 40) (us)
    between them: window 40, summed 35, busy 30, two at once 5."""
    import csv
    from paper_2103_03074_amd import profile_summary as ps
    rows = [(1, ps.COPY_KERNEL, -100, -50), (2, "void tn::a(tn::GemmArgs)", 0, 10),
            (3, "void tn::b(tn::GemmArgs)", 5, 20), (4, "void tn::c(tn::GemmArgs)", 30, 40),
            (5, ps.COPY_KERNEL, 100, 150)]
    d = tmp_path / "run"
    d.mkdir()
    with open(d / "1_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for i, k, t0, t1 in rows:
            w.writerow([i, k, t0 * 1000, t1 * 1000])
    o, table = ps.overlap_summary(str(d))
    assert o["dispatches"] == 3
    assert (o["window_us"], o["sum_us"], o["busy1_us"], o["busy2_us"]) == (40.0, 35.0, 30.0, 5.0)
    assert [r["kernel"] for r in table] == ["b", "a", "c"]
