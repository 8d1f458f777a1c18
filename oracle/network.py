"""The circuit's tensor network, slicing and naive contraction (oracle).

What the method computes, written out plainly:

    A[s2] = <s1; s2| U |0^n>     for every assignment s2 of the open qubits,

where U is the ordered product of the circuit's gates and s1 the fixed bits
of the closed qubits (section "Big-head simulation of quantum circuits": the
end-state qubits split into a closed group with fixed bits and an open group
that is enumerated).

Network (paragraph "Computing bitstring probabilities": single-qubit gates
are absorbed into two-qubit gates).  Canonical rules, shared by reading, not
by code, with the GPU library's planner:

* every single-qubit gate is absorbed *forward* into the next two-qubit gate
  on its qubit; single-qubit gates after a qubit's last two-qubit gate are
  absorbed *backward* into that last gate;
* the initial |0> of a qubit is absorbed into its first two-qubit gate, and
  the projector <s1_q| of a closed qubit into its last one;
* edge (q, t) is the wire of qubit q leaving its t-th two-qubit gate
  (t = 0, 1, ...); for an open qubit the edge leaving its last gate is the
  open leg;
* a qubit that meets no two-qubit gate becomes its own node: a scalar when
  closed, a vector with open leg (q, -1) when open.

Slicing (appendix A "Dynamic slicing"; section "The algorithm"): a set of
edges is fixed; slice j fixes the i-th sliced edge to bit i of j.  The full
result is the sum over all 2^k slices; each slice is an ordinary network.

Contraction: pairwise, in any order (np.tensordot as the single step, no
blocking or fusion).  The order used by default is a plain greedy that picks
the pair whose result is smallest, only so that larger cases fit in memory;
the result does not depend on it (pinned by order-invariance tests).

Pins: equals the state vector (tiny and 25-qubit circuits); sum over slices
equals the unsliced result; order invariance; closed form of product
circuits at any size.
"""

import numpy as np


class Network:
    """A list of tensors, each with a list of edge labels (one per axis).

    Labels are tuples (q, t).  `open_labels` lists the open legs in
    ascending qubit order (= output bit order, most significant first)."""

    def __init__(self, tensors, labels, open_labels):
        self.tensors = tensors
        self.labels = labels
        self.open_labels = open_labels

    def edges(self):
        """All labels with the indices of the tensors that hold them."""
        where = {}
        for i, ls in enumerate(self.labels):
            for lab in ls:
                where.setdefault(lab, []).append(i)
        return where

    def internal_edges(self):
        return sorted(e for e, ts in self.edges().items() if len(ts) == 2)

    def copy(self):
        return Network([t.copy() for t in self.tensors], [list(l) for l in self.labels],
                       list(self.open_labels))


def _apply_on_axis(t, axis, m):
    """new[..., a, ...] = sum_b m[a, b] t[..., b, ...]."""
    out = np.tensordot(m, t, axes=([1], [axis]))
    return np.moveaxis(out, 0, axis)


def build_network(circuit, open_q, fixed_q, bits):
    n = circuit.n_qubits
    open_set = set(open_q)
    if sorted(list(open_q) + list(fixed_q)) != list(range(n)):
        raise ValueError("open and fixed qubits must partition the qubits")
    bit_of = {q: int(b) for q, b in zip(fixed_q, bits)}
    pending = [np.eye(2, dtype=np.complex128) for _ in range(n)]
    count = [0] * n                  # two-qubit gates seen per qubit
    holder = [None] * n              # (tensor index, axis) of q's current out-leg
    tensors, labels = [], []
    for g in circuit.gates:
        if len(g.qubits) == 1:
            q = g.qubits[0]
            pending[q] = g.matrix @ pending[q]
            continue
        q0, q1 = g.qubits
        u = g.matrix @ np.kron(pending[q0], pending[q1])
        pending[q0] = np.eye(2, dtype=np.complex128)
        pending[q1] = np.eye(2, dtype=np.complex128)
        t = u.reshape(2, 2, 2, 2)                  # axes: out0, out1, in0, in1
        labs = [(q0, count[q0]), (q1, count[q1]),
                (q0, count[q0] - 1), (q1, count[q1] - 1)]
        # absorb |0> where this is the qubit's first two-qubit gate
        keep = [True, True, count[q0] > 0, count[q1] > 0]
        for ax in (3, 2):
            if not keep[ax]:
                t = np.take(t, 0, axis=ax)
        labs = [l for l, k in zip(labs, keep) if k]
        tensors.append(t)
        labels.append(labs)
        idx = len(tensors) - 1
        holder[q0] = (idx, 0)
        holder[q1] = (idx, 1)
        count[q0] += 1
        count[q1] += 1
    # trailing single-qubit gates (backward absorption), projectors, open legs
    for q in range(n):
        if count[q] == 0:
            v = pending[q] @ np.array([1.0, 0.0], dtype=np.complex128)
            if q in open_set:
                tensors.append(v)
                labels.append([(q, -1)])
            else:
                tensors.append(np.array(v[bit_of[q]]))
                labels.append([])
            continue
        ti, _ = holder[q]
        lab = (q, count[q] - 1)
        ax = labels[ti].index(lab)
        tensors[ti] = _apply_on_axis(tensors[ti], ax, pending[q])
        if q not in open_set:
            tensors[ti] = np.take(tensors[ti], bit_of[q], axis=ax)
            labels[ti] = [l for l in labels[ti] if l != lab]
    open_labels = []
    for q in sorted(open_q):
        open_labels.append((q, count[q] - 1) if count[q] > 0 else (q, -1))
    return Network(tensors, labels, open_labels)


def slice_network(net, sliced, values):
    """Fix edge sliced[i] to values[i] in both tensors that hold it."""
    out = net.copy()
    opens = set(net.open_labels)
    for e, v in zip(sliced, values):
        e = tuple(e)
        if e in opens:
            raise ValueError(f"open leg {e} cannot be sliced")
        found = 0
        for i in range(len(out.tensors)):
            if e in out.labels[i]:
                ax = out.labels[i].index(e)
                out.tensors[i] = np.take(out.tensors[i], int(v), axis=ax)
                out.labels[i] = [l for l in out.labels[i] if l != e]
                found += 1
        if found != 2:
            raise ValueError(f"edge {e} is not an internal edge")
    return out


def contract_pair(ta, la, tb, lb):
    shared = [l for l in la if l in lb]
    ia = [la.index(l) for l in shared]
    ib = [lb.index(l) for l in shared]
    t = np.tensordot(ta, tb, axes=(ia, ib))
    labs = [l for l in la if l not in shared] + [l for l in lb if l not in shared]
    return t, labs


def greedy_order(labels):
    """Plain greedy pair order: repeatedly pick the pair (sharing an edge if
    any pair does) whose result has the fewest elements; ties go to the
    smallest (size_a + size_b) reduction, then the lowest ids.
    Returns SSA pairs over ids (leaves 0..n-1, results n, n+1, ...)."""
    live = {i: set(l) for i, l in enumerate(labels)}
    nxt = len(labels)
    pairs = []
    while len(live) > 1:
        owners = {}
        for i, ls in live.items():
            for lab in ls:
                owners.setdefault(lab, []).append(i)
        cands = set()
        for ts in owners.values():
            if len(ts) == 2:
                cands.add((min(ts), max(ts)))
        if not cands:                     # disconnected pieces: outer products
            ids = sorted(live, key=lambda i: (len(live[i]), i))
            cands = {(min(ids[0], ids[1]), max(ids[0], ids[1]))}
        best = None
        for a, b in cands:
            out = live[a] ^ live[b]
            key = (len(out), -(2 ** len(live[a]) + 2 ** len(live[b]) - 2 ** len(out)), a, b)
            if best is None or key < best[0]:
                best = (key, a, b, out)
        _, a, b, out = best
        pairs.append((a, b))
        del live[a], live[b]
        live[nxt] = out
        nxt += 1
    return pairs


def random_order(labels, seed):
    """A seeded random pairwise order: each step joins a uniformly drawn pair
    of tensors that share an edge (any pair once none do)."""
    rng = np.random.default_rng(seed)
    live = {i: set(l) for i, l in enumerate(labels)}
    nxt = len(labels)
    pairs = []
    while len(live) > 1:
        owners = {}
        for i, ls in live.items():
            for lab in ls:
                owners.setdefault(lab, []).append(i)
        cands = sorted({(min(ts), max(ts)) for ts in owners.values() if len(ts) == 2})
        if not cands:
            ids = sorted(live)
            cands = [(ids[0], ids[1])]
        a, b = cands[int(rng.integers(len(cands)))]
        pairs.append((a, b))
        live[nxt] = live.pop(a) ^ live.pop(b)
        nxt += 1
    return pairs


def contract(net, order=None):
    """Contract the whole network; returns the output vector over the open
    legs (ascending qubit id, first = most significant bit)."""
    if order is None:
        order = greedy_order(net.labels)
    store = {i: (t, list(l)) for i, (t, l) in enumerate(zip(net.tensors, net.labels))}
    nxt = len(net.tensors)
    for a, b in order:
        ta, la = store.pop(a)
        tb, lb = store.pop(b)
        store[nxt] = contract_pair(ta, la, tb, lb)
        nxt += 1
    if len(store) != 1:
        raise ValueError("order does not contract the network to one tensor")
    (t, labs), = store.values()
    if sorted(labs) != sorted(net.open_labels):
        raise ValueError("result legs are not the open legs")
    perm = [labs.index(l) for l in net.open_labels]
    return np.ascontiguousarray(np.transpose(t, perm)).reshape(-1)


def slice_values(sliced, slice_id):
    """Bit i of the slice id is the value of the i-th sliced edge."""
    return [(int(slice_id) >> i) & 1 for i in range(len(sliced))]


def slice_amplitudes(net, sliced, slice_id, order=None):
    """A_j[s2]: the network with the sliced edges fixed by slice id j."""
    sub = slice_network(net, sliced, slice_values(sliced, slice_id))
    return contract(sub, order)


def amplitudes(circuit, open_q, fixed_q, bits, sliced=(), slice_ids=None):
    """Sum of A_j over the given slice ids (all 2^k when None), in slice-id
    order, complex128."""
    net = build_network(circuit, open_q, fixed_q, bits)
    sliced = [tuple(e) for e in sliced]
    if not sliced:
        return contract(net)
    ids = range(1 << len(sliced)) if slice_ids is None else slice_ids
    acc = None
    sub0 = slice_network(net, sliced, [0] * len(sliced))
    order = greedy_order(sub0.labels)
    for j in ids:
        a = slice_amplitudes(net, sliced, j, order)
        acc = a if acc is None else acc + a
    return acc


def log2_sizes(labels, order):
    """(max log2 size of any intermediate, total complex MACs) of an order
    -- the pairwise cost 2^(nA + nB + nAB) of appendix A, Fig. 3."""
    live = {i: set(l) for i, l in enumerate(labels)}
    nxt = len(labels)
    mx = max((len(l) for l in labels), default=0)
    macs = 0
    for a, b in order:
        la, lb = live.pop(a), live.pop(b)
        out = la ^ lb
        macs += 2 ** len(la | lb)
        mx = max(mx, len(out))
        live[nxt] = out
        nxt += 1
    return mx, macs
