"""Seeded random circuits, open/fixed qubit choices and slice-id samples.

Circuit rule (section "Simulation of the Sycamore circuits"; the reading of
the unspecified details is stated where it is made):

* initial state |0...0>;
* m cycles; cycle i is a single-qubit layer followed by fSim gates on the
  couplers of pattern "ABCDCDAB"[i mod 8];
* single-qubit gates: uniform over {sqrt X, sqrt Y, sqrt W} in the first
  layer, afterwards uniform over the two gates that differ from the qubit's
  previous one;
* fSim angles drawn once per coupler: theta ~ U[pi/2 - 0.05, pi/2 + 0.05],
  phi ~ U[pi/6 - 0.05, pi/6 + 0.05];
* a closing single-qubit layer after the last cycle (reading: the paper is
  silent; Google's circuits end with one).

A circuit is a time-ordered list of gates, each carrying its explicit
complex128 matrix, so every consumer reads the same numbers.
"""

from dataclasses import dataclass, field
from collections import deque

import numpy as np

from . import gates as G
from . import layouts as L


@dataclass
class Gate:
    qubits: tuple           # (q,) or (q0, q1); matrix basis |q0 q1>, q0 = MSB
    matrix: np.ndarray      # complex128, (2,2) or (4,4)
    label: str = ""


@dataclass
class Circuit:
    n_qubits: int
    gates: list
    meta: dict = field(default_factory=dict)

    def two_qubit_gates(self):
        return [g for g in self.gates if len(g.qubits) == 2]

    def to_json(self):
        return {
            "n_qubits": self.n_qubits,
            "gates": [{"q": list(g.qubits),
                       "re": np.real(g.matrix).ravel().tolist(),
                       "im": np.imag(g.matrix).ravel().tolist(),
                       "label": g.label} for g in self.gates],
            "meta": self.meta,
        }

    @staticmethod
    def from_json(d):
        gl = []
        for g in d["gates"]:
            k = 2 ** len(g["q"])
            m = (np.array(g["re"]) + 1j * np.array(g["im"])).reshape(k, k)
            gl.append(Gate(tuple(g["q"]), m.astype(np.complex128), g.get("label", "")))
        return Circuit(d["n_qubits"], gl, d.get("meta", {}))


def _single_qubit_layers(rng, n, layers):
    """Gate names per (layer, qubit) following the no-repeat rule."""
    names = G.SINGLE_QUBIT_GATES
    out = []
    prev = [None] * n
    for _ in range(layers):
        row = []
        for q in range(n):
            if prev[q] is None:
                choice = names[int(rng.integers(3))]
            else:
                others = [x for x in names if x != prev[q]]
                choice = others[int(rng.integers(2))]
            row.append(choice)
            prev[q] = choice
        out.append(row)
    return out


def random_circuit(layout, cycles, seed=0, theta_center=np.pi / 2, phi_center=np.pi / 6,
                   half_width=0.05, closing_layer=True, two_qubit="fsim"):
    """Random grid circuit on `layout` with `cycles` cycles.

    two_qubit = "fsim" (the circuit family) or "product": every fSim is
    replaced by a seeded random G_a (x) G_b, a dense but non-entangling gate,
    so amplitudes factor over qubits (closed-form test circuits of any size).
    """
    rng = np.random.default_rng(seed)
    n = layout.n_qubits
    couplers = layout.couplers()
    angles = {}
    for cp in couplers:
        th = rng.uniform(theta_center - half_width, theta_center + half_width)
        ph = rng.uniform(phi_center - half_width, phi_center + half_width)
        angles[cp] = (th, ph)
    sq = _single_qubit_layers(rng, n, cycles + (1 if closing_layer else 0))
    prod_rng = np.random.default_rng(seed + 7919)
    gl = []
    for i in range(cycles):
        for q in range(n):
            gl.append(Gate((q,), G.single_qubit(sq[i][q]), sq[i][q]))
        pat = L.pattern_for_cycle(i)
        for (a, b) in layout.patterns[pat]:
            if two_qubit == "fsim":
                th, ph = angles[(a, b)]
                gl.append(Gate((a, b), G.fsim(th, ph), f"fsim{pat}"))
            elif two_qubit == "product":
                m = np.kron(G.random_su2(prod_rng), G.random_su2(prod_rng))
                gl.append(Gate((a, b), m, f"prod{pat}"))
            elif two_qubit == "identity":
                gl.append(Gate((a, b), G.fsim(0.0, 0.0), f"id{pat}"))
            else:
                raise ValueError(two_qubit)
    if closing_layer:
        for q in range(n):
            gl.append(Gate((q,), G.single_qubit(sq[cycles][q]), sq[cycles][q]))
    meta = {"layout": layout.name, "cycles": cycles, "seed": seed, "two_qubit": two_qubit,
            "sequence": L.PATTERN_SEQUENCE, "closing_layer": closing_layer}
    return Circuit(n, gl, meta)


def product_circuit(layout, cycles, seed=0, closing_layer=True):
    return random_circuit(layout, cycles, seed=seed, closing_layer=closing_layer,
                          two_qubit="product")


def choose_open_qubits(layout, n_open):
    """Connected open region grown breadth-first from the highest-id qubit
    (neighbours visited in descending id).  The paper reads the open qubits
    off its contraction order; its m=20 choice is a contiguous block."""
    if n_open == 0:
        return []
    nb = layout.neighbours()
    start = layout.n_qubits - 1
    seen = [start]
    mark = {start}
    dq = deque([start])
    while dq and len(seen) < n_open:
        u = dq.popleft()
        for v in sorted(nb[u], reverse=True):
            if v not in mark:
                mark.add(v)
                seen.append(v)
                dq.append(v)
                if len(seen) == n_open:
                    break
    if len(seen) < n_open:      # disconnected layout: fill by descending id
        for q in range(layout.n_qubits - 1, -1, -1):
            if q not in mark and len(seen) < n_open:
                seen.append(q)
                mark.add(q)
    return sorted(seen)


def fixed_bits(n_fixed, seed=1, zeros=False):
    if zeros:
        return np.zeros(n_fixed, dtype=np.uint8)
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2, size=n_fixed).astype(np.uint8)


def sample_slice_ids(n_sliced, count, seed=2):
    """`count` distinct slice ids in [0, 2**n_sliced), sorted, seeded."""
    total = 1 << n_sliced
    if count >= total:
        return np.arange(total, dtype=np.uint64)
    rng = np.random.default_rng(seed)
    if total <= 1 << 24:
        ids = rng.choice(total, size=count, replace=False)
    else:
        got = set()
        while len(got) < count:
            got.update(int(x) for x in rng.integers(0, total, size=count - len(got), dtype=np.uint64))
        ids = np.array(sorted(got)[:count])
    return np.sort(np.asarray(ids, dtype=np.uint64))


# Workloads --------------------------------------------------------------

WORKLOADS = {
    # name: (layout factory, cycles, n_open, sliced edges k (None = planner target), max_log2_size)
    "c1_tiny_3x4_m8": dict(layout=("rect", 3, 4), cycles=8, n_open=6, n_sliced=2, max_log2=None),
    "c2_5x5_m16": dict(layout=("rect", 5, 5), cycles=16, n_open=10, n_sliced=8, max_log2=None),
    "c3_5x8_m16": dict(layout=("rect", 5, 8), cycles=16, n_open=16, n_sliced=16, max_log2=None),
    "c4_diag53_m20": dict(layout=("diag54",), cycles=20, n_open=20, n_sliced=None, max_log2=30,
                          n_sample_slices=256),
}


def make_layout(spec, seed=0):
    if spec[0] == "rect":
        return rect_layout(spec[1], spec[2])
    if spec[0] == "diag54":
        return diag54_layout(seed)
    if spec[0] == "nsq":
        return near_square_layout(spec[1])
    raise ValueError(spec)


def rect_layout(r, c):
    return L.rect_layout(r, c)


def diag54_layout(seed=0):
    return L.diag54_layout(seed)


def near_square_layout(n):
    return L.near_square_layout(n)


def workload(name, circuit_seed=0, bits_seed=1, two_qubit="fsim", zeros=False):
    """Circuit plus open/fixed qubits and fixed bits for a named workload."""
    w = dict(WORKLOADS[name])
    lay = make_layout(w["layout"], seed=circuit_seed)
    circ = random_circuit(lay, w["cycles"], seed=circuit_seed, two_qubit=two_qubit)
    open_q = choose_open_qubits(lay, w["n_open"])
    fixed_q = [q for q in range(lay.n_qubits) if q not in set(open_q)]
    bits = fixed_bits(len(fixed_q), seed=bits_seed, zeros=zeros)
    w.update(name=name, layout_obj=lay, circuit=circ, open_q=open_q, fixed_q=fixed_q, bits=bits)
    return w


def cost_model_corpus(count=200, seed0=0, n_open=16):
    """Circuits of the learned-cost-model study: n ~ U{36..53} qubits on
    near-square grids, m ~ U{12..20} cycles, seeds seed0..seed0+count-1."""
    out = []
    for s in range(seed0, seed0 + count):
        rng = np.random.default_rng(10_000 + s)
        n = int(rng.integers(36, 54))
        m = int(rng.integers(12, 21))
        lay = near_square_layout(n)
        circ = random_circuit(lay, m, seed=s)
        open_q = choose_open_qubits(lay, n_open)
        fixed_q = [q for q in range(n) if q not in set(open_q)]
        out.append(dict(seed=s, n=n, cycles=m, layout_obj=lay, circuit=circ,
                        open_q=open_q, fixed_q=fixed_q,
                        bits=fixed_bits(len(fixed_q), seed=1 + s)))
    return out
