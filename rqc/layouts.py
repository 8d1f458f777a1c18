"""Qubit layouts and the four alternating coupler patterns.

The paper runs the Sycamore circuits, whose coupler patterns A, B, C, D are
alternated in the sequence ABCDCDAB; its layout is shown only as a figure
(appendix "Details of simulations") and its circuit files are not part of
this project.  The synthetic stand-ins used here:

* Rectangular R x C grid, qubit id = r * C + c.
  A: horizontal (r,c)-(r,c+1) with r+c even;  B: horizontal, r+c odd;
  C: vertical (r,c)-(r+1,c) with r+c even;    D: vertical, r+c odd.
  Each pattern is a matching (no qubit appears twice).
* 54-site diagonal-neighbour grid: 9 rows of 6 sites, site (r,c) at
  x = 2c + (r mod 2), y = r; couplers join (x,y) to (x+1,y+1) and (x-1,y+1).
  A/B: direction +1 from even/odd rows, C/D: direction -1 from even/odd rows.
  One seeded boundary site is disabled, leaving 53 active qubits.  This is a
  synthetic layout of the same size and degree, not Google's device.
* Near-square rectangular grids with surplus sites removed from the last row
  (cost-model corpus of 36..53 qubits).
"""

from dataclasses import dataclass, field
import math

import numpy as np

PATTERN_SEQUENCE = "ABCDCDAB"


@dataclass
class Layout:
    name: str
    n_qubits: int
    coords: list                      # per qubit (row, col) or (x, y)
    patterns: dict = field(default_factory=dict)   # "A".."D" -> list of (q0, q1), q0 < q1

    def couplers(self):
        out = []
        for k in "ABCD":
            out.extend(self.patterns[k])
        return sorted(set(out))

    def neighbours(self):
        nb = [[] for _ in range(self.n_qubits)]
        for a, b in self.couplers():
            nb[a].append(b)
            nb[b].append(a)
        return [sorted(x) for x in nb]


def _rect_from_sites(name, sites, ncols):
    """sites: sorted list of active (r, c)."""
    index = {s: i for i, s in enumerate(sites)}
    pats = {k: [] for k in "ABCD"}
    for (r, c), q in index.items():
        right = index.get((r, c + 1))
        if right is not None:
            pats["A" if (r + c) % 2 == 0 else "B"].append((q, right))
        down = index.get((r + 1, c))
        if down is not None:
            pats["C" if (r + c) % 2 == 0 else "D"].append((q, down))
    for k in pats:
        pats[k] = sorted(tuple(sorted(p)) for p in pats[k])
    return Layout(name, len(sites), list(sites), pats)


def rect_layout(rows, cols):
    sites = [(r, c) for r in range(rows) for c in range(cols)]
    return _rect_from_sites(f"rect{rows}x{cols}", sites, cols)


def near_square_layout(n):
    """Smallest near-square grid holding n qubits; surplus sites are dropped
    from the end of the last row."""
    cols = int(math.ceil(math.sqrt(n)))
    rows = int(math.ceil(n / cols))
    sites = [(r, c) for r in range(rows) for c in range(cols)][:n]
    return _rect_from_sites(f"nsq{n}", sites, cols)


def diag54_layout(seed=0):
    rows, per_row = 9, 6
    all_sites = []
    for r in range(rows):
        for c in range(per_row):
            all_sites.append((2 * c + (r % 2), r))
    boundary = [s for s in all_sites
                if s[1] in (0, rows - 1) or s[0] in (0, 2 * (per_row - 1) + 1, 1, 2 * (per_row - 1))]
    boundary = sorted(set(boundary), key=lambda s: (s[1], s[0]))
    rng = np.random.default_rng(seed)
    disabled = boundary[int(rng.integers(len(boundary)))]
    sites = [s for s in sorted(all_sites, key=lambda s: (s[1], s[0])) if s != disabled]
    index = {s: i for i, s in enumerate(sites)}
    pats = {k: [] for k in "ABCD"}
    for (x, y), q in index.items():
        for dx, even_key, odd_key in ((+1, "A", "B"), (-1, "C", "D")):
            other = index.get((x + dx, y + 1))
            if other is None:
                continue
            pats[even_key if y % 2 == 0 else odd_key].append(tuple(sorted((q, other))))
    for k in pats:
        pats[k] = sorted(pats[k])
    return Layout("diag54", len(sites), sites, pats)


def pattern_for_cycle(i):
    return PATTERN_SEQUENCE[i % len(PATTERN_SEQUENCE)]
