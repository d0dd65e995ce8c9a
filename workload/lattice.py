"""Qubit connectivity graphs for the kicked Ising benchmark.

The 127-qubit heavy-hexagon graph follows the IBM Eagle layout used in the
paper (Results, Eq. (u); Fig. 1(a) caption: 144 two-qubit couplings split into
three disjoint sets).  The figure itself is not available, so the layout is
built from its construction rule: seven rows of 14, 15, 15, 15, 15, 15, 14
qubits joined by six layers of four bridge qubits at alternating column
offsets.  Qubits are numbered row by row with each bridge layer numbered
between the two rows it joins, which puts the observable qubit 62 in the
middle row with neighbours 61, 63 and 72.
"""

from __future__ import annotations

from collections import deque
from dataclasses import dataclass, field


@dataclass
class Lattice:
    n: int
    edges: list[tuple[int, int]]
    name: str = ""
    center: int = 0
    adj: list[list[int]] = field(default_factory=list)

    def __post_init__(self):
        adj: list[list[int]] = [[] for _ in range(self.n)]
        seen = set()
        for a, b in self.edges:
            assert a != b and 0 <= a < self.n and 0 <= b < self.n
            key = (min(a, b), max(a, b))
            assert key not in seen, f"duplicate edge {key}"
            seen.add(key)
            adj[a].append(b)
            adj[b].append(a)
        self.adj = [sorted(v) for v in adj]

    def degree(self, q: int) -> int:
        return len(self.adj[q])

    def edge_colouring(self) -> list[list[tuple[int, int]]]:
        """Greedy proper edge colouring (disjoint matchings)."""
        colours: list[list[tuple[int, int]]] = []
        used: list[set[int]] = []
        for a, b in self.edges:
            for c, s in enumerate(used):
                if a not in s and b not in s:
                    colours[c].append((a, b))
                    s.update((a, b))
                    break
            else:
                colours.append([(a, b)])
                used.append({a, b})
        return colours


def _rows_and_bridges(row_cols, bridge_cols):
    """Number rows and bridge layers alternately; return (n, edges, index)."""
    index = {}
    edges = []
    q = 0
    for r, cols in enumerate(row_cols):
        for c in cols:
            index[("row", r, c)] = q
            q += 1
        if r < len(bridge_cols):
            for c in bridge_cols[r]:
                index[("bridge", r, c)] = q
                q += 1
    for r, cols in enumerate(row_cols):
        for c0, c1 in zip(cols[:-1], cols[1:]):
            edges.append((index[("row", r, c0)], index[("row", r, c1)]))
    for r, cols in enumerate(bridge_cols):
        for c in cols:
            b = index[("bridge", r, c)]
            edges.append((index[("row", r, c)], b))
            edges.append((b, index[("row", r + 1, c)]))
    return q, edges, index


def eagle_127() -> Lattice:
    """127-qubit heavy-hex lattice (144 edges), observable qubit 62."""
    row_cols = [list(range(0, 14))] + [list(range(0, 15))] * 5 + [list(range(1, 15))]
    bridge_cols = [[0, 4, 8, 12] if r % 2 == 0 else [2, 6, 10, 14] for r in range(6)]
    n, edges, _ = _rows_and_bridges(row_cols, bridge_cols)
    assert n == 127 and len(edges) == 144
    return Lattice(n=n, edges=edges, name="eagle127", center=62)


def heavy_hex_21() -> Lattice:
    """21-qubit patch: 3 rows of 5 qubits joined by 2 layers of 3 bridges at
    columns 0, 2, 4 (24 edges).  The central qubit is 10 (middle row, col 2)."""
    row_cols = [list(range(5))] * 3
    bridge_cols = [[0, 2, 4], [0, 2, 4]]
    n, edges, _ = _rows_and_bridges(row_cols, bridge_cols)
    assert n == 21 and len(edges) == 24
    return Lattice(n=n, edges=edges, name="heavyhex21", center=10)


def star_graph(d: int) -> Lattice:
    """Centre 0 joined to d leaves; used for closed-form checks."""
    return Lattice(n=d + 1, edges=[(0, k) for k in range(1, d + 1)], name=f"star{d}", center=0)


def chain(n: int) -> Lattice:
    return Lattice(n=n, edges=[(k, k + 1) for k in range(n - 1)], name=f"chain{n}", center=n // 2)


def ball(lat: Lattice, center: int, radius: int) -> list[int]:
    """Qubits within graph distance `radius` of `center` (sorted)."""
    dist = {center: 0}
    dq = deque([center])
    while dq:
        u = dq.popleft()
        if dist[u] == radius:
            continue
        for v in lat.adj[u]:
            if v not in dist:
                dist[v] = dist[u] + 1
                dq.append(v)
    return sorted(dist)


def distances(lat: Lattice, center: int) -> list[int]:
    """Graph distance of every qubit from `center` (-1 if unreachable)."""
    dist = [-1] * lat.n
    dist[center] = 0
    dq = deque([center])
    while dq:
        u = dq.popleft()
        for v in lat.adj[u]:
            if dist[v] < 0:
                dist[v] = dist[u] + 1
                dq.append(v)
    return dist


def induced(lat: Lattice, qubits: list[int]) -> tuple[Lattice, dict[int, int]]:
    """Sub-lattice on `qubits` (relabelled 0..k-1, keeping their order)."""
    m = {q: i for i, q in enumerate(qubits)}
    edges = [(m[a], m[b]) for a, b in lat.edges if a in m and b in m]
    sub = Lattice(n=len(qubits), edges=edges, name=f"{lat.name}_sub{len(qubits)}",
                  center=m.get(lat.center, 0))
    return sub, m
