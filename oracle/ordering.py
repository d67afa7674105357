"""Near-field block ordering (oracle).

Algorithm 1 of the paper: the leaves are the nodes of a graph, near-field
interactions are its edges, a bandwidth-reduction ordering renumbers the
nodes (Sec. 3.3, Figs. 4-5, Table 3: Cuthill-McKee and its reverse). The
paper names no start node or tie rule, so this reading is used:

* degree = number of distinct near neighbours (self pairs excluded);
* components are taken in turn, each from the unvisited node with the
  smallest (degree, id);
* start node: the George-Liu pseudo-peripheral node finder from that node
  (level structure from r; x = the node of smallest (degree, id) in the last
  level; if x's level structure is deeper, r = x and repeat, else x is the
  start; a component whose structure has one level, or one node per level,
  keeps r);
* breadth-first search from the start, marking nodes when they are
  enqueued and enqueueing each popped node's unvisited neighbours in
  ascending (degree, id);
* RCM is the reverse of the whole Cuthill-McKee list.

Sloan's and King's orderings (Table 3, Figs. 6-7; the paper ran Sloan's
for every result of Sec. 5) follow their published algorithms with the same
start-node and tie readings; see ``sloan`` and ``king``.

Output: ``order[new] = old``. Pinned in the tests on hand-worked graphs
(path, star, ring, grid, two components), by the permutation property, and
by the Liu-Sherman result that the reversed ordering's profile is never
larger than that of the unreversed one.
"""
from __future__ import annotations

import numpy as np


def leaf_graph(nb: int, near: np.ndarray):
    """Adjacency lists (sorted) of the leaf graph; self pairs dropped."""
    adj = [set() for _ in range(nb)]
    for i, j in near:
        i, j = int(i), int(j)
        if i != j:
            adj[i].add(j)
            adj[j].add(i)
    return [sorted(a) for a in adj]


def _levels(adj, root, deg):
    """Rooted level structure (list of levels) restricted to root's component."""
    seen = {root}
    levels = [[root]]
    while True:
        nxt = []
        for v in levels[-1]:
            for w in adj[v]:
                if w not in seen:
                    seen.add(w)
                    nxt.append(w)
        if not nxt:
            return levels
        levels.append(nxt)


def pseudo_peripheral(adj, start, deg):
    r = start
    lv = _levels(adj, r, deg)
    size = sum(len(level) for level in lv)
    if len(lv) == 1 or len(lv) == size:
        return r
    while True:
        last = lv[-1]
        x = min(last, key=lambda v: (deg[v], v))
        lx = _levels(adj, x, deg)
        if len(lx) <= len(lv):
            return x
        r, lv = x, lx
        if len(lv) >= size:
            return r


def cuthill_mckee(nb: int, near: np.ndarray) -> np.ndarray:
    adj = leaf_graph(nb, near)
    deg = [len(a) for a in adj]
    visited = np.zeros(nb, dtype=bool)
    order = []
    while len(order) < nb:
        cand = [v for v in range(nb) if not visited[v]]
        s0 = min(cand, key=lambda v: (deg[v], v))
        s = pseudo_peripheral(adj, s0, deg)
        visited[s] = True
        queue = [s]
        head = 0
        while head < len(queue):
            v = queue[head]
            head += 1
            order.append(v)
            nbrs = [w for w in adj[v] if not visited[w]]
            nbrs.sort(key=lambda w: (deg[w], w))
            for w in nbrs:
                visited[w] = True
                queue.append(w)
    return np.array(order, dtype=np.int64)


def reverse_cuthill_mckee(nb: int, near: np.ndarray) -> np.ndarray:
    return cuthill_mckee(nb, near)[::-1].copy()


def _components_starts(adj, deg, nb):
    """Seeds of the components in the order they are taken (the unvisited
    node of smallest (degree, id) each time) with each component's nodes."""
    seen = np.zeros(nb, dtype=bool)
    out = []
    for _ in range(nb):
        cand = [v for v in range(nb) if not seen[v]]
        if not cand:
            break
        s0 = min(cand, key=lambda v: (deg[v], v))
        comp = [w for level in _levels(adj, s0, deg) for w in level]
        for w in comp:
            seen[w] = True
        out.append((s0, comp))
    return out


SLOAN_W1, SLOAN_W2 = 1, 2


def sloan(nb: int, near: np.ndarray, w1: int = SLOAN_W1, w2: int = SLOAN_W2) -> np.ndarray:
    """Sloan's profile and wavefront reduction (Sloan's 1986 algorithm as
    restated by Kumfert and Pothen), per component:

    * start s: the pseudo-peripheral node found from the component's seed
      (as for Cuthill-McKee); end e: the node of smallest (degree, id) in
      the last level of the level structure rooted at s;
    * priority P(i) = w1 dist(i, e) - w2 (deg(i) + 1);
    * states inactive / preactive / active / postactive, s preactive first;
      repeatedly take the queued (preactive or active) node of largest
      priority, ties to the lowest id. If it was preactive, each neighbour
      gains w2 and an inactive neighbour becomes preactive. It is numbered
      (postactive). Each of its preactive neighbours becomes active and gains
      w2, and each non-postactive neighbour of such a node gains w2, an
      inactive one becoming preactive.
    """
    adj = leaf_graph(nb, near)
    deg = [len(a) for a in adj]
    order = []
    INACT, PRE, ACT, POST = 0, 1, 2, 3
    status = [INACT] * nb
    prio = [0] * nb
    for s0, comp in _components_starts(adj, deg, nb):
        s = pseudo_peripheral(adj, s0, deg)
        last = _levels(adj, s, deg)[-1]
        e = min(last, key=lambda v: (deg[v], v))
        for d, level in enumerate(_levels(adj, e, deg)):
            for v in level:
                prio[v] = w1 * d - w2 * (deg[v] + 1)
        status[s] = PRE
        queue = {s}
        while queue:
            i = max(queue, key=lambda v: (prio[v], -v))
            queue.remove(i)
            if status[i] == PRE:
                for j in adj[i]:
                    prio[j] += w2
                    if status[j] == INACT:
                        status[j] = PRE
                        queue.add(j)
            order.append(i)
            status[i] = POST
            for j in adj[i]:
                if status[j] == PRE:
                    status[j] = ACT
                    prio[j] += w2
                    for k in adj[j]:
                        if status[k] != POST:
                            prio[k] += w2
                            if status[k] == INACT:
                                status[k] = PRE
                                queue.add(k)
    return np.array(order, dtype=np.int64)


def king(nb: int, near: np.ndarray) -> np.ndarray:
    """King's front-minimising ordering, per component: number the
    pseudo-peripheral start first (as for Cuthill-McKee); then, of the front
    (unnumbered nodes adjacent to numbered ones), number the node that adds
    the fewest new nodes to the front, ties to the lowest id."""
    adj = leaf_graph(nb, near)
    deg = [len(a) for a in adj]
    order = []
    numbered = np.zeros(nb, dtype=bool)
    for s0, comp in _components_starts(adj, deg, nb):
        s = pseudo_peripheral(adj, s0, deg)
        front = set()
        nxt = s
        while nxt is not None:
            numbered[nxt] = True
            front.discard(nxt)
            order.append(nxt)
            for w in adj[nxt]:
                if not numbered[w]:
                    front.add(w)
            if not front:
                nxt = None
                break
            nxt = min(front, key=lambda v: (sum(1 for w in adj[v] if not numbered[w] and w not in front), v))
    return np.array(order, dtype=np.int64)


def make_order(kind: str, nb: int, near: np.ndarray) -> np.ndarray:
    kind = kind.lower()
    if kind == "natural":
        return np.arange(nb, dtype=np.int64)
    if kind == "cm":
        return cuthill_mckee(nb, near)
    if kind == "rcm":
        return reverse_cuthill_mckee(nb, near)
    if kind == "sloan":
        return sloan(nb, near)
    if kind == "king":
        return king(nb, near)
    raise ValueError(f"unknown ordering {kind}")


def inverse(order: np.ndarray) -> np.ndarray:
    rank = np.empty_like(order)
    rank[order] = np.arange(order.shape[0], dtype=order.dtype)
    return rank


def profile(nb: int, near: np.ndarray, order: np.ndarray) -> int:
    """Envelope size sum_i (i - min{j <= i adjacent to i}) in the new numbering."""
    rank = inverse(order)
    first = np.arange(nb)
    for i, j in near:
        a, b = int(rank[i]), int(rank[j])
        lo, hi = min(a, b), max(a, b)
        first[hi] = min(first[hi], lo)
    return int(np.sum(np.arange(nb) - first))


def bandwidth(nb: int, near: np.ndarray, order: np.ndarray) -> int:
    rank = inverse(order)
    bw = 0
    for i, j in near:
        bw = max(bw, abs(int(rank[i]) - int(rank[j])))
    return bw
