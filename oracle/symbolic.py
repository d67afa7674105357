"""Filled pattern of the scaling coefficients (oracle).

Eliminating leaf block k with Eq. 14/19 couples every pair of blocks that
row k touches: Z_ij receives -Z_ik Z_kk^-1 Z_kj. The set of later blocks in
row k after all earlier eliminations, S_k, is therefore the row pattern of
the combined scaling coefficients (the fill the orderings of Sec. 3.3
reduce, Figs. 3b-7b). This module computes it by the definition:

* U_k = { rank[j] : leaf j adjacent to leaf order[k], rank[j] > k };
* for k ascending: S_k = U_k, then for all i < j in S_k insert j into U_i;
* orig(k, j) = the two leaves are near-field neighbours (else a fill-in
  block, Sec. 3.4);
* etree parent(k) = min S_k (or -1).

Pinned in the tests by dense boolean Gaussian elimination of the permuted
leaf adjacency matrix.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Symbolic:
    order: np.ndarray        # new -> old leaf
    rank: np.ndarray         # old -> new leaf
    rows: list               # S_k as sorted lists of new indices (> k)
    orig: list               # per k, list of bools parallel to rows[k]
    parent: np.ndarray       # elimination tree parent (-1 for roots)

    @property
    def nb(self) -> int:
        return int(self.order.shape[0])

    def nnz_blocks(self) -> int:
        return sum(len(r) for r in self.rows)


def symbolic(nb: int, near: np.ndarray, order: np.ndarray) -> Symbolic:
    rank = np.empty_like(order)
    rank[order] = np.arange(nb, dtype=order.dtype)
    adj = [set() for _ in range(nb)]
    for i, j in near:
        i, j = int(i), int(j)
        if i != j:
            adj[i].add(j)
            adj[j].add(i)
    U = [set() for _ in range(nb)]
    for k in range(nb):
        for j in adj[int(order[k])]:
            if rank[j] > k:
                U[k].add(int(rank[j]))
    rows, origs = [], []
    parent = np.full(nb, -1, dtype=np.int64)
    for k in range(nb):
        S = sorted(U[k])
        rows.append(S)
        old_k = int(order[k])
        origs.append([int(order[j]) in adj[old_k] for j in S])
        if S:
            parent[k] = S[0]
        for a in range(len(S)):
            for b in range(a + 1, len(S)):
                U[S[a]].add(S[b])
    return Symbolic(order=order.copy(), rank=rank, rows=rows, orig=origs, parent=parent)
