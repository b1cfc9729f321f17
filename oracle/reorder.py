"""Oracle for the hub-and-spoke matrix reordering (Section 3.2, Algorithm 2).

TEST INFRASTRUCTURE ONLY: this module is imported by tests, the smoke check and
the CPU baseline leg of the benchmark, never by the product path.

The feature matrix is read as a bipartite graph (Definition 1): instance nodes
are rows, feature nodes are columns and every stored non-zero is an edge.
Each iteration picks the ceil(k|V_T|) and ceil(k|V_F|) highest-degree nodes of
the current graph as hubs and gives them the highest free ids, finds the
connected components of what is left, gives every component except the giant
one the lowest free ids, and continues on the giant component. It stops once
the giant component has fewer instance nodes than this iteration's instance hub
count, or fewer feature nodes than its feature hub count (or is empty).

Readings of points the paper leaves open (each one is written down because the
permutation must be reproduced bit for bit by the host library):

* degree = number of neighbours inside the current graph; hubs are taken in
  (degree descending, original index ascending) order;
* the hub counts use the current graph's node counts, ceil evaluated in IEEE
  double as ceil(k * count), clamped to the count;
* inside one hub batch the first hub in that order gets the highest free id;
* components are discovered by scanning instance nodes in ascending original
  index, then feature nodes in ascending original index; the giant component is
  the one with the most nodes (instances + features), ties to the first found;
* non-giant components take the lowest free ids in discovery order; inside one
  component, instances in ascending original index, then features likewise,
  so each component is one contiguous diagonal block;
* isolated nodes are components of their own (blocks of width or height 0);
* the final giant component becomes the last diagonal block.

Implementation: scipy's connected-components routine labels the components;
the discovery order is then the order of each component's smallest node in
the instances-then-features numbering, which is exactly the seed that a scan
in that order would reach first.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


@dataclasses.dataclass
class Reordering:
    piT: np.ndarray          # int32[m]: original row -> new row
    piF: np.ndarray          # int32[n]: original column -> new column
    blocks: np.ndarray       # int64[B, 4]: (row0, col0, rows, cols) in new ids
    m1: int
    n1: int
    m2: int
    n2: int
    iterations: int


def hub_count(k: float, count: int) -> int:
    return min(count, max(0, int(math.ceil(k * float(count)))))


def reorder(m: int, n: int, indptr: np.ndarray, indices: np.ndarray, k: float = 0.01) -> Reordering:
    indptr = np.asarray(indptr, dtype=np.int64)
    indices = np.asarray(indices, dtype=np.int64)
    rows = np.repeat(np.arange(m, dtype=np.int64), np.diff(indptr))
    cols = indices
    aliveT = np.ones(m, dtype=bool)
    aliveF = np.ones(n, dtype=bool)
    piT = np.full(m, -1, dtype=np.int64)
    piF = np.full(n, -1, dtype=np.int64)
    loT = loF = 0
    hiT, hiF = m - 1, n - 1
    blocks = []
    iterations = 0
    while True:
        iterations += 1
        nT = int(aliveT.sum())
        nF = int(aliveF.sum())
        mhub = hub_count(k, nT)
        nhub = hub_count(k, nF)
        live = aliveT[rows] & aliveF[cols]
        degT = np.bincount(rows[live], minlength=m)
        degF = np.bincount(cols[live], minlength=n)
        # hubs: alive nodes ordered by (degree desc, index asc)
        candT = np.flatnonzero(aliveT)
        hubT = candT[np.lexsort((candT, -degT[candT]))][:mhub]
        candF = np.flatnonzero(aliveF)
        hubF = candF[np.lexsort((candF, -degF[candF]))][:nhub]
        piT[hubT] = hiT - np.arange(hubT.size)
        piF[hubF] = hiF - np.arange(hubF.size)
        hiT -= hubT.size
        hiF -= hubF.size
        aliveT[hubT] = False
        aliveF[hubF] = False
        # components of G' (alive nodes, edges between alive nodes)
        live = aliveT[rows] & aliveF[cols]
        g = sp.coo_matrix((np.ones(int(live.sum()), dtype=np.int8), (rows[live], m + cols[live])),
                          shape=(m + n, m + n)).tocsr()
        _, label = connected_components(g, directed=False)
        alive_nodes = np.concatenate([np.flatnonzero(aliveT), m + np.flatnonzero(aliveF)])
        if alive_nodes.size == 0:
            break
        lab = label[alive_nodes]
        uniq_lab, inv = np.unique(lab, return_inverse=True)
        # smallest node of each component in the instances-then-features numbering
        first = np.full(uniq_lab.size, np.iinfo(np.int64).max, dtype=np.int64)
        np.minimum.at(first, inv, alive_nodes)
        sizes = np.bincount(inv, minlength=uniq_lab.size)
        disc = np.argsort(first, kind="stable")          # discovery order of components
        giant = disc[np.argmax(sizes[disc])]               # argmax returns the first maximum
        # members of each component, instances then features, each ascending
        comp_of_T = np.full(m, -1, dtype=np.int64)
        comp_of_F = np.full(n, -1, dtype=np.int64)
        is_T = alive_nodes < m
        comp_of_T[alive_nodes[is_T]] = inv[is_T]
        comp_of_F[alive_nodes[~is_T] - m] = inv[~is_T]
        giant_T = np.flatnonzero(comp_of_T == giant)
        giant_F = np.flatnonzero(comp_of_F == giant)
        rank = np.empty(uniq_lab.size, dtype=np.int64)
        rank[disc] = np.arange(uniq_lab.size)
        # spokes in discovery order
        spT = np.flatnonzero((comp_of_T >= 0) & (comp_of_T != giant))
        spF = np.flatnonzero((comp_of_F >= 0) & (comp_of_F != giant))
        spT = spT[np.lexsort((spT, rank[comp_of_T[spT]]))]
        spF = spF[np.lexsort((spF, rank[comp_of_F[spF]]))]
        cntT = np.bincount(rank[comp_of_T[spT]], minlength=uniq_lab.size)
        cntF = np.bincount(rank[comp_of_F[spF]], minlength=uniq_lab.size)
        piT[spT] = loT + np.arange(spT.size)
        piF[spF] = loF + np.arange(spF.size)
        for c in range(uniq_lab.size):
            if disc[c] == giant:
                continue
            blocks.append((loT, loF, int(cntT[c]), int(cntF[c])))
            loT += int(cntT[c])
            loF += int(cntF[c])
        aliveT[:] = False
        aliveF[:] = False
        aliveT[giant_T] = True
        aliveF[giant_F] = True
        if giant_T.size < mhub or giant_F.size < nhub or (giant_T.size + giant_F.size) == 0:
            break
    # the final giant component is the last diagonal block
    gT = np.flatnonzero(aliveT)
    gF = np.flatnonzero(aliveF)
    if gT.size + gF.size > 0:
        piT[gT] = loT + np.arange(gT.size)
        piF[gF] = loF + np.arange(gF.size)
        blocks.append((loT, loF, int(gT.size), int(gF.size)))
        loT += gT.size
        loF += gF.size
    assert loT == hiT + 1 and loF == hiF + 1, "ids do not meet"
    m1, n1 = loT, loF
    blocks = np.asarray(blocks, dtype=np.int64).reshape(-1, 4)
    return Reordering(piT.astype(np.int32), piF.astype(np.int32), blocks,
                      int(m1), int(n1), int(m - m1), int(n - n1), iterations)
