"""CPU oracle of distance-2 maximal independent sets and the aggregation
that turns them into a restriction operator (Section 5.3, Algorithm 3).

TEST INFRASTRUCTURE ONLY: used by tests/ and nowhere in the product.  It
shares no code with the HIP path; the random numbers come from a
counter-based generator that this file implements from its published
definition (the SplitMix64 output function of Steele, Lea and Flood), as
the HIP side does independently.

What it computes, in the order of Algorithm 3 (vectors are dense here; an
absent entry of a sparse vector is the largest 64-bit key, or False):
  every vertex starts as a candidate;
  while candidates remain:
    each candidate draws a key (random high half, vertex id low half, so
      keys never tie);
    minadj1 = A x keys over (min, select2nd): the smallest candidate key
      among the vertices adjacent to each vertex;
    minadj2 = A x minadj1 over the same semiring: the smallest within two
      hops;
    minadj = elementwise min of the two;
    newS = the candidates whose own key is not larger than minadj (they hold
      the smallest key within distance two);
    the candidates lose newS, then every vertex within two hops of newS
      (two more (min, select2nd) products, here with booleans);
    mis2 gains newS.
Aggregation: each MIS-2 vertex roots an aggregate numbered in vertex order,
together with its distance-1 neighbours (at most one root can be adjacent to
a vertex); every vertex still unassigned joins the aggregate of one of its
assigned neighbours, chosen by the generator.  R(i, agg(i)) = 1.

The pattern of A is read as an undirected graph (symmetric pattern).
"""

from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
ABSENT = np.uint64(MASK64)
GOLDEN = np.uint64(0x9E3779B97F4A7C15)
SALT_CHOICE = np.uint64(0x5DEECE66D2B9A1F3)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output for states x (state advanced by the golden gamma,
    then the variant-13 finalizer), elementwise on uint64."""
    with np.errstate(over="ignore"):
        z = (x.astype(np.uint64) + GOLDEN).astype(np.uint64)
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)).astype(np.uint64)
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)).astype(np.uint64)
        return (z ^ (z >> np.uint64(31))).astype(np.uint64)


def candidate_keys(seed: int, rnd: int, n: int) -> np.ndarray:
    """Key of every vertex in round rnd: random high 32 bits, vertex id low."""
    v = np.arange(n, dtype=np.uint64)
    ctr = (np.uint64(rnd) << np.uint64(32)) | v
    h = splitmix64(np.uint64(seed) ^ ctr)
    return (h & np.uint64(0xFFFFFFFF00000000)) | v


def choice_keys(seed: int, i: np.ndarray, j: np.ndarray) -> np.ndarray:
    """Key by which an unassigned vertex i ranks its assigned neighbour j."""
    ctr = (i.astype(np.uint64) << np.uint64(32)) | j.astype(np.uint64)
    return splitmix64(np.uint64(seed) ^ SALT_CHOICE ^ ctr)


def _row_of_entries(A) -> np.ndarray:
    return np.repeat(np.arange(A.nrows, dtype=np.int64), np.diff(A.row_ptr))


def mxv_min_select2nd(A, x: np.ndarray) -> np.ndarray:
    """y(i) = min over stored A(i,j) of x(j); ABSENT where the row is empty
    or every x(j) is absent."""
    y = np.full(A.nrows, ABSENT, dtype=np.uint64)
    if A.nnz:
        np.minimum.at(y, _row_of_entries(A), x[A.col])
    return y


def mxv_any(A, x: np.ndarray) -> np.ndarray:
    """y(i) = OR over stored A(i,j) of x(j) (booleans)."""
    y = np.zeros(A.nrows, dtype=bool)
    if A.nnz:
        np.logical_or.at(y, _row_of_entries(A), x[A.col])
    return y


def mis2(A, seed: int):
    """Returns (boolean mis2 membership, number of rounds)."""
    n = A.nrows
    cands = np.ones(n, dtype=bool)
    in_mis = np.zeros(n, dtype=bool)
    rnd = 0
    while cands.any():
        keys = np.where(cands, candidate_keys(seed, rnd, n), ABSENT)
        minadj1 = mxv_min_select2nd(A, keys)
        minadj2 = mxv_min_select2nd(A, minadj1)
        minadj = np.minimum(minadj1, minadj2)
        new = cands & (keys <= minadj)
        cands &= ~new
        adj1 = mxv_any(A, new)
        adj2 = mxv_any(A, adj1)
        cands &= ~(adj1 | adj2)
        in_mis |= new
        rnd += 1
    return in_mis, rnd


def aggregate(A, in_mis: np.ndarray, seed: int):
    """Aggregate of every vertex (int32) and the number of aggregates."""
    n = A.nrows
    roots = np.flatnonzero(in_mis)
    agg = np.full(n, -1, dtype=np.int64)
    agg[roots] = np.arange(roots.size)
    rows = _row_of_entries(A)
    # distance-1 neighbours of the roots
    hit = in_mis[A.col] & ~in_mis[rows]
    agg1 = agg.copy()
    agg1[rows[hit]] = agg[A.col[hit]]
    # the rest join an assigned neighbour, the one with the smallest choice key
    agg2 = agg1.copy()
    need = agg1[rows] < 0
    cand = need & (agg1[A.col] >= 0)
    if cand.any():
        r, c = rows[cand], A.col[cand]
        k = choice_keys(seed, r, c)
        order = np.lexsort((k, r))
        r, c = r[order], c[order]
        first = np.ones(r.size, dtype=bool)
        first[1:] = r[1:] != r[:-1]
        agg2[r[first]] = agg1[c[first]]
    if (agg2 < 0).any():
        raise ValueError("a vertex is farther than two hops from every MIS-2 vertex")
    return agg2.astype(np.int32), int(roots.size)


def restriction(n: int, n_agg: int, agg: np.ndarray):
    """R (n x n_agg) and R^T as CSR dataclasses with values 1.0."""
    from synth import canonical_from_coo
    idx = np.arange(n, dtype=np.int64)
    ones = np.ones(n)
    R = canonical_from_coo(n, n_agg, idx, agg.astype(np.int64), ones, dup="first")
    RT = canonical_from_coo(n_agg, n, agg.astype(np.int64), idx, ones, dup="first")
    return R, RT
