"""Test-side helpers that restate the paper's definitions independently of the
oracle and of the GPU library: the neighbour stencil, the order with ties
broken by index, the literal iteration of Alg. 1/Alg. 2, and critical points
of a piecewise-linear field (Sec. II).
"""
from __future__ import annotations

import itertools
import random

import numpy as np


# --------------------------------------------------------------- neighbours
def stencil(nd: int):
    """Edges of the Freudenthal triangulation of the grid: the offsets in
    {-1,0,1}^nd, other than 0, whose nonzero entries all have one sign."""
    out = []
    for d in itertools.product((-1, 0, 1), repeat=nd):
        if all(v == 0 for v in d):
            continue
        if any(v > 0 for v in d) and any(v < 0 for v in d):
            continue
        out.append(d)
    return out


def neighbours(shape, p):
    coords = np.unravel_index(p, shape)
    res = []
    for d in stencil(len(shape)):
        c = [a + b for a, b in zip(coords, d)]
        if all(0 <= c[i] < shape[i] for i in range(len(shape))):
            res.append(int(np.ravel_multi_index(c, shape)))
    return res


def order_keys(x: np.ndarray) -> np.ndarray:
    """Integer keys ordered like the values, -0 equal to +0 (int64)."""
    x = np.ascontiguousarray(x)
    if x.dtype == np.float32:
        u = x.view(np.uint32).astype(np.int64)
        neg = (u >> 31) == 1
        mag = u & 0x7FFFFFFF
    else:
        u = x.view(np.uint64)
        neg = (u >> np.uint64(63)) == 1
        mag = (u & np.uint64(0x7FFFFFFFFFFFFFFF)).astype(np.int64)
        u = u.astype(np.int64)
    return np.where(neg, -mag, mag).astype(np.int64)


# --------------------------------------------------------------- Alg. 1 / 2
def _less(vals, a, b):
    # a "should be less than" b: smaller value, or equal value and lower index
    return vals[a] < vals[b] or (vals[a] == vals[b] and a < b)


def alg2_fixed_point(values, bins, shape, schedule="jacobi", seed=0,
                     max_iter=100000):
    """Run Alg. 1 (flags + worklists) with Alg. 2 iterations until the
    worklist is empty.  ``schedule`` = "jacobi": every point of the worklist
    reads the subbins of the previous iteration; "async": points are visited
    one at a time in a random order and see every earlier update.
    ``values`` are compared as Python floats (exact for float32/float64)."""
    n = int(np.prod(shape))
    vals = [float(v) for v in np.asarray(values).ravel()]
    b = [int(v) for v in np.asarray(bins).ravel()]
    nb = [neighbours(shape, p) for p in range(n)]
    lower = [[q for q in nb[p] if b[q] == b[p] and _less(vals, q, p)] for p in range(n)]
    greater = [[q for q in nb[p] if b[q] == b[p] and _less(vals, p, q)] for p in range(n)]
    s = [0] * n
    work = list(range(n))
    rng = random.Random(seed)
    it = 0
    while work:
        it += 1
        if it > max_iter:
            raise RuntimeError("no convergence")
        nxt = set()
        if schedule == "jacobi":
            snap = list(s)
            for p in work:
                m = 0
                for q in lower[p]:
                    m = max(m, snap[q] + (1 if q > p else 0))
                if s[p] < m:
                    s[p] = m
                    nxt.update(greater[p])
        else:
            order = list(work)
            rng.shuffle(order)
            for p in order:
                m = 0
                for q in lower[p]:
                    m = max(m, s[q] + (1 if q > p else 0))
                if s[p] < m:
                    s[p] = m
                    nxt.update(greater[p])
        work = sorted(nxt)
    return np.array(s, dtype=np.uint64).reshape(shape), it


# --------------------------------------------------------------- critical points
_TABLES = {}


def _components_table(nd):
    """Number of connected components of every subset of the link of an
    interior vertex; two link vertices u, w are joined when w - u is itself
    a stencil offset (they span a triangle with the centre)."""
    if nd in _TABLES:
        return _TABLES[nd]
    st = stencil(nd)
    k = len(st)
    adj = [[j for j in range(k) if j != i and tuple(b - a for a, b in zip(st[i], st[j])) in set(st)]
           for i in range(k)]
    table = np.zeros(1 << k, np.int8)
    for mask in range(1 << k):
        seen = 0
        comps = 0
        for i in range(k):
            if not (mask >> i) & 1 or (seen >> i) & 1:
                continue
            comps += 1
            stack = [i]
            seen |= 1 << i
            while stack:
                u = stack.pop()
                for w in adj[u]:
                    if (mask >> w) & 1 and not (seen >> w) & 1:
                        seen |= 1 << w
                        stack.append(w)
        table[mask] = comps
    _TABLES[nd] = (st, table)
    return _TABLES[nd]


REGULAR, MINIMUM, MAXIMUM, SADDLE = 0, 1, 2, 3


def critical_points(x: np.ndarray) -> np.ndarray:
    """Type of every vertex of the PL field (Sec. II): no lower link vertex ->
    minimum, no upper -> maximum, one connected component each -> regular,
    otherwise saddle.  Ties are broken by linear index.  Boundary vertices use
    the part of the link that lies in the grid."""
    st, table = _components_table(x.ndim)
    key = order_keys(x)
    idx = np.arange(x.size, dtype=np.int64).reshape(x.shape)
    lo = np.zeros(x.shape, np.int64)
    hi = np.zeros(x.shape, np.int64)
    for j, d in enumerate(st):
        src = tuple(slice(max(0, v), x.shape[i] + min(0, v)) for i, v in enumerate(d))
        dst = tuple(slice(max(0, -v), x.shape[i] + min(0, -v)) for i, v in enumerate(d))
        kn = key[src]
        kp = key[dst]
        less = (kn < kp) | ((kn == kp) & (idx[src] < idx[dst]))
        lo[dst] |= less.astype(np.int64) << j
        hi[dst] |= (~less).astype(np.int64) << j
    nlo = table[lo]
    nhi = table[hi]
    t = np.full(x.shape, SADDLE, np.int8)
    t[(nlo == 1) & (nhi == 1)] = REGULAR
    t[nlo == 0] = MINIMUM
    t[nhi == 0] = MAXIMUM
    return t


def edge_orders(x: np.ndarray):
    """For every stencil edge (p, p+d) with d a 'positive' offset, whether p
    comes before p+d in the order (value, index).  Returns a list of arrays."""
    key = order_keys(x)
    res = []
    for d in stencil(x.ndim):
        if not any(v > 0 for v in d):
            continue
        a = tuple(slice(0, x.shape[i] - v) for i, v in enumerate(d))
        b = tuple(slice(v, x.shape[i]) for i, v in enumerate(d))
        res.append(key[a] <= key[b])  # equal keys: p has the lower index
    return res
