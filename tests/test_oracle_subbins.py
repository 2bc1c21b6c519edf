"""Pins of the oracle's subbins (Sec. IV-B, Alg. 1, Alg. 2, Sec. IV-E).

The oracle computes the subbins in one pass over the points sorted by
(value, index).  Here they are checked against the literal worklist
iteration of Alg. 1/Alg. 2 (synchronous and random asynchronous schedules)
on exhaustive and random tiny grids, against closed forms, and against the
bounds of Sec. IV-E."""
import itertools

import numpy as np
import pytest

import topo


def codes(ref, x, eps):
    e, inv = ref.error_params(x, eps, ref.ABS)
    b = ref.bins(x, inv)
    return b, ref.subbins(x, b)


def test_worked_examples(ref):
    # an exact tie becomes strict: the later index of the tie is raised
    x = np.array([[0.3, 0.3, 0.1]])
    b, s = codes(ref, x, 1.0)
    assert b.tolist() == [[0, 0, 0]]
    assert s.tolist() == [[0, 1, 0]]
    # a strict pair whose lower value has the lower index needs no subbin
    x = np.array([[0.2, 0.3]])
    assert codes(ref, x, 1.0)[1].tolist() == [[0, 0]]


@pytest.mark.parametrize("n", [2, 5, 9, 31])
def test_chain_closed_forms(ref, n):
    """Sec. IV-E worst case: a chain of n same-bin points whose value falls as
    the index rises needs subbins n-1 ... 0; a rising chain or a plateau needs
    none."""
    falling = np.linspace(0.9, 0.1, n).reshape(1, n)
    assert codes(ref, falling, 10.0)[1].ravel().tolist() == list(range(n - 1, -1, -1))
    rising = np.linspace(0.1, 0.9, n).reshape(1, n)
    assert not codes(ref, rising, 10.0)[1].any()
    plateau = np.full((1, n), 0.5)
    assert not codes(ref, plateau, 10.0)[1].any()
    # the literal iteration needs n sweeps for the falling chain
    s, it = topo.alg2_fixed_point(falling, np.zeros_like(falling, np.int64), falling.shape)
    assert s.ravel().tolist() == list(range(n - 1, -1, -1))


def _check_against_alg2(ref, x, eps, seeds=(0, 1)):
    b, s = codes(ref, x, eps)
    sj, _ = topo.alg2_fixed_point(x, b, x.shape, "jacobi")
    assert np.array_equal(s, sj), (x, b, s, sj)
    for seed in seeds:
        sa, _ = topo.alg2_fixed_point(x, b, x.shape, "async", seed=seed)
        assert np.array_equal(s, sa)
    return b, s


def test_exhaustive_2x3_small_alphabet(ref):
    """Every assignment of values {0, 1, 2} to a 2x3 grid (729 fields), with a
    bound putting all values in one bin and one putting them in separate bins."""
    for vals in itertools.product((0.0, 0.25, 0.5), repeat=6):
        x = np.array(vals).reshape(2, 3)
        _check_against_alg2(ref, x, 10.0, seeds=(0,))
        b, s = _check_against_alg2(ref, x, 0.1, seeds=())
        assert not s.any()  # no two neighbours share a bin


@pytest.mark.parametrize("shape", [(3, 3), (4, 3), (2, 2, 2), (3, 2, 3), (1, 7), (2, 2, 3)])
def test_random_tiny_grids(ref, shape):
    rng = np.random.default_rng(sum(shape) * 7 + len(shape))
    for t in range(60):
        levels = rng.integers(2, 6)
        x = rng.integers(0, levels, shape).astype(np.float64) / 8.0
        if t % 3 == 0:
            x = rng.standard_normal(shape)
        if t % 4 == 1:
            x = x.astype(np.float32)
        for eps in (10.0, 0.2, 0.05):
            _check_against_alg2(ref, x, eps)


def test_bounds_of_section_iv_e(ref):
    """Subbins of a connected same-bin component of n points lie in [0, n-1];
    points with no lower same-bin neighbour keep 0; a subbin is below the
    number of distinct values between the bin floor and the point."""
    rng = np.random.default_rng(11)
    for t in range(20):
        x = (rng.integers(0, 12, (9, 11)) / 16.0).astype(np.float64)
        x += rng.standard_normal(x.shape) * (1e-3 if t % 2 else 0.0)
        eps = 0.3
        b, s = codes(ref, x, eps)
        n = x.size
        shape = x.shape
        # connected same-bin components
        comp = -np.ones(n, np.int64)
        c = 0
        for p in range(n):
            if comp[p] >= 0:
                continue
            stack = [p]
            comp[p] = c
            while stack:
                u = stack.pop()
                for w in topo.neighbours(shape, u):
                    if comp[w] < 0 and b.flat[w] == b.flat[u]:
                        comp[w] = c
                        stack.append(w)
            c += 1
        sizes = np.bincount(comp)
        assert (s.ravel() <= sizes[comp] - 1).all()
        flat = x.ravel()
        for p in range(n):
            lower = [q for q in topo.neighbours(shape, p)
                     if b.flat[q] == b.flat[p] and (flat[q] < flat[p] or (flat[q] == flat[p] and q < p))]
            if not lower:
                assert s.flat[p] == 0
            same_bin = flat[(b.ravel() == b.flat[p]) & (flat <= flat[p])]
            assert s.flat[p] <= len(np.unique(same_bin)) - 1


def test_tiny_bound_gives_zero_subbins(ref):
    rng = np.random.default_rng(5)
    x = rng.standard_normal((20, 20))
    b, s = codes(ref, x, 1e-9)
    assert not s.any()


def test_subbins_are_a_fixed_point_on_larger_fields(ref):
    """On a 48x40 and a 12x10x9 field the oracle's subbins satisfy the
    equations of Alg. 2 at every point (checked in numpy)."""
    rng = np.random.default_rng(6)
    for shape in [(48, 40), (12, 10, 9)]:
        x = np.cumsum(rng.standard_normal(shape), axis=0)
        b, s = codes(ref, x, 0.5)
        s = s.astype(np.int64)
        key = topo.order_keys(x)
        idx = np.arange(x.size).reshape(shape)
        want = np.zeros(shape, np.int64)
        for d in topo.stencil(x.ndim):
            src = tuple(slice(max(0, v), shape[i] + min(0, v)) for i, v in enumerate(d))
            dst = tuple(slice(max(0, -v), shape[i] + min(0, -v)) for i, v in enumerate(d))
            lower = (b[src] == b[dst]) & ((key[src] < key[dst]) | ((key[src] == key[dst]) & (idx[src] < idx[dst])))
            cand = s[src] + (idx[src] > idx[dst])
            want[dst] = np.maximum(want[dst], np.where(lower, cand, 0))
        assert np.array_equal(want, s)
