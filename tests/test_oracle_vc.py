"""Pins of the oracle's VC-dimension bounds (Sec. 4.3: the range space Q_k
whose ranges are the hyperedges met by a set of at most k nodes; Lemma
vcboundgeneral, Lemma lemmavckbound and the union bound), checked against
VC dimensions computed by brute force on small hyperedge families: a family
built to be shattered reaches d1, random families never pass it, and VC(Q_2)
stays within both bounds of Q_2 and log2 of its number of ranges."""
import itertools
import math

import numpy as np
import pytest

import oracle


def ranges(family, n, k):
    """Every range of Q_k on the family: the set of hyperedges (indices)
    that a node set S with |S| <= k meets."""
    out = set()
    for size in range(k + 1):
        for S in itertools.combinations(range(n), size):
            Sset = set(S)
            out.add(frozenset(i for i, h in enumerate(family) if Sset & h))
    return out


def vc_dimension(family, n, k):
    """Largest number of hyperedges of the family shattered by Q_k."""
    R = ranges(family, n, k)
    best = 0
    for size in range(1, len(family) + 1):
        found = False
        for X in itertools.combinations(range(len(family)), size):
            Xs = frozenset(X)
            if len({r & Xs for r in R}) == 2 ** size:
                found = True
                break
        if not found:
            break
        best = size
    return best


def shattered_family(d):
    """d hyperedges shattered by single nodes: one node per nonempty pattern
    of the d hyperedges, each hyperedge holding the 2^(d-1) nodes of the
    patterns that contain it."""
    patterns = [p for p in range(1, 2 ** d)]
    fam = [frozenset(j for j, p in enumerate(patterns) if p >> i & 1) for i in range(d)]
    return fam, len(patterns)


@pytest.mark.parametrize("b,d1", [(1, 1), (2, 2), (3, 2), (4, 3), (7, 3), (8, 4), (15, 4), (16, 5),
                                  (2 ** 40, 41), (2 ** 63, 64), (2 ** 64 - 1, 64)])
def test_d1_closed_form(b, d1):
    assert oracle.vc_dims(b, 1, 10)[0] == d1


@pytest.mark.parametrize("b", [1, 2, 3, 4, 5, 8])
def test_d1_is_reached(b):
    # the shattered family of d1 hyperedges has hyperedges of 2^(d1-1) <= b
    # nodes, so VC(Q_1) >= d1 on hyperedges of at most b nodes
    d1 = oracle.vc_dims(b, 1, 10)[0]
    fam, n = shattered_family(d1)
    assert max(len(h) for h in fam) <= b
    assert vc_dimension(fam, n, 1) == d1
    # one more hyperedge shattered would need hyperedges of 2^d1 > b nodes
    assert 2 ** d1 > b


@pytest.mark.parametrize("seed", range(6))
def test_random_families_stay_within_the_bounds(seed):
    rng = np.random.default_rng(seed)
    n = 7
    for b in [1, 2, 3, 4]:
        fam = {frozenset(rng.choice(n, size=int(rng.integers(1, b + 1)), replace=False).tolist())
               for _ in range(9)}
        fam = sorted(fam, key=sorted)
        d1, dk1, du1 = oracle.vc_dims(b, 1, n)
        assert vc_dimension(fam, n, 1) <= d1
        v2 = vc_dimension(fam, n, 2)
        _, dk2, du2 = oracle.vc_dims(b, 2, n)
        assert v2 <= dk2 and v2 <= du2
        assert v2 <= math.floor(math.log2(len(ranges(fam, n, 2)))) <= du2


def test_union_bound_closed_form_and_errors():
    # n = 2^j: floor(k log2 n) = k j exactly
    for j in [1, 5, 20, 40]:
        for k in [1, 3, 50]:
            assert oracle.vc_dims(4, k, 2 ** j)[2] == k * j
    # the lemma's bound grows like k log k, the union bound like k log n
    d1, dk, du = oracle.vc_dims(3, 50, 10 ** 6)
    assert d1 == 2 and dk == math.floor(2 * 2 * 50 * math.log2(150)) and du == math.floor(50 * math.log2(10 ** 6))
    assert oracle.vc_dims(0, 1, 1) is None and oracle.vc_dims(1, 0, 1) is None and oracle.vc_dims(1, 1, 0) is None
