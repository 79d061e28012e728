"""Pins of the oracle's Dormand-Prince 5(4) coefficients (the pair ode45 uses,
Sec. 1 and Fig. 2 caption) against what the mathematics fixes: the order
conditions of Butcher's rooted-tree theory in exact rational arithmetic, the
row-sum (consistency) conditions, the first-same-as-last row and the method's
stability polynomial."""
from fractions import Fraction

import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore")


def _rational(x: float) -> Fraction:
    fr = Fraction(x).limit_denominator(10**6)
    assert float(fr) == x, f"{x!r} is not the double nearest to a small rational"
    return fr


@pytest.fixture(scope="module")
def tab(aio):
    t = aio.tableau()
    return {
        "c": [_rational(v) for v in t["c"]],
        "a": [[_rational(v) for v in row] for row in t["a"]],
        "b": [_rational(v) for v in t["b"]],
        "bhat": [_rational(v) for v in t["bhat"]],
        "e": [_rational(v) for v in t["e"]],
    }


def _canon(tree):
    return tuple(sorted(_canon(ch) for ch in tree))


def _attach_everywhere(tree):
    """All trees obtained by adding one leaf to some vertex of ``tree``."""
    out = [_canon(tree + ((),))]
    for i, ch in enumerate(tree):
        for grown in _attach_everywhere(ch):
            out.append(_canon(tree[:i] + (grown,) + tree[i + 1:]))
    return out


def rooted_trees(order):
    level = {()}
    for _ in range(order - 1):
        level = {g for t in level for g in _attach_everywhere(t)}
    return sorted(level)


def _order(t):
    return 1 + sum(_order(c) for c in t)


def _gamma(t):
    g = _order(t)
    for c in t:
        g *= _gamma(c)
    return g


def _phi(t, a):
    s = len(a)
    v = [Fraction(1)] * s
    for c in t:
        pc = _phi(c, a)
        apc = [sum(a[i][j] * pc[j] for j in range(s)) for i in range(s)]
        v = [v[i] * apc[i] for i in range(s)]
    return v


def _condition_holds(t, weights, a):
    return sum(w * p for w, p in zip(weights, _phi(t, a))) == Fraction(1, _gamma(t))


def test_tree_counts():
    # number of rooted trees of order 1..6 (OEIS A000081)
    assert [len(rooted_trees(k)) for k in range(1, 7)] == [1, 1, 2, 4, 9, 20]


def test_explicit_and_consistent(tab):
    a, c = tab["a"], tab["c"]
    for i in range(7):
        assert all(a[i][j] == 0 for j in range(i, 7)), "method must be explicit"
        assert sum(a[i]) == c[i], f"row sum of stage {i + 1} must equal c"


def test_first_same_as_last(tab):
    assert tab["a"][6] == tab["b"]
    assert tab["c"][6] == 1 and tab["b"][6] == 0


def test_fifth_order_weights(tab):
    a, b = tab["a"], tab["b"]
    for k in range(1, 6):
        for t in rooted_trees(k):
            assert _condition_holds(t, b, a), f"order-{k} condition fails for tree {t}"
    failing6 = [t for t in rooted_trees(6) if not _condition_holds(t, b, a)]
    assert failing6, "weights b are not of order 6"


def test_fourth_order_embedded_weights(tab):
    a, bh = tab["a"], tab["bhat"]
    for k in range(1, 5):
        for t in rooted_trees(k):
            assert _condition_holds(t, bh, a), f"order-{k} condition fails for bhat, tree {t}"
    assert any(not _condition_holds(t, bh, a) for t in rooted_trees(5))


def test_error_weights_are_difference(tab):
    assert tab["e"] == [x - y for x, y in zip(tab["b"], tab["bhat"])]
    assert sum(tab["e"]) == 0


def _stability_coeffs(weights, a):
    s = len(a)
    coeffs = [Fraction(1)]
    v = [Fraction(1)] * s
    for _ in range(s):
        coeffs.append(sum(w * x for w, x in zip(weights, v)))
        v = [sum(a[i][j] * v[j] for j in range(s)) for i in range(s)]
    return coeffs


def test_stability_polynomial(tab):
    # R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 + z^5/120 + z^6/600 for this pair
    coeffs = _stability_coeffs(tab["b"], tab["a"])
    expect = [Fraction(1), Fraction(1), Fraction(1, 2), Fraction(1, 6), Fraction(1, 24),
              Fraction(1, 120), Fraction(1, 600), Fraction(0)]
    assert coeffs == expect
