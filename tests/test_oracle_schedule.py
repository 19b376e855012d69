"""Pins for the oracle's dimension-tree schedules against the cost tables
printed in Section 3.4 (Tables 1-6, Corollary 1) and against the update
orders described in Section 3.1."""
import json
import os

import numpy as np
import pytest

import oracle as O
import synthgen as G

GOLD = os.path.join(os.path.dirname(__file__), "golden", "ttm_flops_tables.json")


def _poly_from_terms(terms):
    out = {}
    for coef, modes, rpow in terms:
        key = (tuple(m - 1 for m in sorted(modes)), rpow)
        out[key] = out.get(key, 0) + coef
    return out


def _lead(poly, N):
    return {k: v for k, v in poly.items() if k[1] == 1}


def _entries():
    with open(GOLD) as f:
        return json.load(f)["entries"]


@pytest.mark.parametrize("entry", _entries(), ids=lambda e: e["cite"][:40])
def test_schedule_flops_match_paper_tables(entry):
    N, tree, sweeps = entry["N"], entry["tree"], entry["sweeps"]
    got = O.schedule_flops(O.tree_schedule(N, tree, sweeps), N)
    want = _poly_from_terms(entry["terms"])
    if entry.get("as_printed_conflicts_with_table5"):
        # the printed Table 6 splits Table 5's 6 I2 I4 R^3 into
        # 4 I2 I4 R^3 + 2 I2 I3 R^3; the two agree when I3 = I4
        assert got != want
        I = {0: 3, 1: 5, 2: 7, 3: 7}
        R = 2

        def ev(p):
            return sum(c * np.prod([I[m] for m in k[0]]) * R ** k[1] for k, c in p.items())
        assert ev(got) == ev(want)
        return
    if entry.get("leading_only"):
        assert _lead(got, N) == _lead(want, N)
    else:
        assert got == want


@pytest.mark.parametrize("N", [5, 6])
def test_corollary1_terms(N):
    """Equal sizes: leading two terms and last term of Corollary 1."""
    def collapse(p):
        c = {}
        for (modes, rp), v in p.items():
            c[rp] = c.get(rp, 0) + v
        return c
    none = collapse(O.schedule_flops(O.tree_schedule(N, "none", 3), N))
    std = collapse(O.schedule_flops(O.tree_schedule(N, "standard", 3), N))
    rst = collapse(O.schedule_flops(O.tree_schedule(N, "restructured", 3), N))
    assert none[1] == 6 * N and none[2] == 6 * N and none[N - 1] == 6 * N
    assert std[1] == 12 and std[2] == 18 and std[N - 1] == 6 * N
    assert rst[1] == 8 and rst[2] == 14 and rst[N - 1] == 6 * N
    # the headline: a third less of the dominant term than the standard tree
    assert rst[1] / std[1] == pytest.approx(2 / 3)


@pytest.mark.parametrize("N", [3, 4, 5, 6])
@pytest.mark.parametrize("tree", ["none", "standard", "restructured"])
def test_schedule_orders_match_closed_form(N, tree):
    sched = O.tree_schedule(N, tree, 9)
    for k, steps in enumerate(sched, start=1):
        order = [s[1] for s in steps if s[0] == "update"]
        assert sorted(order) == list(range(N))
        assert order == O.sweep_order(N, tree, k)


def test_restructured_orders_described_in_text():
    """Order 4: the second sweep begins with A(3) (from Y^(3,4)); the third
    begins with A(1) then A(3) (Section 3.1)."""
    assert O.sweep_order(4, "restructured", 2)[0] == 2
    assert O.sweep_order(4, "restructured", 3)[:2] == [0, 2]
    assert O.sweep_order(3, "restructured", 3) == [1, 0, 2]


@pytest.mark.parametrize("N,dims,R", [(3, (6, 5, 7), 3), (4, (4, 5, 3, 6), 3), (5, (4, 3, 5, 3, 4), 2)])
@pytest.mark.parametrize("tree", ["standard", "restructured"])
def test_tree_leaves_equal_direct_multi_ttm(N, dims, R, tree):
    p = G.make_problem(dims, R, seed=60 + N, rho=0.05)
    out = O.run_tree_schedule(p.X, R, p.init, 7, tree)
    assert out["max_leaf_err"] < 1e-12
    ref = O.cp_als_qr(p.X, R, p.init, iters=7, tree=tree)
    assert out["orders"] == ref["orders"]
    for a, b in zip(out["factors"], ref["factors"]):
        assert np.allclose(a, b, atol=1e-11)
    assert np.allclose(out["fits"], ref["fits"], atol=1e-12)


def test_standard_tree_iterates_equal_no_tree():
    p = G.make_problem((7, 6, 5, 4), 3, seed=70, rho=0.03)
    a = O.run_tree_schedule(p.X, 3, p.init, 5, "standard")
    b = O.cp_als_qr(p.X, 3, p.init, iters=5, tree="none")
    for x, y in zip(a["factors"], b["factors"]):
        assert np.allclose(x, y, atol=1e-12)
