"""Pins of the tolerance schedule against the values printed in Sec. 5.2
(Tables tab:1m, tab:2m) and the baselines of eq. (stop_tol)."""
import json
import os

import pytest

import oracle.w1_oracle as o

GOLD = os.path.join(os.path.dirname(__file__), "golden", "tolerance_tables.json")


def _load():
    with open(GOLD) as f:
        return json.load(f)


def _two_digits(x):
    return float(f"{x:.2g}") if x < 1.2e-5 or x >= 1.3e-5 else float(f"{x:.3g}")


@pytest.mark.parametrize("row", _load()["schedules"], ids=lambda r: f"{r['table']}-a{r['alpha']}")
def test_printed_schedules(row):
    got = o.level_tolerances(row["eps_L"], row["alpha"], row["n"], row["L"])
    assert len(got) == len(row["printed"])
    for g, p in zip(got, row["printed"]):
        # printed with two significant digits (1.25e-5 with three)
        assert abs(g - p) <= 0.051 * p, (g, p)


@pytest.mark.parametrize("row", _load()["baselines"], ids=lambda r: r["caption"])
def test_printed_baselines(row):
    got = o.paper_stop_tolerance(row["algo"], row["n"], row["multilevel"])
    assert abs(got - row["printed"]) <= 0.04 * row["printed"]


@pytest.mark.parametrize("row", _load()["eps_L_rule"], ids=lambda r: r["what"])
def test_stop_tol_matches_table_rows(row):
    assert o.paper_stop_tolerance(row["algo"], row["n"], row["multilevel"]) == pytest.approx(row["value"], rel=1e-12)


def test_level_sides():
    assert o.level_sides(512, 4) == [64, 128, 256, 512]
    assert o.level_sides(64, 1) == [64]
    assert o.level_sides(256, 6) == [8, 16, 32, 64, 128, 256]


@pytest.mark.parametrize("algo", [1, 2])
def test_per_level_caps(algo):
    """Per-level iteration caps: with a zero tolerance every level runs to
    its own cap; one cap repeated per level is the scalar cap; a cap above
    a level's stop leaves that level unchanged."""
    import oracle.w1_oracle as o
    import w1data
    n, L = 16, 3
    p0, p1 = w1data.random_pair(n, 5)
    caps = [7, 3, 5]
    r = o.solve(p0, p1, n, L=L, p=2, algo=algo, stop="fpr", tol=0.0, eps_L=0.0, max_iters=caps,
                return_fields=False)
    assert r["iters"] == caps and r["status"] == "maxiter"
    a = o.solve(p0, p1, n, L=L, p=2, algo=algo, stop="fpr", tol=0.0, eps_L=0.0, max_iters=[4, 4, 4],
                return_fields=False)
    b = o.solve(p0, p1, n, L=L, p=2, algo=algo, stop="fpr", tol=0.0, eps_L=0.0, max_iters=4,
                return_fields=False)
    assert a["iters"] == b["iters"] == [4, 4, 4] and a["w1"] == b["w1"]
    eps = 1e-3 if algo == 2 else 1e-5
    free = o.solve(p0, p1, n, L=L, p=2, algo=algo, stop="fpr", eps_L=eps, max_iters=5000, return_fields=False)
    capped = o.solve(p0, p1, n, L=L, p=2, algo=algo, stop="fpr", eps_L=eps,
                     max_iters=[k + 1 for k in free["iters"]], return_fields=False)
    assert capped["iters"] == free["iters"] and capped["w1"] == free["w1"]
    with pytest.raises(ValueError):
        o.solve(p0, p1, n, L=L, p=2, algo=algo, max_iters=[5, 5], return_fields=False)
