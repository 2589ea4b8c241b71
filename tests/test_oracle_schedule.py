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
