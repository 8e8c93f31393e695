"""Eq. 1-2 and the quality ratio against every worked value the paper prints
(Tables I, II, IV; Sec. II.C and III.C)."""
import json
import math
import os

import pytest

from paper_2311_09275_amd import ttt

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_ttt_tables.json")))


def close_sf(computed, printed, sf=3):
    """True when `computed` rounds to `printed` at `sf` significant figures."""
    if printed == 0:
        return computed == 0
    unit = 10 ** (math.floor(math.log10(abs(printed))) - (sf - 1))
    return abs(computed - printed) <= 0.5 * unit * 1.0001


def test_repetition_edge_cases():
    assert ttt.repetitions(1.0) == 1.0
    assert math.isinf(ttt.repetitions(0.0))
    assert ttt.repetitions(0.999) == 1.0  # clamped to at least one run
    assert math.isinf(ttt.time_to_target(2.0, 0.0))
    with pytest.raises(ValueError):
        ttt.repetitions(1.5)


@pytest.mark.parametrize("row", GOLD["table1_speedup"]["rows"], ids=lambda r: r["inst"])
def test_table1(row):
    best = GOLD["best_known"][row["inst"]]
    assert close_sf(ttt.sweeps_to_target(row["sweeps_per_run"], row["ps"]), row["sweeps_to_target"])
    assert close_sf(row["sbm_ttt_s"] / row["ttt_s"], row["speedup"])
    assert abs(100 * ttt.quality(row["sbm_cut"], best) - row["quality_pct"]) <= 0.005 + 1e-9


@pytest.mark.parametrize("row", GOLD["table2_best"]["rows"], ids=lambda r: r["inst"])
def test_table2(row):
    assert close_sf(ttt.sweeps_to_target(row["sweeps_per_run_e6"], row["ps"]), row["sweeps_to_target_e6"])


@pytest.mark.parametrize("row", GOLD["table4_bls"]["rows"], ids=lambda r: r["inst"])
def test_table4(row):
    best = GOLD["best_known"][row["inst"]]
    per_run = row["avg_time_s"] * row["ps"]           # footnote 4
    assert abs(per_run - row["time_per_run_s"]) < 1e-6
    proj = ttt.time_to_target(per_run, row["ps"])
    assert abs(proj - row["projected_ttt_s"]) <= 0.5 + 1e-6   # printed to the second
    # the printed speedup divides the printed (rounded) projection
    assert close_sf(row["projected_ttt_s"] / row["cosm_s"], row["speedup"])
    assert abs(100 * ttt.quality(row["bls_cut"], best) - row["quality_pct"]) <= 0.005 + 1e-9


@pytest.mark.parametrize("row", GOLD["ges_estimates"]["rows"], ids=lambda r: r["target"])
def test_ges(row):
    tt = ttt.time_to_target(row["t_trial_s"], row["ps"])
    assert close_sf(tt / 3600.0, row["ttt_h"], sf=2)
    assert close_sf(tt / row["cosm_s"], row["speedup"], sf=3)


def test_digital_annealer():
    d = GOLD["digital_annealer"]
    assert close_sf(d["ttt_h"] * 3600 / d["cosm_s"], d["speedup"])
    assert abs(100 * ttt.quality(d["cut"], GOLD["best_known"]["G65"]) - d["quality_pct"]) <= 0.005


def test_replica_ttt():
    out = ttt.replica_ttt([10, 12, 12, 9], target=12, wall_s=2.0, sweeps=100)
    assert out["ps"] == 0.5
    assert out["t_trial_s"] == 0.5
    assert abs(out["ttt_s"] - 0.5 * math.log(0.01) / math.log(0.5)) < 1e-12
