"""The synthetic C2 cascade takes its concentration ratios from the paper's
species table (Sec. 3.1), stored verbatim in tests/golden/species_table.txt.
"""
import os

import numpy as np

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def table():
    out = {}
    with open(os.path.join(HERE, "golden", "species_table.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                out[k] = float(v)
    return out


def test_c2_ratios_follow_the_species_table():
    t = table()
    k1, inh, k2, pk2, k3, pk3, ph, k1i = W.C2_BASE_M
    assert k1 == t["BRAF"]
    assert k2 == t["MEK"] + t["pMEK"] + t["ppMEK"]
    assert abs(pk3 - (t["pERK"] + t["ppERK"])) < 1e-12
    assert k3 == t["ERK"]
    assert abs(ph - (t["phosphatase1"] + t["phosphatase2"])) < 1e-15
    # inhibitor: geometric middle of the 3-decade dose range below the top dose
    assert abs(inh / (t["dabrafenib_top"] * 10 ** -1.5) - 1) < 1e-3
    total = sum(v for k, v in t.items() if k != "dabrafenib_top")
    assert abs(W.C2_TOP_DOSE_FRACTION - t["dabrafenib_top"] / (t["dabrafenib_top"] + total)) < 1e-12


def test_counts_are_seeded_and_exact():
    a = W.c2_counts(2_000_000, 0)
    assert a == W.c2_counts(2_000_000, 0) and sum(a) == 2_000_000
    assert a[3] == a[4] == a[7] == 0 and min(a[0], a[1], a[6]) > 0
    f = W.C2_TOP_DOSE_FRACTION
    b = W.c2_counts(100_000, 0, inhibitor_fraction=f)
    assert b[1] == round(f * 100_000) and sum(b) == 100_000
    sizes = [m.n_agents for m in W.c4_sweep()]
    assert len(sizes) == 1024 and 20_000 <= min(sizes) and max(sizes) <= 200_000
    assert abs(np.mean(sizes) / ((2e5 - 2e4) / np.log(10)) - 1) < 0.05
