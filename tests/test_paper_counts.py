"""The simulation counts printed in the paper's Tables 1 and 2 follow from the
particle and iteration counts in its text when one "simulation" is one
particle's forward + adjoint pass over all its data (the unit in which the
throughput of this library is reported: particle-gradients per second)."""
import json
import os

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")


def _load():
    with open(GOLDEN) as f:
        return json.load(f)


def test_fwi_counts():
    c = _load()["fwi"]
    assert c["svgd"]["particles"] * c["svgd"]["iterations"] == c["svgd"]["table_simulations"]
    s = c["ssvgd"]
    assert s["particles"] * (s["iterations"] + s["burn_in"]) == s["table_simulations"]
    assert s["particles"] * s["iterations"] // s["thin"] == s["samples"]


def test_tomography_counts():
    c = _load()["tomography"]
    f = 1.0 + c["gradient_cost_in_forward_simulations"]
    assert c["svgd"]["particles"] * c["svgd"]["iterations"] == c["svgd"]["table_simulations"]
    s = c["ssvgd"]
    assert s["particles"] * (s["iterations"] + s["burn_in"]) == s["table_simulations"]
    assert s["particles"] * s["iterations"] // s["thin"] == s["samples"]
    for k in ("svgd", "ssvgd", "advi"):
        assert round(c[k]["table_simulations"] * f) == c[k]["table_comparable"]


def test_paper_throughput_context():
    # derived context figure: 120,000 sSVGD simulations in 49 h on 40 cores
    w = _load()["fwi"]
    rate = w["ssvgd"]["table_simulations"] / (w["wall_hours"]["ssvgd"] * 3600.0)
    assert abs(rate - 0.680) < 1e-3
