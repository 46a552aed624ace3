"""The parameter tables of the paper (tests/golden/paper_parameters.json,
transcribed from Table II, Sec. IV-B-2 and Table III) are what the workload
definitions hand to both the oracle and the GPU path."""
import json
import os

import pytest

from synth import configs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))


def _check(p, ref):
    for k, v in ref.items():
        if k.startswith("_"):
            continue
        assert p[k] == pytest.approx(v, rel=1e-12), k


@pytest.mark.parametrize("M,key", [(12, "12"), (24, "24"), (4, "12"), (28, "24")])
@pytest.mark.parametrize("level,counts", [("high", 5e6), ("low", 1e5)])
def test_table2_rows(M, key, level, counts):
    c = GOLD["common_2d"]
    for mode, row in (("BSREM", "BSREM"), ("P1", "P1_"), ("P2", "P2_")):
        p = configs.params_2d(M, counts, mode=mode)
        _check(p, GOLD["table2"][row + key if mode != "BSREM" else row + key][level])
        assert p["beta"] == (c["beta_high"] if level == "high" else c["beta_low"])
        for k in ("t_clip", "eps", "gamma_R", "lambda0", "J0", "J1"):
            assert p[k] == c[k]
        if mode == "P2":
            assert p["delta2"] == p["delta1"]           # delta1 = delta2 in the simulations


@pytest.mark.parametrize("M,key", [(12, "12"), (24, "24")])
def test_momentum_rows(M, key):
    m = GOLD["momentum_2d"]
    _check(configs.params_2d(M, 5e6, mode="M1"), m["M1_" + key])
    _check(configs.params_2d(M, 5e6, mode="M2"), m["M2_" + key])


def test_table3_row():
    _check(configs.params_3d(), GOLD["table3_P2_nonTOF"])


@pytest.mark.parametrize("mode,row", [("BSREM", "BSREM24"), ("P1", "P1_24"), ("P2", "P2_24")])
def test_uniform_phantom_rows(mode, row):
    p = configs.params_2d_uniform(mode)
    _check(p, GOLD["table2_uniform"][row]["high"])
    assert p["beta"] == GOLD["common_2d"]["beta_high"]
    if mode == "P2":
        assert p["delta2"] == p["delta1"]


def test_simulation_constants():
    s = GOLD["simulation_2d"]
    assert (configs.TC_HIGH, configs.TC_LOW, configs.SF, configs.RF) == (s["TC_high"], s["TC_low"], s["SF"], s["RF"])
