"""The defaults the paper states (tests/golden/paper_defaults.json, each entry
with its citation) are the defaults of the library and of the oracle."""
import inspect
import json
import os

import pytest

from oracle import densify as OD
from oracle import schedule as OS
from paper_2503_18402_amd import gsmi, train

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_defaults.json")))


def _default(fn, name):
    return inspect.signature(fn).parameters[name].default


def test_resolution_schedule_a():
    a = G["a"]["value"]
    assert _default(train.ResolutionSchedule.__init__, "a") == a
    assert _default(train.Trainer.__init__, "a") == a
    assert _default(gsmi.gs_resolution_schedule, "a") == a
    assert _default(OS.schedule_knots, "a") == a


def test_budget_gamma_eta_and_initial_budget():
    g, e = G["gamma"]["value"], G["eta"]["value"]
    assert train.DensifyConfig().gamma == g and train.DensifyConfig().eta == e
    assert _default(OD.budget_update, "gamma") == g and _default(OD.budget_update, "eta") == e
    assert train.P_FIN_INIT_FACTOR == G["p_fin_init_factor"]["value"]


def test_eq8_factor_at_the_defaults():
    g, e = G["gamma"]["value"], G["eta"]["value"]
    assert e / (1.0 - g) == pytest.approx(G["eq8_steady_state_factor"]["value"], rel=1e-12)
    p = 0.0
    for _ in range(5000):
        p = OD.budget_update(p, 1.0)
    assert p == pytest.approx(G["eq8_steady_state_factor"]["value"], rel=1e-9)
