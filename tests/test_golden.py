"""The oracle still reproduces the stored residual histories, and the paper's
stated parameters are the solver defaults."""

import json
import os

import numpy as np
import pytest

from tests.golden import make_golden

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("name", sorted(make_golden.CASES))
def test_oracle_matches_stored_history(name):
    stored = np.loadtxt(os.path.join(HERE, name + ".txt"))
    got = make_golden.history(make_golden.CASES[name])
    np.testing.assert_allclose(got, stored, rtol=1e-13, atol=0)


def test_paper_facts_are_the_defaults():
    facts = json.load(open(os.path.join(HERE, "paper_facts.json")))
    import paper_1406_5369_amd as mg

    p = mg.Params(dim=2, n=129)
    assert p.omega == facts["rbgs_omega"]["value"]
    assert (p.nu1, p.nu2) == tuple(facts["pre_post_smoothing"]["value"])
    pj = mg.Params(dim=2, n=129, smoother=mg.SMOOTH_JACOBI)
    assert pj.omega == facts["jacobi_omega"]["value"]
