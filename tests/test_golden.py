"""The oracle reproduces its committed golden fixtures (written by
tests/golden/make_golden.py from the oracle and the input generator)."""
import json
import os

import numpy as np

import tests.golden.make_golden as mg

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _check(name, fresh):
    stored = json.load(open(os.path.join(HERE, name)))
    for k in ("seeds", "steps", "code", "out_dest"):
        if k in stored:
            np.testing.assert_array_equal(np.array(fresh[k]), np.array(stored[k]))
    np.testing.assert_allclose(np.array(fresh["final_pos"]), np.array(stored["final_pos"]), rtol=0, atol=1e-12)


def test_abc_golden():
    _check("abc32.json", mg.abc_case())


def test_turbulence_golden():
    _check("turb24.json", mg.turb_case())
