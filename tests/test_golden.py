"""The stored fixture of the tiny configuration (tests/golden/c1_tiny.json,
written by tests/golden/make_golden.py from the oracle alone) still matches
the oracle: a regression check on the oracle, and the reference the GPU test
of the same configuration reads."""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def test_tiny_configuration_fixture_matches_oracle():
    from tests.golden import make_golden
    stored = json.load(open(os.path.join(HERE, "golden", "c1_tiny.json")))
    now = make_golden.compute()
    assert now["cg_iters"] == stored["cg_iters"]
    for k in ("mat_pc_sym_norm2", "solution_norm2"):
        assert abs(now[k] - stored[k]) <= 1e-12 * abs(stored[k])
    for k in ("mat_pc_sym_sites", "solution_sites"):
        for site, v in stored[k].items():
            assert np.allclose(np.array(now[k][site]), np.array(v), rtol=0, atol=1e-12)
    assert stored["full_residual"] < 1e-9
