"""The paper's printed constants (Table 1, Sec. 8) against the defaults."""
import json
import os

from gen.scenes import SolverParams, scene_c2

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1.json")


def test_solver_defaults_follow_table1():
    g = json.load(open(GOLD))
    p = SolverParams()
    assert p.node_sigma == g["node_sigma_m"]
    assert p.lambda_reg == g["lambda_reg"]
    assert p.gn_iters <= g["max_gn_iters"]
