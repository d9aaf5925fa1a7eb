"""The oracle's SQP/ADMM defaults are the values the paper prints
(Section V-A and Table I; fixture tests/golden/paper_parameters.json)."""
import json
import os

from oracle.sqp import SqpParams

HERE = os.path.dirname(__file__)


def test_defaults_are_the_papers_settings():
    with open(os.path.join(HERE, "golden", "paper_parameters.json")) as fh:
        gold = json.load(fh)
    p = SqpParams()
    assert p.mu_merit == gold["sqp_penalty"]
    assert p.tol_primal == gold["sqp_tolerance"]
    # the default ADMM settings are those of the 30- and 57-bus rows of Table I
    row = [r for r in gold["table1_admm"] if r["case_buses"] == 30][0]
    assert (p.rho, p.max_sweeps, p.eps_pri, p.eps_dual) == (row["rho"], row["max_iter"], row["eps"], row["eps"])
