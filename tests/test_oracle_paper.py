"""Pins of the oracle against numbers the paper prints for its own test
problem (Sec. 4), beyond Table 1 (test_oracle_system)."""
import os

import numpy as np
import pytest

from oracle import system
from paper_1901_00654_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table3_condition.txt")


def _golden():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    return {(int(r[0]), int(r[1])): float(r[2]) for r in rows}


def test_table3_condition_number_of_A():
    """Table 3: kappa(A) = 1933.27 at P = 2, G = 5. It depends on the knot
    convention, the penalty (Frobenius norm of the Hessian), the integration
    domain and the basis normalisation all at once; a plausible slip in any
    of them (clamped knots, the squared-sum penalty, a missing factor 2 on
    the mixed terms) moves it far more than the 0.5 % allowed here."""
    ref = _golden()[(2, 5)]
    w = workloads.paper_sigmoid(2, N=32, lam=0.2)
    A, _, _, _ = system.system(w["x"], w["y"], w["lo"], w["hi"], w["N"], w["lam"])
    ev = np.linalg.eigvalsh(A.toarray())
    kappa = ev[-1] / ev[0]
    assert abs(kappa - ref) <= 5e-3 * ref, kappa


@pytest.mark.parametrize("lam", [0.1, 1.0])
def test_condition_number_plateau(lam):
    """kappa(A) stays within 1 % of the Table 3 value for lambda in [0.1, 1]."""
    ref = _golden()[(2, 5)]
    w = workloads.paper_sigmoid(2, N=32, lam=lam, seed=12)
    A, _, _, _ = system.system(w["x"], w["y"], w["lo"], w["hi"], w["N"], w["lam"])
    ev = np.linalg.eigvalsh(A.toarray())
    assert abs(ev[-1] / ev[0] - ref) <= 1e-2 * ref
