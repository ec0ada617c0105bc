"""The stored oracle solutions of the 48 x 24^3 lattice (tests/golden/
c2_oracle_solutions.txt, written by tests/golden/make_c2_oracle_solutions.py
from the oracle alone) are complete and were accepted by the writer's own
check: twelve sources, 64 sites each (the six lattice corners first), every
full-lattice oracle residual at most 1e-12 (the writer asserts 1e-10)."""
import os

import numpy as np

from tests.test_gpu_c2_rhs import GOLDEN, read_oracle_solutions


def test_stored_oracle_solutions_are_complete():
    assert os.path.exists(GOLDEN)
    sites, sols = read_oracle_solutions()
    assert sites.shape == (64,) and len(set(sites.tolist())) == 64
    assert sites[0] == 0 and sites[1] == 48 * 48 * 24 * 24 - 1
    assert sorted(sols) == list(range(12))
    for k, v in sols.items():
        assert v.shape == (64, 4, 3) and np.all(np.isfinite(v)) and np.abs(v).max() > 0
    res = [float(line.split()[7]) for line in open(GOLDEN) if line.startswith("rhs ")]
    its = [int(line.split()[5]) for line in open(GOLDEN) if line.startswith("rhs ")]
    assert len(res) == 12 and max(res) <= 1e-12
    assert min(its) > 100
