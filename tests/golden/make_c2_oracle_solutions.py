"""Write tests/golden/c2_oracle_solutions.txt: the FP64 oracle's solutions of
D x = b on the 48 x 24^3 lattice with C* in three directions (extended
48 x 48 x 24 x 24, sigma 0.3 / 0.3, gauge seed 2), flavour qhat = -2, for the
twelve Gaussian sources of seeds 2000..2011, at 64 fixed sites.

Each solution is the oracle's even-odd reduction (source b_hat = b_e - D_eo
D_oo^-1 b_o), its conjugate-gradient solve of the Schur system to an absolute
normal-residual bound 1e-12 |b_hat|, and its reconstruction of the odd sites;
the full-lattice residual |b - D x| / |b| is recomputed with the oracle's D and
written beside each source.  Calls only the oracle and the input generator.
Run from the repository root: python tests/golden/make_c2_oracle_solutions.py
(about 5 minutes per source on 8 cores)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synthgen as sg  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_oracle_solutions.txt")
NRHS = 12
NSITES = 64


def sample_sites(o):
    """Six lattice corners (where every C* crossing happens) and 58 random sites."""
    corners = o.site(np.array([[0, 0, 0, 0], [o.Le[0] - 1, o.Le[1] - 1, o.Le[2] - 1, o.Le[3] - 1],
                               [0, o.L[1], 0, 0], [0, o.L[1] - 1, o.Le[2] - 1, 0],
                               [o.Le[0] - 1, 0, 0, o.Le[3] - 1], [1, o.Le[1] - 1, 1, 1]]))
    rest = np.random.default_rng(11).choice(np.setdiff1d(np.arange(o.V), corners), NSITES - len(corners),
                                            replace=False)
    return np.concatenate([corners, rest])


def main():
    w = sg.WORKLOADS["c2"]
    o = oracle.Oracle(w["L"], w["cstar"])
    o.set_gauge_physical(sg.gauge_su3(w["gauge_seed"], w["sigma_su3"], o.Vphys),
                         sg.gauge_u1(w["gauge_seed"], w["sigma_u1"], o.Vphys))
    o.set_flavour(**sg.FLAVOURS["d"])
    sites = sample_sites(o)
    lines = ["# oracle solutions of D x = b, 48 x 24^3 physical, C* 3, sigma 0.3/0.3, gauge seed 2, qhat -2",
             "# kappa 0.136377, su3csw 1.90952, u1csw 1; source seeds 2000..2011 (Gaussian, every extended site)",
             "# written by tests/golden/make_c2_oracle_solutions.py (oracle CG on the Schur system)",
             "sites " + " ".join(str(int(s)) for s in sites)]
    for k in range(NRHS):
        t0 = time.time()
        seed = w["source_seed"] + k
        b = sg.spinor(seed, o.V)
        bhat = o.eo_source(b)
        xe, it, _ = o.cg(bhat, 1e-12 * np.linalg.norm(bhat))
        assert it >= 0, "oracle CG did not converge"
        x = o.eo_reconstruct(xe, b)
        res = np.linalg.norm(b - o.dirac(x)) / np.linalg.norm(b)
        assert res <= 1e-10, res
        lines.append("rhs %d seed %d iterations %d residual %.3e" % (k, seed, it, res))
        for s in sites:
            v = x[s].reshape(12)
            lines.append(" ".join("%.17e %.17e" % (c.real, c.imag) for c in v))
        print("rhs %d: %d iterations, residual %.2e, %.0f s" % (k, it, res, time.time() - t0), flush=True)
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
