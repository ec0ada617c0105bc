"""Mixed precision on twelve right-hand sides: 48 x 24^3 physical lattice with
C* in three directions (extended 48 x 48 x 24 x 24), rougher links (sigma 0.3),
flavour qhat = -2.  Every solver (FP64 CG; defect-correction CG and FGCR with
FP32 and with bf16-link inner solves) must reach the FP64 true residual 1e-10
on the full lattice; each solution is compared with the FP64 CG one and with
the oracle's own solution at 64 stored sites (tests/golden/
c2_oracle_solutions.txt, written by the committed script beside it, which
calls only the oracle: CG on the Schur system to a residual near 1e-12), and
the oracle recomputes the residual of two solutions per source on sampled
sites."""
import os

import numpy as np
import pytest

import oracle
import synthgen as sg
from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
qxd = pytest.importorskip("paper_1908_11673_amd")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_oracle_solutions.txt")
W2 = sg.WORKLOADS["c2"]
FD = sg.FLAVOURS["d"]
NRHS = 12
SOLVERS = [("dc_cg_f32", "cg", qxd.F32), ("dc_cg_bf16", "cg", qxd.BF16), ("fgcr_f32", "fgcr", qxd.F32),
           ("fgcr_bf16", "fgcr", qxd.BF16)]


def read_oracle_solutions():
    """{rhs: (V_sites, 4, 3) complex} at the stored sites, and the sites."""
    sites, sols, cur = None, {}, None
    for line in open(GOLDEN):
        if line.startswith("#"):
            continue
        if line.startswith("sites "):
            sites = np.array([int(t) for t in line.split()[1:]])
        elif line.startswith("rhs "):
            cur = int(line.split()[1])
            sols[cur] = []
        else:
            v = np.array([float(t) for t in line.split()])
            sols[cur].append((v[0::2] + 1j * v[1::2]).reshape(4, 3))
    return sites, {k: np.array(v) for k, v in sols.items()}


def test_twelve_sources_all_solvers_reach_1e10():
    L, cstar = W2["L"], W2["cstar"]
    o = oracle.Oracle(L, cstar)
    U = sg.gauge_su3(W2["gauge_seed"], W2["sigma_su3"], o.Vphys)
    A = sg.gauge_u1(W2["gauge_seed"], W2["sigma_u1"], o.Vphys)
    o.set_gauge_physical(U, A)
    o.set_flavour(**FD, cache=False, blocks=False)
    lat = qxd.Lattice(L, cstar)
    lat.setup(U, A, FD)
    rng = np.random.default_rng(7)
    gsites, gsol = read_oracle_solutions()
    assert sorted(gsol) == list(range(NRHS))
    gs_dev = torch.from_numpy(gsites).cuda()
    rows = []
    for k in range(NRHS):
        b = sg.spinor(W2["source_seed"] + k, lat.V)
        bd = lat.pack(to_dev(b))
        x64 = lat.field(qxd.F64, full=True)
        st = qxd.qxd_solve_cg(lat.h, qxd.solver_params(res=1e-10, inner_prec=qxd.F64, check_every=8), x64, bd)
        assert st["status"] == 0 and st["true_residual"] <= 1e-10
        row = {"rhs": k, "cg_f64": (st["inner_it"], st["t_ms"])}
        xr = lat.unpack(x64)
        sols = {"cg_f64": xr}
        eo = float(np.linalg.norm(xr[gs_dev].cpu().numpy() - gsol[k]) / np.linalg.norm(gsol[k]))
        assert eo <= 1e-8, ("cg_f64", eo)
        row["cg_f64"] = row["cg_f64"] + (eo,)
        for name, kind, inner in SOLVERS:
            x = lat.field(qxd.F64, full=True)
            prm = qxd.solver_params(res=1e-10, inner_prec=inner, check_every=8)
            if kind == "cg":
                st = qxd.qxd_solve_cg(lat.h, prm, x, bd)
            else:
                st = qxd.qxd_solve_fgcr(lat.h, prm, None, x, bd)
            assert st["status"] == 0 and st["true_residual"] <= 1e-10, (name, st)
            xs = lat.unpack(x)
            err = float(torch.linalg.norm(xs - xr) / torch.linalg.norm(xr))
            assert err <= 1e-6, (name, err)
            eo = float(np.linalg.norm(xs[gs_dev].cpu().numpy() - gsol[k]) / np.linalg.norm(gsol[k]))
            assert eo <= 1e-8, (name, eo)
            row[name] = (st["inner_it"], st["t_ms"], err, eo)
            sols[name] = xs
        # the oracle's residual on 256 sampled sites, for the FP64 CG solution and
        # one mixed-precision solution (alternating)
        sites = rng.choice(o.V, 256, replace=False)
        for name in ("cg_f64", SOLVERS[k % len(SOLVERS)][0]):
            x = sols[name].cpu().numpy()
            dx = o.dirac_sites(x, sites)
            res = np.linalg.norm(b[sites] - dx) / np.linalg.norm(b[sites])
            assert res <= 1e-9, (name, res)
        rows.append(row)
    print("\nrhs  cg_f64(it,ms,err_vs_oracle)  " + "  ".join("%s(it,ms,err_vs_cg64,err_vs_oracle)" % n
                                                          for n, _, _ in SOLVERS))
    for r in rows:
        print("%3d  %4d %7.1f %.1e  " % (r["rhs"], *r["cg_f64"]) +
              "  ".join("%4d %7.1f %.1e %.1e" % r[n] for n, _, _ in SOLVERS))
    lat.close()
