"""What the trained network gains: on the 32 x 16^3 lattice with C* in three
directions (extended 32 x 32 x 16 x 16), a network trained on pairs harvested
from other fields must cut the FGCR steps to the FP64 true residual 1e-10 on
held-out fields, whose solutions the oracle checks."""
import numpy as np
import pytest

import oracle
import synthgen as sg
from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
qxd = pytest.importorskip("paper_1908_11673_amd")
from paper_1908_11673_amd import learned  # noqa: E402

W = sg.WORKLOADS["c3"]
FD = sg.FLAVOURS["d"]


def test_trained_network_cuts_fgcr_steps_on_held_out_fields():
    L, cstar = W["L"], W["cstar"]
    w, skip, info = learned.harvest_and_train(L, cstar, FD, gauge_seeds=list(range(3000, 3008)), sources=8,
                                              pairs_per_source=10, epochs=6, log=print)
    print("harvest/train", info)
    assert info["loss_history"][-1] < info["loss_history"][0]
    lat = qxd.Lattice(L, cstar)
    net = learned.make_network(lat, w, skip)
    vphys = int(np.prod(L))
    for k, gs in enumerate((3100, 3101)):
        U = sg.gauge_su3(gs, W["sigma_su3"], vphys)
        A = sg.gauge_u1(gs, W["sigma_u1"], vphys)
        lat.setup(U, A, FD)
        b = sg.spinor(3600 + k, lat.V)
        bd = lat.pack(to_dev(b))
        x = lat.field(qxd.F64, full=True)
        plain = qxd.qxd_solve_fgcr(lat.h, qxd.solver_params(res=1e-10, inner_prec=qxd.F32), None, x, bd)
        xn = lat.field(qxd.F64, full=True)
        nn = qxd.qxd_solve_fgcr(lat.h, qxd.solver_params(res=1e-10, inner_prec=qxd.F32), net, xn, bd)
        print("field %d: plain %d steps %.1f ms, network %d steps %.1f ms" % (gs, plain["inner_it"], plain["t_ms"],
                                                                              nn["inner_it"], nn["t_ms"]))
        assert nn["fell_back"] == 0 and nn["true_residual"] <= 1e-10
        assert nn["inner_it"] < 0.9 * plain["inner_it"]
        o = oracle.Oracle(L, cstar)
        o.set_gauge_physical(U, A)
        o.set_flavour(**FD, cache=False, blocks=False)
        res = np.linalg.norm(b - o.dirac(lat.unpack(xn).cpu().numpy())) / np.linalg.norm(b)
        assert res <= 1e-10
    qxd.qxd_nn_destroy(net)
    lat.close()
