"""What the trained network gains, on the 32 x 16^3 lattice with C* in three
directions (extended 32 x 32 x 16 x 16), for both flavours.  A network trained
on 100 pairs per field harvested from 8 fields (seeds 3000-3007) is evaluated on
held-out fields (3100, 3101) by FGCR steps and wall time to the FP64 true
residual 1e-10, beside plain FP32-inner FGCR and FP64 CG; one network solution
per flavour is checked by the oracle's D.  The network also goes through
qxd_nn_save / qxd_nn_load unchanged.

The network is not gauge equivariant: on a held-out field under a random gauge
transformation, plain FGCR takes the same steps and returns the rotated
solution (the operator is covariant), while the network-preconditioned solve
must still reach 1e-10 (its gain is reported, not asserted).

Asserted gains are the measured ones: for the down-type flavour the network
cuts FGCR steps by at least 10 % (measured 88 -> 64 and 87 -> 63); the up-type
flavour converges in about 50 plain steps at this volume and the network gains
no steps there (50 -> 51, 48 -> 48).  In wall time the network-preconditioned
solve is slower than plain FGCR for both flavours (25.6 against 20.0 ms and
20.2 against 11.2 ms): one application of the three convolutions costs more
than the D_hat applications and vector work of the steps it saves, so the times
are printed and bounded only from above.  On the gauge-rotated field the
down-type gain turns into a loss (102 network steps against 88 plain)."""
import numpy as np
import pytest

import oracle
import synthgen as sg
from tests.gpu_common import gauge_rotate, rotate_spinor, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
qxd = pytest.importorskip("paper_1908_11673_amd")
from paper_1908_11673_amd import learned  # noqa: E402

W = sg.WORKLOADS["c3"]
HELD_OUT = (3100, 3101)


def _solves(lat, net, bd):
    prm = qxd.solver_params(res=1e-10, inner_prec=qxd.F32)
    out = {}
    for tag, fn in (("plain", lambda x: qxd.qxd_solve_fgcr(lat.h, prm, None, x, bd)),
                    ("network", lambda x: qxd.qxd_solve_fgcr(lat.h, prm, net, x, bd)),
                    ("cg_f64", lambda x: qxd.qxd_solve_cg(lat.h, qxd.solver_params(res=1e-10), x, bd))):
        x = lat.field(qxd.F64, full=True)
        fn(x)  # warm-up: the first call of a solver allocates its workspace
        x = lat.field(qxd.F64, full=True)
        st = fn(x)
        assert st["status"] == 0 and st["true_residual"] <= 1e-10, (tag, st)
        out[tag] = (st, x)
    return out


@pytest.mark.parametrize("flav_name", ["d", "u"])
def test_trained_network_on_held_out_and_gauge_rotated_fields(flav_name, tmp_path):
    flav = sg.FLAVOURS[flav_name]
    L, cstar = W["L"], W["cstar"]
    w, skip, info = learned.harvest_and_train(L, cstar, flav, gauge_seeds=list(range(3000, 3008)),
                                              pairs_per_field=100, epochs=6, sigma_su3=W["sigma_su3"],
                                              sigma_u1=W["sigma_u1"])
    print("qhat %d: %d pairs, loss %.4f -> %.4f, harvest %.1f s, train %.1f s" % (
        flav["qhat"], info["pairs"], info["loss_history"][0], info["loss_history"][-1], info["harvest_s"],
        info["train_s"]))
    assert info["loss_history"][-1] < info["loss_history"][0]
    lat = qxd.Lattice(L, cstar)
    net0 = learned.make_network(lat, w, skip)
    learned.save_network(str(tmp_path / "net"), net0, {"qhat": flav["qhat"], "pairs": info["pairs"]})
    net, meta = learned.load_network(lat, str(tmp_path / "net"))
    assert meta["pairs"] == info["pairs"]
    assert np.array_equal(qxd.qxd_nn_get_weights(net), qxd.qxd_nn_get_weights(net0))
    qxd.qxd_nn_destroy(net0)
    vphys = int(np.prod(L))
    o = oracle.Oracle(L, cstar)
    for k, gs in enumerate(HELD_OUT):
        U = sg.gauge_su3(gs, W["sigma_su3"], vphys)
        A = sg.gauge_u1(gs, W["sigma_u1"], vphys)
        lat.setup(U, A, flav)
        b = sg.spinor(3600 + k, lat.V)
        r = _solves(lat, net, lat.pack(to_dev(b)))
        (sp, xp), (sn, xn), (sc, _) = r["plain"], r["network"], r["cg_f64"]
        print("qhat %d field %d: plain FGCR %d steps %.1f ms | network FGCR %d steps %.1f ms | FP64 CG %d it %.1f ms"
              % (flav["qhat"], gs, sp["inner_it"], sp["t_ms"], sn["inner_it"], sn["t_ms"], sc["inner_it"],
                 sc["t_ms"]))
        assert sn["fell_back"] == 0
        if flav_name == "d":
            assert sn["inner_it"] < 0.9 * sp["inner_it"]
        # time: never worse than three times plain FGCR (measured about 1.3x)
        assert sn["t_ms"] < 3.0 * sp["t_ms"]
        if k == 0:
            o.set_gauge_physical(U, A)
            o.set_flavour(**flav, cache=False, blocks=False)
            res = np.linalg.norm(b - o.dirac(lat.unpack(xn).cpu().numpy())) / np.linalg.norm(b)
            assert res <= 1e-10
            # the same field and source under a random gauge transformation
            U2, A2, g = gauge_rotate(o, U, A, flav["qhat"], 77)
            lat.setup(U2, A2, flav)
            b2 = rotate_spinor(g, b)
            r2 = _solves(lat, net, lat.pack(to_dev(b2)))
            (sp2, xp2), (sn2, _), _ = r2["plain"], r2["network"], r2["cg_f64"]
            want = rotate_spinor(g, lat.unpack(xp).cpu().numpy())
            dx = np.linalg.norm(lat.unpack(xp2).cpu().numpy() - want) / np.linalg.norm(want)
            print("qhat %d field %d gauge-rotated: plain FGCR %d steps (|x' - g x| / |x| = %.1e), network FGCR %d "
                  "steps %.1f ms (fell back: %d)" % (flav["qhat"], gs, sp2["inner_it"], dx, sn2["inner_it"],
                                                      sn2["t_ms"], sn2["fell_back"]))
            assert abs(sp2["inner_it"] - sp["inner_it"]) <= 2
            assert dx < 1e-8
    qxd.qxd_nn_destroy(net)
    lat.close()


def test_network_file_errors(tmp_path):
    lat = qxd.Lattice((4, 2, 4, 4), 3)
    net = qxd.qxd_nn_create(lat.h)
    w = learned.initial_weights(3)
    qxd.qxd_nn_set_weights(net, w)
    qxd.qxd_nn_set_skip(net, 0.25)
    path = tmp_path / "a.qxdnn"
    qxd.qxd_nn_save(net, str(path))
    other = qxd.qxd_nn_create(lat.h)
    qxd.qxd_nn_load(other, str(path))
    assert np.array_equal(qxd.qxd_nn_get_weights(other), w)
    raw = bytearray(path.read_bytes())
    for name, data in (("flipped weight bit", raw[:40] + bytes([raw[40] ^ 1]) + raw[41:]),
                       ("bad tag", b"X" + raw[1:]), ("truncated", raw[:-4]), ("trailing byte", raw + b"\0")):
        bad = tmp_path / "bad.qxdnn"
        bad.write_bytes(bytes(data))
        with pytest.raises(qxd.QxdError) as e:
            qxd.qxd_nn_load(other, str(bad))
        assert e.value.code == 10, name
    with pytest.raises(qxd.QxdError) as e:
        qxd.qxd_nn_load(other, str(tmp_path / "missing.qxdnn"))
    assert e.value.code == 10
    qxd.qxd_nn_destroy(other)
    qxd.qxd_nn_destroy(net)
    lat.close()
