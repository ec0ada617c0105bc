"""Benchmark of the Wilson-clover / C* hot path on one MI355X.

Workload (default): the 32^3 x 64 lattice with C* in three directions, i.e. the
doubled 64 x 64 x 32 x 32 extended lattice (t, x1, x2, x3), two flavours
(qhat = -2, kappa = 0.136377; qhat = 4, kappa = 0.137312; su3csw 1.90952,
u1csw 1), seeded synthetic SU(3) x U(1) fields (exp of Gaussian traceless
anti-Hermitian matrices, sigma 0.2; U(1) angles sigma 0.3).

One step applies the even-odd Schur operator D_hat once per flavour in FP64
and once in FP32, on in/out buffers rotated over four pairs (so no operand
stays in the 256 MB last-level cache between applications).  `value` is the
algorithmic bytes of all those applications divided by the timed wall time.
Algorithmic bytes of one D_hat application: 552 reals per even site (links read
once per pass: 288; clover blocks H_e and H_o^-1: 144; spinors: 120).

Extra legs (not part of `value`): the time to a true FP64 residual 1e-10 of FP64
CG against mixed-precision FGCR (and, when a trained network is available,
network-preconditioned FGCR) on the same lattice; FP64 shifted normal solves
(the paper's rational operator by multi-shift CG, twisted-mass systems solved
together and one by one); inexactly deflated SAP-FGCR against SAP-FGCR, with
matched and swapped-charge subspaces; and the FP64 CPU oracle timed on a
bounded sample of even sites of the same lattice (`cpu_baseline`).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dw GB/s & %HBM roofline; time-to-1e-10 residual, mixed+learned vs FP64 CG"
HBM_PEAK_GBS = 8000.0
REALS_PER_VE = 552


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def make_fields(w):
    import synthgen as sg
    L = w["L"]
    vphys = L[0] * L[1] * L[2] * L[3]
    U = sg.gauge_su3(w["gauge_seed"], w["sigma_su3"], vphys)
    A = sg.gauge_u1(w["gauge_seed"], w["sigma_u1"], vphys)
    return U, A


def cpu_baseline(w, U, A, flav, seconds=15.0):
    """Oracle D_hat on a bounded sample of even sites of the same lattice."""
    import oracle
    import synthgen as sg
    o = oracle.Oracle(w["L"], w["cstar"])
    o.set_gauge_physical(U, A)
    o.set_flavour(**flav, cache=False, blocks=False)
    psi = sg.spinor(w["source_seed"], o.V)
    par = o.parity()
    psi[par == 1] = 0
    even = np.nonzero(par == 0)[0]
    rng = np.random.default_rng(0)
    n = 64
    done, t_tot = 0, 0.0
    while t_tot < seconds:
        sites = rng.choice(even, size=n, replace=False)
        t0 = time.perf_counter()
        o.schur_sites(psi, sites)
        t_tot += time.perf_counter() - t0
        done += n
        n = min(2 * n, 4096)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    gbs = done * REALS_PER_VE * 8 / t_tot / 1e9
    return {"value": gbs, "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": "%d random even sites of the same lattice (FP64 D_hat, oracle as is), %.1f s" % (done, t_tot)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--nn-fields", type=int, default=10, help="fields for the network training (0: no network)")
    ap.add_argument("--nn-epochs", type=int, default=8)
    ap.add_argument("--legs", default="", help="comma-separated solve legs to run (default: all)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on one GPU (a multi-GPU path with time-slab "
              "halo exchange over xGMI is designed, not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1908_11673_amd as qxd
    import synthgen as sg

    w = sg.WORKLOADS[args.workload]
    # the 128 x 64^3 lattice (175 GB of links and clover per flavour) runs one
    # flavour, one buffer pair, and releases the gauge copy after set-up
    big = args.workload == "c4"
    flavours = [sg.FLAVOURS["d"]] if big else [sg.FLAVOURS["d"], sg.FLAVOURS["u"]]
    log("generating %s fields %s" % (args.workload, w["L"]))
    U, A = make_fields(w)
    lats = []
    for f in flavours:
        lat = qxd.Lattice(w["L"], w["cstar"])
        st = lat.setup(U, A, f)
        log("flavour qhat=%d: clover min pivot %.4f" % (f["qhat"], st["min_pivot"]))
        if big:
            qxd.qxd_trim(lat.h)
        lats.append(lat)
    Ve = lats[0].Ve
    torch.cuda.synchronize()

    nbuf = 1 if big else 4
    psi = sg.spinor(w["source_seed"], lats[0].V)
    src64 = lats[0].pack(torch.from_numpy(psi).cuda())
    src32 = lats[0].pack(torch.from_numpy(psi).cuda(), qxd.F32)
    ins = {qxd.F64: [], qxd.F32: []}
    outs = {qxd.F64: [], qxd.F32: []}
    for i in range(nbuf):
        for p, src in ((qxd.F64, src64), (qxd.F32, src32)):
            t = qxd.field(Ve, p)
            t.copy_(src[:12 * Ve] * (1.0 + 0.01 * i))
            ins[p].append(t)
            outs[p].append(qxd.field(Ve, p))
    del psi, src64, src32

    stream = torch.cuda.current_stream()
    sptr = stream.cuda_stream

    def step(i):
        for lat in lats:
            for p in (qxd.F64, qxd.F32):
                qxd.qxd_dw_eo_schur(lat.h, p, 0, outs[p][i % nbuf], ins[p][i % nbuf], sptr)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for i in range(args.steps):
        step(i)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    bytes_step = len(lats) * (REALS_PER_VE * 8 + REALS_PER_VE * 4) * Ve
    value = bytes_step / (ms_step * 1e-3) / 1e9
    log("timed %d steps: %.3f ms/step (wall %.3f s)" % (args.steps, ms_step, wall))

    # dominant kernel: FP64 D_hat (two launches: odd-site pass and even-site pass), timed alone
    n64 = 50
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(n64):
        qxd.qxd_dw_eo_schur(lats[0].h, qxd.F64, 0, outs[qxd.F64][i % nbuf], ins[qxd.F64][i % nbuf], sptr)
    e1.record(stream)
    torch.cuda.synchronize()
    ms64 = e0.elapsed_time(e1) / n64
    n32 = 100
    e0.record(stream)
    for i in range(n32):
        qxd.qxd_dw_eo_schur(lats[0].h, qxd.F32, 0, outs[qxd.F32][i % nbuf], ins[qxd.F32][i % nbuf], sptr)
    e1.record(stream)
    torch.cuda.synchronize()
    ms32 = e0.elapsed_time(e1) / n32
    ach64 = REALS_PER_VE * 8 * Ve / (ms64 * 1e-3) / 1e9
    ach32 = REALS_PER_VE * 4 * Ve / (ms32 * 1e-3) / 1e9
    log("D_hat FP64 %.3f ms (%.0f GB/s), FP32 %.3f ms (%.0f GB/s)" % (ms64, ach64, ms32, ach32))

    copy_gbs = copy_calibration(torch)
    log("plain copy of 1.5 GiB (not cache resident): %.0f GB/s read+write" % copy_gbs)

    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "D_hat applies, %dx%d^3 physical with C* in %d directions (extended %dx%dx%dx%d), "
                               "%d flavour%s x {FP64, FP32} per step" % (
                                   w["L"][0], w["L"][1], w["cstar"], w["L"][0], 2 * w["L"][1], w["L"][2], w["L"][3],
                                   len(flavours), "s" if len(flavours) > 1 else ""),
                   "extended_lattice": [w["L"][0], 2 * w["L"][1], w["L"][2], w["L"][3]],
                   "even_sites": Ve, "flavours": [{"qhat": f["qhat"], "kappa": f["kappa"]} for f in flavours],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(ach64, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach64 / HBM_PEAK_GBS, 4),
                     "traffic": recorded_traffic("dhat_f64") if args.workload == "c1" else None,
                     "kernel": "D_hat FP64 (k_schur1 + k_schur2)", "ms_per_launch": round(ms64, 4)},
        "dhat_fp32": {"ms": round(ms32, 4), "achieved_gbs": round(ach32, 1), "frac": round(ach32 / HBM_PEAK_GBS, 4)},
        "copy_kernel_gbs": round(copy_gbs, 1),
    }

    if not args.no_solve:
        del ins, outs
        torch.cuda.empty_cache()
        only = tuple(t for t in args.legs.split(",") if t)
        train = not only or "fgcr_f32_nn_in_f64" in only
        result["time_to_solution"] = solve_leg(qxd, torch, lats, w, flavours, args.nn_fields if train else 0,
                                               args.nn_epochs, big, only)
        if not big and (not only or "shifted" in only):
            result["shifted_solves"] = shifted_leg(qxd, torch, lats, w, flavours)
        if not big and (not only or "deflation" in only):
            result["deflation"] = deflation_leg(qxd, torch, lats, w, flavours, U, A)

    if not args.no_cpu_baseline and not big:  # the oracle would hold 60 GB of host fields at 128 x 64^3
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(w, U, A, flavours[0], args.cpu_seconds)
    print(json.dumps(result), flush=True)
    for lat in lats:
        lat.close()


TRAFFIC_SOURCES = ("paper_1908_11673_amd/csrc/dirac.hip", "paper_1908_11673_amd/csrc/wilson_site.hpp",
                   "paper_1908_11673_amd/csrc/qxd_internal.hpp",
                   "paper_1908_11673_amd/build.py")


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration), or None
    when the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "dhat_schur_c1.md")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    for line in open(path):
        if line.startswith("traffic-record:"):
            kv = dict(item.split("=", 1) for item in line.split()[1:])
            if kv.get("kernel") == kernel and kv.get("sources_sha256") == h.hexdigest():
                return int(kv["bytes_per_launch"])
    return None


def copy_calibration(torch):
    """Device-to-device copy of 1.5 GiB whose source was evicted from the
    last-level cache first: the reference for the measured bandwidth and for
    scaling the HBM byte counters."""
    n = 3 * (1 << 29) // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    flush = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    flush.fill_(2.0)
    del flush
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del a, b
    return 2 * n * 8 / (ms * 1e-3) / 1e9


# SAP in the solve leg: plain minimal-residual block solves, two cycles of 8
# steps, the fastest of a sweep at 64 x 32^3.  The even-odd preconditioned block
# solver (the paper's) needs fewer FGCR steps but costs twice as much per step
# here (half the wavefronts wait in each of its two hop exchanges): 153 ms
# against 128 ms at its best setting.  The paper's own setting (5 cycles, 5
# even-odd minimal-residual steps per block) is timed as a leg of its own.
SAP_NCY, SAP_NMR, SAP_PLAIN = 2, 8, 1


def read_rational(path=os.path.join(ROOT, "tests", "golden", "rational0.txt")):
    """The [Rational 0] approximation printed in the paper's sample input file."""
    t = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        key, *vals = line.split()
        t[key] = [float(v) for v in vals]
    return t["A"][0], t["nu"], t["mus"], t["delta"][0]


TM_MU = (0.003, 0.01, 0.03, 0.1)  # twisted masses of the shifted-solve leg


def shifted_leg(qxd, torch, lats, w, flavours):
    """FP64 shifted normal solves on the benchmark lattice, one Gaussian source
    per flavour: the rational operator R of the paper's [Rational 0]
    approximation (ten poles, one multi-shift solve to 1e-11), and the
    twisted-mass systems (D_hat^+ D_hat + mu^2) for the masses TM_MU solved
    together by multi-shift CG against one after another."""
    import synthgen as sg
    A, nu, mu, delta = read_rational()
    out = {}
    b = sg.spinor(w["source_seed"] + 2, lats[0].V)
    for lat, name in zip(lats, ("qhat-2", "qhat+4")):
        res = {}
        phi = lat.pack(torch.from_numpy(b).cuda())[:12 * lat.Ve].clone()
        torch.cuda.empty_cache()
        y = lat.field(qxd.F64)

        def timed(fn):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) * 1e3, st

        ms, st = timed(lambda: qxd.qxd_rational_apply(lat.h, qxd.solver_params(res=1e-11, check_every=8), A, nu, mu,
                                                      y, phi, check=False))
        res["rational_r0"] = {"ms": round(ms, 2), "status": st["status"], "iterations": st["inner_it"],
                              "poles": len(mu), "schur_applies": st["schur_applies"],
                              "recurrence_residual": st["true_residual"], "delta": delta}
        log("%s rational operator (%d poles): %.1f ms, %d iterations" % (name, len(mu), ms, st["inner_it"]))
        prm = qxd.solver_params(res=1e-10, check_every=8)
        xs = [lat.field(qxd.F64) for _ in TM_MU]
        ms_all, st = timed(lambda: qxd.qxd_solve_mscg(lat.h, prm, [m * m for m in TM_MU], xs, phi, check=False))
        res["tm_multishift"] = {"ms": round(ms_all, 2), "status": st["status"], "iterations": st["inner_it"],
                                "true_residual": st["true_residual"], "mu": list(TM_MU)}
        ms_sep, its = 0.0, 0
        for m, x in zip(TM_MU, xs):
            ms1, st = timed(lambda: qxd.qxd_solve_mscg(lat.h, prm, [m * m], [x], phi, check=False))
            ms_sep += ms1
            its += st["inner_it"]
        res["tm_one_by_one"] = {"ms": round(ms_sep, 2), "iterations": its}
        log("%s twisted-mass solves, mu %s: together %.1f ms, one by one %.1f ms" % (name, TM_MU, ms_all, ms_sep))
        del xs, y
        out[name] = res
    return out


DFL_NS, DFL_NIT, DFL_NC = 16, 10, 16  # subspace size, inverse-iteration rounds (4 SAP cycles of 4 steps), coarse steps
LIGHT_KAPPA = 0.1405  # a lighter down-type quark for the deflation leg


def deflation_leg(qxd, torch, lats, w, flavours, U, A):
    """Inexactly deflated SAP-FGCR (DFL+SAP, FP32 inner, FP64 true residual 1e-10)
    against SAP-FGCR with the same SAP settings: per flavour a subspace of
    DFL_NS vectors from DFL_NIT rounds of SAP inverse iteration on seeded
    Gaussian start vectors; then each physical flavour solved with the other
    charge's subspace (the little operator rebuilt for its own operator); and a
    lighter down-type quark (kappa LIGHT_KAPPA) where the low modes matter more."""
    import synthgen as sg
    out = {}

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3, st

    light = dict(flavours[0])
    light["kappa"] = LIGHT_KAPPA
    lat_l = qxd.Lattice(w["L"], w["cstar"])
    lat_l.setup(U, A, light)
    cases = list(zip(lats, ("qhat-2", "qhat+4"))) + [(lat_l, "qhat-2 kappa %.4f" % LIGHT_KAPPA)]
    b = sg.spinor(w["source_seed"] + 1, lats[0].V)
    prm_sap = qxd.solver_params(res=1e-10, inner_prec=qxd.F32, sap_ncy=SAP_NCY, sap_nmr=SAP_NMR, sap_plain=SAP_PLAIN)
    prm_dfl = qxd.solver_params(res=1e-10, inner_prec=qxd.F32, sap_ncy=SAP_NCY, sap_nmr=SAP_NMR, sap_plain=SAP_PLAIN,
                                dfl_nc=DFL_NC)
    dfls = []
    for i, (lat, name) in enumerate(cases):
        torch.cuda.empty_cache()
        gen = torch.Generator(device="cuda").manual_seed(w["source_seed"] + 50 + i)
        v = torch.randn(DFL_NS * 24 * lat.Ve, dtype=torch.complex64, device="cuda", generator=gen)
        d = qxd.qxd_dfl_create(lat.h, DFL_NS)
        ms_gen, _ = timed(lambda: qxd.qxd_dfl_generate(lat.h, d, v, DFL_NIT, 4, 4))
        del v
        dfls.append(d)
        bd = lat.pack(torch.from_numpy(b).cuda())
        x = lat.field(qxd.F64, full=True)
        ms_s, st_s = timed(lambda: qxd.qxd_solve_fgcr(lat.h, prm_sap, None, x, bd, check=False))
        ms_d, st_d = timed(lambda: qxd.qxd_solve_fgcr_dfl(lat.h, prm_dfl, d, x, bd, check=False))
        out[name] = {"subspace_ms": round(ms_gen, 1), "ns": DFL_NS, "nit": DFL_NIT, "nc": DFL_NC,
                     "sap_fgcr": {"ms": round(ms_s, 2), "iterations": st_s["inner_it"], "status": st_s["status"],
                                  "true_residual": st_s["true_residual"]},
                     "dfl_sap_fgcr": {"ms": round(ms_d, 2), "iterations": st_d["inner_it"], "status": st_d["status"],
                                      "true_residual": st_d["true_residual"]}}
        log("%s: subspace %.0f ms; SAP-FGCR %.1f ms (%d it), DFL+SAP-FGCR %.1f ms (%d it)" % (
            name, ms_gen, ms_s, st_s["inner_it"], ms_d, st_d["inner_it"]))
        del x, bd
    # each physical flavour with the other charge's subspace
    for i in (0, 1):
        lat, name = cases[i]
        other = dfls[1 - i]
        qxd.qxd_dfl_little(lat.h, other)
        bd = lat.pack(torch.from_numpy(b).cuda())
        x = lat.field(qxd.F64, full=True)
        ms, st = timed(lambda: qxd.qxd_solve_fgcr_dfl(lat.h, prm_dfl, other, x, bd, check=False))
        out[name]["dfl_sap_fgcr_other_charge_subspace"] = {"ms": round(ms, 2), "iterations": st["inner_it"],
                                                           "status": st["status"], "true_residual": st["true_residual"]}
        log("%s with the other charge's subspace: %.1f ms (%d it)" % (name, ms, st["inner_it"]))
        del x, bd
    for d in dfls:
        qxd.qxd_dfl_destroy(d)
    lat_l.close()
    return out


def solve_leg(qxd, torch, lats, w, flavours, nn_fields, nn_epochs, big=False, only=()):
    """Time to a true FP64 residual 1e-10 on the benchmark lattice, one Gaussian
    source per flavour: FP64 CG against defect-correction CG and FGCR with FP32
    and bf16-link inner solves, FP32-inner FGCR preconditioned by SAP (two
    cycles, 8 plain minimal-residual steps per 4^4 block), and FP32-inner FGCR preconditioned
    by a network trained (per flavour) on pairs harvested from seeded 32 x 16^3
    fields with the same statistics."""
    import synthgen as sg
    from paper_1908_11673_amd import learned
    c3 = sg.WORKLOADS["c3"]
    out = {}
    b = sg.spinor(w["source_seed"] + 1, lats[0].V)
    for lat, flav, name in zip(lats, flavours, ("qhat-2", "qhat+4")):
        res = {}
        net = None
        if nn_fields > 0:
            t0 = time.perf_counter()
            wts, skip, info = learned.harvest_and_train(c3["L"], c3["cstar"], flav,
                                                        gauge_seeds=list(range(3000, 3000 + nn_fields)),
                                                        sigma_su3=w["sigma_su3"], sigma_u1=w["sigma_u1"], sources=8,
                                                        pairs_per_source=10, epochs=nn_epochs)
            net = learned.make_network(lat, wts, skip)
            res["network_training"] = {"pairs": info["pairs"], "harvest_s": round(info["harvest_s"], 2),
                                       "train_s": round(info["train_s"], 2),
                                       "loss_first_last": [round(info["loss_history"][0], 4),
                                                           round(info["loss_history"][-1], 4)],
                                       "lattice": "32x16^3 physical, C* 3", "fields": nn_fields,
                                       "epochs": nn_epochs, "skip": skip}
            log("%s network: %d pairs, harvest %.1f s, train %.1f s, loss %.3f -> %.3f" % (
                name, info["pairs"], info["harvest_s"], info["train_s"], info["loss_history"][0],
                info["loss_history"][-1]))
        bd = lat.pack(torch.from_numpy(b).cuda())
        torch.cuda.empty_cache()  # the library allocates its solver vectors itself
        x = lat.field(qxd.F64, full=True)

        def cg(inner):
            return lambda: qxd.qxd_solve_cg(lat.h, qxd.solver_params(res=1e-10, inner_prec=inner, check_every=8), x,
                                            bd, check=False)

        # at 128 x 64^3 the 2 nkv FGCR directions must fit beside the operator: nkv 4
        nkv = 4 if big else 16

        def fgcr(inner, network=None, sap_ncy=0, sap_nmr=8, sap_plain=0):
            prm = qxd.solver_params(res=1e-10, inner_prec=inner, sap_ncy=sap_ncy, sap_nmr=sap_nmr,
                                    sap_plain=sap_plain, nkv=nkv)
            return lambda: qxd.qxd_solve_fgcr(lat.h, prm, network, x, bd, check=False)

        legs = [("cg_f64", cg(qxd.F64)), ("cg_f32_in_f64", cg(qxd.F32)), ("cg_bf16links_in_f64", cg(qxd.BF16))]
        legs.append(("fgcr_f32_in_f64", fgcr(qxd.F32)))
        if not big:  # the SAP block copies do not fit beside the 128 x 64^3 operator and FGCR's directions
            legs += [("fgcr_bf16links_in_f64", fgcr(qxd.BF16)),
                     ("fgcr_f32_sap_in_f64", fgcr(qxd.F32, sap_ncy=SAP_NCY, sap_nmr=SAP_NMR, sap_plain=SAP_PLAIN)),
                     ("fgcr_f32_sap_eo55_in_f64", fgcr(qxd.F32, sap_ncy=5, sap_nmr=5, sap_plain=0))]
        if net is not None:
            legs.append(("fgcr_f32_nn_in_f64", fgcr(qxd.F32, net)))
        trimmed = False
        for tag, fn in legs:
            if only and tag not in only:
                continue
            if big and tag.startswith("fgcr"):
                if not trimmed:  # drop the CG legs' workspaces before FGCR allocates its own
                    qxd.qxd_trim(lat.h)
                    torch.cuda.empty_cache()
                    trimmed = True
                fn()  # untimed: the first call allocates the 2 nkv directions
            times = []
            for rep in range(1 if big else 3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = fn()
                torch.cuda.synchronize()
                times.append((time.perf_counter() - t0) * 1e3)
            res[tag] = {"ms_median": round(float(np.median(times)), 2), "status": st["status"],
                        "iterations": st["inner_it"], "outer": st["outer_it"], "schur_applies": st["schur_applies"],
                        "nn_applies": st["nn_applies"], "sap_applies": st["sap_applies"], "fell_back": st["fell_back"],
                        "true_residual": st["true_residual"]}
            if tag.startswith("fgcr"):
                res[tag]["nkv"] = nkv
            log("solve %s %s: %.1f ms, %d it, res %.2e, status %d" % (name, tag, np.median(times), st["inner_it"],
                                                                       st["true_residual"], st["status"]))
        if net is not None:
            qxd.qxd_nn_destroy(net)
        out[name] = res
    return out


if __name__ == "__main__":
    main()
