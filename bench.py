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
# bf16 storage: links 288 reals and spinors 120 reals at 2 bytes, clover blocks 144 reals at 4 bytes
BF16_BYTES_PER_VE = (288 + 120) * 2 + 144 * 4


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def make_fields(w):
    import synthgen as sg
    L = w["L"]
    vphys = L[0] * L[1] * L[2] * L[3]
    U = sg.gauge_su3(w["gauge_seed"], w["sigma_su3"], vphys)
    A = sg.gauge_u1(w["gauge_seed"], w["sigma_u1"], vphys)
    return U, A


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n):
    """Set the OpenMP thread count of this process (the oracle's parallel
    loops); returns the previous count."""
    import ctypes
    gomp = ctypes.CDLL("libgomp.so.1")
    old = gomp.omp_get_max_threads()
    gomp.omp_set_num_threads(int(n))
    return old


def _oracle_rate(o, psi, even, seconds, seed):
    """Oracle D_hat on batches of random even sites for about `seconds`:
    sites done and the time they took."""
    rng = np.random.default_rng(seed)
    n, done, t_tot = 64, 0, 0.0
    while t_tot < seconds:
        sites = rng.choice(even, size=n, replace=False)
        t0 = time.perf_counter()
        o.schur_sites(psi, sites)
        t_tot += time.perf_counter() - t0
        done += n
        n = min(2 * n, 4096)
    return done, t_tot


def cpu_baseline(w, U, A, flav, seconds=15.0):
    """The FP64 oracle's D_hat on a bounded sample of even sites of the same
    lattice, with its site clover blocks and their inverses precomputed (the
    oracle's cache; the set-up is timed apart and not in the rate): all host
    threads for about half the time, then one thread; plus the oracle's CG solve
    of the 8 x 4^3 lattice to the same 1e-10 residual (one thread)."""
    import oracle
    import synthgen as sg
    try:  # numpy's BLAS threads spin after each call and starve the oracle's OpenMP loops
        from threadpoolctl import threadpool_limits
        limit = threadpool_limits(1, user_api="blas")
    except ImportError:
        limit = None
    threads = _omp_threads(os.cpu_count() or 1)
    _omp_threads(threads)
    o = oracle.Oracle(w["L"], w["cstar"])
    o.set_gauge_physical(U, A)
    t0 = time.perf_counter()
    o.set_flavour(**flav, cache=True)
    setup_s = time.perf_counter() - t0
    psi = sg.spinor(w["source_seed"], o.V)
    par = o.parity()
    psi[par == 1] = 0
    even = np.nonzero(par == 0)[0]
    done, t_all = _oracle_rate(o, psi, even, seconds / 2, 0)
    old = _omp_threads(1)
    done1, t_one = _oracle_rate(o, psi, even, seconds / 2, 1)
    _omp_threads(old)
    gbs = done * REALS_PER_VE * 8 / t_all / 1e9
    gbs1 = done1 * REALS_PER_VE * 8 / t_one / 1e9
    # the oracle's FP64 CG on the small workload (8 x 4^3, C* in x1), true residual 1e-10
    w0 = sg.WORKLOADS["c0"]
    o0 = oracle.Oracle(w0["L"], w0["cstar"])
    vp = int(np.prod(w0["L"]))
    o0.set_gauge_physical(sg.gauge_su3(w0["gauge_seed"], w0["sigma_su3"], vp), sg.gauge_u1(w0["gauge_seed"],
                                                                                            w0["sigma_u1"], vp))
    o0.set_flavour(**flav)
    b0 = sg.spinor(w0["source_seed"], o0.V)
    old = _omp_threads(1)  # 512 even sites: one thread is fastest
    t0 = time.perf_counter()
    bh = o0.eo_source(b0)
    xe, it0, _ = o0.cg(bh, 1e-10 * np.linalg.norm(b0))
    x0 = o0.eo_reconstruct(xe, b0)
    c0_ms = (time.perf_counter() - t0) * 1e3
    _omp_threads(old)
    res0 = float(np.linalg.norm(b0 - o0.dirac(x0)) / np.linalg.norm(b0))
    if limit is not None:
        limit.unregister()
    return {"value": gbs, "unit": "GB/s", "cores": threads, "kind": "oracle", "cpu_model": _cpu_model(),
            "one_core_gbs": gbs1,
            "sample": "FP64 D_hat of the oracle as is on random even sites of the same lattice (%d sites in %.1f s "
                      "on %d threads, %d sites in %.1f s on 1 thread), site blocks precomputed in %.1f s" % (
                          done, t_all, threads, done1, t_one, setup_s),
            "c0_cg": {"ms": round(c0_ms, 1), "iterations": it0, "true_residual": res0, "threads": 1,
                      "lattice": "8x4^3 physical, C* 1"}}


def solve_summary(tts):
    """Per flavour of a time-to-solution block: FP64 CG, the network-preconditioned
    mixed-precision FGCR and the fastest solve (all to the FP64 true residual
    1e-10), with their speed-ups over FP64 CG."""
    out = {}
    for name, legs in tts.items():
        if not isinstance(legs, dict):  # the lattice description
            continue
        ok = {k: v for k, v in legs.items() if isinstance(v, dict) and v.get("status") == 0 and "ms_median" in v}
        if "cg_f64" not in ok:
            continue
        cg = ok["cg_f64"]["ms_median"]
        best = min(ok, key=lambda k: ok[k]["ms_median"])
        row = {"cg_f64_ms": cg, "fastest": best, "fastest_ms": ok[best]["ms_median"],
               "fastest_speedup_vs_cg_f64": round(cg / ok[best]["ms_median"], 2)}
        if "fgcr_f32_nn_in_f64" in ok:
            nn = ok["fgcr_f32_nn_in_f64"]["ms_median"]
            row.update({"mixed_learned_ms": nn, "mixed_learned_speedup_vs_cg_f64": round(cg / nn, 2)})
        out[name] = row
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-c4", action="store_true", help="skip the 128 x 64^3 time-to-solution leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--nn-fields", type=int, default=20, help="fields for the network training (0: no network)")
    ap.add_argument("--nn-epochs", type=int, default=8)
    ap.add_argument("--legs", default="", help="comma-separated solve legs to run (default: all)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on one GPU (a multi-GPU path with time-slab "
              "halo exchange over xGMI is designed, not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    t_start = time.perf_counter()
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
    log("D_hat FP64 %.3f ms (%.0f GB/s, %.1f %% of the %.0f GB/s HBM peak; 70 %% would take %.3f ms), "
        "FP32 %.3f ms (%.0f GB/s, %.1f %%)" % (
            ms64, ach64, 100 * ach64 / HBM_PEAK_GBS, HBM_PEAK_GBS,
            REALS_PER_VE * 8 * Ve / (0.7 * HBM_PEAK_GBS * 1e9) * 1e3, ms32, ach32, 100 * ach32 / HBM_PEAK_GBS))
    # bf16 storage: links and spinors in bfloat16, clover blocks FP32
    in16 = [qxd.field(Ve, qxd.BF16) for _ in range(nbuf)]
    out16 = [qxd.field(Ve, qxd.BF16) for _ in range(nbuf)]
    for i in range(nbuf):
        full = qxd.field(Ve, qxd.BF16, full=True)
        qxd.qxd_pack(lats[0].h, qxd.BF16, full, lats[0].unpack(
            torch.cat([ins[qxd.F64][i], torch.zeros_like(ins[qxd.F64][i])])))
        in16[i].copy_(full[:full.numel() // 2])
        del full
    for i in range(10):
        qxd.qxd_dw_eo_schur(lats[0].h, qxd.BF16, 0, out16[i % nbuf], in16[i % nbuf], sptr)
    n16 = 100
    e0.record(stream)
    for i in range(n16):
        qxd.qxd_dw_eo_schur(lats[0].h, qxd.BF16, 0, out16[i % nbuf], in16[i % nbuf], sptr)
    e1.record(stream)
    torch.cuda.synchronize()
    ms16 = e0.elapsed_time(e1) / n16
    ach16 = BF16_BYTES_PER_VE * Ve / (ms16 * 1e-3) / 1e9
    log("D_hat bf16 storage %.3f ms (%.0f GB/s, %.1f %%)" % (ms16, ach16, 100 * ach16 / HBM_PEAK_GBS))
    del in16, out16

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
        "dhat_bf16": {"ms": round(ms16, 4), "achieved_gbs": round(ach16, 1), "frac": round(ach16 / HBM_PEAK_GBS, 4),
                      "bytes_per_even_site": BF16_BYTES_PER_VE,
                      "storage": "links and spinors bfloat16, clover blocks FP32"},
        "copy_kernel_gbs": round(copy_gbs, 1),
    }

    if not args.no_solve:
        del ins, outs
        torch.cuda.empty_cache()
        only = tuple(t for t in args.legs.split(",") if t)
        train = (not only or "fgcr_f32_nn_in_f64" in only or "learned" in only) and args.nn_fields > 0
        nets = train_networks(qxd, flavours, args.nn_fields, args.nn_epochs) if train else None
        if nets and not big and (not only or "learned" in only):
            result["learned_c3"] = learned_leg(qxd, torch, flavours, nets)
        result["time_to_solution"] = solve_leg(qxd, torch, lats, w, flavours, nets, big, only)
        if not big and (not only or "shifted" in only):
            result["shifted_solves"] = shifted_leg(qxd, torch, lats, w, flavours)
        if not big and (not only or "deflation" in only):
            result["deflation"] = deflation_leg(qxd, torch, lats, w, flavours, U, A)

    if not args.no_c4 and not big and not args.no_solve and (not only or "c4" in only):
        for lat in lats:
            lat.close()
        lats = []
        torch.cuda.empty_cache()
        result["time_to_solution_c4"] = c4_leg(qxd, torch, nets, t_start)

    if not args.no_cpu_baseline and not big:  # the oracle would hold 60 GB of host fields at 128 x 64^3
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(w, U, A, flavours[0], args.cpu_seconds)
    summary = {k: solve_summary(result[k]) for k in ("time_to_solution", "time_to_solution_c4") if k in result}
    if summary:
        result["solve_summary"] = summary
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


def train_networks(qxd, flavours, nn_fields, nn_epochs, pairs_per_field=100):
    """One network per flavour, trained on `pairs_per_field` (residual, error)
    pairs harvested on each of the 32 x 16^3 fields 3000 .. 3000 + nn_fields - 1
    (the learned form's training set: 20 fields x 100 pairs)."""
    import synthgen as sg
    from paper_1908_11673_amd import learned
    c3 = sg.WORKLOADS["c3"]
    nets = []
    for flav in flavours:
        wts, skip, info = learned.harvest_and_train(c3["L"], c3["cstar"], flav,
                                                    gauge_seeds=list(range(3000, 3000 + nn_fields)),
                                                    sigma_su3=c3["sigma_su3"], sigma_u1=c3["sigma_u1"],
                                                    pairs_per_field=pairs_per_field, epochs=nn_epochs)
        meta = {"pairs": info["pairs"], "harvest_s": round(info["harvest_s"], 2), "train_s": round(info["train_s"], 2),
                "loss_first_last": [round(info["loss_history"][0], 4), round(info["loss_history"][-1], 4)],
                "lattice": "32x16^3 physical, C* 3", "fields": nn_fields, "pairs_per_field_target": pairs_per_field,
                "epochs": nn_epochs, "skip": skip}
        log("qhat %+d network: %d pairs on %d fields, harvest %.1f s, train %.1f s, loss %.3f -> %.3f" % (
            flav["qhat"], info["pairs"], nn_fields, info["harvest_s"], info["train_s"], info["loss_history"][0],
            info["loss_history"][-1]))
        nets.append((wts, skip, meta))
    return nets


NN_HELD_OUT = tuple(range(3100, 3110))  # held-out 32 x 16^3 fields of the learned-form evaluation


def learned_leg(qxd, torch, flavours, nets):
    """The learned form on its own lattice: per flavour, FGCR preconditioned by
    the trained network against plain FGCR (both FP32 inner, FP64 defect
    correction) and FP64 CG, to the FP64 true residual 1e-10 on each held-out
    32 x 16^3 field (one Gaussian source each; median of 3 timed solves)."""
    import synthgen as sg
    from paper_1908_11673_amd import learned
    c3 = sg.WORKLOADS["c3"]
    L, cstar = c3["L"], c3["cstar"]
    vphys = int(np.prod(L))
    out = {}
    lat = qxd.Lattice(L, cstar)
    for flav, (wts, skip, meta) in zip(flavours, nets):
        name = "qhat%+d" % flav["qhat"]
        net = learned.make_network(lat, wts, skip)
        rows = {"network_fgcr": [], "plain_fgcr": [], "cg_f64": []}
        for k, gs in enumerate(NN_HELD_OUT):
            lat.setup(sg.gauge_su3(gs, c3["sigma_su3"], vphys), sg.gauge_u1(gs, c3["sigma_u1"], vphys), flav)
            bd = lat.pack(torch.from_numpy(sg.spinor(3600 + k, lat.V)).cuda())
            x = lat.field(qxd.F64, full=True)
            prm = qxd.solver_params(res=1e-10, inner_prec=qxd.F32)
            legs = (("network_fgcr", lambda: qxd.qxd_solve_fgcr(lat.h, prm, net, x, bd, check=False)),
                    ("plain_fgcr", lambda: qxd.qxd_solve_fgcr(lat.h, prm, None, x, bd, check=False)),
                    ("cg_f64", lambda: qxd.qxd_solve_cg(lat.h, qxd.solver_params(res=1e-10, check_every=8), x, bd,
                                                        check=False)))
            for tag, fn in legs:
                fn()  # warm-up
                times = []
                for _ in range(3):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    st = fn()
                    torch.cuda.synchronize()
                    times.append((time.perf_counter() - t0) * 1e3)
                rows[tag].append({"field": gs, "steps": st["inner_it"], "ms": round(float(np.median(times)), 2),
                                  "status": st["status"], "true_residual": st["true_residual"],
                                  "fell_back": st["fell_back"]})
        qxd.qxd_nn_destroy(net)
        summary = {t: {"steps_mean": round(float(np.mean([r["steps"] for r in v])), 1),
                       "ms_mean": round(float(np.mean([r["ms"] for r in v])), 2)} for t, v in rows.items()}
        out[name] = {"training": meta, "held_out_fields": list(NN_HELD_OUT), "summary": summary, "per_field": rows}
        log("%s learned form at 32x16^3 over %d held-out fields: network FGCR %.1f steps %.1f ms, plain FGCR %.1f "
            "steps %.1f ms, FP64 CG %.1f it %.1f ms" % (
                name, len(NN_HELD_OUT), summary["network_fgcr"]["steps_mean"], summary["network_fgcr"]["ms_mean"],
                summary["plain_fgcr"]["steps_mean"], summary["plain_fgcr"]["ms_mean"],
                summary["cg_f64"]["steps_mean"], summary["cg_f64"]["ms_mean"]))
    lat.close()
    return out


def solve_leg(qxd, torch, lats, w, flavours, nets, big=False, only=(), b=None):
    """Time to a true FP64 residual 1e-10 on the benchmark lattice, one Gaussian
    source per flavour: FP64 CG against defect-correction CG and FGCR with FP32
    and bf16-link inner solves, FP32-inner FGCR preconditioned by SAP (two
    cycles, 8 plain minimal-residual steps per 4^4 block), and FP32-inner FGCR
    preconditioned by the flavour's network (`nets`, trained on 32 x 16^3
    fields with the same statistics; the network is local, so its weights
    apply on any lattice).  `big` (the 128 x 64^3 lattice): one timed solve per
    leg, only the tuned SAP setting, every workspace released before each FGCR
    leg, and each FGCR leg with the largest restart length of 12, 10, ..., 4
    whose directions fit beside the operator (and the SAP block copies)."""
    import synthgen as sg
    from paper_1908_11673_amd import learned
    out = {}
    if b is None:
        b = sg.spinor(w["source_seed"] + 1, lats[0].V)
    for i, (lat, flav) in enumerate(zip(lats, flavours)):
        name = "qhat%+d" % flav["qhat"]
        res = {}
        net = None
        if nets:
            wts, skip, meta = nets[i]
            net = learned.make_network(lat, wts, skip)
            res["network_training"] = meta
        bd = lat.pack(torch.from_numpy(b).cuda())
        torch.cuda.empty_cache()  # the library allocates its solver vectors itself
        x = lat.field(qxd.F64, full=True)

        def cg(inner):
            return lambda: qxd.qxd_solve_cg(lat.h, qxd.solver_params(res=1e-10, inner_prec=inner, check_every=8), x,
                                            bd, check=False)

        nkv = [12 if big else 16]

        def fgcr(inner, network=None, sap_ncy=0, sap_nmr=8, sap_plain=0, nmx=100000):
            return lambda: qxd.qxd_solve_fgcr(
                lat.h, qxd.solver_params(res=1e-10, inner_prec=inner, sap_ncy=sap_ncy, sap_nmr=sap_nmr,
                                         sap_plain=sap_plain, nkv=nkv[0], nmx=nmx), network, x, bd, check=False)

        legs = [("cg_f64", cg(qxd.F64)), ("cg_f32_in_f64", cg(qxd.F32)), ("cg_bf16links_in_f64", cg(qxd.BF16))]
        legs.append(("fgcr_f32_in_f64", (qxd.F32, None)))
        if not big:
            legs.append(("fgcr_bf16links_in_f64", (qxd.BF16, None)))
        legs.append(("fgcr_f32_sap_in_f64", (qxd.F32, None, SAP_NCY, SAP_NMR, SAP_PLAIN)))
        if not big:
            legs.append(("fgcr_f32_sap_eo55_in_f64", (qxd.F32, None, 5, 5, 0)))
        if net is not None:
            legs.append(("fgcr_f32_nn_in_f64", (qxd.F32, net)))
        for tag, fn in legs:
            if only and tag not in only:
                continue
            if tag.startswith("fgcr"):
                spec = fn
                fn = fgcr(*spec)
                if big:
                    # drop the previous legs' workspaces and copies before this one allocates its own
                    qxd.qxd_trim(lat.h)
                    torch.cuda.empty_cache()
                    nkv[0] = 12
                    # untimed one-step call: allocates the 2 nkv directions (fewer if they do not fit)
                    while fgcr(*spec, nmx=1)()["status"] == 3 and nkv[0] > 4:
                        qxd.qxd_trim(lat.h)
                        nkv[0] -= 2
                        log("%s %s: directions do not fit, restart length %d" % (name, tag, nkv[0]))
                    fn = fgcr(*spec)
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
                res[tag]["nkv"] = nkv[0]
            log("solve %s %s: %.1f ms, %d it, res %.2e, status %d" % (name, tag, np.median(times), st["inner_it"],
                                                                       st["true_residual"], st["status"]))
        if net is not None:
            qxd.qxd_nn_destroy(net)
        out[name] = res
    return out


C4_LEGS = {"qhat-2": ("cg_f64", "cg_f32_in_f64", "fgcr_f32_in_f64", "fgcr_f32_sap_in_f64", "fgcr_f32_nn_in_f64"),
           "qhat+4": ("cg_f64", "fgcr_f32_sap_in_f64")}
C4_BUDGET_S = 220.0  # bench seconds elapsed after which the up-type solves at 128 x 64^3 are left out


def c4_leg(qxd, torch, nets, t_start):
    """Time to the FP64 true residual 1e-10 at the largest one-GPU share, the
    128 x 64^3 physical lattice with C* in three directions (extended 128 x 128
    x 64 x 64, 67,108,864 sites), both flavours one after the other on one
    handle; one Gaussian source, one timed solve each.  Down-type: FP64 CG
    against defect-correction CG (FP32 inner), FP32-inner FGCR, SAP-preconditioned
    FP32-inner FGCR and network-preconditioned FP32-inner FGCR.  Up-type: FP64
    CG against SAP-preconditioned FGCR only; at this volume its operator needs
    about 1650 CG iterations (defect-correction CG about 2830 inner ones, 94 s),
    plain FGCR with the restart lengths whose directions fit (12 and less)
    stalls near 1e-6 after 2500 steps, and the network gains no steps for this
    flavour at any volume measured.  The handle holds the FP64 operator (97 GB)
    and only the lower-precision copies the running solve uses.  The up-type
    solves are left out if the bench has already run C4_BUDGET_S seconds."""
    import synthgen as sg
    w4 = sg.WORKLOADS["c4"]
    t0 = time.perf_counter()
    U, A = make_fields(w4)
    lat = qxd.Lattice(w4["L"], w4["cstar"])
    b = sg.spinor(w4["source_seed"], lat.V)
    log("c4 fields and source generated in %.1f s" % (time.perf_counter() - t0))
    out = {}
    flavours = [sg.FLAVOURS["d"], sg.FLAVOURS["u"]]
    for i, flav in enumerate(flavours):
        name = "qhat%+d" % flav["qhat"]
        if name == "qhat+4" and time.perf_counter() - t_start > C4_BUDGET_S:
            log("c4 %s left out: %.0f s of bench elapsed" % (name, time.perf_counter() - t_start))
            out[name] = {"skipped": "bench time budget (%.0f s elapsed)" % (time.perf_counter() - t_start)}
            continue
        t0 = time.perf_counter()
        st = lat.setup(U, A, flav)
        qxd.qxd_trim(lat.h)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        log("c4 qhat %+d set up in %.1f s (min pivot %.4f)" % (flav["qhat"], setup_s, st["min_pivot"]))
        res = solve_leg(qxd, torch, [lat], w4, [flav], [nets[i]] if nets else None, big=True, only=C4_LEGS[name],
                        b=b)
        torch.cuda.empty_cache()
        res[name]["setup_s"] = round(setup_s, 2)
        res[name]["min_pivot"] = st["min_pivot"]
        out[name] = res[name]
        qxd.qxd_trim(lat.h)
    lat.close()
    del U, A, b
    out["lattice"] = "128x64^3 physical, C* 3 (extended 128x128x64x64)"
    return out


if __name__ == "__main__":
    main()
