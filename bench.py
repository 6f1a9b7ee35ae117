"""Benchmark of one space-time P + Sigma step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 3] [--prec fp64|fp32|bf16x3]
    python bench.py --serve [--requests 200] [--slots 4]

The step line also carries a bounded serving leg (--serve-requests, default 40 requests of the
serving mix on the BF16-split path): its throughput and p50 / p99 latency beside the one-at-a-time
FP64 service of the same stream.  Roofline entries are given per kernel and for the whole step.

A step is the whole path on one synthetic cell with inputs resident in HBM:
    G(k,tau) -k2r-> G(R,tau) -> P (Eq. 5) and Sigma (Eq. 8, with W(R,tau))
    -> drain (R->k, tau->Matsubara) of P and of Sigma -> electron count.
The metric is the algorithmic P + Sigma GFLOP/s of the whole step.  The default
(mixed) path stores G, W, P as complex64 and runs both contractions on the BF16
matrix cores with split-precision (hi + lo) products and FP32 accumulation; the lattice and
Matsubara transforms and the electron count are FP64, and the Sigma orbital sums run in FP32 per
row of nine terms and in FP64 across rows.  The FP32 and the plain FP64 paths are timed after it
on the same inputs, each with its error on the oracle's sample.  One JSON line is printed with a roofline entry for the dominant kernel
(timed with events on the launch stream) and the CPU oracle timed on a bounded
sample, whose outputs also give the error of the timed path.
"""
import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15}
HBM_PEAK = 8.0e12

# HBM bytes per launch of a kernel from rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE of
# the kernel, each divided by the same counter's reading per byte of a plain device copy;
# the summaries are in profiles/).  Keyed by (kernel, precision); valid only while the
# source file that defines the kernel has the recorded SHA-256 prefix, else reported null.
TRAFFIC = {
    ("Sigma", "bf16x3"): {"bytes": 62.73e9 + 3.38e9, "source": "paper_1911_05633_amd/csrc/contract_mfma.hip",
                          "sha256": "b3c924ea8cd5cb7c"},
    ("P", "bf16x3"): {"bytes": 3.17e9 + 58.30e9, "source": "paper_1911_05633_amd/csrc/contract_mfma.hip",
                      "sha256": "b3c924ea8cd5cb7c"},
    ("drain_P", "bf16x3"): {"bytes": 57.33e9 + 57.33e9, "source": "paper_1911_05633_amd/csrc/omega_kernels.h",
                            "sha256": "e263b1c8de584bc2"},
    ("k2r", "bf16x3"): {"bytes": 2.58e9 + 1.29e9, "source": "paper_1911_05633_amd/csrc/fourier.hip",
                        "sha256": "a5af6e76c96c7ef9"},
}


def _source_hash(rel):
    import hashlib
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(kernel, prec):
    rec = TRAFFIC.get((kernel, prec))
    if rec is None:
        return None
    try:
        if _source_hash(rec["source"]) != rec["sha256"]:
            return None
    except OSError:
        return None
    return rec["bytes"]


def copy_reference(gib, torch, log):
    """One plain device copy of `gib` GiB (the reference for scaling the HBM byte counters)."""
    n = int(gib * 2**30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy reference: {n * 8} bytes read and {n * 8} bytes written")


def pair_flops(spec):
    """Algorithmic P and Sigma flops per (tau, R) slice: sum over atom pairs of the cheapest
    contraction order (complex x real MAC = 4 flop, complex x complex MAC = 8 flop)."""
    n = spec.atom_norb
    m = spec.atom_npb
    fp = fs = 0.0
    for A in range(spec.n_atoms):
        nA, mA = float(n[A]), float(m[A])
        nB, mB = n.astype(float), m.astype(float)
        p1 = 4 * mA * nA * nA * nB + 8 * mA * nA * nB * nB + 4 * mA * mB * nB * nB
        p2 = 4 * mB * nB * nB * nA + 8 * mB * nB * nA * nA + 4 * mA * mB * nA * nA
        s1 = 4 * mA * mB * nB * nB + 4 * mA * nA * nA * nB + 8 * mA * nA * nB * nB
        s2 = 4 * mA * mB * nA * nA + 4 * mB * nB * nB * nA + 8 * mB * nB * nA * nA
        fp += np.minimum(p1, p2).sum()
        fs += np.minimum(s1, s2).sum()
    return fp, fs


def build_inputs(spec, prec, torch, log):
    import synthcell as sc
    import paper_1911_05633_amd as g

    t0 = time.time()
    hop = sc.hoppings(spec)
    b = sc.bands(spec, hop)
    C = sc.coefficients(spec)
    Gk_h = sc.green_ktau(spec, b)
    A = sc.w_amplitude(spec)
    sR, et = sc.w_factors(spec)
    log(f"inputs built on host in {time.time() - t0:.1f}s")
    cdt = torch.complex128 if prec == "fp64" else torch.complex64
    Gk = torch.from_numpy(Gk_h).cuda()
    GR = torch.empty(Gk.shape, dtype=cdt, device="cuda")
    Ad = torch.from_numpy(A).cuda().to(torch.float64)
    W = torch.empty((spec.n_tau, spec.N_R, spec.N_pb, spec.N_pb), dtype=cdt, device="cuda")
    for t in range(spec.n_tau):
        for R in range(spec.N_R):
            W[t, R].copy_(Ad * float(sR[R] * et[t]))
    del Ad
    P = torch.empty((spec.n_tau, spec.N_R, spec.N_pb, spec.N_pb), dtype=cdt, device="cuda")
    S = torch.empty((spec.n_tau, spec.N_R, spec.N_orb, spec.N_orb), dtype=torch.complex128, device="cuda")
    tau = sc.tau_grid(spec)
    TP = torch.from_numpy(g.gw_tau2omega_matrix(tau, g.matsubara(spec.n_tau, spec.beta, "bosonic"))).cuda()
    TS = torch.from_numpy(g.gw_tau2omega_matrix(tau, g.matsubara(spec.n_tau, spec.beta, "fermionic"))).cuda()
    nd = torch.zeros(1, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    return dict(C=C, Gk=Gk, GR=GR, W=W, P=P, S=S, TP=TP, TS=TS, n=nd, Gk_h=Gk_h, A=A, sR=sR, et=et)


KERNELS = ["k2r", "P", "Sigma", "drain_P", "drain_Sigma", "density"]


def run_step(g, cell, d, spec, prec, ev=None):
    """One pass of the whole path; ev: list of (start, end) events per kernel, or None."""
    calls = [
        lambda: g.gw_fourier_k2r(cell, d["Gk"], d["GR"], basis=0),
        lambda: g.gw_polarizability(cell, d["GR"], d["P"], spec.spin, prec=prec),
        lambda: g.gw_self_energy(cell, d["GR"], d["W"], d["S"], prec=prec),
        lambda: g.gw_drain(cell, d["TP"], d["P"], d["P"], basis=1, parity=1),
        lambda: g.gw_drain(cell, d["TS"], d["S"], d["S"], basis=0, parity=-1),
        (lambda: g.gw_density(cell, d["GR"], spec.spin, d["n"], space=0)) if prec == "fp64" else
        (lambda: g.gw_density(cell, d["Gk"], spec.spin, d["n"], space=1)),
    ]
    for i, f in enumerate(calls):
        if ev is not None:
            ev[i][0].record()
        f()
        if ev is not None:
            ev[i][1].record()


# MFMA instructions per (tau, R, A, B) block of the BF16 split kernels on the 9-orbital /
# 64-padded-function species pair (each 16x16x32, 16384 flop): the polarizability runs 84 per
# wavefront on 4 wavefronts and evaluates the blocks of tau <= beta / 2 only (the mirror gives
# the rest); the self-energy runs 84 per wavefront on 3 wavefronts for every block.
MFMA_PER_BLOCK_BF16 = {"P": 4 * 84, "Sigma": 3 * 84}


def kernel_roofs(spec, prec, fp, fs):
    """Per kernel of the step: algorithmic flops and the peak they run against, algorithmic HBM
    bytes (every operand read once, every result written once), executed flops where the kernel
    runs a different count (BF16 split products, the tau mirror).  The roof of a kernel is
    max(flops / peak, bytes / HBM peak)."""
    es = 16 if prec == "fp64" else 8
    No, Np, NR, nt = spec.N_orb, spec.N_pb, spec.N_R, spec.n_tau
    n_om, half = nt, (nt + 1) // 2
    peak_mfma = {"fp64": PEAK["fp64"], "fp32": PEAK["fp32"], "bf16x3": PEAK["bf16"]}[prec]
    gG, gP = float(nt * NR * No * No), float(nt * NR * Np * Np)
    # R -> k: separable butterflies, N_R log2 N_R complex additions per (tau, element) column
    dft = 2.0 * NR * np.log2(max(NR, 1))
    k = {}
    k["k2r"] = dict(flops=dft * gG / NR, peak=PEAK["fp64"], bytes=gG * (16 + es))
    k["P"] = dict(flops=fp * nt * NR, peak=peak_mfma, bytes=gG * es + gP * es)
    k["Sigma"] = dict(flops=fs * nt * NR, peak=peak_mfma, bytes=gG * es + gP * es + gG * 16)
    # drain with the declared parity: per element and k, two real GEMMs of the n_omega x half
    # matrices (Re T, Im T) on the paired complex columns u, v = y(tau) +- y(beta - tau):
    # 8 n_omega half flop, plus the R -> k butterflies of u and v
    for name, n2, e in (("drain_P", float(Np * Np), es), ("drain_Sigma", float(No * No), 16)):
        k[name] = dict(flops=8.0 * n_om * half * NR * n2 + 2 * dft * half * n2, peak=PEAK["fp64"],
                       bytes=2.0 * nt * NR * n2 * e)
    k["density"] = dict(flops=float(NR * No), peak=PEAK["fp64"], bytes=float(NR * No * 16))
    if prec == "bf16x3" and spec.n_species == 1 and spec.n_orb[0] == 9 and 48 < spec.n_pb[0] <= 64:
        nb = float(NR * spec.n_atoms * spec.n_atoms)
        k["P"]["executed_flops"] = MFMA_PER_BLOCK_BF16["P"] * 16384.0 * half * nb
        k["Sigma"]["executed_flops"] = MFMA_PER_BLOCK_BF16["Sigma"] * 16384.0 * nt * nb
    for v in k.values():
        v["mfma_ms"] = v["flops"] / v["peak"] * 1e3
        v["hbm_ms"] = v["bytes"] / HBM_PEAK * 1e3
        v["bound"] = "mfma" if v["mfma_ms"] >= v["hbm_ms"] else "hbm"
        v["roof_ms"] = max(v["mfma_ms"], v["hbm_ms"])
    return k


def roofline_entries(roofs, per, prec, step_ms):
    """Per-kernel roofline entries from the measured kernel times, and the whole step's."""
    out = {}
    for name, ms in per.items():
        r = roofs[name]
        if r["bound"] == "hbm":
            achieved, peak, unit = r["bytes"] / (ms * 1e-3) / 1e9, HBM_PEAK / 1e9, "GB/s"
        else:
            achieved, peak, unit = r["flops"] / (ms * 1e-3) / 1e12, r["peak"] / 1e12, "TFLOP/s"
        e = {"ms": ms, "bound": r["bound"], "achieved": achieved, "peak": peak, "unit": unit,
             "frac": achieved / peak, "roof_ms": r["roof_ms"], "alg_flops": r["flops"], "alg_bytes": r["bytes"],
             "mfma_roof_ms": r["mfma_ms"], "hbm_roof_ms": r["hbm_ms"], "traffic": traffic_for(name, prec)}
        if "executed_flops" in r:
            e["executed_flops"] = r["executed_flops"]
            e["executed_mfma_ms"] = r["executed_flops"] / r["peak"] * 1e3
        out[name] = e
    roof = sum(roofs[n]["roof_ms"] for n in per)
    return out, {"roof_ms": roof, "ms": step_ms, "frac": roof / step_ms,
                 "kernel_ms_sum": float(sum(per.values()))}


def oracle_sample(spec, d, log, n_slices=2):
    """The FP64 oracle on a bounded sample: P^q(tau) and Sigma^k(tau) for n_slices (tau, q) pairs
    of the same cell.  Returns the slices and the CPU seconds spent on each."""
    import oracle
    tq = [(spec.n_tau // 3, 1), (spec.n_tau - 2, spec.N_R - 1)][:n_slices]
    P, S, tp, ts = [], [], 0.0, 0.0
    for t, q in tq:
        t0 = time.perf_counter()
        P.append(oracle.polarizability_q(d["Gk_h"], spec, d["C"], spec.spin, taus=[t], qs=[q])[0, 0])
        tp += time.perf_counter() - t0
        WR = {t: (d["et"][t] * d["sR"][:, None, None] * d["A"][None]).astype(np.complex128)}
        t0 = time.perf_counter()
        S.append(oracle.self_energy_k(d["Gk_h"], WR, spec, d["C"], taus=[t], ks=[q])[0, 0])
        ts += time.perf_counter() - t0
    log(f"cpu oracle sample ({len(tq)} slices): P {tp:.1f}s, Sigma {ts:.1f}s")
    return dict(tq=tq, P=P, S=S, tp=tp, ts=ts)


def slice_error(g, cell, d, spec, prec, smp, log):
    """Error of the timed path on the oracle's slices (recomputed, then R -> k)."""
    import torch
    g.gw_fourier_k2r(cell, d["Gk"], d["GR"], basis=0)
    g.gw_polarizability(cell, d["GR"], d["P"], spec.spin, prec=prec)
    g.gw_self_energy(cell, d["GR"], d["W"], d["S"], prec=prec)
    g.gw_fourier_r2k(cell, d["P"], d["P"], basis=1)
    g.gw_fourier_r2k(cell, d["S"], d["S"], basis=0)
    torch.cuda.synchronize()
    Pg = np.stack([d["P"][t, q].cpu().numpy().astype(np.complex128) for t, q in smp["tq"]])
    Sg = np.stack([d["S"][t, q].cpu().numpy() for t, q in smp["tq"]])
    err = {}
    for name, a, b in (("P", Pg, np.stack(smp["P"])), ("Sigma", Sg, np.stack(smp["S"]))):
        mx = float(np.max(np.abs(a - b)))
        err[name] = {"max_abs": mx, "rel": mx / float(np.max(np.abs(b)))}
    log(f"{prec}: error vs oracle on the sampled slices: {err}")
    return err


def cpu_baseline(spec, smp, fp, fs):
    """The oracle's sample as a rate: (its share of the step's algorithmic work) / CPU time.
    cores = the BLAS threads the oracle's numpy ran with (its only parallelism)."""
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    try:
        avail = len(os.sched_getaffinity(0))
    except Exception:
        avail = os.cpu_count()
    ns = len(smp["tq"])
    work = ns * (fp + fs)  # each (tau, q) slice of P and of Sigma is 1 / (n_tau N_R) of the step's
    secs = smp["tp"] + smp["ts"]
    return {"value": work / secs / 1e9, "unit": "GFLOP/s", "cores": int(cores), "kind": "oracle",
            "sample": f"k-space FP64 oracle: P^q(tau) and Sigma^k(tau) for {ns} (tau, q) pairs of the "
                      f"{spec.n_atoms}-atom cell ({ns}/{spec.n_tau * spec.N_R} of the step's P and Sigma output), "
                      f"{secs:.1f} s on {cores} BLAS threads ({avail} host cores available)"}


def time_path(g, spec, prec, steps, warmup, torch, log):
    """Build the inputs for one precision, time `steps` steps; returns (d, cell, ms, per-kernel ms)."""
    d = build_inputs(spec, prec, torch, log)
    cell = g.Cell.from_spec(spec, d["C"])
    ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in KERNELS]
          for _ in range(steps)]
    # torch creates an event at its first record: do that before the warm-up
    for row in ev:
        for pair in row:
            for e in pair:
                e.record()
    # no garbage-collector pause while launches are queued (one can leave the GPU idle), and
    # none between the warm-up and the timed steps
    gc.collect()
    gc.disable()
    try:
        for _ in range(warmup):
            run_step(g, cell, d, spec, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            run_step(g, cell, d, spec, prec, ev[s])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        gc.enable()
    per = {k: float(np.mean([ev[s][i][0].elapsed_time(ev[s][i][1]) for s in range(steps)]))
           for i, k in enumerate(KERNELS)}
    log(f"{prec}: {wall / steps * 1e3:.2f} ms/step; per-kernel ms: " +
        ", ".join(f"{k} {v:.3f}" for k, v in per.items()))
    log(f"{prec}: per step, P / Sigma / drain_P ms: " + "; ".join(
        "/".join(f"{ev[s][i][0].elapsed_time(ev[s][i][1]):.2f}" for i in (1, 2, 3)) for s in range(steps)))
    return d, cell, wall / steps * 1e3, per


def serve_runs(n, slots, torch, log, prec="bf16x3"):
    """Serving mix: a seeded stream of n independent P + Sigma requests over 2-, 8-, 24-, 40- and
    72-atom cells with 16-48 tau points, served by the continuous-batching loop on the mixed path
    (burst capacity, then Poisson arrivals at 0.7 of it: throughput, p50 / p99 latency), and the
    same Poisson stream served one request at a time on the plain FP64 path."""
    import synthcell as sc
    from synthcell.device import ServingInputs
    from paper_1911_05633_amd import serve

    def run(ex, reqs, slots):
        t0 = time.perf_counter()
        recs = serve.Server(ex, ex.capacity, slots=slots).run(reqs)
        s = serve.summarize(recs)
        s["wall_s"] = time.perf_counter() - t0
        bad = [(r.request_id, r.status, r.error) for r in recs if r.status != "done"]
        if bad:
            raise RuntimeError(f"requests not served: {bad[:5]}")
        nerr = max(abs(r.result["n"] - r.result["n_expected"]) / r.result["n_expected"] for r in recs)
        s["max_electron_count_rel_err"] = nerr
        return s

    def prepare(ex):
        t0 = time.perf_counter()
        for kind in sc.SERVING_KINDS:
            for nt in sc.SERVING_NTAU:
                ex.prepare(sc.Request(-1, 0.0, kind, nt))
        # one request per kind on the device (kernel and allocator warm-up)
        run(ex, [sc.Request(i, 0.0, kind, sc.SERVING_NTAU[0]) for i, kind in enumerate(sc.SERVING_KINDS)], 1)
        log(f"serving executor ({ex.prec}) prepared in {time.perf_counter() - t0:.1f}s, pool "
            f"{ex.capacity / 2**30:.1f} GiB")

    inputs = ServingInputs()
    ex = serve.GWExecutor(inputs, prec=prec, slots=slots)
    prepare(ex)
    burst = run(ex, sc.request_stream(n, rate=1.0, burst=True), slots)
    log(f"burst: {burst}")
    rate = 0.7 * burst["throughput_req_per_s"]
    reqs = sc.request_stream(n, rate=rate)
    mixed = run(ex, reqs, slots)
    log(f"poisson at {rate:.2f} req/s (0.7 of the burst rate), {prec}: {mixed}")
    del ex
    torch.cuda.empty_cache()
    ex64 = serve.GWExecutor(inputs, prec="fp64", slots=1)
    prepare(ex64)
    base = run(ex64, reqs, 1)
    log(f"same stream, one at a time, FP64: {base}")
    del ex64
    torch.cuda.empty_cache()
    return {"requests": n, "slots": slots, "prec": prec, "rate_req_per_s": rate,
            "throughput_req_per_s": mixed["throughput_req_per_s"], "p50_ms": mixed["p50_ms"],
            "p99_ms": mixed["p99_ms"], "burst_capacity_req_per_s": burst["throughput_req_per_s"],
            "poisson_mixed": mixed, "baseline_fp64_one_at_a_time": base,
            "speedup_throughput_vs_baseline": mixed["throughput_req_per_s"] / base["throughput_req_per_s"],
            "p99_ratio_baseline_over_mixed": base["p99_ms"] / mixed["p99_ms"],
            "workload": f"{n} requests, Poisson arrivals at {rate:.3f} req/s (0.7 of the measured burst rate), "
                        f"cells uniform over {list(sc.SERVING_KINDS)}, n_tau uniform over {list(sc.SERVING_NTAU)}"}


def serve_bench(args, torch, log):
    """The serving mix alone (bench.py --serve), as its own JSON line."""
    r = serve_runs(args.requests, args.slots, torch, log)
    out = {
        "metric": "serving mix: P+Sigma requests/s with p50/p99 latency (continuous batching, mixed path)",
        "value": r["throughput_req_per_s"], "unit": "req/s", "n_gpus": 1, "higher_is_better": True,
        "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"], "dtype": "bf16x3+f64", "data": "synthetic",
        "config": {"workload": r["workload"], "slots": args.slots}, "serving": r,
    }
    print(json.dumps(out), flush=True)


def pairs_bench(args, torch, log):
    """Real-space cutoff path (Sec. 2, Figs. 1 and 2): P + Sigma over the kept blocks (the
    matrix-core kernels walking the block list) of Si cells of 8 to 72 atoms at one cutoff (r_b = 2.5 A, r_c = 4.6 A: each atom with itself, its 4
    neighbours in the B tier with all 60 product functions and the 24 next ones in the C tier
    with 16), beside the dense contraction of every (R, A, B) block of the same cell."""
    import synthcell as sc
    import paper_1911_05633_amd as g

    prec = args.prec
    rows = []
    for kind in ("si8", "si24", "si40", "si72"):
        spec = sc.serving_cell(kind, 48, 0)
        d = build_inputs(spec, prec, torch, log)
        cell = g.Cell.from_spec(spec, d["C"])
        nk = cell.set_pairs(spec.lattice, spec.positions, 2.5, 4.6, [[60, 16]])
        g.gw_fourier_k2r(cell, d["Gk"], d["GR"], basis=0)

        def cut():
            g.gw_polarizability_pairs(cell, d["GR"], d["P"], spec.spin, prec=prec)
            g.gw_self_energy_pairs(cell, d["GR"], d["W"], d["S"], prec=prec)

        def dense():
            g.gw_polarizability(cell, d["GR"], d["P"], spec.spin, prec=prec)
            g.gw_self_energy(cell, d["GR"], d["W"], d["S"], prec=prec)

        def timed(fn, reps=3):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        ms_cut, ms_dense = timed(cut), timed(dense)
        # packed storage: P and W hold the kept blocks only
        per_tau = cell.packed_elems()
        cdt = torch.complex128 if prec == "fp64" else torch.complex64
        Ppk = torch.empty((spec.n_tau, per_tau), dtype=cdt, device="cuda")
        Wpk = torch.empty_like(Ppk)
        g.gw_polarizability_packed(cell, d["GR"], Wpk, spec.spin, prec=prec)  # any finite W will do

        def packed():
            g.gw_polarizability_packed(cell, d["GR"], Ppk, spec.spin, prec=prec)
            g.gw_self_energy_packed(cell, d["GR"], Wpk, d["S"], prec=prec)

        def packed_drain():
            g.gw_drain_packed(cell, d["TP"], Ppk, d["P"], parity=1)

        ms_packed, ms_pdrain = timed(packed), timed(packed_drain)
        es = Ppk.element_size()
        del Ppk, Wpk
        plan = cell.pairs()
        kept_elems = float((plan[:, 3].astype(np.int64) * plan[:, 4]).sum())   # sum over kept blocks of mA mB
        dense_elems = float(spec.N_R) * spec.N_pb ** 2
        row = {"cell": kind, "atoms": spec.n_atoms, "N_R": spec.N_R, "n_tau": spec.n_tau, "kept_blocks": nk,
               "dense_blocks": spec.N_R * spec.n_atoms ** 2, "ms_cutoff": ms_cut, "ms_dense": ms_dense,
               "us_per_kept_block_and_tau": ms_cut * 1e3 / (nk * spec.n_tau),
               "P_elements_per_tau_kept": kept_elems, "P_elements_per_tau_dense": dense_elems,
               "storage_ratio_dense_over_kept": dense_elems / kept_elems,
               "ms_packed": ms_packed, "ms_packed_drain_to_dense_k": ms_pdrain,
               "packed_P_bytes": float(spec.n_tau * per_tau * es),
               "dense_P_bytes": float(spec.n_tau * dense_elems * es)}
        log(f"cutoff {kind}: {row}")
        rows.append(row)
        del d, cell
        torch.cuda.empty_cache()
    a = np.array([r["atoms"] for r in rows], dtype=float)
    t = np.array([r["ms_cutoff"] for r in rows])
    slope = float(np.polyfit(np.log(a), np.log(t), 1)[0])
    out = {"metric": "cutoff path: P+Sigma ms vs cell size at fixed r_c (kernels walking the kept-block list; "
                     "dense and packed storage of P and W)",
           "unit": "ms", "n_gpus": 1, "dtype": prec, "data": "synthetic",
           "config": {"workload": "Si cells of 8, 24, 40, 72 atoms, n_tau 48, r_b 2.5 A, r_c 4.6 A, "
                                  "m_B 60, m_C 16", "prec": prec},
           "rows": rows, "loglog_slope_time_vs_atoms": slope}
    print(json.dumps(out), flush=True)


def dyson_bench(args, torch, log):
    """Screened interaction, Eq. (2): W~ = (V^-1 - P)^-1 - V for every (q, nu) of the 8-atom Si
    cell (N_pb 480, 64 q, 32 nu) and, sampled, of the 72-atom cell (N_pb 4320, 8 q, 4 of its
    48 nu).  Seeded inputs (synthcell.dyson_factors), products for V and P formed on the device
    before timing.  Work: 8 N_pb^3 real flops per inversion (the N_k inversions of V included)."""
    import oracle
    import synthcell as sc
    import paper_1911_05633_amd as g
    rows = []
    cpu = None
    for cfg, n_nu, steps in ((2, None, args.steps), (3, 4, 1)):
        spec = sc.config(cfg)
        cell = g.Cell.from_spec(spec, sc.coefficients(spec))
        n, nk = cell.N_pb, cell.N_R
        n_nu = spec.n_tau if n_nu is None else n_nu
        t0 = time.time()
        B, X, s = sc.dyson_factors(nk, n, n_nu, cfg)
        Bd = torch.from_numpy(B).cuda()
        V = torch.matmul(Bd, Bd.conj().transpose(-1, -2).contiguous()) / n
        V.diagonal(dim1=-2, dim2=-1).add_(0.5)
        del Bd
        Xd = torch.from_numpy(X).cuda()
        XX = torch.matmul(Xd, Xd.conj().transpose(-1, -2).contiguous()) / n
        del Xd
        P = torch.empty((n_nu, nk, n, n), dtype=torch.complex128, device="cuda")
        for m in range(n_nu):
            torch.mul(XX, -float(s[m]), out=P[m])
        W = torch.empty_like(P)
        total = n_nu * nk
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        log(f"dyson {spec.name}: inputs in {time.time() - t0:.1f}s; {total} (q, nu) matrices of {n}")
        Vh = V.cpu().numpy()
        for prec in ("fp64", "fp32"):
            work = torch.empty(g.gw_screened_interaction_workspace(cell, total, prec), dtype=torch.uint8,
                               device="cuda")
            g.gw_screened_interaction(cell, V, P, W, work, info=info, prec=prec)
            torch.cuda.synchronize()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
            for a, b in ev:
                a.record()
                g.gw_screened_interaction(cell, V, P, W, work, info=info, prec=prec)
                b.record()
            torch.cuda.synchronize()
            ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
            flops = 8.0 * n ** 3 * (total + nk)
            # sampled parity against the oracle
            err = 0.0
            for m, q in ((0, 0), (n_nu - 1, nk - 1)):
                ref = oracle.screened_interaction(Vh[q:q + 1], P[m:m + 1, q:q + 1].cpu().numpy())[0, 0]
                got = W[m, q].cpu().numpy()
                err = max(err, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
            peak = PEAK["fp64"] if prec == "fp64" else PEAK["fp32"]
            rows.append({"cell": spec.name, "prec": prec, "N_pb": n, "N_k": nk, "n_nu": n_nu, "matrices": total,
                         "ms": ms, "ms_per_matrix": ms / total, "gflops": flops / (ms * 1e-3) / 1e9,
                         "frac_peak": flops / (ms * 1e-3) / peak, "info": int(info.item()),
                         "max_rel_err_sampled": err})
            log(f"dyson {spec.name} {prec}: {ms:.2f} ms, {rows[-1]['gflops']:.0f} GFLOP/s, info {rows[-1]['info']}, "
                f"sampled rel err {err:.2e}")
            del work
            torch.cuda.empty_cache()
        if cfg == 2 and not args.no_cpu:
            Ph = P[0:1, 0:2].cpu().numpy()
            c0 = time.perf_counter()
            oracle.screened_interaction(Vh[0:2], Ph)
            secs = time.perf_counter() - c0
            cpu = {"value": 8.0 * n ** 3 * 2 / secs / 1e9, "unit": "GFLOP/s", "cores": os.cpu_count(),
                   "kind": "oracle", "sample": f"numpy LU solve of 2 (q, nu) systems of {n}: {secs:.2f} s"}
        del V, XX, P, W
        torch.cuda.empty_cache()
    green, exch = [], []
    for cfg in (2, 3):
        spec = sc.config(cfg)
        C = sc.coefficients(spec)
        cell = g.Cell.from_spec(spec, C)
        n, nk, n_om = cell.N_orb, cell.N_R, spec.n_tau
        b = sc.bands(spec)
        Hk = torch.from_numpy(np.ascontiguousarray(sc.hamiltonian_k(spec, sc.hoppings(spec)))).cuda()
        gen = torch.Generator(device="cuda")
        gen.manual_seed(1000 + cfg)
        X = torch.randn((nk, n, n), dtype=torch.complex128, device="cuda", generator=gen)
        XX = torch.matmul(X, X.conj().transpose(-1, -2).contiguous()) / n
        om = torch.tensor((2.0 * np.arange(n_om) + 1.0) * np.pi / spec.beta, dtype=torch.float64, device="cuda")
        S = 0.2 * XX[None] / (1j * om[:, None, None, None] - 0.3)          # causal one-pole self-energy
        G = torch.empty_like(S)
        work = torch.empty(g.gw_green_dyson_workspace(cell, n_om * nk), dtype=torch.uint8, device="cuda")
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        g.gw_green_dyson(cell, Hk, b.mu, G, work, Sigma=S, info=info)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
        for a, e in ev:
            a.record()
            g.gw_green_dyson(cell, Hk, b.mu, G, work, Sigma=S, info=info)
            e.record()
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(e) for a, e in ev]))
        fl = 8.0 * n ** 3 * n_om * nk
        green.append({"cell": spec.name, "N_orb": n, "N_k": nk, "n_omega": n_om, "matrices": n_om * nk, "ms": ms,
                      "gflops": fl / (ms * 1e-3) / 1e9, "frac_fp64_peak": fl / (ms * 1e-3) / PEAK["fp64"],
                      "info": int(info.item())})
        log(f"green {spec.name}: {ms:.2f} ms for {n_om * nk} matrices of {n}, {green[-1]['gflops']:.0f} GFLOP/s")
        del X, XX, S, G, work
        # static exchange: the self-energy kernels on one time slice, per precision
        for prec in ("fp64", "bf16x3"):
            cdt = torch.complex128 if prec == "fp64" else torch.complex64
            GR = torch.randn((spec.n_tau, nk, n, n), dtype=cdt, device="cuda", generator=gen)
            VR = torch.randn((nk, cell.N_pb, cell.N_pb), dtype=cdt, device="cuda", generator=gen)
            Sx = torch.empty((nk, n, n), dtype=torch.complex128, device="cuda")
            g.gw_exchange(cell, GR, VR, Sx, prec=prec)
            torch.cuda.synchronize()
            a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(3):
                g.gw_exchange(cell, GR, VR, Sx, prec=prec)
            e.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(e) / 3
            fs = pair_flops(spec)[1] * nk
            exch.append({"cell": spec.name, "prec": prec, "ms": ms, "gflops": fs / (ms * 1e-3) / 1e9})
            log(f"exchange {spec.name} {prec}: {ms:.3f} ms, {exch[-1]['gflops']:.0f} GFLOP/s")
            del GR, VR, Sx
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "screened interaction (Eq. 2) GFLOP/s, FP64 blocked Gauss-Jordan",
                      "unit": "GFLOP/s", "higher_is_better": True, "dtype": "f64", "rows": rows,
                      "green_dyson": green, "exchange": exch, "cpu_baseline": cpu}))


def interstitial_bench(args, torch, log):
    """Interstitial-grid blocks of P and Sigma (Eqs. (6), (7), (9), (10)) with n_g grid points per
    cell, complex64 storage (the mixed path's), random seeded blocks on the device.  Per kernel:
    HIP-event time, algorithmic HBM bytes (each block read or written once) and FP64 flops."""
    import synthcell as sc
    import paper_1911_05633_amd as g
    rows = []
    for cfg, n_g in ((2, 256), (3, 256)):
        spec = sc.config(cfg)
        cell = g.Cell.from_spec(spec, sc.coefficients(spec))
        nt, nr, no, npb = spec.n_tau, spec.N_R, spec.N_orb, spec.N_pb
        gen = torch.Generator(device="cuda")
        gen.manual_seed(2000 + cfg)
        rnd = lambda *sh: torch.randn(sh, dtype=torch.complex64, device="cuda", generator=gen)
        G = [rnd(nt, nr, no, n_g), rnd(nt, nr, n_g, no), rnd(nt, nr, n_g, n_g)]
        W = [rnd(nt, nr, npb, n_g), rnd(nt, nr, n_g, npb), rnd(nt, nr, n_g, n_g)]
        P = [torch.empty_like(W[0]), torch.empty_like(W[1]), torch.empty_like(W[2])]
        S = [torch.empty((nt, nr, no, n_g), dtype=torch.complex128, device="cuda"),
             torch.empty((nt, nr, n_g, no), dtype=torch.complex128, device="cuda"),
             torch.empty((nt, nr, n_g, n_g), dtype=torch.complex128, device="cuda")]
        for name, fn in (("P_int", lambda: g.gw_polarizability_int(cell, *G, *P, spec.spin)),
                         ("Sigma_int", lambda: g.gw_self_energy_int(cell, *G, *W, *S))):
            fn()
            torch.cuda.synchronize()
            a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            e.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(e)
            bl = nt * nr
            n2 = float((np.asarray(spec.atom_norb) ** 2 * np.asarray(spec.atom_npb)).sum())
            if name == "P_int":
                byts = bl * 8.0 * (2 * 2 * no * n_g + 2 * npb * n_g + 3 * n_g * n_g)
                flops = bl * n_g * 2 * n2 * 4.0 + bl * n_g * n_g * 8.0
            else:
                byts = bl * (8.0 * (2 * no * n_g + 2 * npb * n_g + 2 * n_g * n_g) + 16.0 * (2 * no * n_g + n_g * n_g))
                flops = bl * n_g * 2 * n2 * 8.0 + bl * n_g * n_g * 8.0
            rows.append({"cell": spec.name, "n_g": n_g, "kernels": name, "ms": ms, "GB": byts / 1e9,
                         "TB_per_s": byts / (ms * 1e-3) / 1e12, "TFLOP_per_s": flops / (ms * 1e-3) / 1e12})
            log(f"{name} {spec.name} n_g={n_g}: {ms:.2f} ms, {rows[-1]['TB_per_s']:.2f} TB/s, "
                f"{rows[-1]['TFLOP_per_s']:.1f} TFLOP/s")
        del G, W, P, S
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "interstitial blocks (Eqs. 6, 7, 9, 10): HBM TB/s and FP64 TFLOP/s", "rows": rows}))


def iteration_bench(args, torch, log):
    """One synthetic scGW iteration of the 72-atom cell on the device, stage by stage (HIP events):
    G(k, tau) -> G^R -> P (BF16 split) -> P(q, i nu) -> W~ (FP64 Dyson, all 48 nu x 8 q) -> W~(q, tau)
    -> W~^R -> Sigma_c (BF16 split) -> Sigma_c(k, i w); Sigma_x; mu search over the G Dyson
    solve (FP64).  Inputs: the seeded cell; V on-site (every q) = v_scale A, A Hermitian positive
    definite (synthcell.dyson_factors); a weak v_scale keeps the synthetic self-energy small
    enough for the tail-summed electron count."""
    import synthcell as sc
    import paper_1911_05633_amd as g
    spec = sc.config(args.config)
    C = sc.coefficients(spec)
    cell = g.Cell.from_spec(spec, C)
    hop = sc.hoppings(spec)
    b = sc.bands(spec, hop)
    nt, nk, no, npb = spec.n_tau, spec.N_R, spec.N_orb, spec.N_pb
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    tau = sc.tau_grid(spec)
    nu = g.matsubara(nt, spec.beta, "bosonic")
    wf = g.matsubara(nt, spec.beta, "fermionic")
    Gk = dev(sc.green_ktau(spec, b)).to(torch.complex64)
    Hk = dev(sc.hamiltonian_k(spec, hop))
    B = dev(sc.dyson_factors(1, npb, 1, 7)[0][0])
    A = torch.matmul(B, B.conj().T.contiguous()) / npb
    A.diagonal().add_(0.5)
    V = (args.v_scale * A)[None].expand(nk, npb, npb).contiguous()
    VR = torch.zeros((nk, npb, npb), dtype=torch.complex64, device="cuda")
    VR[0] = V[0].to(torch.complex64)
    del B, A
    TP, TS = dev(g.gw_tau2omega_matrix(tau, nu)), dev(g.gw_tau2omega_matrix(tau, wf))
    TPi = dev(g.gw_omega2tau_matrix(tau, nu))
    GR = torch.empty_like(Gk)
    P = torch.empty((nt, nk, npb, npb), dtype=torch.complex64, device="cuda")
    S = torch.empty((nt, nk, no, no), dtype=torch.complex128, device="cuda")
    SxR = torch.empty((nk, no, no), dtype=torch.complex128, device="cuda")
    Gw = torch.empty_like(S)
    chunk = min(nt * nk, 64)
    work_w = torch.empty(g.gw_screened_interaction_workspace(cell, chunk, args.w_prec), dtype=torch.uint8,
                         device="cuda")
    work_g = torch.empty(g.gw_green_dyson_workspace(cell, nt * nk), dtype=torch.uint8, device="cuda")
    n_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    stages = []
    mu_box = {}
    Sx_stack = torch.empty((nt, nk, no, no), dtype=torch.complex128, device="cuda")

    def sx_k():
        # Sigma_x(k) = sum_R exp(-i k.R) Sigma_x^R through the library's R -> k sum (slice 0 kept)
        Sx_stack[0].copy_(SxR)
        g.gw_fourier_r2k(cell, Sx_stack, Sx_stack, basis=0)

    def mu_update():
        mu_box["mu"], mu_box["n"] = g.gw_update_mu(cell, Hk, Gw, work_g, n_dev, spec.spin, spec.spin * no / 2.0,
                                                  b.mu - 1.0, b.mu + 1.0, tol=1e-8, max_iter=60, Sigma=S,
                                                  Sigma_x=Sx_stack[0])

    plan = [
        ("k2r G", lambda: g.gw_fourier_k2r(cell, Gk, GR, basis=0)),
        ("P", lambda: g.gw_polarizability(cell, GR, P, spec.spin, prec="bf16x3")),
        ("drain P", lambda: g.gw_drain(cell, TP, P, P, basis=1, parity=1)),
        ("W Dyson", lambda: g.gw_screened_interaction(cell, V, P, P, work_w, info=info, prec=args.w_prec)),
        ("W nu->tau", lambda: g.gw_tau2omega(cell, TPi, P, P, basis=1, parity=0)),
        ("W q->R", lambda: g.gw_fourier_k2r(cell, P, P, basis=1)),
        ("Sigma", lambda: g.gw_self_energy(cell, GR, P, S, prec="bf16x3")),
        ("drain Sigma", lambda: g.gw_drain(cell, TS, S, S, basis=0, parity=-1)),
        ("Sigma_x", lambda: g.gw_exchange(cell, GR, VR, SxR, prec="bf16x3")),
        ("Sigma_x R->k", sx_k),
        ("mu + G Dyson", mu_update),
    ]
    t0 = time.perf_counter()
    for name, fn in plan:
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        e.record()
        torch.cuda.synchronize()
        stages.append({"stage": name, "ms": a.elapsed_time(e)})
        log(f"iteration {spec.name}: {name} {stages[-1]['ms']:.2f} ms")
        if name == "drain Sigma":
            log(f"iteration {spec.name}: max |Sigma_c(k, i w)| = {S.abs().max().item():.4g}, W pivot report "
                f"{int(info.item())}")
    wall = time.perf_counter() - t0
    print(json.dumps({"metric": "one synthetic scGW iteration, stage times (ms)", "cell": spec.name,
                      "w_prec": args.w_prec,
                      "total_s": wall, "stages": stages, "W_info": int(info.item()), "mu": mu_box.get("mu"),
                      "count": mu_box.get("n")}))


def scgw_bench(args, torch, log):
    """The self-consistent loop (Sec. 2, Eqs. (1)-(4)) on the device: --scgw-cycles cycles from the
    band G(k, tau) of the chosen config's cell (FP64, mixing 0.5, weak synthetic V = 0.01 of a
    random positive definite matrix), with the time, mu, counts and iterate change of each cycle."""
    import synthcell as sc
    import paper_1911_05633_amd as g
    from paper_1911_05633_amd.scgw import SCGW
    spec = sc.config(args.config)
    hop = sc.hoppings(spec)
    b = sc.bands(spec, hop)
    C = sc.coefficients(spec)
    Hk = sc.hamiltonian_k(spec, hop)
    V = args.scgw_v_scale * sc.dyson_inputs(spec.N_R, spec.N_pb, 1, 9)[0]
    cell = g.Cell.from_spec(spec, C)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Gd = dev(sc.green_ktau(spec, b))
    target = spec.spin * spec.N_orb / 2.0
    loop = SCGW(cell, dev(Hk), dev(V), Gd, spec.spin, target, mix=0.5)
    torch.cuda.synchronize()
    rows, mu = [], b.mu
    prev = Gd.clone()
    for c in range(args.scgw_cycles):
        t0 = time.perf_counter()
        mu, n_w, n_beta, info = loop.cycle(mu - 1.0, mu + 1.0)
        ms = (time.perf_counter() - t0) * 1e3
        step = float((Gd - prev).abs().max().item())
        prev.copy_(Gd)
        rows.append({"cycle": c, "ms": ms, "mu": mu, "count_matsubara": n_w, "count_beta": n_beta,
                     "max_change_of_G": step, "W_pivot_report": info})
        log(f"scgw {spec.name} cycle {c}: {ms:.1f} ms, mu {mu:.8f}, count {n_w:.8f} / {n_beta:.8f}, "
            f"change {step:.3e}")
    print(json.dumps({"metric": "self-consistent GW cycles on the device (ms per cycle, FP64)", "cell": spec.name,
                      "atoms": spec.n_atoms, "N_R": spec.N_R, "n_tau": spec.n_tau, "v_scale": args.scgw_v_scale,
                      "cycles": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--prec", default="bf16x3", choices=["fp64", "fp32", "bf16x3"],
                    help="contraction arithmetic: bf16x3 = the mixed path of the 72-atom workload (split-precision "
                         "BF16 products, complex64 storage, FP64 transforms and sums; default), fp32 = FP32 "
                         "matrix cores, fp64 = plain FP64")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--serve", action="store_true", help="run the serving mix instead of the step benchmark")
    ap.add_argument("--copy-ref", type=float, default=0.0, metavar="GIB",
                    help="only run one plain device copy of GIB GiB (counter reference) and exit")
    ap.add_argument("--pairs", action="store_true",
                    help="time the real-space cutoff path against the dense one on 8- to 72-atom cells and exit")
    ap.add_argument("--dyson", action="store_true",
                    help="time the screened interaction (Eq. 2) on the 8- and 72-atom cells and exit")
    ap.add_argument("--interstitial", action="store_true",
                    help="time the interstitial-grid blocks of P and Sigma and exit")
    ap.add_argument("--iteration", action="store_true",
                    help="time one synthetic scGW iteration (P, W, Sigma, Sigma_x, mu and G) stage by stage and exit")
    ap.add_argument("--v-scale", type=float, default=1e-4, help="bare interaction scale of --iteration")
    ap.add_argument("--w-prec", default="fp64", choices=["fp64", "fp32"],
                    help="elimination precision of the W step in --iteration")
    ap.add_argument("--scgw", action="store_true",
                    help="run self-consistent GW cycles on the chosen config's cell (FP64) and exit")
    ap.add_argument("--scgw-cycles", type=int, default=5)
    ap.add_argument("--scgw-v-scale", type=float, default=0.01, help="bare interaction scale of --scgw")
    ap.add_argument("--requests", type=int, default=200, help="requests of --serve")
    ap.add_argument("--serve-requests", type=int, default=40,
                    help="requests of the bounded serving leg of the step benchmark (0: none)")
    ap.add_argument("--slots", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    import torch
    import synthcell as sc
    import paper_1911_05633_amd as g

    if args.copy_ref > 0:
        copy_reference(args.copy_ref, torch, log)
        return
    if args.serve:
        serve_bench(args, torch, log)
        return
    if args.pairs:
        pairs_bench(args, torch, log)
        return
    if args.dyson:
        dyson_bench(args, torch, log)
        return
    if args.interstitial:
        interstitial_bench(args, torch, log)
        return
    if args.iteration:
        iteration_bench(args, torch, log)
        return
    if args.scgw:
        scgw_bench(args, torch, log)
        return
    spec = sc.config(args.config)
    log(f"config {args.config}: {spec.name}, {spec.n_atoms} atoms, N_orb {spec.N_orb}, N_pb {spec.N_pb}, "
        f"N_R {spec.N_R}, n_tau {spec.n_tau}, prec {args.prec}")
    fp, fs = pair_flops(spec)
    d, cell, ms, per = time_path(g, spec, args.prec, args.steps, args.warmup, torch, log)
    total_flops = (fp + fs) * spec.n_tau * spec.N_R
    roofs = kernel_roofs(spec, args.prec, fp, fs)
    entries, step_roof = roofline_entries(roofs, per, args.prec, ms)
    dom = max(per, key=per.get)
    de = entries[dom]
    n_val = float(d["n"].cpu()[0])
    dtype = {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64"}[args.prec]
    out = {
        "metric": f"P+Sigma GFLOP/s per scGW step ({spec.n_atoms}-atom cell); frac of the kernels' rooflines; "
                  f"p50/p99 latency of the serving mix",
        "value": total_flops / (ms * 1e-3) / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{spec.name}: {spec.n_atoms} atoms, n_orb {spec.n_orb}, n_pb {spec.n_pb}, "
                               f"mesh {'x'.join(map(str, spec.mesh))}, n_tau {spec.n_tau}, beta {spec.beta}",
                   "precision": args.prec, "per_kernel_ms": per, "electron_count": n_val},
        "roofline": {"kernel": dom, "bound": de["bound"], "achieved": de["achieved"], "peak": de["peak"],
                     "unit": de["unit"], "frac": de["frac"], "traffic": de["traffic"]},
        "roofline_per_kernel": entries,
        "roofline_step": step_roof,
    }
    smp = None
    if not args.no_cpu:
        smp = oracle_sample(spec, d, log)
        out["cpu_baseline"] = cpu_baseline(spec, smp, fp, fs)
        out["config"]["error_vs_oracle"] = slice_error(g, cell, d, spec, args.prec, smp, log)
    del d, cell
    torch.cuda.empty_cache()
    # the other mixed-precision path, then the plain FP64 path, on the same inputs
    others = [] if args.no_fp64 else [x for x in ("fp32", "bf16x3") if x != args.prec] + ["fp64"]
    if args.prec == "fp64":
        others = []
    for alt in others:
        da, cella, msa, pera = time_path(g, spec, alt, max(1, min(args.steps, 3)), 2, torch, log)
        out["config"][f"{alt}_ms_per_step"] = msa
        out["config"][f"{alt}_per_kernel_ms"] = pera
        out["config"][f"speedup_vs_{alt}"] = msa / ms
        if smp is not None:
            out["config"][f"{alt}_error_vs_oracle"] = slice_error(g, cella, da, spec, alt, smp, log)
        del da, cella
        torch.cuda.empty_cache()
    if args.serve_requests > 0:
        out["serving"] = serve_runs(args.serve_requests, args.slots, torch, log)
        out["p50_ms"], out["p99_ms"] = out["serving"]["p50_ms"], out["serving"]["p99_ms"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
