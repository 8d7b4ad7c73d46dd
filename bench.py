#!/usr/bin/env python3
"""Benchmark of the chi0 -> Dyson -> S(q,w) -> F(q,tau) path on one MI355X.

One step = the whole hot path for every q of the workload with the states
already resident in HBM: transitions, pair densities, chi0, K = v + f_xc,
Dyson, S, F.  The headline value is the chi0 contraction's algorithmic
throughput, F_alg = 8 N_w N_G^2 T(q) flops per launch, divided by the chi0
launch time measured with HIP events on the launch stream.  Comparison legs
run the FP64 and FP32 contractions on the first q and report the error of
the chosen form's S and F against the FP64 path.  The FP64 oracle runs on a
bounded sample of the same crystal (q0 on a 4^3 grid, every tenth
frequency): its chi0 step is the CPU baseline, and the GPU path on the same
sample gives the errors of S and F against the oracle in every precision.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"bf16x3": 2516.0, "fp32": 157.3, "fp64": 78.6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def f_alg(n_w, n_g, n_t):
    return 8.0 * n_w * n_g * n_g * n_t


def kernel(tdx, ctx, w, st, qj, gb, fx):
    """K for one q; the q-independent f_xc(G) grid is computed once per
    temperature within one step (fx holds it) and reused for every q."""
    if w.xc == "rpa":
        return tdx.kernel_matrix_from_grid(ctx, st, qj, gb, w.xc)
    if st.temperature not in fx:
        fx[st.temperature] = tdx.xc_kernel_grid(ctx, st, w.dens_grid)
    return tdx.kernel_matrix_from_grid(ctx, st, qj, gb, w.xc, w.dens_grid, fx[st.temperature])


def run_step(tdx, ctx, w, st, setup, prec, qs, torch, keep=False, paired=True):
    """One pass of the path over the q indices `qs`, one chi0 launch per q,
    chi0 bracketed by events (used for the comparison legs)."""
    stream = torch.cuda.current_stream()
    out, fx = [], {}
    for iq in qs:
        T = w.temperatures[iq]
        if st.temperature != T:
            tdx.occupations(ctx, st, T, w.n_electrons, w.f_trunc)
        gb, i_g0, om, tau = setup[iq]
        qj = tuple(w.qs[iq])
        tr = tdx.transitions(ctx, st, qj, w.f_trans_thr, paired=paired)
        P = tdx.pair_density(ctx, st, qj, tr, gb, prec)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        c0 = tdx.chi0(ctx, tr, P, gb.shape[0], prec, om, w.eta, st.chi0_pref)
        e1.record(stream)
        del P
        K = kernel(tdx, ctx, w, st, qj, gb, fx)
        c00 = tdx.dyson(ctx, c0, K, i_g0)
        beta = 1.0 / T
        S = tdx.dsf(ctx, c00, om, beta, st.density)
        F = tdx.itcf(ctx, S, om, beta, tau)
        out.append(dict(iq=iq, n_t=len(tr), n_g=gb.shape[0], n_w=om.shape[0], ev=(e0, e1),
                        S=S if keep else None, F=F if keep else None))
        del c0
    return out


class BatchedStep:
    """The benchmark step: transitions and pair densities of every q into
    fixed buffers, chi0 for every q (one grid launch per q, or with
    persistent=True ONE persistent launch for all q from a plan built once),
    then K, Dyson, S and F per q.  paired: time-reversal paired transition
    lists (half the transitions contracted)."""

    def __init__(self, tdx, ctx, w, st, setup, prec, torch, persistent=False, paired=True):
        self.tdx, self.ctx, self.w, self.st, self.setup, self.prec = tdx, ctx, w, st, setup, prec
        self.torch, self.persistent, self.paired = torch, persistent, paired
        self.tr, self.P, self.items = [], [], []
        pref = st.chi0_pref
        for iq in range(len(w.qs)):
            self._occ(iq)
            gb, i_g0, om, tau = setup[iq]
            tr = tdx.transitions(ctx, st, w.qs[iq], w.f_trans_thr, paired=paired)
            P = tdx.pair_density(ctx, st, w.qs[iq], tr, gb, prec)
            self.tr.append(tr)
            self.P.append(P)
            self.items.append(tdx.Chi0Item(tr, P, gb.shape[0], om, w.eta, pref))
        self.plan = tdx.Chi0Plan(ctx, self.items, prec)

    def _occ(self, iq):
        T = self.w.temperatures[iq]
        if self.st.temperature != T:
            self.tdx.occupations(self.ctx, self.st, T, self.w.n_electrons, self.w.f_trunc)

    def __call__(self, keep=False):
        tdx, ctx, w, st, torch = self.tdx, self.ctx, self.w, self.st, self.torch
        for iq in range(len(w.qs)):
            self._occ(iq)
            gb = self.setup[iq][0]
            n0 = len(self.tr[iq])
            tr = tdx.transitions(ctx, st, w.qs[iq], w.f_trans_thr, out=self.tr[iq],
                                 paired=self.paired)
            assert tr is self.tr[iq] and len(tr) == n0
            tdx.pair_density(ctx, st, w.qs[iq], tr, gb, self.prec, out=self.P[iq])
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if self.persistent:
            self.plan.launch()
        else:
            for it in self.items:
                tdx.chi0(ctx, it.tr, it.P, it.out.shape[1], self.prec, it.omega, w.eta,
                         it.c.pref, out=it.out)
        e1.record(stream)
        out, fx = [], {}
        for iq in range(len(w.qs)):
            self._occ(iq)
            gb, i_g0, om, tau = self.setup[iq]
            T = w.temperatures[iq]
            K = kernel(tdx, ctx, w, st, w.qs[iq], gb, fx)
            c00 = tdx.dyson(ctx, self.items[iq].out, K, i_g0)
            S = tdx.dsf(ctx, c00, om, 1.0 / T, st.density)
            F = tdx.itcf(ctx, S, om, 1.0 / T, tau)
            out.append(dict(iq=iq, n_t=len(self.tr[iq]), n_g=gb.shape[0], n_w=om.shape[0],
                            S=S if keep else None, F=F if keep else None))
        return out, (e0, e1)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "counters_k_chi0_bf16x3_fcc_c2.md")
TRAFFIC_SOURCES = ["paper_2510_01875_amd/csrc/chi0_bf16x3.hip",
                   "paper_2510_01875_amd/csrc/chi0_batch.hip",
                   "paper_2510_01875_amd/csrc/chi0_batch.h",
                   "paper_2510_01875_amd/csrc/chi0_tile.h",
                   "paper_2510_01875_amd/csrc/pair_density.hip"]


def measured_traffic(workload, prec):
    """HBM bytes per step of the split-BF16 chi0 launches from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary (scaled by the plain-copy
    calibration), or None if that summary was taken on other kernel sources
    or another workload."""
    if workload != "fcc_c2" or prec != "bf16x3" or not os.path.exists(TRAFFIC_PROFILE):
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    rec = {}
    with open(TRAFFIC_PROFILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith(("#", "|", "-", "`")):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    if rec.get("kernel_sources_sha256_16") != h.hexdigest()[:16]:
        return None
    return float(rec["traffic_bytes_per_step"])


def errors(S, Sref, F, Fref):
    S, Sref, F, Fref = (np.asarray(x) for x in (S, Sref, F, Fref))
    norm = float(np.max(np.abs(S - Sref)) / np.max(np.abs(Sref)))
    m = Sref > 1e-3 * Sref.max()
    point = float(np.max(np.abs(S[m] - Sref[m]) / Sref[m]))
    ferr = float(np.max(np.abs(F - Fref) / np.abs(Fref)))
    return {"S_max_rel_normwise": norm, "S_max_rel_pointwise": point, "F_max_rel": ferr}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_sample(w, n_w_sample=50):
    """The FP64 oracle on a bounded sample of the workload: the same crystal
    and q0 on a 4^3 grid (the q vector is unchanged), every tenth frequency;
    states, transitions, pair densities, chi0 (timed on all BLAS threads and,
    on a tenth of those frequencies, on one), K, Dyson, S and F.  Returns the
    cpu_baseline record, the sample workload and the oracle's S and F."""
    import oracle
    from oracle import response
    from threadpoolctl import threadpool_info, threadpool_limits
    cores = max([i.get("num_threads", 1) for i in threadpool_info()
                 if i.get("user_api") == "blas"] or [os.cpu_count()])
    N = np.asarray(w.kgrid)
    small = (4, 4, 4)
    qj = tuple(int(x) for x in np.asarray(w.qs[0]) * np.asarray(small) // N)
    om = w.omega_grid(0)[:: max(1, w.n_omega // n_w_sample)]
    ws = w.with_(name=w.name + "_k4", kgrid=small, qs=(qj,), temperatures=w.temperatures[:1],
                 ecut_chi=w.ecut_chi[:1], omega_max=w.omega_max[:1])
    st = oracle.build_states(ws)
    r = oracle.run_q(ws, st, 0, omegas=om)
    t0 = time.perf_counter()
    response.chi0(r.tr, r.P, om, ws.eta, st.n_k, st.omega)
    dt = time.perf_counter() - t0
    om1 = om[:: 5]
    with threadpool_limits(limits=1, user_api="blas"):
        t0 = time.perf_counter()
        response.chi0(r.tr, r.P, om1, ws.eta, st.n_k, st.omega)
        dt1 = time.perf_counter() - t0
    nb = len(r.basis)
    fl, fl1 = f_alg(len(om), nb, len(r.tr)), f_alg(len(om1), nb, len(r.tr))
    base = {"value": fl / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
            "cpu_model": cpu_model(),
            "one_thread": {"value": fl1 / dt1 / 1e12, "unit": "TFLOP/s", "cores": 1,
                           "n_omega": len(om1), "seconds": dt1},
            "sample": (f"{w.name} crystal and q0 on a 4^3 k-grid (T={len(r.tr)} transitions, "
                       f"full list; N_G={nb}), {len(om)} of {w.n_omega} frequencies; FP64 "
                       f"NumPy chi0 step {dt:.2f} s on {cores} BLAS threads, "
                       f"{len(om1)} frequencies {dt1:.2f} s on one"),
            "seconds": dt}
    return base, ws, om, r


def gpu_vs_oracle(tdx, ctx, ws, om, r, precs, paired):
    """The GPU path on the oracle's sample (same states model, q, frequencies
    and tau grid) in each precision: max relative errors of S and F against
    the oracle's."""
    import torch
    st = tdx.build_states(ctx, ws)
    out = {}
    for prec in precs:
        g = tdx.run_q(ctx, ws, st, 0, prec=prec, omega=om, keep_chi0=False, paired=paired)
        out[prec] = errors(g.S.cpu().numpy(), r.S, g.F.cpu().numpy(), r.F)
        del g
    torch.cuda.synchronize()
    del st
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fcc_c2")
    ap.add_argument("--prec", default="bf16x3", choices=["bf16x3", "fp32", "fp64"])
    ap.add_argument("--compare", default="fp64,fp32",
                    help="precisions timed on the first q for comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pairing", action="store_true",
                    help="contract the full transition list instead of one transition per "
                         "time-reversal pair")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the split-BF16 tile shape on q0 first and save the cache")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2510_01875_amd",
                                                         "tune_gfx950.json"),
                    help="tile cache read when not tuning")
    ap.add_argument("--tune-save", default=None,
                    help="where --autotune writes its cache (default: --tune-cache)")
    ap.add_argument("--eta-scan", type=int, default=8,
                    help="also time the eta-convergence test (Sec. 2) on q0 over this many "
                         "eta (powers of two around the workload's eta; 0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (out = in * 1.0, "
                         "five launches): the reference kernel for scaling HBM byte counters")
    args = ap.parse_args()
    if args.copy_probe_mib:
        import torch
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe": {"bytes_read": n * 8, "bytes_written": n * 8,
                                         "launches": 5}}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); across GPUs the path "
              "would split the q-vectors, or the frequencies of one q, with no exchange "
              "inside the chi0 step", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2510_01875_amd as tdx
    import workloads

    w = workloads.get(args.workload)
    ctx = tdx.Context(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = tdx.build_states(ctx, w, w.temperatures[0])
    torch.cuda.synchronize()
    t_states = time.perf_counter() - t0
    log(f"states: {st.n_k} k, {t_states:.2f} s")
    setup = []
    for iq in range(len(w.qs)):
        b, g0 = tdx.response_basis(w.cell, w.kgrid, w.qs[iq], w.ecut_chi[iq])
        setup.append((torch.from_numpy(b).cuda(), g0,
                      torch.as_tensor(w.omega_grid(iq), device="cuda"),
                      torch.as_tensor(w.tau_grid(iq), device="cuda")))
    qs = list(range(len(w.qs)))
    paired = not args.no_pairing
    tuned = None
    if args.prec == "bf16x3":
        if args.autotune:
            b0 = setup[0][0]
            tr0 = tdx.transitions(ctx, st, w.qs[0], w.f_trans_thr, paired=paired)
            P0 = tdx.pair_density(ctx, st, w.qs[0], tr0, b0, "bf16x3")
            probe = tdx.Chi0Item(tr0, P0, b0.shape[0], setup[0][2], w.eta,
                                 st.chi0_pref)
            v, sl, ms = tdx.autotune_chi0(ctx, probe, max_trans=1 << 22)
            tuned = {"variant": v, "slice_log2": sl, "probe_ms": ms, "source": "autotuned now"}
            out = args.tune_save or args.tune_cache
            os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
            tdx.tune_save(ctx, out)
            del P0, tr0, probe
            log(f"autotune: variant {v}, slice 2^{sl}, {ms:.1f} ms on the probe")
        elif os.path.exists(args.tune_cache):
            tdx.tune_load(ctx, args.tune_cache)
            tuned = {"source": os.path.basename(args.tune_cache)}
        v, sl = tdx.chi0_get_config(ctx, setup[0][0].shape[0])
        tuned = dict(tuned or {"source": "default"}, variant=v, slice_log2=sl)

    step = BatchedStep(tdx, ctx, w, st, setup, args.prec, torch, paired=paired)
    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs, evs = [], []
    for i in range(args.steps):
        r, ev = step(keep=(i == 0))
        recs += r
        evs.append(ev)
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0

    launch_ms = [e0.elapsed_time(e1) for e0, e1 in evs]
    flops_step = sum(f_alg(r["n_w"], r["n_g"], r["n_t"]) for r in recs[: len(qs)])
    tflops = flops_step / (sum(launch_ms) / len(launch_ms) * 1e-3) / 1e12
    n_eval = sum(r["n_w"] for r in recs)
    main_q0 = next(r for r in recs if r["iq"] == 0 and r["S"] is not None)
    # the same step with one persistent launch for all q (ragged-batch form)
    step.persistent = True
    step()
    torch.cuda.synchronize()
    _, (p0, p1) = step()
    torch.cuda.synchronize()
    pers_ms = p0.elapsed_time(p1)
    log(f"persistent batch: {pers_ms:.1f} ms")
    step.plan.close()
    del step

    legs = {}
    for prec in [p for p in args.compare.split(",") if p and p != args.prec]:
        torch.cuda.synchronize()
        r = run_step(tdx, ctx, w, st, setup, prec, [0], torch, keep=True, paired=paired)[0]
        torch.cuda.synchronize()
        ms = r["ev"][0].elapsed_time(r["ev"][1])
        legs[prec] = {"chi0_tflops": f_alg(r["n_w"], r["n_g"], r["n_t"]) / (ms * 1e-3) / 1e12,
                      "chi0_ms_q0": ms, "S": r["S"].cpu().numpy(), "F": r["F"].cpu().numpy()}
        log(f"leg {prec}: chi0 {ms:.1f} ms, {legs[prec]['chi0_tflops']:.2f} TFLOP/s")
    err = None
    if "fp64" in legs:
        err = errors(main_q0["S"].cpu().numpy(), legs["fp64"]["S"], main_q0["F"].cpu().numpy(),
                     legs["fp64"]["F"])
        if "fp32" in legs:
            err["fp32"] = errors(legs["fp32"]["S"], legs["fp64"]["S"], legs["fp32"]["F"],
                                 legs["fp64"]["F"])

    eta_info = None
    if args.prec == "bf16x3" and args.eta_scan > 0:
        k = args.eta_scan
        etas = w.eta * 2.0 ** np.arange(-(k // 2), k - k // 2)
        tdx.eta_scan(ctx, w, st, 0, etas, prec=args.prec, paired=paired)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        es = tdx.eta_scan(ctx, w, st, 0, etas, prec=args.prec, paired=paired)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        n_w0, n_g0 = int(es.omega.shape[0]), int(setup[0][0].shape[0])
        eta_info = {
            "n_eta": k, "eta_ha": etas.tolist(), "ms": dt * 1e3,
            "s_eval_per_s": k * n_w0 / dt,
            "chi0_tflops_whole_scan": k * f_alg(n_w0, n_g0, es.n_trans) / dt / 1e12,
            "reference_eta_ha": float(etas[es.ref_index]), "tol": 1e-2,
            "metrics": {"columns": list(tdx.METRICS), "rows": es.metrics.tolist()},
            "form": "q0: transitions, pair densities, one persistent chi0 launch for all eta, "
                    "then Dyson, S, F and the metrics per eta (whole scan timed)"}
        log(f"eta scan: {k} eta in {dt * 1e3:.0f} ms, reference eta {etas[es.ref_index]:.4f}")
        del es

    # dielectric properties of q0 from its S (Kramers-Kronig on the grid)
    stream = torch.cuda.current_stream()
    d0, d1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    om0 = setup[0][2]
    q2 = tdx.q_squared(w.cell, w.kgrid, w.qs[0])
    beta0, dens0 = 1.0 / w.temperatures[0], st.density
    tdx.dielectric(ctx, main_q0["S"], om0, beta0, dens0, q2)
    d0.record(stream)
    tdx.dielectric(ctx, main_q0["S"], om0, beta0, dens0, q2)
    d1.record(stream)
    torch.cuda.synchronize()
    diel = {"ms": d0.elapsed_time(d1), "n_w": int(om0.shape[0]),
            "form": "q0: Im chi by the FDT, Re chi by Kramers-Kronig over the grid, eps^-1, sigma"}

    # attenuation of narrow-band fluctuations on q0's S: the two strongest
    # peaks of the spectrum of dS/dw as targets, then the whole grid search
    # (filter bank, scores, F of every filtered S, residual conditions,
    # per-degree selection)
    tau0 = setup[0][3]
    span = float(om0[-1] - om0[0])
    nus = torch.linspace(4.0 / span, 0.25 * (om0.shape[0] - 1) / span, 400,
                         dtype=torch.float64, device="cuda")
    psd = tdx.derivative_psd(ctx, main_q0["S"], om0, nus).cpu().numpy()[0]
    peaks = [i for i in range(1, len(psd) - 1) if psd[i] >= psd[i - 1] and psd[i] > psd[i + 1]]
    peaks = sorted(peaks, key=lambda i: -psd[i])[:2]
    targets = nus[torch.as_tensor(sorted(peaks), dtype=torch.long, device="cuda")]
    pairs = [(x, p) for p in range(1, 7) for x in range(5, 62, 4) if x > p]
    windows, degrees = [x for x, _ in pairs], [p for _, p in pairs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    at = tdx.attenuate(ctx, main_q0["S"], om0, beta0, tau0, windows, degrees, targets)
    torch.cuda.synchronize()
    dt_att = time.perf_counter() - t0
    atten = {"ms": dt_att * 1e3, "n_filters": len(windows), "n_w": int(om0.shape[0]),
             "targets_per_ha": targets.cpu().tolist(),
             "selected": {str(p): ([windows[b], p] if b >= 0 else None)
                          for p, b in at.best.items()},
             "form": "q0: filter bank, scores, F of each filtered S, residual ITCF "
                     "conditions and per-degree selection (whole search timed)"}
    log(f"attenuation: {len(windows)} filters in {dt_att * 1e3:.1f} ms")

    per_launch = flops_step
    avg_ms = sum(launch_ms) / len(launch_ms)
    line = {
        "metric": "chi0 TFLOP/s + S(q,w) eval/s at stated error vs FP64, plain vs split-BF16",
        "value": tflops,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic (seeded model crystal; no paper data)",
        "config": {"workload": w.name, "kgrid": list(w.kgrid), "n_bands": w.n_bands,
                   "n_q": len(w.qs), "n_omega": w.n_omega,
                   "n_g": [int(s_[0].shape[0]) for s_ in setup],
                   "n_trans": [r["n_t"] for r in recs[: len(qs)]],
                   "transitions": ("one per time-reversal pair (n_trans contracted, about "
                                   "half the screened set)" if paired else "full screened set"),
                   "xc": w.xc,
                   "chi0_launch": "one grid launch per q", "tile": tuned},
        "s_eval_per_s": n_eval / t_total,
        "chi0_ms_per_step": launch_ms,
        "persistent_batch": {"chi0_ms": pers_ms, "tflops": flops_step / (pers_ms * 1e-3) / 1e12,
                             "form": "one persistent launch for all q"},
        "build_states_s": t_states,
        "plain": {p: {"chi0_tflops": v["chi0_tflops"], "chi0_ms_q0": v["chi0_ms_q0"]}
                  for p, v in legs.items()},
        "error_vs_fp64": err,
        "eta_scan": eta_info,
        "dielectric": diel,
        "attenuation": atten,
        "roofline": {"bound": "mfma", "achieved": per_launch / (avg_ms * 1e-3) / 1e12,
                     "peak": PEAK_TFLOPS[args.prec], "unit": "TFLOP/s",
                     "frac": per_launch / (avg_ms * 1e-3) / 1e12 / PEAK_TFLOPS[args.prec],
                     "traffic": measured_traffic(w.name, args.prec),
                     "kernel": {"bf16x3": "k_chi0_bf16x3", "fp32": "k_chi0_fp<float>",
                                "fp64": "k_chi0_fp<double>"}[args.prec],
                     "issued_mfma_frac": (3.0 if args.prec == "bf16x3" else 1.0)
                     * per_launch / (avg_ms * 1e-3) / 1e12 / PEAK_TFLOPS[args.prec]},
    }
    if not args.no_cpu_baseline:
        log("oracle sample ...")
        base, ws, om_s, r_s = oracle_sample(w)
        line["cpu_baseline"] = base
        precs = [args.prec] + [p for p in args.compare.split(",") if p and p != args.prec]
        line["error_vs_oracle"] = dict(
            gpu_vs_oracle(tdx, ctx, ws, om_s, r_s, precs, paired),
            sample=base["sample"].split(";")[0] + "; S normwise and pointwise "
            "(S > 1e-3 max S), F pointwise, GPU and oracle on the same sample")
        log(f"errors vs oracle: {line['error_vs_oracle']}")
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
