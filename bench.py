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
    """HBM bytes per launch (one q, averaged over the step's launches) of the
    split-BF16 chi0 kernel from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary (scaled by the plain-copy calibration), or None if that summary
    was taken on other kernel sources or another workload."""
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
    return float(rec["traffic_bytes_per_launch"])


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


def c1_leg(tdx, ctx):
    """The free-electron configuration (feg_c1: 8^3 k, 56 bands on plane
    waves to 10 Ha, 200 frequencies, RPA, one q): states, then the whole
    step (transitions, pair densities, chi0, K, Dyson, S, F) in FP64 and in
    split-BF16, each timed after a warm-up; the split-BF16 S and F against
    the FP64 ones."""
    import torch
    import workloads
    w = workloads.feg_c1()
    t0 = time.perf_counter()
    st = tdx.build_states(ctx, w, w.temperatures[0])
    torch.cuda.synchronize()
    t_states = time.perf_counter() - t0
    out = {"workload": w.name, "kgrid": list(w.kgrid), "n_omega": w.n_omega,
           "build_states_s": t_states}
    res = {}
    for prec in ("fp64", "bf16x3"):
        tdx.run_q(ctx, w, st, 0, prec=prec, keep_chi0=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = tdx.run_q(ctx, w, st, 0, prec=prec, keep_chi0=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[prec] = r
        out[prec] = {"step_ms": dt * 1e3, "s_eval_per_s": w.n_omega / dt,
                     "n_trans": r.n_trans, "n_g": len(r.basis)}
    out["error_vs_fp64"] = errors(res["bf16x3"].S.cpu().numpy(), res["fp64"].S.cpu().numpy(),
                                  res["bf16x3"].F.cpu().numpy(), res["fp64"].F.cpu().numpy())
    return out


def h16_leg(tdx, ctx, sample_every=50):
    """The 16-proton system at full size (h16_c3: 64 k, about 6290 plane waves
    and 860 bands per k, 304 G, 1000 frequencies on [0, 5] Ha, RPA): q0 with
    split-BF16 chi0 and FP64 Dyson, states built once (timed apart).  The
    step (pair densities, chi0, K, Dyson, S, F) is timed as a whole and the
    chi0 launch with HIP events on its stream.  The FP64 contraction then
    runs on every sample_every-th frequency, and S and F (the latter on that
    coarse grid, for both) of the split-BF16 path are compared with it."""
    import torch
    import workloads
    w = workloads.h16_c3()
    t0 = time.perf_counter()
    st = tdx.build_states(ctx, w, w.temperatures[0])
    torch.cuda.synchronize()
    t_states = time.perf_counter() - t0
    qj = w.qs[0]
    basis, g0 = tdx.response_basis(w.cell, w.kgrid, qj, w.ecut_chi[0])
    n_g = len(basis)
    gb = torch.from_numpy(basis).cuda()
    om = torch.as_tensor(w.omega_grid(0), device="cuda")
    tau = torch.as_tensor(w.tau_grid(0), device="cuda")
    stream = torch.cuda.current_stream()

    def step(prec, omega):
        tr = tdx.transitions(ctx, st, qj, w.f_trans_thr, paired=True)
        P = tdx.pair_density(ctx, st, qj, tr, gb, prec)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        c0 = tdx.chi0(ctx, tr, P, n_g, prec, omega, w.eta, st.chi0_pref)
        e1.record(stream)
        del P
        K = tdx.kernel_matrix_from_grid(ctx, st, qj, gb, w.xc)
        c00 = tdx.dyson(ctx, c0, K, g0)
        S = tdx.dsf(ctx, c00, omega, st.beta, st.density)
        return len(tr), (e0, e1), c00, S

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_t, ev, c00, S = step("bf16x3", om)
    F = tdx.itcf(ctx, S, om, st.beta, tau)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = ev[0].elapsed_time(ev[1])
    fl = f_alg(om.shape[0], n_g, n_t)
    sub = om[::sample_every].contiguous()
    _, ev64, _, S64 = step("fp64", sub)
    torch.cuda.synchronize()
    ms64 = ev64[0].elapsed_time(ev64[1])
    # both paths through S and F on the same coarse grid (S(0) is taken from
    # the grid's next point, so it depends on the grid)
    S_sub = tdx.dsf(ctx, c00[::sample_every].contiguous(), sub, st.beta, st.density)
    F_sub = tdx.itcf(ctx, S_sub, sub, st.beta, tau).cpu().numpy()
    F64 = tdx.itcf(ctx, S64, sub, st.beta, tau).cpu().numpy()
    err = errors(S_sub.cpu().numpy(), S64.cpu().numpy(), F_sub, F64)
    del st
    torch.cuda.empty_cache()
    return {"workload": w.name, "kgrid": list(w.kgrid), "n_bands": w.n_bands, "n_g": n_g,
            "n_omega": int(om.shape[0]), "n_trans": n_t,
            "transitions": "one per time-reversal pair", "dtype": "bf16x3 chi0, FP64 Dyson",
            "build_states_s": t_states, "step_s": dt,
            "s_eval_per_s": int(om.shape[0]) / dt,
            "chi0_ms": ms, "chi0_tflops": fl / (ms * 1e-3) / 1e12,
            "roofline": {"bound": "mfma", "achieved": fl / (ms * 1e-3) / 1e12,
                         "peak": PEAK_TFLOPS["bf16x3"], "unit": "TFLOP/s",
                         "frac": fl / (ms * 1e-3) / 1e12 / PEAK_TFLOPS["bf16x3"]},
            "fp64_sampled": {"n_omega": int(sub.shape[0]), "chi0_ms": ms64,
                             "chi0_tflops": f_alg(sub.shape[0], n_g, n_t) / (ms64 * 1e-3) / 1e12},
            "error_vs_fp64_sampled": err}


def batched_graph_run(tdx, ctx, w, args, budget_bytes=200 << 30, slice_log2=22):
    """A ragged batch of q (fcc_c4: 32 q, per-q temperature and basis) at full
    size: the q are packed longest first into groups whose split-BF16 pair
    densities, chi0 slice partials and outputs fit the budget; each group is
    ONE HIP graph holding pair densities -> one persistent chi0 launch ->
    Dyson -> S -> F for all its q, captured once and replayed once (timed
    with events around the replay).  States, occupations, transition lists,
    f_xc grids and K are set up before the timed graphs."""
    import torch
    t0 = time.perf_counter()
    st = tdx.build_states(ctx, w, w.temperatures[0])
    torch.cuda.synchronize()
    t_states = time.perf_counter() - t0
    log(f"states: {st.n_k} k, {t_states:.1f} s")
    tdx.chi0_set_slice_length(ctx, 1 << slice_log2)
    fx, qs = {}, []
    for iq in range(len(w.qs)):
        T = w.temperatures[iq]
        if st.temperature != T:
            tdx.occupations(ctx, st, T, w.n_electrons, w.f_trunc)
        if T not in fx:
            fx[T] = tdx.xc_kernel_grid(ctx, st, w.dens_grid)
        basis, g0 = tdx.response_basis(w.cell, w.kgrid, w.qs[iq], w.ecut_chi[iq])
        n_g = len(basis)
        gb = torch.from_numpy(basis).cuda()
        tr = tdx.transitions(ctx, st, w.qs[iq], w.f_trans_thr, paired=True)
        K = tdx.kernel_matrix_from_grid(ctx, st, w.qs[iq], gb, w.xc, w.dens_grid, fx[T])
        n_w = w.n_omega
        per = n_w * n_g * n_g * 16
        slices = max(1, -(-len(tr) // (1 << slice_log2)))
        nbytes = (tdx.pair_density_bytes(len(tr), n_g, "bf16x3") + (slices + 2) * per +
                  tdx.pair_density_work_bytes(st, len(tr)))
        qs.append(dict(iq=iq, T=T, beta=1.0 / T, g0=g0, gb=gb, tr=tr, K=K, n_g=n_g, n_w=n_w,
                       bytes=nbytes, n_t=len(tr)))
    dens = st.density
    order = sorted(qs, key=lambda q: -q["bytes"])
    groups, cur, used = [], [], 0
    for q in order:
        if cur and used + q["bytes"] > budget_bytes:
            groups.append(cur)
            cur, used = [], 0
        cur.append(q)
        used += q["bytes"]
    if cur:
        groups.append(cur)
    log(f"{len(qs)} q in {len(groups)} groups; transitions {min(q['n_t'] for q in qs)} .. "
        f"{max(q['n_t'] for q in qs)}")
    stream = torch.cuda.current_stream()
    recs, total_ms, total_flops, n_eval = [], 0.0, 0.0, 0
    S_out = {}
    for gi, grp in enumerate(groups):
        torch.cuda.empty_cache()
        items = []
        for q in grp:
            q["P"] = torch.empty(tdx.pair_density_bytes(q["n_t"], q["n_g"], "bf16x3"),
                                 dtype=torch.uint8, device="cuda")
            q["pdw"] = torch.empty(tdx.pair_density_work_bytes(st, q["n_t"]), dtype=torch.uint8,
                                   device="cuda")
            q["om"] = torch.as_tensor(w.omega_grid(q["iq"]), device="cuda")
            q["tau"] = torch.as_tensor(w.tau_grid(q["iq"]), device="cuda")
            q["dw"] = torch.empty(tdx.dyson_work_bytes(q["n_g"], q["n_w"]), dtype=torch.uint8,
                                  device="cuda")
            q["info"] = torch.zeros(q["n_w"], dtype=torch.int32, device="cuda")
            q["chi00"] = torch.empty(q["n_w"], dtype=torch.complex128, device="cuda")
            q["item"] = tdx.Chi0Item(q["tr"], q["P"], q["n_g"], q["om"], w.eta, st.chi0_pref)
            items.append(q["item"])
        plan = tdx.Chi0Plan(ctx, items, "bf16x3")

        def body():
            for q in grp:
                tdx.pair_density_async(ctx, st, w.qs[q["iq"]], q["tr"], q["gb"], q["P"], q["pdw"],
                                       "bf16x3")
            plan.launch()
            outs = []
            for q in grp:
                tdx.dyson_async(ctx, q["item"].out, q["K"], q["g0"], q["chi00"], q["dw"], q["info"])
                S = tdx.dsf(ctx, q["chi00"], q["om"], q["beta"], dens)
                outs.append((S, tdx.itcf(ctx, S, q["om"], q["beta"], q["tau"])))
            return outs

        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            captured = body()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        fl = sum(f_alg(q["n_w"], q["n_g"], q["n_t"]) for q in grp)
        bad = sum(int(q["info"].abs().max()) != 0 for q in grp)
        for q, (S, F) in zip(grp, captured):
            S_out[q["iq"]] = (S.cpu().numpy(), F.cpu().numpy())
        total_ms += ms
        total_flops += fl
        n_eval += sum(q["n_w"] for q in grp)
        recs.append({"q": [q["iq"] for q in grp], "n_trans": [q["n_t"] for q in grp],
                     "n_g": [q["n_g"] for q in grp], "graph_ms": ms,
                     "tflops_graph": fl / (ms * 1e-3) / 1e12, "singular": bad,
                     "gib": sum(q["bytes"] for q in grp) / 2 ** 30})
        log(f"group {gi + 1}/{len(groups)}: q {recs[-1]['q']} {ms:.0f} ms "
            f"{recs[-1]['tflops_graph']:.0f} TFLOP/s")
        del g, captured, plan, items
        for q in grp:
            for key in ("P", "pdw", "dw", "item"):
                q.pop(key, None)
    finite = all(np.all(np.isfinite(S)) and np.all(np.isfinite(F)) for S, F in S_out.values())
    line = {
        "metric": "chi0 TFLOP/s + S(q,w) eval/s at stated error vs FP64, plain vs split-BF16",
        "value": total_flops / (total_ms * 1e-3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": total_ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3",
        "data": "synthetic (seeded model crystal; no paper data)",
        "config": {"workload": w.name, "kgrid": list(w.kgrid), "n_q": len(w.qs),
                   "n_omega": w.n_omega, "transitions": "one per time-reversal pair",
                   "form": "groups of q, each one HIP graph: pair densities, one persistent "
                           "chi0 launch, Dyson, S, F; value = F_alg / graph time (pair "
                           "densities and Dyson included)",
                   "slice_log2": slice_log2, "budget_gib": budget_bytes / 2 ** 30},
        "s_eval_per_s": n_eval / (total_ms * 1e-3), "build_states_s": t_states,
        "groups": recs, "all_finite": bool(finite),
        "total_transitions": int(sum(q["n_t"] for q in qs))}
    tdx.chi0_set_slice_length(ctx, 0)
    return line


def gradient_run(tdx, ctx, w, prec="bf16x3"):
    """The gradient workload at its full configuration (h16_c5: the
    16-proton system, 4 q, 1000 frequencies, 64 imaginary times on
    [0, beta/2]): the adjoint of a seeded linear functional of F(q, tau) for
    all q with respect to (T, eta, v_1..v_3), time-reversal paired lists,
    pair densities recomputed block by block in the reverse sweep.  The
    forward chi0 runs in `prec` (the reverse sweep is FP64).  Times the
    forward and the reverse pass (wall clock around synchronised steps)."""
    import torch
    from paper_2510_01875_amd.grad import ChainRunner, itcf_differentiable
    T, eta = w.temperatures[0], w.eta
    v0 = np.array(w.potential.shell_v, dtype=np.float64)
    c = np.random.default_rng(11).standard_normal((len(w.qs), w.n_tau))
    runner = ChainRunner(ctx, w, paired=True, block_bytes=8 << 30, prec=prec)
    Tt = torch.tensor(T, dtype=torch.float64, requires_grad=True)
    et = torch.tensor(eta, dtype=torch.float64, requires_grad=True)
    vt = torch.tensor(v0, dtype=torch.float64, requires_grad=True)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    t0 = time.perf_counter()
    F = itcf_differentiable(ctx, w, Tt, et, vt, runner=runner)
    L = (F.cpu() * torch.as_tensor(c)).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    peak_f = torch.cuda.max_memory_allocated()
    log(f"forward: {len(w.qs)} q, {t1 - t0:.1f} s")
    torch.cuda.reset_peak_memory_stats()
    gT, ge, gv = torch.autograd.grad(L, (Tt, et, vt))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    log(f"reverse: {t2 - t1:.1f} s")
    per_q = runner.saved["per_q"]
    n_t = [len(q["tr"]) for q in per_q]
    n_g = [int(q["gb"].shape[0]) for q in per_q]
    flops = sum(f_alg(w.n_omega, g, t) for g, t in zip(n_g, n_t))
    return {
        "metric": "chi0 TFLOP/s + S(q,w) eval/s at stated error vs FP64, plain vs split-BF16",
        "value": flops / (t1 - t0) / 1e12, "unit": "TFLOP/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": (t2 - t0) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": prec,
        "data": "synthetic (seeded model system; no paper data)",
        "config": {"workload": w.name, "kgrid": list(w.kgrid), "n_q": len(w.qs),
                   "n_omega": w.n_omega, "n_tau": w.n_tau, "n_g": n_g, "n_trans": n_t,
                   "transitions": "one per time-reversal pair",
                   "form": "F(q, tau) for all q and its adjoint in (T, eta, v_1..v_3); value = "
                           "F_alg of the forward chi0 / forward wall time (states, pair "
                           "densities, Dyson, S, F included)"},
        "forward_s": t1 - t0, "reverse_s": t2 - t1,
        "peak_gib": {"forward": peak_f / 2 ** 30,
                     "reverse": torch.cuda.max_memory_allocated() / 2 ** 30},
        "grad": {"T": float(gT), "eta": float(ge), "v": [float(x) for x in gv]},
    }


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
    ap.add_argument("--no-h16", dest="h16", action="store_false",
                    help="skip the 16-proton leg (h16_c3 at full size, q0, 1000 frequencies)")
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
    if args.workload == "fcc_c4":
        line = batched_graph_run(tdx, ctx, w, args)
        ctx.close()
        print(json.dumps(line), flush=True)
        return
    if args.workload == "h16_c5":
        if os.path.exists(args.tune_cache):
            tdx.tune_load(ctx, args.tune_cache)
        line = gradient_run(tdx, ctx, w, args.prec)
        ctx.close()
        print(json.dumps(line), flush=True)
        return
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
            # the FP64 and FP32 tiles of the comparison legs, on the first 2^19
            # transitions of the same probe
            for fp in [p for p in args.compare.split(",") if p in ("fp64", "fp32")]:
                Pf = tdx.pair_density(ctx, st, w.qs[0], tr0, b0, fp, n_trans=1 << 19)
                pf = tdx.Chi0Item(tr0, Pf, b0.shape[0], setup[0][2], w.eta, st.chi0_pref,
                                  n_trans=min(len(tr0), 1 << 19))
                vf, _, msf = tdx.autotune_chi0(ctx, pf, max_trans=1 << 19, prec=fp)
                tuned[fp] = {"variant": vf, "probe_ms": msf}
                log(f"autotune {fp}: variant {vf}, {msf:.1f} ms on the probe")
                del Pf, pf
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

    # the Kubo-Greenwood conductivity of the states (Sec. A.3's input) on
    # q0's positive frequencies, then S* from it
    trk = tdx.transitions(ctx, st, (0, 0, 0), w.f_trans_thr)
    omk = om0[1:].contiguous()
    kw = torch.empty(tdx.kg_work_bytes(len(trk), omk.shape[0]), dtype=torch.uint8, device="cuda")
    tdx.kg_conductivity(ctx, st, omk, w.eta, w.f_trans_thr, tr=trk, work=kw)
    d0.record(stream)
    sig = tdx.kg_conductivity(ctx, st, omk, w.eta, w.f_trans_thr, tr=trk, work=kw)
    Sk = tdx.kg_dsf(ctx, sig, omk, beta0, dens0)
    d1.record(stream)
    torch.cuda.synchronize()
    kg = {"ms": d0.elapsed_time(d1), "n_trans": len(trk), "n_w": int(omk.shape[0]),
          "finite": bool(torch.isfinite(Sk).all()),
          "form": "sigma_KG of the states over the q = 0 transitions (trace average, "
                  "Lorentzian eta), then S*"}
    del trk, kw, sig, Sk

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
        "kubo_greenwood": kg,
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
    log("feg_c1 leg ...")
    line["feg_c1"] = c1_leg(tdx, ctx)
    log(f"feg_c1: FP64 step {line['feg_c1']['fp64']['step_ms']:.1f} ms, split-BF16 "
        f"{line['feg_c1']['bf16x3']['step_ms']:.1f} ms, errors {line['feg_c1']['error_vs_fp64']}")
    if args.h16:
        del st
        torch.cuda.empty_cache()
        log("h16_c3 leg ...")
        line["h16_c3"] = h16_leg(tdx, ctx)
        log(f"h16_c3: {line['h16_c3']['chi0_tflops']:.0f} TFLOP/s, step "
            f"{line['h16_c3']['step_s']:.1f} s, errors {line['h16_c3']['error_vs_fp64_sampled']}")
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
