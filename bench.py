#!/usr/bin/env python3
"""Throughput of the coupled D3Q27 RR-LBM + IBM time step on one MI355X.

Workload: the falling-frame scale case -- a 256 x 256 x 768 box (50.3 M
cells), tau from Re = 100, periodic x/y, free-slip top and bottom, sponge of
61 rows, one tilted oblate ellipsoid (semi-axes 32/32/16) carried by 12,252
surface markers, density ratio 2.7.  A step is the whole Table 1 sequence
(body advance, fused stream + collide, IBM coupling with 4 multi-direct
forcing cycles and force/torque, window test).  Populations start at rest
and live in HBM before timing starts.

Output: one JSON line with MLUPS (cells x steps / s / 1e6) and the HBM
roofline of the dominant kernel (the fused stream + collide): algorithmic
bytes per launch (27 reads + 27 writes per cell) over its average launch
time, measured with events on the library's stream during the timed steps.
FP16 and BF16 storage are reported beside FP32 with their drag difference.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM peak, D3Q27 RR+IBM; FP16-store vs FP32 at equal drag error"
HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stream_collide_ellipsoid256x256x768.txt")
KERNEL_SOURCES = ["paper_2408_15115_amd/csrc/stream_collide.hip", "paper_2408_15115_amd/csrc/lattice.hpp",
                  "paper_2408_15115_amd/csrc/pull.hpp", "paper_2408_15115_amd/csrc/internal.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(storage):
    """HBM bytes per launch of the lattice kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha") != kernel_source_hash():
        return None
    v = kv.get(f"traffic_bytes_{storage}")
    return float(v) if v else None


def timed_steps(S, torch, steps, warmup):
    """Eager step sequence; events on the library stream bracket every
    lattice-kernel launch and the whole timed region."""
    st = S.stream
    for _ in range(warmup):
        S.run(1)
    torch.cuda.synchronize()
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(st)
    for k in range(steps):
        S.body_advance()
        pairs[k][0].record(st)
        S.lbm_step()
        pairs[k][1].record(st)
        S.ibm_couple()
        S.window_shift()
    t1.record(st)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    k1 = [a.elapsed_time(b) for a, b in pairs]
    timed_steps.last_k1 = k1
    return total_ms, sum(k1) / len(k1)


def graph_steps(S, torch, steps):
    """Exactly `steps` coupled steps as replays of a captured 10-step graph
    (2-step when `steps` is not a multiple of 10; graphs hold an even number
    of steps), after one untimed replay; ms per step.  Inside a graph the
    window test of one step and the body advance of the next share a kernel."""
    if steps % 2:
        raise ValueError("graph replay times an even number of steps")
    per = 10 if steps % 10 == 0 else 2
    graph_steps.per = per
    S.graph_capture(per)
    S.graph_launch()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(S.stream)
    for _ in range(steps // per):
        S.graph_launch()
    t1.record(S.stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def copy_bandwidth(T, torch, nbytes=4 << 30, reps=10):
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    T.stream_copy(b, a, nbytes)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        T.stream_copy(b, a, nbytes)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def batch_run(T, W, torch, steps, storage, coupling="auto"):
    """The batched form: 64 independent cases (64^3 .. 192x192x384; spheres,
    spheroids, perturbed spheres) in one context; schedule tuned on whole coupled steps
    (coupling "serial" or "beside" overrides the tuner's choice of where the
    coupling runs, keeping its lattice schedule)."""
    from paper_2408_15115_amd import autotune
    batch = W.batch_cases(64)
    cases = [c for c, _ in batch]
    bodies = [b for _, b in batch]
    if storage == "mom":   # moment storage has one schedule: the z-marching column tiles
        tuned = {"best": {}, "cached": False}
    else:
        tuned = autotune.tune_step(cases, bodies, storage=storage)
        log(f"batch: schedule {tuned['best']} ({'cached' if tuned['cached'] else 'tuned'} on whole steps, "
            f"{tuned['ms']:.3f} ms per step, lattice kernel alone {tuned['lattice_ms']:.3f} ms)")
    best = dict(tuned["best"])
    if coupling in ("serial", "beside"):
        best["serial_ibm"] = 1 if coupling == "serial" else 0
    S = T.Solver(cases, bodies, storage=storage, stream=torch.cuda.Stream(), **best)
    total_ms, k1_ms = timed_steps(S, torch, steps, 3)
    errs = [S.body_state(c, check=False)["err"] for c in range(len(cases))]
    for c, e in enumerate(errs):
        if e:
            log(f"  batch case {c} ({cases[c]['nx']}x{cases[c]['ny']}x{cases[c]['nz']}, tau {cases[c]['tau']:.4f}) "
                f"masked, error bits {e}")
    S.close()
    del S
    torch.cuda.empty_cache()
    cells = sum(c["nx"] * c["ny"] * c["nz"] for c in cases)
    eb = T.ELEM_BYTES[T.STORAGE[storage]]
    k1_gbps = 2 * (10 if storage == "mom" else 27) * eb * cells / (k1_ms * 1e-3) / 1e9
    return {"cases": len(cases), "cells": cells, "markers": int(sum(b["x_body"].shape[0] for b in bodies)),
            "steps": steps, "mlups": round(cells * steps / (total_ms * 1e-3) / 1e6, 1),
            "ms_per_step": round(total_ms / steps, 4), "k1_gbps": round(k1_gbps, 1),
            "k1_frac": round(k1_gbps / HBM_PEAK_GBPS, 4), "schedule": best,
            "schedule_cached": tuned["cached"], "masked_cases": int(sum(1 for e in errs if e))}


def learned_run(T, W, torch, storage, train_steps=300, eval_steps=100, skip=10, train_iters=2000, max_cycles=3):
    """The learned form on the batched cases (drag = F_z averaged over the
    second half of the run, its deviation taken over the body's weight kappa V g;
    v_z at the run's end).  The network is trained by the
    library's kernels on samples of a plain run of the 64-case batch (seeds
    2408..2471) and evaluated on a held-out batch of 64 other seeds
    (2472..2535): the residual after k = 1..4 cycles from the plain start,
    from the previous step's h and from the network (gate 0, so those runs
    follow the plain trajectory), then the gated run -- cycles from the
    network start until the case's residual is at or below the largest plain
    four-cycle residual of that case, at most `max_cycles`, else the plain
    cycles -- with its IBM time per step, acceptance and drag deviation
    against the plain run."""
    import numpy as np
    from paper_2408_15115_amd import autotune, learn
    seed_train, seed_eval, nc = 2408, 2408 + 64, 64

    def solver(seed0, diag, cycles=4, serial=1):
        # serial coupling: the events around ibm_couple then time the coupling itself
        batch = W.batch_cases(nc, seed0=seed0)
        cases = [c for c, _ in batch]
        sched = autotune.tune(cases, storage=storage)["best"]
        return T.Solver(cases, [b for _, b in batch], storage=storage, stream=torch.cuda.Stream(), ibm_diag=diag,
                        ibm_cycles=cycles, serial_ibm=serial, **sched)

    def step_ms(S, steps=60):
        """Whole coupled step with the coupling beside the lattice kernel."""
        S.run(5)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(S.stream)
        S.run(steps)
        e1.record(S.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def close(S):
        S.close()
        torch.cuda.empty_cache()

    def run(S, steps, collect=False, hist=False):
        st = S.stream
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        X, Y, H, Fz = [], [], [], []
        for k in range(steps):
            S.body_advance()
            S.lbm_step()
            ev[k][0].record(st)
            S.ibm_couple()
            ev[k][1].record(st)
            S.window_shift()
            if k >= skip and collect and k % 3 == 0:
                f, t = S.ibm_samples()
                sel = torch.arange(0, f.shape[0], 2, device="cuda")
                X.append(f[sel].cpu().numpy())
                Y.append(t[sel].cpu().numpy())
            if k >= steps // 2:
                Fz.append([S.body_state(c, check=False)["F"][2] for c in range(nc)])
            if k >= skip and hist:
                sts = [S.ibm_stats(c) for c in range(nc)]
                H.append([np.concatenate([x["resid_hist"], x["resid_hist_fallback"]]) for x in sts])
        torch.cuda.synchronize()
        ms = [a.elapsed_time(b) for a, b in ev[skip:]]
        stats = [S.ibm_stats(c) for c in range(nc)]
        bs = [S.body_state(c, check=False) for c in range(nc)]
        return {"ms": sum(ms) / len(ms), "X": X, "Y": Y, "H": np.array(H), "stats": stats,
                "Fz": np.array(Fz).mean(0), "vz": np.array([b["v"][2] for b in bs]),
                "errs": np.array([b["err"] for b in bs])}

    # training data: plain run of the training batch
    S = solver(seed_train, 0)
    M_all = S.marker_count()
    tr = run(S, train_steps, collect=True)
    close(S)
    X, Y = np.concatenate(tr["X"]), np.concatenate(tr["Y"])
    net = T.MLP(max_batch=8192, seed=0)
    t0 = time.perf_counter()
    loss = learn.fit(net, X, Y, iters=train_iters)
    train_s = time.perf_counter() - t0
    # held-out batch: plain run (timing, per-step four-cycle residual)
    S = solver(seed_eval, 0)
    plain = run(S, eval_steps, hist=True)
    close(S)
    starts = (("mlp", T.LBM_WARM_MLP, net), ("previous_h", T.LBM_WARM_PREVIOUS, None))
    # residuals after k cycles on the plain trajectory
    diag = {}
    for name, mode, m in starts:
        S = solver(seed_eval, 1)
        S.set_warm_start(mode, m, 4)
        for c in range(nc):
            S.set_ibm_gate(c, 0.0)
        diag[name] = run(S, eval_steps, hist=True)
        close(S)
    # gated runs: the network start, and the previous step's h without a
    # network (control)
    ok0 = plain["errs"] == 0
    r4 = plain["H"][:, :, 3]
    gates = np.where(ok0, r4.max(0), 0.0)
    gated = {}
    for name, mode, m in starts:
        S = solver(seed_eval, 0)
        S.set_warm_start(mode, m, max_cycles)
        for c in range(nc):
            S.set_ibm_gate(c, float(gates[c]))
        gated[name] = run(S, eval_steps)
        close(S)
    # sensitivity of the drag to the IBM residual: plain start, 3 cycles
    S = solver(seed_eval, 0, cycles=3)
    plain3 = run(S, eval_steps)
    close(S)
    # whole steps with the coupling beside the lattice kernel (the default)
    overlapped = {}
    for name, mode, m in (("plain", None, None), ("learned_gated", T.LBM_WARM_MLP, net)):
        S = solver(seed_eval, 0, serial=0)
        if mode is not None:
            S.set_warm_start(mode, m, max_cycles)
            for c in range(nc):
                S.set_ibm_gate(c, float(gates[c]))
        overlapped[name] = round(step_ms(S), 4)
        close(S)
    ok = ok0 & (plain3["errs"] == 0)
    for r_ in gated.values():
        ok &= r_["errs"] == 0
    # the network's forward on every marker of the batch (the warm start's
    # kernel shape), timed alone
    feats = torch.tensor(X[:M_all], device="cuda") if X.shape[0] >= M_all else None
    fwd_us = None
    if feats is not None:
        # into one preallocated output, so that the host keeps ahead of the GPU
        Yf = torch.empty((M_all, 3), dtype=torch.float32, device="cuda")
        for _ in range(5):
            net.forward(feats, out=Yf)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(net.stream)
        for _ in range(100):
            net.forward(feats, out=Yf)
        e1.record(net.stream)
        torch.cuda.synchronize()
        fwd_us = e0.elapsed_time(e1) / 100 * 1e3
    live = np.where(ok)[0]

    eb = W.batch_cases(nc, seed0=seed_eval)
    weight = np.array([b["kappa"] * b["volume"] * c["gravity"] for c, b in eb])

    def dev(r, key):
        # drag over the body's weight (its value at terminal velocity); v_z relative
        scale = weight[ok] if key == "Fz" else np.abs(plain[key][ok])
        d = np.abs(r[key][ok] - plain[key][ok]) / scale
        return {"median": float(np.median(d)), "max": float(d.max())} if d.size else None

    def gated_report(r):
        acc = sum(st["accepts"] for st in r["stats"])
        rej = sum(st["rejects"] for st in r["stats"])
        cyc = sum(st["warm_cycles_accepted"] for st in r["stats"])
        return {"ibm_ms_per_step": round(r["ms"], 4), "accepted": int(acc), "rejected": int(rej),
                "acceptance": round(acc / max(1, acc + rej), 4), "mean_cycles_accepted": round(cyc / max(1, acc), 3),
                "drag_dev_over_weight_vs_plain": dev(r, "Fz"), "vz_rel_dev_vs_plain": dev(r, "vz")}

    med = lambda Hs, k: float(np.median(Hs[:, live, k]))
    Hm, Hp = diag["mlp"]["H"], diag["previous_h"]["H"]
    return {"train_batch_seeds": f"{seed_train}..{seed_train + nc - 1}",
            "eval_batch_seeds": f"{seed_eval}..{seed_eval + nc - 1}", "cases": nc,
            "train_steps": train_steps, "eval_steps": eval_steps, "train_samples": int(X.shape[0]),
            "train_iters": train_iters, "train_seconds": round(train_s, 2), "train_loss_standardized": loss,
            "resid_after_k_cycles_median": {"plain": [med(Hm, 8 + k) for k in range(4)],
                                            "previous_h": [med(Hp, k) for k in range(4)],
                                            "mlp": [med(Hm, k) for k in range(4)]},
            "mlp_forward_us_all_markers": round(fwd_us, 2) if fwd_us else None, "markers": int(M_all),
            "gate": "largest plain four-cycle residual of the case in the plain run",
            "max_learned_cycles": max_cycles,
            "ibm_ms_per_step_plain_4cycles": round(plain["ms"], 4),
            "learned_gated": gated_report(gated["mlp"]),
            "previous_h_gated": gated_report(gated["previous_h"]),
            "step_ms_coupling_beside_lattice": overlapped,
            "plain_3cycles": {"ibm_ms_per_step": round(plain3["ms"], 4),
                              "drag_dev_over_weight_vs_plain": dev(plain3, "Fz"),
                              "vz_rel_dev_vs_plain": dev(plain3, "vz")},
            "masked_cases": int((~ok).sum())}


def settling_run(T, W, torch, steps=8000):
    """Sphere settling at Re 5 (D = 16, kappa 2.7, 160 x 160 x 480): terminal
    velocity over the Clift-Gauvin value, with the stress integral at the
    markers (as written) and on the parallel surface 3 cells outside."""
    import numpy as np
    out = {"workload": "sphere D 16, Re 5, kappa 2.7, box 160x160x480, 8000 steps from rest",
           "steps": steps}
    for name, off in (("markers", 0.0), ("parallel_surface_3", 3.0)):
        case, body, v_t = W.case_sphere_settling(16.0, 5.0, 2.7, force_offset=off)
        S = T.Solver([case], [body], stream=torch.cuda.Stream())
        v = []
        t0 = time.perf_counter()
        for k in range(steps // 250):
            S.run(250)
            if k >= steps // 250 - 8:
                v.append(-S.body_state()["v"][2] / v_t)
        dt = time.perf_counter() - t0
        S.close()
        torch.cuda.empty_cache()
        out[name] = {"vT_over_clift_gauvin": round(float(np.mean(v)), 4),
                     "mlups": round(case["nx"] * case["ny"] * case["nz"] * steps / dt / 1e6, 1)}
    return out


def settling_sweep(T, W, torch, diameters, re=5.0, offsets=(0.0, 3.0), domain="paper", storage="f32"):
    """Sphere terminal velocity over the Clift-Gauvin value against resolution:
    spheres of diameter D cells (kappa 2.7, Re `re`) settling from rest in the
    w* = 10, h* = 30 box of the paper's low-Re cases (no-slip bottom,
    constant-pressure top with domain="paper"), 500 D steps each; v_T is the
    mean of -v_z over the last quarter, `drift` its range there.  One row per
    (D, force-evaluation surface offset)."""
    import numpy as np
    rows = []
    for D in diameters:
        steps = int(500 * D)
        for off in offsets:
            case, body, v_t = W.case_sphere_settling(float(D), re, 2.7, force_offset=off, domain=domain)
            S = T.Solver([case], [body], stream=torch.cuda.Stream(), storage=storage)
            chunk = 250
            nch = steps // chunk
            tail = max(8, nch // 4)
            v = []
            t0 = time.perf_counter()
            for k in range(nch):
                S.run(chunk)
                if k >= nch - tail:
                    v.append(-S.body_state()["v"][2] / v_t)
                if k % 16 == 15:
                    log(f"  D {D}, offset {off}: step {(k + 1) * chunk} of {steps}, v_z / v_T "
                        f"{-S.body_state()['v'][2] / v_t:.4f}")
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            st = S.body_state()
            S.close()
            del S
            torch.cuda.empty_cache()
            cells = case["nx"] * case["ny"] * case["nz"]
            row = {"D": D, "re": re, "force_offset": off, "domain": domain, "storage": storage,
                   "box": [case["nx"], case["ny"], case["nz"]],
                   "markers": int(body["x_body"].shape[0]), "steps": steps, "tau": round(case["tau"], 5),
                   "vT_over_clift_gauvin": round(float(np.mean(v)), 4), "drift": round(float(np.ptp(v)), 4),
                   "window_shifts": int(st["shifts"]), "mlups": round(cells * steps / dt / 1e6, 1)}
            rows.append(row)
            log(f"  {row}")
    return rows


TABLE3_RE = (0.58, 1.39, 4.49, 6.18, 28.3, 127.88)


def settling_table3(T, W, torch, D, res=TABLE3_RE, kappa=2.7, storage="f32"):
    """The terminal-velocity comparison of Table 3 (Sec. 3.2) at one
    resolution: a sphere of diameter D cells settling from rest in the
    paper's box (w* = 10, h* = 30, no-slip bottom, constant-pressure top;
    h_ini* = 27 below Re 20, 23 up to Re 1000 and 20 above, h_end* = 3,
    sponge 2.4 D), force on
    the parallel surface 3 cells out, max(500 D, 8 drag-law relaxation
    times (6 above Re 1000, where the quadratic drag relaxes twice as fast),
    3 Oseen times nu / v^2) steps: at low Re the history force
    approaches the terminal speed as t^(-1/2) until the Oseen time, so the
    speed is also extrapolated by a fit v = v_inf - c t^(-1/2) over the
    second half of the run.  Per Re: the terminal speed over the Clift-Gauvin value
    (the weight balanced by the drag law, solved by bisection) and, below
    Re 1, over Stokes' law; the paper's own measure (the reference speed
    from C_D at the simulated Re); the force balance Delta F = (F_g - F_D) / F_g;
    and p*, the pressure share of the drag on that surface.  The density
    ratio sets only the transient, so a light sphere (kappa 2.7) reaches the
    same steady balance in fewer steps than the paper's 996."""
    import numpy as np
    rows = []
    for re in res:
        h_ini = 27.0 if re < 20 else (23.0 if re < 1000 else 20.0)
        case, body, v_t = W.case_sphere_settling(float(D), re, kappa, force_offset=3.0, domain="paper",
                                                 h_ini_d=h_ini, h_end_d=3.0, sponge_d=2.4)
        nu, g = (case["tau"] - 0.5) / 3.0, case["gravity"]
        t_relax = v_t / g * (kappa + 0.5) / kappa
        chunk = 250
        # a drag quadratic in v (Re above 1000) relaxes twice as fast near the
        # terminal speed: 6 t_relax are 12 of its time constants
        relax = 8 if re < 1000 else 6
        steps = int(max(500 * D, relax * t_relax, 3 * nu / v_t ** 2)) // chunk * chunk + chunk
        S = T.Solver([case], [body], stream=torch.cuda.Stream(), storage=storage)
        nch = steps // chunk
        tail = max(8, nch // 4)
        v, F, Fp, hist = [], [], [], []
        t0 = time.perf_counter()
        for k in range(nch):
            S.run(chunk)
            if k >= nch // 2:
                st = S.body_state()
                hist.append(((k + 1) * chunk, -st["v"][2]))
                if k >= nch - tail:
                    v.append(-st["v"][2])
                    F.append(st["F"][2])
                    Fp.append(st["F_pressure"][2])
            if k % 16 == 15:
                log(f"  Table 3, D {D}, Re {re}: step {(k + 1) * chunk} of {steps}, v_z {S.body_state()['v'][2]:.5f}")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        S.close()
        del S
        torch.cuda.empty_cache()
        vol = float(body["volume"])
        Fg = kappa * g * vol
        area = math.pi * D * D / 4.0

        def drag(u):
            return 0.5 * W.clift_gauvin_cd(u * D / nu) * area * u * u

        lo, hi = 1e-7, 1.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            lo, hi = (mid, hi) if drag(mid) < Fg else (lo, mid)
        v_cg = 0.5 * (lo + hi)
        vT = float(np.mean(v))
        th = np.array(hist)
        fit = np.polyfit(th[:, 0] ** -0.5, th[:, 1], 1)   # v = v_inf + slope t^(-1/2)
        v_inf = float(fit[1])
        re_sim = vT * D / nu
        cd_sim = 24.0 / re_sim if re < 1 else W.clift_gauvin_cd(re_sim)
        v_ref = math.sqrt(8.0 * Fg / (math.pi * D * D * cd_sim))
        Fd = float(np.mean(F))
        row = {"re_target": re, "D": D, "kappa": kappa, "storage": storage, "box": [case["nx"], case["ny"], case["nz"]],
               "tau": round(case["tau"], 5),
               "steps": steps, "v_T_lattice": round(vT, 6), "re_simulated": round(re_sim, 3),
               "vT_over_clift_gauvin": round(vT / v_cg, 4),
               "v_inf_over_clift_gauvin": round(v_inf / v_cg, 4) if re < 1 else None,
               "vT_over_stokes": round(vT / (Fg / (3.0 * math.pi * nu * D)), 4) if re < 1 else None,
               "delta_vT_paper_measure": round((vT - v_ref) / vT, 4),
               "delta_F": round((Fg - Fd) / Fg, 4), "p_star": round(float(np.mean(Fp)) / Fd, 4),
               "drift": round(float(np.ptp(v)) / vT, 4), "mlups": round(case["nx"] * case["ny"] * case["nz"] * steps / dt / 1e6, 1)}
        rows.append(row)
        log(f"  {row}")
    return rows


def stability_run(T, W, torch, n=64, U0=0.1, steps=2000):
    """3-D Taylor-Green vortex (n^3, U0 = 0.1): the smallest relaxation time
    that runs `steps` steps without tripping the lattice kernel's guard, for
    the recursive-regularized collision and for BGK, on D3Q27 and on the D3Q19
    comparison lattice."""
    import numpy as np
    taus = [0.52, 0.51, 0.505, 0.502, 0.501, 0.5005, 0.5002, 0.5001]
    f27 = np.moveaxis(W.taylor_green_populations(n, U0), -1, 0)
    f19 = np.moveaxis(W.taylor_green_populations19(n, U0), -1, 0)
    out = {"workload": f"Taylor-Green vortex {n}^3, U0 {U0}, {steps} steps", "taus_tried": taus}
    for name, coll, q, f0 in (("regularized", 0, 27, f27), ("bgk", 1, 27, f27),
                              ("regularized_d3q19", 0, 19, f19), ("bgk_d3q19", 1, 19, f19)):
        low = None
        for tau in taus:
            S = T.Solver([W.make_case(n, n, n, tau, W.BC_PERIODIC, W.BC_PERIODIC, 0)], collision=coll,
                         stream=torch.cuda.Stream(), lattice=q)
            S.set_populations(f0)
            ok = True
            for _ in range(steps // 250):
                S.run(250)
                if S.body_state(0, check=False)["err"]:
                    ok = False
                    break
            S.close()
            if not ok:
                break
            low = tau
        out[name] = {"smallest_stable_tau": low,
                     "reynolds": round(U0 * n / (2 * math.pi) / ((low - 0.5) / 3.0), 1) if low else None}
    return out


def lattice_rate_run(T, W, torch, n=(256, 256, 768), steps=20, warmup=3):
    """Fluid-only periodic box, FP32, recursive-regularized collision: the
    lattice kernel alone on D3Q27, on the D3Q19 comparison lattice, and on
    D3Q27 with moment storage; GLUPS and the algorithmic bandwidth (the
    stored values read and written: q populations, or 10 moments)."""
    nx, ny, nz = n
    out = {"workload": f"fluid-only periodic {nx}x{ny}x{nz}, FP32, recursive regularized, {steps} steps"}
    for name, q, storage, per_cell in (("d3q27", 27, "f32", 27), ("d3q19", 19, "f32", 19),
                                       ("d3q27_moments", 27, "mom", 10)):
        S = T.Solver([W.make_case(nx, ny, nz, 0.6, W.BC_PERIODIC, W.BC_PERIODIC, 0)], lattice=q, storage=storage,
                     stream=torch.cuda.Stream())
        for _ in range(warmup):
            S.lbm_step()
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(S.stream)
        for _ in range(steps):
            S.lbm_step()
        t1.record(S.stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / steps
        err = S.body_state(0, check=False)["err"]
        S.close()
        cells = nx * ny * nz
        out[name] = {"ms_per_step": round(ms, 4), "glups": round(cells / (ms * 1e-3) / 1e9, 2),
                     "gbps": round(cells * per_cell * 8 / (ms * 1e-3) / 1e9, 1), "err": int(err)}
    torch.cuda.empty_cache()
    return out


def long_run(T, W, torch, which, steps, storage="f32", chunk=None):
    """The stated run lengths, once: the scale case for 20k steps (about five
    window shifts) or the 64-case batch for 5k steps.  Replays of a 10-step
    graph in chunks;
    after each chunk the body states (shifts, drag, velocity, the Reynolds
    number reached, error bits) are read back and logged."""
    import numpy as np
    from paper_2408_15115_amd import autotune
    if which == "scale":
        case, body = W.case_ellipsoid_tall()
        cases, bodies = [case], [body]
        sched = {}
        chunk = chunk or 1000
    else:
        batch = W.batch_cases(64)
        cases, bodies = [c for c, _ in batch], [b for _, b in batch]
        sched = autotune.tune_step(cases, bodies, storage=storage)["best"]
        chunk = chunk or 250
    S = T.Solver(cases, bodies, storage=storage, stream=torch.cuda.Stream(), **sched)
    S.graph_capture(10)
    nu = [(c["tau"] - 0.5) / 3.0 for c in cases]
    rows, done = [], 0
    t0 = time.perf_counter()
    gpu_ms = 0.0
    while done < steps:
        n = min(chunk, steps - done)
        n -= n % 10
        if n == 0:
            break
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(S.stream)
        for _ in range(n // 10):
            S.graph_launch()
        e1.record(S.stream)
        torch.cuda.synchronize()
        gpu_ms += e0.elapsed_time(e1)
        done += n
        st = [S.body_state(c, check=False) for c in range(len(cases))]
        re = [float(np.linalg.norm(b["v"]) * c.get("d_eq", 0.0) / v) for b, c, v in zip(st, cases, nu)]
        masked = [c for c, b in enumerate(st) if b["err"]]
        row = {"step": done, "shifts": [b["shifts"] for b in st] if which != "scale" else st[0]["shifts"],
               "masked": masked}
        if which == "scale":
            row.update(Fz=float(st[0]["F"][2]), vz=float(st[0]["v"][2]), rz=float(st[0]["r"][2]), re=round(re[0], 3),
                       err=st[0]["err"])
        rows.append(row)
        log(f"  {which}: step {done}/{steps}, {gpu_ms / done:.3f} ms per step, shifts "
            f"{row['shifts'] if which == 'scale' else sum(row['shifts'])}, masked {masked}"
            + (f", F_z {row['Fz']:.4e}, v_z {row['vz']:.4e}, Re {row['re']:.2f}" if which == "scale" else ""))
    wall = time.perf_counter() - t0
    st = [S.body_state(c, check=False) for c in range(len(cases))]
    S.close()
    del S
    torch.cuda.empty_cache()
    cells = sum(c["nx"] * c["ny"] * c["nz"] for c in cases)
    out = {"workload": which, "steps": steps, "storage": storage, "cells": cells, "ms_per_step": gpu_ms / steps,
           "mlups": cells * steps / (gpu_ms * 1e-3) / 1e6, "wall_s": round(wall, 1), "chunks": rows}
    if which != "scale":
        out["schedule"] = sched
        out["cases"] = [{"seed": 2408 + c, "shape": cases[c]["shape"], "box": [cases[c]["nx"], cases[c]["ny"], cases[c]["nz"]],
                         "tau": round(cases[c]["tau"], 5), "kappa": round(bodies[c]["kappa"], 3),
                         "re_target": round(cases[c]["re"], 3), "re_reached": round(float(
                             np.linalg.norm(st[c]["v"]) * cases[c]["d_eq"] / nu[c]), 3),
                         "shifts": st[c]["shifts"], "err": st[c]["err"]} for c in range(len(cases))]
    return out


def cpu_model():
    """CPU model name of the host (from /proc/cpuinfo, as lscpu reads it)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_rate(O, case, body, steps, threads):
    """MLUPS of the FP64 oracle's coupled step on `threads` threads (one
    untimed step first)."""
    O.set_threads(threads)
    sim = O.OracleSim(case, body)
    sim.step(1)
    t = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t
    cells = case["nx"] * case["ny"] * case["nz"]
    return {"mlups": round(cells * steps / dt / 1e6, 4), "steps": steps, "threads": threads, "seconds": round(dt, 2)}


def scale_window(case, body, nx, ny, nz):
    """A window of the scale case around its body (same body, tau, walls),
    sponge scaled with the height, no re-injection."""
    c = dict(case)
    c.update(nx=nx, ny=ny, nz=nz, sponge=int(round(0.08 * nz)), h_ini=0.0, h_end=0.0)
    b = dict(body)
    b["r0"] = [(nx - 1) / 2.0, (ny - 1) / 2.0, 0.5 * nz]
    return c, b


def cpu_baseline(case, body, steps, full=False):
    """The FP64 oracle, as it stands, timed on the host cores.  Default: a
    bounded sample -- the 48^3 sphere case for `steps` steps on all threads
    and for 4 steps on one thread, and a 128^3 window of the scale case for
    `steps` steps on all threads (the value: its MLUPS).  full=True: the
    whole set -- the sphere case for 200 and 2,000 steps on all threads and
    200 on one, the 128 x 128 x 384 slice of the scale case for 100 steps on
    all threads and 5 on one."""
    from oracle import oracle as O
    from paper_2408_15115_amd import workloads as W
    threads = O.num_threads()
    s_case, s_body = W.case_sphere48()
    rows = {}
    if full:
        for n in (200, 2000):
            rows[f"sphere48_{n}_steps_all"] = _oracle_rate(O, s_case, s_body, n, threads)
            log(f"  cpu: sphere48 {n} steps, {threads} threads: {rows[f'sphere48_{n}_steps_all']}")
        rows["sphere48_200_steps_1thread"] = _oracle_rate(O, s_case, s_body, 200, 1)
        log(f"  cpu: sphere48 200 steps, 1 thread: {rows['sphere48_200_steps_1thread']}")
        c, b = scale_window(case, body, 128, 128, 384)
        rows["slice128x128x384_100_steps_all"] = _oracle_rate(O, c, b, 100, threads)
        log(f"  cpu: slice 100 steps, {threads} threads: {rows['slice128x128x384_100_steps_all']}")
        rows["slice128x128x384_5_steps_1thread"] = _oracle_rate(O, c, b, 5, 1)
        log(f"  cpu: slice 5 steps, 1 thread: {rows['slice128x128x384_5_steps_1thread']}")
        value = rows["slice128x128x384_100_steps_all"]
        sample = "128 x 128 x 384 slice of the workload (same ellipsoid, 12252 markers, tau, walls), 100 coupled steps"
    else:
        rows["sphere48_all"] = _oracle_rate(O, s_case, s_body, steps, threads)
        rows["sphere48_1thread"] = _oracle_rate(O, s_case, s_body, 4, 1)
        c, b = scale_window(case, body, 128, 128, 128)
        rows["window128_all"] = _oracle_rate(O, c, b, steps, threads)
        value = rows["window128_all"]
        sample = (f"128^3 window of the workload (same ellipsoid, 12252 markers, tau, walls), {steps} coupled steps "
                  f"after 1 untimed, FP64, {value['seconds']} s")
    O.set_threads(threads)
    return {"value": value["mlups"], "unit": "MLUPS", "cores": threads, "kind": "oracle", "sample": sample,
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "one_thread_mlups": (
                rows.get("sphere48_1thread") or rows.get("sphere48_200_steps_1thread"))["mlups"], "runs": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16", "mom"])
    ap.add_argument("--variant-steps", type=int, default=400)
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--cpu-full", action="store_true",
                    help="run only the full CPU-oracle timing set (sphere case 200 / 2,000 steps, slice 100 steps)")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=40)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-settling", action="store_true")
    ap.add_argument("--settling-sweep", type=str, default=None,
                    help="comma-separated sphere diameters: run only the terminal-velocity resolution sweep")
    ap.add_argument("--sweep-offsets", type=str, default="0,3",
                    help="force-surface offsets of the --settling-sweep runs")
    ap.add_argument("--no-stability", action="store_true")
    ap.add_argument("--no-long", action="store_true", help="skip the stated run lengths (20k / 5k steps)")
    ap.add_argument("--kappa", type=float, default=2.7, help="density ratio of the --table3 spheres")
    ap.add_argument("--lattice-rates", action="store_true",
                    help="run only the fluid-only lattice kernel comparison (D3Q27, D3Q19, moment storage)")
    ap.add_argument("--table3", type=str, default=None,
                    help="D[:Re1,Re2,...]: run only the terminal-velocity comparison of Table 3 at diameter D cells")
    ap.add_argument("--long", choices=["scale", "batch"], default=None,
                    help="run only the stated run length of the scale case (20k steps) or the batch (5k steps)")
    ap.add_argument("--long-steps", type=int, default=None)
    ap.add_argument("--coupling", default="auto", choices=["auto", "serial", "beside"],
                    help="where the coupling runs: chosen by timing both (auto), after the lattice kernel, or "
                         "beside it on a second stream; for the batch, auto is the tuner's choice")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(each case runs on a single MI355X); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2408_15115_amd import turret as T
    from paper_2408_15115_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.lattice_rates:
        # the plain copy in the same run calibrates counter-based traffic figures
        copy = None if args.no_copy else round(copy_bandwidth(T, torch), 1)
        print(json.dumps({"metric": "fluid-only lattice kernel rates", "data": "synthetic", "copy_GBps": copy,
                          "rows": lattice_rate_run(T, W, torch, steps=args.steps)}))
        return
    if args.cpu_full:
        case, body = W.case_ellipsoid_tall()
        print(json.dumps({"metric": "FP64 CPU oracle timings", "data": "synthetic",
                          "cpu_baseline": cpu_baseline(case, body, 0, full=True)}), flush=True)
        return
    if args.long:
        n = args.long_steps or (20000 if args.long == "scale" else 5000)
        print(json.dumps({"metric": f"stated run length, {args.long}", "data": "synthetic",
                          "result": long_run(T, W, torch, args.long, n, storage=args.storage)}), flush=True)
        return
    if args.table3:
        d, _, rl = args.table3.partition(":")
        res = [float(r) for r in rl.split(",")] if rl else TABLE3_RE
        rows = settling_table3(T, W, torch, int(d), res, kappa=args.kappa, storage=args.storage)
        print(json.dumps({"metric": "sphere terminal velocity against Clift-Gauvin / Stokes across Re (Table 3)",
                          "data": "synthetic", "rows": rows}))
        return
    if args.settling_sweep:
        rows = settling_sweep(T, W, torch, [int(d) for d in args.settling_sweep.split(",")],
                              offsets=tuple(float(o) for o in args.sweep_offsets.split(",")), storage=args.storage)
        print(json.dumps({"metric": "sphere terminal velocity / Clift-Gauvin against resolution",
                          "data": "synthetic", "rows": rows}))
        return
    case, body = W.case_ellipsoid_tall()
    cells = case["nx"] * case["ny"] * case["nz"]
    M = body["x_body"].shape[0]
    log(f"workload {case['nx']}x{case['ny']}x{case['nz']} ({cells / 1e6:.1f} M cells), {M} markers, "
        f"tau {case['tau']:.5f}, gravity {case['gravity']:.3e}")

    copy_gbps = None if args.no_copy else copy_bandwidth(T, torch)
    if copy_gbps:
        log(f"streaming copy: {copy_gbps:.0f} GB/s")

    def coupling_mode(storage, steps=100):
        """serial_ibm value with the shorter coupled step: the coupling beside
        the lattice kernel (0) or after it (1)."""
        best = None
        for serial in (0, 1):
            S = T.Solver([case], [body], storage=storage, stream=torch.cuda.Stream(), serial_ibm=serial)
            S.run(10)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(S.stream)
            S.run(steps)
            e1.record(S.stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            S.close()
            del S
            torch.cuda.empty_cache()
            if best is None or ms < best[1]:
                best = (serial, ms)
        return best[0]

    modes = {}

    def run_storage(storage, steps, warmup, graph):
        if storage not in modes:
            modes[storage] = {"serial": 1, "beside": 0}.get(args.coupling)
            if modes[storage] is None:
                modes[storage] = coupling_mode(storage)
        S = T.Solver([case], [body], storage=storage, stream=torch.cuda.Stream(), serial_ibm=modes[storage])
        total_ms, k1_ms = timed_steps(S, torch, steps, warmup)
        k1 = timed_steps.last_k1
        n = min(100, len(k1))
        # drift over the run and the two buffer directions (even / odd steps)
        k1_profile = {"first_100_ms": sum(k1[:n]) / n, "last_100_ms": sum(k1[-n:]) / n,
                      "even_steps_ms": sum(k1[0::2]) / len(k1[0::2]),
                      "odd_steps_ms": sum(k1[1::2]) / max(1, len(k1[1::2]))}
        st = S.body_state()
        gms = None if not graph else graph_steps(S, torch, steps)
        S.close()
        del S
        torch.cuda.empty_cache()
        eb = T.ELEM_BYTES[T.STORAGE[storage]]
        kbytes = 2 * (10 if storage == "mom" else 27) * eb * cells   # stored values read and written
        return {"ms_per_step": total_ms / steps, "mlups": cells * steps / (total_ms * 1e-3) / 1e6,
                "k1_ms": k1_ms, "k1_gbps": kbytes / (k1_ms * 1e-3) / 1e9, "k1_bytes": kbytes,
                "graph_ms_per_step": gms, "F": st["F"].tolist(), "v": st["v"].tolist(), "steps": st["steps"],
                "k1_profile": {k: round(v, 4) for k, v in k1_profile.items()}}

    log(f"timed: {args.steps} steps ({args.storage}) after {args.warmup} warm-up")
    main_run = run_storage(args.storage, args.steps, args.warmup, not args.no_graph)
    log(f"  eager {main_run['ms_per_step']:.3f} ms/step, {main_run['mlups']:.0f} MLUPS; lattice kernel "
        f"{main_run['k1_ms']:.3f} ms = {main_run['k1_gbps']:.0f} GB/s")
    # the value: the same number of steps replayed from captured graphs (the
    # eager run brackets every lattice launch with events for the roofline)
    value_ms = main_run["graph_ms_per_step"] or main_run["ms_per_step"]
    if main_run["graph_ms_per_step"]:
        log(f"  graph replay {value_ms:.3f} ms/step, {cells / (value_ms * 1e-3) / 1e6:.0f} MLUPS")

    variants = {}
    if not args.no_variants and not args.no_precision:
        ref = run_storage("f32", args.variant_steps, 5, False)
        for sto in ("f16", "bf16"):
            # eager steps (events around every lattice launch), then the same
            # number of steps graph-replayed like the value
            r = run_storage(sto, args.variant_steps, 5, True)
            fz, fz_ref = r["F"][2], ref["F"][2]
            gm = r["graph_ms_per_step"]
            variants[sto] = {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                             "mlups_graph": round(cells / (gm * 1e-3) / 1e6, 1), "graph_ms_per_step": round(gm, 4),
                             "coupling": "serial" if modes[sto] else "beside",
                             "k1_gbps": round(r["k1_gbps"], 1), "k1_frac": round(r["k1_gbps"] / HBM_PEAK_GBPS, 4),
                             "drag_rel_diff_vs_f32": abs(fz - fz_ref) / abs(fz_ref),
                             "vz_rel_diff_vs_f32": abs(r["v"][2] - ref["v"][2]) / abs(ref["v"][2]),
                             "after_steps": args.variant_steps}
            log(f"  {sto}: {r['mlups']:.0f} MLUPS eager, {variants[sto]['mlups_graph']:.0f} graph-replayed, "
                f"kernel {r['k1_gbps']:.0f} GB/s, drag diff vs f32 "
                f"{variants[sto]['drag_rel_diff_vs_f32']:.2e}")
        variants["f32_same_steps"] = {"mlups": round(ref["mlups"], 1), "k1_gbps": round(ref["k1_gbps"], 1)}
        # moment storage: the same coupled step, ten moments per cell (plus the
        # forcing shifts of the particle region); graph-replayed like the value
        r = run_storage("mom", args.variant_steps, 5, True)
        gm = r["graph_ms_per_step"]
        variants["moments"] = {"mlups_graph": round(cells / (gm * 1e-3) / 1e6, 1), "graph_ms_per_step": round(gm, 4),
                               "mlups_eager": round(r["mlups"], 1), "lattice_kernel_ms": round(r["k1_ms"], 4),
                               "lattice_kernel_gbps": round(r["k1_gbps"], 1),
                               "drag_rel_diff_vs_f32": abs(r["F"][2] - ref["F"][2]) / abs(ref["F"][2]),
                               "vz_rel_diff_vs_f32": abs(r["v"][2] - ref["v"][2]) / abs(ref["v"][2]),
                               "after_steps": args.variant_steps}
        log(f"  moment storage: {variants['moments']['mlups_graph']:.0f} MLUPS (graph), lattice kernel "
            f"{r['k1_ms']:.3f} ms, drag diff vs f32 {variants['moments']['drag_rel_diff_vs_f32']:.2e}")

    if not args.no_variants and not args.no_batch:
        b = batch_run(T, W, torch, args.batch_steps, args.storage, args.coupling)
        variants["batch64"] = b
        log(f"  batch: {b['mlups']:.0f} MLUPS, {b['ms_per_step']:.2f} ms/step, kernel {b['k1_gbps']:.0f} GB/s, "
            f"masked {b['masked_cases']}")
        if args.storage == "f32":
            bm = batch_run(T, W, torch, args.batch_steps, "mom", args.coupling)
            variants["batch64_moments"] = bm
            log(f"  batch, moment storage: {bm['mlups']:.0f} MLUPS, {bm['ms_per_step']:.2f} ms/step, "
                f"masked {bm['masked_cases']}")

    if not args.no_variants and not args.no_learned:
        lr = learned_run(T, W, torch, args.storage)
        variants["learned_batch64"] = lr
        rk = lr["resid_after_k_cycles_median"]
        log(f"  learned: residual after 1..4 cycles plain {['%.2e' % v for v in rk['plain']]}, "
            f"previous h {['%.2e' % v for v in rk['previous_h']]}, network {['%.2e' % v for v in rk['mlp']]}")
        for k in ("learned_gated", "previous_h_gated"):
            g = lr[k]
            log(f"  {k}: IBM {lr['ibm_ms_per_step_plain_4cycles']:.3f} -> {g['ibm_ms_per_step']:.3f} ms/step, "
                f"acceptance {g['acceptance']:.2f}, mean cycles {g['mean_cycles_accepted']}, "
                f"drag dev / weight {g['drag_dev_over_weight_vs_plain']}, v_z dev {g['vz_rel_dev_vs_plain']}")
        log(f"  whole step with the coupling beside the lattice kernel: {lr['step_ms_coupling_beside_lattice']} ms")
        log(f"  plain 3 cycles: drag dev / weight {lr['plain_3cycles']['drag_dev_over_weight_vs_plain']}, "
            f"v_z dev {lr['plain_3cycles']['vz_rel_dev_vs_plain']}")

    if not args.no_variants and not args.no_settling:
        st = settling_run(T, W, torch)
        variants["sphere_settling"] = st
        log(f"  sphere settling, v_T / Clift-Gauvin: stress integral at the markers "
            f"{st['markers']['vT_over_clift_gauvin']}, on the parallel surface 3 cells out "
            f"{st['parallel_surface_3']['vT_over_clift_gauvin']}")

    if not args.no_variants and not args.no_stability:
        sb = stability_run(T, W, torch)
        variants["stability"] = sb
        log(f"  Taylor-Green stability, smallest stable tau: regularized {sb['regularized']}, BGK {sb['bgk']}; "
            f"D3Q19 regularized {sb['regularized_d3q19']}, BGK {sb['bgk_d3q19']}")

    if not args.no_variants and not args.no_stability:
        lr19 = lattice_rate_run(T, W, torch)
        variants["lattice_rate"] = lr19
        log(f"  fluid-only lattice kernel: D3Q27 {lr19['d3q27']}, D3Q19 {lr19['d3q19']}, "
            f"D3Q27 moment storage {lr19['d3q27_moments']}")

    if not args.no_variants and not args.no_long:
        # the stated run lengths: the scale case for 20k steps, the batch for 5k
        runs = {}
        for which, n in (("scale", 20000), ("batch", 5000)):
            r = long_run(T, W, torch, which, n)
            last = r["chunks"][-1]
            runs[which] = {k: v for k, v in r.items() if k not in ("chunks", "cases")}
            runs[which]["final"] = last
            if which == "batch":
                runs[which]["shifts_total"] = int(sum(c["shifts"] for c in r["cases"]))
                runs[which]["masked_seeds"] = [c["seed"] for c in r["cases"] if c["err"]]
                runs[which]["re_reached_over_target"] = sorted(
                    round(c["re_reached"] / c["re_target"], 3) for c in r["cases"])
        variants["stated_run_lengths"] = runs
        log(f"  stated run lengths: scale {runs['scale']['ms_per_step']:.3f} ms/step, "
            f"{runs['scale']['final']['shifts']} shifts; batch {runs['batch']['ms_per_step']:.3f} ms/step, "
            f"{runs['batch']['shifts_total']} shifts, masked {runs['batch']['masked_seeds']}")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: FP64 oracle on bounded samples")
        cpu = cpu_baseline(case, body, args.cpu_steps)
        log(f"  {cpu['value']:.3f} MLUPS on {cpu['cores']} threads ({cpu['cpu_model']}), one thread "
            f"{cpu['one_thread_mlups']:.3f} MLUPS")

    achieved = main_run["k1_gbps"]
    out = {
        "metric": METRIC,
        "value": round(cells / (value_ms * 1e-3) / 1e6, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(value_ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": "falling-frame box 256x256x768, tilted oblate ellipsoid 32/32/16 with 12252 "
                               "markers, kappa 2.7, Re 100, sponge 61, free-slip z, 4 IBM cycles",
                   "cells": cells, "markers": M, "storage": args.storage,
                   "launch": (f"graph replay of {graph_steps.per}-step graphs" if main_run["graph_ms_per_step"]
                              else "eager"),
                   "coupling": "after the lattice kernel" if modes.get(args.storage) else "beside the lattice kernel",
                   "eager_ms_per_step": round(main_run["ms_per_step"], 5)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": stored_traffic(args.storage),
                     "kernel": f"k_stream_collide<{args.storage}>",
                     "algorithmic_bytes_per_launch": main_run["k1_bytes"],
                     "avg_launch_ms": round(main_run["k1_ms"], 5), "launch_profile": main_run["k1_profile"],
                     "copy_GBps": round(copy_gbps, 1) if copy_gbps else None},
        "cpu_baseline": cpu,
        "variants": variants or None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
