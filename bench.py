#!/usr/bin/env python3
"""Throughput of the decode + DAS hot path on one MI355X.

Workload (default): HERCULES volume, 128x128 TOBE array at 0.1 mm, 128
Hadamard transmits x 128 channels x 2048 int16 samples at 30 MHz, output
128 x 128 x 256 FP32 voxels, cubic Hermite reads, F# 1 (seeded synthetic
scene of 64 points + 10^4 speckle scatterers).  One step = decode + DAS of
one volume with the RF already resident in HBM.

Metric: G voxel*tx*ch samples/s = Nx*Ny*Nz*n_tx*n_ch / step time (nominal:
apodization-skipped terms are counted), plus volumes/s.  The JSON line also
carries the DAS kernel's roofline figures (HIP events around each DAS launch
on the launch stream) and the FP64 CPU oracle's rate on a bounded sample.
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

# FP32 vector peaks of MI355X (256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz, an FMA
# counting 2 flops): the published 157.3 TFLOP/s counts packed FP32 (two FP32
# operations per lane and instruction); this build disables packed FP32
# instructions, so its ceiling is half of that.
FP32_PUBLISHED_TFLOPS = 157.3
FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12
# LDS read bandwidth: 256 CUs x 128 bytes per clock x 2.4 GHz.
LDS_PEAK_TBPS = 256 * 128 * 2.4e9 / 1e12
# Bytes of LDS taps per cubic FP32 read: four samples (the kernels read them
# as one 16-byte coefficient quad).
LDS_BYTES_PER_TERM = 16


def alu_roofline(tflops: float, traffic=None) -> dict:
    """FP32 ALU roofline object: against the published peak (frac) and the
    non-packed ceiling of this build (frac_nonpacked)."""
    return {"bound": "alu", "achieved": round(tflops, 2), "peak": FP32_PUBLISHED_TFLOPS,
            "unit": "TFLOP/s", "frac": round(tflops / FP32_PUBLISHED_TFLOPS, 4),
            "traffic": traffic, "peak_nonpacked": round(FP32_NONPACKED_TFLOPS, 1),
            "frac_nonpacked": round(tflops / FP32_NONPACKED_TFLOPS, 4)}


def lds_roofline(n_terms: int, n_nominal: int, ms: float) -> dict:
    """LDS-gather roofline of a DAS launch: 16 bytes of taps per term read
    from LDS, over the active terms (apodization > 0) and over the nominal
    count of the metric."""
    act = LDS_BYTES_PER_TERM * n_terms / (ms * 1e-3) / 1e12
    nom = LDS_BYTES_PER_TERM * n_nominal / (ms * 1e-3) / 1e12
    return {"bound": "lds", "achieved": round(act, 2), "peak": round(LDS_PEAK_TBPS, 1),
            "unit": "TB/s", "frac": round(act / LDS_PEAK_TBPS, 4),
            "achieved_nominal": round(nom, 2), "frac_nominal": round(nom / LDS_PEAK_TBPS, 4)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def active_terms(desc, dev) -> int:
    """Number of (voxel, tx, ch) terms with non-zero apodization (geometry only;
    bookkeeping for the roofline figure, evaluated with torch on the device)."""
    import torch
    px, py = desc["pitch"]
    M = torch.tensor(np.asarray(desc["xdc"], dtype=np.float64).reshape(4, 4), device=dev)
    axes = [torch.linspace(desc["gmin"][a], desc["gmax"][a], desc["dims"][a], dtype=torch.float64,
                           device=dev) for a in range(3)]
    gx, gy, gz = torch.meshgrid(axes[0], axes[1], axes[2], indexing="ij")
    P = torch.stack([gx, gy, gz], -1).reshape(-1, 3) @ M[:3, :3].T + M[:3, 3]
    x, y, z = P[:, 0], P[:, 1], P[:, 2]
    F2 = float(desc["f_number"]) ** 2
    thr = torch.where(z > 0, 0.25 * z * z, torch.full_like(z, -1.0))
    xt = torch.tensor(np.asarray(desc["tx_elements"], dtype=np.float64) * px, device=dev)
    total = 0
    if desc["mode"] == "hercules":
        for yj in np.asarray(desc["channel_map"], dtype=np.float64) * py:
            r2 = (x[:, None] - xt[None, :]) ** 2 + (y[:, None] - yj) ** 2
            total += int(torch.count_nonzero(F2 * r2 < thr[:, None]))
        return total
    if desc["mode"] in ("tpw", "vls"):        # row receivers: apodization on |y - y_j|
        for yj in np.asarray(desc["channel_map"], dtype=np.float64) * py:
            total += int(torch.count_nonzero(F2 * (y - yj) ** 2 < thr)) * len(xt)
        return total
    for xj in np.asarray(desc["channel_map"], dtype=np.float64) * px:
        total += int(torch.count_nonzero(F2 * (x - xj) ** 2 < thr)) * len(xt)
    return total


def algorithmic_flops(desc, n_act: int, iq: bool = False, adjoint_c: bool = False) -> float:
    """FP32 flops (FMA = 2; a floor, fract, square root or reciprocal = 1) of
    one DAS launch (or its dL/dc adjoint) with n_act active terms
    (apodization > 0), counted as the kernels evaluate each term.  The cubic
    read's coefficients of a trace's sample interval are formed once (10
    flops; 20 for IQ's real and imaginary parts; the adjoint forms the
    derivative's 3 coefficients, 10) and every term evaluates its polynomial
    by Horner's rule (6; the derivative's quadratic 4).

    Per active term: HERCULES (one receive path per term) delay 12 (dx,
    rho^2, (d/k)^2, sqrt, d/k + z/k, rcp, fma, floor, fract) + apodization 4
    (the Hann table: scale, floor, and one fma from the entry's base and
    slope); FORCES, TPW and
    VLS separate the path into a transmit part per (point, transmit)
    (FORCES distance to the column 8, TPW x sin + z (cos - 1) 4, VLS signed
    distance to the line 11) and a receive part with its weight per active
    (point, row) (path 9 + Hann polynomial in u^2 13 = 22), and a term adds
    the two and takes floor and fract (3).  Then the read (Horner 6) and the
    accumulation: real 2; IQ two reads (12) + phase 2 + the rotation 13
    (fract, sine, cosine, two weight products, complex multiply-add 8);
    dL/dc the derivative (4) + the sums of w v' and w v' s (4)."""
    mode = desc["mode"]
    traces = desc["n_tx"] * desc["n_ch"]
    coef = 10.0 * traces * desc["n_samples"] * (2 if iq else 1)
    if adjoint_c:
        per_term = 4 + 4
    elif iq:
        per_term = 12 + 2 + 13
    else:
        per_term = 6 + 2
    if mode == "hercules":
        return n_act * (12 + 4 + per_term) + coef
    n_tx = desc["n_tx"]
    n_pts = int(np.prod(desc["dims"]))
    f_tx = {"forces": 8, "tpw": 4, "vls": 11}[mode]
    return n_act * (3 + per_term + 22.0 / n_tx) + f_tx * n_pts * n_tx + coef


def _oracle_rate(desc, H, rf, n_vox=None, seed=0):
    """Seconds of the FP64 oracle's decode and of its DAS over one whole frame
    (DAS on n_vox random points scaled to the frame when n_vox is given)."""
    import oracle
    t = time.perf_counter()
    e = oracle.decode(H, rf)
    t_dec = time.perf_counter() - t
    nv = int(np.prod(desc["dims"]))
    t = time.perf_counter()
    if n_vox is None or n_vox >= nv:
        oracle.das(desc, e)
        t_das = time.perf_counter() - t
    else:
        vox = np.sort(np.random.default_rng(seed).choice(nv, n_vox, replace=False))
        oracle.das_points(desc, e, vox)
        t_das = (time.perf_counter() - t) * nv / n_vox
    return t_dec, t_das


def cpu_baseline_per_config(stream4=None):
    """The oracle on the other workloads, all host cores and one thread:
    workload 0 (FORCES 128x128 B-scan) and one frame of workload 3 (FORCES
    256x256, 64 x 64 x 2048) decode + DAS of the whole image (one thread:
    DAS on a quarter of the pixels, scaled); workload 4 on 8 of its 64 frames
    (the first four planes and the first four volumes), DAS on random points
    scaled to each frame, as a rate for the whole stream."""
    import oracle
    import synth
    cores = oracle.threads()
    out = {}
    for k, name in ((0, "workload0_forces_128x128"), (3, "workload3_forces_256x256_per_frame")):
        if k == 0:
            desc, H, rf, _ = synth.make_inputs(0)
        else:
            desc, H, rfs, _ = synth.make_inputs(3, frame=0)
            rf = rfs[0]
        nv = int(np.prod(desc["dims"]))
        nominal = nv * desc["n_tx"] * desc["n_ch"]
        rec = {}
        for threads, n_vox in ((cores, None), (1, nv // 4)):
            oracle.threads(threads)
            t_dec, t_das = _oracle_rate(desc, H, rf, n_vox)
            rec[f"threads_{threads}"] = {
                "decode_s": round(t_dec, 4), "das_s": round(t_das, 4),
                "G_samples_per_s": round(nominal / (t_dec + t_das) / 1e9, 4),
                "frames_per_s": round(1.0 / (t_dec + t_das), 3),
                "sample": "whole image" if n_vox is None else
                          f"DAS on {n_vox} random pixels of {nv}, scaled"}
        oracle.threads(cores)
        out[name] = rec
    if stream4 is not None:
        descs, Hs, rfs = stream4
        kinds = ["2d" if d["mode"] == "forces" else "3d" for d in descs]
        pick = [i for i, k in enumerate(kinds) if k == "2d"][:4] + \
               [i for i, k in enumerate(kinds) if k == "3d"][:4]
        t_tot, nom = 0.0, 0
        for i in pick:
            t_dec, t_das = _oracle_rate(descs[i], Hs[i], rfs[i], n_vox=400, seed=i)
            t_tot += t_dec + t_das
            nom += int(np.prod(descs[i]["dims"])) * descs[i]["n_tx"] * descs[i]["n_ch"]
        rate = nom / t_tot
        total = sum(int(np.prod(d["dims"])) * d["n_tx"] * d["n_ch"] for d in descs)
        out["workload4_stream"] = {
            f"threads_{cores}": {"G_samples_per_s": round(rate / 1e9, 4),
                                 "stream_s": round(total / rate, 1),
                                 "sample": f"frames {pick} (n_tx "
                                           f"{[descs[i]['n_tx'] for i in pick]}): full decode, "
                                           "DAS on 400 random points per frame scaled to the "
                                           "frame; stream time extrapolated at that rate"}}
    return out


def cpu_baseline(desc, H, rf, budget_s: float):
    """FP64 oracle on the host cores: full decode + DAS on a random voxel sample."""
    import oracle
    threads = oracle.threads()
    t = time.perf_counter()
    e = oracle.decode(H, rf)
    t_dec = time.perf_counter() - t
    nv = int(np.prod(desc["dims"]))
    rng = np.random.default_rng(99)
    probe = rng.choice(nv, 512, replace=False)
    t = time.perf_counter()
    oracle.das_points(desc, e, probe)
    per_vox = (time.perf_counter() - t) / probe.size
    n = int(min(nv, max(1024, (budget_s - t_dec) / max(per_vox, 1e-9))))
    vox = np.sort(rng.choice(nv, n, replace=False))
    t = time.perf_counter()
    ref = oracle.das_points(desc, e, vox)
    t_das = time.perf_counter() - t
    step = t_dec + t_das * nv / n          # one full volume at the sampled rate
    nominal = nv * desc["n_tx"] * desc["n_ch"]
    return dict(value=nominal / step / 1e9, unit="G voxel*tx*ch samples/s", cores=threads,
                kind="oracle",
                sample=f"full decode ({t_dec:.1f} s) + DAS of {n} random voxels of {nv} "
                       f"({t_das:.1f} s), scaled to one volume"), e, vox, ref


def precision_study(torch, bfm, desc, H, rf_d, e_mfma, out_f32, e64, vox, ref, n_ref=20000):
    """The precision variants on the headline data (workload 2), against the
    FP64 oracle: decode by int8 MFMA (the default, e_mfma) and by FP32 FMA --
    max-abs error over the whole decoded set; DAS of FP32 and of BF16-stored
    decoded data (FP32 accumulation) -- max-abs and relative L2 error on the
    oracle's sampled voxels (vox, ref).  For BF16 the error of the kernel
    alone is also given, against the oracle's DAS of the BF16-rounded data
    (the first n_ref sampled voxels)."""
    import oracle
    res = {}
    e_fma = bfm.Plan(desc, H, decode_algo="fma").decode(rf_d)
    for name, e in (("decode_mfma", e_mfma), ("decode_fma", e_fma)):
        err = float(np.max(np.abs(e.cpu().numpy().astype(np.float64) - e64)))
        res[name] = {"max_abs": err, "bit_exact": err == 0.0}
    del e_fma
    pb = bfm.Plan(desc, H, e_type="bf16")
    e_b = pb.decode(rf_d)
    out_b = pb.das(e_b)
    torch.cuda.synchronize()
    scale = float(np.max(np.abs(ref)))
    for name, out in (("das_f32", out_f32), ("das_bf16", out_b)):
        got = out.cpu().numpy().reshape(-1)[vox].astype(np.float64)
        res[name] = {"max_abs": float(np.max(np.abs(got - ref))),
                     "max_abs_rel_to_peak": float(np.max(np.abs(got - ref)) / scale),
                     "rel_l2": float(np.linalg.norm(got - ref) / np.linalg.norm(ref))}
    sub = vox[:n_ref]
    e_round = e_b.float().cpu().numpy().astype(np.float64)
    ref_r = oracle.das_points(desc, e_round, sub)
    got_b = out_b.cpu().numpy().reshape(-1)[sub].astype(np.float64)
    res["das_bf16"]["rel_l2_vs_rounded_data"] = float(np.linalg.norm(got_b - ref_r) /
                                                       np.linalg.norm(ref_r))
    res["sample"] = (f"{len(vox)} random voxels of {int(np.prod(desc['dims']))} "
                     f"({len(sub)} for the rounded-data reference)")
    return res


VARIANT_NAMES = {0: "lds", 1: "gather", 2: "lds2"}
KERNEL_SOURCES = ("paper_2512_11086_amd/csrc/bf_das_lds.hip", "paper_2512_11086_amd/csrc/bf_das_lds_block.h",
                  "paper_2512_11086_amd/csrc/bf_common.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "das_hercules_128x128x256_traffic.json")


def kernel_hash() -> str:
    """Hash of the DAS kernel sources without their comments and with
    whitespace collapsed: it changes with the code the counters measured, not
    with its comments."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fp:
            text = fp.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per DAS launch from the committed rocprofv3 counter summary,
    or None when the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fp:
            t = json.load(fp)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("das_hbm_bytes_per_launch")


def traffic_run():
    """Short fixed sequence for rocprofv3 --pmc runs: a plain 512 MiB copy
    (counter calibration), then 3 decodes and 3 DAS launches of the workload."""
    import torch
    import paper_2512_11086_amd as bfm
    import synth
    dev = torch.device("cuda:0")
    src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    desc, H, rf, _ = synth.make_inputs(1)
    plan = bfm.Plan(desc, H)
    rf_d = torch.from_numpy(rf).to(dev)
    e_d = torch.empty(rf.shape, dtype=torch.float32, device=dev)
    out_d = torch.empty(plan.out_shape, dtype=torch.float32, device=dev)
    for _ in range(3):
        plan.decode(rf_d, out=e_d)
    torch.cuda.synchronize()
    for _ in range(3):
        plan.das(e_d, out=out_d)
    torch.cuda.synchronize()
    print(json.dumps({"traffic_run": "done", "kernel_hash": kernel_hash(),
                      "das_config": plan.info()}), flush=True)


def _counter_per_dispatch(db: str, counter: str) -> list:
    """(kernel name, value) per dispatch of one rocprofv3 --pmc results
    database, in dispatch order."""
    import sqlite3
    con = sqlite3.connect(db)
    try:
        rows = con.execute("select dispatch_id, kernel_name, sum(value) from counters_collection "
                           "where counter_name = ? group by dispatch_id order by dispatch_id",
                           (counter,)).fetchall()
    finally:
        con.close()
    return [(n, float(v)) for _, n, v in rows]


def traffic_summary(fetch_db: str, write_db: str):
    """Write the HBM traffic summary of the DAS kernel from the results of
    the two counter runs of --traffic (FETCH_SIZE, then WRITE_SIZE, KiB per
    dispatch).  Each counter is scaled by what it reads for the plain 512 MiB
    copy at the start of the sequence (the dispatch outside this library that
    fetches the most; its write is read from the same kernel)."""
    fetch = _counter_per_dispatch(fetch_db, "FETCH_SIZE")
    write = _counter_per_dispatch(write_db, "WRITE_SIZE")
    mib512 = 512.0 * 1024.0           # KiB
    copy_name, copy_fetch = max(((n, v) for n, v in fetch if "bf::" not in n), key=lambda t: t[1])
    copy_write = max(v for n, v in write if n == copy_name)
    das_f = [v for n, v in fetch if "das_lds_kernel" in n]
    das_w = [v for n, v in write if "das_lds_kernel" in n]
    das_name = next(n for n, _ in fetch if "das_lds_kernel" in n)
    f_scale, w_scale = mib512 / copy_fetch, mib512 / copy_write
    f_raw, w_raw = sum(das_f) / len(das_f), sum(das_w) / len(das_w)
    out = {
        "kernel": das_name,
        "workload": "HERCULES 128 tx x 128 ch x 2048 -> 128x128x256, c = 1540 m/s",
        "kernel_hash": kernel_hash(),
        "fetch_kib_raw": f_raw,
        "write_kib_raw": w_raw,
        "fetch_scale": f_scale,
        "write_scale": w_scale,
        "das_hbm_bytes_per_launch": int(round((f_raw * f_scale + w_raw * w_scale) * 1024)),
        "algorithmic_hbm_bytes_per_launch": 128 * 128 * 2048 * 4 + 128 * 128 * 256 * 4,
        "calibration_kernel": copy_name[:120],
        "commands": [
            "rocprofv3 --pmc FETCH_SIZE --kernel-trace -d <dir> -o run -- python bench.py --traffic",
            "rocprofv3 --pmc WRITE_SIZE --kernel-trace -d <dir> -o run -- python bench.py --traffic",
            "python bench.py --traffic-summary <fetch dir>/run_results.db <write dir>/run_results.db",
        ],
    }
    with open(TRAFFIC_FILE, "w") as fp:
        json.dump(out, fp, indent=1)
        fp.write("\n")
    print(json.dumps(out))


def plane_run():
    """Short fixed sequence for rocprofv3 runs on the 256 x 256 FORCES plane
    (one frame of workload 3, 64 x 64 x 2048): 3 DAS launches, 3 dL/dc
    adjoint launches and 3 RF-gradient adjoint launches, then 20 timed DAS
    and 20 timed dL/dc launches (HIP events on the launch stream)."""
    import torch
    import paper_2512_11086_amd as bfm
    import synth
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    desc, H, rfs, info = synth.make_inputs(3, frame=0)
    plan = bfm.Plan(desc, H)
    e = plan.decode(torch.from_numpy(rfs[0]).to(dev))
    c = float(info["c_true"])
    img = plan.das(e, c=c)
    _, g = bfm.sharpness(img.reshape(1, -1))
    g = g.reshape(img.shape)
    ge = torch.empty(e.shape, dtype=torch.float32, device=dev)
    for _ in range(3):
        plan.das(e, c=c, out=img)
    for _ in range(3):
        plan.das_adjoint(e, g, c=c, want_e=False)
    for _ in range(3):
        plan.das_adjoint(None, g, c=c, want_c=False, out_e=ge)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(stream)
    for _ in range(20):
        plan.das(e, c=c, out=img)
    ev[1].record(stream)
    for _ in range(20):
        plan.das_adjoint(e, g, c=c, want_e=False)
    ev[2].record(stream)
    torch.cuda.synchronize()
    print(json.dumps({"plane_run": "done", "das_ms": ev[0].elapsed_time(ev[1]) / 20,
                      "adjoint_c_ms": ev[1].elapsed_time(ev[2]) / 20, "config": plan.info()}),
          flush=True)


def batched_comparison(torch, bfm, stream4, reps: int):
    """64-frame uFORCES/uHERCULES stream: plain per-frame launches vs one
    persistent launch per kernel class vs the same captured in a hipGraph.
    The per-frame loop is also timed as its decode launches alone and its
    DAS launches alone (the decode share of the stream).  Per-frame and graph
    are timed twice, the second time after the others, and the faster pass
    of each is reported."""
    descs, Hs, rfs = stream4
    dev = torch.device("cuda:0")
    rf_d = [torch.from_numpy(r).to(dev) for r in rfs]
    bp = bfm.BatchPlan(descs, Hs)
    plans = [bfm.Plan(d, H) for d, H in zip(descs, Hs)]
    outs_b = [torch.empty(s, device=dev) for s in bp.out_shapes]
    outs_g = [torch.empty(s, device=dev) for s in bp.out_shapes]
    outs_p = [torch.empty(p.out_shape, device=dev) for p in plans]
    es = [torch.empty(r.shape, dtype=torch.float32, device=dev) for r in rfs]

    def per_frame():
        for p, r, e, o in zip(plans, rf_d, es, outs_p):
            p.decode(r, out=e)
            p.das(e, out=o)

    def decode_only():
        for p, r, e in zip(plans, rf_d, es):
            p.decode(r, out=e)

    def das_only():
        for p, e, o in zip(plans, es, outs_p):
            p.das(e, out=o)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    ms_pf = timed(per_frame)
    ms_dec = timed(decode_only)
    ms_das = timed(das_only)
    ms_ps = timed(lambda: bp.run(rf_d, outs_b))
    ms_gr = timed(lambda: bp.graph_launch(rf_d, outs_g))
    # a second, alternated pass of the two paths the speedup compares (the
    # clock differs between the first and later passes); the faster of each
    ms_pf = min(ms_pf, timed(per_frame))
    ms_gr = min(ms_gr, timed(lambda: bp.graph_launch(rf_d, outs_g)))
    # the same stream with tiles autotuned per problem-shape class (no cache:
    # every class is timed on the device)
    t = time.perf_counter()
    bp_t = bfm.BatchPlan(descs, Hs)
    bp_t.autotune(None)
    tune_s = time.perf_counter() - t
    outs_t = [torch.empty(s, device=dev) for s in bp_t.out_shapes]
    ms_gt = timed(lambda: bp_t.graph_launch(rf_d, outs_t))
    worst = 0.0
    for a_, b_, c_, d_ in zip(outs_p, outs_b, outs_g, outs_t):
        worst = max(worst, float((a_ - b_).norm() / a_.norm().clamp_min(1e-30)),
                    float((b_ - c_).norm() / b_.norm().clamp_min(1e-30)),
                    float((b_ - d_).norm() / b_.norm().clamp_min(1e-30)))
    paths = [bp.frame_info(f) for f in range(len(descs))]
    nominal = sum(int(np.prod(d["dims"])) * d["n_tx"] * d["n_ch"] for d in descs)
    n3 = sum(1 for d in descs if d["mode"] == "hercules")
    log(f"batched: per-frame {ms_pf:.2f} ms (decode {ms_dec:.2f}, DAS {ms_das:.2f}), "
        f"persistent {ms_ps:.2f} ms, graph {ms_gr:.2f} ms, autotuned graph {ms_gt:.2f} ms "
        f"(tuning {tune_s:.1f} s)")
    return {"frames": len(descs), "frames_3d": n3, "nominal_G_samples": round(nominal / 1e9, 2),
            "per_frame_ms": round(ms_pf, 3), "per_frame_decode_ms": round(ms_dec, 3),
            "per_frame_das_ms": round(ms_das, 3), "persistent_ms": round(ms_ps, 3),
            "graph_ms": round(ms_gr, 3), "autotuned_graph_ms": round(ms_gt, 3),
            "autotune_s": round(tune_s, 1),
            "speedup_graph_vs_per_frame": round(ms_pf / ms_gr, 3),
            "speedup_autotuned_graph_vs_per_frame": round(ms_pf / ms_gt, 3),
            "speedup_persistent_vs_per_frame": round(ms_pf / ms_ps, 3),
            "graph_G_samples_per_s": round(nominal / (ms_gr * 1e-3) / 1e9, 1),
            "frames_on_persistent_lds": sum(1 for p in paths if p["das_path"] == "persistent_lds"),
            "max_rel_l2_between_paths": worst}


def decode_share(torch, bfm, synth, reps: int = 20):
    """Decode and DAS times of the plane workloads (0: FORCES 128x128 from 32 x
    32 x 1024; 3: one FORCES 256x256 frame from 64 x 64 x 2048): the largest
    saving a decode fused into DAS could give is the decode's own time.  The
    fused kernel (bf_das_fused: the decode inside the DAS staging, one
    launch, same image bit for bit) is timed beside them."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = {}
    for k, name in ((0, "workload0"), (3, "workload3_per_frame")):
        if k == 0:
            desc, H, rf, _ = synth.make_inputs(0)
        else:
            desc, H, rfs, _ = synth.make_inputs(3, frame=0)
            rf = rfs[0]
        plan = bfm.Plan(desc, H)
        rf_d = torch.from_numpy(rf).to(dev)
        e = plan.decode(rf_d)
        img = plan.das(e)
        torch.cuda.synchronize()
        fused_img = plan.das_fused(rf_d)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        for _ in range(reps):
            plan.decode(rf_d, out=e)
        ev[1].record(stream)
        for _ in range(reps):
            plan.das(e, out=img)
        ev[2].record(stream)
        for _ in range(reps):
            plan.das_fused(rf_d, out=fused_img)
        ev[3].record(stream)
        torch.cuda.synchronize()
        dec = ev[0].elapsed_time(ev[1]) / reps
        das = ev[1].elapsed_time(ev[2]) / reps
        fused = ev[2].elapsed_time(ev[3]) / reps
        out[name] = {"decode_ms": round(dec, 4), "das_ms": round(das, 4),
                     "decode_share": round(dec / (dec + das), 4),
                     "fused_ms": round(fused, 4),
                     "fused_vs_decode_plus_das": round(fused / (dec + das), 3),
                     "fused_bitwise_equal": bool(torch.equal(fused_img, img))}
    return out


def iq_pipeline(torch, bfm, synth, desc, H, rf_d, n_act, reps: int):
    """Demodulate (Eq. 4) + decode complex int16 + IQ DAS of the same RF:
    36-tap low-pass (the paper's volume filter length), decimation 2 ->
    1024 complex samples at 15 MHz."""
    from synth.configs import iq_frontend
    taps, D, dq = iq_frontend(desc)
    n_tr = desc["n_tx"] * desc["n_ch"]
    dm = bfm.Demod(n_tr, desc["n_samples"], taps, desc["fc"], desc["fs"], D)
    plan = bfm.Plan(dq, H)
    stream = torch.cuda.current_stream()
    iq = dm(rf_d)
    e = plan.decode(iq)
    img = plan.das(e)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(reps)]
    for k in range(reps):
        ev[k][0].record(stream)
        dm(rf_d, out=iq)
        ev[k][1].record(stream)
        plan.decode(iq, out=e)
        ev[k][2].record(stream)
        plan.das(e, out=img)
        ev[k][3].record(stream)
    torch.cuda.synchronize()
    t = np.array([[ev[k][i].elapsed_time(ev[k][i + 1]) for i in range(3)] for k in range(reps)])
    _, _, das_ms = (float(v) for v in t.mean(axis=0))
    # the short kernels: 10 back-to-back launches each (single launches
    # between 40 ms DAS launches carry the event gaps)
    ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev2[0].record(stream)
    for _ in range(10):
        dm(rf_d, out=iq)
    ev2[1].record(stream)
    for _ in range(10):
        plan.decode(iq, out=e)
    ev2[2].record(stream)
    torch.cuda.synchronize()
    dem_ms = ev2[0].elapsed_time(ev2[1]) / 10
    dec_ms = ev2[1].elapsed_time(ev2[2]) / 10
    step = dem_ms + dec_ms + das_ms
    n_out = dm.n_out
    # demodulation: per output 2 flops per non-zero real or imaginary part of
    # the mixed taps h[k] exp(j 2 pi r k) (a real filter under quadrature
    # sampling, r = 1/4, has one non-zero part per tap) + the rotation (6);
    # HBM: 2 bytes in per input sample, 4 bytes out per output
    r = desc["fc"] / desc["fs"]
    q = 4.0 * ((r * np.arange(len(taps))) % 1.0)
    quarter = np.abs(q - np.round(q)) < 1e-12
    mix = np.where(quarter, 1j ** np.round(q), np.exp(2j * np.pi * q / 4.0))
    g = np.asarray(taps) * mix
    parts = int(np.count_nonzero(np.abs(g.real) > 0) + np.count_nonzero(np.abs(g.imag) > 0))
    dem_flops = n_tr * n_out * (2 * parts + 6)
    dem_bytes = n_tr * (2 * desc["n_samples"] + 4 * n_out)
    dem_tf = dem_flops / (dem_ms * 1e-3) / 1e12
    das_tf = algorithmic_flops(dq, n_act, iq=True) / (das_ms * 1e-3) / 1e12
    nominal = int(np.prod(dq["dims"])) * dq["n_tx"] * dq["n_ch"]
    return {
        "workload": "same RF -> demodulate (36-tap low-pass, D = 2, fd = 7.5 MHz) -> "
                    "decode complex int16 (128 x 128 x 1024 x 2) -> IQ DAS 128x128x256 complex",
        "ms_per_step": round(step, 4), "value": round(nominal / (step * 1e-3) / 1e9, 3),
        "unit": "G samples/s", "demod_ms": round(dem_ms, 4), "decode_ms": round(dec_ms, 4),
        "das_ms": round(das_ms, 4),
        "demod_roofline": {**alu_roofline(dem_tf),
                           "hbm_GBps": round(dem_bytes / (dem_ms * 1e-3) / 1e9, 1)},
        "das_roofline": alu_roofline(das_tf),
        "das_config": plan.info(),
    }


def envelope_stage(torch, bfm, img, reps: int = 10):
    """Envelope + log compression (60 dB) of the beamformed RF volume: one
    FFT analytic signal per depth column.  Timed with a given reference level
    (one fused pass) and with the image maximum (envelope pass + max, then a
    compression pass)."""
    env = bfm.Envelope(img.shape)
    out = torch.empty(img.shape, dtype=torch.float32, device=img.device)
    stream = torch.cuda.current_stream()
    res = {}
    for name, ref in (("fused_ms", 1.0), ("image_max_ms", 0.0)):
        env(img, "log", ref, 60.0, out=out)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            env(img, "log", ref, 60.0, out=out)
        b.record(stream)
        torch.cuda.synchronize()
        res[name] = round(a.elapsed_time(b) / reps, 4)
    # algorithmic HBM bytes of the fused pass: the image read once, written once
    nbytes = 2 * img.numel() * 4
    gbps = nbytes / (res["fused_ms"] * 1e-3) / 1e9
    res["workload"] = (f"log envelope (60 dB) of the {tuple(img.shape)} RF volume, "
                       f"FFT analytic signal along depth ({img.shape[-1]})")
    res["roofline"] = {"bound": "hbm", "achieved": round(gbps, 1), "peak": 8000.0, "unit": "GB/s",
                       "frac": round(gbps / 8000.0, 4), "traffic": None}
    return res


def autofocus_stage(torch, bfm, synth, reps: int = 5):
    """Differentiable FORCES workload (256x256 plane, 64 tx x 64 ch, 2048
    samples, 8 frames).  The gradient step -- forward DAS, the sharpness loss
    with its image gradient, and the adjoint for dL/dc alone (the autofocus
    gradient) -- is timed two ways: with the 8 frames stacked (bf_das_frames,
    one DAS launch per frame; one sharpness launch for the 8 images;
    bf_das_adjoint_frames, one launch per gradient for all frames), and frame
    by frame (bf_das / bf_das_adjoint per frame).  Also timed: the adjoint with the RF gradient
    (8 x 64 x 64 x 2048, LDS windows added to it with FP32 atomics), with and
    without dL/dc.  Adjoint roofline: algorithmic_flops(..., adjoint_c=True)
    (the separable FORCES path, derivative coefficients once per trace sample
    interval) over the stacked launch."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    desc, H, rfs, info = synth.make_inputs(3)
    plan = bfm.Plan(desc, H)
    nf = len(rfs)
    es = torch.stack([plan.decode(torch.from_numpy(r).to(dev)) for r in rfs]).contiguous()
    c = float(info["c_true"])
    imgs = plan.das(es, c=c)
    loss, g = bfm.sharpness(imgs.reshape(nf, -1))
    g = g.reshape(imgs.shape)
    ge, gc = plan.das_adjoint(es, g, c=c)
    torch.cuda.synchronize()

    def timed(fn):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(reps):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / (reps * nf)      # ms per frame

    st = {
        "das_ms": timed(lambda: plan.das(es, c=c, out=imgs)),
        "sharpness_ms": timed(lambda: bfm.sharpness(imgs.reshape(nf, -1))),
        "adjoint_c_ms": timed(lambda: plan.das_adjoint(es, g, c=c, want_e=False)),
        "adjoint_e_and_c_ms": timed(lambda: plan.das_adjoint(es, g, c=c, out_e=ge)),
        "adjoint_e_ms": timed(lambda: plan.das_adjoint(None, g, c=c, want_c=False, out_e=ge)),
    }
    img1, ge1 = imgs[0].clone(), ge[0].clone()

    def per_frame(fn):
        return lambda: [fn(f) for f in range(nf)]

    pf = {
        "das_ms": timed(per_frame(lambda f: plan.das(es[f], c=c, out=img1))),
        "sharpness_ms": timed(per_frame(lambda f: bfm.sharpness(img1.reshape(1, -1)))),
        "adjoint_c_ms": timed(per_frame(lambda f: plan.das_adjoint(es[f], g[f], c=c,
                                                                   want_e=False))),
        "adjoint_e_and_c_ms": timed(per_frame(lambda f: plan.das_adjoint(es[f], g[f], c=c,
                                                                         out_e=ge1))),
        "adjoint_e_ms": timed(per_frame(lambda f: plan.das_adjoint(None, g[f], c=c, want_c=False,
                                                                   out_e=ge1))),
    }
    n_act = active_terms(desc, dev)
    tf = algorithmic_flops(desc, n_act, adjoint_c=True) / (st["adjoint_c_ms"] * 1e-3) / 1e12
    nominal = int(np.prod(desc["dims"])) * desc["n_tx"] * desc["n_ch"]
    out = {"workload": "FORCES 256x256 plane, 64 tx x 64 ch x 2048 samples, 8 frames: "
                       "DAS + sharpness + adjoint dL/dc with the 8 frames stacked (one call "
                       "each: the DAS one launch per frame, the sharpness and each adjoint "
                       "gradient one launch for all 8); per_frame_calls: one call per frame; "
                       "times in ms per frame"}
    for k, v in st.items():
        out[k] = round(v, 4)
    step = st["das_ms"] + st["sharpness_ms"] + st["adjoint_c_ms"]
    step_pf = pf["das_ms"] + pf["sharpness_ms"] + pf["adjoint_c_ms"]
    out["gradient_step_ms_per_frame"] = round(step, 4)
    out["value"] = round(nominal / (step * 1e-3) / 1e9, 2)
    out["unit"] = "G samples/s"
    out["per_frame_calls"] = {k: round(v, 4) for k, v in pf.items()}
    out["per_frame_calls"]["gradient_step_ms_per_frame"] = round(step_pf, 4)
    out["adjoint_roofline"] = alu_roofline(tf)
    return out


def n4_workloads(torch, bfm, synth, reps: int = 6):
    """Decode + DAS of the additional transmit models at the headline volume
    size (128x128 array, 2048 samples, 128x128x256 voxels): diverging-wave
    HERCULES (LDS kernel, two points per lane), TPW with 32 angles and
    VLS-128 (separable LDS kernels, unencoded data), and the cross-plane
    FORCES pair as one captured graph of the batched path against plain
    per-frame calls."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    res = {}
    names = {5: "diverging_hercules", 6: "tpw_32", 7: "vls_128"}
    for k, name in names.items():
        desc, H, rf, _ = synth.make_inputs(k)
        plan = bfm.Plan(desc, H)
        rf_d = torch.from_numpy(rf).to(dev)
        e = plan.decode(rf_d)
        img = plan.das(e)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        for _ in range(reps):
            plan.decode(rf_d, out=e)
        ev[1].record(stream)
        for _ in range(reps):
            plan.das(e, out=img)
        ev[2].record(stream)
        torch.cuda.synchronize()
        dec_ms = ev[0].elapsed_time(ev[1]) / reps
        das_ms = ev[1].elapsed_time(ev[2]) / reps
        n_act = active_terms(desc, dev)
        tf = algorithmic_flops(desc, n_act) / (das_ms * 1e-3) / 1e12
        nominal = int(np.prod(desc["dims"])) * desc["n_tx"] * desc["n_ch"]
        res[name] = {"n_tx": desc["n_tx"], "decode_ms": round(dec_ms, 4),
                     "das_ms": round(das_ms, 3),
                     "value": round(nominal / ((dec_ms + das_ms) * 1e-3) / 1e9, 2),
                     "unit": "G samples/s", "variant": VARIANT_NAMES[plan.info()["variant"]],
                     "roofline": alu_roofline(tf)}
        log(f"{name}: decode {dec_ms:.3f} ms, DAS {das_ms:.3f} ms")
        del plan, rf_d, e, img
    descs, Hs, rfs, _ = synth.make_inputs(8)
    bp = bfm.BatchPlan(descs, Hs)
    rf_d = [torch.from_numpy(r).to(dev) for r in rfs]
    outs = [torch.empty(s, device=dev) for s in bp.out_shapes]
    bp.graph_launch(rf_d, outs)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    xreps = 2 * reps          # (about a millisecond per pass)
    # the same pair as plain per-frame calls (decode + DAS of each plane)
    plans = [bfm.Plan(d, H) for d, H in zip(descs, Hs)]
    es = [p.decode(r) for p, r in zip(plans, rf_d)]
    outs_p = [p.das(e) for p, e in zip(plans, es)]

    def per_frame():
        for p, r, e, o in zip(plans, rf_d, es, outs_p):
            p.decode(r, out=e)
            p.das(e, out=o)

    def graph():
        bp.graph_launch(rf_d, outs)

    per_frame()
    torch.cuda.synchronize()
    # the two measured twice, alternating (the first pass after the other
    # workloads runs at a different clock), the faster pass of each reported
    times = {"graph": [], "per_frame": []}
    for _ in range(2):
        for name, fn in (("graph", graph), ("per_frame", per_frame)):
            a.record(stream)
            for _ in range(xreps):
                fn()
            b.record(stream)
            torch.cuda.synchronize()
            times[name].append(a.elapsed_time(b) / xreps)
    res["cross_plane_graph_ms"] = round(min(times["graph"]), 3)
    res["cross_plane_per_frame_ms"] = round(min(times["per_frame"]), 3)
    res["cross_plane"] = ("FORCES x-z (columns) + y-z (rows) planes, 256x256 each, 128 tx x 128 ch "
                          "x 2048: one graph of the batched path vs per-frame calls")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-frame batched comparison")
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--no-iq", action="store_true", help="skip the demodulation + IQ pipeline")
    ap.add_argument("--iq-reps", type=int, default=3)
    ap.add_argument("--no-n4", action="store_true", help="skip the TPW / VLS / diverging workloads")
    ap.add_argument("--no-autofocus", action="store_true",
                    help="skip the differentiable FORCES workload (adjoint, sharpness)")
    ap.add_argument("--traffic", action="store_true",
                    help="only run the short kernel sequence used for counter collection")
    ap.add_argument("--plane", action="store_true",
                    help="only run the short FORCES-plane sequence used for profiles")
    ap.add_argument("--fused", action="store_true",
                    help="only time decode, DAS and the fused decode + DAS on the FORCES "
                         "planes of workloads 0 and 3 (the decode_share object)")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="write the DAS traffic summary from the two --traffic counter runs")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary)
        return
    if args.traffic:
        traffic_run()
        return
    if args.plane:
        plane_run()
        return
    if args.fused:
        import torch
        import paper_2512_11086_amd as bfm
        import synth
        print(json.dumps({"decode_share": decode_share(torch, bfm, synth, reps=5)}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU; multi-GPU runs are not part of this build "
              "(frames or receive channels would shard with no or one all-reduce).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2512_11086_amd as bfm
    import synth

    dev = torch.device("cuda:0")
    t = time.perf_counter()
    desc, H, rf, _ = synth.make_inputs(1)
    log(f"inputs generated in {time.perf_counter() - t:.1f} s")
    plan = bfm.Plan(desc, H)
    rf_d = torch.from_numpy(rf).to(dev)
    e_d = torch.empty(rf.shape, dtype=torch.float32, device=dev)
    out_d = torch.empty(plan.out_shape, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        plan.decode(rf_d, out=e_d)
        plan.das(e_d, out=out_d)
    torch.cuda.synchronize()
    log("warmup done")

    K = args.steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record(stream)
    for k in range(K):
        ev[k][0].record(stream)
        plan.decode(rf_d, out=e_d)
        ev[k][1].record(stream)
        plan.das(e_d, out=out_d)
        ev[k][2].record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_step = start.elapsed_time(stop) / K
    dec_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    das_ms = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    log(f"step {ms_step:.3f} ms (decode {dec_ms:.3f} ms, DAS {das_ms:.3f} ms), wall {t_wall:.2f} s")

    nv = int(np.prod(desc["dims"]))
    nominal = nv * desc["n_tx"] * desc["n_ch"]
    value = nominal / (ms_step * 1e-3) / 1e9
    n_act = active_terms(desc, dev)
    # algorithmic FP32 work of the launch (algorithmic_flops)
    achieved = algorithmic_flops(desc, n_act) / (das_ms * 1e-3) / 1e12
    dec_bytes = rf.size * 2 + rf.size * 4
    res = {
        "metric": "G voxel*tx*ch samples/s (+ volumes/s), decode + DAS at oracle accuracy",
        "value": round(value, 3),
        "unit": "G samples/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded point + speckle scene, int16 RF)",
        "config": {"workload": "HERCULES volume 128x128 array, 128 tx x 128 ch x 2048 samples "
                               "-> 128x128x256 voxels, cubic",
                   "n_tx": 128, "n_ch": 128, "n_samples": 2048, "out_dims": [128, 128, 256]},
        "volumes_per_s": round(1e3 / ms_step, 3),
        "decode_ms": round(dec_ms, 4), "das_ms": round(das_ms, 4),
        "decode_hbm_GBps": round(dec_bytes / (dec_ms * 1e-3) / 1e9, 1),
        "active_term_fraction": round(n_act / nominal, 4),
        "roofline": alu_roofline(achieved, measured_traffic()),
        "lds_roofline": lds_roofline(n_act, nominal, das_ms),
        "das_ms_median": round(float(np.median([b.elapsed_time(c) for _, b, c in ev])), 4),
    }
    res["das_config"] = plan.info()
    res["envelope"] = envelope_stage(torch, bfm, out_d)
    log(f"envelope {res['envelope']['fused_ms']:.4f} ms")
    if not args.no_iq:
        res["iq"] = iq_pipeline(torch, bfm, synth, desc, H, rf_d, n_act, args.iq_reps)
        log(f"IQ pipeline {res['iq']['ms_per_step']:.3f} ms")
    if not args.no_n4:
        res["n4"] = n4_workloads(torch, bfm, synth)
    if not args.no_autofocus:
        res["autofocus"] = autofocus_stage(torch, bfm, synth)
        log(f"autofocus step {res['autofocus']['gradient_step_ms_per_frame']:.3f} ms per frame "
            f"(stacked frames; one call per frame: "
            f"{res['autofocus']['per_frame_calls']['gradient_step_ms_per_frame']:.3f} ms)")
    res["decode_share"] = decode_share(torch, bfm, synth)
    res["decode_share"]["workload1"] = {"decode_ms": round(dec_ms, 4), "das_ms": round(das_ms, 4),
                                        "decode_share": round(dec_ms / (dec_ms + das_ms), 4)}
    stream4 = None
    if not args.no_batch or not args.no_cpu:
        t = time.perf_counter()
        descs4, Hs4, rfs4, _ = synth.make_inputs(4)
        stream4 = (descs4, Hs4, rfs4)
        log(f"batched inputs ({len(descs4)} frames) generated in {time.perf_counter() - t:.1f} s")
    if not args.no_batch:
        res["batched"] = batched_comparison(torch, bfm, stream4, args.batch_reps)
        b = res["batched"]
        res["decode_share"]["workload4_per_frame_loop"] = {
            "decode_ms": b["per_frame_decode_ms"], "das_ms": b["per_frame_das_ms"],
            "decode_share": round(b["per_frame_decode_ms"] /
                                  (b["per_frame_decode_ms"] + b["per_frame_das_ms"]), 4)}
    if not args.no_cpu:
        cb, e64, vox, ref = cpu_baseline(desc, H, rf, args.cpu_budget)
        cb["per_config"] = cpu_baseline_per_config(stream4)
        res["cpu_baseline"] = cb
        got = out_d.cpu().numpy().reshape(-1)[vox].astype(np.float64)
        res["sampled_rel_l2_vs_oracle"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        res["precision"] = precision_study(torch, bfm, desc, H, rf_d, e_d, out_d, e64, vox, ref)
        log("precision study: " + json.dumps(res["precision"]))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
