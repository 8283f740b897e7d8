#!/usr/bin/env python3
"""Throughput of the batched fused RSFT hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): 128 frames of
1024x1024 complex64, each with K = 20 off-grid tones (frequencies uniform in
[0,1)^2, Rayleigh amplitudes at per-sample SNR uniform in [-10, 10] dB) in
CN(0,1) noise; B = 64x64 buckets, T = 3 permutation rounds, Pfa = 1e-4,
60 dB Dolph-Chebyshev windows, one sigma set for the batch. Seeded synthetic
data (no dataset is involved).

One step = one rsft_execute over the batch: fold (window, permutation, flat
window, aliasing for all rounds), MFMA DFT + first-stage threshold, voting +
second stage, ordered compaction + off-grid estimates; the detection records
end in device memory. Inputs are resident in HBM before timing starts; two
1 GiB input buffers alternate so the 256 MB last-level cache cannot serve
repeated reads.

The same JSON line also reports the other batched workloads (1024 x 256x256
complex128, 64 radar cubes of 256x128x32, 512 frames of uneven shapes,
16 x 2048x2048; --skip-workloads leaves them out), a refinement run, the
SRUR radar cubes, the same-GPU comparators and the CPU oracle on a sample.

Prints one JSON line on stdout; progress goes to stderr.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from synth import scoring  # noqa: E402

METRIC = "frames/s + HBM GB/s: batched fused RSFT vs per-frame RSFT at equal Pd/Pfa"
HBM_PEAK_GBS = 8000.0
WORKLOAD = "offgrid_1024x1024"
FRAMES = 128
COUNTERS_FILE = os.path.join(ROOT, "profiles", "fold_1024x1024x128_hbm_counters.json")
# the sources the fold kernel is built from: its counters stay valid while
# these are unchanged
FOLD_SOURCES = [os.path.join(ROOT, "paper_1610_01050_amd", "csrc", f)
                for f in ("fold.hip", "device_common.h", "rsft_internal.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for path in FOLD_SOURCES:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def fold_kernel_key(rounds, fold_cfg):
    """Template signature of the fold kernel variant a launch shape selects."""
    nt = "true" if fold_cfg["nontemporal"] else "false"
    return f"fold_kernel<{min(rounds, 4)}, {fold_cfg['vec']}, {fold_cfg['threads']}, false, {nt}>"


def measured_traffic(rounds, fold_cfg):
    """HBM bytes per fold launch of the chosen variant, from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source;
    else None."""
    try:
        with open(COUNTERS_FILE) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    v = c.get("variants", {}).get(fold_kernel_key(rounds, fold_cfg))
    return None if v is None else v["hbm_bytes_per_launch"]


def _counter_rows(directory):
    """(kernel name, counter, value) of every dispatch in rocprofv3's CSV
    counter-collection output under `directory`."""
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True):
        with open(path, newline="") as fh:
            for r in csv.DictReader(fh):
                rows.append((r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])))
    if not rows:
        raise SystemExit(f"no counter_collection.csv under {directory}")
    return rows


def summarize_counters(fetch_dir, write_dir, command_fetch, command_write):
    """Turn two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE; KiB per
    dispatch) into HBM bytes per fold launch. Both counters are scaled by what
    they read for the elementwise negation that makes the second input buffer,
    a kernel that reads and writes exactly 1 GiB."""
    calib_bytes = FRAMES * int(np.prod(synth.WORKLOADS[WORKLOAD]["shape"])) * 8
    out = {"kernel_source_sha256_16": kernel_source_hash(),
           "commands": {"FETCH_SIZE": command_fetch, "WRITE_SIZE": command_write},
           "calibration": {"kernel": "elementwise negation (torch.neg) of the 1 GiB input batch",
                           "bytes_read": calib_bytes, "bytes_written": calib_bytes},
           "variants": {}}
    per = {}
    for counter, directory in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        vals = {}
        for name, cn, v in _counter_rows(directory):
            if cn != counter:
                continue
            vals.setdefault(name, []).append(v)
        calib = [np.mean(v) for n, v in vals.items() if "neg" in n]
        if not calib:
            raise SystemExit(f"{counter}: no negation kernel in {directory}")
        scale = calib_bytes / (calib[0] * 1024.0)
        out["calibration"][counter + "_kib"] = calib[0]
        out["calibration"][counter + "_scale"] = scale
        for name, v in vals.items():
            if "fold_kernel<" not in name:
                continue
            key = name[name.index("fold_kernel<"):name.index(">", name.index("fold_kernel<")) + 1]
            per.setdefault(key, {})[counter] = (float(np.mean(v)), len(v), scale)
    N = int(np.prod(synth.WORKLOADS[WORKLOAD]["shape"]))
    B = int(np.prod(synth.WORKLOADS[WORKLOAD]["buckets"]))
    T = synth.WORKLOADS[WORKLOAD]["rounds"]
    algorithmic = FRAMES * (N * 8 + T * B * 8)
    for key, c in sorted(per.items()):
        if "FETCH_SIZE" not in c or "WRITE_SIZE" not in c:
            continue
        fetch = c["FETCH_SIZE"][0] * 1024.0 * c["FETCH_SIZE"][2]
        write = c["WRITE_SIZE"][0] * 1024.0 * c["WRITE_SIZE"][2]
        out["variants"][key] = {"fetch_kib": c["FETCH_SIZE"][0], "write_kib": c["WRITE_SIZE"][0],
                                "dispatches": [c["FETCH_SIZE"][1], c["WRITE_SIZE"][1]],
                                "hbm_fetch_bytes": fetch, "hbm_write_bytes": write,
                                "hbm_bytes_per_launch": fetch + write,
                                "algorithmic_bytes_per_launch": algorithmic,
                                "traffic_over_algorithmic": (fetch + write) / algorithmic}
    with open(COUNTERS_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out, indent=1))


def _short_kernel_name(name):
    """A kernel's name without its argument list and namespace."""
    n = name.split("(")[0]
    return n.replace("rsft::", "").replace("void ", "").strip()


def summarize_trace(directory, title, command):
    """Markdown summary of a rocprofv3 --kernel-trace --stats run: per
    kernel, calls, average / min / max duration (us) and share of the GPU
    time, from the kernel_stats.csv files under `directory`."""
    import csv
    import glob
    rows = {}
    for path in glob.glob(os.path.join(directory, "**", "*kernel_stats.csv"), recursive=True):
        with open(path, newline="") as fh:
            for r in csv.DictReader(fh):
                k = _short_kernel_name(r["Name"])
                c = rows.setdefault(k, [0, 0.0, math.inf, 0.0])
                calls = int(r["Calls"])
                c[0] += calls
                c[1] += float(r["TotalDurationNs"])
                c[2] = min(c[2], float(r["MinNs"]))
                c[3] = max(c[3], float(r["MaxNs"]))
    if not rows:
        raise SystemExit(f"no kernel_stats.csv under {directory}")
    total = sum(v[1] for v in rows.values())
    lines = [f"# {title}", "", "Command (from the repository root `R` on an MI355X, ROCm 7.2 rocprofv3):",
             "", "```", command, "```", "",
             "| Kernel | Calls | Average (us) | Min (us) | Max (us) | Share of GPU time |",
             "|---|---|---|---|---|---|"]
    for k, v in sorted(rows.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| `{k}` | {v[0]} | {v[1] / v[0] / 1e3:.1f} | {v[2] / 1e3:.1f} | {v[3] / 1e3:.1f} | "
                     f"{100 * v[1] / total:.1f}% |")
    print("\n".join(lines))


def summarize_pmc(directories, title, commands, kernels):
    """Markdown summary of rocprofv3 --pmc runs: for each kernel whose name
    contains one of `kernels`, the number of dispatches and each counter's
    average per dispatch, from the counter_collection.csv files under the
    given directories (one run per counter pass)."""
    per = {}
    for directory in directories:
        for name, counter, value in _counter_rows(directory):
            k = _short_kernel_name(name)
            if kernels and not any(q in k for q in kernels):
                continue
            per.setdefault(k, {}).setdefault(counter, []).append(value)
    counters = sorted({c for v in per.values() for c in v})
    lines = [f"# {title}", "", "Commands (from the repository root `R` on an MI355X, ROCm 7.2 rocprofv3):",
             "", "```"] + list(commands) + ["```", "",
             "Average per dispatch (SQ counters are summed over the chip; cycle counters of "
             "the SQ are in quad-cycles where rocprofv3 documents them so).", "",
             "| Kernel | Dispatches | " + " | ".join(counters) + " |",
             "|---|---|" + "---|" * len(counters)]
    for k, v in sorted(per.items()):
        n = max(len(x) for x in v.values())
        cells = [f"{np.mean(v[c]):,.0f}" if c in v else "" for c in counters]
        lines.append(f"| `{k}` | {n} | " + " | ".join(cells) + " |")
    print("\n".join(lines))


def score(recs, counts, metas, shape, frames):
    hits = tgt = fa = outside = 0
    D = len(shape)
    for f in frames:
        sel = recs[recs["frame"] == f]
        cells = [int(np.ravel_multi_index(tuple(int(v) for v in r["idx"][:D]), shape)) for r in sel]
        h, k, a, o = scoring.pd_pfa(cells, metas[f]["freqs"], shape)
        hits += h
        tgt += k
        fa += a
        outside += o
    return {"pd": hits / max(tgt, 1), "pfa": fa / max(outside, 1), "frames": len(frames)}


def cpu_baseline(frames_np, metas, shape, buckets, sigma, pfa, nsample):
    """The FP64 oracle on the first `nsample` frames of the batch, one thread:
    the whole step (literal Algorithm 1 in numpy, then the off-grid estimate
    of every detection)."""
    from threadpoolctl import threadpool_limits
    from oracle import rsft as oracle_rsft
    with threadpool_limits(limits=1):
        plan = oracle_rsft.OraclePlan(shape, buckets, sigma, 60.0, None, pfa)
        dets = []
        outs = []
        t0 = time.perf_counter()
        for f in range(nsample):
            out = oracle_rsft.rsft(frames_np[f], plan)
            out["estimates"] = oracle_rsft.estimate(out["detections"], out["buckets"], plan)
            dets.append(out["detections"])
            outs.append(out)
        dt = time.perf_counter() - t0
    hits = tgt = fa = outside = 0
    for f in range(nsample):
        h, k, a, o = scoring.pd_pfa(dets[f], metas[f]["freqs"], shape)
        hits += h
        tgt += k
        fa += a
        outside += o
    return {"value": nsample / dt, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"first {nsample} of the {FRAMES} frames of this workload: literal "
                      f"FP64 Algorithm 1 plus the estimate of every detection (numpy, "
                      f"one thread), {dt:.1f} s",
            "pd": hits / max(tgt, 1), "pfa": fa / max(outside, 1)}, dets, outs


def host_cpu():
    """The host's CPU model (from /proc/cpuinfo), its logical CPU count
    (os.cpu_count, what nproc reports without limits) and the CPUs this
    process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count(), "cpus_allowed": allowed}


def dense_cpu_leg(frames_np, shape, atten_db, pfa, nsample, workers):
    """The dense detector on the host: windowed 2-D FFT with
    scipy.fft.fftn(workers=...), |X|^2 and the exact exponential threshold
    sigma_n^2 ||w||^2 ln(1/Pfa) (Algorithm 2, one segment), on the first
    `nsample` frames; frames/s."""
    import scipy.fft
    from oracle import windows as oracle_windows
    w = np.multiply.outer(oracle_windows.dolph_chebyshev(shape[0], atten_db),
                          oracle_windows.dolph_chebyshev(shape[1], atten_db))
    thr = float(np.sum(w ** 2)) * math.log(1.0 / pfa)
    t0 = time.perf_counter()
    for f in range(nsample):
        X = scipy.fft.fftn(frames_np[f].astype(np.complex128) * w, workers=workers)
        np.flatnonzero((X.real ** 2 + X.imag ** 2) >= thr)
    dt = time.perf_counter() - t0
    return {"value": nsample / dt, "unit": "frames/s", "workers": workers,
            "sample": f"first {nsample} frames: FP64 windowed fftn + |X|^2 + threshold, {dt:.1f} s"}


def precision_report(gpu_buckets, gpu_flags, recs, outs, shape, buckets):
    """The FP32 path against the FP64 oracle on the same frames, stage by
    stage: bucket errors per round relative to the round's rms (max and
    99th percentile), first-stage flags that differ and how close their
    oracle power was to the threshold (|P - gamma| / gamma), detection-set
    differences, and for the detections both report, the magnitude's
    relative error and (cells both call peaks) the off-grid frequency's
    error in bins."""
    T = len(outs[0]["buckets"])
    B = int(np.prod(buckets))
    D = len(shape)
    bmax, bp99 = [], []
    flips, flip_band = 0, 0.0
    sym, common = 0, 0
    mag, frq = [], []
    peak_diff = 0
    for f, o in enumerate(outs):
        g = gpu_buckets[f].reshape((T,) + tuple(buckets))
        for r in range(T):
            rms = np.sqrt(np.mean(np.abs(o["buckets"][r]) ** 2))
            e = np.abs(g[r] - o["buckets"][r]).ravel() / rms
            bmax.append(float(e.max()))
            bp99.append(float(np.percentile(e, 99)))
        words = gpu_flags[f].reshape(T, -1).astype(np.uint32)
        j = np.arange(B)
        gfl = ((words[:, j // 32] >> (j % 32).astype(np.uint32)) & 1).astype(bool)
        ofl = o["flags"].reshape(T, -1)
        diff = gfl != ofl
        if diff.any():
            pw = np.abs(o["buckets"].reshape(T, -1)) ** 2
            band = np.abs(pw - o["gamma"][:, None]) / o["gamma"][:, None]
            flips += int(diff.sum())
            flip_band = max(flip_band, float(band[diff].max()))
        sel = recs[recs["frame"] == f]
        cells = np.ravel_multi_index(tuple(sel["idx"][:, d].astype(np.int64) for d in range(D)), shape)
        gmap = {int(c): r for c, r in zip(cells, sel)}
        est = {e["cell"]: e for e in o["estimates"]}
        sym += len(set(gmap) ^ set(est))
        for c in set(gmap) & set(est):
            common += 1
            r, e = gmap[c], est[c]
            mag.append(abs(float(r["magnitude"]) / e["magnitude"] - 1))
            if bool(r["is_peak"]) != e["is_peak"]:
                peak_diff += 1
            elif e["is_peak"]:
                frq.append(max(abs(((float(r["freq"][d]) - e["freq"][d] + 0.5) % 1.0) - 0.5) * shape[d]
                               for d in range(D)))
    mag = np.array(mag) if mag else np.zeros(1)
    frq = np.array(frq) if frq else np.zeros(1)
    return {"frames": len(outs),
            "bucket_rel_err": {"max": max(bmax), "p99_max_over_rounds": max(bp99)},
            "flag_flips": flips, "flip_max_distance_to_threshold": flip_band,
            "detections_common": common, "detections_differing": sym,
            "magnitude_rel_err": {"median": float(np.median(mag)), "max": float(mag.max())},
            "peak_flag_differences": peak_diff,
            "peak_freq_err_bins": {"p99": float(np.percentile(frq, 99)), "max": float(frq.max())}}


def paper_complexity(shape, buckets, T, K, measured_speedup, eta_m_per_dim=2.03, eta_p=1.0):
    """The paper's operation-count model for one frame (eq. RSFT_complexity,
    Table 2, with the FFT cost B log2 B that reproduces its argmins):
    RSFT T (N + B + B log2 B + K eta_m N / (B eta_p)) + N against one dense
    windowed FFT, N (1 + log2 N) + N; eta_m is the 6-dB width of the 60 dB
    window in bins per dimension. The paper names no hardware: context for
    the measured speedup over the dense FFT detector, not a target."""
    N = int(np.prod(shape))
    B = int(np.prod(buckets))
    eta_m = eta_m_per_dim ** len(shape)
    rsft = T * (N + B + B * math.log2(B) + K * eta_m * N / (B * eta_p)) + N
    dense = N * (1 + math.log2(N)) + N
    return {"rsft_ops_per_frame": rsft, "dense_ops_per_frame": dense, "model_ratio": dense / rsft,
            "measured_speedup_vs_dense_fft": measured_speedup,
            "note": "operation counts of the paper's complexity model (eq. RSFT_complexity, Table 2; "
                    "B log2 B, eta_m = 2.03 bins per dimension, eta_p = 1); the paper reports no "
                    "hardware, throughput or bandwidth"}


def refine_section(dev, steps=20, oracle_frames=1):
    """Detect -> estimate -> refine on 16 frames of 2048x2048 (K = 32
    off-grid tones, B = 128x128): the fused RSFT of the frames; starting
    tones chosen among the detector's peak records (select_tones: per-round
    agreement, then peeling on the residual of the tones found); their
    detector frequencies and amplitudes from the buckets
    (rsft_initial_amplitudes); then `steps` refinement iterations
    (rsft_refine) timed with events. Every true tone within one bin of a
    chosen start is scored before and after, by amplitude class. The
    least-squares fit the refinement converges to is compared with the one
    reached from the true parameters (the noise decides how far that fit is
    from the truth), and each frame's final loss with the loss at the true
    parameters. The FP64 oracle refines the first `oracle_frames` frames
    from the same start and observed buckets."""
    import torch
    from paper_1610_01050_amd import Plan
    from paper_1610_01050_amd.refine import refine, select_tones
    cfg = synth.WORKLOADS["offgrid_2048x2048"]
    F, K = 16, cfg["K"]
    shape = cfg["shape"]
    log(f"refinement: generating {F} frames {shape} ...")
    frames, metas = synth.make_batch("offgrid_2048x2048", F)
    sigma = synth.shared_sigma("offgrid_2048x2048")
    plan = Plan(shape, cfg["buckets"], rounds=cfg["rounds"], sigma=sigma, pfa=cfg["pfa"], max_batch=F,
                max_detections=1 << 17)
    x = torch.from_numpy(frames).to(dev)
    plan.execute(x)
    recs, _ = plan.detect()
    obs = torch.cat([b.reshape(-1) for b in plan.buckets()]).contiguous()
    t0 = time.perf_counter()
    f0, a0, counts = select_tones(plan, recs, K, observed=obs)
    torch.cuda.synchronize()
    select_s = time.perf_counter() - t0
    start = f0.cpu().numpy()
    passed = counts.cpu().numpy()
    refine(plan, obs, f0, a0, steps=2, record_loss=False, counts=counts)          # warm-up
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    fr, ar, _ = refine(plan, obs, f0, a0, steps=steps, record_loss=False, counts=counts)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    _, _, losses = refine(plan, obs, f0, a0, steps=steps, record_loss=True, counts=counts)
    losses = losses.cpu().numpy()
    end = fr.cpu().numpy()
    amp0 = a0.cpu().numpy()
    amp1 = ar.cpu().numpy()
    # the fit reached from the true parameters, and the loss there
    tf = torch.tensor(np.stack([m["freqs"] for m in metas]), dtype=torch.float64, device=dev).contiguous()
    ta = torch.tensor(np.stack([m["amps"] for m in metas]).astype(np.complex64), device=dev).contiguous()
    f_ml, _, _ = refine(plan, obs, tf, ta, steps=steps, record_loss=False)
    f_ml = f_ml.cpu().numpy()
    _, _, loss_truth = refine(plan, obs, tf, ta, steps=0, record_loss=True)
    loss_truth = loss_truth.cpu().numpy()[0]

    def circ(a, b):
        return (((a - b + 0.5) % 1.0) - 0.5) * np.array(shape)

    tones = []   # per true tone with a chosen start within one bin
    ml_diff = []
    complete = 0
    for f in range(F):
        found = 0
        for t, ft in enumerate(metas[f]["freqs"]):
            if passed[f] == 0:
                continue
            d = np.abs(circ(start[f, :passed[f]], ft)).max(axis=1)
            u = int(np.argmin(d))
            if d[u] >= 1.0:
                continue
            found += 1
            tones.append((f, t, float(abs(metas[f]["amps"][t]) ** 2), float(d[u]),
                          float(np.abs(circ(end[f, u], ft)).max()),
                          float(abs(amp1[f, u] / metas[f]["amps"][t] - 1)),
                          float(np.abs(circ(end[f, u], f_ml[f, t])).max())))
        if found == K and passed[f] == K:
            complete += 1
            ml_diff += [v[6] for v in tones[-K:]]
    ev = np.array([v[2:] for v in tones]) if tones else np.zeros((0, 5))

    def cls(lo, hi):
        q = (ev[:, 0] >= lo) & (ev[:, 0] < hi)
        if not q.any():
            return {"tones": 0}
        b, a = ev[q, 1], ev[q, 2]
        return {"tones": int(q.sum()),
                "err_rms_bins": [float(np.sqrt(np.mean(b ** 2))), float(np.sqrt(np.mean(a ** 2)))],
                "err_max_bins": [float(b.max()), float(a.max())],
                "tones_worse_after": int(np.sum(a > b))}

    out = {"workload": f"{F} frames of 2048x2048 complex64, K={K} off-grid tones, B=128x128, T=3",
           "start": f"per frame up to {K} of the {64 * K} strongest detected peaks: those whose per-round "
                    "amplitudes agree (spread <= 0.5), then two peeling rounds (5 refinement steps, "
                    "the residual after the tones found, the other peaks' agreement on it); the "
                    "chosen records' detector frequencies, amplitudes from rsft_initial_amplitudes",
           "select_s": select_s,
           "tones_refined": int(passed.sum()),
           "steps": steps, "ms_per_step": ms / steps, "ms_total": ms,
           "true_tones": F * K, "true_tones_started": len(tones),
           "frames_with_all_tones_started": complete,
           "by_amplitude": {"|b|^2<0.1": cls(0.0, 0.1), "0.1<=|b|^2<1": cls(0.1, 1.0),
                            "|b|^2>=1": cls(1.0, np.inf)},
           "err_rms_bins": [float(np.sqrt(np.mean(ev[:, 1] ** 2))), float(np.sqrt(np.mean(ev[:, 2] ** 2)))],
           "err_max_bins": [float(ev[:, 1].max()), float(ev[:, 2].max())],
           "amp_rel_err_median_after": float(np.median(ev[:, 3])),
           "vs_fit_from_truth_max_bins": float(max(ml_diff)) if ml_diff else None,
           "loss_sum": {"start": float(losses[0].sum()), "end": float(losses[-1].sum()),
                        "at_true_parameters": float(loss_truth.sum())},
           "frames_end_loss_at_or_below_truth": int(np.sum(losses[-1] <= loss_truth))}
    log(f"refinement: {out['ms_per_step']:.3f} ms/step, {len(tones)} tones started, "
        f"{complete} complete frames; rms {out['err_rms_bins'][0]:.4f} -> {out['err_rms_bins'][1]:.4f} bin; "
        f"strong {out['by_amplitude']['|b|^2>=1']}; vs fit from truth {out['vs_fit_from_truth_max_bins']}")
    per = cfg["rounds"] * int(np.prod(cfg["buckets"]))
    obs_np = obs.cpu().numpy()
    handoff = {"sigma": sigma, "steps": steps,
               "frames": [{"start_f": start[f], "start_a": amp0[f], "end_f": end[f], "end_a": amp1[f],
                           "active": int(passed[f]),
                           "observed": obs_np[f * per:(f + 1) * per].reshape(
                               (cfg["rounds"],) + tuple(cfg["buckets"]))}
                          for f in range(oracle_frames)]}
    plan.close()
    return out, handoff


def refine_vs_oracle(handoff):
    """The FP64 oracle's refinement of the handed-over frames from the same
    start (frequencies, amplitudes) and observed buckets as the GPU's: the
    largest difference of the refined frequencies (bins) and amplitudes."""
    from oracle import refine as oracle_refine
    from oracle import rsft as oracle_rsft
    cfg = synth.WORKLOADS["offgrid_2048x2048"]
    shape = cfg["shape"]
    oplan = oracle_rsft.OraclePlan(shape, cfg["buckets"], handoff["sigma"], 60.0, None, cfg["pfa"])
    df, da = [], []
    t0 = time.perf_counter()
    for fr in handoff["frames"]:
        k = fr["active"]
        wf, wa, _, _ = oracle_refine.refine(fr["start_f"], fr["start_a"].astype(np.complex128), oplan,
                                            fr["observed"].astype(np.complex128), handoff["steps"], active=k)
        df.append(np.abs((((fr["end_f"][:k] - wf[:k] + 0.5) % 1.0) - 0.5) * np.array(shape)).max())
        da.append(np.max(np.abs(fr["end_a"][:k] / wa[:k] - 1)))
    return {"frames": len(handoff["frames"]), "refined_freq_max_diff_bins": float(max(df)),
            "refined_amp_max_rel_diff": float(max(da)), "oracle_seconds": time.perf_counter() - t0}


# The other batched workloads, each at its full batch: (name, frames,
# max detections per frame).
OTHER_WORKLOADS = (
    ("ongrid_256x256_c128", 1024, 1 << 15),
    ("cube_256x128x32", 64, 1 << 16),
    ("uneven_128_to_2048", 512, 1 << 17),
    ("offgrid_2048x2048", 16, 1 << 17),
)


def _workload_plan(name, nframes, max_det):
    """Plan, input array and per-frame metadata for one batched workload.
    Workloads with one sigma per frame get one descriptor per frame."""
    cfg = synth.WORKLOADS[name]
    if not cfg["sigma_per_frame"]:
        frames, metas = synth.make_batch(name, nframes)
        for m in metas:
            m["buckets"] = cfg["buckets"]
        return _plan_for(name, nframes, max_det, metas), frames, metas
    metas = [synth.make_frame(name, f) for f in range(nframes)]
    for m in metas:
        m["buckets"] = cfg["buckets"] or tuple(n // 16 for n in m["shape"])
    frames = np.concatenate([m.pop("frame").ravel() for m in metas])
    return _plan_for(name, nframes, max_det, metas), frames, metas


def _plan_for(name, nframes, max_det, metas):
    """The plan of a batched workload for frames described by `metas`."""
    from paper_1610_01050_amd import Plan
    cfg = synth.WORKLOADS[name]
    dtype = "c128" if cfg["dtype"] == np.complex128 else "c64"
    if not cfg["sigma_per_frame"]:
        return Plan(cfg["shape"], cfg["buckets"], rounds=cfg["rounds"], sigma=synth.shared_sigma(name),
                    window_atten_db=cfg["atten_db"], pfa=cfg["pfa"], dtype=dtype,
                    max_batch=nframes, max_detections=max_det)
    descs = [dict(shape=m["shape"], buckets=m["buckets"], rounds=cfg["rounds"], sigma=m["sigma"],
                  window_atten_db=cfg["atten_db"], pfa=cfg["pfa"], dtype=dtype, max_detections=max_det)
             for m in metas]
    return Plan.uneven(descs)


def pipelined_ms(plans, bufs, steps, warmup):
    """Milliseconds per batch with batches alternating over two plans: the
    fold of batch k (rsft_execute_fold, one stream for all folds) beside the
    tail of batch k - 1 (rsft_execute_tail, one stream per plan), ordered by
    events; wall time over `steps` batches between two synchronizations."""
    import torch
    sF = torch.cuda.Stream()
    sT = [torch.cuda.Stream(), torch.cuda.Stream()]
    fdone = [torch.cuda.Event(), torch.cuda.Event()]
    tdone = [torch.cuda.Event(), torch.cuda.Event()]

    def run(n):
        for k in range(n):
            i = k % 2
            sF.wait_event(tdone[i])
            plans[i].execute_fold(bufs[k % len(bufs)], stream=sF)
            fdone[i].record(sF)
            sT[i].wait_event(fdone[i])
            plans[i].execute_tail(stream=sT[i])
            tdone[i].record(sT[i])

    run(max(warmup, 2))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def workloads_section(dev, steps, warmup, names=None):
    """Every other batched workload at its full batch, in the launch
    configuration of the headline measurement: autotuned fold, graph replay
    over two alternating input buffers (throughput), then eager launches
    with events around each stage (fold bandwidth)."""
    import torch
    from paper_1610_01050_amd import OPT_GRAPH, OPT_TIMING
    out = {}
    for name, nframes, max_det in OTHER_WORKLOADS:
        if names is not None and name not in names:
            continue
        cfg = synth.WORKLOADS[name]
        log(f"workload {name}: generating {nframes} frames ...")
        plan, frames_np, metas = _workload_plan(name, nframes, max_det)
        esize = np.dtype(cfg["dtype"]).itemsize
        T = cfg["rounds"]
        in_bytes = sum(int(np.prod(m["shape"])) for m in metas) * esize
        part_bytes = sum(T * int(np.prod(m["buckets"])) * 8 for m in metas)
        xa = torch.from_numpy(frames_np).to(dev)
        del frames_np
        xb = torch.neg(xa)
        bufs = [xa, xb]
        plan.autotune(xa, repeats=3)
        plan.set_option(OPT_TIMING, 0)
        plan.set_option(OPT_GRAPH, 1)
        for w in range(warmup):
            plan.execute(bufs[w % 2])
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record()
        for k in range(steps):
            plan.execute(bufs[k % 2])
            ev[k + 1].record()
        torch.cuda.synchronize()
        replay = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
        plan.set_option(OPT_GRAPH, 0)
        plan.set_option(OPT_TIMING, 1)
        for w in range(warmup):
            plan.execute(bufs[w % 2])
        torch.cuda.synchronize()
        plan.stage_times(reset=True)
        for k in range(steps):
            plan.execute(bufs[k % 2])
        torch.cuda.synchronize()
        stages, _ = plan.stage_times(reset=True)
        plan.set_option(OPT_TIMING, 0)
        # the same batches pipelined over two plans (fold beside the previous tail)
        plan2 = _plan_for(name, nframes, max_det, metas)
        plan2.autotune(xa, repeats=3)
        pipe_ms = pipelined_ms([plan, plan2], bufs, max(steps, 20), warmup)
        plan2.close()
        plan.execute(xa)
        recs, counts = plan.detect()
        hits = tgt = fa = outside = 0
        starts = np.searchsorted(recs["frame"], np.arange(nframes + 1))
        for f, m in enumerate(metas):
            sel = recs[starts[f]:starts[f + 1]]
            D = len(m["shape"])
            cells = np.ravel_multi_index(tuple(sel["idx"][:, d].astype(np.int64) for d in range(D)),
                                         m["shape"]) if len(sel) else []
            h, k, a, o = scoring.pd_pfa(cells, m["freqs"], m["shape"])
            hits, tgt, fa, outside = hits + h, tgt + k, fa + a, outside + o
        # records per compaction chunk (2^15 cells), the estimate's unit of work
        D = len(metas[0]["shape"])
        shapes = np.array([m["shape"] for m in metas], dtype=np.int64)
        strides = np.cumprod(shapes[:, ::-1], axis=1)[:, ::-1]
        strides = np.concatenate([strides[:, 1:], np.ones((nframes, 1), np.int64)], axis=1)
        fr = recs["frame"].astype(np.int64)
        flat = (recs["idx"][:, :D].astype(np.int64) * strides[fr]).sum(axis=1)
        _, per_chunk = np.unique(fr * (1 << 40) + (flat >> 15), return_counts=True)
        med = float(np.median(replay))
        fold_gbs = (in_bytes + part_bytes) / (stages["fold"] * 1e-3) / 1e9
        out[name] = {
            "frames": nframes, "input_bytes": in_bytes,
            "fold_launch": plan.info()["fold"],
            "estimate_workers": plan.info()["estimate_workers"],
            "vote_kernel": plan.info()["vote_kernel"],
            "graph_replay_ms": {"p10": float(np.percentile(replay, 10)), "median": med,
                                "p90": float(np.percentile(replay, 90))},
            "frames_per_s": nframes / (med * 1e-3),
            "pipelined_two_plans": {"ms_per_batch": pipe_ms, "frames_per_s": nframes / (pipe_ms * 1e-3)},
            "input_gbs": in_bytes / (med * 1e-3) / 1e9,
            "stage_ms": stages,
            "fold_algorithmic_bytes": in_bytes + part_bytes,
            "fold_gbs": fold_gbs, "fold_frac_of_peak": fold_gbs / HBM_PEAK_GBS,
            "detections": int(counts.sum()),
            "records_per_chunk": {"chunks": int(per_chunk.size), "max": int(per_chunk.max(initial=0)),
                                  "mean": float(per_chunk.mean()) if per_chunk.size else 0.0,
                                  "over_2048": int((per_chunk > 2048).sum())},
            "pd": hits / max(tgt, 1), "pfa": fa / max(outside, 1),
        }
        log(f"  {med:.3f} ms per batch ({nframes / (med * 1e-3):.0f} frames/s), fold "
            f"{stages['fold']:.3f} ms = {fold_gbs:.0f} GB/s, stages {stages}")
        plan.close()
        del xa, xb, bufs
        torch.cuda.empty_cache()
    return out


def radar_section(dev, cpis=8, reps=10):
    """3-D RSFT on SRUR cubes (Table III: 32 RIs x 64 elements x 2048 range
    samples; Table IV targets, different-SNR setting), T = 4 bursts per CPI in
    segment mode, B = 8x16x128, mu = 3, Pfa = 1e-6; against the dense
    windowed 3-D FFT with the Bartlett sum over the bursts and the exact
    Gamma(T) threshold, both on this GPU, with target recovery."""
    import torch
    from scipy import stats
    from synth import radar
    from paper_1610_01050_amd import Plan, chebyshev_window
    shape = radar.cube_shape()
    T, mu, pfa = 4, 3, 1e-6
    log(f"radar: generating {cpis} CPIs of {T} bursts {shape} ...")
    data = [radar.make_cpi(c, T, "different") for c in range(cpis)]
    x = torch.from_numpy(np.stack([d[0] for d in data])).to(dev)
    sigma = synth.draw_sigma(np.random.default_rng(radar.RADAR_SEED), T, shape)
    plan = Plan(shape, (8, 16, 128), rounds=T, sigma=sigma, mu=mu, pfa=pfa, segments=True,
                max_batch=cpis, max_detections=1 << 16)
    plan.execute(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.execute(x)
    e1.record()
    torch.cuda.synchronize()
    rsft_ms = e0.elapsed_time(e1) / reps
    recs, counts = plan.detect()

    def recovered(cells_of_cpi):
        found = 0
        for c, (_, freqs, _) in enumerate(data):
            idx = cells_of_cpi(c)
            for f in freqs:
                cell = np.round(f * np.array(shape)) % np.array(shape)
                if len(idx):
                    d = np.abs(idx - cell)
                    d = np.minimum(d, np.array(shape) - d).max(axis=1)
                    found += int(d.min() <= 3)
        return found / (cpis * len(data[0][1]))

    rsft_rec = recovered(lambda c: recs[(recs["frame"] == c) & (recs["is_peak"] == 1)]["idx"][:, :3])
    # dense comparator: windowed 3-D FFT per burst, |X|^2 summed over bursts
    w = [torch.tensor(chebyshev_window(n, 60.0), dtype=torch.float32, device=dev) for n in shape]
    wnd = w[0][:, None, None] * w[1][None, :, None] * w[2][None, None, :]
    energy = float((wnd.double() ** 2).sum())
    thr = float(stats.gamma.isf(pfa, T, scale=energy))

    def dense():
        acc = None
        for s in range(T):
            X = torch.fft.fftn(x[:, s] * wnd, dim=(1, 2, 3))
            p = X.real ** 2 + X.imag ** 2
            acc = p if acc is None else acc + p
        return acc >= thr

    det = dense()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        det = dense()
    e1.record()
    torch.cuda.synchronize()
    dense_ms = e0.elapsed_time(e1) / reps
    nz = torch.nonzero(det).cpu().numpy()
    dense_rec = recovered(lambda c: nz[nz[:, 0] == c][:, 1:].astype(np.float64))
    in_bytes = x.numel() * 8
    plan.close()
    out = {"workload": f"{cpis} CPIs x {T} bursts of 32x64x2048 complex64 (SRUR, Table III/IV targets, "
                       "different SNRs), B=8x16x128, mu=3, Pfa=1e-6, segment mode",
           "rsft_ms_per_batch": rsft_ms, "rsft_cpis_per_s": cpis / rsft_ms * 1e3,
           "rsft_input_gbs": in_bytes / (rsft_ms * 1e-3) / 1e9,
           "dense_fft_ms_per_batch": dense_ms, "speedup_over_dense_fft": dense_ms / rsft_ms,
           "targets_recovered": {"rsft": rsft_rec, "dense_fft": dense_rec},
           "detections_per_cpi": float(np.mean(counts)),
           "dense_detections_per_cpi": len(nz) / cpis}
    log(f"radar: RSFT {rsft_ms:.3f} ms, dense 3-D FFT {dense_ms:.3f} ms per batch; recovered "
        f"{rsft_rec:.2f} / {dense_rec:.2f}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=40)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-comparators", action="store_true")
    ap.add_argument("--skip-refine", action="store_true")
    ap.add_argument("--skip-radar", action="store_true")
    ap.add_argument("--workloads", nargs="?", const="all", default="all",
                    help="the other batched workloads to measure as well: all (default) or a "
                         "comma-separated list of names (about a minute in all)")
    ap.add_argument("--skip-workloads", action="store_true")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the fold HBM-traffic summary from two rocprofv3 --pmc "
                         "CSV output folders (FETCH_SIZE, WRITE_SIZE) and exit; no GPU")
    ap.add_argument("--counter-commands", nargs=2, default=["", ""],
                    help="the two rocprofv3 commands, recorded in the summary")
    ap.add_argument("--skip-headline", action="store_true",
                    help="skip the headline workload (with --workloads NAME: profile one workload)")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("DIR", "TITLE", "COMMAND"),
                    help="print a markdown summary of a rocprofv3 --kernel-trace --stats run and "
                         "exit; no GPU")
    ap.add_argument("--summarize-pmc", nargs="+", metavar="ARG",
                    help="TITLE KERNELS(comma-separated) DIR COMMAND [DIR COMMAND ...]: print a "
                         "markdown summary of rocprofv3 --pmc runs and exit; no GPU")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, *args.counter_commands)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_pmc:
        a = args.summarize_pmc
        summarize_pmc(a[2::2], a[0], a[3::2], [k for k in a[1].split(",") if k])
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(frames would shard across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1610_01050_amd import OPT_GRAPH, OPT_TIMING, Plan, load_library
    load_library()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.skip_headline:
        # profiling runs: the named other workloads alone
        names = None if args.workloads == "all" else args.workloads.split(",")
        print(json.dumps({"workloads": workloads_section(dev, min(args.steps, 20), args.warmup, names)}),
              flush=True)
        return
    cfg = synth.WORKLOADS[WORKLOAD]
    shape, buckets, T, pfa = cfg["shape"], cfg["buckets"], cfg["rounds"], cfg["pfa"]
    N = int(np.prod(shape))
    B = int(np.prod(buckets))

    log(f"generating {FRAMES} frames {shape} ...")
    t0 = time.perf_counter()
    frames_np, metas = synth.make_batch(WORKLOAD, FRAMES)
    log(f"  done in {time.perf_counter() - t0:.1f} s")
    xa = torch.from_numpy(frames_np).to(dev)
    xb = torch.neg(xa)   # second buffer: same statistics, other bytes; this kernel reads
                         # and writes exactly 1 GiB and calibrates the HBM counters
    bufs = [xa, xb]
    # measured copy bandwidth: the same elementwise negation, 1 GiB read + 1 GiB written
    copy_ms = []
    for _ in range(6):
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        torch.neg(xa, out=xb)
        c1.record()
        torch.cuda.synchronize()
        copy_ms.append(c0.elapsed_time(c1))
    copy_gbs = 2 * xa.numel() * 8 / (float(np.median(copy_ms[1:])) * 1e-3) / 1e9
    log(f"copy (negation, 2 GiB moved): {copy_gbs:.0f} GB/s")
    # measured read bandwidth: torch's sum over rows of 1024 floats of the same
    # 1 GiB (reads it all, writes 1 MiB), the read-only reference of the fold
    rows = torch.view_as_real(xa).view(-1, 1024)
    rsum = torch.empty(rows.shape[0], device=dev)
    read_ms = []
    for _ in range(6):
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        torch.sum(rows, dim=1, out=rsum)
        c1.record()
        torch.cuda.synchronize()
        read_ms.append(c0.elapsed_time(c1))
    del rows, rsum
    read_gbs = xa.numel() * 8 / (float(np.median(read_ms[1:])) * 1e-3) / 1e9
    log(f"read (row sums of the 1 GiB input): {read_gbs:.0f} GB/s")
    sigma = synth.shared_sigma(WORKLOAD)
    plan = Plan(shape, buckets, rounds=T, sigma=sigma, window_atten_db=cfg["atten_db"],
                pfa=pfa, dtype="c64", max_batch=FRAMES, max_detections=1 << 16)
    torch.cuda.synchronize()
    tuned_ms = plan.autotune(xa, repeats=5)          # fold launch shape, untimed
    fold_cfg = plan.info()["fold"]
    log(f"autotuned fold: {fold_cfg} ({tuned_ms:.4f} ms), estimate workers "
        f"{plan.info()['estimate_workers']}")

    # graph replay (production launch mode)
    plan.set_option(OPT_TIMING, 0)
    plan.set_option(OPT_GRAPH, 1)
    for w in range(args.warmup):
        plan.execute(bufs[w % 2])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        plan.execute(bufs[k % 2])
    torch.cuda.synchronize()
    graph_s = time.perf_counter() - t0
    # per-replay durations from events around each replay, on the launch stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record()
    for k in range(args.steps):
        plan.execute(bufs[k % 2])
        ev[k + 1].record()
    torch.cuda.synchronize()
    replay_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    graph_pct = {"p10": float(np.percentile(replay_ms, 10)), "median": float(np.median(replay_ms)),
                 "p90": float(np.percentile(replay_ms, 90))}
    log(f"graph mode: {graph_s / args.steps * 1e3:.3f} ms/step, per replay {graph_pct}")

    # timed region: eager launches with HIP events around every stage on the
    # stream the kernels run on
    plan.set_option(OPT_TIMING, 1)
    for w in range(args.warmup):
        plan.execute(bufs[w % 2])
    torch.cuda.synchronize()
    plan.stage_times(reset=True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        plan.execute(bufs[k % 2])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages, nstaged = plan.stage_times(reset=True)
    plan.set_option(OPT_TIMING, 0)
    ms_per_step = elapsed / args.steps * 1e3
    value = FRAMES * args.steps / elapsed
    log(f"eager+events: {ms_per_step:.3f} ms/step, stages {stages}")

    # detections of buffer A
    plan.execute(xa)
    recs, counts = plan.detect()
    fused_score = score(recs, counts, metas, shape, range(FRAMES))
    log(f"fused: {int(counts.sum())} detections, {fused_score}")

    fold_ms = stages["fold"]
    fold_bytes = FRAMES * (N * 8 + T * B * 8)        # input once + T x B partial buckets
    achieved = fold_bytes / (fold_ms * 1e-3) / 1e9
    traffic = measured_traffic(T, fold_cfg)
    out = {
        "metric": METRIC, "value": value, "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "128 frames of 1024x1024 complex64, K=20 off-grid tones, "
                               "SNR U[-10,10] dB Rayleigh, B=64x64, T=3, Pfa=1e-4, 60 dB "
                               "Dolph-Chebyshev, shared sigma",
                   "frames": FRAMES, "shape": list(shape), "buckets": list(buckets),
                   "rounds": T, "pfa": pfa},
        "hbm_gbs": FRAMES * N * 8 * args.steps / elapsed / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": "fold",
                     "measured_copy_gbs": copy_gbs, "frac_of_measured_copy": achieved / copy_gbs,
                     "measured_read_gbs": read_gbs, "frac_of_measured_read": achieved / read_gbs,
                     "algorithmic_bytes_per_launch": fold_bytes,
                     "avg_launch_ms": fold_ms},
        "stage_ms": stages,
        "fold_launch": fold_cfg,
        "estimate_workers": plan.info()["estimate_workers"],
        "vote_kernel": plan.info()["vote_kernel"],
        "graph_ms_per_step": graph_s / args.steps * 1e3,
        "graph_replay_ms": graph_pct,
        "detections": {"total": int(counts.sum()), **fused_score},
    }

    if not args.skip_comparators:
        # per-frame plain RSFT: literal Algorithm 1, one launch chain per frame
        plan.execute_per_frame(xa)
        torch.cuda.synchronize()
        reps = 2
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.execute_per_frame(xa)
        torch.cuda.synchronize()
        pf_s = (time.perf_counter() - t0) / reps
        precs, pcounts = plan.detect()
        pf_score = score(precs, pcounts, metas, shape, range(FRAMES))
        same = int(np.array_equal(precs[["frame", "idx"]], recs[["frame", "idx"]]))
        out["per_frame_rsft"] = {"frames_per_s": FRAMES / pf_s, "ms_per_batch": pf_s * 1e3,
                                 "speedup_of_fused": value / (FRAMES / pf_s),
                                 "same_detections": bool(same), **pf_score}
        log(f"per-frame: {pf_s * 1e3:.2f} ms/batch, {pf_score}")

        # dense windowed 2-D FFT (rocFFT through torch) + exact T=1 NP threshold
        from paper_1610_01050_amd import chebyshev_window
        w0 = torch.tensor(chebyshev_window(shape[0], cfg["atten_db"]), dtype=torch.float32, device=dev)
        w1 = torch.tensor(chebyshev_window(shape[1], cfg["atten_db"]), dtype=torch.float32, device=dev)
        wnd = torch.outer(w0, w1)
        thr = float((wnd.double() ** 2).sum().item() * math.log(1.0 / pfa))

        def dense(x):
            X = torch.fft.fft2(x * wnd)
            return (X.real ** 2 + X.imag ** 2) >= thr

        def timed(fn, reps=5):
            fn()
            torch.cuda.synchronize()
            d0, d1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            d0.record()
            for _ in range(reps):
                r = fn()
            d1.record()
            torch.cuda.synchronize()
            return d0.elapsed_time(d1) / reps * 1e-3, r

        dn_s, det = timed(lambda: dense(xa))
        fft_s, _ = timed(lambda: torch.fft.fft2(xa))
        nz = torch.nonzero(det.view(FRAMES, -1)).cpu().numpy()
        hits = tgt = fa = outside = 0
        for f in range(FRAMES):
            cells = nz[nz[:, 0] == f, 1]
            h, k, a, o = scoring.pd_pfa(cells, metas[f]["freqs"], shape)
            hits += h
            tgt += k
            fa += a
            outside += o
        out["dense_fft"] = {"frames_per_s": FRAMES / dn_s, "ms_per_batch": dn_s * 1e3,
                            "what": "window multiply, rocFFT 2-D FFT (torch.fft.fft2), |X|^2 >= "
                                    "threshold as a mask; the cell list is taken after timing",
                            "fft_only_ms_per_batch": fft_s * 1e3,
                            "speedup_of_fused": value / (FRAMES / dn_s),
                            "speedup_of_fused_vs_fft_only": value / (FRAMES / fft_s),
                            "pd": hits / max(tgt, 1), "pfa": fa / max(outside, 1)}
        log(f"dense: {dn_s * 1e3:.2f} ms/batch")
        out["paper_complexity_model"] = paper_complexity(shape, buckets, T, cfg["K"],
                                                         out["dense_fft"]["speedup_of_fused"])

    refine_handoff = None
    if not args.skip_refine:
        out["refine"], refine_handoff = refine_section(dev)
    if not args.skip_radar:
        out["radar"] = radar_section(dev)
    if args.workloads and not args.skip_workloads:
        names = None if args.workloads == "all" else args.workloads.split(",")
        out["workloads"] = workloads_section(dev, min(args.steps, 20), args.warmup, names)

    if not args.skip_cpu and args.cpu_sample > 0:
        n = min(args.cpu_sample, FRAMES)
        log(f"cpu baseline: oracle on {n} frames ...")
        cb, odets, oouts = cpu_baseline(frames_np, metas, shape, buckets, sigma, pfa, n)
        gb = [b.cpu().numpy() for b in plan.buckets()[:n]]
        gw = [w.cpu().numpy().view(np.uint32) for w in plan.flags()[:n]]
        out["precision"] = precision_report(gb, gw, recs, oouts, shape, buckets)
        log(f"precision: {out['precision']}")
        if refine_handoff is not None:
            out["refine"]["vs_fp64_oracle"] = refine_vs_oracle(refine_handoff)
            log(f"refinement vs FP64 oracle: {out['refine']['vs_fp64_oracle']}")
        gpu_sample = score(recs, counts, metas, shape, range(n))
        cb["gpu_pd_same_frames"] = gpu_sample["pd"]
        cb["gpu_pfa_same_frames"] = gpu_sample["pfa"]
        agree = 0
        total = 0
        D = len(shape)
        for f in range(n):
            sel = recs[recs["frame"] == f]
            g = set(int(np.ravel_multi_index(tuple(int(v) for v in r["idx"][:D]), shape)) for r in sel)
            o = set(int(v) for v in odets[f])
            agree += len(g & o)
            total += len(g | o)
        cb["detection_jaccard_vs_gpu"] = agree / max(total, 1)
        cb["host"] = host_cpu()
        workers = max(1, min(16, cb["host"]["cpus_allowed"]))
        cb["dense_leg"] = dense_cpu_leg(frames_np, shape, cfg["atten_db"], pfa, n, workers)
        log(f"cpu dense leg: {cb['dense_leg']}")
        out["cpu_baseline"] = cb
        log(f"cpu: {cb['value']:.2f} frames/s")

    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
