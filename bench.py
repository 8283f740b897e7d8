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
        t0 = time.perf_counter()
        for f in range(nsample):
            out = oracle_rsft.rsft(frames_np[f], plan)
            oracle_rsft.estimate(out["detections"], out["buckets"], plan)
            dets.append(out["detections"])
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
            "pd": hits / max(tgt, 1), "pfa": fa / max(outside, 1)}, dets


def refine_section(dev, steps=20):
    """Gauss-Newton refinement through the bucketized forward model on 16
    frames of 2048x2048 (K = 32 off-grid tones, B = 128x128): observed buckets
    from the fused RSFT of the frames, start = truth perturbed by N(0, 0.1 bin)
    in frequency and 10% in amplitude; `steps` steps timed with events."""
    import torch
    from paper_1610_01050_amd import Plan
    from paper_1610_01050_amd.refine import refine
    cfg = synth.WORKLOADS["offgrid_2048x2048"]
    F, K = 16, cfg["K"]
    shape = cfg["shape"]
    log(f"refinement: generating {F} frames {shape} ...")
    frames, metas = synth.make_batch("offgrid_2048x2048", F)
    plan = Plan(shape, cfg["buckets"], rounds=cfg["rounds"], sigma=synth.shared_sigma("offgrid_2048x2048"),
                pfa=cfg["pfa"], max_batch=F)
    x = torch.from_numpy(frames).to(dev)
    plan.execute(x)
    obs = torch.cat([b.reshape(-1) for b in plan.buckets()]).contiguous()
    truth_f = np.stack([m["freqs"] for m in metas])
    truth_a = np.stack([m["amps"] for m in metas])
    rng = np.random.default_rng(1610)
    start_f = truth_f + rng.normal(0.0, 0.1, truth_f.shape) / np.array(shape)
    start_a = truth_a * (1 + 0.1 * (rng.standard_normal(truth_a.shape)
                                    + 1j * rng.standard_normal(truth_a.shape)) / np.sqrt(2))
    f0 = torch.tensor(start_f, dtype=torch.float64, device=dev)
    a0 = torch.tensor(start_a.astype(np.complex64), device=dev)
    refine(plan, obs, f0, a0, steps=2, record_loss=False)          # warm-up
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    fr, ar, _ = refine(plan, obs, f0, a0, steps=steps, record_loss=False)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    _, _, losses = refine(plan, obs, f0, a0, steps=steps, record_loss=True)
    losses = losses.cpu().numpy()

    def err(f):
        e = (((f - truth_f + 0.5) % 1.0) - 0.5) * np.array(shape)
        return float(np.sqrt(np.mean(e ** 2))), float(np.max(np.abs(e)))

    # loss of the true parameters: a fit at or below it is noise-limited
    ws = plan.model_workspace(F, K)
    tm = plan.model_forward(torch.tensor(truth_f, dtype=torch.float64, device=dev),
                            torch.tensor(truth_a.astype(np.complex64), device=dev), ws)
    r = tm - obs
    truth_loss = float((r.real.double() ** 2 + r.imag.double() ** 2).sum())
    before, after = err(start_f), err(fr.cpu().numpy())
    amp_err = float(np.median(np.abs(ar.cpu().numpy() / truth_a - 1)))
    plan.close()
    out = {"workload": f"{F} frames of 2048x2048 complex64, K={K} off-grid tones, B=128x128, T=3",
           "start": "truth + N(0, 0.1 bin) frequency, 10% amplitude error",
           "steps": steps, "ms_per_step": ms / steps, "ms_total": ms,
           "freq_err_rms_bins": [before[0], after[0]], "freq_err_max_bins": [before[1], after[1]],
           "amp_rel_err_median_after": amp_err,
           "loss_first_last": [float(losses[0]), float(losses[-1])],
           "loss_at_truth": truth_loss}
    log(f"refinement: {out['ms_per_step']:.3f} ms/step, freq rms {before[0]:.4f} -> {after[0]:.4f} bin")
    return out


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
    from paper_1610_01050_amd import Plan
    cfg = synth.WORKLOADS[name]
    dtype = "c128" if cfg["dtype"] == np.complex128 else "c64"
    if not cfg["sigma_per_frame"]:
        frames, metas = synth.make_batch(name, nframes)
        for m in metas:
            m["buckets"] = cfg["buckets"]
        plan = Plan(cfg["shape"], cfg["buckets"], rounds=cfg["rounds"], sigma=synth.shared_sigma(name),
                    window_atten_db=cfg["atten_db"], pfa=cfg["pfa"], dtype=dtype,
                    max_batch=nframes, max_detections=max_det)
        return plan, frames, metas
    metas = [synth.make_frame(name, f) for f in range(nframes)]
    descs = []
    for m in metas:
        m["buckets"] = cfg["buckets"] or tuple(n // 16 for n in m["shape"])
        descs.append(dict(shape=m["shape"], buckets=m["buckets"], rounds=cfg["rounds"], sigma=m["sigma"],
                          window_atten_db=cfg["atten_db"], pfa=cfg["pfa"], dtype=dtype,
                          max_detections=max_det))
    frames = np.concatenate([m.pop("frame").ravel() for m in metas])
    return Plan.uneven(descs), frames, metas


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
            "graph_replay_ms": {"p10": float(np.percentile(replay, 10)), "median": med,
                                "p90": float(np.percentile(replay, 90))},
            "frames_per_s": nframes / (med * 1e-3),
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
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, *args.counter_commands)
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
                     "algorithmic_bytes_per_launch": fold_bytes,
                     "avg_launch_ms": fold_ms},
        "stage_ms": stages,
        "fold_launch": fold_cfg,
        "estimate_workers": plan.info()["estimate_workers"],
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

        det = dense(xa)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            det = dense(xa)
            nz = torch.nonzero(det.view(FRAMES, -1))
        torch.cuda.synchronize()
        dn_s = (time.perf_counter() - t0) / 3
        nz = nz.cpu().numpy()
        hits = tgt = fa = outside = 0
        for f in range(FRAMES):
            cells = nz[nz[:, 0] == f, 1]
            h, k, a, o = scoring.pd_pfa(cells, metas[f]["freqs"], shape)
            hits += h
            tgt += k
            fa += a
            outside += o
        out["dense_fft"] = {"frames_per_s": FRAMES / dn_s, "ms_per_batch": dn_s * 1e3,
                            "speedup_of_fused": value / (FRAMES / dn_s),
                            "pd": hits / max(tgt, 1), "pfa": fa / max(outside, 1)}
        log(f"dense: {dn_s * 1e3:.2f} ms/batch")

    if not args.skip_refine:
        out["refine"] = refine_section(dev)
    if not args.skip_radar:
        out["radar"] = radar_section(dev)
    if args.workloads and not args.skip_workloads:
        names = None if args.workloads == "all" else args.workloads.split(",")
        out["workloads"] = workloads_section(dev, min(args.steps, 20), args.warmup, names)

    if not args.skip_cpu and args.cpu_sample > 0:
        n = min(args.cpu_sample, FRAMES)
        log(f"cpu baseline: oracle on {n} frames ...")
        cb, odets = cpu_baseline(frames_np, metas, shape, buckets, sigma, pfa, n)
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
        out["cpu_baseline"] = cb
        log(f"cpu: {cb['value']:.2f} frames/s")

    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
