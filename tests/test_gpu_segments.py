"""GPU parity of segment mode (a frame is T data segments and round s
processes segment s with sigma_s; votes accumulate over the segments) and of
a given first-stage false-alarm probability, against the FP64 oracle; plus
the exact binomial false-alarm rate of independent noise segments measured
on the GPU path."""

import math
import zlib

import numpy as np
import pytest

import synth
from oracle import rsft as OR

from helpers import check_frame

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _segments(shape, T, K, seed):
    """T segments of the same K tones with Rayleigh amplitudes redrawn per
    segment (Swerling-I across segments) in independent noise."""
    rng = np.random.default_rng(seed)
    freqs, _ = synth.draw_frequencies(rng, shape, K, False, 2.05)
    segs = []
    for s in range(T):
        amps = synth.complex_noise(rng, (K,), 1.0) * np.sqrt(10.0 ** (rng.uniform(5, 15, K) / 10))
        segs.append(synth.synthesize(shape, freqs, None, amps) + synth.complex_noise(rng, shape))
    return np.stack(segs).astype(np.complex64), freqs


CASES = {
    # name: (shape, buckets, T, mu, stage1_pfa, batch)
    "two_dim_T5_mu3": ((256, 256), (16, 16), 5, 3, 0.0, 2),
    "one_dim_T40_mu12_given_p1": ((4096,), (64,), 40, 12, 0.2, 2),
    "three_dim_T3": ((64, 32, 16), (8, 4, 4), 3, 0, 0.0, 2),
    "one_dim_T64_mu20_given_p1": ((2048,), (32,), 64, 20, 0.2, 1),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("per_frame", [False, True])
def test_segment_mode_matches_oracle(name, per_frame):
    from paper_1610_01050_amd import Plan
    shape, buckets, T, mu, p1, batch = CASES[name]
    print(f"case {name} per_frame={per_frame}", flush=True)
    seed = zlib.crc32(name.encode()) % 100000
    frames = [_segments(shape, T, 3, seed + f)[0] for f in range(batch)]
    sigma = synth.draw_sigma(np.random.default_rng(seed), T, shape)
    plan = Plan(shape, buckets, rounds=T, sigma=sigma, pfa=1e-3, mu=mu, max_batch=batch,
                segments=True, stage1_pfa=p1, max_detections=1 << 16)
    xd = torch.from_numpy(np.stack(frames)).to("cuda")
    if per_frame:
        plan.execute_per_frame(xd)
    else:
        plan.execute(xd)
    recs, counts = plan.detect()
    gbk = [b.cpu().numpy() for b in plan.buckets()]
    gfl = [w.cpu().numpy().view(np.uint32) for w in plan.flags()]
    oplan = OR.OraclePlan(shape, buckets, sigma, 60.0, None, 1e-3, None if mu == 0 else mu, 1.0,
                          p1 if p1 > 0 else None)
    for f in range(batch):
        ref = OR.rsft(frames[f], oplan, segments=True)
        check_frame(f, oplan, ref, recs, gbk[f], gfl[f])
    plan.close()


def test_uneven_segment_plan_matches_oracle():
    from paper_1610_01050_amd import Plan
    shapes = [(128, 256), (512, 128), (256, 256)]
    T = 4
    descs, frames, sigmas = [], [], []
    for i, sh in enumerate(shapes):
        sg = synth.draw_sigma(np.random.default_rng(700 + i), T, sh)
        descs.append(dict(shape=sh, buckets=tuple(n // 16 for n in sh), rounds=T, mu=3,
                          sigma=sg, pfa=1e-3, segments=True, max_detections=1 << 16))
        frames.append(_segments(sh, T, 4, 800 + i)[0])
        sigmas.append(sg)
    plan = Plan.uneven(descs)
    plan.execute(torch.from_numpy(np.concatenate([x.ravel() for x in frames])).to("cuda"))
    recs, counts = plan.detect()
    gbk = [b.cpu().numpy() for b in plan.buckets()]
    gfl = [w.cpu().numpy().view(np.uint32) for w in plan.flags()]
    for f, sh in enumerate(shapes):
        oplan = OR.OraclePlan(sh, tuple(n // 16 for n in sh), sigmas[f], 60.0, None, 1e-3, 3)
        check_frame(f, oplan, OR.rsft(frames[f], oplan, segments=True), recs, gbk[f], gfl[f])
    plan.close()


@pytest.mark.timeout(300)
def test_independent_noise_segments_final_pfa_on_gpu():
    """T = mu = 3, Pfa = 1e-3: independent noise segments make the rounds'
    flags independent Bernoulli(p1), so the rate of detected cells is exactly
    1e-3; 2048 frames of 256 x 256 (134 M cells), within 3 standard errors
    computed over frames."""
    from paper_1610_01050_amd import Plan
    shape, buckets, T = (256, 256), (16, 16), 3
    sigma = synth.draw_sigma(np.random.default_rng(99), T, shape)
    batch = 256
    plan = Plan(shape, buckets, rounds=T, sigma=sigma, pfa=1e-3, max_batch=batch,
                segments=True, max_detections=1 << 12)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1610)
    rates = []
    N = shape[0] * shape[1]
    for rep in range(8):
        x = torch.randn((batch, T) + shape, dtype=torch.complex64, device="cuda", generator=gen)
        plan.execute(x)
        rates.append(plan.detect()[1] / N)
    rates = np.concatenate(rates)
    se = rates.std(ddof=1) / math.sqrt(len(rates))
    print(f"false-alarm rate {rates.mean():.4e} +- {se:.1e}")
    assert abs(rates.mean() - 1e-3) < 3 * se
    plan.close()
