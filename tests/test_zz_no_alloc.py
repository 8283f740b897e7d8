"""The no-allocation model entry point (rsft_model_forward_noalloc) against
rsft_model_forward, which takes a caller workspace: same kernels, so the
model buckets must agree to the bucket tolerance of the parity tests (they
are expected bit for bit). Two calls in a row on one plan, the second with a
smaller input (fewer frames and tones), so the second reuses the static
array the first filled; then a request beyond the array's size is refused
with a clear error and no launch."""

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _inputs(rng, batch, K, shape):
    freqs = np.stack([synth.draw_frequencies(rng, shape, K, False, 2.05)[0] for _ in range(batch)])
    amps = (rng.standard_normal((batch, K)) + 1j * rng.standard_normal((batch, K))) * 2.0
    return (torch.tensor(freqs, dtype=torch.float64, device="cuda").contiguous(),
            torch.tensor(amps.astype(np.complex64), device="cuda").contiguous())


def _compare(plan, f_d, a_d):
    batch, K = int(f_d.shape[0]), int(f_d.shape[1])
    ws = plan.model_workspace(batch, K)
    want = plan.model_forward(f_d, a_d, ws)
    got = torch.full_like(want, complex(float("nan"), float("nan")))
    plan.model_forward_noalloc(f_d, a_d, got)
    torch.cuda.synchronize()
    w = want.cpu().numpy()
    g = got.cpu().numpy()
    T = plan.rounds
    B = int(np.prod(plan.descs[0]["buckets"]))
    for f in range(batch):
        for s in range(T):
            ref = w[(f * T + s) * B:(f * T + s + 1) * B]
            out = g[(f * T + s) * B:(f * T + s + 1) * B]
            rms = np.sqrt(np.mean(np.abs(ref) ** 2))
            assert np.all(np.isfinite(out))
            assert np.max(np.abs(out - ref)) <= 1e-4 * rms
    return int(np.sum(g != w))


def test_noalloc_model_matches_workspace_model_twice():
    from paper_1610_01050_amd import Plan
    from paper_1610_01050_amd.binding import RsftError
    shape, buckets = (2048, 2048), (128, 128)
    rng = np.random.default_rng(20)
    sigma = synth.draw_sigma(rng, 3, shape)
    plan = Plan(shape, buckets, rounds=3, sigma=sigma, pfa=1e-4, max_batch=16)
    print("no-alloc model: 16 frames x 32 tones, then 5 frames x 7 tones", flush=True)
    f1, a1 = _inputs(rng, 16, 32, shape)       # 6.3 MB of factors: most of the array
    diff1 = _compare(plan, f1, a1)
    f2, a2 = _inputs(rng, 5, 7, shape)         # smaller: the array keeps the first call's tail
    diff2 = _compare(plan, f2, a2)
    print(f"elements differing: {diff1}, {diff2}", flush=True)
    # 16 frames x 64 tones need 12.6 MB of factors: refused before any launch
    f3, a3 = _inputs(rng, 16, 64, shape)
    out = torch.empty(plan.model_size(16), dtype=torch.complex64, device="cuda")
    with pytest.raises(RsftError, match="static scratch"):
        plan.model_forward_noalloc(f3, a3, out)
    plan.close()
