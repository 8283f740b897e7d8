"""Off-grid refinement of detected tones through the bucketized forward model.

The round-s buckets of a frame (eq. f) are linear in the signal, so a set of
K complex tones with continuous frequencies f_t (cycles/sample) and
amplitudes b_t predicts them as

    model_s[k] = sum_t b_t prod_d G_{s,d}(f_{t,d})[k_d]

(the per-dimension factors of the window, permutation, flat window, aliasing
and B-point DFT of the plan). ``BucketModel`` exposes this model and its
hand-written backward (HIP kernels behind rsft_model_forward /
rsft_model_backward) as a torch.autograd.Function, with gradients with
respect to the frequencies (float64) and the complex amplitudes (complex64).
``refine`` fits frequencies and amplitudes to observed buckets by per-tone
trust-region Gauss-Newton steps with step acceptance and a per-frame loss
check (rsft_refine), ``initial_amplitudes`` gives detected tones their
starting amplitudes (rsft_initial_amplitudes), and ``select_tones`` chooses
which detections to refine, peeling found tones off the buckets
(rsft_model_residual).

Everything runs in the library's kernels; torch provides device memory and
the autograd plumbing.
"""

import torch


class BucketModel(torch.autograd.Function):
    """model = BucketModel.apply(freqs, amps, plan)

    freqs: CUDA float64 [batch, K, D]; amps: CUDA complex64 [batch, K];
    plan: a Plan. Returns the model buckets as a flat complex64 tensor in the
    layout of Plan.buckets() (per frame [T, *B])."""

    @staticmethod
    def forward(ctx, freqs, amps, plan):
        freqs = freqs.contiguous()
        amps = amps.contiguous()
        ws = plan.model_workspace(freqs.shape[0], freqs.shape[1])
        out = plan.model_forward(freqs, amps, ws)
        ctx.plan = plan
        ctx.workspace = ws
        ctx.save_for_backward(amps)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        (amps,) = ctx.saved_tensors
        gf, ga = ctx.plan.model_backward(amps, grad_out, ctx.workspace)
        return gf, ga, None


def bucket_model(freqs, amps, plan):
    return BucketModel.apply(freqs, amps, plan)


def model_loss(freqs, amps, plan, observed):
    """sum_{s,k} |model_s[k] - observed_s[k]|^2, differentiable."""
    r = bucket_model(freqs, amps, plan) - observed
    return (r.real ** 2 + r.imag ** 2).sum()


@torch.no_grad()
def refine(plan, observed, freqs, amps, steps=20, record_loss=True, trust_bins=0.25, counts=None):
    """Refinement of (freqs, amps) against observed buckets (flat complex64,
    layout of Plan.buckets(); None: the plan's own buckets of the last
    execute) by per-tone trust-region Gauss-Newton steps with step
    acceptance and a per-frame loss guard, all in the library (rsft_refine).
    counts (int32 CUDA [batch], optional): tones taking part per frame.
    Returns (freqs, amps, losses), losses [steps + 1, batch] (FP64, on the
    device) holding each frame's lowest loss so far before each iteration
    and after the last, or None."""
    f = freqs.detach().clone().contiguous()
    a = amps.detach().clone().contiguous()
    ws = plan.refine_workspace(f.shape[0], f.shape[1])
    loss = (torch.empty((steps + 1) * f.shape[0], dtype=torch.float64, device=f.device)
            if record_loss else None)
    plan.refine(f, a, steps, ws, observed=observed, trust_bins=trust_bins, loss=loss, counts=counts)
    return f, a, (loss.view(steps + 1, f.shape[0]) if record_loss else None)


@torch.no_grad()
def initial_amplitudes(plan, freqs, observed=None, with_spread=False):
    """Starting amplitudes of tones at `freqs` (float64 [batch, K, D]) from
    the buckets their nearest cells fall in (rsft_initial_amplitudes); with
    with_spread also each tone's per-round spread."""
    f = freqs.contiguous()
    ws = plan.refine_workspace(f.shape[0], f.shape[1])
    return plan.initial_amplitudes(f, ws, observed=observed, with_spread=with_spread)


@torch.no_grad()
def select_tones(plan, recs, K, candidates=64, max_spread=0.5, observed=None, peel_rounds=2, peel_steps=5):
    """Starting tones for refinement from a detection list (host-side choice
    of which detections to refine).

    Candidates: per frame the candidates * K peak records of largest
    magnitude. A detected cell whose rounds hold different tones' energy
    (the ambiguity of Remark 1) can outrank real tones, but its per-round
    amplitudes disagree; a real tone's agree unless another tone shares its
    bucket in some round.
    1. Amplitudes and spreads of the candidates on the observed buckets
       (rsft_initial_amplitudes); chosen: up to K with spread <= max_spread,
       by magnitude.
    2. peel_rounds times: the chosen tones refined peel_steps iterations (a
       scratch copy; rsft_refine), the residual of the observed buckets after
       them (rsft_model_residual), the other candidates' amplitudes and
       spreads on that residual, where a tone that shared a bucket with a
       chosen one stands alone; chosen becomes the K of largest amplitude
       among the refined chosen tones and the candidates consistent on the
       residual.
    Returns (freqs float64 [batch, K, D], amps complex64 [batch, K], counts
    int32 [batch]) on the device: the chosen records' detector frequencies
    and their amplitudes on the observed buckets; frame f's first counts[f]
    tones are the chosen ones, the rest are zero-amplitude padding that
    rsft_refine leaves out (pass counts)."""
    import numpy as np
    batch = plan.last_batch
    D = len(plan.descs[0]["shape"])
    C = candidates * K
    cand = np.zeros((batch, C, D))
    nvalid = np.zeros(batch, dtype=np.int64)
    for f in range(batch):
        sel = recs[(recs["frame"] == f) & (recs["is_peak"] == 1)]
        sel = sel[np.argsort(-sel["magnitude"], kind="stable")][:C]
        nvalid[f] = len(sel)
        if len(sel) == 0:
            continue
        cand[f, :len(sel)] = sel["freq"][:, :D]
        cand[f, len(sel):] = sel["freq"][0, :D]
    fc = torch.tensor(cand, dtype=torch.float64, device="cuda").contiguous()
    ac_d, sp_d = initial_amplitudes(plan, fc, observed=observed, with_spread=True)
    ac, ok = ac_d.cpu().numpy(), (sp_d <= max_spread).cpu().numpy()
    chosen = [[c for c in range(int(nvalid[f])) if ok[f, c]][:K] for f in range(batch)]

    def gather(amp_src):
        pick = np.zeros((batch, K), dtype=np.int64)
        counts = np.zeros(batch, dtype=np.int32)
        amps = np.zeros((batch, K), dtype=np.complex64)
        for f in range(batch):
            counts[f] = len(chosen[f])
            pick[f, :counts[f]] = chosen[f]
            amps[f, :counts[f]] = amp_src[f, chosen[f]]
        freqs = cand[np.arange(batch)[:, None], pick]
        return (torch.tensor(freqs, dtype=torch.float64, device="cuda").contiguous(),
                torch.tensor(amps, device="cuda").contiguous(),
                torch.tensor(counts, device="cuda"))

    mws = plan.model_workspace(batch, K)
    for _ in range(peel_rounds):
        f0, a0, counts = gather(ac)
        fr, ar, _ = refine(plan, observed, f0, a0, steps=peel_steps, record_loss=False, counts=counts)
        resid = plan.model_residual(fr, ar, mws, observed=observed, counts=counts)
        a2_d, sp2_d = initial_amplitudes(plan, fc, observed=resid, with_spread=True)
        mag_r = np.abs(ar.cpu().numpy())
        mag2, ok2 = np.abs(a2_d.cpu().numpy()), (sp2_d <= max_spread).cpu().numpy()
        for f in range(batch):
            have = set(chosen[f])
            pool = [(float(mag_r[f, k]), c) for k, c in enumerate(chosen[f])]
            pool += [(float(mag2[f, c]), c) for c in range(int(nvalid[f])) if ok2[f, c] and c not in have]
            pool.sort(key=lambda v: -v[0])
            chosen[f] = [c for _, c in pool[:K]]
    return gather(ac)
