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
trust-region Gauss-Newton steps with step acceptance (rsft_refine), and
``initial_amplitudes`` gives detected tones their starting amplitudes
(rsft_initial_amplitudes).

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
def refine(plan, observed, freqs, amps, steps=20, record_loss=True, trust_bins=0.25):
    """Refinement of (freqs, amps) against observed buckets (flat complex64,
    layout of Plan.buckets(); None: the plan's own buckets of the last
    execute) by per-tone trust-region Gauss-Newton steps with step
    acceptance, all in the library (rsft_refine). Returns (freqs, amps,
    losses), losses [steps + 1, batch] (FP64, on the device) holding the loss
    before each step and after the last, or None."""
    f = freqs.detach().clone().contiguous()
    a = amps.detach().clone().contiguous()
    ws = plan.refine_workspace(f.shape[0], f.shape[1])
    loss = (torch.empty((steps + 1) * f.shape[0], dtype=torch.float64, device=f.device)
            if record_loss else None)
    plan.refine(f, a, steps, ws, observed=observed, trust_bins=trust_bins, loss=loss)
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
def select_tones(plan, recs, K, candidates=4, max_spread=0.5, observed=None):
    """Starting tones for refinement from a detection list (host-side choice
    of which detections to refine): per frame the candidates * K peak
    records of largest magnitude, their amplitudes and per-round spreads
    from rsft_initial_amplitudes, then the K of largest magnitude among
    those with spread <= max_spread (a peak whose rounds disagree is the
    Remark-1 ambiguity, not a tone), filled up with the strongest remaining
    candidates when fewer pass. Returns (freqs float64 [batch, K, D],
    amps complex64 [batch, K], passed [batch]) on the device."""
    import numpy as np
    batch = plan.last_batch
    D = len(plan.descs[0]["shape"])
    C = candidates * K
    cand = np.zeros((batch, C, D))
    for f in range(batch):
        sel = recs[(recs["frame"] == f) & (recs["is_peak"] == 1)]
        sel = sel[np.argsort(-sel["magnitude"], kind="stable")][:C]
        if len(sel) == 0:
            continue
        cand[f, :len(sel)] = sel["freq"][:, :D]
        cand[f, len(sel):] = sel["freq"][0, :D]
    fc = torch.tensor(cand, dtype=torch.float64, device="cuda").contiguous()
    ac, sp = initial_amplitudes(plan, fc, observed=observed, with_spread=True)
    ok = (sp <= max_spread).cpu().numpy()
    freqs = np.zeros((batch, K, D))
    pick = np.zeros((batch, K), dtype=np.int64)
    passed = np.zeros(batch, dtype=np.int64)
    for f in range(batch):
        order = [c for c in range(C) if ok[f, c]]
        passed[f] = min(len(order), K)
        order += [c for c in range(C) if not ok[f, c]]
        pick[f] = order[:K]
        freqs[f] = cand[f, pick[f]]
    idx = torch.tensor(pick, device="cuda")
    amps = torch.gather(ac, 1, idx).contiguous()
    return torch.tensor(freqs, dtype=torch.float64, device="cuda").contiguous(), amps, passed
