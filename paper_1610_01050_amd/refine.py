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
``refine`` fits frequencies and amplitudes to observed buckets by Gauss-Newton
steps that the backward kernel solves per tone.

Everything runs in the library's kernels; torch provides device memory, the
autograd plumbing and the elementwise residual.
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
def refine(plan, observed, freqs, amps, steps=20, record_loss=True):
    """Gauss-Newton refinement of (freqs, amps) against observed buckets
    (flat complex64, layout of Plan.buckets()). Each step evaluates the model,
    its residual and, in the backward kernel, every tone's Gauss-Newton step
    over (b_t, f_t) (tones decoupled). Returns (freqs, amps, losses), losses
    being the loss before each step and after the last (on the device)."""
    f = freqs.detach().clone().contiguous()
    a = amps.detach().clone().contiguous()
    ws = plan.model_workspace(f.shape[0], f.shape[1])
    model = torch.empty(plan.model_size(f.shape[0]), dtype=torch.complex64, device=f.device)
    losses = []
    for _ in range(steps):
        plan.model_forward(f, a, ws, out=model)
        r = model - observed
        if record_loss:
            losses.append((r.real.double() ** 2 + r.imag.double() ** 2).sum())
        _, _, sf, sa = plan.model_backward(a, 2.0 * r, ws, steps=True)
        f += sf
        a += sa
    if record_loss:
        plan.model_forward(f, a, ws, out=model)
        r = model - observed
        losses.append((r.real.double() ** 2 + r.imag.double() ** 2).sum())
    return f, a, (torch.stack(losses) if losses else None)
