"""rsft_autotune's choices carry over to a later plan of the same signature
(device, batch capacity, rounds, mu, dtype, segment mode, frame shapes,
buckets and noise modes), and only to such a plan."""

import numpy as np
import pytest

import synth

from helpers import make_input

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

KEYS = ("fold", "estimate_workers", "vote_kernel", "dft_two_pass", "dft_threads")


def _plan(max_batch):
    from paper_1610_01050_amd import Plan
    shape, buckets = (512, 1024), (32, 64)
    sigma = synth.draw_sigma(np.random.default_rng(8011), 3, shape)
    return Plan(shape, buckets, rounds=3, sigma=sigma, pfa=1e-3, max_batch=max_batch,
                max_detections=1 << 16)


def test_autotuned_shapes_carry_to_a_plan_of_the_same_signature():
    print("autotune cache: 3-frame plan of 512x1024", flush=True)
    a = _plan(3)
    frames = np.stack([make_input((512, 1024), 5, seed=8100 + f)[0] for f in range(3)])
    x = torch.from_numpy(frames).to("cuda")
    a.autotune(x, repeats=2)
    tuned = {k: a.info()[k] for k in KEYS}
    recs_a, counts_a = a.detect()
    b = _plan(3)
    assert {k: b.info()[k] for k in KEYS} == tuned
    b.execute(x)
    recs_b, counts_b = b.detect()
    assert np.array_equal(counts_a, counts_b)
    assert recs_a.tobytes() == recs_b.tobytes()
    # another batch capacity is another signature: the defaults
    c = _plan(7)
    info = c.info()
    assert info["fold"] == {"threads": 256, "vec": 4, "nontemporal": 0}
    assert info["dft_two_pass"] == 1 and info["estimate_workers"] == 0
    for p in (a, b, c):
        p.close()
