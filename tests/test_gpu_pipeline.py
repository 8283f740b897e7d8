"""The execute in two halves (rsft_execute_fold / rsft_execute_tail) and
batches pipelined over two plans: results bit for bit those of whole
rsft_execute calls on the same inputs, graph replay on and off."""

import numpy as np
import pytest

import synth
from helpers import make_input

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

SHAPE, BUCKETS, BATCH = (512, 256), (32, 16), 4


def _plan():
    from paper_1610_01050_amd import Plan
    sigma = synth.draw_sigma(np.random.default_rng(5), 3, SHAPE)
    return Plan(SHAPE, BUCKETS, rounds=3, sigma=sigma, pfa=1e-3, max_batch=BATCH)


def _inputs(n):
    out = []
    for k in range(n):
        frames = np.stack([make_input(SHAPE, 6, 100 * k + f)[0] for f in range(BATCH)])
        out.append(torch.from_numpy(frames).to("cuda"))
    return out


def _result(plan, stream=None):
    recs, counts = plan.detect(stream=stream)
    bk = torch.cat([b.reshape(-1) for b in plan.buckets()]).cpu().numpy()
    return recs, counts, bk


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("graph", [1, 0])
def test_fold_then_tail_equals_execute(graph):
    from paper_1610_01050_amd import OPT_GRAPH, RsftError
    print(f"graph {graph}", flush=True)
    plan = _plan()
    plan.set_option(OPT_GRAPH, graph)
    (x,) = _inputs(1)
    plan.execute(x)
    want = _result(plan)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    done = torch.cuda.Event()
    for _ in range(2):   # the second time from the captured graphs
        plan.execute_fold(x, stream=s1)
        done.record(s1)
        s2.wait_event(done)
        plan.execute_tail(stream=s2)
        s2.synchronize()
        assert _same(_result(plan, s2), want)
    with pytest.raises(RsftError):
        plan.execute_tail(stream=s2)    # no fold pending
    plan.close()


def test_two_plans_pipelined_equal_whole_executes():
    """Six batches alternating over two plans, each plan's fold ordered
    after its own previous tail and its tail after its own fold; every
    batch's results (read after its tail) equal a whole execute of the same
    input on a third plan."""
    plans = [_plan(), _plan()]
    ref = _plan()
    xs = _inputs(6)
    sF = torch.cuda.Stream()
    sT = [torch.cuda.Stream(), torch.cuda.Stream()]
    fdone = [torch.cuda.Event(), torch.cuda.Event()]
    tdone = [torch.cuda.Event(), torch.cuda.Event()]
    got = []
    for k, x in enumerate(xs):
        i = k % 2
        if k >= 2:
            got.append(_result(plans[i], sT[i]))   # batch k - 2, before the plan is reused
        sF.wait_event(tdone[i])
        plans[i].execute_fold(x, stream=sF)
        fdone[i].record(sF)
        sT[i].wait_event(fdone[i])
        plans[i].execute_tail(stream=sT[i])
        tdone[i].record(sT[i])
    got.append(_result(plans[0], sT[0]))
    got.append(_result(plans[1], sT[1]))
    for k, x in enumerate(xs):
        ref.execute(x)
        assert _same(got[k], _result(ref)), f"batch {k}"
    for p in plans + [ref]:
        p.close()
