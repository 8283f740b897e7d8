"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs, element by element.

Contract (FP32 path vs FP64 oracle):
* buckets fhat_s (eq. f): max |gpu - oracle| <= 1e-4 * rms of the round;
* first-stage flags: a flag may differ only where |P - gamma| / gamma <= 1e-3
  (an FP32 rounding of |fhat|^2 can cross the threshold only there);
* detections and votes: identical except on cells whose T buckets include
  such an ambiguous bucket; with the oracle's flags injected, identical bit
  for bit;
* estimates of matched detections: magnitude within 1e-3 relative, off-grid
  frequency within 1e-3 bin.
"""

import zlib

import numpy as np
import pytest

import synth
from oracle import rsft as OR

from helpers import (ambiguous, cells_from_records, free_cells, make_input, oracle_plan,
                     pack_flags, unpack_flags)
from helpers import check_frame as _check_frame

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _seed(name):
    return zlib.crc32(name.encode())


def _plan(**kw):
    from paper_1610_01050_amd import Plan
    return Plan(**kw)


CASES = {
    # name: (shape, buckets, rounds, mu, dtype, batch, K, pfa, atten)
    "ongrid_256x256_c128": ((256, 256), (16, 16), 3, 0, "c128", 3, 4, 1e-3, 60.0),
    "offgrid_1024x1024": ((1024, 1024), (64, 64), 3, 0, "c64", 2, 20, 1e-4, 60.0),
    "cube_256x128x32": ((256, 128, 32), (32, 16, 8), 3, 0, "c64", 2, 6, 1e-4, 60.0),
    "one_dim_4096": ((4096,), (64,), 3, 0, "c64", 3, 3, 1e-3, 60.0),
    "four_dim": ((16, 8, 16, 32), (4, 2, 4, 8), 3, 0, "c64", 2, 3, 1e-3, 60.0),
    "short_rows_512x64": ((512, 64), (32, 8), 3, 0, "c64", 2, 5, 1e-3, 60.0),
    "tiny_last_bucket": ((128, 256), (32, 2), 3, 0, "c64", 2, 3, 1e-3, 60.0),
    "wide_rows_multichunk": ((16, 65536), (8, 128), 3, 0, "c64", 1, 1, 1e-3, 60.0),
    "single_round": ((256, 512), (16, 32), 1, 1, "c64", 2, 5, 1e-3, 60.0),
    "t3_mu2_512x256": ((512, 256), (32, 16), 3, 2, "c64", 2, 5, 1e-3, 60.0),
    "five_rounds_mu3": ((256, 256), (16, 16), 5, 3, "c64", 2, 5, 1e-3, 60.0),
    "rectangular_windows": ((256, 256), (16, 16), 3, 0, "c64", 2, 5, 1e-3, 0.0),
    "forty_db": ((1024, 256), (32, 16), 3, 0, "c64", 2, 8, 1e-3, 40.0),
    "max_rounds_64": ((512, 256), (16, 16), 64, 40, "c64", 1, 4, 1e-3, 60.0),
    # rows of 32 cells take the bit-parallel vote; T = 5 and 9 need 3- and
    # 7-bit vote counters
    "rows_of_32_T5_mu3": ((256, 32), (16, 8), 5, 3, "c64", 2, 4, 1e-3, 60.0),
    "rows_of_32_T9_mu5": ((128, 32), (8, 4), 9, 5, "c64", 1, 3, 1e-3, 60.0),
    # the word-parallel vote's largest table (B_last * N_last / 32 = 16384 words)
    "rows_of_4096_b128": ((64, 4096), (8, 128), 3, 0, "c64", 1, 4, 1e-3, 60.0),
    "rows_of_128_T6_mu4": ((256, 128), (16, 8), 6, 4, "c64", 2, 4, 1e-3, 60.0),
}


def _run_case(name, per_frame=False, noise="known", vote_words=1, dft_split=1, dft_threads=None):
    from paper_1610_01050_amd import OPT_DFT_SPLIT, OPT_DFT_THREADS, OPT_VOTE_WORDS
    shape, buckets, T, mu, dtype, batch, K, pfa, atten = CASES[name]
    print(f"case {name} per_frame={per_frame} noise={noise} vote_words={vote_words}", flush=True)
    npdt = np.complex128 if dtype == "c128" else np.complex64
    frames = []
    freqs = []
    for f in range(batch):
        x, fr = make_input(shape, K, seed=_seed(name) % 100000 + f, dtype=npdt)
        frames.append(x)
        freqs.append(fr)
    sigma = synth.draw_sigma(np.random.default_rng(_seed(name) % 7919), T, shape)
    flat = 0.0 if atten == 0.0 else -1.0
    plan = _plan(shape=shape, buckets=buckets, rounds=T, sigma=sigma, window_atten_db=atten,
                 flat_atten_db=flat, pfa=pfa, mu=mu, dtype=dtype, max_batch=batch,
                 noise_mode=noise, max_detections=1 << 18)
    plan.set_option(OPT_VOTE_WORDS, vote_words)
    plan.set_option(OPT_DFT_SPLIT, dft_split)
    if dft_threads is not None:
        plan.set_option(OPT_DFT_THREADS, dft_threads)
    xd = torch.from_numpy(np.stack(frames)).to("cuda")
    if per_frame:
        plan.execute_per_frame(xd)
    else:
        plan.execute(xd)
    recs, counts = plan.detect()
    gbk = [b.cpu().numpy() for b in plan.buckets()]
    gfl = [w.cpu().numpy().view(np.uint32) for w in plan.flags()]
    oplan = oracle_plan(shape, buckets, sigma, atten, flat, pfa, mu)
    refs = [OR.rsft(x, oplan, noise=noise) for x in frames]
    return plan, oplan, frames, refs, recs, counts, gbk, gfl


@pytest.mark.parametrize("name", list(CASES))
def test_fused_path_matches_oracle(name):
    plan, oplan, frames, refs, recs, counts, gbk, gfl = _run_case(name)
    for f, ref in enumerate(refs):
        _check_frame(f, oplan, ref, recs, gbk[f], gfl[f])
        assert counts[f] == len(cells_from_records(recs, oplan.shape, f))
    plan.close()


@pytest.mark.parametrize("name", ["ongrid_256x256_c128", "offgrid_1024x1024", "cube_256x128x32",
                                  "four_dim", "tiny_last_bucket", "max_rounds_64"])
def test_single_workgroup_dft_matches_oracle(name):
    """The DFT stage with one work-group per (round, frame) instead of the
    two passes (RSFT_OPT_DFT_SPLIT = 0), the rest unchanged."""
    plan, oplan, frames, refs, recs, counts, gbk, gfl = _run_case(name, dft_split=0)
    for f, ref in enumerate(refs):
        _check_frame(f, oplan, ref, recs, gbk[f], gfl[f])
    plan.close()


@pytest.mark.parametrize("threads", [64, 256, 1024])
@pytest.mark.parametrize("name", ["ongrid_256x256_c128", "offgrid_1024x1024", "cube_256x128x32",
                                  "one_dim_4096", "four_dim", "tiny_last_bucket"])
def test_dft_work_group_sizes_match_oracle(name, threads):
    """The one-work-group DFT at each work-group size (RSFT_OPT_DFT_THREADS:
    one, four or sixteen waves per transform)."""
    plan, oplan, frames, refs, recs, counts, gbk, gfl = _run_case(name, dft_split=0, dft_threads=threads)
    for f, ref in enumerate(refs):
        _check_frame(f, oplan, ref, recs, gbk[f], gfl[f])
    plan.close()


@pytest.mark.parametrize("threads", [64, 256])
def test_dft_work_group_sizes_estimated_noise_match_oracle(threads):
    """The estimated noise floor (radix selection of the lower median in the
    DFT kernel) with one and four waves per transform."""
    plan, oplan, frames, refs, recs, counts, gbk, gfl = _run_case("short_rows_512x64", noise="estimated",
                                                                  dft_split=0, dft_threads=threads)
    for f, ref in enumerate(refs):
        _check_frame(f, oplan, ref, recs, gbk[f], gfl[f])
    plan.close()


@pytest.mark.parametrize("name", ["ongrid_256x256_c128", "cube_256x128x32", "one_dim_4096"])
def test_per_frame_path_matches_oracle(name):
    plan, oplan, frames, refs, recs, counts, gbk, gfl = _run_case(name, per_frame=True)
    for f, ref in enumerate(refs):
        _check_frame(f, oplan, ref, recs, gbk[f], gfl[f])
    plan.close()


@pytest.mark.parametrize("name", ["offgrid_1024x1024", "short_rows_512x64"])
def test_estimated_noise_floor_matches_oracle(name):
    plan, oplan, frames, refs, recs, counts, gbk, gfl = _run_case(name, noise="estimated")
    for f, ref in enumerate(refs):
        _check_frame(f, oplan, ref, recs, gbk[f], gfl[f])
    plan.close()


@pytest.mark.parametrize("name,vote_words", [
    ("ongrid_256x256_c128", 1), ("ongrid_256x256_c128", 0), ("cube_256x128x32", 1),
    ("four_dim", 1), ("five_rounds_mu3", 1), ("one_dim_4096", 1), ("one_dim_4096", 0),
    ("rows_of_32_T5_mu3", 1), ("rows_of_32_T9_mu5", 1), ("offgrid_1024x1024", 1),
    ("offgrid_1024x1024", 0), ("rows_of_4096_b128", 1), ("rows_of_128_T6_mu4", 1),
    ("short_rows_512x64", 1), ("t3_mu2_512x256", 0), ("t3_mu2_512x256", 1)])
def test_votes_bit_exact_from_oracle_flags(name, vote_words):
    """Voting, second stage and ordering are integer work: given the oracle's
    flags, the detections and their votes must match exactly (word-parallel
    masks where the rows suit them, and the candidate enumeration)."""
    plan, oplan, frames, refs, recs, counts, gbk, gfl = _run_case(name, vote_words=vote_words)
    words = np.concatenate([pack_flags(r["flags"]).ravel() for r in refs]).view(np.int32)
    plan.vote_flags(torch.from_numpy(words.copy()).to("cuda"))
    recs2, counts2 = plan.detect()
    for f, ref in enumerate(refs):
        got = cells_from_records(recs2, oplan.shape, f)
        assert sorted(got) == [int(v) for v in ref["detections"]]
        votes = ref["votes"].ravel()
        assert all(int(r["votes"]) == int(votes[c]) for c, r in got.items())
        assert counts2[f] == len(ref["detections"])
    # records are sorted by (frame, row-major cell)
    keys = [(int(r["frame"]), int(np.ravel_multi_index(tuple(r["idx"][:len(oplan.shape)]),
                                                        oplan.shape))) for r in recs2]
    assert keys == sorted(keys)
    plan.close()


def test_uneven_batch_matches_oracle():
    """Frames of different shapes, each with its own sigma, in one launch."""
    shapes = [(128, 256), (256, 128), (512, 512), (128, 128), (1024, 256), (256, 2048)]
    descs, frames, sigmas = [], [], []
    for i, sh in enumerate(shapes):
        sg = synth.draw_sigma(np.random.default_rng(400 + i), 3, sh)
        bk = tuple(n // 16 for n in sh)
        descs.append(dict(shape=sh, buckets=bk, rounds=3, sigma=sg, pfa=1e-4))
        x, _ = make_input(sh, 6, seed=500 + i)
        frames.append(x)
        sigmas.append(sg)
    from paper_1610_01050_amd import Plan
    plan = Plan.uneven([dict(dsc, max_detections=1 << 16) for dsc in descs])
    xd = torch.from_numpy(np.concatenate([x.ravel() for x in frames])).to("cuda")
    plan.execute(xd)
    recs, counts = plan.detect()
    gbk = [b.cpu().numpy() for b in plan.buckets()]
    gfl = [w.cpu().numpy().view(np.uint32) for w in plan.flags()]
    for f, sh in enumerate(shapes):
        oplan = oracle_plan(sh, tuple(n // 16 for n in sh), sigmas[f], pfa=1e-4)
        ref = OR.rsft(frames[f], oplan)
        _check_frame(f, oplan, ref, recs, gbk[f], gfl[f])
    plan.close()


@pytest.mark.parametrize("threads,vec,nt", [(256, 2, 1), (256, 4, 0), (512, 2, 1), (512, 4, 0)])
def test_fold_shapes_on_short_rows_match_oracle(threads, vec, nt):
    """Every fold launch shape on frames whose rows are shorter than the
    smallest fold pass, where one work-group folds several residue classes
    (rows of 32, 64, 128 and 256 cells, up to 16 classes per tile), uneven
    and uniform: every frame's full result against the oracle."""
    from paper_1610_01050_amd import Plan
    from paper_1610_01050_amd.binding import OPT_FOLD_NONTEMPORAL, OPT_FOLD_THREADS, OPT_FOLD_VEC
    print(f"fold {threads} x {vec}, nt {nt}", flush=True)
    cases = [((128, 32), (8, 4)), ((512, 64), (32, 8)), ((128, 128), (8, 8)),
             ((256, 128), (16, 8)), ((64, 256), (4, 16)), ((256, 256), (16, 16))]
    descs, frames, sigmas = [], [], []
    for i, (sh, bk) in enumerate(cases):
        sg = synth.draw_sigma(np.random.default_rng(470 + i), 3, sh)
        descs.append(dict(shape=sh, buckets=bk, rounds=3, sigma=sg, pfa=1e-3, max_detections=1 << 14))
        x, _ = make_input(sh, 4, seed=570 + i)
        frames.append(x)
        sigmas.append(sg)

    def shaped(plan):
        plan.set_option(OPT_FOLD_THREADS, threads)
        plan.set_option(OPT_FOLD_VEC, vec)
        plan.set_option(OPT_FOLD_NONTEMPORAL, nt)
        return plan

    plan = shaped(Plan.uneven(descs))
    plan.execute(torch.from_numpy(np.concatenate([x.ravel() for x in frames])).to("cuda"))
    recs, counts = plan.detect()
    gbk = [b.cpu().numpy() for b in plan.buckets()]
    gfl = [w.cpu().numpy().view(np.uint32) for w in plan.flags()]
    plan.close()
    refs = []
    for f, (sh, bk) in enumerate(cases):
        oplan = oracle_plan(sh, bk, sigmas[f], pfa=1e-3)
        refs.append((oplan, OR.rsft(frames[f], oplan)))
        _check_frame(f, oplan, refs[-1][1], recs, gbk[f], gfl[f])
    # the same shapes as uniform batches of two frames
    for f, (sh, bk) in enumerate(cases):
        plan = shaped(Plan(sh, bk, rounds=3, sigma=sigmas[f], pfa=1e-3, max_batch=2,
                           max_detections=1 << 14))
        plan.execute(torch.from_numpy(np.stack([frames[f], frames[f]])).to("cuda"))
        recs, counts = plan.detect()
        gbk = [b.cpu().numpy() for b in plan.buckets()]
        gfl = [w.cpu().numpy().view(np.uint32) for w in plan.flags()]
        plan.close()
        for g in range(2):
            _check_frame(g, refs[f][0], refs[f][1], recs, gbk[g], gfl[g])


def test_uneven_3d_mixed_fold_views_matches_oracle():
    """Frames whose fold rows are the last dimension (N_last = 64) or the last
    two flattened (N_last = 32 or 16), of one or two compaction chunks (so
    the vote and estimate take the chunk list), in one launch; both estimate
    layouts give the same records."""
    from paper_1610_01050_amd import OPT_ESTIMATE_WORKERS, Plan
    cases = [((64, 32, 32), (8, 8, 8)), ((32, 16, 64), (4, 4, 8)),
             ((16, 128, 32), (4, 16, 4)), ((8, 64, 16), (4, 8, 4))]
    descs, frames, sigmas = [], [], []
    for i, (sh, bk) in enumerate(cases):
        sg = synth.draw_sigma(np.random.default_rng(450 + i), 3, sh)
        descs.append(dict(shape=sh, buckets=bk, rounds=3, sigma=sg, pfa=1e-3, max_detections=1 << 15))
        x, _ = make_input(sh, 5, seed=550 + i)
        frames.append(x)
        sigmas.append(sg)
    xd = torch.from_numpy(np.concatenate([x.ravel() for x in frames])).to("cuda")
    out = []
    for workers in (0, 1):
        plan = Plan.uneven(descs)
        plan.set_option(OPT_ESTIMATE_WORKERS, workers)
        plan.execute(xd)
        recs, counts = plan.detect()
        gbk = [b.cpu().numpy() for b in plan.buckets()]
        gfl = [w.cpu().numpy().view(np.uint32) for w in plan.flags()]
        plan.close()
        out.append((recs, counts, gbk, gfl))
    assert np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][0], out[1][0])
    recs, counts, gbk, gfl = out[0]
    for f, (sh, bk) in enumerate(cases):
        oplan = oracle_plan(sh, bk, sigmas[f], pfa=1e-3)
        ref = OR.rsft(frames[f], oplan)
        _check_frame(f, oplan, ref, recs, gbk[f], gfl[f])


def test_graph_replay_equals_eager():
    """The captured launch sequence gives the same results on every replay as
    the eager launches, with eager work in between."""
    from paper_1610_01050_amd import OPT_GRAPH
    shape, buckets = (512, 512), (32, 32)
    xs = [make_input(shape, 8, seed=700 + f)[0] for f in range(4)]
    xd = torch.from_numpy(np.stack(xs)).to("cuda")
    sigma = synth.draw_sigma(np.random.default_rng(3), 3, shape)
    plan = _plan(shape=shape, buckets=buckets, rounds=3, sigma=sigma, pfa=1e-3, max_batch=4)
    plan.set_option(OPT_GRAPH, 0)
    plan.execute(xd)
    ref_recs, _ = plan.detect()
    ref_bk = plan.buckets()[0].cpu().numpy()
    for rep in range(3):
        plan.set_option(OPT_GRAPH, 1)
        plan.execute(xd)
        recs, _ = plan.detect()
        assert np.array_equal(plan.buckets()[0].cpu().numpy(), ref_bk)
        assert np.array_equal(recs, ref_recs)
        plan.set_option(OPT_GRAPH, 0)
        plan.execute(xd)
        torch.cuda.synchronize()
    plan.close()


def test_empty_batch_and_nan_frame():
    shape, buckets = (256, 256), (16, 16)
    sigma = synth.draw_sigma(np.random.default_rng(8), 3, shape)
    plan = _plan(shape=shape, buckets=buckets, rounds=3, sigma=sigma, pfa=1e-3, max_batch=2)
    xs = [make_input(shape, 4, seed=800 + f)[0] for f in range(2)]
    xs[0][10, 20] = np.nan
    xd = torch.from_numpy(np.stack(xs)).to("cuda")
    plan.execute(xd, batch=0)
    recs, counts = plan.detect()
    assert len(recs) == 0 and len(counts) == 0
    plan.execute(xd)
    recs, counts = plan.detect()
    bk = [b.cpu().numpy() for b in plan.buckets()]
    assert np.all(np.isnan(bk[0]))          # the NaN spreads to every bucket
    assert counts[0] == 0                    # and no flag is set (NaN >= gamma is false)
    oplan = oracle_plan(shape, buckets, sigma)
    ref = OR.rsft(xs[1], oplan)
    _check_frame(1, oplan, ref, recs, bk[1], plan.flags()[1].cpu().numpy().view(np.uint32))
    plan.close()


def test_capacity_overflow_keeps_exact_counts():
    """A frame over max_detections keeps its first max_detections records in
    row-major order; the counts stay exact and detect() reports CAPACITY."""
    from paper_1610_01050_amd import RsftError
    shape, buckets = (256, 256), (16, 16)
    sigma = synth.draw_sigma(np.random.default_rng(9), 3, shape)
    xs = [make_input(shape, 4, seed=900 + f)[0] for f in range(2)]
    xd = torch.from_numpy(np.stack(xs)).to("cuda")
    full = _plan(shape=shape, buckets=buckets, rounds=3, sigma=sigma, pfa=1e-2, max_batch=2)
    full.execute(xd)
    frecs, fcounts = full.detect()
    small = _plan(shape=shape, buckets=buckets, rounds=3, sigma=sigma, pfa=1e-2,
                  max_batch=2, max_detections=8)
    small.execute(xd)
    with pytest.raises(RsftError):
        small.detect()
    recs, counts = small.detect(allow_truncation=True)
    assert np.array_equal(counts, fcounts)
    for f in range(2):
        assert counts[f] > 8
        want = frecs[frecs["frame"] == f][:8]
        assert np.array_equal(recs[recs["frame"] == f], want)
    oplan = oracle_plan(shape, buckets, sigma, pfa=1e-2)
    for f in range(2):
        ref = OR.rsft(xs[f], oplan)
        amb = ambiguous(ref["buckets"], ref["gamma"])
        n_free = int(free_cells(amb, oplan).sum())
        assert abs(int(counts[f]) - len(ref["detections"])) <= n_free
    full.close()
    small.close()


def test_dense_chunk_every_cell_detected():
    """Noise 20 dB above the design variance flags every bucket, so all
    32768 cells of the frame's single compaction chunk are detected: the
    compaction's multi-pass path (more detections than one listing holds),
    with every record compared to the oracle, plus a capacity cut inside a
    later pass."""
    shape, buckets = (128, 256), (16, 16)
    sigma = synth.draw_sigma(np.random.default_rng(17), 3, shape)
    x = (synth.noise_only(shape, 31, 0, dtype=np.complex128) * 10.0).astype(np.complex64)
    xd = torch.from_numpy(x[None]).to("cuda")
    plan = _plan(shape=shape, buckets=buckets, rounds=3, sigma=sigma, pfa=1e-3, max_batch=1,
                 max_detections=1 << 16)
    plan.execute(xd)
    recs, counts = plan.detect()
    gbk = [b.cpu().numpy() for b in plan.buckets()]
    gfl = [w.cpu().numpy().view(np.uint32) for w in plan.flags()]
    oplan = oracle_plan(shape, buckets, sigma, pfa=1e-3)
    ref = OR.rsft(x, oplan)
    assert len(ref["detections"]) > 20000
    _check_frame(0, oplan, ref, recs, gbk[0], gfl[0])
    cut = _plan(shape=shape, buckets=buckets, rounds=3, sigma=sigma, pfa=1e-3, max_batch=1,
                max_detections=5000)
    cut.execute(xd)
    crecs, ccounts = cut.detect(allow_truncation=True)
    assert np.array_equal(ccounts, counts)
    assert np.array_equal(crecs, recs[:5000])
    plan.close()
    cut.close()


DENSE = {
    # name: (shape, buckets): at Pfa 0.3 (p1 = 0.67 per round) about 45% of
    # the cells are detected, ~15000 per compaction chunk of 2^15 cells
    "dense_256x256": ((256, 256), (16, 16)),
    "dense_64x32x32": ((64, 32, 32), (8, 8, 8)),
}


@pytest.mark.parametrize("cap", [None, 20000])
@pytest.mark.parametrize("name", sorted(DENSE))
def test_estimate_layouts_on_dense_chunks(name, cap):
    """Chunks far beyond 1024 detections: the estimate without and with
    overflow workers gives the same records bit for bit, and they match the
    oracle; a frame capacity that cuts the list keeps its first records."""
    from paper_1610_01050_amd import OPT_ESTIMATE_WORKERS
    shape, buckets = DENSE[name]
    print(f"dense case {name} cap={cap}", flush=True)
    xs = [make_input(shape, 6, seed=901 + f)[0] for f in range(2)]
    xd = torch.from_numpy(np.stack(xs)).to("cuda")
    sigma = synth.draw_sigma(np.random.default_rng(5), 3, shape)

    def run(max_det, workers):
        plan = _plan(shape=shape, buckets=buckets, rounds=3, sigma=sigma, pfa=0.3, max_batch=2,
                     max_detections=max_det)
        plan.set_option(OPT_ESTIMATE_WORKERS, workers)
        assert plan.info()["estimate_workers"] == workers
        plan.execute(xd)
        recs, counts = plan.detect(allow_truncation=True)
        gbk = [b.cpu().numpy() for b in plan.buckets()]
        gfl = [w.cpu().numpy().view(np.uint32) for w in plan.flags()]
        plan.close()
        return recs, counts, gbk, gfl

    full = 1 << 16
    r0, c0, _, _ = run(cap or full, 0)
    r1, c1, gbk, gfl = run(cap or full, 1)
    assert np.array_equal(c0, c1)
    assert np.array_equal(r0, r1)
    oplan = oracle_plan(shape, buckets, sigma, pfa=0.3)
    if cap is None:
        assert int(c1.max()) > 2 * 1024          # overflow items exist
        ref = OR.rsft(xs[0], oplan)
        _check_frame(0, oplan, ref, r1, gbk[0], gfl[0])
    else:
        assert int(c1.min()) > cap               # every frame is cut
        ru, _, _, _ = run(full, 0)
        for f in range(2):
            got = r1[r1["frame"] == f]
            assert len(got) == cap
            assert np.array_equal(got, ru[ru["frame"] == f][:cap])


def test_autotuned_fold_keeps_parity():
    """Whatever launch shape the tuner picks, the results stay within the
    parity contract."""
    name = "offgrid_1024x1024"
    plan, oplan, frames, refs, recs, counts, gbk, gfl = _run_case(name)
    xd = torch.from_numpy(np.stack(frames)).to("cuda")
    ms = plan.autotune(xd, repeats=2)
    assert ms > 0
    cfg = plan.info()["fold"]
    assert cfg["threads"] in (256, 512) and cfg["vec"] in (2, 4)
    plan.execute(xd)
    recs, counts = plan.detect()
    gbk = [b.cpu().numpy() for b in plan.buckets()]
    gfl = [w.cpu().numpy().view(np.uint32) for w in plan.flags()]
    for f, ref in enumerate(refs):
        _check_frame(f, oplan, ref, recs, gbk[f], gfl[f], check_estimates=False)
    plan.close()
