"""Host-side checks of two reformulations the kernels rely on, each against
its plain definition (no GPU, no shared code with the HIP path).

* Vote of a 32-cell row in bit-parallel form: in round s the cells of a row
  share their bucket in every dimension but the last, so the round's votes
  for the row are the OR of per-bucket 32-bit masks over the row's flagged
  buckets; a bit-sliced counter adds the rounds and a bit-sliced comparison
  with mu gives the detections. Must equal {i : sum_s c_s[M(i, sigma_s)] >=
  mu} (Def. 3, eq. a_i) cell by cell.
* The word-parallel vote of rows of 128..4096 cells: per round a table
  M_s[b][w] built by scattering each column's preimages x = [sigma^-1 u]
  (Def. 4); per bucket row r (leading bucket indices) the mask E_s[r] = OR
  of the flagged columns' table rows, built once for all cell rows that map
  to r; each cell row then gathers E_s[r_s(row)] four words at a time, and
  the rounds are combined by AND (mu = T) or a bit-sliced counter. Must
  equal the same per-cell sum.
* Segmented scan of many small frames in one 256-wide block: each frame's
  exclusive chunk offsets, records and overflow items (records beyond the
  first 1024 of a chunk that fit the frame's capacity, in items of 256) must
  equal a frame-by-frame running sum.
"""

import numpy as np
import pytest

BLOCK = 256
CHUNK_RECORDS = 1024
ITEM = 256


def votes_per_cell(shape, buckets, sigma, flags, mu):
    """Detections by the definition: sum over rounds of the flag of the
    cell's bucket M(i, sigma_s) (floor hashing, row-major buckets)."""
    D = len(shape)
    idx = np.indices(shape).reshape(D, -1)
    votes = np.zeros(idx.shape[1], dtype=np.int64)
    for s, sig in enumerate(sigma):
        j = np.zeros(idx.shape[1], dtype=np.int64)
        for d in range(D):
            L = shape[d] // buckets[d]
            j = j * buckets[d] + ((sig[d] * idx[d]) % shape[d]) // L
        votes += flags[s][j]
    return votes >= mu


def votes_mask32(shape, buckets, sigma, flags, mu):
    """The bit-parallel form for rows of exactly 32 cells."""
    assert shape[-1] == 32
    D, T = len(shape), len(sigma)
    bl = buckets[-1]
    lsl = int(np.log2(32 // bl))
    nb = 2 if T <= 3 else 3 if T <= 7 else 7
    masks = [[sum(1 << x for x in range(32) if ((sig[-1] * x) & 31) >> lsl == b) for b in range(bl)]
             for sig in sigma]
    out = np.zeros(int(np.prod(shape)), dtype=bool)
    for r in range(out.size // 32):
        coords = np.unravel_index(r * 32, shape)
        acc = [0] * nb
        for s, sig in enumerate(sigma):
            rowpart = 0
            for d in range(D - 1):
                L = shape[d] // buckets[d]
                rowpart = rowpart * buckets[d] + ((sig[d] * coords[d]) % shape[d]) // L
            rowpart *= bl
            m = 0
            for b in range(bl):
                if flags[s][rowpart + b]:
                    m |= masks[s][b]
            for k in range(nb):             # acc += m
                carry = acc[k] & m
                acc[k] ^= m
                m = carry
        ge, eq = 0, 0xFFFFFFFF               # acc >= mu
        for k in range(nb - 1, -1, -1):
            mk = 0xFFFFFFFF if (mu >> k) & 1 else 0
            ge |= eq & acc[k] & ~mk & 0xFFFFFFFF
            eq &= ~(acc[k] ^ mk) & 0xFFFFFFFF
        hit = ge | eq
        out[r * 32:(r + 1) * 32] = [(hit >> x) & 1 for x in range(32)]
    return out


@pytest.mark.parametrize("shape,buckets,T,mu,p", [
    ((16, 8, 32), (4, 2, 8), 3, 3, 0.5),
    ((8, 32), (4, 16), 5, 3, 0.4),
    ((32,), (4,), 3, 2, 0.5),
    ((4, 4, 4, 32), (2, 2, 2, 2), 7, 4, 0.6),
    ((16, 32), (4, 1), 9, 5, 0.5),
    ((8, 32), (2, 8), 2, 1, 0.3),
])
def test_mask32_vote_equals_per_cell_sum(shape, buckets, T, mu, p):
    rng = np.random.default_rng(sum(shape) * 31 + T)
    sigma = [[int(rng.integers(0, n // 2)) * 2 + 1 for n in shape] for _ in range(T)]
    flags = [rng.random(int(np.prod(buckets))) < p for _ in range(T)]
    want = votes_per_cell(shape, buckets, sigma, flags, mu)
    got = votes_mask32(shape, buckets, sigma, flags, mu)
    assert np.array_equal(got, want)
    assert 0 < want.sum() < want.size       # both outcomes occur


def votes_words(shape, buckets, sigma, flags, mu):
    """The word-parallel form for rows of 128..4096 cells: per round the
    bucket-row masks, then four words per thread gathered from them."""
    D, T = len(shape), len(sigma)
    nl, bl = shape[-1], buckets[-1]
    W = nl // 32
    L = nl // bl
    nb = 0 if mu == T else 2 if T <= 3 else 3 if T <= 7 else 7
    nwords = int(np.prod(shape)) // 32
    acc = np.zeros((max(nb, 1), nwords), dtype=np.uint64)
    if nb == 0:
        acc[:] = 0xFFFFFFFF
    for s, sig in enumerate(sigma):
        sinv = pow(int(sig[-1]), -1, nl)
        tab = np.zeros((bl, W), dtype=np.uint64)
        for u in range(nl):                     # scatter the preimages
            x = (sinv * u) % nl
            tab[u // L, x // 32] |= np.uint64(1 << (x % 32))
        nrows = int(np.prod(buckets)) // bl     # bucket rows
        E = np.zeros((nrows, W), dtype=np.uint64)
        for r in range(nrows):                  # expand: once per bucket row
            for b in range(bl):
                if flags[s][r * bl + b]:
                    E[r] |= tab[b]
        for g in range(0, nwords, 4):           # gather: four words of one cell row
            coords = np.unravel_index(g * 32, shape)
            r = 0
            for d in range(D - 1):
                Ld = shape[d] // buckets[d]
                r = r * buckets[d] + ((sig[d] * coords[d]) % shape[d]) // Ld
            w0 = g % W
            m = E[r, w0:w0 + 4]
            for q in range(4):
                if nb == 0:
                    acc[0, g + q] &= m[q]
                    continue
                carry = m[q]
                for k in range(nb):
                    t = acc[k, g + q] & carry
                    acc[k, g + q] ^= carry
                    carry = t
    if nb == 0:
        hit = acc[0]
    else:
        full = np.uint64(0xFFFFFFFF)
        ge = np.zeros(nwords, dtype=np.uint64)
        eq = np.full(nwords, full, dtype=np.uint64)
        for k in range(nb - 1, -1, -1):
            mk = full if (mu >> k) & 1 else np.uint64(0)
            ge |= eq & acc[k] & (~mk & full)
            eq &= ~(acc[k] ^ mk) & full
        hit = ge | eq
    bits = (hit[:, None] >> np.arange(32, dtype=np.uint64)[None, :]) & np.uint64(1)
    return bits.astype(bool).ravel()


@pytest.mark.parametrize("shape,buckets,T,mu,p", [
    ((8, 1024), (4, 64), 3, 3, 0.3),
    ((4, 4096), (2, 128), 3, 2, 0.2),
    ((16, 128), (4, 8), 5, 3, 0.4),
    ((4, 8, 256), (2, 4, 16), 9, 5, 0.5),
    ((2, 2048), (2, 128), 1, 1, 0.1),
    ((512,), (32,), 4, 4, 0.6),
])
def test_word_parallel_vote_equals_per_cell_sum(shape, buckets, T, mu, p):
    rng = np.random.default_rng(sum(shape) * 17 + T)
    sigma = [[int(rng.integers(0, n // 2)) * 2 + 1 for n in shape] for _ in range(T)]
    flags = [rng.random(int(np.prod(buckets))) < p for _ in range(T)]
    want = votes_per_cell(shape, buckets, sigma, flags, mu)
    got = votes_words(shape, buckets, sigma, flags, mu)
    assert np.array_equal(got, want)
    assert 0 < want.sum() < want.size       # both outcomes occur


def scan_per_frame(counts, cap):
    offs, items, tot, itot = [], [], [], []
    for row in counts:
        run = irun = 0
        o, it = [], []
        for v in row:
            fit = min(max(cap - run, 0), v)
            n = -(-max(fit - CHUNK_RECORDS, 0) // ITEM)
            o.append(run)
            it.append(irun)
            run += v
            irun += n
        offs.append(o)
        items.append(it)
        tot.append(run)
        itot.append(irun)
    return np.array(offs), np.array(items), tot, itot


def scan_segmented(counts, cap):
    """256 threads per block, thread t = chunk t mod cch of the block's frame
    t // cch; frame prefixes from the block-wide inclusive sums."""
    nframes, cch = counts.shape
    fpb = BLOCK // cch
    offs = np.zeros_like(counts)
    items = np.zeros_like(counts)
    tot, itot = [0] * nframes, [0] * nframes
    for f0 in range(0, nframes, fpb):
        v = np.zeros(BLOCK, dtype=np.int64)
        for t in range(BLOCK):
            if f0 + t // cch < nframes:
                v[t] = counts[f0 + t // cch, t % cch]
        incl = np.cumsum(v)
        it = np.zeros(BLOCK, dtype=np.int64)
        off = np.zeros(BLOCK, dtype=np.int64)
        for t in range(BLOCK):
            s0 = (t // cch) * cch
            off[t] = incl[t] - v[t] - (incl[s0 - 1] if s0 else 0)
            fit = min(max(cap - off[t], 0), v[t])
            it[t] = -(-max(fit - CHUNK_RECORDS, 0) // ITEM)
        iincl = np.cumsum(it)
        for t in range(BLOCK):
            fi, c = divmod(t, cch)
            f, s0 = f0 + fi, fi * cch
            if f >= nframes:
                continue
            offs[f, c] = off[t]
            items[f, c] = iincl[t] - it[t] - (iincl[s0 - 1] if s0 else 0)
            if c == cch - 1:
                tot[f] = incl[t] - (incl[s0 - 1] if s0 else 0)
                itot[f] = iincl[t] - (iincl[s0 - 1] if s0 else 0)
    return offs, items, tot, itot


@pytest.mark.parametrize("cch,nframes,cap", [(2, 300, 5000), (32, 20, 16384), (128, 5, 60000),
                                             (1, 7, 3000), (64, 9, 30000)])
def test_segmented_scan_equals_per_frame_scan(cch, nframes, cap):
    counts = np.random.default_rng(cch * 1000 + nframes).integers(0, 4000, size=(nframes, cch))
    want = scan_per_frame(counts, cap)
    got = scan_segmented(counts, cap)
    assert np.array_equal(got[0], want[0])
    assert np.array_equal(got[1], want[1])
    assert got[2] == want[2] and got[3] == want[3]
    assert max(want[3]) > 0                  # overflow items occur
