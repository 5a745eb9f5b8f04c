"""Bucket tiles (BLSH_TILES): LSH banding handed over as 16 x 16 tiles of each
bucket's members (bayeslsh_band_tiles) must list exactly the oracle's banding
pairs in the oracle's tiled order (Section 2), and Algorithm 1 over the tiles
(bayeslsh_verify) must give the oracle's decisions, levels, m and S_hat for
those pairs -- and the same output as the PAIRS path over the same pairs."""
import numpy as np
import pytest
import torch

import paper_1110_1328_amd as P
from oracle import reference as R
from synth import generators as G

from gpu_util import assert_same_as_oracle, decode_result, down, sigs_tensor, up

pytestmark = pytest.mark.gpu

EPS, DELTA, GAMMA = 0.03, 0.05, 0.03


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = P.bayeslsh_create(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def mix():
    return G.dense_mixture(n=3000, d=64, n_comp=30, seed=G.SEED_BASE + 61)


def _bits(mix, n_bits, seed):
    planes = G.gaussian_planes(mix.x.shape[1], n_bits, seed)
    return G.pack_bits((mix.x.astype(np.float64) @ planes >= 0).astype(np.uint8))


TW = 24   # int64 words per 192-byte tile descriptor


def expand(tiles_i64, n_tiles):
    """Host expansion of tile descriptors into (x, y) in candidate order; also
    checks that each tile numbers its candidates right after the previous one."""
    d = tiles_i64[: n_tiles * TW].reshape(n_tiles, TW)
    first = d[:, 0]
    n_rows = (d[:, 1] & 0xFFFFFFFF).astype(np.int64)
    n_cols = ((d[:, 1] >> 32) & 0xFFFFFFFF).astype(np.int64)
    keep = np.ascontiguousarray(d[:, 2:6]).view(np.uint64)
    ids = np.ascontiguousarray(d[:, 6:22]).view(np.uint32).reshape(n_tiles, 32)
    bits = np.unpackbits(keep.view(np.uint8).reshape(n_tiles, 32), axis=1, bitorder="little").astype(bool)
    counts = bits.sum(axis=1)
    assert np.array_equal(first, np.concatenate([[0], np.cumsum(counts)[:-1]]))
    assert np.all((n_rows >= 1) & (n_rows <= 16) & (n_cols >= 1) & (n_cols <= 16))
    t_idx, p = np.nonzero(bits)
    r, c = p // 16, p % 16
    assert np.all(r < n_rows[t_idx]) and np.all(c < n_cols[t_idx])
    return ids[t_idx, r], ids[t_idx, 16 + c]


def band_tiles(ctx, S, nb, b, max_bucket=0, cap=1 << 16):
    tl, nt, npairs, trunc = P.bayeslsh_band_tiles(ctx, S, nb, b, cap, max_bucket=max_bucket)
    assert not trunc
    return tl, nt, npairs


@pytest.mark.parametrize("nb,b,max_bucket", [(8, 8, 0), (5, 11, 0), (3, 5, 40), (20, 3, 40), (4, 16, 0)])
def test_band_tiles_list_the_oracle_pairs(ctx, mix, nb, b, max_bucket):
    """Both layouts; keys that straddle a word; bucket caps that are not a
    multiple of 16; 20 bands of 3 bits (the earlier-band test drops most
    pairs, so keep masks have holes): the tiles expand to the oracle's tiled
    pairs, numbered consecutively."""
    print("band tiles nb=%d b=%d max_bucket=%d" % (nb, b, max_bucket), flush=True)
    bits = _bits(mix, 64, G.SEED_BASE + 62)
    wx, wy = R.band_candidates(bits, nb, b, max_bucket, tile=16)
    assert len(wx) > 1000
    for layout in (P.OBJECT_MAJOR, P.WORD_MAJOR):
        tl, nt, npairs = band_tiles(ctx, sigs_tensor(bits, P.COSINE, layout), nb, b, max_bucket)
        assert npairs == len(wx)
        gx, gy = expand(tl.cpu().numpy(), nt)
        np.testing.assert_array_equal(gx, wx)
        np.testing.assert_array_equal(gy, wy)


@pytest.fixture(scope="module")
def banded(mix):
    """16 bands x 6 bits of an independent 96-bit projection: the oracle's
    tiled pairs (about 1.2M), computed once."""
    band = _bits(mix, 96, G.SEED_BASE + 63)
    return band, R.band_candidates(band, 16, 6, 0, tile=16)


@pytest.mark.parametrize("k,n_max,t", [(32, 1024, 0.8), (16, 256, 0.7), (64, 512, 0.7), (32, 128, 0.7),
                                       (64, 2048, 0.8), (16, 1024, 0.9)])
def test_tiles_verify_matches_oracle(ctx, mix, banded, k, n_max, t):
    """Algorithm 1 over the tiles of a banding of the mixture (16 bands x 6
    bits, buckets of a few to a few hundred members, keep masks with holes),
    on an independent n_max-bit projection, every group width of the row
    kernel (n_max / 128 = 1 .. 16 lanes), every k and both acceptance tests
    (interval bounds, accept bitmask): the oracle's output on the oracle's
    banding pairs, and the PAIRS path's output."""
    print("tiles verify k=%d n_max=%d t=%.1f" % (k, n_max, t), flush=True)
    band, (wx, wy) = banded
    sig = _bits(mix, n_max, G.SEED_BASE + 64 + n_max)
    tl, nt, npairs = band_tiles(ctx, sigs_tensor(band, P.COSINE, P.OBJECT_MAJOR), 16, 6)
    assert npairs == len(wx)
    want = R.verify(wx, wy, P.COSINE, sig, k, n_max // k, t, EPS, DELTA, GAMMA)
    # pruned and concentrated everywhere; accepted at n_max too except where
    # every pair concentrates first (2048 hashes; t = 0.9)
    assert {0, 1} <= set(want["decision"].tolist())
    S = sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR)
    # acceptance tested with the two bounds of each level's accept interval,
    # then with the accept bitmask (the path for tables whose accept sets are
    # not intervals): the same output
    for bitmask in (1, 0):
        P.bayeslsh_set_tuning(ctx, tiles_accept_bitmask=bitmask)
        res = P.make_result(npairs, npairs, m_debug=True)
        P.bayeslsh_verify(ctx, P.tiles(tl, nt, npairs), S, t, EPS, DELTA, GAMMA, (1, 1), k, res)
        P.bayeslsh_sync(ctx)
        got = decode_result(res, npairs)
        assert_same_as_oracle(got, want)
    P.bayeslsh_set_tuning(ctx)
    res_p = P.make_result(npairs, npairs, m_debug=True)
    P.bayeslsh_verify(ctx, P.pairs(up(wx), up(wy)), S, t, EPS, DELTA, GAMMA, (1, 1), k, res_p)
    P.bayeslsh_sync(ctx)
    gp = decode_result(res_p, npairs)
    np.testing.assert_array_equal(got["code"], gp["code"])
    np.testing.assert_array_equal(got["acc_val"], gp["acc_val"])


def _tile(first, row_ids, col_ids, positions):
    n_rows, n_cols = len(row_ids), len(col_ids)
    keep = np.zeros(4, np.uint64)
    for p_ in positions:
        keep[p_ // 64] |= np.uint64(1) << np.uint64(p_ % 64)
    ids = np.full(32, 0xFFFFFFFF, np.uint32)
    ids[:n_rows] = row_ids
    ids[16:16 + n_cols] = col_ids
    head = np.array([first, n_rows | (n_cols << 32)], np.int64)
    return np.concatenate([head, keep.view(np.int64), ids.view(np.int64), np.zeros(2, np.int64)])


def test_tiles_by_hand_and_malformed(ctx):
    """Hand-made tiles: partial rows and columns, sparse keep masks, more tiles
    than one launch of the persistent grid takes at once; then a member id >=
    n_obj (code 0xFF, BLSH_EBADID), a position past n_rows and numbering past
    n_cand (BLSH_EINVAL), an empty tile list."""
    rng = np.random.default_rng(8)
    n_obj, n_max, k = 500, 256, 32
    sig = G.pack_bits(G.calibration_bits(n_obj // 2, n_max, rng.uniform(0.6, 1.0, n_obj // 2), 81))
    tiles, xs, ys, first = [], [], [], 0
    for _ in range(9000):
        nr, nc = int(rng.integers(1, 17)), int(rng.integers(1, 17))
        rows = rng.integers(0, n_obj, nr).astype(np.uint32)
        cols = rng.integers(0, n_obj, nc).astype(np.uint32)
        pos = sorted(int(16 * r + c) for r in range(nr) for c in range(nc) if rng.random() < 0.7)
        if not pos:
            continue
        tiles.append(_tile(first, rows, cols, pos))
        xs += [rows[q // 16] for q in pos]
        ys += [cols[q % 16] for q in pos]
        first += len(pos)
    x, y = np.array(xs, np.uint32), np.array(ys, np.uint32)
    S = sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR)
    want = R.verify(x, y, P.COSINE, sig, k, n_max // k, 0.7, EPS, DELTA, GAMMA)
    tl = up(np.stack(tiles).reshape(-1))
    res = P.make_result(first, first, m_debug=True)
    P.bayeslsh_verify(ctx, P.tiles(tl, len(tiles), first), S, 0.7, EPS, DELTA, GAMMA, (1, 1), k, res)
    P.bayeslsh_sync(ctx)
    assert_same_as_oracle(decode_result(res, first), want)

    def run_one(tile, n_cand):
        r = P.make_result(max(n_cand, 1), 16)
        r.code.fill_(0xEE)
        P.bayeslsh_verify(ctx, P.tiles(up(tile), 1, n_cand), S, 0.7, EPS, DELTA, GAMMA, (1, 1), k, r)
        with pytest.raises(P.BayesLSHError) as e:
            P.bayeslsh_sync(ctx)
        return e.value.code, r.code[:n_cand].cpu().numpy()

    rows = np.arange(4, dtype=np.uint32)
    cols = np.arange(8, 12, dtype=np.uint32)
    bad_rows = rows.copy()
    bad_rows[3] = n_obj + 5                                             # row member 3 is a bad id
    code, got = run_one(_tile(0, bad_rows, cols, [16 * r + c for r in range(4) for c in range(4)]), 16)
    assert code == -5 and np.all(got[12:16] == 0xFF) and np.all(got[:12] != 0xFF)   # BLSH_EBADID
    code, got = run_one(_tile(0, rows[:2], cols[:2], [0, 1, 16, 17, 34]), 5)          # position past n_rows
    assert code == -1 and got[4] == 0xFF and np.all(got[:4] != 0xFF)
    code, got = run_one(_tile(3, rows[:2], cols[:2], [0, 1, 16, 17]), 5)              # numbering past n_cand
    assert code == -1 and np.all(got == 0xEE)                                         # the tile is skipped
    r = P.make_result(1, 1)
    r.n_accepted.fill_(9)
    P.bayeslsh_verify(ctx, P.tiles(tl, 0, 0), S, 0.7, EPS, DELTA, GAMMA, (1, 1), k, r)
    P.bayeslsh_sync(ctx)
    assert int(r.n_accepted.item()) == 0



@pytest.mark.parametrize("per_launch,stage_cap", [(97, 0), (1000, 0), (97, 64)])
def test_tiles_many_launches(ctx, per_launch, stage_cap):
    """A call cut into many launches (tiles_per_launch), each launch's staged
    accepted pairs appended to the caller's list after it; with a tiny staging
    most pairs go to the list directly from the tile kernel.  Same codes, m
    and accepted list as one launch, and as the oracle."""
    rng = np.random.default_rng(13)
    n_obj, n_max, k = 500, 256, 32
    sig = G.pack_bits(G.calibration_bits(n_obj // 2, n_max, rng.uniform(0.6, 1.0, n_obj // 2), 131))
    tiles, xs, ys, first = [], [], [], 0
    for _ in range(6000):
        nr, nc = int(rng.integers(1, 17)), int(rng.integers(1, 17))
        rows = rng.integers(0, n_obj, nr).astype(np.uint32)
        cols = rng.integers(0, n_obj, nc).astype(np.uint32)
        pos = sorted(int(16 * r + c) for r in range(nr) for c in range(nc) if rng.random() < 0.7)
        if not pos:
            continue
        tiles.append(_tile(first, rows, cols, pos))
        xs += [rows[q // 16] for q in pos]
        ys += [cols[q % 16] for q in pos]
        first += len(pos)
    x, y = np.array(xs, np.uint32), np.array(ys, np.uint32)
    S = sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR)
    want = R.verify(x, y, P.COSINE, sig, k, n_max // k, 0.7, EPS, DELTA, GAMMA)
    cand = P.tiles(up(np.stack(tiles).reshape(-1)), len(tiles), first)
    one = P.make_result(first, first, m_debug=True)
    P.bayeslsh_verify(ctx, cand, S, 0.7, EPS, DELTA, GAMMA, (1, 1), k, one)
    P.bayeslsh_sync(ctx)
    P.bayeslsh_set_tuning(ctx, tiles_per_launch=per_launch, acc_stage_cap=stage_cap)
    try:
        for _ in range(2):   # twice: the second call reuses the staging
            res = P.make_result(first, first, m_debug=True)
            P.bayeslsh_verify(ctx, cand, S, 0.7, EPS, DELTA, GAMMA, (1, 1), k, res)
            P.bayeslsh_sync(ctx)
            got = decode_result(res, first)
            assert_same_as_oracle(got, want)
            ref = decode_result(one, first)
            np.testing.assert_array_equal(got["code"], ref["code"])
            np.testing.assert_array_equal(got["m"], ref["m"])
            np.testing.assert_array_equal(got["acc_val"], ref["acc_val"])
    finally:
        P.bayeslsh_set_tuning(ctx)


def test_tiles_per_launch_rejected_out_of_range(ctx):
    for v in (-1, (1 << 22) + 1):
        with pytest.raises(P.BayesLSHError) as e:
            P.bayeslsh_set_tuning(ctx, tiles_per_launch=v)
        assert e.value.code == -1
    P.bayeslsh_set_tuning(ctx, tiles_per_launch=1 << 22)
    assert P.bayeslsh_get_tuning(ctx)["tiles_per_launch"] == 1 << 22
    P.bayeslsh_set_tuning(ctx)


@pytest.mark.parametrize("order", ["ascending", "descending", "shuffled"])
def test_tiles_numbered_past_two_to_the_31_and_32(ctx, order):
    """Tiles whose candidates are numbered beyond 2^31 and 2^32 (a result of
    4.3e9 candidates, most of them outside these tiles), handed over in
    ascending, descending or shuffled order of their numbering (one launch
    holds them all): codes, m and accepted indices land at those numbers,
    equal to the oracle's output for the same pairs."""
    rng = np.random.default_rng(9)
    n_obj, n_max, k = 600, 512, 32
    sig = G.pack_bits(G.calibration_bits(n_obj // 2, n_max, rng.uniform(0.6, 1.0, n_obj // 2), 91))
    S = sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR)
    n_cand = (1 << 32) + 5000
    # three full tiles (768 numbers) from each start: straddling 2^31 and 2^32, disjoint
    starts = [(1 << 31) - 300, (1 << 31) + 1000, (1 << 32) - 400, (1 << 32) + 1000]
    tiles, xs, ys, idx = [], [], [], []
    for st in starts:
        for u in range(3):
            rows = np.sort(rng.choice(n_obj, 16, replace=False)).astype(np.uint32)
            cols = np.sort(rng.choice(n_obj, 16, replace=False)).astype(np.uint32)
            pos = list(range(256))
            first = st + 256 * u
            tiles.append(_tile(first, rows, cols, pos))
            xs += [rows[q // 16] for q in pos]
            ys += [cols[q % 16] for q in pos]
            idx += list(range(first, first + 256))
    x, y, idx = np.array(xs, np.uint32), np.array(ys, np.uint32), np.array(idx, np.int64)
    want = R.verify(x, y, P.COSINE, sig, k, n_max // k, 0.7, EPS, DELTA, GAMMA)
    tiles = np.stack(tiles)
    if order == "descending":
        tiles = tiles[::-1]
    elif order == "shuffled":
        tiles = tiles[np.random.default_rng(10).permutation(len(tiles))]
    res = P.make_result(n_cand, 1 << 16, m_debug=True)
    res.code.fill_(0xEE)
    P.bayeslsh_verify(ctx, P.tiles(up(np.ascontiguousarray(tiles).reshape(-1)), len(tiles), n_cand), S, 0.7, EPS,
                      DELTA, GAMMA, (1, 1), k, res)
    P.bayeslsh_sync(ctx)
    idx_d = torch.from_numpy(idx).cuda()
    code = res.code[idx_d].cpu().numpy()
    m = res.m_debug.view(torch.int16)[idx_d].cpu().numpy().view(np.uint16).astype(np.int32)
    np.testing.assert_array_equal(code >> 6, want["decision"])
    np.testing.assert_array_equal(code & 63, want["level"])
    np.testing.assert_array_equal(m, want["m"])
    ai, av = res.accepted()
    emit = (want["decision"] == 1) | (want["decision"] == 2)
    np.testing.assert_array_equal(ai, idx[emit])
    np.testing.assert_allclose(av, want["shat"][emit], atol=1e-6, rtol=0)
    assert int((res.code == 0xEE).sum().item()) == n_cand - len(idx)   # nothing else written



def test_tiles_member_ids_past_two_to_the_24(ctx):
    """An index of 2^24 + 300 objects (128-bit rows): the tile kernel reads
    rows through 32-bit buffer offsets only while n_obj <= 2^24 and the rows
    fit 4 GiB, else through 64-bit addresses.  Tiles mixing members below and
    above 2^24 take the second way; the same tiles over an index of the low
    objects only take the first; both equal the oracle."""
    rng = np.random.default_rng(12)
    n_small, n_max, k = 600, 128, 32
    sig = G.pack_bits(G.calibration_bits(n_small // 2, n_max, rng.uniform(0.6, 1.0, n_small // 2), 121))
    lo, hi = np.arange(300), np.arange(300, 600)
    big = (1 << 24) + 300
    ids = np.concatenate([lo, hi - 300 + (1 << 24)]).astype(np.uint32)   # object i of sig at ids[i]
    words = torch.zeros(big * 4, dtype=torch.int32, device="cuda")
    words.view(big, 4)[torch.from_numpy(ids.astype(np.int64)).cuda()] = torch.from_numpy(sig.view(np.int32)).cuda()
    S_big = P.Signatures(words.view(torch.uint32), P.COSINE, P.OBJECT_MAJOR, big, n_max)
    tiles, xs, ys, first = [], [], [], 0
    for _ in range(40):
        rows = rng.choice(n_small, 16, replace=False)
        cols = rng.choice(n_small, 16, replace=False)
        pos = [q for q in range(256) if rng.random() < 0.8]
        tiles.append(_tile(first, ids[rows], ids[cols], pos))
        xs += [rows[q // 16] for q in pos]
        ys += [cols[q % 16] for q in pos]
        first += len(pos)
    x, y = np.array(xs, np.uint32), np.array(ys, np.uint32)
    want = R.verify(x, y, P.COSINE, sig, k, n_max // k, 0.7, EPS, DELTA, GAMMA)
    res = P.make_result(first, first, m_debug=True)
    P.bayeslsh_verify(ctx, P.tiles(up(np.stack(tiles).reshape(-1)), len(tiles), first), S_big, 0.7, EPS, DELTA,
                      GAMMA, (1, 1), k, res)
    P.bayeslsh_sync(ctx)
    assert_same_as_oracle(decode_result(res, first), want)
    # the low half alone, as an index of 300 objects (buffer offsets)
    low_tiles, lx, ly, first = [], [], [], 0
    for _ in range(40):
        rows = rng.choice(300, 16, replace=False)
        cols = rng.choice(300, 16, replace=False)
        pos = [q for q in range(256) if rng.random() < 0.8]
        low_tiles.append(_tile(first, ids[rows], ids[cols], pos))
        lx += [rows[q // 16] for q in pos]
        ly += [cols[q % 16] for q in pos]
        first += len(pos)
    S_low = sigs_tensor(sig[:300], P.COSINE, P.OBJECT_MAJOR)
    want = R.verify(np.array(lx, np.uint32), np.array(ly, np.uint32), P.COSINE, sig, k, n_max // k, 0.7, EPS, DELTA,
                    GAMMA)
    res = P.make_result(first, first, m_debug=True)
    P.bayeslsh_verify(ctx, P.tiles(up(np.stack(low_tiles).reshape(-1)), len(low_tiles), first), S_low, 0.7, EPS,
                      DELTA, GAMMA, (1, 1), k, res)
    P.bayeslsh_sync(ctx)
    assert_same_as_oracle(decode_result(res, first), want)
    del words

def test_tiles_rejected_where_unsupported(ctx, mix, banded):
    band = banded[0]
    tl, nt, npairs = band_tiles(ctx, sigs_tensor(band, P.COSINE, P.OBJECT_MAJOR), 16, 6)
    cand = P.tiles(tl, nt, npairs)
    res = P.make_result(npairs, 16)
    sig = _bits(mix, 256, 5)
    for S in (sigs_tensor(sig, P.COSINE, P.WORD_MAJOR), sigs_tensor(_bits(mix, 96, 6), P.COSINE, P.OBJECT_MAJOR),
              sigs_tensor(np.zeros((3000, 64), np.uint32), P.JACCARD, P.OBJECT_MAJOR)):
        with pytest.raises(P.BayesLSHError) as e:
            P.bayeslsh_verify(ctx, cand, S, 0.7, EPS, DELTA, GAMMA, (1, 1), 32, res)
        assert e.value.code == -1
    S = sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR)
    with pytest.raises(P.BayesLSHError):   # Lite over tiles: h a multiple of 128
        P.bayeslsh_lite_verify(ctx, cand, S, P.dense_vectors(up(mix.x)), 0.7, EPS, (1, 1), 64, 32, res)
    with pytest.raises(P.BayesLSHError):
        P.bayeslsh_exhaustive_verify(ctx, cand, S, None, 0.7, EPS, DELTA, GAMMA, (1, 1), 32, 0, P.REPLAY, res)
    with pytest.raises(P.BayesLSHError):
        P.bayeslsh_verify_noalloc(ctx, cand, S, 0.7, EPS, DELTA, GAMMA, (1, 1), 32, res)
    with pytest.raises(P.BayesLSHError):    # tiles must be 16-byte aligned
        P.bayeslsh_verify(ctx, P.tiles(tl.view(torch.int32)[1:], nt, npairs), S, 0.7, EPS, DELTA, GAMMA, (1, 1), 32,
                          res)


@pytest.mark.parametrize("k,h,t", [(32, 128, 0.7), (16, 256, 0.8), (64, 512, 0.7)])
def test_tiles_lite_matches_oracle(ctx, mix, banded, k, h, t):
    """Algorithm 2 (BayesLSH-Lite) over the tiles: prune tests on the first h
    hashes, then the exact cosine of the mixture rows for the survivors,
    emitted iff s > t: the oracle's decisions, levels, m and exact values on
    the oracle's banding pairs, and the PAIRS Lite path's output."""
    print("tiles lite k=%d h=%d t=%.1f" % (k, h, t), flush=True)
    band, (wx, wy) = banded
    sig = _bits(mix, 1024, G.SEED_BASE + 65)
    tl, nt, npairs = band_tiles(ctx, sigs_tensor(band, P.COSINE, P.OBJECT_MAJOR), 16, 6)
    want = R.verify(wx, wy, P.COSINE, sig, k, h // k, t, EPS, 0, 0, lite=True)
    exact_fn = lambda a_, b_: R.exact_cosine_dense(mix.x, a_, b_)
    want = R.lite_finish(want, exact_fn, wx, wy, t)
    assert {0, 3} <= set(want["decision"].tolist())
    S = sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR)
    vec = P.dense_vectors(up(mix.x))
    res = P.make_result(npairs, npairs, m_debug=True)
    P.bayeslsh_lite_verify(ctx, P.tiles(tl, nt, npairs), S, vec, t, EPS, (1, 1), h, k, res)
    P.bayeslsh_sync(ctx)
    got = decode_result(res, npairs)
    assert_same_as_oracle(got, want, lite_exact=want["exact"])
    assert got["n_accepted"] > 10
    res_p = P.make_result(npairs, npairs, m_debug=True)
    P.bayeslsh_lite_verify(ctx, P.pairs(up(wx), up(wy)), S, vec, t, EPS, (1, 1), h, k, res_p)
    P.bayeslsh_sync(ctx)
    gp = decode_result(res_p, npairs)
    np.testing.assert_array_equal(got["code"], gp["code"])
    np.testing.assert_array_equal(got["acc_idx"], gp["acc_idx"])
    np.testing.assert_array_equal(got["acc_val"], gp["acc_val"])
    # the same call in launches of 7 tiles
    P.bayeslsh_set_tuning(ctx, tiles_per_launch=7)
    try:
        res_m = P.make_result(npairs, npairs, m_debug=True)
        P.bayeslsh_lite_verify(ctx, P.tiles(tl, nt, npairs), S, vec, t, EPS, (1, 1), h, k, res_m)
        P.bayeslsh_sync(ctx)
    finally:
        P.bayeslsh_set_tuning(ctx)
    assert nt > 14
    gm = decode_result(res_m, npairs)
    for key in ("code", "m", "acc_idx", "acc_val"):
        np.testing.assert_array_equal(gm[key], got[key])


@pytest.mark.parametrize("k", [32, 64])
def test_tiles_level0_accept_before_level1_prune(ctx, k):
    """The tile kernel decides levels 0 and 1 in its first pass.  A pair that
    agrees on every hash of level 0 is accepted there (the table concentrates
    at m = n = k) even when it disagrees on every hash of level 1, which would
    prune it at level 1 had level 0 not ended its loop (Algorithm 1 tests
    acceptance before going on).  One tile: row 0 an all-zero object, columns
    objects with chosen disagreement counts in levels 0 and 1: the oracle's
    decisions, levels and m."""
    n_max, t = 512, 0.8
    words = n_max // 32
    rng = np.random.default_rng(17)
    combos = [(0, k), (0, k), (0, k // 2), (1, k), (2, k), (k // 4, k), (0, 0), (3, 0), (k // 2, 0), (1, 1),
              (0, k - 1), (k - 1, k), (5, 5), (0, 3), (2, k - 2)]
    sig = np.zeros((len(combos) + 1, words), np.uint32)
    for j, (d0, d1) in enumerate(combos, start=1):
        bits = np.zeros(n_max, np.uint8)
        bits[rng.choice(k, d0, replace=False)] = 1            # level 0 disagreements
        bits[k + rng.choice(k, d1, replace=False)] = 1        # level 1 disagreements
        bits[2 * k:] = rng.integers(0, 2, n_max - 2 * k) * (rng.random(n_max - 2 * k) < 0.1)
        sig[j] = G.pack_bits(bits[None, :])[0]
    m_cols = len(combos)
    tile = _tile(0, np.array([0], np.uint32), np.arange(1, m_cols + 1, dtype=np.uint32), list(range(m_cols)))
    x = np.zeros(m_cols, np.uint32)
    y = np.arange(1, m_cols + 1, dtype=np.uint32)
    want = R.verify(x, y, P.COSINE, sig, k, n_max // k, t, EPS, DELTA, GAMMA)
    # the case under test is there: accepted at level 0 with level 1 all disagreeing
    assert want["decision"][0] == 1 and want["level"][0] == 0
    S = sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR)
    res = P.make_result(m_cols, m_cols, m_debug=True)
    P.bayeslsh_verify(ctx, P.tiles(up(tile), 1, m_cols), S, t, EPS, DELTA, GAMMA, (1, 1), k, res)
    P.bayeslsh_sync(ctx)
    assert_same_as_oracle(decode_result(res, m_cols), want)
