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


def expand(members, tiles_i64, n_tiles):
    """Host expansion of tile descriptors into (x, y) in candidate order; also
    checks that each tile numbers its candidates right after the previous one."""
    d = tiles_i64[: n_tiles * 8].reshape(n_tiles, 8)
    first, row0, col0 = d[:, 0], d[:, 1], d[:, 2]
    n_rows = (d[:, 3] & 0xFFFFFFFF).astype(np.int64)
    n_cols = ((d[:, 3] >> 32) & 0xFFFFFFFF).astype(np.int64)
    keep = d[:, 4:8].view(np.uint64)
    bits = np.unpackbits(keep.view(np.uint8).reshape(n_tiles, 32), axis=1, bitorder="little").astype(bool)
    counts = bits.sum(axis=1)
    assert np.array_equal(first, np.concatenate([[0], np.cumsum(counts)[:-1]]))
    assert np.all((n_rows >= 1) & (n_rows <= 16) & (n_cols >= 1) & (n_cols <= 16))
    t_idx, p = np.nonzero(bits)
    r, c = p // 16, p % 16
    assert np.all(r < n_rows[t_idx]) and np.all(c < n_cols[t_idx])
    return members[row0[t_idx] + r], members[col0[t_idx] + c]


def band_tiles(ctx, S, nb, b, max_bucket=0, cap=1 << 16):
    mem, tl, nt, npairs, trunc = P.bayeslsh_band_tiles(ctx, S, nb, b, cap, max_bucket=max_bucket)
    assert not trunc
    return mem, tl, nt, npairs


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
        mem, tl, nt, npairs = band_tiles(ctx, sigs_tensor(bits, P.COSINE, layout), nb, b, max_bucket)
        assert npairs == len(wx)
        gx, gy = expand(down(mem), tl.cpu().numpy(), nt)
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
    kernel (n_max / 128 = 1 .. 16 lanes) and every k: the oracle's output on
    the oracle's banding pairs, and the PAIRS path's output."""
    print("tiles verify k=%d n_max=%d t=%.1f" % (k, n_max, t), flush=True)
    band, (wx, wy) = banded
    sig = _bits(mix, n_max, G.SEED_BASE + 64 + n_max)
    mem, tl, nt, npairs = band_tiles(ctx, sigs_tensor(band, P.COSINE, P.OBJECT_MAJOR), 16, 6)
    assert npairs == len(wx)
    want = R.verify(wx, wy, P.COSINE, sig, k, n_max // k, t, EPS, DELTA, GAMMA)
    # pruned and concentrated everywhere; accepted at n_max too except where
    # every pair concentrates first (2048 hashes; t = 0.9)
    assert {0, 1} <= set(want["decision"].tolist())
    S = sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR)
    res = P.make_result(npairs, npairs, m_debug=True)
    P.bayeslsh_verify(ctx, P.tiles(mem, tl, nt, npairs), S, t, EPS, DELTA, GAMMA, (1, 1), k, res)
    P.bayeslsh_sync(ctx)
    got = decode_result(res, npairs)
    assert_same_as_oracle(got, want)
    res_p = P.make_result(npairs, npairs, m_debug=True)
    P.bayeslsh_verify(ctx, P.pairs(up(wx), up(wy)), S, t, EPS, DELTA, GAMMA, (1, 1), k, res_p)
    P.bayeslsh_sync(ctx)
    gp = decode_result(res_p, npairs)
    np.testing.assert_array_equal(got["code"], gp["code"])
    np.testing.assert_array_equal(got["acc_val"], gp["acc_val"])


def _tile(first, row0, col0, n_rows, n_cols, positions):
    keep = np.zeros(4, np.uint64)
    for p_ in positions:
        keep[p_ // 64] |= np.uint64(1) << np.uint64(p_ % 64)
    return np.array([first, row0, col0, n_rows | (n_cols << 32)] + list(keep.view(np.int64)), np.int64)


def test_tiles_by_hand_and_malformed(ctx):
    """Hand-made tiles: partial rows and columns, sparse keep masks, several
    launches' worth of tiles; then a member id >= n_obj (code 0xFF,
    BLSH_EBADID), a position past the members array and numbering past n_cand
    (BLSH_EINVAL), an empty tile list."""
    rng = np.random.default_rng(8)
    n_obj, n_max, k = 500, 256, 32
    sig = G.pack_bits(G.calibration_bits(n_obj // 2, n_max, rng.uniform(0.6, 1.0, n_obj // 2), 81))
    members = rng.permutation(n_obj).astype(np.uint32)
    tiles, xs, ys, first = [], [], [], 0
    for _ in range(700):
        nr, nc = int(rng.integers(1, 17)), int(rng.integers(1, 17))
        r0, c0 = int(rng.integers(0, n_obj - 16)), int(rng.integers(0, n_obj - 16))
        pos = sorted(int(16 * r + c) for r in range(nr) for c in range(nc) if rng.random() < 0.7)
        if not pos:
            continue
        tiles.append(_tile(first, r0, c0, nr, nc, pos))
        xs += [members[r0 + q // 16] for q in pos]
        ys += [members[c0 + q % 16] for q in pos]
        first += len(pos)
    x, y = np.array(xs, np.uint32), np.array(ys, np.uint32)
    S = sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR)
    want = R.verify(x, y, P.COSINE, sig, k, n_max // k, 0.7, EPS, DELTA, GAMMA)
    tl = up(np.stack(tiles))
    mem = up(members)
    res = P.make_result(first, first, m_debug=True)
    P.bayeslsh_verify(ctx, P.tiles(mem, tl.view(-1), len(tiles), first), S, 0.7, EPS, DELTA, GAMMA, (1, 1), k, res)
    P.bayeslsh_sync(ctx)
    assert_same_as_oracle(decode_result(res, first), want)

    def run_one(tile, members_arr, n_cand):
        r = P.make_result(max(n_cand, 1), 16)
        r.code.fill_(0xEE)
        P.bayeslsh_verify(ctx, P.tiles(up(members_arr), up(tile[None, :]).view(-1), 1, n_cand), S, 0.7, EPS, DELTA,
                          GAMMA, (1, 1), k, r)
        with pytest.raises(P.BayesLSHError) as e:
            P.bayeslsh_sync(ctx)
        return e.value.code, r.code[:n_cand].cpu().numpy()

    bad_mem = members.copy()
    bad_mem[3] = n_obj + 5                                   # row member 3 is a bad id
    code, got = run_one(_tile(0, 0, 8, 4, 4, [16 * r + c for r in range(4) for c in range(4)]), bad_mem, 16)
    assert code == -5 and np.all(got[12:16] == 0xFF) and np.all(got[:12] != 0xFF)   # BLSH_EBADID
    code, got = run_one(_tile(0, n_obj - 2, 0, 4, 4, [0, 1, 16, 17, 32]), members, 5)   # rows past members[]
    assert code == -1 and got[4] == 0xFF and np.all(got[:4] != 0xFF)
    code, got = run_one(_tile(0, 0, 8, 2, 2, [0, 1, 16, 17, 34]), members, 5)           # position past n_rows
    assert code == -1 and got[4] == 0xFF
    code, got = run_one(_tile(3, 0, 8, 2, 2, [0, 1, 16, 17]), members, 5)               # numbering past n_cand
    assert code == -1 and np.all(got[3:5] != 0xEE) and np.all(got[:3] == 0xEE)
    r = P.make_result(1, 1)
    r.n_accepted.fill_(9)
    P.bayeslsh_verify(ctx, P.tiles(mem, tl.view(-1), 0, 0), S, 0.7, EPS, DELTA, GAMMA, (1, 1), k, r)
    P.bayeslsh_sync(ctx)
    assert int(r.n_accepted.item()) == 0


def test_tiles_rejected_where_unsupported(ctx, mix, banded):
    band = banded[0]
    mem, tl, nt, npairs = band_tiles(ctx, sigs_tensor(band, P.COSINE, P.OBJECT_MAJOR), 16, 6)
    cand = P.tiles(mem, tl, nt, npairs)
    res = P.make_result(npairs, 16)
    sig = _bits(mix, 256, 5)
    for S in (sigs_tensor(sig, P.COSINE, P.WORD_MAJOR), sigs_tensor(_bits(mix, 96, 6), P.COSINE, P.OBJECT_MAJOR),
              sigs_tensor(np.zeros((3000, 64), np.uint32), P.JACCARD, P.OBJECT_MAJOR)):
        with pytest.raises(P.BayesLSHError) as e:
            P.bayeslsh_verify(ctx, cand, S, 0.7, EPS, DELTA, GAMMA, (1, 1), 32, res)
        assert e.value.code == -1
    S = sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR)
    with pytest.raises(P.BayesLSHError):
        P.bayeslsh_lite_verify(ctx, cand, S, P.dense_vectors(up(mix.x)), 0.7, EPS, (1, 1), 128, 32, res)
    with pytest.raises(P.BayesLSHError):
        P.bayeslsh_verify_noalloc(ctx, cand, S, 0.7, EPS, DELTA, GAMMA, (1, 1), 32, res)
    with pytest.raises(P.BayesLSHError):    # members buffer smaller than n_bands * n_obj
        P.bayeslsh_band_tiles(ctx, sigs_tensor(band, P.COSINE, P.OBJECT_MAJOR), 16, 6, 16,
                              members_out=mem[:100])
