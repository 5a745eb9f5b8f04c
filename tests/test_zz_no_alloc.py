"""The allocation-free entry point (bayeslsh_verify_noalloc) against
bayeslsh_verify through the C ABI: the same codes, match counts, accepted set
and S_hat on two calls in a row, the second smaller than the first (the
library's scratch array keeps the first call's contents), for the SRP prefix +
tail path (survivor queue and staging), SRP word-major slabs (staging only) and
minhash; then a call with another threshold (a new table image)."""
import numpy as np
import pytest
import torch

import paper_1110_1328_amd as P
from synth import generators as G

from gpu_util import decode_result, up

pytestmark = pytest.mark.gpu

EPS, DELTA, GAMMA = 0.03, 0.05, 0.03


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    c = P.bayeslsh_create(0)
    yield c
    c.close()


def _pairs(n_obj, n, seed):
    """Planted pairs (2i, 2i + 1) among uniform random pairs, in random order."""
    rng = np.random.default_rng(seed)
    planted = rng.integers(0, n_obj // 2, n // 8)
    x = np.concatenate([2 * planted, rng.integers(0, n_obj, n - len(planted))]).astype(np.uint32)
    y = np.concatenate([2 * planted + 1, rng.integers(0, n_obj, n - len(planted))]).astype(np.uint32)
    o = rng.permutation(n)
    return x[o], y[o]


def _same(ctx, cand, S, t, k, n):
    ref = P.make_result(n, n, m_debug=True)
    got = P.make_result(n, n, m_debug=True)
    got.code.fill_(0xEE)
    got.n_accepted.fill_(-7)
    P.bayeslsh_verify(ctx, cand, S, t, EPS, DELTA, GAMMA, (1, 1), k, ref)
    P.bayeslsh_sync(ctx)
    P.bayeslsh_verify_noalloc(ctx, cand, S, t, EPS, DELTA, GAMMA, (1, 1), k, got)
    P.bayeslsh_sync(ctx)
    a, b = decode_result(ref, n), decode_result(got, n)
    np.testing.assert_array_equal(b["code"], a["code"])
    np.testing.assert_array_equal(b["m"], a["m"])
    assert b["n_accepted"] == a["n_accepted"] > 0
    np.testing.assert_array_equal(b["acc_idx"], a["acc_idx"])
    np.testing.assert_array_equal(b["acc_val"], a["acc_val"])
    return a


@pytest.mark.parametrize("case", ["srp_prefix_tail", "srp_word_major", "minhash"])
def test_noalloc_equals_verify_on_consecutive_calls(ctx, case):
    print("no-alloc: %s" % case, flush=True)
    n_pairs_obj = 20_000
    rng = np.random.default_rng(3)
    if case == "minhash":
        n_hashes, k = 256, 32
        s = rng.uniform(0.0, 1.0, n_pairs_obj)
        sig = G.calibration_minhash(n_pairs_obj, n_hashes, s, 31)
        S = P.Signatures(up(sig.reshape(-1)), P.JACCARD, P.OBJECT_MAJOR, sig.shape[0], n_hashes)
        t = 0.7
    else:
        n_hashes, k = 1024, 32
        s = rng.uniform(0.5, 1.0, n_pairs_obj)
        sig = G.pack_bits(G.calibration_bits(n_pairs_obj, n_hashes, s, 32))
        if case == "srp_prefix_tail":
            S = P.Signatures(up(sig.reshape(-1)), P.COSINE, P.OBJECT_MAJOR, sig.shape[0], n_hashes,
                             prefix=up(np.ascontiguousarray(sig[:, :4]).reshape(-1)))
        else:
            S = P.Signatures(up(np.ascontiguousarray(sig.T).reshape(-1)), P.COSINE, P.WORD_MAJOR, sig.shape[0],
                             n_hashes)
        t = 0.8
    n_obj = sig.shape[0]
    # first call: more than two launches of the scratch's 2^20 candidates;
    # second: a smaller input after it
    for n, seed in (((1 << 21) + 12345, 5), (50_001, 6)):
        x, y = _pairs(n_obj, n, seed)
        out = _same(ctx, P.pairs(up(x), up(y)), S, t, k, n)
        assert len(set(out["decision"].tolist())) == 3
    # another threshold: the table image in the scratch array is replaced
    x, y = _pairs(n_obj, 70_000, 7)
    _same(ctx, P.pairs(up(x), up(y)), S, t - 0.1, k, 70_000)


def test_noalloc_empty_and_invalid(ctx):
    sig = np.zeros((8, 32), np.uint32)
    S = P.Signatures(up(sig.reshape(-1)), P.COSINE, P.OBJECT_MAJOR, 8, 1024)
    res = P.make_result(1, 1)
    res.n_accepted.fill_(5)
    e = up(np.zeros(0, np.uint32))
    P.bayeslsh_verify_noalloc(ctx, P.pairs(e, e), S, 0.8, EPS, DELTA, GAMMA, (1, 1), 32, res)
    P.bayeslsh_sync(ctx)
    assert int(res.n_accepted.item()) == 0
    with pytest.raises(P.BayesLSHError) as err:
        P.bayeslsh_verify_noalloc(ctx, P.pairs(e, e), S, 0.8, EPS, DELTA, GAMMA, (1, 1), 24, res)
    assert err.value.code == -1
