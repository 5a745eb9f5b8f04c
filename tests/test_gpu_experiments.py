"""The experiment analogs (pruning curve, gamma/delta/epsilon sweep, LSH
Approx, BayesLSH vs Lite by threshold) against the same statistics worked out
from the oracle's decisions on the same signatures and exact similarities.

Decisions are bit-exact, so every count (positives, accepted, recall) must
match exactly and every error statistic within 1e-6."""
import numpy as np
import pytest
import torch

import paper_1110_1328_amd as P
from paper_1110_1328_amd import experiments as E
from oracle import reference as R
from synth import generators as G

from gpu_util import csr_device, sigs_tensor, up

pytestmark = pytest.mark.gpu
K, NB, H = 32, 512, 128


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    c = P.bayeslsh_create(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def setup():
    corpus = G.tfidf_corpus(n_docs=2500, dim=1 << 16, mean_nnz=40, dup_frac=0.2, seed=G.SEED_BASE + 71)
    x, y = G.sparse_band_candidates(corpus, n_bands=12, band_bits=5, seed=G.SEED_BASE + 72)
    proj = R.srp_sparse_projections(corpus.offsets, corpus.indices, corpus.values, NB, 9,
                                    np.arange(corpus.n, dtype=np.int64))
    sig = R.bits_from_projections(proj)
    truth = R.exact_cosine_csr(corpus.offsets, corpus.indices, corpus.values, x, y)
    return corpus, x, y, sig, truth


def oracle_quality(accepted, values, truth, t, bound=0.05):
    pos = truth >= t
    acc = np.flatnonzero(accepted)
    err = np.abs(values[acc].astype(np.float32).astype(np.float64) - truth[acc])
    return dict(positives=int(pos.sum()), accepted=len(acc), accepted_positives=int((pos & accepted).sum()),
                mean_error=float(err.mean()) if len(acc) else 0.0, max_error=float(err.max()) if len(acc) else 0.0,
                frac_error_gt=float((err > bound).mean()) if len(acc) else 0.0)


def same(got, want):
    for key in ("positives", "accepted", "accepted_positives"):
        assert got[key] == want[key], (key, got[key], want[key])
    for key in ("mean_error", "max_error", "frac_error_gt"):
        assert abs(got[key] - want[key]) <= 1e-6, (key, got[key], want[key])


def test_truth_and_pruning_curve(ctx, setup):
    corpus, x, y, sig, truth = setup
    print("experiments: truth and pruning curve, %d candidates" % len(x), flush=True)
    cand = P.pairs(up(x), up(y))
    t_gpu, _ = E.exact_truth(ctx, cand, csr_device(corpus))
    np.testing.assert_allclose(t_gpu.cpu().numpy(), truth, atol=1e-6, rtol=0)
    res = P.make_result(len(x), len(x))
    P.bayeslsh_verify(ctx, cand, sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR), 0.7, 0.03, 0.05, 0.03, (1, 1), K, res)
    P.bayeslsh_sync(ctx)
    want = R.verify(x, y, P.COSINE, sig, K, NB // K, 0.7, 0.03, 0.05, 0.03)
    curve = E.pruning_curve(res.code[:len(x)], K, NB // K)
    lv = want["level"]
    for j, (nh, frac) in enumerate(curve):
        assert nh == (j + 1) * K
        assert abs(frac - np.mean(lv > j)) < 1e-12
    assert curve[-1][1] == 0.0


def test_parameter_sweep_matches_oracle(ctx, setup):
    corpus, x, y, sig, truth = setup
    print("experiments: parameter sweep", flush=True)
    cand = P.pairs(up(x), up(y))
    S = sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR)
    truth_d = torch.from_numpy(truth).cuda()
    rows = E.parameter_sweep(ctx, cand, S, truth_d, 0.7, K, values=(0.01, 0.09), steps=1)
    assert [(r["vary"], r["value"]) for r in rows] == [(w, v) for w in ("gamma", "delta", "epsilon")
                                                       for v in (0.01, 0.09)]
    for r in rows:
        want = R.verify(x, y, P.COSINE, sig, K, NB // K, 0.7, r["epsilon"], r["delta"], r["gamma"])
        acc = (want["decision"] == R.DEC_CONC) | (want["decision"] == R.DEC_NMAX)
        same(r, oracle_quality(acc, want["shat"], truth, 0.7))
        assert r["recall"] == (r["accepted_positives"] / r["positives"])


def test_lsh_approx_and_thresholds_match_oracle(ctx, setup):
    corpus, x, y, sig, truth = setup
    print("experiments: LSH Approx and thresholds", flush=True)
    cand = P.pairs(up(x), up(y))
    S = sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR)
    truth_d = torch.from_numpy(truth).cuda()
    a = E.lsh_approx(ctx, cand, S, truth_d, 0.7, K, steps=1)
    m = R.mle(x, y, P.COSINE, sig, NB, 0.7)
    same(a, oracle_quality(m["accepted"], m["shat"], truth, 0.7))
    S_pf = sigs_tensor(np.ascontiguousarray(sig[:, : H // 32]), P.COSINE, P.OBJECT_MAJOR)
    rows = E.threshold_sweep(ctx, cand, S, S_pf, csr_device(corpus), truth_d, (0.5, 0.8), K, H, steps=1)
    for r in rows:
        t = r["t"]
        wb = R.verify(x, y, P.COSINE, sig, K, NB // K, t, 0.03, 0.05, 0.03)
        accb = (wb["decision"] == R.DEC_CONC) | (wb["decision"] == R.DEC_NMAX)
        qb = oracle_quality(accb, wb["shat"], truth, t)
        assert r["bayeslsh_accepted"] == qb["accepted"] and r["positives"] == qb["positives"]
        assert abs(r["bayeslsh_recall"] - qb["accepted_positives"] / qb["positives"]) < 1e-12
        wl = R.lite_finish(R.verify(x, y, P.COSINE, sig, K, H // K, t, 0.03, 0, 0, lite=True),
                           lambda p, q: R.exact_cosine_csr(corpus.offsets, corpus.indices, corpus.values, p, q),
                           x, y, t)
        ql = oracle_quality(wl["accepted"], np.nan_to_num(wl["exact"]), truth, t)
        assert r["lite_accepted"] == ql["accepted"]
        assert abs(r["lite_recall"] - ql["accepted_positives"] / ql["positives"]) < 1e-12
