"""GPU parity of sparse SRP with 2-byte plane entries (Section 4.3,
BLSH_SRP_PLANES_Q16) against the oracle's projection over the same entries
read back from their codes, in FP64, under the sign-flip rule: a bit may
differ only where the FP64 projection is within summation-order rounding of
0.  The table path (terms repeat) and the per-nonzero path give identical
bits, and the bits differ from the fp32-entry ones only where the projection
is within sum |x_i| 2^-13 of 0."""
import numpy as np
import pytest
import torch

import paper_1110_1328_amd as P
from oracle import reference as R
from synth import generators as G

from gpu_util import csr_device, down, up

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = P.bayeslsh_create(0)
    yield c
    c.close()


def _bits(ctx, vec, n, n_bits, seed, layout, flags):
    W = n_bits // 32
    out = torch.empty(n * W, dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_srp_sigs(ctx, vec, None, n_bits, seed, layout, out, flags=flags)
    P.bayeslsh_sync(ctx)
    got = down(out).reshape((W, n) if layout == P.WORD_MAJOR else (n, W))
    return got.T.copy() if layout == P.WORD_MAJOR else got


def _flips(a, b, n, n_bits):
    return np.unpackbits((a ^ b).view(np.uint8), bitorder="little").reshape(n, n_bits).astype(bool)


@pytest.mark.parametrize("n_bits,layout,table", [(2048, P.WORD_MAJOR, False), (256, P.OBJECT_MAJOR, False),
                                                 (2048, P.OBJECT_MAJOR, True), (96, P.WORD_MAJOR, True)])
def test_sparse_srp_q16_flip_rule(ctx, n_bits, layout, table):
    print("srp q16: %d bits layout %d table %s" % (n_bits, layout, table), flush=True)
    if table:   # more nonzeros than twice the dimension: the codes are drawn once per term into a table
        corpus = G.tfidf_corpus(n_docs=1500, dim=1 << 12, mean_nnz=40, seed=G.SEED_BASE + 24)
        assert len(corpus.indices) > 2 * corpus.dim
    else:
        corpus = G.tfidf_corpus(n_docs=300, dim=1 << 20, seed=G.SEED_BASE + 25)
        assert len(corpus.indices) <= 2 * corpus.dim
    seed = 0x5151_2626_3737
    n = corpus.n
    got = _bits(ctx, csr_device(corpus), n, n_bits, seed, layout, P.SRP_PLANES_Q16)
    rows = np.arange(n, dtype=np.int64)
    projq = R.srp_sparse_projections(corpus.offsets, corpus.indices, corpus.values, n_bits, seed, rows, q16=True)
    diff = _flips(got, R.bits_from_projections(projq), n, n_bits)
    assert np.all(np.abs(projq[diff]) < 1e-5), np.abs(projq[diff]).max()
    assert diff.sum() <= max(1, 1e-6 * diff.size)
    # the same CSR data declared with a dimension too large for a table: codes drawn per nonzero
    off, idx, val = up(corpus.offsets), up(corpus.indices.astype(np.uint32)), up(corpus.values)
    other = _bits(ctx, P.csr_vectors(off, idx, val, 1 << 40), n, n_bits, seed, layout, P.SRP_PLANES_Q16)
    np.testing.assert_array_equal(got, other)
    # against the fp32-entry signatures: flips only within the storage error bound
    full = _bits(ctx, csr_device(corpus), n, n_bits, seed, layout, 0)
    proj = R.srp_sparse_projections(corpus.offsets, corpus.indices, corpus.values, n_bits, seed, rows)
    l1 = np.array([np.abs(corpus.row(r)[1].astype(np.float64)).sum() for r in rows])
    d2 = _flips(got, full, n, n_bits)
    bound = np.broadcast_to(l1[:, None] * 2.0 ** -13 + 1e-5, proj.shape)
    assert np.all(np.abs(proj[d2]) <= bound[d2])


def test_q16_flag_rejected(ctx):
    corpus = G.tfidf_corpus(n_docs=20, dim=1 << 12, mean_nnz=10, seed=G.SEED_BASE + 26)
    out = torch.empty(corpus.n * 4, dtype=torch.int32, device="cuda").view(torch.uint32)
    with pytest.raises(P.BayesLSHError) as e:
        P.bayeslsh_srp_sigs(ctx, csr_device(corpus), None, 128, 1, P.OBJECT_MAJOR, out, flags=2)
    assert e.value.code == -1
    x = torch.randn(64, 64, device="cuda")
    planes = torch.randn(64, 64, device="cuda")
    out_d = torch.empty(64 * 2, dtype=torch.int32, device="cuda").view(torch.uint32)
    with pytest.raises(P.BayesLSHError) as e:
        P.bayeslsh_srp_sigs(ctx, P.dense_vectors(x), planes, 64, 0, P.OBJECT_MAJOR, out_d, flags=P.SRP_PLANES_Q16)
    assert e.value.code == -1
