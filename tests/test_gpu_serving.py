"""GPU tests of the serving loop (bayeslsh_server_*): continuous batching with
memory admission.  Each request's output must equal the oracle's, and be the
same whether the request runs alone or mixed with others."""
import time

import numpy as np
import pytest
import torch

import paper_1110_1328_amd as P
from oracle import reference as R
from synth import generators as G

from gpu_util import sigs_tensor, up

pytestmark = pytest.mark.gpu
EPS, DELTA, GAMMA = 0.03, 0.05, 0.03


@pytest.fixture(scope="module")
def index():
    rng = np.random.default_rng(99)
    n = 20000
    sig = G.pack_bits(G.calibration_bits(n // 2, 1024, rng.uniform(0.5, 1.0, n // 2), 98))
    return sig


def make_requests(n_obj, n_req, seed, lo=1, hi=4.0):
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n_req):
        q = int(rng.integers(0, n_obj))
        L = int(10 ** rng.uniform(lo, hi))
        c = rng.integers(0, n_obj, L).astype(np.uint32)
        c[: max(1, L // 100)] = q ^ 1
        reqs.append((q, np.sort(c), float(rng.choice([0.6, 0.8]))))
    return reqs


def oracle_request(sig, q, c, t, k=32):
    r = R.verify(np.full(len(c), q, np.uint32), c, 1, sig, k, 1024 // k, t, EPS, DELTA, GAMMA)
    acc = np.flatnonzero((r["decision"] == 1) | (r["decision"] == 2))
    return acc, r["shat"][acc]


def test_serving_alone_equals_mixed_and_oracle(index):
    print("serving alone vs mixed", flush=True)
    ctx = P.bayeslsh_create(0)
    S = sigs_tensor(index, P.COSINE, P.WORD_MAJOR)
    srv = P.Server(ctx, S, mem_budget_bytes=4 << 20, max_active=4, k=32, max_batch_candidates=1 << 16)
    try:
        reqs = make_requests(index.shape[0], 60, 5)
        alone = []
        for q, c, t in reqs:
            rid = srv.submit(q, c, t)
            alone.append(srv.wait(rid))
            srv.release(rid)
        # mixed: everything at once (admission limited by slots and the 4 MB arena)
        ids = [srv.submit(q, c, t) for q, c, t in reqs]
        mixed = [srv.wait(r) for r in ids]
        for a, b, (q, c, t) in zip(alone, mixed, reqs):
            np.testing.assert_array_equal(a["acc_idx"], b["acc_idx"])
            np.testing.assert_array_equal(a["acc_val"], b["acc_val"])
            acc, sh = oracle_request(index, q, c, t)
            np.testing.assert_array_equal(b["acc_idx"], acc)
            np.testing.assert_allclose(b["acc_val"], sh, atol=1e-6)
            assert b["done"] >= b["admit"] >= b["submit"]
        assert srv.stats()["deferred"] > 0     # admission made some requests wait
        assert sum(len(a["acc_idx"]) for a in alone) > 0
    finally:
        srv.close()
        ctx.close()


def test_serving_poisson_arrivals_and_limits(index):
    print("serving poisson", flush=True)
    ctx = P.bayeslsh_create(0)
    S = sigs_tensor(index, P.COSINE, P.WORD_MAJOR)
    srv = P.Server(ctx, S, mem_budget_bytes=1 << 20, max_active=8, k=32, max_batch_candidates=1 << 15)
    try:
        reqs = make_requests(index.shape[0], 40, 6, lo=1, hi=5.2)   # some exceed 256k candidates = 1 MB
        rng = np.random.default_rng(1)
        gaps = rng.exponential(0.002, len(reqs))
        ids, big = [], 0
        for (q, c, t), g in zip(reqs, gaps):
            time.sleep(g)
            if len(c) * 4 > (1 << 20):
                with pytest.raises(P.BayesLSHError) as e:
                    srv.submit(q, c, t)
                assert e.value.code == -2
                big += 1
                continue
            ids.append((srv.submit(q, c, t), q, c, t))
        for rid, q, c, t in ids:
            res = srv.wait(rid)
            acc, _ = oracle_request(index, q, c, t)
            np.testing.assert_array_equal(res["acc_idx"], acc)
        with pytest.raises(P.BayesLSHError):
            srv.submit(0, np.array([index.shape[0]], np.uint32), 0.8)      # id out of range
        assert srv.stats()["iterations"] > 0
    finally:
        srv.close()
        ctx.close()


def test_serving_device_submit_equals_host_and_oracle(index):
    """Candidate ids submitted from device memory give the same output as the
    same request submitted from the host, mixed in one stream of requests; a
    device request with ids >= n_obj finishes with BLSH_EBADID, its other
    candidates verified as usual, and does not mark the requests after it."""
    print("serving device submit", flush=True)
    ctx = P.bayeslsh_create(0)
    S = sigs_tensor(index, P.COSINE, P.WORD_MAJOR)
    n_obj = index.shape[0]
    srv = P.Server(ctx, S, mem_budget_bytes=2 << 20, max_active=6, k=32, max_batch_candidates=1 << 15)
    try:
        reqs = make_requests(n_obj, 40, 7)
        reqs.append((3, np.zeros(0, np.uint32), 0.8))                        # empty request
        dev = [up(c.astype(np.uint32)) for _, c, _ in reqs]
        ids = []
        for i, (q, c, t) in enumerate(reqs):                                  # interleave host and device
            ids.append((srv.submit(q, c, t), srv.submit_device(q, dev[i], t)))
        for (rh, rd), (q, c, t) in zip(ids, reqs):
            a, b = srv.wait(rh), srv.wait(rd)
            assert a["status"] == 0 and b["status"] == 0
            np.testing.assert_array_equal(a["acc_idx"], b["acc_idx"])
            np.testing.assert_array_equal(a["acc_val"], b["acc_val"])
            acc, sh = oracle_request(index, q, c, t)
            np.testing.assert_array_equal(b["acc_idx"], acc)
            np.testing.assert_allclose(b["acc_val"], sh, atol=1e-6)
            assert b["n_candidates"] == len(c)
            srv.release(rh)
            srv.release(rd)
        assert not srv._held
        # bad ids: positions 5 and 77 out of range
        q, c, t = reqs[1]
        c = np.resize(c, max(len(c), 100)).astype(np.uint32)
        bad = c.copy()
        bad[[5, 77]] = [n_obj, 0xFFFFFFFF]
        rb = srv.submit_device(q, up(bad), t)
        rg = srv.submit_device(q, up(c), t)
        res_b, res_g = srv.wait(rb), srv.wait(rg)
        assert res_b["status"] == -5 and res_g["status"] == 0
        ok = np.setdiff1d(np.arange(len(c)), [5, 77])
        acc, sh = oracle_request(index, q, c[ok], t)
        np.testing.assert_array_equal(res_b["acc_idx"], ok[acc])
        np.testing.assert_allclose(res_b["acc_val"], sh, atol=1e-6)
        acc, _ = oracle_request(index, q, c, t)
        np.testing.assert_array_equal(res_g["acc_idx"], acc)
        # a later request is clean
        rn = srv.submit_device(q, up(c), t)
        assert srv.wait(rn)["status"] == 0
        with pytest.raises(P.BayesLSHError):
            srv.submit_device(n_obj, dev[0], 0.8)                             # query out of range
        with pytest.raises(TypeError):
            srv.submit_device(0, dev[0].view(torch.int32), 0.8)
    finally:
        srv.close()
        ctx.close()


def test_serving_device_submit_many_per_admission(index):
    """More device-submitted requests admitted at once than one copy launch
    takes (64): every request still equals the oracle."""
    print("serving device submit, 150 at once", flush=True)
    ctx = P.bayeslsh_create(0)
    S = sigs_tensor(index, P.COSINE, P.WORD_MAJOR)
    srv = P.Server(ctx, S, mem_budget_bytes=16 << 20, max_active=256, k=32, max_batch_candidates=1 << 20)
    try:
        reqs = make_requests(index.shape[0], 150, 8, lo=0, hi=3.8)
        dev = [up(c) for _, c, _ in reqs]
        torch.cuda.synchronize()
        ids = [srv.submit_device(q, d, t) for (q, _, t), d in zip(reqs, dev)]
        for rid, (q, c, t) in zip(ids, reqs):
            res = srv.wait(rid)
            assert res["status"] == 0
            acc, sh = oracle_request(index, q, c, t)
            np.testing.assert_array_equal(res["acc_idx"], acc)
            np.testing.assert_allclose(res["acc_val"], sh, atol=1e-6)
    finally:
        srv.close()
        ctx.close()


def test_serving_device_submit_rejects_non_device_ranges(index):
    """bayeslsh_server_submit_device checks its pointer on the host: host
    memory, and a device range past the end of its allocation, are refused
    (BLSH_EINVAL) before anything reads them; a valid request still runs."""
    import ctypes as C
    from paper_1110_1328_amd import api as A
    print("serving device submit: pointer checks", flush=True)
    ctx = P.bayeslsh_create(0)
    S = sigs_tensor(index, P.COSINE, P.WORD_MAJOR)
    srv = P.Server(ctx, S, mem_budget_bytes=64 << 20, max_active=4, k=32, max_batch_candidates=1 << 16)
    try:
        lib = A._lib()
        rid = C.c_int64(-1)
        host = np.arange(64, dtype=np.uint32)
        rc = lib.bayeslsh_server_submit_device(srv.handle, 1, host.ctypes.data_as(C.c_void_p), 64, 0.8, C.byref(rid))
        assert rc == -1 and rid.value == -1
        small = up(np.arange(16, dtype=np.uint32))     # a 64-byte tensor: its allocation is far below 32 MB
        rc = lib.bayeslsh_server_submit_device(srv.handle, 1, C.c_void_p(small.data_ptr()), 8 << 20, 0.8,
                                               C.byref(rid))
        assert rc == -1 and rid.value == -1
        q, c, t = make_requests(index.shape[0], 1, 9)[0]
        res = srv.wait(srv.submit_device(q, up(c), t))
        acc, _ = oracle_request(index, q, c, t)
        assert res["status"] == 0
        np.testing.assert_array_equal(res["acc_idx"], acc)
    finally:
        srv.close()
        ctx.close()
