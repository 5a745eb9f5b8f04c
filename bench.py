#!/usr/bin/env python3
"""Benchmark: candidate pairs verified per second, BayesLSH vs exhaustive hash
compare with the same output, on one MI355X.

Workload (default): dense cosine estimation, the largest workload one GPU
holds -- 1M x 256 unit vectors from a 1000-component Gaussian mixture, 1024
sign-random-projection bits per vector (FP32 MFMA projection), candidates
from GPU LSH banding (16 bands x 12 bits of an independent 192-bit
projection, each bucket's pairs in 16 x 16 tiles of its members; about 2.4e9
pairs; timed apart from the step), Algorithm 1 at t = 0.8, epsilon = gamma =
0.03, delta = 0.05, k = 32.

One step = one bayeslsh_verify call over all candidates with signatures and
candidates resident in HBM and the posterior table cached.  The exhaustive
comparator (bayeslsh_exhaustive_verify, mode REPLAY: all 1024 bits of both
object-major rows, then the same decision sequence replayed) is timed the same
way and its output is checked to be identical.  The line carries the roofline
of the dominant kernel (algorithmic bytes over its HIP-event duration), the
oracle timed on the host over a seeded sample, and the sample's parity.  The
cosine BayesLSH-Lite workload (100k sparse tf-idf vectors, ~8e7 candidates)
follows under its own key.

Prints one JSON line (stdout).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "candidate pairs verified/sec, BayesLSH vs exhaustive hash compare, same output"
T, EPS, H, K, N_BITS = 0.7, 0.03, 128, 32, 2048
SRP_SEED = 0x5EED_1110_1328
HBM_PEAK_GBS = 8000.0
# the paper's own speedups, for context only (other hardware, whole pipeline
# including candidate generation, real datasets)
PAPER_CONTEXT = {
    "speedup_over_baselines": "2x-20x in most comparisons (abstract; Section 5)",
    "speedup_over_lsh_approx": "tf-idf cosine 2.0x-3.0x, binary Jaccard 2.8x-4.2x, binary cosine 1.2x "
                               "(Table 2, time summed over thresholds)",
    "hardware": "single-threaded C/C++, dual-socket dual-core 2.3 GHz Opteron, 8 GB RAM (Section 5)",
}


def log(msg):
    print("[bench %7.1fs] %s" % (time.time() - T0, msg), file=sys.stderr, flush=True)


T0 = time.time()


def up(torch, a):
    a = np.ascontiguousarray(a)
    m = {np.dtype(np.uint32): (np.int32, torch.uint32), np.dtype(np.uint64): (np.int64, torch.uint64)}
    if a.dtype in m:
        sd, td = m[a.dtype]
        return torch.from_numpy(a.view(sd)).cuda().view(td)
    return torch.from_numpy(a).cuda()


def build_workload(small: bool):
    from synth import generators as G
    if small:
        corpus = G.tfidf_corpus(n_docs=20_000, seed=G.SEED_BASE + 2)
        x, y = G.sparse_band_candidates(corpus, n_bands=16, band_bits=8, seed=G.SEED_BASE + 102)
    else:
        corpus = G.tfidf_corpus(seed=G.SEED_BASE + 2)
        x, y = G.sparse_band_candidates(corpus, n_bands=16, band_bits=10, seed=G.SEED_BASE + 102)
    return corpus, x, y


def lite_candidates(torch, P, ctx, corpus, small):
    """The 16-band LSH candidates of the tf-idf corpus, generated on the device:
    the band keys are the sign bits of the independent Gaussian projection that
    build_workload bands (10 bits a band; 8 for the small corpus), and
    bayeslsh_band_candidates lists each bucket's pairs in 16 x 16 tiles of its
    members (first-band dedupe), the order the compare kernel reads best; and
    the same candidates, numbered alike, as bucket tiles (bayeslsh_band_tiles).
    The candidate set is the one build_workload lists.  Returns device x, y,
    the count, the time of a second, timed banding call in ms, then the tiles,
    their count and the timed tile banding call in ms."""
    from synth import generators as G
    bb = 8 if small else 10
    words = G.sparse_band_bits(corpus, n_bands=16, band_bits=bb, seed=G.SEED_BASE + 102)
    S_band = P.Signatures(up(torch, words.reshape(-1)), P.COSINE, P.OBJECT_MAJOR, corpus.n, words.shape[1] * 32)
    cap = 1 << 27
    xo = torch.empty(cap, dtype=torch.int32, device="cuda").view(torch.uint32)
    yo = torch.empty(cap, dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_band_candidates(ctx, S_band, 16, bb, cap, x_out=xo, y_out=yo, order_tile=16)   # sizes its buffers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, n, trunc = P.bayeslsh_band_candidates(ctx, S_band, 16, bb, cap, x_out=xo, y_out=yo, order_tile=16)
    band_ms = (time.perf_counter() - t0) * 1e3
    if trunc:
        raise RuntimeError("banding: %d candidates exceed the %d-entry buffers" % (n, cap))
    tile_cap = 1 << 21
    tl = torch.empty(tile_cap * 24, dtype=torch.int64, device="cuda")
    P.bayeslsh_band_tiles(ctx, S_band, 16, bb, tile_cap, tiles_out=tl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, nt, n_t, trunc = P.bayeslsh_band_tiles(ctx, S_band, 16, bb, tile_cap, tiles_out=tl)
    band_t_ms = (time.perf_counter() - t0) * 1e3
    if trunc or n_t != n:
        raise RuntimeError("banding into tiles: %d candidates in %d tiles (pairs: %d)" % (n_t, nt, n))
    return xo[:n], yo[:n], n, band_ms, tl, nt, band_t_ms


def cpu_baseline(corpus, x, y, gpu_codes, gpu_m, gpu_acc):
    """The oracle (plain C loop of Algorithm 2 + FP64 exact cosine), timed over the
    whole candidate set on the host's cores, on signatures the oracle computes
    itself (the first h bits of every object; not timed, as the GPU's signature
    generation is not in its step either).  Also compares its output with the
    GPU's on every candidate whose two objects have no near-zero projection
    (only there can an FP32-vs-FP64 rounding flip a signature bit): decision,
    level and m exact, the accepted set equal, exact cosines within 1e-6."""
    from oracle import reference as R
    from oracle import posterior as OP
    rows = np.arange(corpus.n, dtype=np.int64)
    proj = R.srp_sparse_projections(corpus.offsets, corpus.indices, corpus.values, H, SRP_SEED, rows)
    sig = R.bits_from_projections(proj)
    OP.decision_memo(1, T, EPS, 0.0, 0.0, 1.0, 1.0, K, H // K, False)   # table, outside the timed region
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        res = R.verify(x, y, 1, sig, K, H // K, T, EPS, 0.0, 0.0, lite=True)
        res = R.lite_finish(res, lambda p, q: R.exact_cosine_csr(corpus.offsets, corpus.indices, corpus.values, p, q),
                            x, y, T)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    fragile = np.any(np.abs(proj) < 1e-5, axis=1)
    ok = ~(fragile[x] | fragile[y])
    g = gpu_codes
    acc_idx, acc_val = gpu_acc
    gpu_accepted = np.zeros(len(x), bool)
    gpu_accepted[acc_idx] = True
    gpu_val = np.full(len(x), np.nan)
    gpu_val[acc_idx] = acc_val
    both = ok & gpu_accepted & res["accepted"]
    parity = dict(compared=int(ok.sum()), skipped_fragile=int((~ok).sum()),
                  decision_mismatches=int(np.sum((g[ok] >> 6) != res["decision"][ok])),
                  level_mismatches=int(np.sum((g[ok] & 63) != res["level"][ok])),
                  m_mismatches=int(np.sum(gpu_m[ok] != res["m"][ok])),
                  accepted_set_mismatches=int(np.sum(gpu_accepted[ok] != res["accepted"][ok])),
                  accepted_compared=int(both.sum()),
                  max_abs_exact_cosine_error=float(np.max(np.abs(gpu_val[both] - res["exact"][both]), initial=0.0)))
    return dict(value=len(x) / dt, unit="pairs/s", cores=threads, cpu_model=cpu_model(), kind="oracle",
                sample="all %d candidates of the workload, median of 3 runs (%.2f s each)" % (len(x), dt)), parity, res


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "verify_bits_prefix_cosine_lite_100k_traffic.txt")
KERNEL_SOURCES = ("paper_1110_1328_amd/csrc/verify.hip", "paper_1110_1328_amd/csrc/device_common.h",
                  "paper_1110_1328_amd/csrc/api.hip")


def measured_traffic():
    """HBM bytes per verify launch from the committed FETCH_SIZE/WRITE_SIZE
    counter runs (scaled by a plain copy's counters), or None when the kernel
    sources have changed since those counters were taken."""
    import hashlib
    try:
        kv = dict(l.split() for l in open(TRAFFIC_FILE) if l.strip())
    except OSError:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return int(kv["traffic_bytes_per_launch"]) if kv.get("kernel_source_sha256") == h.hexdigest() else None


def copy_calibration(n_bytes=1 << 30, reps=20):
    """A plain device copy of known size (torch's copy kernel), for scaling rocprof
    FETCH_SIZE/WRITE_SIZE and as the achievable-bandwidth reference."""
    import torch
    a = torch.empty(n_bytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    print(json.dumps({"copy_bytes_read": n_bytes, "copy_bytes_written": n_bytes, "ms": ms,
                      "GBps_read_plus_write": 2 * n_bytes / ms / 1e6}), flush=True)


def dense_index(torch, P, ctx, layouts, prefix=False):
    """Dense cosine index: 1M x 256 unit vectors from a 1000-component Gaussian
    mixture, 1024 SRP bits from the MFMA projection against Gaussian planes,
    in each of the given layouts; with prefix=True each set also carries the
    16 B/object array of hashes 0..127 (the first 128 plane columns), checked
    against the object-major rows when those are built."""
    from synth import generators as G
    mix = G.dense_mixture(seed=G.SEED_BASE + 4)
    planes = up(torch, G.gaussian_planes(256, 1024, G.SEED_BASE + 204))
    xd = up(torch, mix.x)
    n = mix.x.shape[0]
    pfx = None
    if prefix:
        pfx = torch.empty(n * 4, dtype=torch.int32, device="cuda").view(torch.uint32)
        P.bayeslsh_srp_sigs(ctx, P.dense_vectors(xd), planes[:, :128].contiguous(), 128, 0, P.OBJECT_MAJOR, pfx)
    sigs = []
    for layout in layouts:
        out = torch.empty(n * 32, dtype=torch.int32, device="cuda").view(torch.uint32)
        P.bayeslsh_srp_sigs(ctx, P.dense_vectors(xd), planes, 1024, 0, layout, out)
        if pfx is not None and layout == P.OBJECT_MAJOR:
            assert torch.equal(out.view(torch.int32).view(n, 32)[:, :4], pfx.view(torch.int32).view(n, 4))
        sigs.append(P.Signatures(out, P.COSINE, layout, n, 1024, prefix=pfx))
    P.bayeslsh_sync(ctx)
    del xd
    return mix, sigs


def groups_of(labels):
    """related(q): the other objects with q's label (label < 0: none)."""
    order = np.argsort(labels, kind="stable")
    lab = labels[order]
    starts = np.searchsorted(lab, labels, side="left")
    ends = np.searchsorted(lab, labels, side="right")

    def related(q):
        if labels[q] < 0:
            return np.zeros(0, np.int64)
        m = order[starts[q]:ends[q]]
        return m[m != q]
    return related


def run_batched(args, torch, P):
    """4096 candidate lists (lengths 10^U(2,6)), measure ~ Bernoulli(1/2), t in
    {0.5, 0.7, 0.9}; Jaccard lists against 1M minhash signatures (256 hashes),
    cosine lists against the dense 1M x 1024-bit SRP index; one graph launch
    with k, in-register levels and grid autotuned; the exhaustive batched
    comparator at the chosen k must give the same output."""
    from synth import generators as G
    eps, delta, gamma = 0.03, 0.05, 0.03
    ctx = P.bayeslsh_create(0)
    log("jaccard index (1M sets, 256 minhashes)")
    sets = G.jaccard_sets_large(seed=G.SEED_BASE + 5)
    a, b = G.minhash_coeffs(256, G.SEED_BASE + 205)
    sig_j = torch.empty(sets.n * 256, dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_minhash_sigs(ctx, P.set_vectors(up(torch, sets.offsets), up(torch, sets.elems), sets.vocab),
                            up(torch, a), up(torch, b), sig_j)
    S_j = P.Signatures(sig_j, P.JACCARD, P.OBJECT_MAJOR, sets.n, 256)
    log("cosine index (1M x 256 dense, 1024 SRP bits)")
    # BayesLSH: word-major slabs (one per level) plus the 16 B/object prefix array,
    # so one gather serves the first 128 hashes; the comparator reads whole
    # object-major rows (also timed for BayesLSH, and word-major without the prefix)
    mix, (S_c, S_c_om) = dense_index(torch, P, ctx, (P.WORD_MAJOR, P.OBJECT_MAJOR), prefix=True)
    S_c_wm = P.Signatures(S_c.data, P.COSINE, P.WORD_MAJOR, S_c.n_obj, 1024)
    S_c_om = P.Signatures(S_c_om.data, P.COSINE, P.OBJECT_MAJOR, S_c_om.n_obj, 1024)
    n_lists = 4096
    rng = np.random.default_rng(G.SEED_BASE + 3)
    meas = rng.integers(0, 2, n_lists).astype(np.int32)
    ts = rng.choice([0.5, 0.7, 0.9], n_lists)
    log("lists")
    qj, oj, cj = G.member_lists(int(np.sum(meas == 0)), sets.n, 2, 6, groups_of(sets.group), seed=G.SEED_BASE + 31)
    qc, oc, cc = G.member_lists(int(np.sum(meas == 1)), mix.x.shape[0], 2, 6, groups_of(mix.comp),
                                seed=G.SEED_BASE + 32)
    cand = np.concatenate([cj, cc])
    query = np.empty(n_lists, np.uint32)
    offset = np.empty(n_lists, np.int64)
    length = np.empty(n_lists, np.int64)
    ij, ic = np.flatnonzero(meas == 0), np.flatnonzero(meas == 1)
    query[ij], offset[ij], length[ij] = qj, oj[:-1], np.diff(oj)
    query[ic], offset[ic], length[ic] = qc, oc[:-1] + len(cj), np.diff(oc)
    lists = P.list_descs(meas, ts, query, offset, length)
    n = len(cand)
    log("%d lists, %d candidates (%d Jaccard, %d cosine)" % (n_lists, n, len(cj), len(cc)))
    cand_d = up(torch, cand)
    cap = 1 << 24
    res = P.make_result(n, cap)
    res_ex = P.make_result(n, cap)
    stream = torch.cuda.current_stream()
    k_used = P.bayeslsh_verify_batched(ctx, lists, cand_d, S_j, S_c, eps, delta, gamma, (1, 1), 0, res, stream)
    P.bayeslsh_sync(ctx, stream)
    tune = P.bayeslsh_get_tuning(ctx)
    log("autotuned: k=%s tiles srp %d / minhash %d, inreg=%d blocks/CU=%d" % (
        k_used, tune["last_batch_srp_tile"], tune["last_batch_mh_tile"], tune["last_batch_inreg"],
        tune["last_batch_blocks_per_cu"]))

    def timed(fn, steps):
        for _ in range(2):
            fn()
        P.bayeslsh_sync(ctx, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        P.bayeslsh_sync(ctx, stream)
        return el * 1e3 / steps

    steps = max(3, args.steps // 5)
    ms = timed(lambda: P.bayeslsh_verify_batched(ctx, lists, cand_d, S_j, S_c, eps, delta, gamma, (1, 1), k_used,
                                                 res, stream), steps)
    log("batched: %.3f ms" % ms)
    # every phase-1 tile shape at the tuned k, in-register depth and blocks per
    # CU (the autotuner's choice among them is the one timed above)
    shapes = {}
    r2 = P.make_result(n, cap)
    for ts in (128, 256, 512):
        for tm in (64, 128):
            P.bayeslsh_set_tuning(ctx, batch_inreg=tune["last_batch_inreg"],
                                  batch_blocks_per_cu=tune["last_batch_blocks_per_cu"], batch_srp_tile=ts,
                                  batch_mh_tile=tm)
            t_ms = timed(lambda: P.bayeslsh_verify_batched(ctx, lists, cand_d, S_j, S_c, eps, delta, gamma, (1, 1),
                                                           k_used, r2, stream), 3)
            shapes["srp%d_mh%d" % (ts, tm)] = {"ms": t_ms, "same_codes": bool(torch.equal(r2.code[:n], res.code[:n]))}
    P.bayeslsh_set_tuning(ctx)
    del r2
    log("tile shapes: %s" % ", ".join("%s %.3f ms" % (kk, v["ms"]) for kk, v in shapes.items()))
    # the same batch split by measure, at every k (where the time goes)
    split = {}
    r2 = P.make_result(n, cap)
    for name, me in (("jaccard", 0), ("cosine", 1)):
        sub = lists[meas == me]
        split[name] = {}
        for kk in (16, 32, 64):
            split[name]["k%d" % kk] = timed(lambda: P.bayeslsh_verify_batched(
                ctx, sub, cand_d, S_j if me == 0 else None, S_c if me == 1 else None, eps, delta, gamma, (1, 1),
                kk, r2, stream), 3)
            P.bayeslsh_set_tuning(ctx, batch_inreg=64)      # every level in registers, no survivor queue
            split[name]["k%d_inreg_all" % kk] = timed(lambda: P.bayeslsh_verify_batched(
                ctx, sub, cand_d, S_j if me == 0 else None, S_c if me == 1 else None, eps, delta, gamma, (1, 1),
                kk, r2, stream), 3)
            P.bayeslsh_set_tuning(ctx)
            if me == 1:
                for lname, Sl in (("word_major", S_c_wm), ("object_major", S_c_om)):
                    split[name]["k%d_%s" % (kk, lname)] = timed(lambda: P.bayeslsh_verify_batched(
                        ctx, sub, cand_d, None, Sl, eps, delta, gamma, (1, 1), kk, r2, stream), 3)
        split[name]["exhaustive_k%d" % k_used[me]] = timed(lambda: P.bayeslsh_exhaustive_batched(
            ctx, sub, cand_d, S_j if me == 0 else None, S_c_om if me == 1 else None, eps, delta, gamma, (1, 1),
            k_used, r2, stream), 2)
        log("  %s: %s" % (name, ", ".join("%s %.2f ms" % kv for kv in split[name].items())))
    del r2
    ms_ex = timed(lambda: P.bayeslsh_exhaustive_batched(ctx, lists, cand_d, S_j, S_c_om, eps, delta, gamma, (1, 1),
                                                        k_used, res_ex, stream), max(2, steps // 3))
    log("exhaustive batched: %.3f ms" % ms_ex)
    diff_codes = int(res.code[:n].ne(res_ex.code[:n]).sum().item())
    ia, va = res.accepted()
    ib, vb = res_ex.accepted()
    same = diff_codes == 0 and np.array_equal(ia, ib) and np.array_equal(va, vb)
    if not same:
        log("outputs differ: %d codes, accepted %d vs %d" % (diff_codes, len(ia), len(ib)))
    codes = res.code[:n].cpu().numpy()
    dec, lvl = codes >> 6, (codes & 63).astype(np.int64)
    # algorithmic bytes: 4 B id + 1 B code per candidate, plus the candidate's
    # signature chunk per level reached (the query's chunk is read once per tile)
    per_level = np.where(np.repeat(meas, length) == 0, 4 * k_used[0], k_used[1] // 8)
    alg = n * 5 + int(np.sum((lvl + 1) * per_level))
    ctx.close()
    return {
        "metric": "candidate pairs verified/sec, batched BayesLSH vs exhaustive batched hash compare, same output",
        "value": n / (ms * 1e-3), "unit": "pairs/s", "n_gpus": 1, "steps": steps, "ms_per_step": ms,
        "higher_is_better": True, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "batched: 4096 lists, lengths 10^U(2,6), measure ~ Bernoulli(1/2), t in {0.5,0.7,0.9}; "
                               "Jaccard: 1M planted-group sets, 256 minhashes; cosine: 1M x 256 Gaussian-mixture "
                               "vectors, 1024 SRP bits (word-major + 128-bit prefix array; the comparator reads object-major rows); eps=0.03, delta=0.05, gamma=0.03",
                   "n_candidates": n, "n_jaccard": int(len(cj)), "n_cosine": int(len(cc)),
                   "k_jaccard": k_used[0], "k_cosine": k_used[1], "inreg_levels": tune["last_batch_inreg"],
                   "blocks_per_cu": tune["last_batch_blocks_per_cu"], "srp_tile": tune["last_batch_srp_tile"],
                   "minhash_tile": tune["last_batch_mh_tile"]},
        "tile_shapes": shapes,
        "decisions": {"pruned": int(np.sum(dec == 0)), "accept_conc": int(np.sum(dec == 1)),
                      "accept_nmax": int(np.sum(dec == 2)), "accepted_listed": int(len(ia))},
        "exhaustive": {"ms_per_step": ms_ex, "value": n / (ms_ex * 1e-3), "speedup": ms_ex / ms,
                       "same_output": same},
        "algorithmic_bytes": alg, "algorithmic_GBps": alg / (ms * 1e-3) / 1e9,
        "by_measure_ms": split,
    }


def run_serving(args, torch, P):
    """Poisson arrivals of query objects against the dense cosine index
    (candidate counts 10^U(3,6), t = 0.8): first all at once (saturated rate),
    then at rho x that rate for rho in {0.5, 0.8, 0.95}; latency = arrival to
    host-visible result; then all at once from 4 client threads.  Then the same requests submitted from device memory
    (candidate ids resident on the GPU, no host copy of them): saturated and at
    rho = 0.95 of that rate.  Rates are given twice: over the client's elapsed
    time (which includes the Python client's submission and per-request result
    conversion) and over the server's own span, first submission to last
    completion on its clock."""
    from synth import generators as G
    ctx = P.bayeslsh_create(0)
    log("cosine index (1M x 256 dense, 1024 SRP bits)")
    mix, (S,) = dense_index(torch, P, ctx, (P.WORD_MAJOR,), prefix=True)
    nq = args.queries
    log("%d queries" % nq)
    rng = np.random.default_rng(G.SEED_BASE + 6)
    queries = rng.integers(0, mix.x.shape[0], nq).astype(np.uint32)
    q, off, cand = G.member_lists(nq, mix.x.shape[0], 3, 6, groups_of(mix.comp), seed=G.SEED_BASE + 61,
                                  queries=queries)
    lens = np.diff(off)
    total = int(off[-1])
    log("%d candidates" % total)
    srv = P.Server(ctx, S, mem_budget_bytes=2 << 30, max_active=128, k=32, max_batch_candidates=1 << 23)

    dcand = None

    def run(gaps):
        ids = []
        t0 = time.perf_counter()
        for i in range(nq):
            if gaps is not None:
                due = t0 + gaps[i]
                while time.perf_counter() < due:
                    pass
            if dcand is None:
                ids.append(srv.submit(int(q[i]), cand[off[i]:off[i + 1]], 0.8))
            else:
                ids.append(srv.submit_device(int(q[i]), dcand[off[i]:off[i + 1]], 0.8))
        run.submit_s = time.perf_counter() - t0              # when the client had submitted everything
        out = [srv.wait(r) for r in ids]
        el = time.perf_counter() - t0
        for r in ids:
            srv.release(r)
        lat = np.array([o["done"] - o["submit"] for o in out])
        # the server's own span: first submission to last completion, on its clock
        run.server_s = max(o["done"] for o in out) - min(o["submit"] for o in out)
        return el, lat, out

    def run_clients(n_clients):
        """All requests at once from n_clients threads (request i from thread
        i mod n_clients); each submits its share, then waits for it."""
        import threading
        out = [None] * nq
        t0 = time.perf_counter()

        def client(c):
            mine = range(c, nq, n_clients)
            ids = [srv.submit(int(q[i]), cand[off[i]:off[i + 1]], 0.8) for i in mine]
            for i, r in zip(mine, ids):
                out[i] = srv.wait(r)
                srv.release(r)

        th = [threading.Thread(target=client, args=(c,)) for c in range(n_clients)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        el = time.perf_counter() - t0
        run.submit_s = None
        run.server_s = max(o["done"] for o in out) - min(o["submit"] for o in out)
        return el, np.array([o["done"] - o["submit"] for o in out]), out

    def stats(el, lat, out, ref):
        d = {"queries_per_s": nq / el, "pairs_per_s": total / el, "p50_ms": float(np.percentile(lat, 50) * 1e3),
             "p99_ms": float(np.percentile(lat, 99) * 1e3), "client_submit_s": run.submit_s, "elapsed_s": el,
             "server_span_s": run.server_s, "server_pairs_per_s": total / run.server_s}
        if ref is not None:
            d["same_results"] = all(np.array_equal(a["acc_idx"], b["acc_idx"]) and
                                    np.array_equal(a["acc_val"], b["acc_val"]) for a, b in zip(ref, out))
        return d

    res, out0 = {}, None
    if args.serving_legs == "all":
        run(None)                                        # warm (graphs, tables)
        el, lat, out0 = run(None)
        sat_qps = nq / el
        res["saturated"] = stats(el, lat, out0, None)
        log("saturated: %.0f q/s, %.3g pairs/s" % (sat_qps, total / el))
        for rho in (0.5, 0.8, 0.95):
            gaps = np.cumsum(np.random.default_rng(int(rho * 100)).exponential(1.0 / (rho * sat_qps), nq))
            key = "rho_%.2f" % rho
            res[key] = stats(*run(gaps), out0)
            log("rho %.2f: p50 %.2f ms p99 %.2f ms" % (rho, res[key]["p50_ms"], res[key]["p99_ms"]))
        # the same requests from 4 client threads at once (ids in host memory)
        res["saturated_4_clients"] = stats(*run_clients(4), out0)
        log("4 clients, saturated: %.0f q/s, %.3g pairs/s" % (res["saturated_4_clients"]["queries_per_s"],
                                                             res["saturated_4_clients"]["pairs_per_s"]))
    # the same requests with candidate ids already resident on the device
    dcand = up(torch, cand)
    run(None)
    el, lat, out = run(None)
    dev_qps = nq / el
    res["device_saturated"] = stats(el, lat, out, out0)
    log("device submit, saturated: %.0f q/s, %.3g pairs/s (server span %.1f ms: %.3g pairs/s)" % (
        dev_qps, total / el, run.server_s * 1e3, total / run.server_s))
    gaps = np.cumsum(np.random.default_rng(95).exponential(1.0 / (0.95 * dev_qps), nq))
    res["device_rho_0.95"] = stats(*run(gaps), out0 if out0 is not None else out)
    log("device submit, rho 0.95: p50 %.2f ms p99 %.2f ms" % (res["device_rho_0.95"]["p50_ms"],
                                                               res["device_rho_0.95"]["p99_ms"]))
    dcand = None
    st = srv.stats()
    srv.close()
    ctx.close()
    return {"metric": "serving: candidate pairs verified/sec and query latency", "unit": "pairs/s",
            "value": res["saturated" if "saturated" in res else "device_saturated"]["pairs_per_s"], "n_gpus": 1,
            "data": "synthetic", "dtype": "u32",
            "config": {"workload": "serving: %d queries against 1M x 1024-bit dense cosine index, candidates "
                                   "10^U(3,6) per query (1%% from the query's mixture component), t=0.8, k=32, "
                                   "max_active=128, 8M candidates per iteration, 2 GiB arena%s" % (
                                       nq, "" if args.serving_legs == "all" else "; device-memory submissions only"),
                       "n_candidates": total,
                       "mean_candidates": float(lens.mean())},
            "latency": res, "server_stats": st}


def run_sigs(args, torch, P):
    """Signature generation (untimed in every verification step), each call
    timed with HIP events on its stream, median of 5 after a warm-up:
    - dense SRP of the 1M x 256 mixture against 1024 Gaussian planes on the
      FP32 matrix cores: 2 d n_bits flops per row, against the 157.3 TFLOP/s
      dense FP32 MFMA peak;
    - sparse SRP of the 100k-document tf-idf corpus at 2048 bits (plane
      entries from Philox-4x32-10 + Box-Muller, drawn once per term into a
      table since terms repeat; FP64 accumulation): n_bits entries applied
      per nonzero;
    - 256 minhashes of the 1M planted-group sets: one multiply-mod and min per
      (element, hash)."""
    from synth import generators as G
    ctx = P.bayeslsh_create(0)
    s = torch.cuda.current_stream()

    def timed(fn, reps=5):
        fn()
        P.bayeslsh_sync(ctx, s)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ts = []
        for _ in range(reps):
            e0.record(s)
            fn()
            e1.record(s)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        P.bayeslsh_sync(ctx, s)
        return float(np.median(ts)), float(min(ts))

    log("dense mixture (1M x 256), 1024 planes")
    mix = G.dense_mixture(seed=G.SEED_BASE + 4)
    planes = up(torch, G.gaussian_planes(256, 1024, G.SEED_BASE + 204))
    xd = up(torch, mix.x)
    n_d = mix.x.shape[0]
    out_d = torch.empty(n_d * 32, dtype=torch.int32, device="cuda").view(torch.uint32)
    dense_ms, dense_min = timed(lambda: P.bayeslsh_srp_sigs(ctx, P.dense_vectors(xd), planes, 1024, 0,
                                                            P.OBJECT_MAJOR, out_d, s))
    flops = 2.0 * n_d * 256 * 1024
    tflops = flops / (dense_ms * 1e-3) / 1e12
    log("dense SRP: %.3f ms, %.1f TFLOP/s" % (dense_ms, tflops))
    del xd, out_d
    log("tf-idf corpus (100k documents)")
    corpus = G.tfidf_corpus(seed=G.SEED_BASE + 2)
    nnz = len(corpus.indices)
    vec = P.csr_vectors(up(torch, corpus.offsets), up(torch, corpus.indices), up(torch, corpus.values), corpus.dim)
    out_s = torch.empty(corpus.n * (N_BITS // 32), dtype=torch.int32, device="cuda").view(torch.uint32)
    sparse_ms, sparse_min = timed(lambda: P.bayeslsh_srp_sigs(ctx, vec, None, N_BITS, SRP_SEED, P.OBJECT_MAJOR,
                                                              out_s, s))
    log("sparse SRP: %.3f ms, %.3g Gaussians/s" % (sparse_ms, nnz * N_BITS / (sparse_ms * 1e-3)))
    # the same with every plane entry stored in 2 bytes (Section 4.3): the table
    # of codes is half the bytes; bits differ only where |r . x| is within the
    # storage error of 0
    out_q = torch.empty_like(out_s)
    q16_ms, q16_min = timed(lambda: P.bayeslsh_srp_sigs(ctx, vec, None, N_BITS, SRP_SEED, P.OBJECT_MAJOR,
                                                        out_q, s, flags=P.SRP_PLANES_Q16))
    x = out_q.view(torch.int32) ^ out_s.view(torch.int32)
    flipped = sum(int(((x >> b) & 1).sum().item()) for b in range(32))
    log("sparse SRP, 2-byte plane entries: %.3f ms; %d of %d bits differ from the fp32-entry signatures"
        % (q16_ms, flipped, corpus.n * N_BITS))
    del vec, out_s, out_q, x
    log("planted-group sets (1M), 256 minhashes")
    sets = G.jaccard_sets_large(seed=G.SEED_BASE + 5)
    a, b = G.minhash_coeffs(256, G.SEED_BASE + 205)
    sv = P.set_vectors(up(torch, sets.offsets), up(torch, sets.elems), sets.vocab)
    da, db = up(torch, a), up(torch, b)
    out_m = torch.empty(sets.n * 256, dtype=torch.int32, device="cuda").view(torch.uint32)
    mh_ms, mh_min = timed(lambda: P.bayeslsh_minhash_sigs(ctx, sv, da, db, out_m, s))
    n_el = len(sets.elems)
    log("minhash: %.3f ms, %.3g hash evaluations/s" % (mh_ms, n_el * 256 / (mh_ms * 1e-3)))
    ctx.close()
    return {"metric": "signature generation: dense SRP on the FP32 matrix cores", "value": tflops,
            "unit": "TFLOP/s", "n_gpus": 1, "ms_per_step": dense_ms, "higher_is_better": True, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "signature generation: dense SRP 1M x 256 fp32 rows x 1024 planes; sparse SRP "
                                   "100k tf-idf documents x 2048 bits (plane entries drawn once per term); 256 "
                                   "minhashes of 1M sets"},
            "roofline": {"bound": "mfma", "achieved": tflops, "peak": 157.3, "unit": "TFLOP/s",
                         "frac": tflops / 157.3, "traffic": None, "kernel": "k_srp_dense_mfma<256>",
                         "flops_per_launch": flops},
            "dense_srp": {"ms": dense_ms, "min_ms": dense_min, "rows": n_d, "dim": 256, "n_bits": 1024,
                          "tflops": tflops},
            "sparse_srp": {"ms": sparse_ms, "min_ms": sparse_min, "rows": corpus.n, "nnz": nnz, "n_bits": N_BITS,
                           "gaussians_per_s": nnz * N_BITS / (sparse_ms * 1e-3)},
            "sparse_srp_q16": {"ms": q16_ms, "min_ms": q16_min, "gaussians_per_s": nnz * N_BITS / (q16_ms * 1e-3),
                               "bits_differing_from_fp32_entries": flipped,
                               "note": "plane entries as 2-byte codes (Section 4.3), table of dim x n_bits codes"},
            "minhash": {"ms": mh_ms, "min_ms": mh_min, "sets": sets.n, "elements": n_el, "n_hashes": 256,
                        "hash_evals_per_s": n_el * 256 / (mh_ms * 1e-3)}}


DENSE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "verify_tiles_dense_1m_traffic.txt")
# the kernels' sources and the host code that cuts a call into launches (the
# counters are per launch)
DENSE_KERNEL_SOURCES = ("paper_1110_1328_amd/csrc/verify.hip", "paper_1110_1328_amd/csrc/device_common.h",
                        "paper_1110_1328_amd/csrc/api.hip")
# the verification call's kernels, by the names their launches are profiled under
TILE_KERNELS = ("verify_tiles", "tiles_flush")
PAIR_KERNELS = ("verify_bits_prefix", "verify_tail", "acc_flush")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def kernel_profile(P, ctx, stream, fn, steps, names):
    """Average duration and launches per step of each named kernel, from HIP
    events recorded around every launch on its stream (a pass of its own, so
    that event creation stays out of the timed steps)."""
    P.bayeslsh_profile_enable(ctx, True)
    P.bayeslsh_profile_reset(ctx)
    for _ in range(steps):
        fn()
    P.bayeslsh_sync(ctx, stream)
    out = {}
    for nm in names:
        ms, nl = P.bayeslsh_profile_read(ctx, nm)
        out[nm] = {"avg_ms": ms / max(nl, 1), "launches_per_step": nl / steps, "ms_per_step": ms / steps}
    P.bayeslsh_profile_enable(ctx, False)
    return out


def measured_traffic_of(path, sources, key):
    """A value from a committed counter summary, or None when the kernel sources
    hash differently from when the counters were taken."""
    import hashlib
    try:
        kv = dict(l.split() for l in open(path) if l.strip())
    except OSError:
        return None
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return int(float(kv[key])) if kv.get("kernel_source_sha256") == h.hexdigest() and key in kv else None


def timed_steps(torch, P, ctx, stream, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    P.bayeslsh_sync(ctx, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) * 1e3 / steps
    P.bayeslsh_sync(ctx, stream)
    return ms


def same_output(torch, n, ra, rb):
    """Codes equal and accepted lists equal as sets of (index, value), on the device."""
    diff = int(ra.code[:n].ne(rb.code[:n]).sum().item())
    na, nb = int(ra.n_accepted.item()), int(rb.n_accepted.item())
    same = diff == 0 and na == nb
    if same:
        ia, oa = torch.sort(ra.acc_idx[:na].view(torch.int64))
        ib, ob = torch.sort(rb.acc_idx[:nb].view(torch.int64))
        same = bool(torch.equal(ia, ib)) and bool(torch.equal(ra.acc_val[:na][oa], rb.acc_val[:nb][ob]))
    return same, diff


def run_dense(args, torch, P):
    """Dense cosine estimation, the largest single-GPU workload: 1M x 256
    Gaussian-mixture vectors, 1024 SRP bits (object-major rows) for
    verification; candidates from GPU LSH banding (16 bands x 12 bits of an
    independent 192-bit projection; each bucket's pairs by 16 x 16 tiles of its
    members, ~2.4e9 pairs).  One step = Algorithm 1 (t = 0.8, eps = gamma =
    0.03, delta = 0.05, k = 32, n_max = 1024) over every candidate, the
    candidates handed over as bucket tiles (bayeslsh_band_tiles); the same
    candidates as explicit id pairs (bayeslsh_band_candidates, with the 16 B
    prefix array) are timed beside it and must give the same output, and so
    must the exhaustive REPLAY comparator (all 1024 bits of both object-major
    rows).  A seeded sample of the candidates is checked against the oracle on
    the GPU's own signatures (decision, level and m exact, S_hat within 1e-6),
    and the oracle's Algorithm 1 is timed over that sample on the host."""
    from synth import generators as G
    from oracle import reference as R
    from oracle import posterior as OP
    t, eps, delta, gamma, k = 0.8, 0.03, 0.05, 0.03, 32
    ctx = P.bayeslsh_create(0)
    stream = torch.cuda.current_stream()
    log("dense index (1M x 256, 1024 verification bits)")
    mix, (S_pfx,) = dense_index(torch, P, ctx, (P.OBJECT_MAJOR,), prefix=True)
    n_obj = mix.x.shape[0]
    S_om = P.Signatures(S_pfx.data, P.COSINE, P.OBJECT_MAJOR, n_obj, 1024)
    band_planes = up(torch, G.gaussian_planes(256, 192, G.SEED_BASE + 104))
    band_sig = torch.empty(n_obj * 6, dtype=torch.int32, device="cuda").view(torch.uint32)
    xd = up(torch, mix.x)
    P.bayeslsh_srp_sigs(ctx, P.dense_vectors(xd), band_planes, 192, 0, P.OBJECT_MAJOR, band_sig)
    P.bayeslsh_sync(ctx)
    del xd, mix
    S_band = P.Signatures(band_sig, P.COSINE, P.OBJECT_MAJOR, n_obj, 192)

    # the candidates as bucket tiles (banding once to size its buffers, then timed)
    tile_cap = 1 << 25
    tl = torch.empty(tile_cap * 24, dtype=torch.int64, device="cuda")
    P.bayeslsh_band_tiles(ctx, S_band, 16, 12, tile_cap, tiles_out=tl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, n_tiles, n, trunc = P.bayeslsh_band_tiles(ctx, S_band, 16, 12, tile_cap, tiles_out=tl)
    band_tiles_ms = (time.perf_counter() - t0) * 1e3
    assert not trunc, n_tiles
    log("banding as tiles: %d candidates in %d tiles, %.1f ms" % (n, n_tiles, band_tiles_ms))
    # and as explicit id pairs
    cap = int(2.6e9)
    xo = torch.empty(cap, dtype=torch.int32, device="cuda").view(torch.uint32)
    yo = torch.empty(cap, dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_band_candidates(ctx, S_band, 16, 12, cap, x_out=xo, y_out=yo, order_tile=16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, n_p, trunc = P.bayeslsh_band_candidates(ctx, S_band, 16, 12, cap, x_out=xo, y_out=yo, order_tile=16)
    band_ms = (time.perf_counter() - t0) * 1e3
    assert not trunc and n_p == n, (n_p, n)
    log("banding as pairs: %d candidates in %.1f ms" % (n, band_ms))
    acc_cap = 1 << 28

    # headline: Algorithm 1 over the tiles
    cand_t = P.tiles(tl, n_tiles, n)
    res = P.make_result(n, acc_cap)

    def step():
        P.bayeslsh_verify(ctx, cand_t, S_om, t, eps, delta, gamma, (1, 1), k, res, stream)

    ms = timed_steps(torch, P, ctx, stream, step, args.steps, args.warmup)
    log("BayesLSH over tiles: %.3f ms/step (%.3g pairs/s)" % (ms, n / ms * 1e3))
    prof = kernel_profile(P, ctx, stream, step, min(args.steps, 10), TILE_KERNELS)
    log("kernels: %s" % ", ".join("%s %.3f ms x %.0f" % (k_, v["avg_ms"], v["launches_per_step"])
                                  for k_, v in prof.items()))

    # the same candidates as id pairs (prefix array + tail)
    cand_p = P.pairs(xo[:n], yo[:n])
    res_p = P.make_result(n, acc_cap)

    def step_p():
        P.bayeslsh_verify(ctx, cand_p, S_pfx, t, eps, delta, gamma, (1, 1), k, res_p, stream)

    ms_p = timed_steps(torch, P, ctx, stream, step_p, max(3, args.steps // 2), 2)
    prof_p = kernel_profile(P, ctx, stream, step_p, min(args.steps, 5), PAIR_KERNELS)
    same_p, diff_p = same_output(torch, n, res, res_p)
    log("BayesLSH over id pairs: %.3f ms/step; same output as tiles: %s" % (ms_p, same_p))
    del res_p

    # the exhaustive comparator: every candidate compares all 1024 bits, then the
    # decision sequence is replayed -> the same output
    res_ex = P.make_result(n, acc_cap)

    def step_ex():
        P.bayeslsh_exhaustive_verify(ctx, cand_p, S_om, None, t, eps, delta, gamma, (1, 1), k, 0, P.REPLAY, res_ex,
                                     stream)

    ms_ex = timed_steps(torch, P, ctx, stream, step_ex, max(2, args.steps // 10), 1)
    log("exhaustive: %.3f ms/step" % ms_ex)
    same, diff_codes = same_output(torch, n, res, res_ex)
    if not same:
        log("outputs differ: %d codes" % diff_codes)
    del res_ex
    codes = res.code[:n]
    lvl = (codes & 63).to(torch.int64)
    dec = codes >> 6
    dec_counts = [int(dec.eq(d).sum().item()) for d in range(3)]
    levels_reached = int(lvl.sum().item()) + n
    levels_past_prefix = int((lvl - 3).clamp_(min=0).sum().item())
    lvl_mean = levels_reached / n - 1.0
    n_acc = int(res.n_accepted.item())
    del lvl, dec
    # decisions by level (index j: taken after (j + 1) k hashes): a histogram of
    # the code bytes, in chunks of 2^30 candidates
    hist = torch.zeros(256, dtype=torch.int64, device="cuda")
    for c0 in range(0, n, 1 << 30):
        hist += torch.bincount(codes[c0:c0 + (1 << 30)].to(torch.int32), minlength=256)
    hist = hist.cpu().numpy()
    by_level = {name: hist[64 * d: 64 * d + 1024 // k].tolist()
                for d, name in ((0, "pruned"), (1, "accept_conc"), (2, "accept_nmax"))}

    # parity pass with m recorded (not timed), on a seeded sample against the oracle
    res_m = P.make_result(n, acc_cap, m_debug=True)
    P.bayeslsh_verify(ctx, cand_t, S_om, t, eps, delta, gamma, (1, 1), k, res_m, stream)
    P.bayeslsh_sync(ctx, stream)
    assert bool(torch.equal(res_m.code[:n], res.code[:n]))
    # stratified sample: one candidate drawn uniformly from each of n_sample
    # equal strata of the candidate numbering (already in candidate order)
    rng = np.random.default_rng(G.SEED_BASE + 105)
    n_sample = min(n, args.cpu_sample)
    stride = n // n_sample
    pick = np.arange(n_sample, dtype=np.int64) * stride + rng.integers(0, stride, size=n_sample, dtype=np.int64)
    pick_d = torch.from_numpy(pick).cuda()
    xs = xo[:n].view(torch.int32)[pick_d].cpu().numpy().view(np.uint32)
    ys = yo[:n].view(torch.int32)[pick_d].cpu().numpy().view(np.uint32)
    got_code = res_m.code[:n][pick_d].cpu().numpy()
    got_m = res_m.m_debug[:n].view(torch.int16)[pick_d].cpu().numpy().view(np.uint16).astype(np.int32)
    n_acc_m = int(res_m.n_accepted.item())
    shat_all = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    shat_all[res_m.acc_idx[:n_acc_m].view(torch.int64)] = res_m.acc_val[:n_acc_m]
    got_shat = shat_all[pick_d].cpu().numpy()
    del shat_all, res_m, pick_d
    sig_host = S_om.data.view(torch.int32).cpu().numpy().view(np.uint32).reshape(n_obj, 32)
    log("cpu baseline and sampled parity: oracle Algorithm 1 over %d candidates" % n_sample)
    OP.decision_memo(1, t, eps, delta, gamma, 1.0, 1.0, k, 1024 // k, True)   # table, outside the timed runs
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    times = []
    for _ in range(3):
        t1 = time.perf_counter()
        want = R.verify(xs, ys, P.COSINE, sig_host, k, 1024 // k, t, eps, delta, gamma)
        times.append(time.perf_counter() - t1)
    dt = float(np.median(times))
    emit = np.isfinite(want["shat"])
    parity = {
        "sample": n_sample,
        "path": "bucket tiles (the headline call)",
        "decision_mismatches": int(np.sum((got_code >> 6) != want["decision"])),
        "level_mismatches": int(np.sum((got_code & 63) != want["level"])),
        "m_mismatches": int(np.sum(got_m != want["m"])),
        "emitted_in_sample": int(emit.sum()),
        "emitted_set_mismatches": int(np.sum(np.isfinite(got_shat) != emit)),
        "max_abs_shat_error": float(np.max(np.abs(got_shat[emit] - want["shat"][emit]), initial=0.0)),
    }
    log("sampled parity: %s" % parity)
    cpu = dict(value=n_sample / dt, unit="pairs/s", cores=threads, cpu_model=cpu_model(), kind="oracle",
               sample="seeded stratified sample of %d of the %d candidates (one uniform draw per stratum), oracle "
                      "Algorithm 1 (plain C loop, OpenMP) on the GPU's own signatures, median of 3 runs "
                      "(%.2f s each)" % (n_sample, n, dt))
    log("cpu baseline: %.3g pairs/s on %d threads" % (cpu["value"], threads))
    del xs, ys, sig_host, want

    # Algorithmic bytes.  Per candidate: 1 B of code, both sides' 4 B chunk per
    # level reached (8 B), 12 B per emitted pair; the candidate ids: 8 B per
    # pair for id pairs, for tiles the 64 B descriptor and 32 member ids (4 B)
    # per tile.  Tiles: the tile kernel owns the ids, the code and level 0, the
    # row kernel the later levels and the emission; id pairs: the prefix kernel
    # owns ids, code and levels 0-3, the tail the rest.
    chunk = 2 * (k // 8)
    accepted = dec_counts[1] + dec_counts[2]
    id_bytes_t = n_tiles * 192
    call_bytes = id_bytes_t + n + chunk * levels_reached + 12 * accepted
    per = {"verify_tiles": id_bytes_t + n + chunk * levels_reached + 12 * accepted, "tiles_flush": 12 * accepted}
    per_p = {"verify_bits_prefix": 9 * n + chunk * (levels_reached - levels_past_prefix),
             "verify_tail": chunk * levels_past_prefix + 12 * accepted, "acc_flush": 12 * accepted}

    def with_bytes(pr, bb):
        return {k_: dict(v, algorithmic_bytes_per_step=bb[k_],
                         algorithmic_GBps=bb[k_] / (v["ms_per_step"] * 1e-3) / 1e9 if v["ms_per_step"] else None)
                for k_, v in pr.items()}

    kern_ms = sum(v["ms_per_step"] for v in prof.values())
    dom = "verify_tiles"
    launches = prof[dom]["launches_per_step"]
    dom_bytes = per[dom] / launches
    achieved = dom_bytes / (prof[dom]["avg_ms"] * 1e-3) / 1e9
    traffic = measured_traffic_of(DENSE_TRAFFIC_FILE, DENSE_KERNEL_SOURCES, "traffic_bytes_per_launch_" + dom)

    def issue_of(kernel_ms):
        """VALU issue utilisation: the kernel's VALU instructions per launch (SQ
        counters, committed with the traffic) over what 256 CUs issue at one
        wave instruction per cycle at 2.4 GHz in the launch's live duration."""
        valu = measured_traffic_of(DENSE_TRAFFIC_FILE, DENSE_KERNEL_SOURCES, "valu_insts_per_launch_" + dom)
        if valu is None:
            return None
        cap = 256 * 2.4e9 * kernel_ms * 1e-3
        return {"valu_insts_per_launch": valu, "valu_issue_capacity_per_launch": cap, "valu_busy_frac": valu / cap,
                "valu_insts_per_tile": valu / (n_tiles / launches), "source": "SQ_INSTS_VALU, " + os.path.relpath(DENSE_TRAFFIC_FILE, ROOT)}
    roofline = {
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "traffic_frac": traffic / (prof[dom]["avg_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS if traffic else None,
        "kernel": dom, "kernel_avg_ms": prof[dom]["avg_ms"], "launches_per_step": launches,
        "algorithmic_bytes_per_launch": dom_bytes,
        "kernels": with_bytes(prof, per),
        "call": {"algorithmic_bytes": call_bytes, "kernel_ms": kern_ms,
                 "achieved": call_bytes / (kern_ms * 1e-3) / 1e9,
                 "frac": call_bytes / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "traffic": measured_traffic_of(DENSE_TRAFFIC_FILE, DENSE_KERNEL_SOURCES, "traffic_bytes_per_call")},
        "bytes_model": "per candidate 1 B code + 8 B per level reached (4 B chunk per side at k = 32) + 12 B per "
                       "emitted pair, plus the 192 B descriptor (member ids included) per tile; the tile kernel "
                       "does all of it, the flush copies the staged accepted pairs to the caller's list",
        "issue": issue_of(prof[dom]["avg_ms"]),
        "note": "frac counts each candidate's level chunks as if read for it alone; the tile kernel reads a "
                "tile's 32 rows once into LDS for its 256 positions, so the counted HBM traffic (traffic, "
                "traffic_frac) is a fraction of the algorithmic bytes and the kernel is bound by instruction "
                "issue rather than by HBM (issue.valu_busy_frac)",
    }
    ctx.close()
    return {
        "metric": METRIC,
        "value": n / (ms * 1e-3), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "dense cosine estimation: 1M x 256 Gaussian-mixture vectors (1000 components), 1024 SRP "
                               "bits, GPU LSH banding 16 x 12 bits on an independent 192-bit projection, candidates "
                               "handed over as 16 x 16 bucket tiles, Algorithm 1 t=0.8, eps=gamma=0.03, "
                               "delta=0.05, k=32, n_max=1024",
                   "n_candidates": n, "n_tiles": n_tiles, "banding_tiles_ms": band_tiles_ms,
                   "banding_pairs_ms": band_ms, "banding_pairs_per_s": n / (band_tiles_ms * 1e-3)},
        "decisions": {"pruned": dec_counts[0], "accept_conc": dec_counts[1], "accept_nmax": dec_counts[2],
                      "mean_level": lvl_mean, "accepted_listed": n_acc, "by_level": by_level},
        "id_pairs": {"ms_per_step": ms_p, "value": n / (ms_p * 1e-3), "same_output_as_tiles": same_p,
                     "differing_codes": diff_p,
                     "note": "the same candidates as 8 B id pairs (bayeslsh_band_candidates) with the 16 B/object "
                             "prefix array: one 16-byte gather per side per candidate, survivors to the tail kernel",
                     "kernels": with_bytes(prof_p, per_p)},
        "exhaustive": {"ms_per_step": ms_ex, "value": n / (ms_ex * 1e-3), "speedup": ms_ex / ms, "same_output": same,
                       "differing_codes": diff_codes,
                       "mode": "REPLAY over id pairs, all 1024 bits of both object-major rows"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "sampled_parity": parity,
        "paper_context": PAPER_CONTEXT,
    }


def run_sweep(args, torch, P):
    """Synthetic analogs of the paper's experiments on the cosine tf-idf
    workload (100k documents, 16-band LSH candidates, 2048 SRP bits): exact
    similarity of every candidate as ground truth ("LSH"), the classical
    estimate over all hashes ("LSH Approx"), the pruning curve, gamma / delta /
    epsilon varied one at a time around 0.05 at t = 0.7 (time, recall, mean
    error, fraction of errors > 0.05), and BayesLSH vs BayesLSH-Lite by
    threshold."""
    from paper_1110_1328_amd import experiments as E
    corpus, x, y = build_workload(args.small)
    n = len(x)
    log("sweep workload: %d docs, %d candidates" % (corpus.n, n))
    ctx = P.bayeslsh_create(0)
    vec = P.csr_vectors(up(torch, corpus.offsets), up(torch, corpus.indices), up(torch, corpus.values), corpus.dim)
    cand = P.pairs(up(torch, x), up(torch, y))
    W = N_BITS // 32
    sig_om = torch.empty(corpus.n * W, dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_srp_sigs(ctx, vec, None, N_BITS, SRP_SEED, P.OBJECT_MAJOR, sig_om)
    sig_pf = torch.empty(corpus.n * (H // 32), dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_srp_sigs(ctx, vec, None, H, SRP_SEED, P.OBJECT_MAJOR, sig_pf)
    P.bayeslsh_sync(ctx)
    S = P.Signatures(sig_om, P.COSINE, P.OBJECT_MAJOR, corpus.n, N_BITS)
    S_pf = P.Signatures(sig_pf, P.COSINE, P.OBJECT_MAJOR, corpus.n, H)
    stream = torch.cuda.current_stream()
    truth, exact_ms = E.exact_truth(ctx, cand, vec, stream)
    log("exact similarity of every candidate (LSH): %.1f ms" % exact_ms)
    approx = E.lsh_approx(ctx, cand, S, truth, T, K, stream=stream)
    log("LSH Approx: %.2f ms, recall %.4f, mean error %.4f" % (approx["ms"], approx["recall"], approx["mean_error"]))
    # the paper's defaults: epsilon = gamma = 0.03, delta = 0.05
    res = P.make_result(n, n)
    ms = E._timed(ctx, lambda: P.bayeslsh_verify(ctx, cand, S, T, 0.03, 0.05, 0.03, (1.0, 1.0), K, res, stream),
                  max(3, args.steps // 10), stream)
    q = E.quality(*E.accepted_mask(res, n), truth, T)
    curve = E.pruning_curve(res.code[:n], K, N_BITS // K)
    log("BayesLSH t=%.1f: %.2f ms, recall %.4f, mean error %.4f" % (T, ms, q["recall"], q["mean_error"]))
    res_l = P.make_result(n, n)
    P.bayeslsh_lite_verify(ctx, cand, S_pf, vec, T, 0.03, (1.0, 1.0), H, K, res_l, stream)
    P.bayeslsh_sync(ctx, stream)
    curve_lite = E.pruning_curve(res_l.code[:n], K, H // K)
    sweep = E.parameter_sweep(ctx, cand, S, truth, T, K, stream=stream)
    for r in sweep:
        log("vary %-7s %.2f: %.2f ms, recall %.4f, mean error %.4f, errors > 0.05: %.4f" % (
            r["vary"], r["value"], r["ms"], r["recall"], r["mean_error"], r["frac_error_gt"]))
    by_t = E.threshold_sweep(ctx, cand, S, S_pf, vec, truth, (0.5, 0.6, 0.7, 0.8, 0.9), K, H, stream=stream)
    for r in by_t:
        log("t=%.1f: BayesLSH %.2f ms (recall %.4f), Lite %.2f ms (recall %.4f)" % (
            r["t"], r["bayeslsh_ms"], r["bayeslsh_recall"], r["lite_ms"], r["lite_recall"]))
    ctx.close()
    return {
        "metric": "candidate pairs verified/sec, BayesLSH vs exhaustive hash compare, same output",
        "value": n / (ms * 1e-3), "unit": "pairs/s", "n_gpus": 1, "ms_per_step": ms, "higher_is_better": True,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "experiment analogs: %d tf-idf documents, %d 16-band LSH candidates, 2048 SRP bits, "
                               "cosine t=%.1f, k=%d; Algorithm 1 at epsilon=gamma=0.03, delta=0.05" % (corpus.n, n, T, K)},
        "quality": q,
        "lsh_exact_ms": exact_ms,
        "lsh_approx": approx,
        "pruning_curve": [[nh, f] for nh, f in curve],
        "pruning_curve_lite": [[nh, f] for nh, f in curve_lite],
        "parameter_sweep": sweep,
        "by_threshold": by_t,
    }


def run_lite(args, torch, P):
    """The cosine BayesLSH-Lite workload: 100,000 sparse tf-idf vectors
    (dimension 2^20, Poisson(100) nonzeros, Zipf(1.1) terms, 5% planted
    near-duplicates), 2048 SRP bits per vector, candidates from 16-band x
    10-bit LSH banding on an independent projection (on the device, each
    bucket's pairs in 16 x 16 tiles of its members; timed apart from the step),
    t = 0.7, epsilon = 0.03, h = 128, k = 32, exact cosine on survivors.  One
    step = one bayeslsh_lite_verify call over all candidates.  Two exhaustive
    comparators with the same output: all 2048 bits of both object-major rows,
    and only the h = 128 bits Lite may use (all h/k level counts, no early
    exit) -- the second isolates the gain of Algorithm 2's early pruning.  The
    same candidates as bucket tiles (bayeslsh_band_tiles, 16 x 16 member tiles
    over the 128-bit object-major rows) are timed beside the step and must give
    the same output."""
    log("generating workload")
    from synth import generators as G
    corpus = G.tfidf_corpus(n_docs=20_000, seed=G.SEED_BASE + 2) if args.small else G.tfidf_corpus(seed=G.SEED_BASE + 2)
    ctx = P.bayeslsh_create(0)
    xd, yd, n, band_ms, tl, n_tiles, band_t_ms = lite_candidates(torch, P, ctx, corpus, args.small)
    x = xd.view(torch.int32).cpu().numpy().view(np.uint32)      # host copies for the oracle baseline
    y = yd.view(torch.int32).cpu().numpy().view(np.uint32)
    log("corpus %d docs, %d nnz; %d candidates (GPU banding: %.1f ms as pairs, %.1f ms as %d tiles)"
        % (corpus.n, len(corpus.indices), n, band_ms, band_t_ms, n_tiles))
    vec = P.csr_vectors(up(torch, corpus.offsets), up(torch, corpus.indices), up(torch, corpus.values), corpus.dim)
    W = N_BITS // 32
    sig_wm = torch.empty(corpus.n * W, dtype=torch.int32, device="cuda").view(torch.uint32)
    sig_om = torch.empty(corpus.n * W, dtype=torch.int32, device="cuda").view(torch.uint32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.bayeslsh_srp_sigs(ctx, vec, None, N_BITS, SRP_SEED, P.WORD_MAJOR, sig_wm)
    P.bayeslsh_sync(ctx)
    sig_ms = (time.perf_counter() - t0) * 1e3
    P.bayeslsh_srp_sigs(ctx, vec, None, N_BITS, SRP_SEED, P.OBJECT_MAJOR, sig_om)
    # Lite reads at most h bits: object-major rows of the first h bits (the plane of
    # hash b does not depend on how many hashes are generated, so these are the
    # first h bits of the full signatures)
    sig_pf = torch.empty(corpus.n * (H // 32), dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_srp_sigs(ctx, vec, None, H, SRP_SEED, P.OBJECT_MAJOR, sig_pf)
    P.bayeslsh_sync(ctx)
    log("signatures: %.1f ms for %d x %d bits" % (sig_ms, corpus.n, N_BITS))
    S_wm = P.Signatures(sig_wm, P.COSINE, P.WORD_MAJOR, corpus.n, N_BITS)
    S_om = P.Signatures(sig_om, P.COSINE, P.OBJECT_MAJOR, corpus.n, N_BITS)
    S_pf = P.Signatures(sig_pf, P.COSINE, P.OBJECT_MAJOR, corpus.n, H)
    S_run = S_pf if args.layout == "prefix" else S_wm
    same_prefix = bool(torch.equal(sig_pf.view(torch.int32).view(corpus.n, H // 32),
                                   sig_om.view(torch.int32).view(corpus.n, N_BITS // 32)[:, : H // 32]))
    cand = P.pairs(xd, yd)
    # the step runs over id pairs (Lite reads 128 bits: one 16-byte gather per
    # side); the same candidates as bucket tiles over the 128-bit object-major
    # rows are timed beside it (same output)
    tiles = False
    with_tiles = args.layout == "prefix"
    cand_t = P.tiles(tl, n_tiles, n)
    main_cand = cand
    cap = max(1 << 20, n // 100)
    res = P.make_result(n, cap)
    res_ex = P.make_result(n, cap)
    stream = torch.cuda.current_stream()

    def step():
        P.bayeslsh_lite_verify(ctx, main_cand, S_run, vec, T, EPS, (1.0, 1.0), H, K, res, stream)

    res_p = P.make_result(n, cap)

    def step_tiles():
        P.bayeslsh_lite_verify(ctx, cand_t, S_run, vec, T, EPS, (1.0, 1.0), H, K, res_p, stream)

    def step_ex():
        P.bayeslsh_exhaustive_verify(ctx, cand, S_om, vec, T, EPS, 0.5, 0.5, (1.0, 1.0), K, H, P.REPLAY_LITE, res_ex,
                                     stream)

    res_exh = P.make_result(n, cap)

    def step_ex_h():   # only the h bits Lite may use: all h/k level counts, no early exit
        P.bayeslsh_exhaustive_verify(ctx, cand, S_pf, vec, T, EPS, 0.5, 0.5, (1.0, 1.0), K, H, P.REPLAY_LITE, res_exh,
                                     stream)

    for _ in range(args.warmup):
        step()
    P.bayeslsh_sync(ctx, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    P.bayeslsh_sync(ctx, stream)
    ms_step = el * 1e3 / args.steps
    # per-kernel durations: HIP events around each launch on the same stream, in a
    # separate pass so that event creation does not enter the timed steps above
    P.bayeslsh_profile_enable(ctx, True)
    P.bayeslsh_profile_reset(ctx)
    for _ in range(args.steps):
        step()
    P.bayeslsh_sync(ctx, stream)
    k_ms, k_n = P.bayeslsh_profile_read(ctx, "verify_tiles" if tiles else "verify_bits")
    k_name = ("k_verify_bits, object-major 128-bit rows (one 16-byte gather per side); Lite survivors queued "
              "for k_exact" if args.layout == "prefix" else "k_verify_bits, word-major slabs, fused Lite exact")
    x_ms, x_n = P.bayeslsh_profile_read(ctx, "exact")   # exact similarity of the survivors
    f_ms, f_n = P.bayeslsh_profile_read(ctx, "flush")
    P.bayeslsh_profile_enable(ctx, False)
    log("BayesLSH-Lite: %.3f ms/step (verify kernel %.3f ms)" % (ms_step, k_ms / max(k_n, 1)))
    # the same candidates as bucket tiles: the 32 rows of a tile staged once
    ms_tiles, kt_ms, kt_n = None, 0.0, 0
    if with_tiles:
        for _ in range(2):
            step_tiles()
        P.bayeslsh_sync(ctx, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step_tiles()
        torch.cuda.synchronize()
        ms_tiles = (time.perf_counter() - t0) * 1e3 / args.steps
        P.bayeslsh_sync(ctx, stream)
        P.bayeslsh_profile_enable(ctx, True)
        P.bayeslsh_profile_reset(ctx)
        step_tiles()
        P.bayeslsh_sync(ctx, stream)
        kt_ms, kt_n = P.bayeslsh_profile_read(ctx, "verify_tiles")
        P.bayeslsh_profile_enable(ctx, False)
        log("BayesLSH-Lite over bucket tiles: %.3f ms/step (k_verify_tiles %.3f ms x %d)"
            % (ms_tiles, kt_ms / max(kt_n, 1), kt_n))
    # exhaustive comparators
    ex_steps = max(3, args.steps // 5)

    def timed_ex(fn):
        for _ in range(2):
            fn()
        P.bayeslsh_sync(ctx, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(ex_steps):
            fn()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        P.bayeslsh_sync(ctx, stream)
        return el * 1e3 / ex_steps

    ex_ms = timed_ex(step_ex)
    exh_ms = timed_ex(step_ex_h)
    log("exhaustive: %.3f ms/step over 2048 bits, %.3f ms/step over the h = %d bits" % (ex_ms, exh_ms, H))
    codes = res.code[:n].cpu().numpy()
    ia, va = res.accepted()

    def same_as(r):
        ib, vb = r.accepted()
        return bool(torch.equal(res.code[:n], r.code[:n])) and np.array_equal(ia, ib) and np.array_equal(va, vb)

    same = same_as(res_ex)
    same_h = same_as(res_exh)
    same_p = same_as(res_p) if with_tiles else None
    del res_ex, res_exh, res_p
    # m of every candidate, from a pass with m recorded (not timed)
    res_m = P.make_result(n, cap, m_debug=True)
    P.bayeslsh_lite_verify(ctx, main_cand, S_run, vec, T, EPS, (1.0, 1.0), H, K, res_m, stream)
    P.bayeslsh_sync(ctx, stream)
    assert bool(torch.equal(res_m.code[:n], res.code[:n]))
    gpu_m = res_m.m_debug[:n].view(torch.int16).cpu().numpy().view(np.uint16).astype(np.int32)
    del res_m
    dec, lvl = codes >> 6, codes & 63
    n_surv = int(np.sum(dec == 3))
    # Algorithmic bytes of the verify kernel per launch.  HBM stream: candidate ids
    # (8 B) and one code byte per candidate.  The signature bytes examined
    # (2 x k/8 B per level reached) come from a 1.6 MB array (prefix layout) or
    # 400 KB slabs (word-major) that stay in L2; the exact cosine of the rare
    # survivors reads their two sparse rows (~2 x 100 x 8 B).
    # (tiles: the 192 B descriptor per tile instead of 8 B of ids per candidate)
    hbm_bytes = n_tiles * 192 + n if tiles else n * 9
    gather_bytes = int(np.sum(lvl.astype(np.int64) + 1)) * 2 * (K // 8)
    k_avg_ms = k_ms / max(k_n, 1)
    per_step = max(k_n, 1) / args.steps                 # verify launches per step (candidate chunks)
    hbm_bytes = int(hbm_bytes / per_step)               # per launch
    gather_bytes = int(gather_bytes / per_step)
    # algorithmic bytes per launch: ids + code + both sides' chunk per level
    # reached (the survivors' exact cosines are computed by k_exact)
    alg_bytes = hbm_bytes + gather_bytes
    achieved = alg_bytes / (k_avg_ms * 1e-3) / 1e9
    traffic = measured_traffic() if args.layout == "prefix" else None
    out = {
        "metric": METRIC,
        "value": n / (ms_step * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": ("cosine BayesLSH-Lite: %d sparse tf-idf vectors (dim 2^20, Poisson(100) nnz, Zipf(1.1), 5%% "
                         "planted near-duplicates), 2048 SRP bits, 16-band LSH candidates (GPU banding, 16 x 16 "
                         "tiles per bucket), t=0.7, eps=0.03, h=128, k=32, exact FP64-accumulated cosine on "
                         "survivors" % corpus.n),
            "n_candidates": n,
            "n_tiles": n_tiles if tiles else None,
            "banding_ms": band_t_ms if tiles else band_ms,
            "banding_pairs_ms": band_ms,
            "survivors_after_h": n_surv,
            "accepted": int(len(ia)),
            "pruned_at_level": [int(np.sum((dec == 0) & (lvl == j))) for j in range(H // K)],
        },
        "bucket_tiles": {"ms_per_step": ms_tiles, "value": n / (ms_tiles * 1e-3) if ms_tiles else None,
                         "same_output": same_p, "n_tiles": n_tiles, "banding_ms": band_t_ms,
                         "kernel": "k_verify_tiles (Lite) + k_tiles_exact + flush",
                         "verify_kernel_ms": kt_ms / max(kt_n, 1), "launches": kt_n},
        "exhaustive": {"ms_per_step": ex_ms, "value": n / (ex_ms * 1e-3), "speedup": ex_ms / ms_step,
                       "same_output": same, "mode": "REPLAY_LITE, all 2048 bits per object"},
        "exhaustive_h_bits": {"ms_per_step": exh_ms, "value": n / (exh_ms * 1e-3), "speedup": exh_ms / ms_step,
                              "same_output": same_h,
                              "mode": "REPLAY_LITE over the h = 128 bits Lite may use (128-bit object-major "
                                      "rows): every level counted, no early exit, then the same decisions "
                                      "replayed -- the gain of Algorithm 2's pruning alone"},
        "signature_ms": sig_ms,
        "prefix_rows_equal_full_signature_prefix": same_prefix,
        "paper_context": PAPER_CONTEXT,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": k_name,
                     "kernel_ms": k_avg_ms, "kernel_launches_timed": k_n,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "bytes_model": ("per tile the 192 B descriptor, per candidate 1 B code + 8 B per level "
                                     "reached (4 B chunk per side at k = 32); survivors' exact cosines are "
                                     "k_tiles_exact's" if tiles else
                                     "per candidate 8 B ids + 1 B code + 8 B per level reached (4 B chunk per "
                                     "side at k = 32)"),
                     "hbm_stream_bytes_per_launch": hbm_bytes,
                     "stream_frac": hbm_bytes / (k_avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic_frac": traffic / (k_avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if traffic else None,
                     "exact_kernel_ms": x_ms / max(x_n, 1) if x_n else None,
                     "flush_kernel_ms": f_ms / max(f_n, 1) if f_n else None},
    }
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        cb, parity, _ = cpu_baseline(corpus, x, y, codes, gpu_m, (ia, va))
        out["cpu_baseline"] = cb
        out["full_size_parity"] = parity
        log("cpu baseline: %.3g pairs/s; parity %s" % (cb["value"], parity))
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--small", action="store_true", help="20k-document workload (quick check)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-calibration", action="store_true", help="time a plain 1 GiB device copy and exit")
    ap.add_argument("--layout", choices=["prefix", "word-major"], default="prefix",
                    help="SRP layout verified: object-major 128-bit rows (prefix) or word-major slabs of all bits")
    ap.add_argument("--workload", choices=["headline", "lite", "batched", "serving", "dense", "sweep", "sigs"],
                    default="headline",
                    help="headline (default): the dense line below, with the cosine BayesLSH-Lite line under its "
                         "own key; dense: GPU LSH banding of 1M dense vectors then Algorithm 1 over all ~2.4e9 "
                         "candidates; lite: the cosine BayesLSH-Lite line alone; batched: 4096 mixed query lists "
                         "in one graph launch vs the exhaustive batched comparator; serving: Poisson arrivals "
                         "against the dense cosine index, p50/p99 latency; sweep: the paper's experiments on the "
                         "tf-idf workload (pruning curve, gamma/delta/epsilon, BayesLSH vs Lite by threshold); "
                         "sigs: signature generation (dense SRP on MFMA, sparse SRP, minhash)")
    ap.add_argument("--no-lite", action="store_true", help="headline: skip the cosine BayesLSH-Lite leg")
    ap.add_argument("--cpu-sample", type=int, default=1 << 29,
                    help="dense: candidates in the seeded sample the oracle is timed on and compared over")
    ap.add_argument("--queries", type=int, default=10000, help="serving: number of queries")
    ap.add_argument("--serving-legs", choices=["all", "device"], default="all",
                    help="serving: all legs, or only the device-memory submissions (for a kernel trace)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1110_1328_amd as P

    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "batched":
        print(json.dumps(run_batched(args, torch, P)), flush=True)
        return
    if args.workload == "serving":
        print(json.dumps(run_serving(args, torch, P)), flush=True)
        return
    if args.workload == "dense":
        print(json.dumps(run_dense(args, torch, P)), flush=True)
        return
    if args.workload == "sweep":
        print(json.dumps(run_sweep(args, torch, P)), flush=True)
        return
    if args.workload == "sigs":
        print(json.dumps(run_sigs(args, torch, P)), flush=True)
        return
    if args.workload == "lite":
        print(json.dumps(run_lite(args, torch, P)), flush=True)
        return
    # default: the dense estimation workload is the headline line; the cosine
    # BayesLSH-Lite workload rides along under its own key
    out = run_dense(args, torch, P)
    torch.cuda.empty_cache()
    if not args.no_lite:
        try:
            out["cosine_lite_100k"] = run_lite(args, torch, P)
        except Exception as e:   # the headline stands on its own; the failure is reported, not hidden
            log("lite leg failed: %r" % (e,))
            out["cosine_lite_100k"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
