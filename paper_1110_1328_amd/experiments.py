"""Synthetic analogs of the paper's experiments (Section 5), on top of the C ABI.

* Pruning curve (Section 5, the pruning figure): the fraction of candidates
  still undecided after each k hashes.
* Parameter sweep (Section 5, the parameter figure and its table): gamma,
  delta and epsilon varied one at a time while the other two stay at a base
  value; for each setting the verification time, recall against the exact
  similarities, mean estimation error and the fraction of estimates off by
  more than 0.05.
* BayesLSH vs BayesLSH-Lite by threshold (Section 5, observation 3 of the
  results): time and recall of both at several thresholds.
* The paper's two LSH baselines: "LSH" (exact similarity of every candidate)
  and "LSH Approx" (the classical estimate m/n over all hashes).

Every verification here is a library call; the statistics are reductions of
its outputs (codes, accepted lists) against the exact similarities, on the
device.  Ground truth is bayeslsh_exact_similarity of every candidate.
"""
from __future__ import annotations

import time

import torch

from . import api as P


def exact_truth(ctx, cand: P.Candidates, vectors: P.Vectors, stream=None) -> tuple[torch.Tensor, float]:
    """Exact similarity of every candidate (FP64, on the device) and the time
    the call took in ms ("LSH" in the paper's comparisons)."""
    n = cand.count
    out = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream() if stream is None else stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.bayeslsh_exact_similarity(ctx, cand, vectors, out, s)
    P.bayeslsh_sync(ctx, s)
    return out[:n], (time.perf_counter() - t0) * 1e3


def accepted_mask(res: P.Result, n: int) -> tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
    """(mask over candidates, accepted indices, accepted values) of a result
    whose list did not overflow."""
    na = int(res.n_accepted.item())
    if na > res.acc_idx.numel():
        raise ValueError("accepted list truncated (%d > %d)" % (na, res.acc_idx.numel()))
    idx = res.acc_idx[:na].view(torch.int64)
    val = res.acc_val[:na].to(torch.float64)
    mask = torch.zeros(n, dtype=torch.bool, device=res.code.device)
    mask[idx] = True
    return mask, idx, val


def quality(mask: torch.Tensor, idx: torch.Tensor, val: torch.Tensor, truth: torch.Tensor, t: float,
            err_bound: float = 0.05) -> dict:
    """Output quality against exact similarities: positives are the candidates
    with similarity >= t; recall = accepted positives / positives; errors
    |value - similarity| over the accepted pairs."""
    pos = truth >= t
    n_pos = int(pos.sum().item())
    n_found = int((pos & mask).sum().item())
    err = (val - truth[idx]).abs()
    n_acc = int(idx.numel())
    return {
        "positives": n_pos,
        "accepted": n_acc,
        "accepted_positives": n_found,
        "recall": n_found / n_pos if n_pos else 1.0,
        "false_positives": n_acc - n_found,
        "mean_error": float(err.mean().item()) if n_acc else 0.0,
        "max_error": float(err.max().item()) if n_acc else 0.0,
        "frac_error_gt": float((err > err_bound).double().mean().item()) if n_acc else 0.0,
        "error_bound": err_bound,
    }


def pruning_curve(code: torch.Tensor, k: int, n_levels: int) -> list[tuple[int, float]]:
    """[(n hashes compared, fraction of candidates still undecided after
    them)] for n = k, 2k, ..., n_levels k, from the per-candidate codes
    (decision << 6 | level of the decision)."""
    n = code.numel()
    lvl = (code & 63).to(torch.int64)
    hist = torch.bincount(lvl, minlength=n_levels)[:n_levels].cpu().tolist()
    out, decided = [], 0
    for j in range(n_levels):
        decided += hist[j]
        out.append(((j + 1) * k, (n - decided) / n if n else 0.0))
    return out


def _timed(ctx, fn, steps: int, stream) -> float:
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


def parameter_sweep(ctx, cand: P.Candidates, sigs: P.Signatures, truth: torch.Tensor, t: float, k: int,
                    values=(0.01, 0.03, 0.05, 0.07, 0.09), base: float = 0.05, steps: int = 3,
                    stream=None, capacity: int | None = None) -> list[dict]:
    """Algorithm 1 with gamma, delta, epsilon varied one at a time (the other
    two at `base`): one row per setting with its time and output quality."""
    n = cand.count
    s = torch.cuda.current_stream() if stream is None else stream
    res = P.make_result(n, capacity or n)
    rows = []
    for which in ("gamma", "delta", "epsilon"):
        for v in values:
            p = {"gamma": base, "delta": base, "epsilon": base, which: v}
            ms = _timed(ctx, lambda: P.bayeslsh_verify(ctx, cand, sigs, t, p["epsilon"], p["delta"], p["gamma"],
                                                       (1.0, 1.0), k, res, s), steps, s)
            mask, idx, val = accepted_mask(res, n)
            rows.append({"vary": which, "value": v, **p, "ms": ms, **quality(mask, idx, val, truth, t)})
    return rows


def lsh_approx(ctx, cand: P.Candidates, sigs_om: P.Signatures, truth: torch.Tensor, t: float, k: int,
               steps: int = 3, stream=None, capacity: int | None = None) -> dict:
    """The classical estimate m/n over all n_max hashes, emitted if >= t
    ("LSH Approx"): time and output quality."""
    n = cand.count
    s = torch.cuda.current_stream() if stream is None else stream
    res = P.make_result(n, capacity or n)
    ms = _timed(ctx, lambda: P.bayeslsh_exhaustive_verify(ctx, cand, sigs_om, None, t, 0.5, 0.5, 0.5, (1.0, 1.0), k,
                                                          0, P.MLE, res, s), steps, s)
    mask, idx, val = accepted_mask(res, n)
    return {"ms": ms, **quality(mask, idx, val, truth, t)}


def threshold_sweep(ctx, cand: P.Candidates, sigs: P.Signatures, lite_sigs: P.Signatures, vectors: P.Vectors,
                    truth: torch.Tensor, thresholds, k: int, h: int, epsilon: float = 0.03, delta: float = 0.05,
                    gamma: float = 0.03, steps: int = 3, stream=None, capacity: int | None = None) -> list[dict]:
    """BayesLSH (Algorithm 1) and BayesLSH-Lite (Algorithm 2, h hashes) at
    each threshold: time, recall and accepted counts of both."""
    n = cand.count
    s = torch.cuda.current_stream() if stream is None else stream
    res = P.make_result(n, capacity or n)
    rows = []
    for t in thresholds:
        ms_b = _timed(ctx, lambda: P.bayeslsh_verify(ctx, cand, sigs, t, epsilon, delta, gamma, (1.0, 1.0), k, res, s),
                      steps, s)
        qb = quality(*accepted_mask(res, n), truth, t)
        ms_l = _timed(ctx, lambda: P.bayeslsh_lite_verify(ctx, cand, lite_sigs, vectors, t, epsilon, (1.0, 1.0), h, k,
                                                          res, s), steps, s)
        ql = quality(*accepted_mask(res, n), truth, t)
        rows.append({"t": t, "bayeslsh_ms": ms_b, "bayeslsh_recall": qb["recall"], "bayeslsh_accepted": qb["accepted"],
                     "bayeslsh_mean_error": qb["mean_error"], "lite_ms": ms_l, "lite_recall": ql["recall"],
                     "lite_accepted": ql["accepted"], "positives": qb["positives"]})
    return rows
