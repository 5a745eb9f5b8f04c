"""Helpers shared by the GPU parity tests: upload seeded inputs, run the HIP
path through the C ABI, and compare its outputs with the oracle's."""
from __future__ import annotations

import numpy as np
import torch

import paper_1110_1328_amd as P
from oracle import reference as R

DEV = "cuda"


_SIGNED = {np.dtype(np.uint32): (np.int32, torch.uint32), np.dtype(np.uint64): (np.int64, torch.uint64),
           np.dtype(np.uint16): (np.int16, torch.uint16)}


def up(a: np.ndarray) -> torch.Tensor:
    """Host array -> device tensor (unsigned types travel as same-width signed views)."""
    a = np.ascontiguousarray(a)
    if a.dtype in _SIGNED:
        sd, td = _SIGNED[a.dtype]
        return torch.from_numpy(a.view(sd)).to(DEV).view(td)
    return torch.from_numpy(a).to(DEV)


def down(t: torch.Tensor) -> np.ndarray:
    back = {torch.uint32: (torch.int32, np.uint32), torch.uint64: (torch.int64, np.uint64),
            torch.uint16: (torch.int16, np.uint16)}
    if t.dtype in back:
        sd, nd = back[t.dtype]
        return t.view(sd).cpu().numpy().view(nd)
    return t.cpu().numpy()


def sigs_tensor(sig_obj_major: np.ndarray, measure: int, layout: int, n_max: int = 0) -> P.Signatures:
    """Signature rows [n_obj][row] (minhash hashes or SRP words) on the device."""
    n_obj, row = sig_obj_major.shape
    n_hashes = row if measure == P.JACCARD else 32 * row
    data = sig_obj_major if layout == P.OBJECT_MAJOR else np.ascontiguousarray(sig_obj_major.T)
    return P.Signatures(up(data.astype(np.uint32)), measure, layout, n_obj, n_hashes, n_max)


def decode_result(res: P.Result, n: int):
    code = res.code[:n].cpu().numpy()
    dec, lvl = code >> 6, code & 63
    m = down(res.m_debug[:n]).astype(np.int32) if res.m_debug is not None else None
    idx, val = res.accepted()
    return dict(code=code, decision=dec, level=lvl, m=m, acc_idx=idx, acc_val=val,
                n_accepted=int(res.n_accepted.item()))


def assert_same_as_oracle(got: dict, want: dict, shat_tol: float = 1e-6, lite_exact: np.ndarray | None = None):
    """Decisions, levels and m bit-exact; the accepted set identical; values within tolerance."""
    np.testing.assert_array_equal(got["decision"], want["decision"])
    np.testing.assert_array_equal(got["level"], want["level"])
    if got["m"] is not None:
        np.testing.assert_array_equal(got["m"], want["m"])
    if lite_exact is None:
        acc = np.flatnonzero((want["decision"] == R.DEC_CONC) | (want["decision"] == R.DEC_NMAX))
        np.testing.assert_array_equal(got["acc_idx"], acc)
        np.testing.assert_allclose(got["acc_val"], want["shat"][acc], atol=shat_tol, rtol=0)
    else:
        acc = np.flatnonzero(want["accepted"])
        np.testing.assert_array_equal(got["acc_idx"], acc)
        np.testing.assert_allclose(got["acc_val"], lite_exact[acc], atol=shat_tol, rtol=0)
    assert got["n_accepted"] == len(acc)


def sets_device(sets) -> P.Vectors:
    return P.set_vectors(up(sets.offsets), up(sets.elems.astype(np.uint32)), sets.vocab)


def csr_device(corpus) -> P.Vectors:
    return P.csr_vectors(up(corpus.offsets), up(corpus.indices.astype(np.uint32)), up(corpus.values), corpus.dim)
