"""Python binding of libbayeslsh.so: argument marshalling only.

Functions carry the C names.  Device memory is held in torch tensors; each
helper checks dtype, device and contiguity, fills the ctypes struct of the
header with raw pointers, and calls the library on the current torch stream
(or the stream passed in).  Every computation happens in the HIP library.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import torch

from . import _abi as A
from ._abi import (ACCEPT_CONC, ACCEPT_NMAX, ALL_PAIRS, COSINE, CSR, DENSE, JACCARD, LITE_EXACT, MLE,  # noqa: F401
                   OBJECT_MAJOR, PAIRS, PRUNED, QUERY_LISTS, REPLAY, REPLAY_LITE, SETS, SRP_PLANES_Q16, TILES,
                   WORD_MAJOR)


class BayesLSHError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (A.STATUS_NAMES.get(code, str(code)), msg))
        self.code = code


def _lib():
    return A.load()


def _check(rc: int) -> int:
    if rc != A.OK:
        msg = _lib().bayeslsh_last_error()
        raise BayesLSHError(rc, msg.decode() if msg else "")
    return rc


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _dev(t: torch.Tensor, dtype, name: str):
    if t is None:
        return None
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _cached(obj, build, *tensors):
    """Rebuild the ctypes struct only when a tensor (or scalar field) changed."""
    key = tuple(t.data_ptr() if isinstance(t, torch.Tensor) else t for t in tensors)
    c = obj.__dict__.get("_cstruct")
    if c is not None and c[0] == key:
        return c[1]
    st = build()
    obj.__dict__["_cstruct"] = (key, st)
    return st


# ---------------------------------------------------------------------------
# argument holders (keep the tensors alive next to their structs)
# ---------------------------------------------------------------------------
@dataclass
class Signatures:
    data: torch.Tensor
    measure: int
    layout: int
    n_obj: int
    n_hashes: int
    n_max: int = 0
    prefix: torch.Tensor = None   # SRP: optional [n_obj][4] words = hashes 0..127 of every object

    def struct(self):
        return _cached(self, self._build, self.data, self.measure, self.layout, self.n_obj, self.n_hashes, self.n_max,
                       self.prefix)

    def _build(self):
        _dev(self.data, torch.int32 if self.data.dtype == torch.int32 else torch.uint32, "signature data")
        if self.prefix is not None:
            _dev(self.prefix, torch.int32 if self.prefix.dtype == torch.int32 else torch.uint32, "signature prefix")
            if self.prefix.numel() < 4 * self.n_obj:
                raise ValueError("signature prefix holds %d words for %d objects" % (self.prefix.numel(), self.n_obj))
        return A.Sigs(self.measure, self.layout, _p(self.data), self.n_obj, self.n_hashes, self.n_max,
                      _p(self.prefix))


@dataclass
class Candidates:
    kind: int
    x: torch.Tensor = None
    y: torch.Tensor = None
    query: torch.Tensor = None
    offsets: torch.Tensor = None
    cand: torch.Tensor = None
    n_cand: int = 0
    all_n: int = 0
    tiles: torch.Tensor = None
    n_tiles: int = 0

    @property
    def count(self) -> int:
        if self.kind == PAIRS:
            return int(self.x.numel())
        if self.kind in (QUERY_LISTS, TILES):
            return int(self.n_cand)
        return self.all_n * (self.all_n - 1) // 2

    def struct(self):
        return _cached(self, self._build, self.kind, self.x, self.y, self.query, self.offsets, self.cand, self.n_cand,
                       self.all_n, self.tiles, self.n_tiles)

    def _build(self):
        c = A.Candidates()
        c.kind = self.kind
        if self.kind == PAIRS:
            _dev(self.x, torch.uint32, "x")
            _dev(self.y, torch.uint32, "y")
            if self.x.numel() != self.y.numel():
                raise ValueError("x and y differ in length")
            c.x, c.y, c.n_pairs = _p(self.x), _p(self.y), self.x.numel()
        elif self.kind == QUERY_LISTS:
            _dev(self.query, torch.uint32, "query")
            _dev(self.offsets, torch.int64, "offsets")
            _dev(self.cand, torch.uint32, "cand")
            c.query, c.offsets, c.cand = _p(self.query), _p(self.offsets), _p(self.cand)
            c.n_lists, c.n_cand = self.query.numel(), self.n_cand
        elif self.kind == TILES:
            if self.tiles.device.type != "cuda" or not self.tiles.is_contiguous():
                raise ValueError("tiles: contiguous device tensor expected")
            if self.tiles.numel() * self.tiles.element_size() < self.n_tiles * A.TILE_BYTES:
                raise ValueError("tiles: tensor smaller than n_tiles descriptors")
            c.tiles, c.n_tiles, c.n_cand = _p(self.tiles), self.n_tiles, self.n_cand
        else:
            c.all_n = self.all_n
        return c


def tiles(tiles_buf: torch.Tensor, n_tiles: int, n_cand: int) -> Candidates:
    """BLSH_TILES candidates from bayeslsh_band_tiles' output (tiles_buf: a
    device tensor holding n_tiles 192-byte descriptors, 16-byte aligned)."""
    return Candidates(TILES, tiles=tiles_buf, n_tiles=int(n_tiles), n_cand=int(n_cand))


def pairs(x: torch.Tensor, y: torch.Tensor) -> Candidates:
    return Candidates(PAIRS, x=x, y=y)


def query_lists(query: torch.Tensor, offsets: torch.Tensor, cand: torch.Tensor, n_cand: int | None = None) -> Candidates:
    return Candidates(QUERY_LISTS, query=query, offsets=offsets, cand=cand,
                      n_cand=int(cand.numel()) if n_cand is None else int(n_cand))


def all_pairs(n: int) -> Candidates:
    return Candidates(ALL_PAIRS, all_n=int(n))


@dataclass
class Vectors:
    kind: int
    n_obj: int
    dim: int
    dense: torch.Tensor = None
    offsets: torch.Tensor = None
    indices: torch.Tensor = None
    values: torch.Tensor = None

    def struct(self):
        return _cached(self, self._build, self.kind, self.n_obj, self.dim, self.dense, self.offsets, self.indices,
                       self.values)

    def _build(self):
        if self.kind == DENSE:
            _dev(self.dense, torch.float32, "dense")
        else:
            _dev(self.offsets, torch.int64, "offsets")
            _dev(self.indices, torch.uint32, "indices")
            if self.kind == CSR:
                _dev(self.values, torch.float32, "values")
        return A.Vectors(self.kind, self.n_obj, self.dim, _p(self.dense), _p(self.offsets), _p(self.indices),
                         _p(self.values))


def dense_vectors(x: torch.Tensor) -> Vectors:
    return Vectors(DENSE, x.shape[0], x.shape[1], dense=x)


def csr_vectors(offsets, indices, values, dim) -> Vectors:
    return Vectors(CSR, offsets.numel() - 1, int(dim), offsets=offsets, indices=indices, values=values)


def set_vectors(offsets, indices, dim) -> Vectors:
    return Vectors(SETS, offsets.numel() - 1, int(dim), offsets=offsets, indices=indices)


@dataclass
class Result:
    code: torch.Tensor
    acc_idx: torch.Tensor
    acc_val: torch.Tensor
    n_accepted: torch.Tensor
    m_debug: torch.Tensor = None
    _s: object = field(default=None, repr=False)

    def struct(self):
        return _cached(self, self._build, self.code, self.acc_idx, self.acc_val, self.n_accepted, self.m_debug)

    def _build(self):
        _dev(self.code, torch.uint8, "code")
        _dev(self.acc_idx, torch.uint64, "acc_idx")
        _dev(self.acc_val, torch.float32, "acc_val")
        _dev(self.n_accepted, torch.int64, "n_accepted")
        _dev(self.m_debug, torch.uint16, "m_debug")
        return A.Result(_p(self.code), _p(self.acc_idx), _p(self.acc_val), self.acc_idx.numel(),
                        _p(self.n_accepted), _p(self.m_debug))

    def accepted(self):
        """(idx, val) of the output set on the host, sorted by candidate index."""
        n = min(int(self.n_accepted.item()), self.acc_idx.numel())
        idx = self.acc_idx[:n].view(torch.int64).cpu().numpy()
        val = self.acc_val[:n].cpu().numpy()
        o = idx.argsort(kind="stable")
        return idx[o], val[o]


def make_result(n_cand: int, capacity: int, device="cuda", m_debug: bool = False) -> Result:
    return Result(code=torch.empty(max(n_cand, 1), dtype=torch.uint8, device=device),
                  acc_idx=torch.empty(max(capacity, 1), dtype=torch.int64, device=device).view(torch.uint64),
                  acc_val=torch.empty(max(capacity, 1), dtype=torch.float32, device=device),
                  n_accepted=torch.zeros(1, dtype=torch.int64, device=device),
                  m_debug=(torch.empty(max(n_cand, 1), dtype=torch.int16, device=device).view(torch.uint16)
                           if m_debug else None))


def decode(code):
    """code byte -> (decision, level); 0xFF marks a bad object id."""
    return code >> 6, code & 63


# ---------------------------------------------------------------------------
# context and entry points (C names)
# ---------------------------------------------------------------------------
class Context:
    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(_lib().bayeslsh_create(C.byref(h), device))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            _lib().bayeslsh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bayeslsh_create(device: int = 0) -> Context:
    return Context(device)


def bayeslsh_destroy(ctx: Context) -> None:
    ctx.close()


def bayeslsh_version() -> int:
    return _lib().bayeslsh_version()


def bayeslsh_sync(ctx: Context, stream=None) -> int:
    return _check(_lib().bayeslsh_sync(ctx.handle, _stream(stream)))


def bayeslsh_profile_enable(ctx: Context, enable: bool = True):
    _check(_lib().bayeslsh_profile_enable(ctx.handle, int(enable)))


def bayeslsh_profile_reset(ctx: Context):
    _check(_lib().bayeslsh_profile_reset(ctx.handle))


def bayeslsh_profile_read(ctx: Context, name: str):
    ms, n = C.c_double(), C.c_int64()
    _check(_lib().bayeslsh_profile_read(ctx.handle, name.encode(), C.byref(ms), C.byref(n)))
    return ms.value, n.value


def bayeslsh_set_tuning(ctx: Context, gather: int = 0, batch_inreg: int = 0, batch_blocks_per_cu: int = 0,
                        batch_spill_cap: int = 0, acc_stage_cap: int = 0, batch_srp_tile: int = 0,
                        batch_mh_tile: int = 0, tiles_accept_bitmask: int = 0, tiles_per_launch: int = 0):
    t = A.Tuning()
    t.gather, t.batch_inreg, t.batch_blocks_per_cu, t.batch_spill_cap = gather, batch_inreg, batch_blocks_per_cu, batch_spill_cap
    t.acc_stage_cap = acc_stage_cap
    t.batch_srp_tile, t.batch_mh_tile = batch_srp_tile, batch_mh_tile
    t.tiles_accept_bitmask = tiles_accept_bitmask
    t.tiles_per_launch = tiles_per_launch
    _check(_lib().bayeslsh_set_tuning(ctx.handle, C.byref(t)))


def bayeslsh_get_tuning(ctx: Context) -> dict:
    t = A.Tuning()
    _check(_lib().bayeslsh_get_tuning(ctx.handle, C.byref(t)))
    return {name: getattr(t, name) for name, _ in A.Tuning._fields_}


def bayeslsh_reserve_workspace(ctx: Context, n_bytes: int, fixed: bool = False):
    _check(_lib().bayeslsh_reserve_workspace(ctx.handle, int(n_bytes), int(bool(fixed))))


def bayeslsh_workspace_bytes(ctx: Context) -> int:
    n = C.c_size_t()
    _check(_lib().bayeslsh_workspace_bytes(ctx.handle, C.byref(n)))
    return n.value


LIST_DTYPE = None


def list_descs(measure, t, query, offset, length):
    """Host array of blsh_list_desc built from per-list columns (numpy, zero-copy into the call)."""
    import numpy as np
    global LIST_DTYPE
    if LIST_DTYPE is None:
        f = A.ListDesc
        LIST_DTYPE = np.dtype({"names": ["measure", "t", "query", "offset", "length"],
                               "formats": [np.int32, np.float64, np.uint32, np.int64, np.int64],
                               "offsets": [f.measure.offset, f.t.offset, f.query.offset, f.offset.offset,
                                           f.length.offset],
                               "itemsize": C.sizeof(f)})
    n = len(query)
    arr = np.zeros(n, LIST_DTYPE)
    arr["measure"], arr["t"], arr["query"], arr["offset"], arr["length"] = measure, t, query, offset, length
    return arr


def _k_pair(k):
    """k: one value for both measures or a (k_jaccard, k_cosine) pair; 0 = autotune."""
    if isinstance(k, (tuple, list)):
        return int(k[0]), int(k[1])
    return int(k), int(k)


def bayeslsh_verify_batched(ctx: Context, lists, cand: torch.Tensor, jaccard_sigs: Signatures | None,
                            cosine_sigs: Signatures | None, epsilon, delta, gamma, prior=(1.0, 1.0), k=32,
                            res: Result = None, stream=None) -> tuple:
    """lists: array from list_descs(); k: int or (k_jaccard, k_cosine), 0 = autotune.
    Returns the (k_jaccard, k_cosine) used."""
    import numpy as np
    _dev(cand, torch.uint32, "cand")
    lists = np.ascontiguousarray(lists)
    if lists.dtype != LIST_DTYPE:
        raise TypeError("lists must come from list_descs()")
    if res.code.numel() < cand.numel():
        raise ValueError("result.code smaller than cand")
    js = jaccard_sigs.struct() if jaccard_sigs is not None else None
    cs = cosine_sigs.struct() if cosine_sigs is not None else None
    rs = res.struct()
    k_used = (C.c_int32 * 2)()
    kj, kc = _k_pair(k)
    _check(_lib().bayeslsh_verify_batched(ctx.handle, lists.ctypes.data_as(C.POINTER(A.ListDesc)), len(lists),
                                          _p(cand), cand.numel(), C.byref(js) if js is not None else None,
                                          C.byref(cs) if cs is not None else None, epsilon, delta, gamma,
                                          _prior(prior), kj, kc, k_used, C.byref(rs), _stream(stream)))
    return int(k_used[0]), int(k_used[1])


def bayeslsh_posterior_table(ctx, measure, t, epsilon, delta, gamma, prior=(1.0, 1.0), k=32, n_levels=8,
                             lite=False):
    """ctx may be None (host-only build, no GPU needed)."""
    import numpy as np
    words = (k * n_levels + 1 + 31) // 32
    mm = np.zeros(n_levels, np.int32)
    acc = np.zeros(n_levels * words, np.uint32)
    margin = C.c_double()
    _check(_lib().bayeslsh_posterior_table(ctx.handle if ctx is not None else None, measure, t, epsilon, delta, gamma, A.Prior(*prior), k,
                                           n_levels, int(lite), mm.ctypes.data_as(C.c_void_p),
                                           acc.ctypes.data_as(C.c_void_p), C.byref(margin)))
    return mm, acc.reshape(n_levels, words), margin.value


def bayeslsh_minhash_sigs(ctx: Context, sets: Vectors, a: torch.Tensor, b: torch.Tensor, out: torch.Tensor,
                          stream=None):
    _dev(a, torch.uint32, "a")
    _dev(b, torch.uint32, "b")
    _dev(out, torch.uint32, "sigs_out")
    if out.numel() < sets.n_obj * a.numel():
        raise ValueError("sigs_out too small")
    v = sets.struct()
    _check(_lib().bayeslsh_minhash_sigs(ctx.handle, C.byref(v), _p(a), _p(b), a.numel(), _p(out), _stream(stream)))
    return out


def bayeslsh_srp_sigs(ctx: Context, vecs: Vectors, planes, n_bits: int, seed: int, layout: int, out: torch.Tensor,
                      stream=None, flags: int = 0):
    """flags: 0 or SRP_PLANES_Q16 (generated plane entries in 2 bytes)."""
    _dev(out, torch.uint32, "bits_out")
    if planes is not None:
        _dev(planes, torch.float32, "planes")
    if out.numel() < vecs.n_obj * (n_bits // 32):
        raise ValueError("bits_out too small")
    v = vecs.struct()
    _check(_lib().bayeslsh_srp_sigs(ctx.handle, C.byref(v), _p(planes), n_bits, seed, layout, flags, _p(out),
                                    _stream(stream)))
    return out


_PRIORS = {}


def _prior(prior):
    prior = tuple(prior)
    p = _PRIORS.get(prior)
    if p is None:
        p = _PRIORS[prior] = A.Prior(*prior)
    return p


def _check_result_size(res: Result, cand: Candidates):
    if res.code.numel() < cand.count:
        raise ValueError("result.code holds %d bytes for %d candidates" % (res.code.numel(), cand.count))
    if res.m_debug is not None and res.m_debug.numel() < cand.count:
        raise ValueError("result.m_debug too small")


def bayeslsh_verify(ctx: Context, cand: Candidates, sigs: Signatures, t, epsilon, delta, gamma, prior=(1.0, 1.0),
                    k=32, res: Result = None, stream=None):
    _check_result_size(res, cand)
    cs, ss, rs = cand.struct(), sigs.struct(), res.struct()
    _check(_lib().bayeslsh_verify(ctx.handle, C.byref(cs), C.byref(ss), t, epsilon, delta, gamma, _prior(prior), k,
                                  C.byref(rs), _stream(stream)))
    return res


def bayeslsh_verify_noalloc(ctx: Context, cand: Candidates, sigs: Signatures, t, epsilon, delta, gamma,
                            prior=(1.0, 1.0), k=32, res: Result = None, stream=None):
    """bayeslsh_verify without device allocation inside the call (its scratch is
    the library's fixed per-GPU array); same output."""
    _check_result_size(res, cand)
    cs, ss, rs = cand.struct(), sigs.struct(), res.struct()
    _check(_lib().bayeslsh_verify_noalloc(ctx.handle, C.byref(cs), C.byref(ss), t, epsilon, delta, gamma,
                                          _prior(prior), k, C.byref(rs), _stream(stream)))
    return res


def bayeslsh_lite_verify(ctx: Context, cand: Candidates, sigs: Signatures, exact: Vectors, t, epsilon,
                         prior=(1.0, 1.0), h=128, k=32, res: Result = None, stream=None):
    _check_result_size(res, cand)
    cs, ss, vs, rs = cand.struct(), sigs.struct(), exact.struct(), res.struct()
    _check(_lib().bayeslsh_lite_verify(ctx.handle, C.byref(cs), C.byref(ss), C.byref(vs), t, epsilon,
                                       _prior(prior), h, k, C.byref(rs), _stream(stream)))
    return res


def bayeslsh_exact_similarity(ctx: Context, cand: Candidates, vecs: Vectors, out: torch.Tensor = None,
                              stream=None) -> torch.Tensor:
    """Exact similarity of every candidate (FP64 device tensor of cand.count)."""
    if out is None:
        out = torch.empty(max(cand.count, 1), dtype=torch.float64, device="cuda")
    _dev(out, torch.float64, "sim_out")
    if out.numel() < cand.count:
        raise ValueError("sim_out too small")
    cs, vs = cand.struct(), vecs.struct()
    _check(_lib().bayeslsh_exact_similarity(ctx.handle, C.byref(cs), C.byref(vs), _p(out), _stream(stream)))
    return out


def bayeslsh_band_candidates(ctx: Context, band_sigs: Signatures, n_bands: int, band_bits: int, capacity: int,
                             max_bucket: int = 0, x_out: torch.Tensor = None, y_out: torch.Tensor = None,
                             stream=None, order_tile: int = 16):
    """LSH banding on the device.  Returns (x, y, n_pairs, truncated): uint32
    device tensors of `capacity` entries, the first min(n_pairs, capacity) valid.
    order_tile: 16 (16 x 16 tiles of each bucket's members, the default: the
    faster order to band and to verify) or 0 (row-major pairs per bucket)."""
    if x_out is None:
        x_out = torch.empty(max(capacity, 1), dtype=torch.int32, device="cuda").view(torch.uint32)
    if y_out is None:
        y_out = torch.empty(max(capacity, 1), dtype=torch.int32, device="cuda").view(torch.uint32)
    _dev(x_out, torch.uint32, "x_out")
    _dev(y_out, torch.uint32, "y_out")
    if x_out.numel() < capacity or y_out.numel() < capacity:
        raise ValueError("outputs smaller than capacity")
    st = band_sigs.struct()
    n = C.c_int64(0)
    rc = _lib().bayeslsh_band_candidates(ctx.handle, C.byref(st), n_bands, band_bits, max_bucket, order_tile,
                                         _p(x_out), _p(y_out), capacity, C.byref(n), _stream(stream))
    if rc == A.ETRUNCATED:
        return x_out, y_out, n.value, True
    _check(rc)
    return x_out, y_out, n.value, False


def bayeslsh_band_tiles(ctx: Context, band_sigs: Signatures, n_bands: int, band_bits: int, tile_capacity: int,
                        max_bucket: int = 0, tiles_out: torch.Tensor = None, stream=None):
    """LSH banding as bucket tiles (the order_tile = 16 candidates, same
    numbering).  Returns (tiles, n_tiles, n_pairs, truncated): tiles an int64
    device tensor of tile_capacity 192-byte descriptors (24 int64 each); pass
    tiles(tiles, n_tiles, n_pairs) to bayeslsh_verify."""
    words = A.TILE_BYTES // 8
    if tiles_out is None:
        tiles_out = torch.empty(max(tile_capacity, 1) * words, dtype=torch.int64, device="cuda")
    if tiles_out.numel() * tiles_out.element_size() < tile_capacity * A.TILE_BYTES:
        raise ValueError("tiles_out smaller than tile_capacity descriptors")
    st = band_sigs.struct()
    nt, npairs = C.c_int64(0), C.c_int64(0)
    rc = _lib().bayeslsh_band_tiles(ctx.handle, C.byref(st), n_bands, band_bits, max_bucket, _p(tiles_out),
                                    tile_capacity, C.byref(nt), C.byref(npairs), _stream(stream))
    if rc == A.ETRUNCATED:
        return tiles_out, nt.value, npairs.value, True
    _check(rc)
    return tiles_out, nt.value, npairs.value, False


def bayeslsh_fit_prior(sims) -> tuple:
    """Method-of-moments Beta prior from a host sample of similarities:
    returns ((alpha, beta), fell_back_to_uniform)."""
    import numpy as np
    s = np.ascontiguousarray(sims, dtype=np.float64)
    pr = A.Prior()
    uni = C.c_int32(0)
    _check(_lib().bayeslsh_fit_prior(s.ctypes.data_as(C.c_void_p), len(s), C.byref(pr), C.byref(uni)))
    return (pr.alpha, pr.beta), bool(uni.value)


def bayeslsh_exhaustive_verify(ctx: Context, cand: Candidates, sigs: Signatures, exact: Vectors | None, t, epsilon,
                               delta, gamma, prior=(1.0, 1.0), k=32, h=0, mode=REPLAY, res: Result = None,
                               stream=None):
    _check_result_size(res, cand)
    cs, ss, rs = cand.struct(), sigs.struct(), res.struct()
    vs = exact.struct() if exact is not None else None
    _check(_lib().bayeslsh_exhaustive_verify(ctx.handle, C.byref(cs), C.byref(ss),
                                             C.byref(vs) if vs is not None else None, t, epsilon, delta, gamma,
                                             A.Prior(*prior), k, h, mode, C.byref(rs), _stream(stream)))
    return res


def bayeslsh_exhaustive_batched(ctx: Context, lists, cand: torch.Tensor, jaccard_sigs: Signatures | None,
                                cosine_sigs: Signatures | None, epsilon, delta, gamma, prior=(1.0, 1.0), k=32,
                                res: Result = None, stream=None):
    import numpy as np
    _dev(cand, torch.uint32, "cand")
    lists = np.ascontiguousarray(lists)
    if lists.dtype != LIST_DTYPE:
        raise TypeError("lists must come from list_descs()")
    if res.code.numel() < cand.numel():
        raise ValueError("result.code smaller than cand")
    js = jaccard_sigs.struct() if jaccard_sigs is not None else None
    cs = cosine_sigs.struct() if cosine_sigs is not None else None
    rs = res.struct()
    kj, kc = _k_pair(k)
    _check(_lib().bayeslsh_exhaustive_batched(ctx.handle, lists.ctypes.data_as(C.POINTER(A.ListDesc)), len(lists),
                                              _p(cand), cand.numel(), C.byref(js) if js is not None else None,
                                              C.byref(cs) if cs is not None else None, epsilon, delta, gamma,
                                              _prior(prior), kj, kc, C.byref(rs), _stream(stream)))
    return res


# ---------------------------------------------------------------------------
# serving (bayeslsh_server_*)
# ---------------------------------------------------------------------------
class Server:
    """Owns a blsh_server; the context passed in is used by the server alone."""

    def __init__(self, ctx: Context, index: Signatures, mem_budget_bytes: int, max_active: int = 64, k: int = 32,
                 max_batch_candidates: int = 1 << 24, epsilon=0.03, delta=0.05, gamma=0.03, prior=(1.0, 1.0)):
        cfg = A.ServerConfig(mem_budget_bytes, max_active, k, max_batch_candidates, epsilon, delta, gamma,
                             _prior(prior))
        self._index = index
        self._held = {}   # device candidate arrays of requests submitted from the device
        st = index.struct()
        h = C.c_void_p()
        _check(_lib().bayeslsh_server_create(ctx.handle, C.byref(st), C.byref(cfg), C.byref(h)))
        self.handle = h
        self.ctx = ctx

    def clock(self) -> float:
        return _lib().bayeslsh_server_clock(self.handle)

    def submit(self, query: int, cand, t: float) -> int:
        import numpy as np
        cand = np.ascontiguousarray(cand, dtype=np.uint32)
        rid = C.c_int64()
        _check(_lib().bayeslsh_server_submit(self.handle, int(query), cand.ctypes.data_as(C.c_void_p), len(cand),
                                             float(t), C.byref(rid)))
        return rid.value

    def submit_device(self, query: int, cand: torch.Tensor, t: float) -> int:
        """Candidate ids already on the device (uint32 tensor): no host copy.
        The server's stream does not wait for the caller's: the tensor's
        values must be complete (synchronised) before the call.  The tensor
        is held until release()."""
        _dev(cand, torch.uint32, "cand")
        rid = C.c_int64()
        _check(_lib().bayeslsh_server_submit_device(self.handle, int(query), _p(cand), int(cand.numel()), float(t),
                                                    C.byref(rid)))
        self._held[rid.value] = cand
        return rid.value

    @staticmethod
    def _result(r: "A.RequestResult"):
        import numpy as np
        n = r.n_accepted
        # positions come in increasing order; string_at copies the server's
        # arrays (cheaper per call than np.ctypeslib.as_array)
        idx = np.frombuffer(C.string_at(r.acc_idx_host, n * 8), np.uint64).astype(np.int64) if n \
            else np.zeros(0, np.int64)
        val = np.frombuffer(C.string_at(r.acc_val_host, n * 4), np.float32).copy() if n else np.zeros(0, np.float32)
        return dict(n_candidates=r.n_candidates, acc_idx=idx, acc_val=val,
                    submit=r.submit_time_s, admit=r.admit_time_s, done=r.done_time_s, status=r.status)

    def poll(self, rid: int):
        r = A.RequestResult()
        rc = _lib().bayeslsh_server_poll(self.handle, rid, C.byref(r))
        if rc == A.EAGAIN:
            return None
        if rc != A.EBADID:   # finished with bad device ids: the result says so in "status"
            _check(rc)
        return self._result(r)

    def wait(self, rid: int):
        r = A.RequestResult()
        rc = _lib().bayeslsh_server_wait(self.handle, rid, C.byref(r))
        if rc != A.EBADID:
            _check(rc)
        return self._result(r)

    def release(self, rid: int):
        _check(_lib().bayeslsh_server_release(self.handle, rid))
        self._held.pop(rid, None)

    def stats(self):
        it, pe, ac, de = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(_lib().bayeslsh_server_stats(self.handle, C.byref(it), C.byref(pe), C.byref(ac), C.byref(de)))
        return dict(iterations=it.value, pending=pe.value, active=ac.value, deferred=de.value)

    def close(self):
        if self.handle:
            _lib().bayeslsh_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bayeslsh_server_create(ctx: Context, index: Signatures, **cfg) -> Server:
    return Server(ctx, index, **cfg)
