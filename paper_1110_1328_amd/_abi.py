"""ctypes mirror of include/bayeslsh.h (struct layouts, enums, prototypes)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbayeslsh.so")

# status codes
OK, EINVAL, ENOMEM, EDEVICE, ETRUNCATED, EBADID, EAGAIN = 0, -1, -2, -3, -4, -5, 1
STATUS_NAMES = {OK: "BLSH_OK", EINVAL: "BLSH_EINVAL", ENOMEM: "BLSH_ENOMEM", EDEVICE: "BLSH_EDEVICE",
                ETRUNCATED: "BLSH_ETRUNCATED", EBADID: "BLSH_EBADID", EAGAIN: "BLSH_EAGAIN"}
# enums
JACCARD, COSINE = 0, 1
PRUNED, ACCEPT_CONC, ACCEPT_NMAX, LITE_EXACT = 0, 1, 2, 3
OBJECT_MAJOR, WORD_MAJOR = 0, 1
PAIRS, QUERY_LISTS, ALL_PAIRS, TILES = 0, 1, 2, 3
DENSE, CSR, SETS = 0, 1, 2
REPLAY, REPLAY_LITE, MLE = 0, 1, 2
SRP_PLANES_Q16 = 1

p = C.c_void_p


class Prior(C.Structure):
    _fields_ = [("alpha", C.c_double), ("beta", C.c_double)]


class Sigs(C.Structure):
    _fields_ = [("measure", C.c_int), ("layout", C.c_int), ("data", p), ("n_obj", C.c_int64),
                ("n_hashes", C.c_int32), ("n_max", C.c_int32), ("prefix", p)]


class Candidates(C.Structure):
    _fields_ = [("kind", C.c_int), ("x", p), ("y", p), ("n_pairs", C.c_int64), ("query", p), ("offsets", p),
                ("cand", p), ("n_lists", C.c_int64), ("n_cand", C.c_int64), ("all_n", C.c_int64),
                ("tiles", p), ("n_tiles", C.c_int64)]


class Tile(C.Structure):
    _fields_ = [("first", C.c_int64), ("n_rows", C.c_uint32), ("n_cols", C.c_uint32), ("keep", C.c_uint64 * 4),
                ("ids", C.c_uint32 * 32), ("reserved", C.c_uint32 * 4)]


TILE_BYTES = 192
assert C.sizeof(Tile) == TILE_BYTES


class Vectors(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_obj", C.c_int64), ("dim", C.c_int64), ("dense", p), ("offsets", p),
                ("indices", p), ("values", p)]


class Result(C.Structure):
    _fields_ = [("code", p), ("acc_idx", p), ("acc_val", p), ("acc_capacity", C.c_int64), ("n_accepted", p),
                ("m_debug", p)]


class Tuning(C.Structure):
    _fields_ = [("gather", C.c_int32), ("batch_inreg", C.c_int32), ("batch_blocks_per_cu", C.c_int32),
                ("last_batch_k_jaccard", C.c_int32), ("last_batch_inreg", C.c_int32),
                ("last_batch_blocks_per_cu", C.c_int32), ("batch_spill_cap", C.c_int32),
                ("last_batch_k_cosine", C.c_int32), ("acc_stage_cap", C.c_int32),
                ("batch_srp_tile", C.c_int32), ("batch_mh_tile", C.c_int32),
                ("last_batch_srp_tile", C.c_int32), ("last_batch_mh_tile", C.c_int32),
                ("tiles_accept_bitmask", C.c_int32), ("tiles_per_launch", C.c_int32)]


class ListDesc(C.Structure):
    _fields_ = [("measure", C.c_int), ("t", C.c_double), ("query", C.c_uint32), ("offset", C.c_int64),
                ("length", C.c_int64)]


class ServerConfig(C.Structure):
    _fields_ = [("mem_budget_bytes", C.c_size_t), ("max_active", C.c_int32), ("k", C.c_int32),
                ("max_batch_candidates", C.c_int64), ("epsilon", C.c_double), ("delta", C.c_double),
                ("gamma", C.c_double), ("prior", Prior)]


class RequestResult(C.Structure):
    _fields_ = [("n_candidates", C.c_int64), ("n_accepted", C.c_int64), ("acc_idx_host", C.POINTER(C.c_uint64)),
                ("acc_val_host", C.POINTER(C.c_float)), ("submit_time_s", C.c_double),
                ("admit_time_s", C.c_double), ("done_time_s", C.c_double), ("status", C.c_int32)]


# (name, restype, argtypes) for every symbol of the header
PROTOTYPES = [
    ("bayeslsh_create", C.c_int, [C.POINTER(p), C.c_int]),
    ("bayeslsh_destroy", None, [p]),
    ("bayeslsh_reserve_workspace", C.c_int, [p, C.c_size_t, C.c_int32]),
    ("bayeslsh_workspace_bytes", C.c_int, [p, C.POINTER(C.c_size_t)]),
    ("bayeslsh_sync", C.c_int, [p, p]),
    ("bayeslsh_last_error", C.c_char_p, []),
    ("bayeslsh_version", C.c_int, []),
    ("bayeslsh_profile_enable", C.c_int, [p, C.c_int]),
    ("bayeslsh_profile_reset", C.c_int, [p]),
    ("bayeslsh_profile_read", C.c_int, [p, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    ("bayeslsh_set_tuning", C.c_int, [p, C.POINTER(Tuning)]),
    ("bayeslsh_get_tuning", C.c_int, [p, C.POINTER(Tuning)]),
    ("bayeslsh_posterior_table", C.c_int,
     [p, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, Prior, C.c_int32, C.c_int32, C.c_int32, p, p,
      C.POINTER(C.c_double)]),
    ("bayeslsh_minhash_sigs", C.c_int, [p, C.POINTER(Vectors), p, p, C.c_int32, p, p]),
    ("bayeslsh_srp_sigs", C.c_int, [p, C.POINTER(Vectors), p, C.c_int32, C.c_uint64, C.c_int, C.c_int32, p, p]),
    ("bayeslsh_verify", C.c_int,
     [p, C.POINTER(Candidates), C.POINTER(Sigs), C.c_double, C.c_double, C.c_double, C.c_double, Prior, C.c_int32,
      C.POINTER(Result), p]),
    ("bayeslsh_verify_noalloc", C.c_int,
     [p, C.POINTER(Candidates), C.POINTER(Sigs), C.c_double, C.c_double, C.c_double, C.c_double, Prior, C.c_int32,
      C.POINTER(Result), p]),
    ("bayeslsh_lite_verify", C.c_int,
     [p, C.POINTER(Candidates), C.POINTER(Sigs), C.POINTER(Vectors), C.c_double, C.c_double, Prior, C.c_int32,
      C.c_int32, C.POINTER(Result), p]),
    ("bayeslsh_exact_similarity", C.c_int, [p, C.POINTER(Candidates), C.POINTER(Vectors), p, p]),
    ("bayeslsh_fit_prior", C.c_int, [p, C.c_int64, C.POINTER(Prior), C.POINTER(C.c_int32)]),
    ("bayeslsh_band_candidates", C.c_int, [p, C.POINTER(Sigs), C.c_int32, C.c_int32, C.c_int32, C.c_int32, p, p, C.c_int64,
                                           C.POINTER(C.c_int64), p]),
    ("bayeslsh_band_tiles", C.c_int, [p, C.POINTER(Sigs), C.c_int32, C.c_int32, C.c_int32, p, C.c_int64,
                                      C.POINTER(C.c_int64), C.POINTER(C.c_int64), p]),
    ("bayeslsh_verify_batched", C.c_int,
     [p, C.POINTER(ListDesc), C.c_int64, p, C.c_int64, C.POINTER(Sigs), C.POINTER(Sigs), C.c_double, C.c_double,
      C.c_double, Prior, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(Result), p]),
    ("bayeslsh_exhaustive_batched", C.c_int,
     [p, C.POINTER(ListDesc), C.c_int64, p, C.c_int64, C.POINTER(Sigs), C.POINTER(Sigs), C.c_double, C.c_double,
      C.c_double, Prior, C.c_int32, C.c_int32, C.POINTER(Result), p]),
    ("bayeslsh_server_create", C.c_int, [p, C.POINTER(Sigs), C.POINTER(ServerConfig), C.POINTER(p)]),
    ("bayeslsh_server_submit", C.c_int, [p, C.c_uint32, p, C.c_int64, C.c_double, C.POINTER(C.c_int64)]),
    ("bayeslsh_server_submit_device", C.c_int, [p, C.c_uint32, p, C.c_int64, C.c_double, C.POINTER(C.c_int64)]),
    ("bayeslsh_server_poll", C.c_int, [p, C.c_int64, C.POINTER(RequestResult)]),
    ("bayeslsh_server_wait", C.c_int, [p, C.c_int64, C.POINTER(RequestResult)]),
    ("bayeslsh_server_release", C.c_int, [p, C.c_int64]),
    ("bayeslsh_server_stats", C.c_int,
     [p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    ("bayeslsh_server_clock", C.c_double, [p]),
    ("bayeslsh_server_destroy", None, [p]),
    ("bayeslsh_exhaustive_verify", C.c_int,
     [p, C.POINTER(Candidates), C.POINTER(Sigs), C.POINTER(Vectors), C.c_double, C.c_double, C.c_double, C.c_double,
      Prior, C.c_int32, C.c_int32, C.c_int, C.POINTER(Result), p]),
]


def header_symbols(header_path: str) -> list[str]:
    """Names of the functions declared in a header (for the export check)."""
    import re
    txt = open(header_path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bayeslsh_[a-z_0-9]+)\s*\(", txt)))


_lib = None


def load(path: str = LIB_PATH):
    """Load libbayeslsh.so and attach prototypes.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libbayeslsh.so is not built (run `python -m paper_1110_1328_amd.build`): %s" % path)
    lib = C.CDLL(path)
    for name, res, args in PROTOTYPES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
