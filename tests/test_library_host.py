"""Host-side checks of libbayeslsh.so that need no GPU: the exported symbols,
the FP64 posterior-table builder against the oracle, and argument validation."""
import ctypes as C
import os

import numpy as np
import pytest

from oracle import posterior as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bayeslsh.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1110_1328_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_1110_1328_amd import build
        build.build()
    return _abi.load()


def test_every_declared_symbol_is_exported(lib):
    from paper_1110_1328_amd import _abi
    declared = _abi.header_symbols(HEADER)
    assert len(declared) >= 14
    for name in declared:
        assert hasattr(lib, name), name
    # and the binding declares a prototype for each
    assert sorted(n for n, _, _ in _abi.PROTOTYPES) == declared
    assert lib.bayeslsh_version() == 4


TABLE_CASES = [
    (0, 0.7, 32, 8, False, (1, 1)),     # Jaccard workload: t=0.7, 256 hashes, k=32
    (0, 0.5, 16, 16, False, (1, 1)),
    (0, 0.9, 64, 4, False, (1, 1)),
    (0, 0.7, 32, 8, False, (2, 3)),     # non-uniform integer prior
    (0, 0.3, 32, 8, True, (1, 1)),      # Lite (no concentration bits)
    (0, 0.7, 32, 8, False, (0.37, 2.9)),  # learned (real) priors: continued fraction
    (0, 0.5, 16, 16, False, (2.5, 7.25)),
    (0, 0.9, 64, 4, False, (0.8, 0.6)),
    (0, 0.3, 32, 8, True, (1.7, 4.2)),
    (1, 0.7, 32, 4, True, (1, 1)),      # cosine Lite, h = 128
    (1, 0.8, 32, 32, False, (1, 1)),    # dense cosine, 1024 bits
    (1, 0.5, 64, 16, False, (1, 1)),
    (1, 0.9, 16, 16, False, (1, 1)),
]


@pytest.mark.parametrize("measure,t,k,L,lite,prior", TABLE_CASES)
def test_posterior_table_matches_oracle(lib, measure, t, k, L, lite, prior):
    import paper_1110_1328_amd as P
    eps, delta, gamma = 0.03, 0.05, 0.03
    mm, acc, margin = P.bayeslsh_posterior_table(None, measure, t, eps, delta, gamma, prior, k, L, lite)
    memo = O.decision_memo(measure, t, eps, 0.0 if lite else delta, 0.0 if lite else gamma,
                           float(prior[0]), float(prior[1]), k, L, not lite)
    for j in range(L):
        n = (j + 1) * k
        surv = memo["survive"][j, :n + 1]
        want = int(np.argmax(surv)) if surv.any() else n + 1
        assert mm[j] == want, (j, mm[j], want)
        if not lite:
            bits = np.array([(int(acc[j, m >> 5]) >> (m & 31)) & 1 for m in range(n + 1)], np.uint8)
            np.testing.assert_array_equal(bits, memo["accept"][j, :n + 1])
    assert margin > 1e-9


def test_posterior_table_rejects_bad_arguments(lib):
    import paper_1110_1328_amd as P
    from paper_1110_1328_amd.api import BayesLSHError
    bad = [
        dict(t=1.2), dict(t=0.0), dict(epsilon=0.0), dict(delta=1.0), dict(gamma=-0.1),
        dict(measure=1, prior=(2.0, 1.0)),      # cosine needs the uniform prior
        dict(prior=(0.0, 1.0)),                 # Jaccard prior: 0 < alpha, beta <= 1e6
        dict(prior=(1.0, -2.0)),
        dict(prior=(2e6, 1.0)),
        dict(n_levels=65), dict(k=0), dict(measure=7),
    ]
    for kw in bad:
        args = dict(measure=0, t=0.7, epsilon=0.03, delta=0.05, gamma=0.03, prior=(1.0, 1.0), k=32, n_levels=4)
        args.update(kw)
        with pytest.raises(BayesLSHError) as e:
            P.bayeslsh_posterior_table(None, args["measure"], args["t"], args["epsilon"], args["delta"],
                                       args["gamma"], args["prior"], args["k"], args["n_levels"])
        assert e.value.code == -1, kw


def test_calls_without_a_context_fail_cleanly(lib):
    from paper_1110_1328_amd import _abi
    assert lib.bayeslsh_verify(None, None, None, 0.7, 0.03, 0.05, 0.03, _abi.Prior(1, 1), 32, None, None) == -1
    assert b"context" in lib.bayeslsh_last_error()
    assert lib.bayeslsh_sync(None, None) == -1
    assert lib.bayeslsh_minhash_sigs(None, None, None, None, 0, None, None) == -1
    assert lib.bayeslsh_reserve_workspace(None, 1 << 20, 1) == -1
    n = C.c_size_t()
    assert lib.bayeslsh_workspace_bytes(None, C.byref(n)) == -1
    h = C.c_void_p()
    rc = lib.bayeslsh_create(C.byref(h), 0)
    if rc == 0:   # a GPU is visible
        lib.bayeslsh_destroy(h)
    else:
        assert rc == -3 and b"device" in lib.bayeslsh_last_error().lower()


def test_fit_prior_matches_oracle(lib):
    """bayeslsh_fit_prior (Section 4.1, method of moments) against the oracle's
    fit, including the cases that fall back to the uniform prior."""
    import paper_1110_1328_amd as P
    from paper_1110_1328_amd.api import BayesLSHError
    rng = np.random.default_rng(5)
    samples = [rng.beta(2.0, 5.0, 5000), rng.beta(0.4, 3.0, 777), rng.uniform(0.2, 0.9, 31), [0.2, 0.4],
               [0.3, 0.3, 0.3], [0.0, 1.0], [0.7], [], [0.5 - 1e-5, 0.5 + 1e-5]]
    for smp in samples:
        (a, b), fell = P.bayeslsh_fit_prior(smp)
        wa, wb, wfell = O.fit_beta_moments(smp)
        assert fell == wfell
        assert a == pytest.approx(wa, rel=1e-12) and b == pytest.approx(wb, rel=1e-12)
    with pytest.raises(BayesLSHError):
        P.bayeslsh_fit_prior([0.3, 1.5])


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits (status 2) with a
    message before anything touches a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("measure,t,k,L,n,m,kind", [
    (0, 0.7, 32, 8, 32, 18, "prune"),         # epsilon placed on Pr[S >= t | M(18, 32)]
    (0, 0.7, 32, 8, 128, 80, "prune"),
    (1, 0.8, 32, 8, 64, 45, "prune"),
    (0, 0.7, 32, 8, 96, 90, "concentration"),  # 1 - gamma placed on Pr[|S - S_hat| < delta | M(90, 96)]
    (1, 0.7, 32, 4, 128, 120, "concentration"),
])
def test_posterior_table_refuses_near_ties(lib, measure, t, k, L, n, m, kind):
    """Section 4.3's precomputed decisions are unique only when no posterior
    probability sits on its threshold.  A parameter set that puts epsilon (or
    1 - gamma) exactly on a probability the oracle computes at some (n, m) is
    refused with BLSH_EINVAL naming that (n, m), rather than decided one way
    by rounding; a nearby parameter set (threshold moved by 1e-6) builds."""
    import paper_1110_1328_amd as P
    from paper_1110_1328_amd.api import BayesLSHError
    eps, delta, gamma = 0.03, 0.05, 0.03
    if kind == "prune":
        eps = O.prune_prob(measure, m, n, t)
        assert 1e-6 < eps < 0.5
    else:
        c = O.concentration(measure, m, n, delta)
        gamma = 1.0 - c
        assert 1e-6 < gamma < 0.5
        # the pair must reach the concentration test there (not pruned first)
        assert O.prune_prob(measure, m, n, t) >= eps
    with pytest.raises(BayesLSHError) as e:
        P.bayeslsh_posterior_table(None, measure, t, eps, delta, gamma, (1.0, 1.0), k, L, False)
    assert e.value.code == -1
    msg = str(e.value)
    assert "n=%d, m=%d" % (n, m) in msg, msg
    if kind == "prune":
        eps += 1e-6
    else:
        gamma += 1e-6
    _, _, margin = P.bayeslsh_posterior_table(None, measure, t, eps, delta, gamma, (1.0, 1.0), k, L, False)
    assert margin > 1e-9
