"""Pins of the CPU oracle against things other than itself (no GPU).

Each test checks the oracle against what the paper or the mathematics fixes:
exact rational arithmetic, 50-digit quadrature, closed forms, published
known-answer vectors, brute force on tiny inputs, and Bayesian calibration by
Monte Carlo.  A plausible slip in the oracle (a dropped term, a wrong tail,
a swapped Beta parameter, an off-by-one in the hash range) fails at least one.
"""
import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle import posterior as P
from oracle import reference as R
from synth import generators as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------------------
# Exact binomial tails with integer arithmetic
# ---------------------------------------------------------------------------
def binom_cdf_exact(N, m, x: Fraction) -> Fraction:
    """Pr[Binomial(N, x) <= m] as an exact rational."""
    if m < 0:
        return Fraction(0)
    if m >= N:
        return Fraction(1)
    p, q = x.numerator, x.denominator
    s = 0
    c = 1
    for j in range(0, m + 1):
        if j:
            c = c * (N - j + 1) // j
        s += c * p ** j * (q - p) ** (N - j)
    return Fraction(s, q ** N)


def reg_inc_beta_exact(x: Fraction, a: int, b: int) -> Fraction:
    """I_x(a, b) = Pr[Binomial(a+b-1, x) >= a] for integer a, b >= 1."""
    if x <= 0:
        return Fraction(0)
    if x >= 1:
        return Fraction(1)
    return 1 - binom_cdf_exact(a + b - 1, a - 1, x)


def test_philox_known_answers():
    for row in _golden("philox4x32_10_kat.txt"):
        v = [int(h, 16) for h in row]
        ctr, key, want = v[0:4], v[4:6], v[6:10]
        assert list(R.philox4x32_10(ctr, key)) == want
        assert R.philox4x32_10_py(ctr, key) == want


def test_paper_printed_values():
    vals = {r[0]: (float(r[1]), float(r[2])) for r in _golden("paper_values.txt")}
    v, tol = vals["c2r_of_0.70"]
    assert abs(P.c2r(0.70) - v) <= tol
    # Beta(1,1) is uniform: MAP = m/n (Section 4.1), cosine R_hat = m/n (Section 4.2)
    for n in (32, 64, 256):
        for m in range(0, n + 1, 7):
            assert P.jaccard_map(m, n, 1.0, 1.0) == pytest.approx(m / n, abs=1e-15)
            if m / n >= 0.5:
                assert P.cosine_map(m, n) == pytest.approx(math.cos(math.pi * (1 - m / n)), abs=1e-15)
    # the example of Section 3.2: 10 agreements among the first 100 hashes at t = 0.8
    assert P.jaccard_prune_prob(10, 100, 0.8) < 1e-30
    assert P.cosine_prune_prob(10, 100, 0.8) < 1e-30


def test_r2c_c2r_inverse():
    for c in np.linspace(0.0, 1.0, 101):
        assert P.r2c(P.c2r(c)) == pytest.approx(c, abs=1e-14)
    assert P.c2r(0.0) == pytest.approx(0.5, abs=1e-16)
    assert P.c2r(1.0) == 1.0


@pytest.mark.parametrize("t,alpha,beta,k,L", [
    (Fraction(7, 10), 1, 1, 32, 8),      # the Jaccard workload's parameters
    (Fraction(1, 2), 2, 3, 16, 6),       # a non-uniform integer prior
    (Fraction(9, 10), 1, 1, 64, 4),
])
def test_jaccard_tables_exact_rational(t, alpha, beta, k, L):
    """Survive/accept decisions and the raw probabilities against exact rationals
    (t, epsilon, delta, gamma as decimal fractions)."""
    eps, delta, gamma = Fraction(3, 100), Fraction(5, 100), Fraction(3, 100)
    memo = P.decision_memo(0, float(t), float(eps), float(delta), float(gamma), float(alpha), float(beta), k, L, True)
    for j in range(L):
        n = (j + 1) * k
        for m in range(n + 1):
            a, b = m + alpha, n - m + beta
            p_ge = 1 - reg_inc_beta_exact(t, a, b)
            assert abs(memo["p_ge"][j, m] - float(p_ge)) < 1e-13
            surv = p_ge >= eps
            assert bool(memo["survive"][j, m]) == surv, (n, m)
            mode = Fraction(m + alpha - 1, n + alpha + beta - 2)
            mode = min(Fraction(1), max(Fraction(0), mode))
            assert memo["shat"][j, m] == pytest.approx(float(mode), abs=1e-15)
            if surv:
                hi = min(Fraction(1), mode + delta)
                lo = max(Fraction(0), mode - delta)
                c = reg_inc_beta_exact(hi, a, b) - reg_inc_beta_exact(lo, a, b)
                assert abs(memo["conc"][j, m] - float(c)) < 1e-12
                assert bool(memo["accept"][j, m]) == (c >= 1 - gamma), (n, m)
            else:
                assert not memo["accept"][j, m]


def _cos_integral(m, n, lo, hi):
    """int_lo^hi r^m (1-r)^(n-m) dr, as mpmath's incomplete beta (a hypergeometric
    series) evaluated with 700 digits so that differences of values as small as
    1e-310 keep full relative precision."""
    with mpmath.workdps(700):
        return mpmath.betainc(m + 1, n - m + 1, mpmath.mpf(lo), mpmath.mpf(hi))


def _cos_quad(m, n, lo, hi):
    """The same integral by tanh-sinh quadrature on 256 panels."""
    f = lambda r: r ** m * (1 - r) ** (n - m)
    return mpmath.quad(f, mpmath.linspace(lo, hi, 257))


def test_cosine_posterior_against_quadrature():
    """Cosine prune/concentration probabilities against high-precision integrals of
    r^m (1-r)^(n-m) over sub-intervals of [0.5, 1] (Section 4.2), an independent
    route from the oracle's log-space binomial-tail form."""
    mpmath.mp.dps = 50
    t, delta = 0.7, 0.05
    tr = mpmath.mpf(1) - mpmath.acos(mpmath.mpf(t)) / mpmath.pi
    cases = [(0, 32), (16, 32), (20, 32), (31, 32), (32, 32), (42, 64), (63, 64), (87, 128),
             (120, 128), (0, 256), (200, 256), (800, 1024), (1024, 1024), (512, 1024)]
    for m, n in cases:
        den = _cos_integral(m, n, mpmath.mpf("0.5"), 1)
        num = _cos_integral(m, n, tr, 1)
        p = float(num / den)
        assert P.cosine_prune_prob(m, n, t) == pytest.approx(p, rel=1e-9, abs=1e-300)
        s = mpmath.cos(mpmath.pi * (1 - max(mpmath.mpf("0.5"), mpmath.mpf(m) / n)))
        r_lo = max(mpmath.mpf("0.5"), 1 - mpmath.acos(max(-1, s - delta)) / mpmath.pi)
        r_hi = 1 - mpmath.acos(min(1, s + delta)) / mpmath.pi
        c = float(_cos_integral(m, n, r_lo, r_hi) / den)
        assert P.cosine_concentration(m, n, delta) == pytest.approx(c, abs=1e-12)
        if 0 < m < n:   # interior peak: plain quadrature agrees too
            cq = float(_cos_quad(m, n, r_lo, r_hi) / _cos_quad(m, n, mpmath.mpf("0.5"), 1))
            assert P.cosine_concentration(m, n, delta) == pytest.approx(cq, abs=1e-9)


def test_cosine_table_decisions_against_quadrature():
    """Every survive decision of the cosine table at n <= 96 (k = 32, t = 0.8)
    against quadrature."""
    mpmath.mp.dps = 30
    t, eps = 0.8, 0.03
    memo = P.decision_memo(1, t, eps, 0.05, 0.03, 1.0, 1.0, 32, 3, False)
    tr = mpmath.mpf(1) - mpmath.acos(mpmath.mpf(t)) / mpmath.pi
    for j in range(3):
        n = 32 * (j + 1)
        for m in range(n + 1):
            den = _cos_integral(m, n, mpmath.mpf("0.5"), 1)
            p = _cos_integral(m, n, tr, 1) / den
            assert bool(memo["survive"][j, m]) == (p >= eps), (n, m)


@pytest.mark.parametrize("measure", [0, 1])
def test_prune_probability_monotone_in_m(measure):
    """Pr[S >= t | M(m,n)] increases with m for fixed n (Section 4.3), up to
    FP64 rounding (values within 1e-14 of 1 may wobble in the last bits)."""
    for t in (0.5, 0.7, 0.9):
        for n in (16, 64, 256):
            p = [P.prune_prob(measure, m, n, t) for m in range(n + 1)]
            assert all(b >= a - 1e-14 for a, b in zip(p, p[1:]))
            assert p[-1] > p[0]


def _sig_pairs_with_m(measure, ms, k_total):
    """Object pairs (2i, 2i+1) agreeing on exactly the first ms[i] hashes."""
    n = len(ms)
    if measure == 0:
        sig = np.zeros((2 * n, k_total), np.uint32)
        for i, m in enumerate(ms):
            sig[2 * i] = np.arange(k_total) + 1000 * i
            sig[2 * i + 1] = sig[2 * i]
            sig[2 * i + 1, m:] += 7
        return sig
    bits = np.zeros((2 * n, k_total), np.uint8)
    for i, m in enumerate(ms):
        bits[2 * i + 1, m:] = 1
    return G.pack_bits(bits)


def test_hand_decisions_single_level():
    """k = n_max = 32, Jaccard t = 0.7, Beta(1,1): closed forms give the outcome.
    The smallest surviving m is the least m with Pr[Bin(33, 0.7) <= m] >= 0.03;
    a surviving pair is concentrated iff I_{m/32+0.05} - I_{m/32-0.05} >= 0.97 with
    Beta(m+1, 33-m), which at n = 32 never happens (the best case m = 32 gives
    1 - 0.95^33 = 0.816), so survivors are emitted at n_max with S_hat = m/32."""
    t = Fraction(7, 10)
    m_min = next(m for m in range(33) if binom_cdf_exact(33, m, t) >= Fraction(3, 100))
    assert float(1 - Fraction(95, 100) ** 33) < 0.97
    ms = list(range(33))
    sig = _sig_pairs_with_m(0, ms, 32)
    x = np.arange(0, 66, 2, dtype=np.uint32)
    y = x + 1
    for res in (R.verify(x, y, 0, sig, 32, 1, 0.7, 0.03, 0.05, 0.03),
                R.verify_py(x, y, 0, sig, 32, 1, 0.7, 0.03, 0.05, 0.03)):
        for m in ms:
            assert res["m"][m] == m
            if m < m_min:
                assert res["decision"][m] == R.DEC_PRUNED
            else:
                assert res["decision"][m] == R.DEC_NMAX
                assert res["shat"][m] == pytest.approx(m / 32, abs=1e-15)


@pytest.mark.parametrize("measure,lite", [(0, False), (1, False), (0, True), (1, True)])
def test_c_loop_matches_pure_python(measure, lite):
    rng = np.random.default_rng(5)
    npairs, k, L = 300, 32, 4
    s = rng.uniform(0.5 if measure else 0.0, 1.0, npairs)
    sig = (G.calibration_minhash(npairs, k * L, s, 17) if measure == 0
           else G.pack_bits(G.calibration_bits(npairs, k * L, s, 17)))
    x = np.arange(0, 2 * npairs, 2, dtype=np.uint32)
    y = x + 1
    a = R.verify(x, y, measure, sig, k, L, 0.7, 0.03, 0.05, 0.03, lite=lite)
    b = R.verify_py(x, y, measure, sig, k, L, 0.7, 0.03, 0.05, 0.03, lite=lite)
    for key in ("decision", "level", "m"):
        np.testing.assert_array_equal(a[key], b[key])
    np.testing.assert_allclose(a["shat"], b["shat"], atol=1e-15, equal_nan=True)
    assert len(set(a["decision"].tolist())) >= 2


def test_all_pairs_enumeration_matches_explicit_pairs():
    rng = np.random.default_rng(3)
    n_obj, nh = 40, 128
    sig = rng.integers(0, 4, size=(n_obj, nh)).astype(np.uint32)   # many agreements
    x, y = R.all_pairs_xy(n_obj)
    a = R.verify(None, None, 0, sig, 32, 4, 0.3, 0.03, 0.05, 0.03, all_n=n_obj)
    b = R.verify(x, y, 0, sig, 32, 4, 0.3, 0.03, 0.05, 0.03)
    for key in ("decision", "level", "m"):
        np.testing.assert_array_equal(a[key], b[key])


def test_minhash_brute_force():
    sets = G.jaccard_sets(n_sets=30, vocab=500, median=12, n_groups=3, seed=7)
    a, b = G.minhash_coeffs(16, 9)
    sig = R.minhash_signatures(sets.offsets, sets.elems, a, b)
    for i in range(sets.n):
        assert sig[i].tolist() == R.minhash_signature_py(sets.row(i).tolist(), a, b)


def test_minhash_agreement_estimates_jaccard():
    """Pr[h(x) = h(y)] = J(x, y) for the family (Section 2, eqn lshmain; Section 4.1)."""
    rng = np.random.default_rng(11)
    A = np.sort(rng.choice(5000, 300, replace=False))
    B = np.sort(np.concatenate([A[:200], rng.choice(np.setdiff1d(np.arange(5000, 9000), A), 100, replace=False)]))
    J = len(np.intersect1d(A, B)) / len(np.union1d(A, B))
    offsets = np.array([0, len(A), len(A) + len(B)], np.int64)
    a, b = G.minhash_coeffs(8192, 12)
    sig = R.minhash_signatures(offsets, np.concatenate([A, B]), a, b)
    est = np.mean(sig[0] == sig[1])
    assert abs(est - J) < 4.5 * math.sqrt(J * (1 - J) / 8192)


def test_gaussian_plane_entries_are_standard_normal():
    from scipy import stats
    vals = np.array([R.srp_gauss(123, term, bit) for term in range(50) for bit in range(400)])
    assert stats.kstest(vals, "norm").pvalue > 1e-3
    assert abs(vals.mean()) < 0.03 and abs(vals.std() - 1) < 0.03
    # Box-Muller on the Philox words, restated directly
    w = R.philox4x32_10_py([7, 5 >> 2, 0, 0], [99, 0])
    u0, u1 = (w[0] + 0.5) / 2 ** 32, (w[1] + 0.5) / 2 ** 32
    z1 = math.sqrt(-2 * math.log(u0)) * math.sin(2 * math.pi * u1)
    assert R.srp_gauss(99, 7, 5) == np.float32(z1)


def test_q16_codes_are_the_midpoints_of_a_uniform_grid():
    """2-byte plane storage (Section 4.3), all 65,536 codes: the values read
    back form a uniform grid of 2^16 cells over (-8, 8), one value at the
    middle of each cell, symmetric about 0; every value encodes to its own
    code; each cell's lower edge belongs to it and its upper edge to the next
    (the floor of the printed encoding); samples outside (-8, 8) saturate."""
    codes = np.arange(1 << 16, dtype=np.uint16)
    d = R.q16_decode(codes)
    step = 2.0 ** -12                       # 16 / 2^16
    assert np.all(np.diff(d) == step)
    assert d[0] == -8 + step / 2 and d[-1] == 8 - step / 2
    assert np.all(d + d[::-1] == 0)
    np.testing.assert_array_equal(R.q16_encode(d), codes)
    lo = -8.0 + codes.astype(np.float64) * step
    np.testing.assert_array_equal(R.q16_encode(lo), codes)
    hi = lo + (step - 2.0 ** -32)           # just below the upper edge (exact, also after the shift by 8)
    np.testing.assert_array_equal(R.q16_encode(hi), codes)
    np.testing.assert_array_equal(R.q16_encode(lo[1:] - 2.0 ** -32), codes[:-1])
    np.testing.assert_array_equal(R.q16_encode([-1e9, -8.5, -8.0, 8.0 - 1e-9, 8.0, 1e9]),
                                  [0, 0, 0, 65535, 65535, 65535])


def test_q16_error_bound_and_the_printed_claim():
    """Read back at the cell midpoint the error is at most half a cell,
    2^-13 = 1.22e-4, and that bound is reached; it exceeds the 1e-4 the
    paper prints for the encoding.  A generated plane entry never leaves
    (-8, 8): the smallest uniform Box-Muller sees is 0.5 / 2^32."""
    rng = np.random.default_rng(5)
    x = rng.uniform(-8, 8, 1 << 20)
    err = np.abs(R.q16_decode(R.q16_encode(x)) - x)
    assert err.max() <= 2.0 ** -13
    assert err.max() > 0.999 * 2.0 ** -13 > 1e-4
    assert math.sqrt(-2 * math.log(0.5 / 2 ** 32)) < 7.0
    g = np.array([R.srp_gauss(31, t, b) for t in range(40) for b in range(256)])
    assert np.all(np.abs(R.q16_decode(R.q16_encode(g)) - g) <= 2.0 ** -13)


def test_q16_sparse_projection():
    """Projections over 2-byte plane entries: a numpy recomputation from the
    entries read back, and within sum |x_i| 2^-13 of the fp32-entry ones."""
    corpus = G.tfidf_corpus(n_docs=40, dim=1 << 12, mean_nnz=30, seed=22)
    rows = np.arange(corpus.n, dtype=np.int64)
    nb = 64
    proj = R.srp_sparse_projections(corpus.offsets, corpus.indices, corpus.values, nb, 78, rows)
    projq = R.srp_sparse_projections(corpus.offsets, corpus.indices, corpus.values, nb, 78, rows, q16=True)
    for r in rows[:3]:
        idx, val = corpus.row(r)
        g = np.array([[R.srp_gauss(78, int(t), b) for b in range(nb)] for t in idx], np.float64)
        gq = R.q16_decode(R.q16_encode(g.ravel())).reshape(g.shape)
        assert np.any(gq != g)
        np.testing.assert_allclose(projq[r], val.astype(np.float64) @ gq, rtol=1e-12, atol=1e-14)
    l1 = np.array([np.abs(corpus.row(r)[1].astype(np.float64)).sum() for r in rows])
    assert np.all(np.abs(projq - proj) <= l1[:, None] * 2.0 ** -13 + 1e-12)
    assert np.any(projq != proj)


def test_sparse_projection_and_angle_agreement():
    """r . x in FP64 equals a numpy recomputation from the plane entries, and the
    sign bits agree with probability 1 - theta/pi (Section 4.2)."""
    corpus = G.tfidf_corpus(n_docs=60, dim=1 << 12, mean_nnz=40, seed=21)
    rows = np.array([0, 1, 2], np.int64)
    nb = 64
    proj = R.srp_sparse_projections(corpus.offsets, corpus.indices, corpus.values, nb, 77, rows)
    for r in rows:
        idx, val = corpus.row(r)
        g = np.array([[R.srp_gauss(77, int(t), b) for b in range(nb)] for t in idx], np.float64)
        np.testing.assert_allclose(proj[r], val.astype(np.float64) @ g, rtol=1e-12, atol=1e-14)
    # angle agreement on a dense pair with many planes
    rng = np.random.default_rng(4)
    u = rng.standard_normal(64).astype(np.float32)
    v = (u + 0.9 * rng.standard_normal(64)).astype(np.float32)
    Rm = G.gaussian_planes(64, 8192, 5)
    bits = R.bits_from_projections(R.srp_dense_projections(np.stack([u, v]), Rm))
    agree = 8192 - sum(bin(int(a ^ b)).count("1") for a, b in zip(bits[0], bits[1]))
    cos = float(np.dot(u.astype(np.float64), v) / np.linalg.norm(u.astype(np.float64)) / np.linalg.norm(v.astype(np.float64)))
    r = P.c2r(cos)
    assert abs(agree / 8192 - r) < 4.5 * math.sqrt(r * (1 - r) / 8192)


def test_bits_packing_lsb_first():
    proj = np.full((1, 64), -1.0)
    proj[0, [0, 5, 31, 32, 63]] = [1.0, 0.0, 2.0, 3.0, 4.0]   # 0.0 is a tie -> bit 1
    w = R.bits_from_projections(proj)
    assert w[0, 0] == (1 | (1 << 5) | (1 << 31)) and w[0, 1] == (1 | (1 << 31))


def test_exact_similarity_brute_force():
    sets = G.jaccard_sets(n_sets=25, vocab=200, median=15, n_groups=3, seed=8)
    x, y = R.all_pairs_xy(sets.n)
    got = R.exact_jaccard(sets.offsets, sets.elems, x, y)
    for p, (i, j) in enumerate(zip(x.tolist(), y.tolist())):
        A, B = set(sets.row(i).tolist()), set(sets.row(j).tolist())
        assert got[p] == len(A & B) / len(A | B)
    corpus = G.tfidf_corpus(n_docs=30, dim=1 << 10, mean_nnz=30, seed=9)
    x, y = R.all_pairs_xy(corpus.n)
    got = R.exact_cosine_csr(corpus.offsets, corpus.indices, corpus.values, x, y)
    dense = np.zeros((corpus.n, corpus.dim))
    for i in range(corpus.n):
        idx, val = corpus.row(i)
        dense[i, idx] = val
    want = [(dense[i] @ dense[j]) / np.linalg.norm(dense[i]) / np.linalg.norm(dense[j]) for i, j in zip(x, y)]
    np.testing.assert_allclose(got, want, atol=1e-14)
    got_d = R.exact_cosine_dense(dense.astype(np.float32), x, y)
    np.testing.assert_allclose(got_d, want, atol=1e-7)
    assert max(got) > 0.5   # planted duplicates present


@pytest.mark.parametrize("measure", [0, 1])
def test_bayesian_calibration_monte_carlo(measure):
    """With S drawn from the prior and hashes agreeing independently with
    probability S, the stopping rule cannot change the posterior, so:
      - among pruned pairs the fraction with S >= t is below epsilon (guarantee 1);
      - among concentrated accepts the fraction with |S_hat - S| >= delta is
        below gamma (guarantee 2);
      - recall over S ~ prior restricted to S >= t is at least 1 - epsilon.
    For cosine the prior is uniform on r = c2r(S) in [0.5, 1]."""
    rng = np.random.default_rng(100 + measure)
    t, eps, delta, gamma, k = 0.7, 0.03, 0.05, 0.03, 32
    L = 8 if measure == 0 else 16
    npairs = 60000
    u = rng.uniform(0.0 if measure == 0 else 0.5, 1.0, npairs)      # similarity in hash space
    sig = (G.calibration_minhash(npairs, k * L, u, 31) if measure == 0
           else G.pack_bits(G.calibration_bits(npairs, k * L, u, 31)))
    S = u if measure == 0 else np.cos(np.pi * (1 - u))
    x = np.arange(0, 2 * npairs, 2, dtype=np.uint32)
    res = R.verify(x, x + 1, measure, sig, k, L, t, eps, delta, gamma)
    d = res["decision"]
    pruned = d == R.DEC_PRUNED
    conc = d == R.DEC_CONC
    assert pruned.sum() > 1000 and conc.sum() > 1000
    assert np.mean(S[pruned] >= t) < eps
    err = np.abs(res["shat"][conc] - S[conc]) >= delta
    se = math.sqrt(gamma * (1 - gamma) / conc.sum())
    assert np.mean(err) < gamma + 2 * se
    # recall with S restricted to [t, 1] under the prior
    u2 = rng.uniform(t if measure == 0 else P.c2r(t), 1.0, 20000)
    sig2 = (G.calibration_minhash(20000, k * L, u2, 32) if measure == 0
            else G.pack_bits(G.calibration_bits(20000, k * L, u2, 32)))
    x2 = np.arange(0, 40000, 2, dtype=np.uint32)
    res2 = R.verify(x2, x2 + 1, measure, sig2, k, L, t, eps, delta, gamma)
    assert np.mean(res2["decision"] != R.DEC_PRUNED) >= 1 - eps


def test_lite_finishes_with_exact_similarity():
    sets = G.jaccard_sets(n_sets=200, vocab=3000, median=40, n_groups=20, seed=13)
    a, b = G.minhash_coeffs(64, 14)
    sig = R.minhash_signatures(sets.offsets, sets.elems, a, b)
    x, y = R.all_pairs_xy(sets.n)
    res = R.verify(x, y, 0, sig, 32, 2, 0.5, 0.03, 0.05, 0.03, lite=True)
    out = R.lite_finish(res, lambda xs, ys: R.exact_jaccard(sets.offsets, sets.elems, xs, ys), x, y, 0.5)
    surv = out["decision"] == R.DEC_LITE
    J = R.exact_jaccard(sets.offsets, sets.elems, x, y)
    np.testing.assert_array_equal(out["accepted"], surv & (J > 0.5))
    # no true pair above t was lost to pruning on this input
    assert np.all(out["accepted"][J > 0.6])


def test_mle_estimate():
    rng = np.random.default_rng(2)
    sig = rng.integers(0, 2, size=(10, 64)).astype(np.uint32)
    x, y = R.all_pairs_xy(10)
    out = R.mle(x, y, 0, sig, 64, 0.5)
    want = [(sig[i] == sig[j]).mean() for i, j in zip(x, y)]
    np.testing.assert_allclose(out["shat"], want)


def _bit_rows(n_bits, agree_counts):
    """Object 0 = all-zero bits; object i+1 agrees with it on exactly
    agree_counts[i] of the first n_bits bits (packed LSB-first words)."""
    words = n_bits // 32
    rows = np.zeros((len(agree_counts) + 1, words), np.uint32)
    for i, m in enumerate(agree_counts):
        bits = np.zeros(n_bits, np.uint8)
        bits[m:] = 1                     # the last n_bits - m bits disagree
        rows[i + 1] = np.packbits(bits.reshape(words, 32)[:, ::-1], axis=1).view(">u4").ravel()
    return rows


def test_mle_cosine_branch_hand_values():
    """Cosine LSH Approx (Section 3 estimator through the Section 4.2 map
    r -> cos(pi (1 - r))): at m/n = 1, 3/4, 1/2, 1/4 and 0 the estimate is
    cos 0 = 1, cos(pi/4) = sqrt(2)/2, cos(pi/2) = 0, cos(3 pi/4) = -sqrt(2)/2
    and cos(pi) = -1 (values of the cosine, not retyped from the oracle's
    expression); emission is inclusive at t (checked on the Jaccard branch,
    where 3/4 is exact)."""
    n = 64
    rows = _bit_rows(n, [64, 48, 32, 16, 0])
    x = np.zeros(5, np.uint32)
    y = np.arange(1, 6, dtype=np.uint32)
    assert np.array_equal(R.counts_all(x, y, 1, rows, n), [64, 48, 32, 16, 0])
    out = R.mle(x, y, 1, rows, n, 0.7)
    h = np.sqrt(2.0) / 2.0
    np.testing.assert_allclose(out["shat"], [1.0, h, 0.0, -h, -1.0], atol=1e-15)
    assert out["accepted"].tolist() == [True, True, False, False, False]
    # inclusive threshold: 48/64 = 0.75 exactly, t = 0.75 accepts (a strict
    # rule would reject it)
    jac = np.zeros((2, n), np.uint32)
    jac[1, 48:] = 7
    o = R.mle(np.array([0], np.uint32), np.array([1], np.uint32), 0, jac, n, 0.75)
    assert o["shat"][0] == 0.75 and bool(o["accepted"][0])


def test_mle_cosine_branch_recovers_the_angle():
    """Sign random projections agree with probability 1 - theta/pi (Section
    4.2), so the cosine estimate over many hashes approaches cos(theta): two
    unit vectors at a chosen angle, 2^16 Gaussian planes drawn here with
    numpy (not the oracle's generator), bits packed LSB-first.  A reading such
    as cos(pi r) would return -cos(theta) and fail."""
    rng = np.random.default_rng(11)
    d, n = 32, 1 << 16
    for theta in (0.3, 1.0, 2.2):
        u = rng.standard_normal(d)
        u /= np.linalg.norm(u)
        w = rng.standard_normal(d)
        w -= (w @ u) * u
        w /= np.linalg.norm(w)
        v = np.cos(theta) * u + np.sin(theta) * w
        planes = rng.standard_normal((d, n))
        bits = np.stack([(u @ planes) >= 0, (v @ planes) >= 0]).astype(np.uint8)
        rows = np.packbits(bits.reshape(2, n // 32, 32)[:, :, ::-1], axis=2).view(">u4").reshape(2, n // 32)
        rows = rows.astype(np.uint32)
        o = R.mle(np.array([0], np.uint32), np.array([1], np.uint32), 1, rows, n, 0.5)
        # std of m/n <= 0.002 at n = 2^16; through cos that is <= pi * 0.002
        assert abs(o["shat"][0] - np.cos(theta)) < 0.03, (theta, o["shat"][0])


# ---------------------------------------------------------------------------
# Learned prior (Section 4.1): method of moments, and the posterior with real
# Beta parameters
# ---------------------------------------------------------------------------
def test_fit_beta_moments_hand_example():
    """{0.2, 0.4}: mean 3/10, variance 1/100, so s(1-s)/v - 1 = 20 and
    Beta(6, 14) (worked by hand in exact fractions)."""
    mean = Fraction(3, 10)
    var = (Fraction(1, 10) ** 2 + Fraction(1, 10) ** 2) / 2
    c = mean * (1 - mean) / var - 1
    assert (mean * c, (1 - mean) * c) == (6, 14)
    a, b, fell = P.fit_beta_moments([0.2, 0.4])
    assert not fell
    assert a == pytest.approx(6.0, rel=1e-12) and b == pytest.approx(14.0, rel=1e-12)


@pytest.mark.parametrize("alpha,beta", [(0.37, 2.9), (2.0, 5.0), (7.5, 0.8), (40.0, 60.0)])
def test_fit_beta_moments_inverts_the_beta_moments(alpha, beta):
    """A two-point sample {mu - sd, mu + sd} has mean mu and variance sd^2; with
    the Beta's own moments mu = a/(a+b), sd^2 = ab/((a+b)^2 (a+b+1)) the fit
    returns (a, b)."""
    mu = alpha / (alpha + beta)
    sd = math.sqrt(alpha * beta / ((alpha + beta) ** 2 * (alpha + beta + 1.0)))
    a, b, fell = P.fit_beta_moments([mu - sd, mu + sd])
    assert not fell
    assert a == pytest.approx(alpha, rel=1e-10) and b == pytest.approx(beta, rel=1e-10)


def test_fit_beta_moments_large_sample_and_degenerate_cases():
    rng = np.random.default_rng(17)
    a, b, fell = P.fit_beta_moments(rng.beta(2.0, 5.0, 200_000))
    assert not fell and abs(a - 2.0) < 0.05 and abs(b - 5.0) < 0.12
    for bad in ([0.4], [0.3, 0.3, 0.3], [0.0, 1.0], [0.0, 0.0, 1.0, 1.0]):
        assert P.fit_beta_moments(bad) == (1.0, 1.0, True), bad
    # a sample too concentrated for the tables' range falls back too
    assert P.fit_beta_moments([0.5 - 1e-5, 0.5 + 1e-5])[2]


@pytest.mark.parametrize("m,n,alpha,beta,t", [(3, 32, 0.37, 2.9, 0.7), (20, 64, 2.5, 7.25, 0.5),
                                              (60, 64, 0.8, 0.6, 0.9), (0, 16, 1.7, 4.2, 0.3)])
def test_jaccard_posterior_with_real_prior(m, n, alpha, beta, t):
    """Real (learned) Beta parameters: the prune and concentration
    probabilities equal the regularized incomplete beta of the posterior
    Beta(m + alpha, n - m + beta) at 50 digits."""
    mpmath.mp.dps = 50
    a, b = mpmath.mpf(m) + mpmath.mpf(alpha), mpmath.mpf(n - m) + mpmath.mpf(beta)
    want = 1 - mpmath.betainc(a, b, 0, mpmath.mpf(t), regularized=True)
    assert P.jaccard_prune_prob(m, n, t, alpha, beta) == pytest.approx(float(want), rel=1e-10, abs=1e-15)
    s = P.jaccard_map(m, n, alpha, beta)
    lo, hi = max(0.0, s - 0.05), min(1.0, s + 0.05)
    want_c = mpmath.betainc(a, b, mpmath.mpf(lo), mpmath.mpf(hi), regularized=True)
    assert P.jaccard_concentration(m, n, 0.05, alpha, beta) == pytest.approx(float(want_c), rel=1e-10, abs=1e-15)


# ---------------------------------------------------------------------------
# LSH banding (Section 2)
# ---------------------------------------------------------------------------
def test_banding_against_brute_force():
    """Every pair whose keys agree in some band is listed exactly once, in its
    first agreeing band, in bucket-major order; no other pair is listed."""
    rng = np.random.default_rng(8)
    n, nb, b = 300, 6, 3
    bits = G.pack_bits(rng.integers(0, 2, size=(n, 32), dtype=np.uint8))
    x, y = R.band_candidates(bits, nb, b)
    keys = np.zeros((n, nb), np.int64)
    for i in range(n):                      # keys by hand, one bit at a time
        for j in range(nb):
            for t in range(b):
                h = j * b + t
                keys[i, j] |= ((int(bits[i, h // 32]) >> (h % 32)) & 1) << t
    first = {}
    for i in range(n):
        for k in range(i + 1, n):
            eq = np.flatnonzero(keys[i] == keys[k])
            if len(eq):
                first[(i, k)] = int(eq[0])
    got = list(zip(x.tolist(), y.tolist()))
    assert len(got) == len(set(got)) == len(first)
    assert set(got) == set(first)
    # order: band of first agreement, then key, then (x, y)
    order = [(first[p], keys[p[0], first[p]], p[0], p[1]) for p in got]
    assert order == sorted(order)


def test_banding_tiled_order():
    """The tiled order lists exactly the row-major order's pairs of each band
    and bucket, rearranged: for member positions (a, b) of one bucket, by tile
    row a // T, tile column b // T, then (a, b)."""
    rng = np.random.default_rng(9)
    n, nb, b, T = 400, 4, 2, 3
    bits = G.pack_bits(rng.integers(0, 2, size=(n, 32), dtype=np.uint8))
    x0, y0 = R.band_candidates(bits, nb, b)
    x1, y1 = R.band_candidates(bits, nb, b, tile=T)
    assert sorted(zip(x0.tolist(), y0.tolist())) == sorted(zip(x1.tolist(), y1.tolist()))
    keys = R.band_keys(bits, nb, b)
    # by hand: band of first agreement, bucket key, positions among the bucket's members
    def band_of(p):
        return int(np.flatnonzero(keys[p[0]] == keys[p[1]])[0])
    members = {}
    for j in range(nb):
        for i in range(n):
            members.setdefault((j, int(keys[i, j])), []).append(i)
    order = []
    for p in zip(x1.tolist(), y1.tolist()):
        j = band_of(p)
        mem = members[(j, int(keys[p[0], j]))]
        a, c = mem.index(p[0]), mem.index(p[1])
        order.append((j, int(keys[p[0], j]), a // T, c // T, a, c))
    assert order == sorted(order)
    assert any(o[2] != o[3] for o in order) and any(o[2] == o[3] for o in order)


@pytest.mark.parametrize("r", [0.6, 0.8])
def test_banding_collision_probability(r):
    """Section 2: with l bands of b bits, a pair whose bits agree independently
    with probability r becomes a candidate with probability 1 - (1 - r^b)^l."""
    rng = np.random.default_rng(int(r * 100))
    n_pairs, nb, b = 3000, 8, 6
    bits = G.pack_bits(G.calibration_bits(n_pairs, 64, np.full(n_pairs, r), int(r * 1000)))
    x, y = R.band_candidates(bits, nb, b, max_bucket=0)
    planted = np.sum((x % 2 == 0) & (y == x + 1))
    p = 1.0 - (1.0 - r ** b) ** nb
    sd = math.sqrt(n_pairs * p * (1 - p))
    assert abs(planted - n_pairs * p) < 4 * sd + 1, (planted, n_pairs * p)
