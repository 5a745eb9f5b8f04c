// Host FP64 builder of the posterior decision tables (Section 4.3).
//
// For each level j (n = (j+1) k hashes compared) the table holds
//   minMatches(n): the smallest m with Pr[S >= t | M(m,n)] >= epsilon, found by
//                  binary search because that probability grows with m;
//   accept bits:   for m >= minMatches(n), whether Pr[|S - S_hat| < delta | M(m,n)]
//                  >= 1 - gamma (the cached concentration test).
//
// Jaccard (Section 4.1): the posterior is Beta(a, b), a = m + alpha,
// b = n - m + beta.  With integer a, b the regularized incomplete beta is a
// binomial tail, I_x(a, b) = Pr[Bin(a+b-1, x) >= a], so every probability is a
// finite sum of binomial terms (the Beta-binomial closed form), summed in FP64
// from log-space terms.  A learned prior (real alpha, beta > 0, fitted by the
// method of moments of Section 4.1) uses the continued fraction of I_x(a, b)
// instead, evaluated by the modified Lentz method, on the side of the mean
// where it converges fast (the other side through I_x(a,b) = 1 - I_{1-x}(b,a)).
//
// Cosine (Section 4.2): with r = 1 - theta/pi the posterior density of the
// angle is proportional to f(theta) = (1 - theta/pi)^m (theta/pi)^(n-m) on
// [0, pi/2], and the events of interest are angle intervals: S >= t is
// theta <= arccos(t), and |S - S_hat| < delta is
// arccos(min(1, S_hat + delta)) < theta < arccos(max(0, S_hat - delta)).
// Each probability is a ratio of integrals of f, computed by composite
// Gauss-Legendre quadrature over the angle, in log space relative to the
// peak of f so that no integral underflows.
#include <algorithm>
#include <cmath>
#include <thread>

#include "internal.h"

namespace blsh {
namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// ---------------- Jaccard: binomial sums ----------------
// Pr[Bin(N, x) <= c] for integer N >= 0, c, x in [0, 1].
double binom_cdf(int N, int c, double x) {
  if (c < 0) return 0.0;
  if (c >= N) return 1.0;
  if (x <= 0.0) return 1.0;
  if (x >= 1.0) return 0.0;
  const double lx = std::log(x), l1x = std::log1p(-x);
  const double lgN = std::lgamma(N + 1.0);
  // Sum whichever tail is shorter; all terms are positive.
  const double mean = N * x;
  if (c <= mean) {
    double s = 0.0;
    for (int j = 0; j <= c; ++j)
      s += std::exp(lgN - std::lgamma(j + 1.0) - std::lgamma(N - j + 1.0) + j * lx + (N - j) * l1x);
    return std::min(1.0, s);
  }
  double s = 0.0;
  for (int j = c + 1; j <= N; ++j)
    s += std::exp(lgN - std::lgamma(j + 1.0) - std::lgamma(N - j + 1.0) + j * lx + (N - j) * l1x);
  return std::max(0.0, 1.0 - s);
}

// I_x(a, b) for integer a, b >= 1.
double reg_inc_beta_int(int a, int b, double x) {
  if (x <= 0.0) return 0.0;
  if (x >= 1.0) return 1.0;
  return 1.0 - binom_cdf(a + b - 1, a - 1, x);
}

// Continued fraction of I_x(a, b) (real a, b > 0):
//   I_x(a,b) = x^a (1-x)^b / (a B(a,b)) / F,  F = 1 + d1 / (1 + d2 / (1 + ...)),
//   d_{2i+1} = -(a+i)(a+b+i) x / ((a+2i)(a+2i+1)),  d_{2i} = i(b-i) x / ((a+2i-1)(a+2i)),
// with F evaluated by the modified Lentz method; accurate where
// x < (a+1)/(a+b+2).
double inc_beta_cf(double a, double b, double x) {
  const double tiny = 1e-300, eps = 1e-16;
  double f = 1.0, C = 1.0, D = 0.0;
  for (int j = 1; j <= 20000; ++j) {
    double dj;
    if (j & 1) {
      const double i = (j - 1) / 2;
      dj = -(a + i) * (a + b + i) * x / ((a + 2.0 * i) * (a + 2.0 * i + 1.0));
    } else {
      const double i = j / 2;
      dj = i * (b - i) * x / ((a + 2.0 * i - 1.0) * (a + 2.0 * i));
    }
    D = 1.0 + dj * D;
    if (std::fabs(D) < tiny) D = tiny;
    D = 1.0 / D;
    C = 1.0 + dj / C;
    if (std::fabs(C) < tiny) C = tiny;
    const double step = C * D;
    f *= step;
    if (std::fabs(step - 1.0) < eps) break;
  }
  const double lpre = a * std::log(x) + b * std::log1p(-x) - std::log(a) -
                      (std::lgamma(a) + std::lgamma(b) - std::lgamma(a + b));
  return std::exp(lpre) / f;
}

// I_x(a, b) and its complement 1 - I_x(a, b), each without cancellation.
double reg_inc_beta(double a, double b, double x) {
  if (x <= 0.0) return 0.0;
  if (x >= 1.0) return 1.0;
  if (x < (a + 1.0) / (a + b + 2.0)) return inc_beta_cf(a, b, x);
  return 1.0 - inc_beta_cf(b, a, 1.0 - x);
}
double reg_inc_beta_upper(double a, double b, double x) {
  if (x <= 0.0) return 1.0;
  if (x >= 1.0) return 0.0;
  if (x < (a + 1.0) / (a + b + 2.0)) return 1.0 - inc_beta_cf(a, b, x);
  return inc_beta_cf(b, a, 1.0 - x);
}

struct Jaccard {
  double t, delta, alpha, beta;
  int ia, ib;
  bool integer;   // alpha, beta integers: exact binomial sums
  double prune_prob(int m, int n) const {   // 1 - I_t(m+alpha, n-m+beta)
    if (!integer) return reg_inc_beta_upper(m + alpha, n - m + beta, t);
    const int a = m + ia, b = n - m + ib;
    return binom_cdf(a + b - 1, a - 1, t);
  }
  double shat(int m, int n) const {
    double s = (m + alpha - 1.0) / (n + alpha + beta - 2.0);
    return std::min(1.0, std::max(0.0, s));
  }
  double concentration(int m, int n) const {
    const double s = shat(m, n);
    const double hi = std::min(1.0, s + delta), lo = std::max(0.0, s - delta);
    if (!integer) {
      const double a = m + alpha, b = n - m + beta;
      return reg_inc_beta(a, b, hi) - reg_inc_beta(a, b, lo);
    }
    const int a = m + ia, b = n - m + ib;
    return reg_inc_beta_int(a, b, hi) - reg_inc_beta_int(a, b, lo);
  }
};

// ---------------- Cosine: quadrature over the angle ----------------
// 16-point Gauss-Legendre nodes/weights on [-1, 1] (positive half; symmetric).
const double kGLx[8] = {0.0950125098376374401853193, 0.2816035507792589132304605, 0.4580167776572273863424194,
                        0.6178762444026437484466718, 0.7554044083550030338951012, 0.8656312023878317438804679,
                        0.9445750230732325760779884, 0.9894009349916499325961542};
const double kGLw[8] = {0.1894506104550684962853967, 0.1826034150449235888667637, 0.1691565193950025381893121,
                        0.1495959888165767320815017, 0.1246289712555338720524763, 0.0951585116824927848099251,
                        0.0622535239386478928628438, 0.0271524594117540948517806};

struct CosinePair {
  int m, n;
  double lmax, lo_eff, hi_eff;  // effective support of f on [0, pi/2]
  double logf(double th) const {
    double v = 0.0;
    if (m) v += m * std::log1p(-th / kPi);
    if (n - m) v += (th > 0.0) ? (n - m) * std::log(th / kPi) : -INFINITY;
    return v;
  }
  CosinePair(int m_, int n_) : m(m_), n(n_) {
    const double half = kPi / 2.0;
    double peak = kPi * (1.0 - double(m) / n);
    peak = std::min(half, std::max(0.0, peak));
    lmax = logf(peak);
    const double drop = 75.0;  // e^-75 ~ 3e-33 relative: negligible
    // f is unimodal: bisection on each side for logf = lmax - drop
    auto edge = [&](double in, double out) {
      if (logf(out) >= lmax - drop) return out;
      for (int it = 0; it < 80; ++it) {
        double mid = 0.5 * (in + out);
        if (logf(mid) >= lmax - drop) in = mid; else out = mid;
      }
      return out;
    };
    lo_eff = edge(peak, 0.0);
    hi_eff = edge(peak, half);
  }
  // integral of f(theta) e^{-lmax} over [a, b] intersected with the support
  double integral(double a, double b) const {
    a = std::max(a, lo_eff);
    b = std::min(b, hi_eff);
    if (!(b > a)) return 0.0;
    const double width = hi_eff - lo_eff;
    int panels = int(std::ceil(96.0 * (b - a) / width)) + 2;
    const double h = (b - a) / panels;
    double s = 0.0;
    for (int p = 0; p < panels; ++p) {
      const double c = a + (p + 0.5) * h, r = 0.5 * h;
      double ps = 0.0;
      for (int q = 0; q < 8; ++q) {
        ps += kGLw[q] * (std::exp(logf(c - r * kGLx[q]) - lmax) + std::exp(logf(c + r * kGLx[q]) - lmax));
      }
      s += ps * r;
    }
    return s;
  }
};

struct Cosine {
  double t, delta;
  double prune_prob(int m, int n) const {
    CosinePair f(m, n);
    const double den = f.integral(0.0, kPi / 2.0);
    return f.integral(0.0, std::acos(t)) / den;
  }
  double shat(int m, int n) const { return std::cos(kPi * (1.0 - std::max(0.5, double(m) / n))); }
  double concentration(int m, int n) const {
    CosinePair f(m, n);
    const double den = f.integral(0.0, kPi / 2.0);
    const double s = shat(m, n);
    const double th_lo = std::acos(std::min(1.0, s + delta));
    const double th_hi = std::min(kPi / 2.0, std::acos(std::max(0.0, s - delta)));
    return f.integral(th_lo, th_hi) / den;
  }
};

// Where a level's smallest margin was found: |probability - threshold| at
// (n, m), for the prune test (kind 0) or the concentration test (kind 1).
struct Margin {
  double v = 1.0;
  int n = 0, m = 0, kind = 0;
  void take(double d, int n_, int m_, int kind_) {
    if (d < v) { v = d; n = n_; m = m_; kind = kind_; }
  }
};

template <class Model>
void build_level(const Model &mdl, const TableKey &key, int j, HostTable *out, Margin *margin) {
  const int n = (j + 1) * key.k;
  // minMatches(n): binary search for the first m with prune_prob >= epsilon.
  int lo = 0, hi = n + 1;  // answer in [lo, hi]; hi = n+1 means "always prune"
  while (lo < hi) {
    int mid = (lo + hi) / 2;
    if (mdl.prune_prob(mid, n) >= key.epsilon) hi = mid; else lo = mid + 1;
  }
  const int mm = lo;
  out->min_matches[j] = mm;
  Margin mg;
  if (mm <= n) mg.take(std::fabs(mdl.prune_prob(mm, n) - key.epsilon), n, mm, 0);
  if (mm > 0 && mm - 1 <= n) mg.take(std::fabs(mdl.prune_prob(mm - 1, n) - key.epsilon), n, mm - 1, 0);
  if (!key.lite) {
    for (int m = mm; m <= n; ++m) {
      const double c = mdl.concentration(m, n);
      mg.take(std::fabs(c - (1.0 - key.gamma)), n, m, 1);
      if (c >= 1.0 - key.gamma) out->accept[size_t(j) * out->words + (m >> 5)] |= 1u << (m & 31);
    }
  }
  *margin = mg;
}

template <class Model>
void build_all(const Model &mdl, const TableKey &key, HostTable *out) {
  std::vector<Margin> margins(key.n_levels);
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nt = std::min<unsigned>(nt, key.n_levels);
  std::vector<std::thread> th;
  for (unsigned w = 0; w < nt; ++w)
    th.emplace_back([&, w] {
      for (int j = int(w); j < key.n_levels; j += int(nt)) build_level(mdl, key, j, out, &margins[j]);
    });
  for (auto &x : th) x.join();
  const Margin *lo = &margins[0];
  for (const Margin &m : margins)
    if (m.v < lo->v) lo = &m;
  out->min_margin = lo->v;
  out->margin_n = lo->n;
  out->margin_m = lo->m;
  out->margin_kind = lo->kind;
}

}  // namespace

int build_table(const TableKey &key, HostTable *out) {
  out->k = key.k;
  out->n_levels = key.n_levels;
  out->n_max = key.k * key.n_levels;
  out->words = (out->n_max + 1 + 31) / 32;
  out->min_matches.assign(key.n_levels, 0);
  out->accept.assign(size_t(key.n_levels) * out->words, 0u);
  if (key.measure == BLSH_JACCARD) {
    const bool integer = key.alpha == std::floor(key.alpha) && key.beta == std::floor(key.beta) && key.alpha >= 1.0 &&
                         key.beta >= 1.0;
    Jaccard mdl{key.t, key.delta, key.alpha, key.beta, int(key.alpha), int(key.beta), integer};
    build_all(mdl, key, out);
  } else {
    Cosine mdl{key.t, key.delta};
    build_all(mdl, key, out);
  }
  // A probability this close to its threshold could fall on either side of it
  // under another (equally valid) evaluation of the posterior: the decision at
  // that (n, m) is not determined, so the parameter set is refused rather
  // than answered one way silently.
  if (out->min_margin < kTieMargin)
    return fail(BLSH_EINVAL,
                "posterior table: %s at n=%d, m=%d lies within %.3g of its threshold (%s = %.17g); decisions "
                "there are not determined in FP64 -- change the parameters slightly",
                out->margin_kind == 0 ? "Pr[S >= t | M(m,n)]" : "Pr[|S - S_hat| < delta | M(m,n)]", out->margin_n,
                out->margin_m, out->min_margin, out->margin_kind == 0 ? "epsilon" : "1 - gamma",
                out->margin_kind == 0 ? key.epsilon : 1.0 - key.gamma);
  return BLSH_OK;
}

}  // namespace blsh
