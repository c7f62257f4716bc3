"""Pins of three readings the oracle takes where the paper leaves a choice, each
against a value computed here by other means, so that a plausible slip in the
oracle (and in the library, which matches it bit for bit) fails a test:

* Lloyd's stop (Section 5: at most 300 iterations, relative tolerance 1e-4),
  read as f_prev - f <= tol * f over the objective, at most max_iter centroid
  updates: checked on a 1-D instance whose whole Lloyd trace is computed here
  in exact rational arithmetic.  A tolerance taken against f_prev, a strict
  '<', or an off-by-one update cap each stop at another update.
* The re-evaluation of an incumbent after a size change (Section 4.2;
  Algorithm 1): one fresh sample of the new size, drawn from the RECALC
  stream with counter t, only when the worker has an incumbent and its size
  changed.  Every sample the oracle draws is recorded and compared with the
  list these rules give.
* The size draws (Algorithm 1: s uniform in [s_min, s_max]; the log-uniform
  and bin laws of the measured workloads): exact sizes for chosen random words,
  including both ends of the range, against 60-digit decimal arithmetic.
"""

import math
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

from oracle import bigmeans, kmeans, rng

# ---------------------------------------------------------------------------
# Lloyd's stopping rule
# ---------------------------------------------------------------------------
# Ten points on a line and two starting centres; every cluster mean along the
# way is an integer, so every objective is an integer and exact in FP64.
LINE_X = [2, 6, 16, 20, 26, 38, 40, 42, 47, 53]
LINE_C0 = [2, 6]


def _exact_lloyd_trace(X, C, steps):
    """Objective and centres before each of `steps` updates, in exact rationals
    (nearest centre with the lowest index on ties; an empty cluster keeps its
    centre)."""
    C = [Fraction(c) for c in C]
    trace, cents = [], []
    for _ in range(steps + 1):
        lab = []
        for x in X:
            best = 0
            for j in range(1, len(C)):
                if (x - C[j]) ** 2 < (x - C[best]) ** 2:
                    best = j
            lab.append(best)
        trace.append(sum((x - C[a]) ** 2 for x, a in zip(X, lab)))
        cents.append(list(C))
        for j in range(len(C)):
            mem = [x for x, a in zip(X, lab) if a == j]
            if mem:
                C[j] = Fraction(sum(mem), len(mem))
    return trace, cents


def _oracle_line(tol, max_iter=300):
    X = np.array(LINE_X, dtype=np.float64)[:, None]
    C0 = np.array(LINE_C0, dtype=np.float64)[:, None]
    return kmeans.lloyd(X, C0, max_iter=max_iter, tol=tol)


def test_line_instance_trace_is_exact():
    trace, cents = _exact_lloyd_trace(LINE_X, LINE_C0, 5)
    assert [int(f) for f in trace] == [8062, 1258, 718, 628, 538, 538]
    assert all(f.denominator == 1 for f in trace)
    assert all(c.denominator == 1 for cc in cents for c in cc)
    out = _oracle_line(0.0)
    assert out["trace"] == [float(f) for f in trace]
    assert out["iters"] == 5


@pytest.mark.parametrize("tol,iters", [
    (10.0, 1),    # the first update already decreases by less than 10 f
    (0.5, 3),     # (f_prev - f)/f: 5.41, 0.752, 0.143 -> stop after 3 updates
    (0.15, 3),
    (0.1, 5),     # 0.143 and then 0.167 exceed 0.1; the fifth update changes nothing
    (0.0, 5),
])
def test_tolerance_is_relative_to_the_new_objective(tol, iters):
    trace, cents = _exact_lloyd_trace(LINE_X, LINE_C0, 5)

    def expected_stop(rel_to_prev, strict):
        for t in range(1, len(trace)):
            dec = trace[t - 1] - trace[t]
            bound = Fraction(tol) * (trace[t - 1] if rel_to_prev else trace[t])
            if (dec < bound) if strict else (dec <= bound):
                return t
        return len(trace) - 1

    assert expected_stop(False, False) == iters
    out = _oracle_line(tol)
    assert out["iters"] == iters
    assert out["f"] == float(trace[iters])
    assert np.array_equal(out["C"][:, 0], [float(c) for c in cents[iters]])


def test_tolerance_against_f_prev_would_stop_earlier():
    # at tol = 0.5 the second update decreases f by 540: more than 0.5 * 718
    # (the reading: continue) but less than 0.5 * 1258 (against f_prev: stop)
    trace, _ = _exact_lloyd_trace(LINE_X, LINE_C0, 5)
    dec = trace[1] - trace[2]
    assert Fraction(1, 2) * trace[2] < dec <= Fraction(1, 2) * trace[1]
    assert _oracle_line(0.5)["iters"] == 3


def test_tolerance_equality_stops():
    # tol = fl(45/314): after the third update f_prev - f = 90 and tol * f
    # = fl(45/314) * 628 rounds to exactly 90.0, so '<=' stops there; a strict
    # '<' would run on (the fourth decrease, 90/538, exceeds tol) to the fifth
    tol = 45 / 314
    assert tol * 628.0 == 90.0
    assert 90.0 / 538.0 > tol
    out = _oracle_line(tol)
    assert out["iters"] == 3 and out["f"] == 628.0


@pytest.mark.parametrize("cap", [0, 1, 2, 4])
def test_update_cap_counts_updates(cap):
    # at most `cap` centroid updates; the returned f is that of the returned C
    trace, cents = _exact_lloyd_trace(LINE_X, LINE_C0, 5)
    out = _oracle_line(0.0, max_iter=cap)
    assert out["iters"] == cap
    assert out["f"] == float(trace[cap])
    assert np.array_equal(out["C"][:, 0], [float(c) for c in cents[cap]])


def test_nonfinite_objective_stops_before_any_update():
    X = np.array(LINE_X + [float("nan")], dtype=np.float64)[:, None]
    out = kmeans.lloyd(X, np.array(LINE_C0, dtype=np.float64)[:, None], tol=0.0)
    assert out["iters"] == 0 and math.isnan(out["f"])
    assert np.array_equal(out["C"][:, 0], LINE_C0)


# ---------------------------------------------------------------------------
# Re-evaluation of the incumbent after a size change
# ---------------------------------------------------------------------------
@pytest.fixture
def recorded_samples(monkeypatch):
    """Record every sample the oracle's Algorithm 1 draws, with the objective
    it computes on each re-evaluation sample."""
    calls = []
    orig_sample = bigmeans._sample
    orig_objective = kmeans.objective

    def sample(X, s, seed, worker, purpose, g):
        calls.append({"purpose": purpose, "worker": worker, "g": g, "s": s, "f": None})
        return orig_sample(X, s, seed, worker, purpose, g)

    def objective(X, C):
        f = orig_objective(X, C)
        if calls and calls[-1]["purpose"] == rng.PURPOSE_RECALC and calls[-1]["f"] is None:
            calls[-1]["f"] = f
            calls[-1]["C"] = np.array(C, dtype=np.float64)
        return f

    monkeypatch.setattr(bigmeans, "_sample", sample)
    monkeypatch.setattr(kmeans, "objective", objective)
    return calls


def _blobs(m=3000, seed=0):
    r = np.random.default_rng(seed)
    mu = r.uniform(-10, 10, size=(4, 2))
    return (mu[r.integers(4, size=m)] + r.standard_normal((m, 2))).astype(np.float32)


def _expected_recalcs(P, X_m, finite_from=None):
    """(worker, g, s) of every re-evaluation the reading implies: round t >= 1
    of worker w when its size differs from round t-1's and the worker holds an
    incumbent (it has one after any round whose first pass beat +inf)."""
    out = []
    for w in range(P.workers):
        prev = None
        for t in range(P.rounds_T):
            s, _ = bigmeans.draw_size(P, w, t, {"acc": [0] * 5, "passes": [0] * 5})
            has_inc = t >= 1 if finite_from is None else finite_from(w, t)
            if has_inc and prev is not None and s != prev:
                out.append((w, t, s))
            prev = s
    return sorted(out)


def test_recalc_samples_follow_the_reading(recorded_samples):
    X = _blobs()
    # a narrow log-uniform range: sizes repeat between rounds often enough
    # that both branches (changed and unchanged) occur
    P = bigmeans.Params(k=3, workers=4, rounds_T=6, passes_p=2, s_min=300, s_max=303,
                        size_policy=bigmeans.SIZE_LOGUNIFORM, seed=7)
    bigmeans.bigmeans_run(X, P)
    rec = [c for c in recorded_samples if c["purpose"] == rng.PURPOSE_RECALC]
    exp = _expected_recalcs(P, X.shape[0])
    unchanged = sum(1 for w in range(4) for t in range(1, 6)
                    if bigmeans.draw_size(P, w, t, None)[0] == bigmeans.draw_size(P, w, t - 1, None)[0])
    assert unchanged > 0 and len(exp) > 0
    assert sorted((c["worker"], c["g"], c["s"]) for c in rec) == exp
    # every other sample is a pass sample: purpose SAMPLE, counter t * p + q
    passes = [c for c in recorded_samples if c["purpose"] == rng.PURPOSE_SAMPLE]
    assert len(passes) == P.workers * P.rounds_T * P.passes_p
    assert sorted((c["worker"], c["g"]) for c in passes) == sorted(
        (w, g) for w in range(P.workers) for g in range(P.rounds_T * P.passes_p))
    # the re-scored f_hat is f(C_w, S) on exactly that sample (brute force)
    Xd = X.astype(np.float64)
    for c in rec:
        idx = rng.sample_indices(X.shape[0], c["s"], P.seed, c["worker"], rng.PURPOSE_RECALC,
                                 c["g"])
        S = Xd[idx]
        d = ((S[:, None, :] - c["C"][None, :, :]) ** 2).sum(axis=2).min(axis=1)
        assert c["f"] == pytest.approx(math.fsum(d.tolist()), rel=1e-12)


def test_no_recalc_at_fixed_size(recorded_samples):
    X = _blobs()
    P = bigmeans.Params(k=3, workers=3, rounds_T=4, passes_p=2, s_min=400, s_max=400,
                        size_policy=bigmeans.SIZE_FIXED, seed=2)
    bigmeans.bigmeans_run(X, P)
    assert not [c for c in recorded_samples if c["purpose"] == rng.PURPOSE_RECALC]


def test_no_recalc_without_incumbent(recorded_samples):
    # NaN rows in every sample: no pass is ever accepted, f_hat stays +inf, so
    # no size change triggers a re-evaluation
    X = _blobs()
    X[::5] = np.nan
    P = bigmeans.Params(k=3, workers=2, rounds_T=4, passes_p=1, s_min=200, s_max=900,
                        size_policy=bigmeans.SIZE_UNIFORM, seed=3)
    out = bigmeans.bigmeans_run(X, P)
    assert out["L"] == []
    sizes = [[bigmeans.draw_size(P, w, t, None)[0] for t in range(4)] for w in range(2)]
    assert any(a != b for row in sizes for a, b in zip(row, row[1:]))
    assert not [c for c in recorded_samples if c["purpose"] == rng.PURPOSE_RECALC]


# ---------------------------------------------------------------------------
# Size draws at chosen random words
# ---------------------------------------------------------------------------
getcontext().prec = 60
MAXW = (1 << 64) - 1


def _u(w):
    return Decimal(w >> 11) / Decimal(2 ** 53)


def _floor_dec(x):
    return int(x.to_integral_value(rounding="ROUND_FLOOR"))


def _with_words(monkeypatch, words):
    """Make every Philox block the oracle's size draw asks for return `words`."""
    monkeypatch.setattr(rng, "philox_block_scalar", lambda ctr, key: tuple(words))


def _draw(P, t=0, stats=None):
    return bigmeans.draw_size(P, 0, t, stats or {"acc": [0] * 5, "passes": [0] * 5})


@pytest.mark.parametrize("a,b", [(4096, 65536), (1 << 12, 1 << 17), (3000, 50000), (1024, 262144)])
def test_loguniform_exact_sizes(monkeypatch, a, b):
    P = bigmeans.Params(k=1, workers=1, rounds_T=1, s_min=a, s_max=b,
                        size_policy=bigmeans.SIZE_LOGUNIFORM)
    la, lb1 = Decimal(a).ln(), Decimal(b + 1).ln()
    r = np.random.default_rng(a)
    words = [0, MAXW, 1 << 63, 1 << 62, 3 << 62] + [int(x) for x in r.integers(0, 2 ** 63, 40)]
    checked = 0
    for w0 in words:
        _with_words(monkeypatch, (w0, 0, 0, 0))
        exact = (la + _u(w0) * (lb1 - la)).exp()
        frac = exact - exact.to_integral_value(rounding="ROUND_FLOOR")
        if Decimal("1e-9") < frac < 1 - Decimal("1e-9") or w0 in (0, MAXW):
            want = min(max(_floor_dec(exact), a), b)
            assert _draw(P)[0] == want, (w0, exact)
            checked += 1
    assert checked >= 40
    # the ends: the smallest word gives s_min, the largest s_max (the law
    # reaches b + 1 exclusive, so s_max has probability ln((b+1)/b)/ln((b+1)/a);
    # with ln b in place of ln(b + 1) the largest word would give b - 1)
    _with_words(monkeypatch, (0, 0, 0, 0))
    assert _draw(P)[0] == a
    _with_words(monkeypatch, (MAXW, 0, 0, 0))
    assert _draw(P)[0] == b
    assert _floor_dec((la + _u(MAXW) * (Decimal(b).ln() - la)).exp()) == b - 1


def test_uniform_exact_sizes(monkeypatch):
    a, b = 1000, 4000
    P = bigmeans.Params(k=1, workers=1, rounds_T=1, s_min=a, s_max=b,
                        size_policy=bigmeans.SIZE_UNIFORM)
    for w0, want in [(0, a), (MAXW, b), (1 << 63, a + 3001 // 2), ((1 << 64) // 3001 * 7, a + 6),
                     ((1 << 64) // 3001 * 7 - 1, a + 6)]:
        _with_words(monkeypatch, (w0, 0, 0, 0))
        assert _draw(P)[0] == want == a + (w0 * (b - a + 1) >> 64)


def test_bins_exact_sizes(monkeypatch):
    a, b = 1 << 12, 1 << 17
    P = bigmeans.Params(k=1, workers=1, rounds_T=1, s_min=a, s_max=b,
                        size_policy=bigmeans.SIZE_BINS)
    stats = {"acc": [0, 3, 0, 9, 1], "passes": [8, 8, 4, 10, 30]}
    wts = [Fraction(stats["acc"][i] + 1, stats["passes"][i] + 2) for i in range(5)]
    tot = sum(wts)
    la, lb1 = Decimal(a).ln(), Decimal(b + 1).ln()
    width = (lb1 - la) / 5
    r = np.random.default_rng(5)
    for _ in range(60):
        w1, w2 = (int(x) for x in r.integers(0, 2 ** 63, 2))
        _with_words(monkeypatch, (0, w1, w2, 0))
        x = Fraction(w1 >> 11, 2 ** 53) * tot
        acc, want_bin = Fraction(0), 4
        for i in range(5):
            acc += wts[i]
            if x < acc:
                want_bin = i
                break
        exact = (la + (Decimal(want_bin) + _u(w2)) * width).exp()
        s, got_bin = _draw(P, t=1, stats=stats)
        assert got_bin == want_bin
        if Decimal("1e-9") < exact - _floor_dec(exact) < 1 - Decimal("1e-9"):
            assert s == min(max(_floor_dec(exact), a), b)
    # round 0 is the log-uniform draw over the whole range
    _with_words(monkeypatch, (MAXW, 0, 0, 0))
    assert _draw(P, t=0, stats=stats)[0] == b
