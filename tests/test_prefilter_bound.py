"""The half-precision prefilter's limit, checked on the CPU.

The matrix-core join screens a candidate with fp16 pieces of the float32
coordinates (x = xh + xl + e, each piece rounded toward zero), three products
per dimension and the query's limit L as two more pieces, and passes it when
the accumulated score is >= -h (h = -pn (1 - c0) / 2 from the candidate's
row).  The limit is widened so that every candidate the float32 direct form
accepts (dd <= thr) passes even if the matrix core's accumulation loses up
to 2^-22 of the summed magnitudes per product.  Here that claim is checked
directly: the pieces are formed as the kernel forms them, the score is
summed exactly (math.fsum of exact products), the worst-case accumulation
loss is subtracted, and the result must still reach -h, on adversarial pairs
(distances at the threshold, large norms against tiny distances,
coordinates at the range edge +-32, near the fp16 subnormal range,
duplicates).  A limit widened too little must fail the same check, and a
candidate far beyond the threshold must not pass.

The constants restate the kernel's (c0 = (8d + 24) 2^-24 in the row's h,
c16 = (139 NS + 120 + d) 2^-24 and cabs = (d + 8) 2^-24 in the limit,
L clamped at -30000).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

U = 2.0 ** -24


def f32(v):
    return float(np.float32(v))


def fma32(a, b, c):
    # a*b is exact in float64 for float32 inputs; one rounding to float32
    return f32(float(a) * float(b) + float(c))


def rtz16(x: float) -> float:
    """x rounded toward zero to half precision (fp16 subnormals kept)."""
    h = np.float16(x)
    if abs(float(h)) > abs(x):
        h = np.nextafter(h, np.float16(0.0))
    return float(h)


def split(x: float):
    hi = rtz16(x)
    lo = rtz16(f32(x - hi))            # the remainder is exact in float32
    return hi, lo


def steps(d: int) -> int:
    m = (d + 1) // 2
    words = 3 * (m // 2) + (2 if m % 2 else 1)
    return (words + 3) // 4


def direct(q, p):
    dd = 0.0
    for a, b in zip(q, p):
        t = f32(a - b)
        dd = fma32(t, t, dd)
    return dd


def norm(v):
    s = 0.0
    for a in v:
        s = fma32(a, a, s)
    return s


def h_of(p, d):
    c0 = f32((8 * d + 24) * U)
    return f32(-0.5 * f32(norm(p) * f32(1.0 - c0)))


def limit(qn, thr, d, widen=1.0):
    c16 = f32((139 * steps(d) + 120 + d) * U * widen)
    cabs = f32((d + 8) * U * widen)
    l = f32(fma32(-c16, f32(qn + thr), f32(0.5 * f32(qn - thr))) - cabs)
    return max(l, -30000.0)


def worst_score(q, p, L, d):
    """The exact score of the pieces minus the largest accumulation loss the
    limit allows for."""
    terms = []
    for a, b in zip(q, p):
        ah, al = split(a)
        bh, bl = split(b)
        terms += [ah * bh, ah * bl, al * bh]           # exact in float64
    nl = -L
    nlh = rtz16(nl)
    terms += [nlh, rtz16(f32(nl - nlh))]
    exact = math.fsum(terms)
    loss = (16 * steps(d) + 1) * 2.0 ** -22 * math.fsum(abs(t) for t in terms)
    return exact, loss


def pairs(kind, d, rng, count):
    """Query / candidate pairs of float32 coordinates."""
    out = []
    for _ in range(count):
        if kind == "unit":
            q = rng.random(d)
            p = q + rng.normal(0, 0.02, d)
        elif kind == "large_norm":            # tiny distances against |q| ~ 31 * sqrt(d)
            q = 31.0 + 1e-3 * rng.random(d)
            p = q + rng.normal(0, 1e-5, d)
        elif kind == "edge":                  # coordinates at the range edge
            q = rng.choice([-32.0, 32.0], d) * (1 - 1e-7 * rng.random(d))
            p = q + rng.normal(0, 1e-3, d)
        elif kind == "subnormal":             # pieces near the fp16 subnormal range
            q = 3e-6 * rng.random(d)
            p = q + rng.normal(0, 3e-8, d)
        else:                                 # duplicates: dd = 0 = thr
            q = rng.random(d)
            p = q.copy()
        q = np.clip(q, -32, 32).astype(np.float32)
        p = np.clip(p, -32, 32).astype(np.float32)
        out.append(([float(v) for v in q], [float(v) for v in p]))
    return out


KINDS = ["unit", "large_norm", "edge", "subnormal", "duplicate"]


@pytest.mark.parametrize("d", [2, 3, 5, 8, 10, 11, 15, 16])
def test_every_accepted_candidate_passes(d):
    rng = np.random.default_rng(700 + d)
    worst = math.inf
    for kind in KINDS:
        for q, p in pairs(kind, d, rng, 60):
            dd = direct(q, p)
            for thr in (dd, f32(dd * (1 + 4 * U))):          # at and just above the threshold
                L = limit(norm(q), thr, d)
                exact, loss = worst_score(q, p, L, d)
                slack = (exact - loss) - (-h_of(p, d))
                worst = min(worst, slack)
                assert slack >= 0.0, f"{kind} d={d}: a candidate with dd <= thr fails the screen by {-slack:.3e}"
    assert math.isfinite(worst)


@pytest.mark.parametrize("d", [3, 8, 15])
def test_a_limit_widened_too_little_fails(d):
    """The check has teeth: with a quarter of the widening, some adversarial
    candidate with dd <= thr is rejected."""
    rng = np.random.default_rng(900 + d)
    fails = 0
    for kind in ("large_norm", "edge"):
        for q, p in pairs(kind, d, rng, 60):
            dd = direct(q, p)
            L = limit(norm(q), dd, d, widen=0.25)
            exact, loss = worst_score(q, p, L, d)
            fails += (exact - loss) < -h_of(p, d)
    assert fails > 0


@pytest.mark.parametrize("d", [3, 8, 15])
def test_far_candidates_do_not_pass(d):
    """A candidate at twice the threshold distance (unit-range data) scores
    below -h even with the most favourable accumulation: the limit is not
    vacuous."""
    rng = np.random.default_rng(950 + d)
    for q, p in pairs("unit", d, rng, 60):
        dd = direct(q, p)
        if dd < 1e-4:
            continue
        L = limit(norm(q), f32(dd / 4.0), d)
        exact, loss = worst_score(q, p, L, d)
        assert exact + loss < -h_of(p, d)


# The alert kernel's object side (a pair must also pass when dd < rk_p, the
# population object's own k-th neighbour dd): the column's pass threshold is
# -h_p + min(0, A_q + B_p) with A_q = (1/2 + c16 - K u) T_q - 2 K u qn and
# B_p = -(1/2 + c16 + K u) rk_p - 4 u |h_p| (K = 64 NS + 32, twice what the
# accumulation bound of both limits needs), the alert's accumulator carrying
# its own limit L_q = limit(qn, T_q).


def k_slack(d):
    return 64 * steps(d) + 32


def object_side_threshold(qn, T, rk, hp, d):
    K = k_slack(d)
    c16 = f32((139 * steps(d) + 120 + d) * U)
    ca = f32(f32(0.5 + c16) - f32(K * U))
    cr = f32(f32(0.5 + c16) + f32(K * U))
    aq = fma32(ca, T, f32(f32(-2.0 * K * U) * qn))
    bp = fma32(-cr, rk, f32(-4 * U * abs(hp)))
    return f32(-hp + min(0.0, f32(aq + bp)))


@pytest.mark.parametrize("d", [2, 3, 5, 8, 10, 11, 15, 16])
def test_object_side_passes_every_counting_object(d):
    """Every object whose own k-th dd exceeds its direct-form distance to the
    alert passes, whatever the alert's own threshold (down to 0)."""
    rng = np.random.default_rng(1300 + d)
    for kind in KINDS:
        for q, p in pairs(kind, d, rng, 40):
            dd = direct(q, p)
            rk = float(np.nextafter(np.float32(dd), np.float32(np.inf)))     # dd < rk, tightest
            hp = h_of(p, d)
            for T in (0.0, f32(dd / 8), f32(dd * 0.999), rk, f32(4 * rk + 1e-3), 1e9):   # 1e9: clamped limit
                L = limit(norm(q), T, d)
                exact, loss = worst_score(q, p, L, d)
                x = object_side_threshold(norm(q), T, rk, hp, d)
                assert exact - loss >= x, f"{kind} d={d} T={T}: a counting object fails by {x - exact + loss:.3e}"


def object_side_variant(qn, T, rk, hp, d, mode):
    """Two plausible mistakes: B without its rk term (the object side adds
    nothing to the alert side), and A taken from a larger threshold than the
    row's own (the block row's largest instead of its smallest)."""
    K = k_slack(d)
    c16 = f32((139 * steps(d) + 120 + d) * U)
    ca = f32(f32(0.5 + c16) - f32(K * U))
    cr = f32(f32(0.5 + c16) + f32(K * U))
    if mode == "largest_row":
        T = f32(4 * T + 4 * rk)
    aq = fma32(ca, T, f32(f32(-2.0 * K * U) * qn))
    bp = f32(-4 * U * abs(hp)) if mode == "no_rk" else fma32(-cr, rk, f32(-4 * U * abs(hp)))
    return f32(-hp + min(0.0, f32(aq + bp)))


@pytest.mark.parametrize("mode", ["no_rk", "largest_row"])
@pytest.mark.parametrize("d", [3, 8, 15])
def test_object_side_check_catches_mistakes(d, mode):
    rng = np.random.default_rng(1400 + d)
    fails = 0
    for kind in ("unit", "large_norm", "edge"):
        for q, p in pairs(kind, d, rng, 40):
            dd = direct(q, p)
            rk = float(np.nextafter(np.float32(dd), np.float32(np.inf)))
            T = f32(dd / 8)
            L = limit(norm(q), T, d)
            exact, loss = worst_score(q, p, L, d)
            fails += (exact - loss) < object_side_variant(norm(q), T, rk, h_of(p, d), d, mode)
    assert fails > 0


@pytest.mark.parametrize("d", [3, 8, 15])
def test_object_side_is_not_vacuous(d):
    """An object at four times its own k-th dd from the alert (alert
    threshold 0) fails the object side even with the most favourable
    accumulation, once that dd is above the widening's scale (10^-3 qn)."""
    rng = np.random.default_rng(1500 + d)
    tested = 0
    for q, p in pairs("unit", d, rng, 40):
        dd = direct(q, p)
        if dd < 1e-3 * norm(q):
            continue
        L = limit(norm(q), 0.0, d)
        exact, loss = worst_score(q, p, L, d)
        assert exact + loss < object_side_threshold(norm(q), 0.0, f32(dd / 4), h_of(p, d), d)
        tested += 1
    assert tested >= 20
