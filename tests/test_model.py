"""Pins for the reading of the truncated reduction (Section 5, Theorems 1-2).

Every variant of oracle/montred_model.py is compared with the exact
Montgomery integer (T + qN)/R, the value Algorithm 5 returns, exhaustively
over small limb widths and randomly at the library's limb width.
"""
import random

import pytest

import oracle
from oracle import montred_model as m

SMALL = [(2, 2), (3, 2), (4, 2), (3, 3), (4, 3), (3, 4)]


def _cases(L, n, cap=None):
    """Every odd N <= R/4 and evenly spaced T < 4N^2 (all T when few enough), plus T = 4N^2 - 1."""
    R = 1 << (L * n)
    mods = range(3, R // 4 + 1, 2)
    if cap is None:
        cap = max(64, 60000 // len(mods))
    for N in mods:
        lim = 4 * N * N
        step = max(1, lim // cap)
        for T in range(0, lim, step):
            yield N, T
        yield N, lim - 1


@pytest.mark.parametrize("L,n", SMALL)
def test_theorem1_and_ceil_reading_exhaustive(L, n):
    for N, T in _cases(L, n):
        e = m.redc_exact(T, N, L, n)
        assert m.theorem1_form(T, N, L, n) == e
        if 2 * n - 3 < (1 << L):
            assert m.redc_truncated(T, N, L, n, "floor") == e
        if n - 1 < (1 << (L - 1)):
            assert m.redc_truncated(T, N, L, n, "nearest") == e
        if m.fullcol_condition(L, n):
            assert m.redc_truncated_fullcol(T, N, L, n) == e


def test_ceil_reading_needs_its_condition():
    """At L=2, n=4 the unknown carry reaches 2^L and the ceil reading must fail somewhere."""
    L, n = 2, 4
    bad = sum(m.redc_truncated(T, N, L, n) != m.redc_exact(T, N, L, n) for N, T in _cases(L, n, 400))
    assert bad > 0


def test_literal_reading_disagrees_with_exact_redc():
    """Feeding c_add in as the carry into column n-1 (equations (3)-(5) read literally) is wrong."""
    for L, n in SMALL:
        bad = sum(m.redc_truncated_literal(T, N, L, n) != m.redc_exact(T, N, L, n)
                  for N, T in _cases(L, n, 300))
        assert bad > 0, (L, n)


def test_fullcol_reading_fails_when_window_too_narrow():
    rng = random.Random(11)
    L, n = 1, 8
    assert not m.fullcol_condition(L, n)
    R = 1 << (L * n)
    bad = 0
    for _ in range(3000):
        N = rng.randrange(3, R // 4 + 1) | 1
        if N > R // 4:
            N -= 2
        T = rng.randrange(4 * N * N)
        bad += m.redc_truncated_fullcol(T, N, L, n) != m.redc_exact(T, N, L, n)
    assert bad > 0


@pytest.mark.parametrize("n", [3, 5, 10, 19, 37, 74, 110, 147])
def test_fullcol_reading_random_at_28bit_limbs(n):
    rng = random.Random(100 + n)
    L = 28
    assert m.fullcol_condition(L, n)
    R = 1 << (L * n)
    t = L * n - 2
    for trial in range(40):
        N = rng.getrandbits(t) | 1 | (1 << (t - 1))
        specials = [0, 1, N, 2 * N - 1, (2 * N - 1) ** 2, 1 << t, (1 << t) << L, R - 1, R]
        T = specials[trial] if trial < len(specials) else rng.randrange(4 * N * N)
        e = m.redc_exact(T, N, L, n)
        assert m.redc_truncated_fullcol(T, N, L, n) == e
        assert e == oracle.redc(T, N, L * n)
        if T < 4 * N * N:
            assert e < 2 * N


def test_counts_formulas():
    # products per operation derived from the schedules; n=33 / 65 at 32-bit limbs
    for n, mul_p, mul_t, sqr_p, sqr_t in ((33, 2739, 2243, 2211, 1715), (65, 10595, 8579, 8515, 6499),
                                          (129, 41667, 33539, 33411, 25283)):
        c = m.counts(n)
        assert (c["mul_plain"], c["mul_trunc"], c["sqr_plain"], c["sqr_trunc"]) == (mul_p, mul_t, sqr_p, sqr_t)
    # the truncated partial-product set of Theorem 2 has n(n+1)/2 + n - 1 members
    for n in (2, 3, 7, 33):
        cnt = sum(1 for i in range(n) for j in range(n) if i + j >= n - 2)
        assert cnt == n * (n + 1) // 2 + n - 1


def _cios_operands(L, n, cap):
    """Odd N <= R/4 and operand pairs A, B < 2N (evenly spaced, plus the extremes)."""
    R = 1 << (L * n)
    for N in range(3, R // 4 + 1, 2):
        lim = 2 * N
        step = max(1, lim // cap)
        vals = list(range(0, lim, step)) + [lim - 1]
        for A in vals:
            for B in vals:
                yield N, A, B


@pytest.mark.parametrize("L,n", SMALL)
def test_cios_equals_exact_redc_exhaustive(L, n):
    """Algorithm 4 with lazy column sums returns the exact Montgomery integer (AB + qN)/R."""
    for N, A, B in _cios_operands(L, n, 24):
        got, _ = m.redc_cios(A, B, N, L, n)
        assert got == m.redc_exact(A * B, N, L, n), (L, n, N, A, B)


@pytest.mark.parametrize("n", [3, 10, 37, 74])
def test_cios_random_at_28bit_limbs_and_column_bound(n):
    """At the library's limb width the lazy column sums stay below 2n 2^(2L), within 64 bits up to n = 127."""
    rng = random.Random(300 + n)
    L = 28
    t = L * n - 2
    worst = 0
    for trial in range(12):
        if trial < 3:
            # every limb of N at its maximum below 2^t: the largest q_i N_j products
            N = (1 << t) - 1
        else:
            N = rng.getrandbits(t) | 1 | (1 << (t - 1))
        ops = [(2 * N - 1, 2 * N - 1), (0, 2 * N - 1), (1, 1)]
        A, B = ops[trial] if trial < 3 else (rng.randrange(2 * N), rng.randrange(2 * N))
        got, peak = m.redc_cios(A, B, N, L, n)
        e = m.redc_exact(A * B, N, L, n)
        assert got == e == oracle.redc(A * B, N, L * n)
        assert e < 2 * N
        worst = max(worst, peak)
    assert worst < 2 * n * (1 << (2 * L))
    assert 2 * 127 * (1 << (2 * L)) <= 1 << 64


def test_cios_and_truncated_counts():
    """CIOS needs 2n^2 + n products for a product and a square alike; truncation wins on squares."""
    for n in (37, 74):
        c = m.counts(n)
        assert c["mul_cios"] == c["sqr_cios"] == 2 * n * n + n
        assert c["sqr_trunc"] < c["sqr_cios"]
        # the multiplication counts differ by n - 1: 2n^2 + 2n - 1 against 2n^2 + n
        assert c["mul_trunc"] - c["mul_cios"] == n - 1


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_karatsuba_columns_equal_schoolbook_columns(levels):
    """Limb-wise half sums make D1 - D0 - D2 exact column by column, so every column matches the schoolbook's."""
    rng = random.Random(400 + levels)
    for k in (1, 2, 3, 4, 5, 7, 8, 19, 37, 74):
        a = [rng.getrandbits(28) for _ in range(k)]
        b = [rng.getrandbits(28) for _ in range(k)]
        sb, cnt_sb = m.kara_columns(a, b, 0)
        assert cnt_sb == k * k
        for xmin in sorted({0, k - 2, k - 1, k, 2 * k - 2}):
            got, _ = m.kara_columns(a, b, levels, xmin)
            for x in range(max(xmin, 0), 2 * k - 1):
                assert got[x] == sb[x], (k, levels, xmin, x)


@pytest.mark.parametrize("L,n", [(2, 2), (3, 2), (4, 2), (3, 3), (2, 4), (3, 4)])
def test_truncated_karatsuba_reduction_exhaustive(L, n):
    for N, T in _cases(L, n, 200):
        if not m.fullcol_condition(L, n):
            continue
        e = m.redc_exact(T, N, L, n)
        for levels in (1, 2):
            got, _ = m.redc_truncated_karatsuba(T, N, L, n, levels)
            assert got == e, (L, n, N, T, levels)


@pytest.mark.parametrize("n", [4, 37, 74, 111, 148])
def test_truncated_karatsuba_reduction_random_at_28bit_limbs(n):
    rng = random.Random(500 + n)
    L = 28
    t = L * n - 2
    for trial in range(6):
        N = rng.getrandbits(t) | 1 | (1 << (t - 1))
        T = [0, (2 * N - 1) ** 2][trial] if trial < 2 else rng.randrange(4 * N * N)
        e = m.redc_exact(T, N, L, n)
        for levels in (1, 2):
            got, _ = m.redc_truncated_karatsuba(T, N, L, n, levels)
            assert got == e, (n, trial, levels)


def test_truncated_karatsuba_counts():
    """One level: the truncated high half of q*N costs about two thirds of a whole one-level Karatsuba product
    (D2 whole, the upper halves of D1 and D0), i.e. about n^2 / 2, the truncated schoolbook's leading term."""
    for n in (74, 148):
        mm = (n + 1) // 2
        rng = random.Random(n)
        q = [rng.getrandbits(28) for _ in range(n)]
        N = [rng.getrandbits(28) for _ in range(n)]
        _, full = m.kara_columns(q, N, 1, 0)
        _, trunc = m.kara_columns(q, N, 1, n - 2)
        assert full == 3 * mm * mm
        assert 0.6 < trunc / full < 0.72, trunc / full
        sb_trunc = n * (n + 1) // 2 + n - 1
        assert abs(trunc - sb_trunc) < 3 * n, (trunc, sb_trunc)
