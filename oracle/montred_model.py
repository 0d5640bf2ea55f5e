"""Limb-level model of the truncated Montgomery reduction -- TEST INFRASTRUCTURE.

Written from Section 5 (Algorithm 6, Theorem 1, Theorem 2 and equations
(1)-(5)); ``redc_cios`` from Section 4 (Algorithm 4); ``kara_columns`` and
``redc_truncated_karatsuba`` from Section 3 and the Karatsuba part of
Section 5.  It is a checker of the *reading* of the paper, not part of the GPU
library, and shares nothing with it.

Setting: limbs of L bits, R = 2^(L*n), N odd with 4N <= R, T < 4N^2,
N' = -N^{-1} mod R.  Algorithm 6 returns

    C = floor(T / R) + floor(q*N / R) + c_add,     q = T*N' mod R,

where (Theorem 1) c_add = 1 exactly when T mod R != 0: the low n limbs of
T + q*N are zero, and their sum produces a carry out iff T's low part is
non-zero.

Theorem 2 says floor(q*N / R) needs only the partial products of q*N that
land at limb weight >= n-1.  With each partial product q_i*N_j split as
lo + hi*2^L, write

    S  = sum_{i+j=n-1} lo(q_i N_j) + sum_{i+j=n-2} hi(q_i N_j)          (column n-1)
    H' = sum_{i+j>=n} lo(q_i N_j) 2^{L(i+j-n)} + sum_{i+j>=n-1} hi(q_i N_j) 2^{L(i+j+1-n)}

The carry gamma that the skipped columns (< n-1) of T + q*N push into
column n-1 lies in [0, 2n-3] and column n-1 of T + q*N is zero mod 2^L
(equation (3)), so for 2n-3 < 2^L it is fixed: gamma = -(T[n-1] + S) mod 2^L.
Hence (the reading used throughout the library):

    C = floor(T / R) + H' + ceil((T[n-1] + S) / 2^L)

The printed equations (3)-(5) instead feed c_add in as the carry into column
n-1; ``redc_truncated_literal`` implements that reading and the tests show it
differs from exact REDC, which is why the ceil reading is used.

For a split that rounds to nearest (lo in [-2^(L-1), 2^(L-1)), as produced by
a double-precision FMA split) the same argument gives a carry in
[-(n-1), n-1] and the ceil becomes round-to-nearest, provided n-1 < 2^(L-1).
"""


def limbs(x, L, n):
    m = (1 << L) - 1
    return [(x >> (L * i)) & m for i in range(n)]


def split_floor(p, L):
    """Partial product as (lo, hi) with lo in [0, 2^L): madd52lo/madd52hi style."""
    return p & ((1 << L) - 1), p >> L


def split_nearest(p, L):
    """Partial product as (lo, hi) with hi = round(p / 2^L), ties to even."""
    half = 1 << (L - 1)
    hi = p >> L
    lo = p - (hi << L)
    if lo > half or (lo == half and (hi & 1)):
        hi += 1
        lo -= 1 << L
    return lo, hi


def redc_exact(T, N, L, n):
    """Algorithm 5: q = T*N' mod R, C = (T + q*N) / R."""
    R = 1 << (L * n)
    Np = (-pow(N, -1, R)) % R
    q = (T * Np) % R
    s = T + q * N
    assert s % R == 0
    return s // R


def theorem1_form(T, N, L, n):
    """Algorithm 6 with the exact quotient: floor(T/R) + floor(qN/R) + c_add."""
    R = 1 << (L * n)
    Np = (-pow(N, -1, R)) % R
    q = (T * Np) % R
    c_add = 1 if T % R != 0 else 0
    return T // R + (q * N) // R + c_add


def _columns(q, N, L, n, split):
    """S (column n-1) and H' (columns >= n) of q*N from the needed partial products only."""
    ql, Nl = limbs(q, L, n), limbs(N, L, n)
    S = 0
    H = 0
    for i in range(n):
        for j in range(n):
            w = i + j
            if w < n - 2:
                continue  # never computed: the point of the truncation
            lo, hi = split(ql[i] * Nl[j], L)
            if w == n - 2:
                S += hi
            elif w == n - 1:
                S += lo
                H += hi
            else:
                H += lo << (L * (w - n))
                H += hi << (L * (w + 1 - n))
    return S, H


def redc_truncated(T, N, L, n, split="floor"):
    """Algorithm 6 with Theorem 2's partial-product set and the exact carry reading."""
    R = 1 << (L * n)
    Np = (-pow(N, -1, R)) % R
    q = (T * Np) % R  # step 1: low half of T*N'
    sp = split_floor if split == "floor" else split_nearest
    S, H = _columns(q, N, L, n, sp)  # step 2: truncated high half
    Tn1 = (T >> (L * (n - 1))) & ((1 << L) - 1)
    v = Tn1 + S
    B = 1 << L
    if split == "floor":
        k = -((-v) // B)  # ceil(v / 2^L)
    else:
        k = (v + (B >> 1)) // B  # nearest (carry in is centred)
    return (T >> (L * n)) + H + k  # step 4


def redc_truncated_literal(T, N, L, n):
    """Equations (3)-(5) read literally: c_add is the carry into column n-1."""
    R = 1 << (L * n)
    Np = (-pow(N, -1, R)) % R
    q = (T * Np) % R
    S, H = _columns(q, N, L, n, split_floor)
    c_add = 1 if T % R != 0 else 0
    return (T >> (L * n)) + H + ((S + c_add) >> L) + c_add


def redc_truncated_fullcol(T, N, L, n):
    """Algorithm 6 when every partial product q_i*N_j is kept whole (2L bits).

    A single L x L -> 2L multiply-accumulate yields both halves of a partial
    product, so the products of Theorem 2 (lo halves at weight >= n-1, hi
    halves at weight n-2) are taken as the full products at weight >= n-2:
    the same n(n+1)/2 + n-1 multiplications.  With column sums
    P_w = sum_{i+j=w} q_i N_j,

        a2 = T[n-2] + P_{n-2}
        a1 = T[n-1] + P_{n-1} + floor(a2 / 2^L)
        k  = floor(a1 / 2^L) + [ (a1 mod 2^L) or (a2 mod 2^L) != 0 ]
        C  = floor(T / R) + sum_{w>=n} P_w 2^{L(w-n)} + k

    The skipped columns (< n-2) push a carry rho into column n-2 with
    0 <= rho < (n-2)(2^L + 2) + 1; column n-1 and below of T + q*N vanish
    (equation (3)), so k = ceil(U / 2^{2L}) with U = a1*2^L + (a2 mod 2^L),
    exact whenever (n-2)(2^L + 2) + 1 <= 2^{2L}.  The indicator plays the
    role of c_add (equation (1)): an OR of low words being non-zero.
    """
    R = 1 << (L * n)
    M = (1 << L) - 1
    Np = (-pow(N, -1, R)) % R
    q = (T * Np) % R
    ql, Nl = limbs(q, L, n), limbs(N, L, n)
    Tl = limbs(T, L, 2 * n)
    P = [0] * (2 * n)
    for i in range(n):
        for j in range(n):
            if i + j >= n - 2:
                P[i + j] += ql[i] * Nl[j]
    a2 = (Tl[n - 2] + P[n - 2]) if n >= 2 else 0
    a1 = Tl[n - 1] + P[n - 1] + (a2 >> L)
    k = (a1 >> L) + (1 if ((a1 & M) | (a2 & M)) else 0)
    H = sum(P[w] << (L * (w - n)) for w in range(n, 2 * n))
    return (T >> (L * n)) + H + k


def redc_cios(A, B, N, L, n):
    """Algorithm 4 (word-interleaved, CIOS): returns (A*B*R^{-1} as REDC gives it, largest column sum).

    For each limb a_i of A: Y += a_i * B; q_i = (Y mod 2^L) * N'_0 mod 2^L
    with N'_0 = -N^{-1} mod 2^L; Y = (Y + q_i * N) / 2^L.  Y is held as
    column sums that are never normalised inside the loop: after adding
    q_i * N the lowest column is divisible by 2^L, and only its carry moves
    up with the shift.  The q_i are the limbs of q = -A*B*N^{-1} mod R, so the
    result is (A*B + q*N) / R, the exact Montgomery integer of Algorithm 5.
    The peak column sum bounds the accumulator width a word-sliced
    implementation needs.
    """
    B_ = 1 << L
    M = B_ - 1
    al, bl, Nl = limbs(A, L, n), limbs(B, L, n), limbs(N, L, n)
    n0 = (-pow(N, -1, B_)) % B_
    Y = [0] * (n + 1)
    peak = 0
    for i in range(n):
        for j in range(n):
            Y[j] += al[i] * bl[j]
        qi = ((Y[0] & M) * n0) & M
        for j in range(n):
            Y[j] += qi * Nl[j]
        peak = max(peak, max(Y))
        assert Y[0] & M == 0
        carry = Y[0] >> L
        Y = Y[1:] + [0]
        Y[0] += carry
    peak = max(peak, max(Y))
    return sum(y << (L * j) for j, y in enumerate(Y)), peak


def kara_columns(a, b, levels, xmin=0):
    """Column sums of the product of two limb vectors (lists of equal length k), by Karatsuba.

    Returns (cols, products): cols[x] = sum_{i+j=x} a_i b_j for x >= xmin
    (None below), products = the multiplications used.  Section 3: the
    operands split at m = ceil(k/2) limbs, a = a0 + B a1, b = b0 + B b1, and
    D0 = a0 b0, D1 = (a0 + a1)(b0 + b1), D2 = a1 b1.  The half sums are taken
    limb by limb, without carries, so the recombination D1 - D0 - D2 =
    a0 b1 + a1 b0 holds for every column on its own, not only for the whole
    number.  Column x of the product is then D0[x] + (D1 - D0 - D2)[x - m]
    + D2[x - 2m], and only the sub-columns that reach columns >= xmin are
    formed (the truncation of Section 5 applied to the sub-products).
    levels = 0 is the schoolbook product restricted to those columns.
    """
    k = len(a)
    ncol = 2 * k - 1
    if levels == 0 or k < 2:
        cols = [None] * ncol
        cnt = 0
        for x in range(max(xmin, 0), ncol):
            v = 0
            for i in range(max(0, x - k + 1), min(x, k - 1) + 1):
                v += a[i] * b[x - i]
                cnt += 1
            cols[x] = v
        return cols, cnt
    m = (k + 1) // 2
    a0, a1 = a[:m], a[m:] + [0] * (2 * m - k)
    b0, b1 = b[:m], b[m:] + [0] * (2 * m - k)
    sa = [x + y for x, y in zip(a0, a1)]
    sb = [x + y for x, y in zip(b0, b1)]
    d0, c0 = kara_columns(a0, b0, levels - 1, min(xmin, xmin - m))
    d1, c1 = kara_columns(sa, sb, levels - 1, xmin - m)
    d2, c2 = kara_columns(a1, b1, levels - 1, xmin - 2 * m)
    cols = [None] * ncol
    for x in range(max(xmin, 0), ncol):
        v = 0
        if x <= 2 * m - 2:
            v += d0[x]
        y = x - m
        if 0 <= y <= 2 * m - 2:
            v += d1[y] - d0[y] - d2[y]
        z = x - 2 * m
        if 0 <= z <= 2 * m - 2:
            v += d2[z]
        cols[x] = v
    return cols, c0 + c1 + c2


def redc_truncated_karatsuba(T, N, L, n, levels=1):
    """Algorithm 6 with the truncated high half of q*N formed by Karatsuba (Section 5, Karatsuba).

    Only the columns n-2 .. 2n-2 of q*N are formed, through kara_columns;
    they equal the schoolbook columns, so the exact two-column carry reading
    of redc_truncated_fullcol applies unchanged.  Returns (C, products of the
    q*N part).
    """
    R = 1 << (L * n)
    M = (1 << L) - 1
    Np = (-pow(N, -1, R)) % R
    q = (T * Np) % R
    cols, cnt = kara_columns(limbs(q, L, n), limbs(N, L, n), levels, n - 2)
    P = cols + [0]
    Tl = limbs(T, L, 2 * n)
    a2 = Tl[n - 2] + P[n - 2]
    a1 = Tl[n - 1] + P[n - 1] + (a2 >> L)
    k = (a1 >> L) + (1 if ((a1 & M) | (a2 & M)) else 0)
    H = sum(P[w] << (L * (w - n)) for w in range(n, 2 * n - 1))
    return (T >> (L * n)) + H + k, cnt


def fullcol_condition(L, n):
    """True when the carry window of redc_truncated_fullcol is provably wide enough."""
    return (n - 2) * ((1 << L) + 2) + 1 <= (1 << (2 * L))


def counts(n):
    """Partial products (L x L -> 2L) per operation, from the schedules above.

    plain: full product + low-half q + full q*N; truncated: the q*N part keeps
    only weights >= n-2 (hi) / >= n-1 (lo), i.e. n(n+1)/2 + n - 1 products;
    CIOS (Algorithm 4): n products a_i*b_j and n products q_i*N_j per limb of A,
    plus one product for q_i, for squares too.
    """
    tri = n * (n + 1) // 2
    return {
        "mul_cios": 2 * n * n + n,
        "sqr_cios": 2 * n * n + n,
        "mul_plain": n * n + tri + n * n,
        "sqr_plain": tri + tri + n * n,
        "mul_trunc": n * n + tri + tri + n - 1,
        "sqr_trunc": tri + tri + tri + n - 1,
    }
