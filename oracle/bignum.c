/*
 * oracle/bignum.c -- plain, slow CPU arithmetic used ONLY as test
 * infrastructure (the parity checker for the GPU library).  Nothing in the
 * product path may link or call this file; tests, the smoke check and the
 * CPU-baseline leg of the benchmark are its only users.
 *
 * Numbers are little-endian arrays of 32-bit limbs with 64-bit
 * intermediates.  Every routine is the textbook definition of what it
 * computes, with no blocking, fusion or reordering:
 *
 *   ora_mul      schoolbook product (the operation of Section 2, Algorithm 1:
 *                all n*n partial products summed at their weights).
 *   ora_mod      bit-serial remainder: scan x from its top bit, r = 2r + bit,
 *                subtract N whenever r >= N.
 *   ora_redc     the exact Montgomery reduction of Algorithm 5,
 *                (T + q*N) / 2^r with the unique q in [0, 2^r) that makes the
 *                division exact, computed one bit of q at a time
 *                (add N when the running value is odd, then halve).
 *   ora_nprime   N' = -N^{-1} mod 2^r, i.e. the q that the bit-serial REDC
 *                picks for T = 1 (Section 4, the precomputed value N').
 *   ora_r2       R^2 mod N = ora_mod(2^{2r}, N) (Section 4, conversion into
 *                Montgomery form).
 *   ora_modexp   a^e mod N by left-to-right binary square-and-multiply with
 *                ora_mul + ora_mod (no Montgomery arithmetic at all), the
 *                value that the fixed-window exponentiation of Algorithm 7
 *                must produce; e = 0 gives 1 mod N.
 *
 * Status codes: 0 on success, -1 on a bad argument.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- small helpers on limb arrays ------------------------------------ */

static int cmp_n(const uint32_t *a, const uint32_t *b, int n) {
  for (int i = n - 1; i >= 0; --i) {
    if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  }
  return 0;
}

/* a -= b over n limbs, returns the borrow out. */
static uint32_t sub_n(uint32_t *a, const uint32_t *b, int n) {
  uint64_t borrow = 0;
  for (int i = 0; i < n; ++i) {
    uint64_t d = (uint64_t)a[i] - b[i] - borrow;
    a[i] = (uint32_t)d;
    borrow = (d >> 63) & 1u;
  }
  return (uint32_t)borrow;
}

/* a += b over n limbs, returns the carry out. */
static uint32_t add_n(uint32_t *a, const uint32_t *b, int n) {
  uint64_t carry = 0;
  for (int i = 0; i < n; ++i) {
    uint64_t s = (uint64_t)a[i] + b[i] + carry;
    a[i] = (uint32_t)s;
    carry = s >> 32;
  }
  return (uint32_t)carry;
}

static int bit_at(const uint32_t *x, int i) { return (x[i >> 5] >> (i & 31)) & 1u; }

/* ---- schoolbook product ---------------------------------------------- */

int ora_mul(const uint32_t *a, int na, const uint32_t *b, int nb, uint32_t *out) {
  if (na <= 0 || nb <= 0 || !a || !b || !out) return -1;
  memset(out, 0, sizeof(uint32_t) * (size_t)(na + nb));
  for (int i = 0; i < na; ++i) {
    uint64_t carry = 0;
    for (int j = 0; j < nb; ++j) {
      uint64_t t = (uint64_t)a[i] * b[j] + out[i + j] + carry;
      out[i + j] = (uint32_t)t;
      carry = t >> 32;
    }
    out[i + nb] = (uint32_t)carry;
  }
  return 0;
}

/* ---- bit-serial remainder -------------------------------------------- */

/* r = x mod m, where m has nm limbs (m != 0); r has nm limbs. */
int ora_mod(const uint32_t *x, int nx, const uint32_t *m, int nm, uint32_t *r) {
  if (nx <= 0 || nm <= 0 || !x || !m || !r) return -1;
  int nz = 0;
  for (int i = 0; i < nm; ++i) nz |= (m[i] != 0);
  if (!nz) return -1;
  /* running remainder needs one extra limb for the doubling */
  uint32_t *acc = (uint32_t *)calloc((size_t)nm + 1, sizeof(uint32_t));
  uint32_t *mm = (uint32_t *)calloc((size_t)nm + 1, sizeof(uint32_t));
  if (!acc || !mm) { free(acc); free(mm); return -1; }
  memcpy(mm, m, sizeof(uint32_t) * (size_t)nm);
  for (int bit = nx * 32 - 1; bit >= 0; --bit) {
    /* acc = 2*acc + bit */
    uint32_t carry = (uint32_t)bit_at(x, bit);
    for (int i = 0; i <= nm; ++i) {
      uint32_t hi = acc[i] >> 31;
      acc[i] = (acc[i] << 1) | carry;
      carry = hi;
    }
    if (cmp_n(acc, mm, nm + 1) >= 0) sub_n(acc, mm, nm + 1);
  }
  memcpy(r, acc, sizeof(uint32_t) * (size_t)nm);
  free(acc); free(mm);
  return 0;
}

/* ---- exact Montgomery reduction, one bit of q at a time -------------- */

/* out = (t + q*m) / 2^rbits with q in [0, 2^rbits) such that the division is
 * exact; m odd.  out has nout limbs (nout*32 must hold the result: for
 * t < 2^rbits * m it is < 2m).  Returns -1 if the result does not fit. */
int ora_redc(const uint32_t *t, int nt, const uint32_t *m, int nm, int rbits,
             uint32_t *out, int nout) {
  if (nt <= 0 || nm <= 0 || rbits <= 0 || !t || !m || !out || nout <= 0) return -1;
  if ((m[0] & 1u) == 0) return -1;
  int w = (nt > nm ? nt : nm) + 2;
  uint32_t *x = (uint32_t *)calloc((size_t)w, sizeof(uint32_t));
  uint32_t *mm = (uint32_t *)calloc((size_t)w, sizeof(uint32_t));
  if (!x || !mm) { free(x); free(mm); return -1; }
  memcpy(x, t, sizeof(uint32_t) * (size_t)nt);
  memcpy(mm, m, sizeof(uint32_t) * (size_t)nm);
  for (int s = 0; s < rbits; ++s) {
    if (x[0] & 1u) add_n(x, mm, w);
    for (int i = 0; i < w; ++i) x[i] = (x[i] >> 1) | (i + 1 < w ? (x[i + 1] << 31) : 0u);
  }
  int rc = 0;
  for (int i = nout; i < w; ++i) if (x[i]) rc = -1;
  for (int i = 0; i < nout; ++i) out[i] = i < w ? x[i] : 0u;
  free(x); free(mm);
  return rc;
}

/* ---- N' = -N^{-1} mod 2^rbits: the q of the bit-serial REDC of 1 ------ */

int ora_nprime(const uint32_t *m, int nm, int rbits, uint32_t *out /* ceil(rbits/32) */) {
  if (nm <= 0 || rbits <= 0 || !m || !out) return -1;
  if ((m[0] & 1u) == 0) return -1;
  int nq = (rbits + 31) / 32;
  int w = nm + 2;
  uint32_t *x = (uint32_t *)calloc((size_t)w, sizeof(uint32_t));
  uint32_t *mm = (uint32_t *)calloc((size_t)w, sizeof(uint32_t));
  if (!x || !mm) { free(x); free(mm); return -1; }
  memcpy(mm, m, sizeof(uint32_t) * (size_t)nm);
  memset(out, 0, sizeof(uint32_t) * (size_t)nq);
  x[0] = 1u;
  for (int s = 0; s < rbits; ++s) {
    if (x[0] & 1u) { add_n(x, mm, w); out[s >> 5] |= 1u << (s & 31); }
    for (int i = 0; i < w; ++i) x[i] = (x[i] >> 1) | (i + 1 < w ? (x[i + 1] << 31) : 0u);
  }
  free(x); free(mm);
  return 0;
}

/* ---- R^2 mod N --------------------------------------------------------- */

int ora_r2(const uint32_t *m, int nm, int rbits, uint32_t *out /* nm */) {
  if (nm <= 0 || rbits <= 0 || !m || !out) return -1;
  int nx = (2 * rbits) / 32 + 1;
  uint32_t *x = (uint32_t *)calloc((size_t)nx, sizeof(uint32_t));
  if (!x) return -1;
  x[(2 * rbits) >> 5] |= 1u << ((2 * rbits) & 31);
  int rc = ora_mod(x, nx, m, nm, out);
  free(x);
  return rc;
}

/* ---- modular exponentiation by square-and-multiply --------------------- */

/* out = a^e mod m, e given by its ebits low bits (leading zeros allowed). */
int ora_modexp(const uint32_t *a, int na, const uint32_t *e, int ebits,
               const uint32_t *m, int nm, uint32_t *out /* nm */) {
  if (na <= 0 || nm <= 0 || ebits < 0 || !a || !m || !out || (ebits > 0 && !e)) return -1;
  uint32_t *base = (uint32_t *)calloc((size_t)nm, sizeof(uint32_t));
  uint32_t *y = (uint32_t *)calloc((size_t)nm, sizeof(uint32_t));
  uint32_t *prod = (uint32_t *)calloc((size_t)2 * nm, sizeof(uint32_t));
  uint32_t *one = (uint32_t *)calloc((size_t)nm, sizeof(uint32_t));
  if (!base || !y || !prod || !one) { free(base); free(y); free(prod); free(one); return -1; }
  int rc = ora_mod(a, na, m, nm, base);
  one[0] = 1u;
  if (!rc) rc = ora_mod(one, nm, m, nm, y); /* y = 1 mod m */
  for (int bit = ebits - 1; bit >= 0 && !rc; --bit) {
    rc |= ora_mul(y, nm, y, nm, prod);
    rc |= ora_mod(prod, 2 * nm, m, nm, y);
    if (bit_at(e, bit)) {
      rc |= ora_mul(y, nm, base, nm, prod);
      rc |= ora_mod(prod, 2 * nm, m, nm, y);
    }
  }
  memcpy(out, y, sizeof(uint32_t) * (size_t)nm);
  free(base); free(y); free(prod); free(one);
  return rc;
}

/* Batch helper for timing only: `count` instances of ora_modexp laid out
 * back to back (a: count*na limbs, e: count*ceil(ebits/32), m and out:
 * count*nm).  Returns the number of failed instances. */
int ora_modexp_many(const uint32_t *a, int na, const uint32_t *e, int ebits,
                    const uint32_t *m, int nm, uint32_t *out, int count) {
  int ne = (ebits + 31) / 32;
  int bad = 0;
  for (int k = 0; k < count; ++k)
    bad += ora_modexp(a + (size_t)k * na, na, e + (size_t)k * ne, ebits,
                      m + (size_t)k * nm, nm, out + (size_t)k * nm) != 0;
  return bad;
}
