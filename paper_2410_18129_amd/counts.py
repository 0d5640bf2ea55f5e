"""Algorithmic work of the method: 28x28-bit partial products per operation.

Host-side bookkeeping for throughput / roofline reporting.  n is the limb
count of the size class, n = ceil((bits + 2) / 28): the work the method needs,
not the padded count of the block kernels above 2048 bits (which compute
whole 37-limb blocks and are charged only this).

  product  (Section 2): mul n^2, sqr n(n+1)/2 (off-diagonal once + diagonal)
  q        (Algorithm 6 step 1 / Algorithm 3 step 1): low half, n(n+1)/2
  q*N      truncated (Theorem 2): n(n+1)/2 + n - 1;  plain (B_fma): n^2
  CIOS     (Algorithm 4): per limb a_i, n products a_i b_j, one for q_i and n
           for q_i N_j: 2n^2 + n, for a square too
Exponentiation (Algorithm 7) with W = ceil(ebits / w) windows runs 2^w - 1
multiplications for the conversion and the table, (W - 1) w squarings,
W - 1 multiplications and one final multiplication by 1 (leaving
Montgomery form).
"""
LIMB_BITS = 28
VALU_LANES = 256 * 64          # CUs x lanes issuing one v_mad_u64_u32 per cycle
CLOCK_HZ = 2.4e9
PEAK_MAD_PER_S = VALU_LANES * CLOCK_HZ  # 3.93e13 28x28->64 multiply-accumulates per second


BLOCK_LIMBS = 37


def limbs(bits, padded=False):
    """Limbs of a size class: the method's ceil((bits + 2) / 28), which sets the algorithmic work
    (110 at 3072 bits, 147 at 4096); padded=True gives the kernels' count, rounded up to whole 37-limb
    blocks above 2048 bits (111 and 148), which also sets R."""
    n = (bits + 2 + LIMB_BITS - 1) // LIMB_BITS
    if padded and bits > 2048:
        n = BLOCK_LIMBS * ((n + BLOCK_LIMBS - 1) // BLOCK_LIMBS)
    return n


def op_products(n, trunc=True, cios=False):
    if cios:
        return {"mul": 2 * n * n + n, "sqr": 2 * n * n + n}
    tri = n * (n + 1) // 2
    qn = tri + n - 1 if trunc else n * n
    return {"mul": n * n + tri + qn, "sqr": tri + tri + qn}


def modexp_schedule(ebits, w):
    nwin = (ebits + w - 1) // w if ebits else 1
    return {"mul": (1 << w) - 1 + (nwin - 1) + 1, "sqr": (nwin - 1) * w, "windows": nwin}


def modexp_products(bits, ebits, w, trunc=True, cios=False):
    n = limbs(bits)
    p = op_products(n, trunc, cios)
    s = modexp_schedule(ebits, w)
    return s["mul"] * p["mul"] + s["sqr"] * p["sqr"]


def table_scan_bytes(bits, ebits, w):
    """Bytes of table entries read by the constant-time scans of one exponentiation."""
    n = limbs(bits)
    s = modexp_schedule(ebits, w)
    return s["windows"] * (1 << w) * n * 4


def mul_products(bits, levels=0):
    """Partial products of one raw product of bits-bit operands (n = ceil(bits / 28) limbs): n^2 by
    schoolbook; with L levels of Karatsuba, 3^L products of ceil(n / 2^L)-limb parts."""
    n = (bits + LIMB_BITS - 1) // LIMB_BITS
    part = -(-n // (1 << levels))
    return 3 ** levels * part * part
