"""CPU oracle for the batched Montgomery / modexp library -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never links, calls or
imports it, and it shares no code, tables or helpers with the GPU path.

The arithmetic lives in ``bignum.c`` (plain C, 32-bit limbs, 64-bit
intermediates, bit-serial reductions); this module only converts Python ints
to limb arrays and back.  ``montred_model`` holds a limb-level model of the
truncated reduction (Section 5, Algorithm 6 with Theorems 1-2) that pins the
reading of the paper's carry equations.

Functions (all on non-negative Python ints):
  mul(a, b)               schoolbook a*b                          (Section 2)
  mod(x, N)               bit-serial x mod N
  redc(T, N, rbits)       exact Montgomery reduction (T+qN)/2^rbits  (Algorithm 5)
  nprime(N, rbits)        -N^{-1} mod 2^rbits                      (Section 4)
  r2(N, rbits)            2^(2 rbits) mod N                        (Section 4)
  montmul(a, b, N, rbits) redc(mul(a, b))                          (Algorithms 3/5)
  modexp(a, e, N, ebits)  a^e mod N by left-to-right square-and-multiply (Algorithm 7's result)
"""
import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "bignum.c")
_lib = None


def build():
    """Compile bignum.c with gcc -O2 into liboracle.so (always rebuilds)."""
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-Wall", "-o", _SO, _SRC])


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_SO)
    P = ctypes.POINTER(ctypes.c_uint32)
    I = ctypes.c_int
    lib.ora_mul.argtypes = [P, I, P, I, P]
    lib.ora_mod.argtypes = [P, I, P, I, P]
    lib.ora_redc.argtypes = [P, I, P, I, I, P, I]
    lib.ora_nprime.argtypes = [P, I, I, P]
    lib.ora_r2.argtypes = [P, I, I, P]
    lib.ora_modexp.argtypes = [P, I, P, I, P, I, P]
    lib.ora_modexp_many.argtypes = [P, I, P, I, P, I, P, I]
    for f in (lib.ora_mul, lib.ora_mod, lib.ora_redc, lib.ora_nprime, lib.ora_r2,
              lib.ora_modexp, lib.ora_modexp_many):
        f.restype = I
    _lib = lib
    return lib


def nlimbs(x):
    """Number of 32-bit limbs needed to hold x (at least 1)."""
    return max(1, (x.bit_length() + 31) // 32)


def to_limbs(x, n):
    if x < 0 or x.bit_length() > 32 * n:
        raise ValueError("value does not fit in %d limbs" % n)
    arr = (ctypes.c_uint32 * n)()
    for i in range(n):
        arr[i] = (x >> (32 * i)) & 0xFFFFFFFF
    return arr


def from_limbs(arr, n=None):
    n = len(arr) if n is None else n
    v = 0
    for i in range(n - 1, -1, -1):
        v = (v << 32) | int(arr[i])
    return v


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s failed (rc=%d)" % (what, rc))


def mul(a, b):
    lib = _load()
    na, nb = nlimbs(a), nlimbs(b)
    out = (ctypes.c_uint32 * (na + nb))()
    _check(lib.ora_mul(to_limbs(a, na), na, to_limbs(b, nb), nb, out), "mul")
    return from_limbs(out)


def mod(x, N):
    lib = _load()
    nx, nm = nlimbs(x), nlimbs(N)
    out = (ctypes.c_uint32 * nm)()
    _check(lib.ora_mod(to_limbs(x, nx), nx, to_limbs(N, nm), nm, out), "mod")
    return from_limbs(out)


def redc(T, N, rbits):
    lib = _load()
    nt, nm = nlimbs(T), nlimbs(N)
    nout = max(nt, nm) + 1
    out = (ctypes.c_uint32 * nout)()
    _check(lib.ora_redc(to_limbs(T, nt), nt, to_limbs(N, nm), nm, rbits, out, nout), "redc")
    return from_limbs(out)


def nprime(N, rbits):
    lib = _load()
    nm = nlimbs(N)
    nq = (rbits + 31) // 32
    out = (ctypes.c_uint32 * nq)()
    _check(lib.ora_nprime(to_limbs(N, nm), nm, rbits, out), "nprime")
    return from_limbs(out)


def r2(N, rbits):
    lib = _load()
    nm = nlimbs(N)
    out = (ctypes.c_uint32 * nm)()
    _check(lib.ora_r2(to_limbs(N, nm), nm, rbits, out), "r2")
    return from_limbs(out)


def montmul(a, b, N, rbits):
    return redc(mul(a, b), N, rbits)


def modexp(a, e, N, ebits=None):
    lib = _load()
    if ebits is None:
        ebits = e.bit_length()
    nm, na = nlimbs(N), nlimbs(a)
    ne = max(1, (ebits + 31) // 32)
    out = (ctypes.c_uint32 * nm)()
    _check(lib.ora_modexp(to_limbs(a, na), na, to_limbs(e, ne), ebits,
                          to_limbs(N, nm), nm, out), "modexp")
    return from_limbs(out)


def modexp_many(bases, exps, mods, ebits):
    """Batch of square-and-multiply modexps through one C call (timing helper)."""
    lib = _load()
    cnt = len(mods)
    nm = max(nlimbs(N) for N in mods)
    ne = max(1, (ebits + 31) // 32)
    A = (ctypes.c_uint32 * (cnt * nm))()
    E = (ctypes.c_uint32 * (cnt * ne))()
    M = (ctypes.c_uint32 * (cnt * nm))()
    O = (ctypes.c_uint32 * (cnt * nm))()
    for k in range(cnt):
        for i in range(nm):
            A[k * nm + i] = (bases[k] >> (32 * i)) & 0xFFFFFFFF
            M[k * nm + i] = (mods[k] >> (32 * i)) & 0xFFFFFFFF
        for i in range(ne):
            E[k * ne + i] = (exps[k] >> (32 * i)) & 0xFFFFFFFF
    bad = lib.ora_modexp_many(A, nm, E, ebits, M, nm, O, cnt)
    if bad:
        raise ValueError("oracle modexp_many: %d failures" % bad)
    return [from_limbs(O[k * nm:(k + 1) * nm]) for k in range(cnt)]
