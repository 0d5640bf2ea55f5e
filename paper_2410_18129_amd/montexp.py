"""ctypes binding of libmontexp.so (C ABI in include/montexp.h).

Argument marshalling only: every arithmetic step runs in the library's HIP
kernels.  Device buffers are torch tensors (int64 words holding the raw
64-bit limbs of each value, one row per instance) and streams are torch
streams; torch is used for device memory and streams, nothing else.  If the
library is missing this module raises -- there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmontexp.so")

MX_OK, MX_EINVAL, MX_ENOMEM, MX_EDEVICE, MX_EUNSUPPORTED = 0, 1, 2, 3, 4
MX_REDC_TRUNC, MX_REDC_PLAIN, MX_IMPL_BLOCK, MX_MUL_KARATSUBA, MX_ONE_LANE, MX_REDC_CIOS, MX_TWO_LANES = \
    0, 1, 2, 4, 8, 16, 32
MX_REDC_KARATSUBA = 64
MX_MUL_KARATSUBA2 = 128
MX_CHECK_INPUTS = 256
MX_FOUR_LANES = 512
SIZE_CLASSES = (64, 128, 256, 512, 1024, 2048, 3072, 4096)
LIMB_BITS = 28

# exported symbols and their ctypes signatures (mirrors include/montexp.h)
_P = ctypes.c_void_p
_U32 = ctypes.c_uint32
_SIGS = {
    "mont_ctx_init": (ctypes.c_int, [ctypes.POINTER(_P), _P, _U32, _U32, _P]),
    "mont_ctx_query": (ctypes.c_int, [_P, ctypes.POINTER(_U32), ctypes.POINTER(_U32), ctypes.POINTER(_U32),
                                      ctypes.POINTER(_U32), ctypes.POINTER(ctypes.c_size_t)]),
    "mont_ctx_export": (ctypes.c_int, [_P, _U32, _P, _P, _P]),
    "mont_ctx_destroy": (None, [_P]),
    "mont_ctx_reserve": (ctypes.c_int, [_P, ctypes.c_size_t]),
    "mont_ws_bytes": (ctypes.c_int, [_P, _U32, _U32, ctypes.POINTER(ctypes.c_size_t)]),
    "mont_mul_batch": (ctypes.c_int, [_P, _P, _P, _P, _P, _U32, _U32, _P]),
    "mont_sqr_batch": (ctypes.c_int, [_P, _P, _P, _P, _U32, _U32, _P]),
    "modexp_batch": (ctypes.c_int, [_P, _P, _P, _P, _U32, _U32, _P, _U32, _U32, _P]),
    "modexp_batch_noalloc": (ctypes.c_int, [_P, _P, _P, _P, _U32, _U32, _P, _U32, _U32, _P]),
    "modexp_batch_ws": (ctypes.c_int, [_P, _P, _P, _P, _U32, _U32, _P, _U32, _U32, _P, ctypes.c_size_t, _P]),
    "modexp_ws_bytes": (ctypes.c_int, [_P, _U32, _U32, _U32, ctypes.POINTER(ctypes.c_size_t)]),
    "rsa_crt_batch": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _U32, _P, _U32, _U32, _P]),
    "rsa_crt_batch_ws": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _U32, _P, _U32, _U32, _P, ctypes.c_size_t,
                                        _P]),
    "rsa_crt_ws_bytes": (ctypes.c_int, [_P, _U32, _U32, _U32, ctypes.POINTER(ctypes.c_size_t)]),
    "mp_mul_batch": (ctypes.c_int, [_P, _P, _P, _U32, _U32, _U32, _P, ctypes.c_size_t, _P]),
    "mp_mul_ws_bytes": (ctypes.c_int, [_U32, _U32, _U32, ctypes.POINTER(ctypes.c_size_t)]),
    "mx_mixed_plan_create": (ctypes.c_int, [ctypes.POINTER(_P), _P, _U32]),
    "mx_mixed_plan_launch": (ctypes.c_int, [_P, _P]),
    "mx_mixed_plan_launch_graph": (ctypes.c_int, [_P, _P]),
    "mx_mixed_plan_query": (ctypes.c_int, [_P, ctypes.POINTER(_U32), ctypes.POINTER(_U32), _P]),
    "mx_mixed_plan_destroy": (None, [_P]),
    "mx_tune_modexp": (ctypes.c_int, [_P, _U32, _U32, _P, _U32, _U32, _U32, ctypes.POINTER(_U32),
                                      ctypes.POINTER(_U32), ctypes.POINTER(ctypes.c_float), _P]),
    "mont_last_error": (ctypes.c_char_p, []),
}


class BatchDesc(ctypes.Structure):
    """mx_batch_desc of include/montexp.h."""
    _fields_ = [("ctx", _P), ("ctx_idx", _P), ("base", _P), ("exp", _P), ("out", _P), ("n", _U32),
                ("exp_bits", _U32), ("window", _U32), ("flags", _U32), ("tile_cost", ctypes.c_float)]
EXPORTS = tuple(_SIGS)

_lib = None


class MontError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d)" % (msg, status))
        self.status = status


def lib():
    """Loads libmontexp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmontexp.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2410_18129_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st):
    if st != MX_OK:
        msg = lib().mont_last_error().decode(errors="replace")
        raise MontError(st, msg)


def words_for(bits):
    return (bits + 63) // 64


BLOCK_LIMBS = 37  # classes above 2048 bits use whole 37-limb blocks


def limbs_for(bits):
    n = (bits + 2 + LIMB_BITS - 1) // LIMB_BITS
    if bits > 2048:
        n = BLOCK_LIMBS * ((n + BLOCK_LIMBS - 1) // BLOCK_LIMBS)
    return n


def r_bits_for(bits):
    return LIMB_BITS * limbs_for(bits)


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev_words(x, words, device):
    """numpy uint64 [n, words] / torch tensor -> contiguous int64 device tensor."""
    import torch
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint64).view(np.int64))
    if x.dtype != torch.int64 or x.dim() != 2 or x.shape[1] != words:
        raise ValueError("expected an int64 tensor of shape [n, %d]" % words)
    return x.to(device).contiguous()


class Context:
    """Device-resident Montgomery contexts for a batch of moduli of one size class."""

    def __init__(self, moduli_words, bits, stream=None):
        moduli_words = np.ascontiguousarray(moduli_words, dtype=np.uint64)
        if moduli_words.ndim != 2 or moduli_words.shape[1] != words_for(bits):
            raise ValueError("moduli must be uint64 [count, ceil(bits/64)]")
        self._h = ctypes.c_void_p()
        L = lib()
        _check(L.mont_ctx_init(ctypes.byref(self._h), moduli_words.ctypes.data_as(_P), bits,
                               moduli_words.shape[0], _stream_ptr(stream)))
        b, rb, lb, cnt = _U32(), _U32(), _U32(), _U32()
        nb = ctypes.c_size_t()
        _check(L.mont_ctx_query(self._h, ctypes.byref(b), ctypes.byref(rb), ctypes.byref(lb), ctypes.byref(cnt),
                                ctypes.byref(nb)))
        self.bits, self.r_bits, self.limb_bits, self.count = b.value, rb.value, lb.value, cnt.value
        self.words = words_for(self.bits)
        self.mont_words = words_for(self.r_bits)

    @property
    def handle(self):
        if not self._h:
            raise ValueError("context destroyed")
        return self._h

    def reserve(self, nbytes):
        """Grows the context's library workspace to at least nbytes (mont_ctx_reserve; allocates)."""
        _check(lib().mont_ctx_reserve(self.handle, nbytes))

    def device_bytes(self):
        nb = ctypes.c_size_t()
        _check(lib().mont_ctx_query(self.handle, None, None, None, None, ctypes.byref(nb)))
        return nb.value

    def export(self, idx):
        """(N' mod R, R^2 mod N, R mod N) of context idx as Python ints."""
        arrs = [np.zeros(self.mont_words, dtype=np.uint64) for _ in range(3)]
        _check(lib().mont_ctx_export(self.handle, idx, *[a.ctypes.data_as(_P) for a in arrs]))
        return tuple(int.from_bytes(a.tobytes(), "little") for a in arrs)

    def close(self):
        if self._h:
            lib().mont_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _impl_flags(block):
    """block: False (default kernels), True (block kernels) or "karatsuba"."""
    if block == "karatsuba":
        return MX_MUL_KARATSUBA
    return MX_IMPL_BLOCK if block else 0


def _redc_flags(plain, cios):
    """plain: full q*N product (Algorithm 3); cios: word-interleaved (Algorithm 4); else truncated."""
    return (MX_REDC_PLAIN if plain else MX_REDC_TRUNC) | (MX_REDC_CIOS if cios else 0)


def _check_rows(name, t, n, words):
    """Shape/dtype/device checks that keep every kernel access inside the buffers."""
    import torch
    if t.dtype != torch.int64 or t.dim() != 2 or t.shape[0] != n or t.shape[1] != words:
        raise ValueError("%s: expected int64 [%d, %d], got %s %s" % (name, n, words, t.dtype, tuple(t.shape)))
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s: expected a contiguous device tensor" % name)


def _check_idx(ctx_idx, n, ctx):
    import torch
    if ctx_idx is None:
        if n > ctx.count:
            raise ValueError("n=%d exceeds the context count %d (pass ctx_idx)" % (n, ctx.count))
        return
    if ctx_idx.dtype != torch.int32 or ctx_idx.dim() != 1 or ctx_idx.shape[0] != n or not ctx_idx.is_cuda:
        raise ValueError("ctx_idx: expected int32 device tensor [%d]" % n)


def _reserve_mont(ctx, n, flags):
    """One launch's workspace for the block kernels' single operations (none for the others)."""
    if not n or flags & MX_MUL_KARATSUBA == 0 and flags & MX_IMPL_BLOCK == 0 and ctx.bits <= 2048:
        return
    nb = ctypes.c_size_t()
    if lib().mont_ws_bytes(ctx.handle, n, flags & (MX_IMPL_BLOCK | MX_MUL_KARATSUBA), ctypes.byref(nb)) == MX_OK:
        ctx.reserve(nb.value)


def mont_mul(ctx, a, b, out=None, ctx_idx=None, plain=False, stream=None, block=False, cios=False,
             kara_redc=False, check_inputs=False):
    """REDC(a*b) per instance; a, b: int64 device tensors [n, mont_words]."""
    n = a.shape[0]
    if out is None:
        import torch
        out = torch.empty_like(a)
    for nm, t in (("a", a), ("b", b), ("out", out)):
        _check_rows(nm, t, n, ctx.mont_words)
    _check_idx(ctx_idx, n, ctx)
    flags = (_redc_flags(plain, cios) | _impl_flags(block) | (MX_REDC_KARATSUBA if kara_redc else 0) |
             (MX_CHECK_INPUTS if check_inputs else 0))
    _reserve_mont(ctx, n, flags)
    _check(lib().mont_mul_batch(ctx.handle, _ptr(ctx_idx), _ptr(a), _ptr(b), _ptr(out), n, flags,
                                _stream_ptr(stream)))
    return out


def mont_sqr(ctx, a, out=None, ctx_idx=None, plain=False, stream=None, block=False, cios=False,
             kara_redc=False, check_inputs=False):
    """REDC(a^2) per instance; a: int64 device tensor [n, mont_words]."""
    n = a.shape[0]
    if out is None:
        import torch
        out = torch.empty_like(a)
    for nm, t in (("a", a), ("out", out)):
        _check_rows(nm, t, n, ctx.mont_words)
    _check_idx(ctx_idx, n, ctx)
    flags = (_redc_flags(plain, cios) | _impl_flags(block) | (MX_REDC_KARATSUBA if kara_redc else 0) |
             (MX_CHECK_INPUTS if check_inputs else 0))
    _reserve_mont(ctx, n, flags)
    _check(lib().mont_sqr_batch(ctx.handle, _ptr(ctx_idx), _ptr(a), _ptr(out), n, flags, _stream_ptr(stream)))
    return out


def modexp(ctx, base, exp, exp_bits, window=0, out=None, ctx_idx=None, plain=False, stream=None, block=False,
           one_lane=False, cios=False, two_lanes=False, kara_redc=False, check_inputs=False, four_lanes=False):
    """base^exp mod N per instance; base: int64 [n, words], exp: int64 [n, ceil(exp_bits/64)].

    one_lane: block kernels keep one lane per instance for small batches too (MX_ONE_LANE);
    two_lanes: at most two lanes per instance (MX_TWO_LANES);
    four_lanes: four lanes per instance at any batch size (MX_FOUR_LANES; block schoolbook kernels).
    cios: word-interleaved Montgomery products (Algorithm 4, MX_REDC_CIOS; classes up to 2048 bits).
    kara_redc: truncated high half of q N by one-level Karatsuba (MX_REDC_KARATSUBA; the register-resident
    classes, and the block kernels at 2048 and 4096 bits with one lane per instance).
    check_inputs: check base < N first (MX_CHECK_INPUTS; the call then waits for the stream)."""
    n = base.shape[0]
    if out is None:
        import torch
        out = torch.empty_like(base)
    for nm, t in (("base", base), ("out", out)):
        _check_rows(nm, t, n, ctx.words)
    if exp_bits:
        _check_rows("exp", exp, n, words_for(exp_bits))
    _check_idx(ctx_idx, n, ctx)
    flags = (_redc_flags(plain, cios) | _impl_flags(block) | (MX_ONE_LANE if one_lane else 0) |
             (MX_TWO_LANES if two_lanes else 0) | (MX_REDC_KARATSUBA if kara_redc else 0) |
             (MX_CHECK_INPUTS if check_inputs else 0) | (MX_FOUR_LANES if four_lanes else 0))
    if n:  # one launch's workspace (0, a no-op, for arguments the call itself rejects)
        ctx.reserve(modexp_ws_bytes(ctx, n, window, flags=flags))
    _check(lib().modexp_batch(ctx.handle, _ptr(ctx_idx), _ptr(base), _ptr(exp) if exp_bits else None, exp_bits,
                              window, _ptr(out), n, flags, _stream_ptr(stream)))
    return out


class MixedPlan:
    """One persistent launch over several size-class batches (mx_mixed_plan_*).

    batches: list of dicts with keys ctx, base, exp, exp_bits, out and
    optionally window, block (bool), karatsuba (bool), flags (MX_IMPL_BLOCK,
    MX_MUL_KARATSUBA, MX_ONE_LANE, MX_TWO_LANES, MX_FOUR_LANES), ctx_idx, tile_cost.  The device buffers
    are captured by the plan; every launch reads and writes them.
    """

    def __init__(self, batches):
        descs = (BatchDesc * len(batches))()
        self._keep = []
        for k, b in enumerate(batches):
            ctx, base, exp, out = b["ctx"], b["base"], b["exp"], b["out"]
            n = base.shape[0]
            _check_rows("base", base, n, ctx.words)
            _check_rows("out", out, n, ctx.words)
            if b["exp_bits"]:
                _check_rows("exp", exp, n, words_for(b["exp_bits"]))
            _check_idx(b.get("ctx_idx"), n, ctx)
            d = descs[k]
            d.ctx, d.ctx_idx = ctx.handle, _ptr(b.get("ctx_idx"))
            d.base, d.exp, d.out = _ptr(base), _ptr(exp) if b["exp_bits"] else None, _ptr(out)
            d.n, d.exp_bits, d.window = n, b["exp_bits"], b.get("window", 0)
            d.flags = ((MX_MUL_KARATSUBA if b.get("karatsuba") else 0) | (MX_IMPL_BLOCK if b.get("block") else 0) |
                       int(b.get("flags", 0)))
            d.tile_cost = float(b.get("tile_cost", 0.0))
            self._keep.append(b)
        self._h = ctypes.c_void_p()
        _check(lib().mx_mixed_plan_create(ctypes.byref(self._h), descs, len(batches)))
        nj, ns = _U32(), _U32()
        win = (_U32 * len(batches))()
        _check(lib().mx_mixed_plan_query(self._h, ctypes.byref(nj), ctypes.byref(ns), win))
        self.njobs, self.nslots, self.windows = nj.value, ns.value, list(win)

    def launch(self, stream=None, graph=False):
        f = lib().mx_mixed_plan_launch_graph if graph else lib().mx_mixed_plan_launch
        _check(f(self._h, _stream_ptr(stream)))

    def close(self):
        if self._h:
            lib().mx_mixed_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_modexp(ctx, n, exp_bits, windows=(3, 4, 5, 6), try_block=True, reps=2, stream=None):
    """Fastest (window, flags) for this context's class; returns (window, flags, ms_per_64_tile)."""
    arr = (_U32 * len(windows))(*windows)
    bw, bf, bms = _U32(), _U32(), ctypes.c_float()
    _check(lib().mx_tune_modexp(ctx.handle, n, exp_bits, arr, len(windows), 1 if try_block else 0, reps,
                                ctypes.byref(bw), ctypes.byref(bf), ctypes.byref(bms), _stream_ptr(stream)))
    return bw.value, bf.value, bms.value


def modexp_ws_bytes(ctx, n, window=0, block=False, flags=None):
    """Workspace bytes of one exponentiation launch over n instances (modexp_ws_bytes)."""
    nb = ctypes.c_size_t()
    f = _impl_flags(block) if flags is None else flags
    st = lib().modexp_ws_bytes(ctx.handle, n, window, f & (MX_IMPL_BLOCK | MX_MUL_KARATSUBA | MX_ONE_LANE |
                                                          MX_TWO_LANES | MX_FOUR_LANES), ctypes.byref(nb))
    if st != MX_OK:  # the batch call reports the same error with its own name
        return 0
    return nb.value


def modexp_ws(ctx, base, exp, exp_bits, ws, window=0, out=None, ctx_idx=None, plain=False, stream=None,
              block=False, n=None, one_lane=False, cios=False, two_lanes=False, four_lanes=False):
    """modexp with a caller-owned workspace tensor (uint8/any dtype, device); n rows of base/exp used."""
    n = base.shape[0] if n is None else n
    if out is None:
        import torch
        out = torch.empty_like(base)
    if n > base.shape[0] or n > out.shape[0] or (exp_bits and n > exp.shape[0]):
        raise ValueError("n exceeds the buffers")
    for nm, t in (("base", base), ("out", out)):
        _check_rows(nm, t, t.shape[0], ctx.words)
    if exp_bits:
        _check_rows("exp", exp, exp.shape[0], words_for(exp_bits))
    if ctx_idx is not None:
        if ctx_idx.dtype.__str__() != "torch.int32" or ctx_idx.shape[0] < n or not ctx_idx.is_cuda:
            raise ValueError("ctx_idx: expected int32 device tensor with >= n entries")
    elif n > ctx.count:
        raise ValueError("n exceeds the context count (pass ctx_idx)")
    if not ws.is_cuda or not ws.is_contiguous():
        raise ValueError("ws: expected a contiguous device tensor")
    flags = (_redc_flags(plain, cios) | _impl_flags(block) | (MX_ONE_LANE if one_lane else 0) |
             (MX_TWO_LANES if two_lanes else 0) | (MX_FOUR_LANES if four_lanes else 0))
    _check(lib().modexp_batch_ws(ctx.handle, _ptr(ctx_idx), _ptr(base), _ptr(exp) if exp_bits else None,
                                 exp_bits, window, _ptr(out), n, flags, _ptr(ws), ws.numel() * ws.element_size(),
                                 _stream_ptr(stream)))
    return out


def rsa_crt(ctx_p, ctx_q, c, dp, dq, qinv, window=0, out=None, key_idx=None, plain=False, cios=False, stream=None,
            ws=None):
    """RSA private-key operation by the CRT (rsa_crt_batch, or rsa_crt_batch_ws with a caller workspace ws):
    c^d mod p q per instance.

    ctx_p, ctx_q: Contexts of the primes (same class, 1024 or 2048 bits); c, out: int64 [n, 2 W];
    dp, dq, qinv: int64 [n, W] with W = bits / 64; key_idx: int32 device tensor or None."""
    n = c.shape[0]
    W = ctx_p.words
    if out is None:
        import torch
        out = torch.empty_like(c)
    for nm, t, w in (("c", c, 2 * W), ("out", out, 2 * W), ("dp", dp, W), ("dq", dq, W), ("qinv", qinv, W)):
        _check_rows(nm, t, n, w)
    if key_idx is not None:
        _check_idx(key_idx, n, ctx_p)
    elif n > min(ctx_p.count, ctx_q.count):
        raise ValueError("n exceeds the key count (pass key_idx)")
    flags = _redc_flags(plain, cios)
    if n and ws is None:
        nb = ctypes.c_size_t()
        if lib().rsa_crt_ws_bytes(ctx_p.handle, n, window, flags, ctypes.byref(nb)) == MX_OK:
            ctx_p.reserve(nb.value)
    if ws is None:
        _check(lib().rsa_crt_batch(ctx_p.handle, ctx_q.handle, _ptr(key_idx), _ptr(c), _ptr(dp), _ptr(dq),
                                   _ptr(qinv), window, _ptr(out), n, flags, _stream_ptr(stream)))
    else:
        if not ws.is_cuda or not ws.is_contiguous():
            raise ValueError("ws: expected a contiguous device tensor")
        _check(lib().rsa_crt_batch_ws(ctx_p.handle, ctx_q.handle, _ptr(key_idx), _ptr(c), _ptr(dp), _ptr(dq),
                                      _ptr(qinv), window, _ptr(out), n, flags, _ptr(ws), ws.numel() * ws.element_size(),
                                      _stream_ptr(stream)))
    return out


def rsa_crt_ws_bytes(ctx_p, n, window=0, plain=False, cios=False):
    """Workspace bytes of rsa_crt over n instances as one paired launch (rsa_crt_ws_bytes)."""
    nb = ctypes.c_size_t()
    _check(lib().rsa_crt_ws_bytes(ctx_p.handle, n, window, _redc_flags(plain, cios), ctypes.byref(nb)))
    return nb.value


MUL_METHODS = {"schoolbook": 0, "karatsuba": MX_MUL_KARATSUBA, "karatsuba2": MX_MUL_KARATSUBA2}


def mp_mul_ws_bytes(bits, n, method="schoolbook"):
    nb = ctypes.c_size_t()
    _check(lib().mp_mul_ws_bytes(bits, n, MUL_METHODS[method], ctypes.byref(nb)))
    return nb.value


def mp_mul(a, b, bits, method="schoolbook", out=None, ws=None, stream=None):
    """Full products a[i] * b[i] (a[i]^2 when b is None) of bits-bit values (mp_mul_batch).

    a, b: int64 device tensors [n, ceil(bits/64)]; out: [n, ceil(2 bits/64)]; ws: a device workspace
    tensor (allocated here for one launch when None); method: schoolbook, karatsuba or karatsuba2."""
    import torch
    n = a.shape[0]
    _check_rows("a", a, n, words_for(bits))
    if b is not None:
        _check_rows("b", b, n, words_for(bits))
    if out is None:
        out = torch.empty((n, words_for(2 * bits)), dtype=torch.int64, device=a.device)
    _check_rows("out", out, n, words_for(2 * bits))
    if ws is None:
        ws = torch.empty(max(1, mp_mul_ws_bytes(bits, n, method)), dtype=torch.uint8, device=a.device)
    if not ws.is_cuda or not ws.is_contiguous():
        raise ValueError("ws: expected a contiguous device tensor")
    _check(lib().mp_mul_batch(_ptr(a), _ptr(b), _ptr(out), bits, n, MUL_METHODS[method], _ptr(ws),
                              ws.numel() * ws.element_size(), _stream_ptr(stream)))
    return out


def to_device(words_u64, device="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(words_u64, dtype=np.uint64).view(np.int64)).to(device)


def to_host(t):
    return t.cpu().numpy().view(np.uint64)
