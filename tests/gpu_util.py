"""Helpers shared by the GPU tests (inputs, conversions, oracle sampling)."""
import numpy as np

from paper_2410_18129_amd import workload as wl

LIMB = 28


def r_bits(bits):
    n = (bits + 2 + LIMB - 1) // LIMB
    if bits > 2048:  # whole 37-limb blocks
        n = 37 * ((n + 36) // 37)
    return LIMB * n


def ints_dev(vals, words, device="cuda"):
    import torch
    arr = wl.ints_to_words(vals, words)
    return torch.from_numpy(arr.view(np.int64)).to(device)


def dev_ints(t):
    return wl.words_to_ints(t.cpu().numpy().view(np.uint64))


def adversarial_pairs(N, bits, L=LIMB):
    """Operand pairs in [0, 2N) that stress carries and the low-word indicator."""
    t = bits - 1
    cands = [(0, 0), (1, 1), (N - 1, N - 1), (N, N), (2 * N - 1, 2 * N - 1), (1 << t, 1), (1 << t, 1 << L),
             (2 * N - 1, 1), (N, 2 * N - 1), ((1 << t) - 1, (1 << t) + 1), (2 * N - 2, 2 * N - 1)]
    return [(a % (2 * N), b % (2 * N)) for a, b in cands]
