"""Batched truncated-Montgomery modular arithmetic for AMD MI355X (gfx950).

The GPU library is ``libmontexp.so`` (C ABI declared in include/montexp.h);
``paper_2410_18129_amd.montexp`` is its thin ctypes binding.  Nothing here
falls back to CPU arithmetic: if the library is missing, calls raise.
"""
