"""Builds libmontexp.so (the HIP library) in-tree for gfx950.

Each size class is its own translation unit (-DMX_CLASS_BITS=<bits>) so the
heavily unrolled kernels compile in parallel; the C ABI layer is one more.
Usage: python -m paper_2410_18129_amd.build [--jobs J] [--only 1024,2048]
"""
import argparse
import concurrent.futures as cf
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmontexp.so")
CLASSES = (64, 128, 256, 512, 1024, 2048, 3072, 4096)
CIOS_CLASSES = tuple(c for c in CLASSES if c <= 2048)  # register-resident classes
CRT_CLASSES = (1024, 2048)  # prime classes of the CRT-RSA operation (RSA-2048, RSA-4096)
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# hipcc flags: packed FP32 ops stay off (the kernels are integer-only anyway)
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    t = time.time()
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), out))
    return time.time() - t


def build(jobs=None, only=None, verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    classes = CLASSES if not only else tuple(c for c in CLASSES if c in only)
    units = [("mx_abi", [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, "mx_abi.hip"),
                                          "-o", os.path.join(BUILD, "mx_abi.o")])]
    units.append(("mx_mixed", [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, "mx_mixed.hip"),
                                                "-o", os.path.join(BUILD, "mx_mixed.o")]))
    units.append(("mx_mul", [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, "mx_mul.hip"),
                                              "-o", os.path.join(BUILD, "mx_mul.o")]))
    for b in classes:
        units.append(("class_%d" % b, [HIPCC] + FLAGS + ["-DMX_CLASS_BITS=%d" % b, "-c",
                                                       os.path.join(CSRC, "mx_class.hip"),
                                                       "-o", os.path.join(BUILD, "mx_class_%d.o" % b)]))
        if b in CIOS_CLASSES:  # the alternative-reduction kernels of the class, compiled alongside
            units.append(("cios_%d" % b, [HIPCC] + FLAGS + ["-DMX_CLASS_BITS=%d" % b, "-DMX_CIOS_UNIT", "-c",
                                                          os.path.join(CSRC, "mx_class.hip"),
                                                          "-o", os.path.join(BUILD, "mx_cios_%d.o" % b)]))
            units.append(("kredc_%d" % b, [HIPCC] + FLAGS + ["-DMX_CLASS_BITS=%d" % b, "-DMX_KREDC_UNIT", "-c",
                                                           os.path.join(CSRC, "mx_class.hip"),
                                                           "-o", os.path.join(BUILD, "mx_kredc_%d.o" % b)]))
    for b in CRT_CLASSES:
        units.append(("crt_%d" % b, [HIPCC] + FLAGS + ["-DMX_CLASS_BITS=%d" % b, "-c", os.path.join(CSRC, "mx_crt.hip"),
                                                     "-o", os.path.join(BUILD, "mx_crt_%d.o" % b)]))
    # the issue-rate probe: a standalone program that measures the ALU roofline's issue rates
    units.append(("issue_rate", [HIPCC] + FLAGS + ["-o", os.path.join(HERE, "issue_rate"),
                                                  os.path.join(CSRC, "issue_rate.hip")]))
    jobs = jobs or min(len(units), max(1, os.cpu_count() or 1))
    t0 = time.time()
    # largest classes first so they overlap with the small ones
    units.sort(key=lambda u: -int(u[0].split("_")[1]) if u[0].startswith(("class_", "cios_", "kredc_", "crt_")) else
               (-4096 if u[0] in ("mx_mixed", "mx_mul") else 0))
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = {ex.submit(_run, cmd): name for name, cmd in units}
        for f in cf.as_completed(futs):
            dt = f.result()
            if verbose:
                print("  built %-10s %6.1fs" % (futs[f], dt), flush=True)
    objs = ([os.path.join(BUILD, "mx_abi.o"), os.path.join(BUILD, "mx_mixed.o"), os.path.join(BUILD, "mx_mul.o")] +
            [os.path.join(BUILD, "mx_class_%d.o" % b) for b in CLASSES] +
            [os.path.join(BUILD, "mx_cios_%d.o" % b) for b in CLASSES if b in CIOS_CLASSES] +
            [os.path.join(BUILD, "mx_kredc_%d.o" % b) for b in CLASSES if b in CIOS_CLASSES] +
            [os.path.join(BUILD, "mx_crt_%d.o" % b) for b in CRT_CLASSES])
    missing = [o for o in objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError("missing objects (build the other classes first): %s" % missing)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        print("libmontexp.so built in %.1fs" % (time.time() - t0), flush=True)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--only", type=str, default="")
    a = ap.parse_args()
    only = tuple(int(x) for x in a.only.split(",") if x) or None
    build(jobs=a.jobs, only=only)
    sys.exit(0)
