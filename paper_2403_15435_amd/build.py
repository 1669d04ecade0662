"""Build the HIP library (libgeoflood.so) in-tree for gfx950.

The FP32 kernels are compiled with FMA contraction allowed, the FP64 kernels
and the host core without it.  Packed FP32 instructions are disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgeoflood.so")
ARCH = os.environ.get("GF_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

UNITS = [
    ("gf_kernels_f32.hip", ["-ffp-contract=on"]),
    ("gf_kernels_f64.hip", ["-ffp-contract=off"]),
    ("gf_net.hip", ["-ffp-contract=off"]),
    ("gf_static.hip", ["-ffp-contract=off"]),
    ("gf_probe.hip", ["-ffp-contract=off"]),
    ("gf_host.cpp", ["-ffp-contract=off", "-pthread"]),
]


def source_digest() -> str:
    """SHA-256 over the device-code sources (kernels and the layouts they
    share with the host) and their compile flags; names the exact kernels a
    profile was taken on.  Host-only code does not enter it."""
    import hashlib
    h = hashlib.sha256()
    h.update(" ".join(COMMON).encode())
    for src, extra in UNITS:
        if src.endswith(".hip"):
            h.update(" ".join(extra).encode())
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".inc", ".h")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD, exist_ok=True)
    objs = [os.path.join(BUILD, os.path.splitext(src)[0] + ".o") for src, _ in UNITS]
    cmds = [["hipcc", *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
            for (src, extra), obj in zip(UNITS, objs)]
    # the units are independent: compile them side by side
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        outs = list(ex.map(_run, cmds))
    if verbose:
        for out in outs:
            if out:
                print(out)
    tmp = LIB + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    if "--digest" in sys.argv:
        print(source_digest())
    else:
        print(build(verbose="-v" in sys.argv))
