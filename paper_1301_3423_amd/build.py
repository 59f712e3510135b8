"""Builds the HIP library librlb.so for gfx950 in-tree with hipcc.

    python -m paper_1301_3423_amd.build
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "rlb_capi.hip")
OUT = os.path.join(PKG, "librlb.so")
# streaming-ceiling kernels for the benchmark (not part of the method)
PROBE_SRC = os.path.join(PKG, "csrc", "stream_probe.hip")
PROBE_OUT = os.path.join(PKG, "libstream_probe.so")

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++20",
    "-fPIC",
    "-shared",
    # no packed fp32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds fuse only within one source expression: the rounding of
    # every kernel then follows the source alone, not how the compiler splits
    # the code into blocks, so kernel variants that run the same arithmetic
    # (two-buffer pull and in-place AA steps) give identical bits
    "-ffp-contract=on",
    "-I", os.path.join(REPO, "include"),
]


def source_digest():
    """sha256 over the kernel sources and compiled-in tables: identifies the
    kernels a profile was taken of."""
    import hashlib
    h = hashlib.sha256()
    files = []
    for d in (os.path.join(PKG, "csrc"), os.path.join(PKG, "lattice")):
        for f in sorted(os.listdir(d)):
            if f.endswith((".hip", ".hpp", ".inc", ".sha")):
                files.append(os.path.join(d, f))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(a for a in HIP_FLAGS if os.sep not in a).encode())
    return h.hexdigest()


def hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(extra=(), out=OUT, verbose=False, src=SRC):
    cmd = [hipcc()] + HIP_FLAGS + list(extra) + [src, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building %s" % out)
    os.replace(out + ".tmp", out)
    return out


def build_probe(verbose=False):
    return build(out=PROBE_OUT, verbose=verbose, src=PROBE_SRC)


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_probe(verbose=True))
