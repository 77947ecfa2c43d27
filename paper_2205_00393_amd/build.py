"""Build libltn.so (host planner + HIP kernels for gfx950) in-tree.

Usage: python -m paper_2205_00393_amd.build   (or call ``build()``).
Objects go to ``<repo>/_build/``; the library to
``paper_2205_00393_amd/libltn.so``.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "libltn.so")
BUILD = os.path.join(ROOT, "_build")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}", "-Wall",
          "-Wno-unused-function", "-Wno-unused-variable"]
# device code: no packed-FP32 instructions (the compiler would otherwise form
# them from ordinary float code)
HIP_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-ffp-contract=off"]

SOURCES = [
    ("common.cpp", "host"),
    ("network.cpp", "host"),
    ("planner.cpp", "host"),
    ("plan.cpp", "host"),
    ("runtime.hip", "hip"),
    ("k_misc.hip", "hip"),
    ("k_mfma.hip", "hip"),
    ("k_permute.hip", "hip"),
    ("k_narrow.hip", "hip"),
    ("k_fused.hip", "hip"),
    ("k_skinny.hip", "hip"),
]


def _compile(src_kind):
    src, kind = src_kind
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC] + COMMON
    if kind == "hip":
        cmd += HIP_FLAGS + ["-x", "hip"]
    else:
        cmd += HOST_FLAGS + ["-x", "c++"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l]
    return src, r.returncode, "\n".join(msgs), obj


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source and link the shared library; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_compile, SOURCES))
    errors = [(s, m) for s, rc, m, _ in results if rc != 0]
    if verbose or errors:
        for s, rc, m, _ in results:
            if m.strip():
                print(f"--- {s}\n{m}", file=sys.stderr)
    if errors:
        raise RuntimeError("libltn build failed in: " + ", ".join(s for s, _ in errors))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + \
          [o for _, _, _, o in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("libltn link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
