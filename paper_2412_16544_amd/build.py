"""Builds the HIP library ``libhtrise.so`` for gfx950 in-tree.

    python -m paper_2412_16544_amd.build

Every kernel is hand-written HIP for CDNA4; hipcc cross-compiles without a GPU.
The translation units compile in parallel (device code does not cross them: each
kernel is launched from the file that defines it) and are linked into one shared
library.
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["ht_kernels.hip", "ht_eig.hip", "ht_abi.hip", "ht_testing.hip", "ht_profile.hip", "ht_datagen.hip"]
LIB = os.path.join(HERE, "libhtrise.so")
OBJDIR = os.path.join(HERE, "_build")
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _clean(text: str) -> str:
    return "\n".join(line for line in text.splitlines() if "packed-fp32-ops" not in line)


def build(verbose: bool = False) -> str:
    csrc = os.path.join(HERE, "csrc")
    os.makedirs(OBJDIR, exist_ok=True)
    flags = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"), "-I", csrc]
    srcs = [f for f in SOURCES if os.path.exists(os.path.join(csrc, f))]

    def compile_one(f):
        obj = os.path.join(OBJDIR, os.path.splitext(f)[0] + ".o")
        cmd = [hipcc(), *flags, "-c", os.path.join(csrc, f), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        return obj, res.returncode, _clean(res.stdout + res.stderr)

    with ThreadPoolExecutor(max_workers=min(len(srcs), max(1, os.cpu_count() or 1))) as ex:
        results = list(ex.map(compile_one, srcs))
    errs = [out for _, rc, out in results if rc != 0]
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
    if verbose:
        for _, _, out in results:
            if out.strip():
                print(out)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", *[o for o, _, _ in results], "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + _clean(res.stdout + res.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
