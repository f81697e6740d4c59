"""Build libpfm.so for gfx950 in-tree (hipcc cross-compiles; no GPU needed).

Steps: generate the coefficient/θ tables with csrc/gen_tables.py, then one
hipcc invocation compiles the kernels and the C-ABI runtime (pfm.hip) and
the serving runtime (serve.hip) into paper_2210_03714_amd/libpfm.so.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpfm.so")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # no packed FP32 instructions (v_pk_*_f32): some of their forms have
    # given silently wrong results on gfx950
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc():
    for cand in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(cand) or cand == "hipcc":
            return cand


def build(verbose=False):
    tables = os.path.join(CSRC, "pfm_tables.inc")
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_tables.py"), tables])
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC,
                                      os.path.join(CSRC, "pfm.hip"), os.path.join(CSRC, "serve.hip"),
                                      "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
    if verbose and errs:
        print("\n".join(errs))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
