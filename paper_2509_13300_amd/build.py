"""Build libah.so (and the generator's GPU filler) in-tree for gfx950.

    python -m paper_2509_13300_amd.build

Compiles every HIP source with hipcc --offload-arch=gfx950, embeds the scan
core (csrc/scan_core.hip) into the host runtime as a string for run-time
specialisation, and compiles a few specialisations through the new library
so that a mistake in the core or its generator fails the build rather than
the first call.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are disabled for all device code.
DEVFLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", f"-I{INCLUDE}", f"-I{CSRC}",
          f"-I{BUILD}"]

# Run-time specialisations compiled once at build time (through the built
# library's own generator and hipRTC) so that a mistake in the scan core or
# the generator fails the build rather than the first call: degenerate sets,
# N, a clamp and a non-ACGT mask; then several pairs in several groups.
CHECK = r"""
import os, sys
sys.path.insert(0, sys.argv[1])
from paper_2509_13300_amd import _lib as L
L.LIB_PATH = sys.argv[2]
assert L.ah_scan_program_compile([("ACGTNRYSWKMBDHVACG", "NNNNNAAAACGTGCATG", 2, 3)], True) > 1000
os.environ["AH_SCAN_GROUP"] = "3"
assert L.ah_scan_program_compile([("ACGTACGTACGTACG", "GGCCAATTGGCCAAT", 0, 0),
                                  ("ACRTACGTNNGTACGAAT", "GGCYAATTGGSCAATCC", 1, 1),
                                  ("ACGTACGWACGTACGTACGTAC", "GGCCAATTGGCCAATTAAGG", 3, 0)],
                                 False) > 1000
"""


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(x for x in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in x)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    return out


def _embed(src_path, dst_path):
    text = open(src_path).read()
    delim = "AHSRC"
    assert f"){delim}\"" not in text
    with open(dst_path, "w") as f:
        f.write(f'R"{delim}(' + text + f'){delim}"\n')


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    _embed(os.path.join(CSRC, "scan_core.hip"), os.path.join(BUILD, "scan_core_src.inc"))
    objs = []
    for name in ("ah_kernels.hip", "ah_host.cpp", "ah_stream.cpp", "ah_serve.cpp",
                 "ah_fasta_io.cpp"):
        src = os.path.join(CSRC, name)
        obj = os.path.join(BUILD, name + ".o")
        lang = ["-x", "hip"] if name.endswith(".hip") else []
        _run([HIPCC, *COMMON, *DEVFLAGS, *lang, "-c", src, "-o", obj])
        objs.append(obj)
    # the compile helper: scan programs compile in processes of their own
    helper = os.path.join(HERE, "ah_jitc")
    _run([HIPCC, "-O2", "-std=c++17", os.path.join(CSRC, "ah_jitc.cpp"), "-o", helper + ".tmp",
          "-L/opt/rocm/lib", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"])
    os.replace(helper + ".tmp", helper)
    lib = os.path.join(HERE, "libah.so")
    tmp = lib + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs,
          "-L/opt/rocm/lib", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"])
    # specialisation check with the new library, in a process of its own
    _run([sys.executable, "-c", CHECK, ROOT, tmp])
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.path.insert(0, ROOT)
    from synth import build_gpu  # noqa: E402

    build_gpu.build(verbose=True)
