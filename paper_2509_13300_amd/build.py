"""Build libah.so (and the generator's GPU filler) in-tree for gfx950.

    python -m paper_2509_13300_amd.build

Compiles every HIP source with hipcc --offload-arch=gfx950, embeds the scan
core (csrc/scan_core.hip) into the host runtime as a string for run-time
specialisation, and compiles that core offline once with a sample pattern
program so that a mistake in it fails the build rather than the first call.
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

SAMPLE_PROGRAM = r"""
#define AH_U 8
#define AH_HALO 19
#define AH_HAS_N 1
"""
SAMPLE_TAIL = r"""
__device__ __forceinline__ void ah_pat_0(const u32* h, const u32* l, const AhCtx& c, u32 t) {
  u32 cl = 0u;
  cl |= (~h[19] | l[19]);
  const u32 a0 = (h[0] | l[0]);
  const u32 a1 = l[1];
  u32 c1 = ~a0;
  c1 |= ~a1;
  u32 cand = c1 & ~cl;
  if (!cand) return;
  cand &= ah_valid(c, t, 20u);
  if (!cand) return;
  u32 nm[20];
#pragma unroll
  for (int j = 0; j < 20; ++j) nm[j] = c.gn[t + j];
  u32 x, cf = 0u; u32 s0 = 0u; u32 s1 = 0u; u32 s2 = 0u;
  x = ((h[0] | l[0]) | nm[0]); s2 |= s1 & x; s1 |= s0 & x; s0 |= x;
  x = (l[1] | nm[1]); s2 |= s1 & x; s1 |= s0 & x; s0 |= x;
  x = ((~h[19] | l[19]) | nm[19]); cf |= x;
  const u32 hb = cand & ~(s2 | cf);
  if (hb) { const u32 lv[2] = {s0, s1}; ah_emit<2>(c, t, hb, lv, 0u, 0u); }
}
__device__ __forceinline__ void ah_group_0(ah_lds_uint2* tw, u32 t0, AhCtx c) {
  for (u32 i = threadIdx.x; i < (u32)AH_TILE; i += AH_BLOCK) {
    const u32 t = t0 + i;
    if (t >= c.S) break;
    u32 h[20], l[20];
#pragma unroll
    for (int j = 0; j < 20; ++j) { const uint2 v = tw[i + (u32)j]; h[j] = v.x; l[j] = v.y; }
    ah_pat_0(h, l, c, t);
  }
}
__device__ void ah_groups(ah_lds_uint2* tw, u32 t0, const AhCtx& c) {
  ah_group_0(tw, t0, c);
}
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
    # offline check of the run-time-compiled core with a sample program
    sample = os.path.join(BUILD, "scan_core_check.hip")
    with open(sample, "w") as f:
        f.write(SAMPLE_PROGRAM + open(os.path.join(CSRC, "scan_core.hip")).read() + SAMPLE_TAIL)
    _run([HIPCC, *COMMON, *DEVFLAGS, "--cuda-device-only", "-include", "hip/hip_runtime.h",
          "-c", sample, "-o",
          os.path.join(BUILD, "scan_core_check.o")])
    objs = []
    for name in ("ah_kernels.hip", "ah_host.cpp", "ah_stream.cpp", "ah_serve.cpp"):
        src = os.path.join(CSRC, name)
        obj = os.path.join(BUILD, name + ".o")
        lang = ["-x", "hip"] if name.endswith(".hip") else []
        _run([HIPCC, *COMMON, *DEVFLAGS, *lang, "-c", src, "-o", obj])
        objs.append(obj)
    lib = os.path.join(HERE, "libah.so")
    tmp = lib + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs,
          "-L/opt/rocm/lib", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"])
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.path.insert(0, ROOT)
    from synth import build_gpu  # noqa: E402

    build_gpu.build(verbose=True)
