"""Build the HIP library liblbm81.so for gfx950 in-tree.

Each storage form's kernels live in their own translation unit
(csrc/kernels_<storage>.hip) so that they compile in parallel; the C ABI is
csrc/lbm81.hip.  The objects are linked into paper_2409_05114_amd/liblbm81.so.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblbm81.so")
BUILD = os.path.join(ROOT, "_build")
SOURCES = ["lbm81.hip", "kernels_f64.hip", "kernels_f32.hip",
           "kernels_f16.hip", "kernels_bf16.hip", "kernels_f64_ent.hip",
           "kernels_f32_ent.hip", "kernels_f16_ent.hip", "kernels_bf16_ent.hip",
           "kernels_f64_ser.hip", "kernels_f32_ser.hip", "kernels_f16_ser.hip",
           "kernels_bf16_ser.hip",
           "diagnostics.hip", "placement.hip"]
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    f"-I{INCLUDE}", f"-I{CSRC}",
    # no packed FP32 instructions (v_pk_*_f32) anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def _compile(src, extra=(), verbose=False):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    return obj, out


def build(verbose=False, extra=()):
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        futs = [ex.submit(_compile, s, extra, verbose) for s in SOURCES]
        objs = []
        for f in futs:
            obj, out = f.result()
            if verbose and out.strip():
                print(out)
            objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
           *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


PROBE_SRC = os.path.join(HERE, "probes", "pattern_ceiling.hip")
PROBE = os.path.join(HERE, "probes", "pattern_ceiling")


def build_probe(verbose=False):
    """The memory-pattern measurement program (probes/pattern_ceiling.hip),
    a standalone executable beside its source; not part of the library."""
    cmd = [HIPCC, *COMMON, PROBE_SRC, "-o", PROBE + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {PROBE_SRC}:\n{r.stdout}{r.stderr}")
    os.replace(PROBE + ".tmp", PROBE)
    return PROBE


if __name__ == "__main__":
    extra = [a for a in sys.argv[1:] if a.startswith("-") and a != "-v"]
    print(build(verbose="-v" in sys.argv, extra=extra))
    print(build_probe(verbose="-v" in sys.argv))
