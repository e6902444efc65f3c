"""Build libdedisp.so (HIP for gfx950) in-tree.

    python -m paper_1107_2516_amd.build

Compiles every csrc/*.hip (device + host) and csrc/*.cpp (host) with hipcc
and links paper_1107_2516_amd/libdedisp.so.  Device code is built for gfx950
only, with packed-FP32 instruction selection disabled.
"""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdedisp.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result",
          "-I", os.path.join(HERE, "..", "include"), "-I", BUILD]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]
# host files whose floating-point results decide integers (the delay table)
NO_CONTRACT = {"dd_plan.cpp"}


def _compile(src: str, verbose: bool) -> str:
    name = os.path.basename(src)
    obj = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC] + COMMON
    if name.endswith(".hip"):
        cmd += ["-x", "hip"] + DEVICE
    else:
        cmd += ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include")]
    if name in NO_CONTRACT:
        cmd += ["-ffp-contract=off"]
    cmd += ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {name}\n{r.stdout}\n{r.stderr}")
    errs = [ln for ln in r.stderr.splitlines() if "warning" in ln and "packed-fp32-ops" not in ln]
    if errs and verbose:
        print("\n".join(errs), file=sys.stderr)
    return obj


def _generate(verbose: bool) -> None:
    """Generated sources: the inline-assembly inner steps of the register-window
    kernels (csrc/gen_window_asm.py -> _build/dd_window_asm.inc)."""
    out = os.path.join(BUILD, "dd_window_asm.inc")
    r = subprocess.run([sys.executable, os.path.join(CSRC, "gen_window_asm.py")],
                       capture_output=True, text=True, check=True)
    tmp = out + ".tmp"
    with open(tmp, "w") as f:
        f.write(r.stdout)
    os.replace(tmp, out)
    if verbose:
        print(f"generated {out}", file=sys.stderr)


def build(verbose: bool = False, jobs: int = 8) -> str:
    if not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(BUILD, exist_ok=True)
    _generate(verbose)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def clean() -> None:
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
