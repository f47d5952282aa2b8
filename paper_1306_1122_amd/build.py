"""Builds libdbie.so (all HIP sources of csrc/, gfx950) in the package directory.

    python -m paper_1306_1122_amd.build
"""
import concurrent.futures
import glob
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdbie.so")

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-fPIC", "-shared", "-std=c++17", "-fvisibility=hidden",
    # packed FP32 instructions are kept out of every kernel of this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + msg)
    if verbose and msg.strip():
        print(msg)


def build_library(verbose: bool = False, out: str = LIB) -> str:
    """Compile every source to an object (in parallel, at most 8 at a time), then link."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include")]
    cflags = [f for f in HIPCC_FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="dbie_build_") as td:
        objs = [os.path.join(td, os.path.basename(src) + ".o") for src in sources()]
        jobs = [[hipcc] + cflags + inc + ["-c", src, "-o", obj] for src, obj in zip(sources(), objs)]
        with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
            for f in [ex.submit(_run, j, verbose) for j in jobs]:
                f.result()
        tmp = out + ".tmp"
        _run([hipcc] + HIPCC_FLAGS + objs + ["-o", tmp], verbose)
        os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build_library(verbose="-v" in sys.argv)
    print(LIB)
