"""Build libffsga.so (HIP, gfx950) in the package directory."""
import hashlib
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libffsga.so")
SRCS = [os.path.join(HERE, "csrc", f) for f in ("ffsga.hip", "surrogate.hip")]
INCLUDE = os.path.join(ROOT, "include")
HEADERS = [os.path.join(INCLUDE, f) for f in ("ffsga.h", "ffs_surrogate.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build_id() -> str:
    """First 16 hex digits of sha256 over the HIP sources and the ABI headers."""
    h = hashlib.sha256()
    for path in (*SRCS, *HEADERS):
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# The device-peak measurements (include/ffs_peaks.h), a library of their own so
# that the decoder's build id does not depend on them.
PEAKS_LIB = os.path.join(HERE, "libffspeaks.so")
PEAKS_SRC = os.path.join(HERE, "csrc", "peaks.hip")


def _compile(out, srcs, extra, verbose):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, *extra, "-I", INCLUDE, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(verbose: bool = False, extra=()) -> str:
    _compile(LIB, SRCS, [*extra, f'-DFFS_BUILD_ID="{build_id()}"'], verbose)
    _compile(PEAKS_LIB, [PEAKS_SRC], list(extra), verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
