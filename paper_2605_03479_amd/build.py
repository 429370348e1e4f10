"""Build the gfx950 HIP library libhbugks.so in-tree with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", "hb_lib.hip")]
DEPS = SRCS + [os.path.join(HERE, "csrc", f) for f in ("hb_runtime.hip", "hb_batch.hip")] + [os.path.join(HERE, "csrc", f) for f in ("hb_kernels.h", "hb_batch_kernels.h", "hb_handle.h",
                                                       "hb_device.h", "hb_layout.h", "hb_mixed.h")] + [
    os.path.join(ROOT, "include", "hb_ugks.h")]
LIB = os.path.join(HERE, "libhbugks.so")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC",
         # packed FP32 VALU forms are kept out of the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-o", LIB + ".tmp", *SRCS]
    if verbose:
        print(" ".join(cmd))
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stderr[-4000:])
    os.replace(LIB + ".tmp", LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
