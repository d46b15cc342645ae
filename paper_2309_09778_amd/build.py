"""Build the HIP library libpwrel.so for gfx950 (in-tree, next to this file)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpwrel.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("pwrel_codec.hip", "pwrel_compress.hip",
                                                   "pwrel_decode.hip", "pwrel_train.hip",
                                                   "pwrel_api.hip", "pwrel_noalloc.hip",
                                                   "pwrel_huffman.hip", "pwrel_decode_lanes.hip",
                                                   "pwrel_batch.hip", "pwrel_openloop.hip", "pwrel_datablocks.hip")]
HEADERS = [os.path.join(HERE, "csrc", f) for f in ("pwrel_device.h", "pwrel_internal.h",
                                                   "pwrel_kernels.h", "pwrel_bf16.h",
                                                   "pwrel_train.h", "pwrel_huffman.h",
                                                   "pwrel_decode.h", "pwrel_wavesort.h")] + \
    [os.path.join(ROOT, "include", "pwrel.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # every a*b+c outside an explicit fma rounds twice, on host and device
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-variable", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def build(force=True, extra=()):
    """Compile every source to an object in parallel, then link libpwrel.so."""
    if not force and os.path.exists(LIB):
        t = os.path.getmtime(LIB)
        if all(os.path.getmtime(s) <= t for s in SOURCES + HEADERS):
            return LIB
    os.makedirs(OBJDIR, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
        objs.append(obj)
        procs.append((src, subprocess.Popen([HIPCC] + FLAGS + list(extra) +
                                            ["-c", "-o", obj, src])))
    failed = [src for src, p in procs if p.wait() != 0]
    if failed:
        raise RuntimeError(f"hipcc failed on {failed}")
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs,
                   check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
