"""Build libccd.so (all HIP kernels and the C ABI) for gfx950 with hipcc.

Device code is compiled with floating-point contraction off (every fused
multiply-add is an explicit fma) and without denormal flushing, because the
narrow phase's error bound is derived for exactly that arithmetic.
"""
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["broad.hip", "narrow.hip", "wide.hip", "learned.hip", "api.hip"]
HEADERS = ["ccd_internal.h", "interval.h", "mlp_tile.h"]
LIB = os.path.join(HERE, "libccd.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
# The wide stage's atomics are issued by one lane or are rare; the atomic
# optimizer's wave-level rewriting of them only lengthens its node loop.
EXTRA = {"wide.hip": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]}


def build(verbose=False):
    """Compile every source to an object (in parallel), then link the shared library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory() as d:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(d, src + ".o")
            cmd = [hipcc] + FLAGS + EXTRA.get(src, []) + inc + ["-c", os.path.join(HERE, "csrc", src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        failed = []
        for src, pr in procs:
            out, _ = pr.communicate()
            if pr.returncode != 0:
                sys.stderr.write(out)
                failed.append(src)
        if failed:
            raise RuntimeError("hipcc failed compiling " + ", ".join(failed))
        cmd = [hipcc, "--offload-arch=gfx950", "-fPIC", "-shared"] + objs + ["-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking libccd.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
