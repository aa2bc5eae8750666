"""Build the HIP library libjsvd.so for gfx950 (in-tree).

All kernels and the C ABI are compiled by hipcc into one shared library with
contraction of a*b+c disabled (every fma is written out explicitly, so the
results are the bit patterns of the paper's operation sequences), IEEE
division and square root, and packed-FP32 instructions disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libjsvd.so")
ARCH = os.environ.get("JSVD_ARCH", "gfx950")

HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "--offload-arch=" + ARCH, "-Wall", "-Wno-unused-result"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def build(verbose: bool = False, jobs: int = 8) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, procs = [], []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [hipcc] + HIPFLAGS + ["-x", "hip", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        # the host pass warns that it does not know the packed-fp32 feature; drop that line
        procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True), src))
        objs.append(obj)
        while len([p for p, _ in procs if p.poll() is None]) >= jobs:
            procs[[p.poll() is None for p, _ in procs].index(True)][0].wait()
    for p, src in procs:
        err = p.communicate()[1]
        err = "\n".join(l for l in err.splitlines() if "packed-fp32-ops" not in l)
        if err.strip():
            print(err, file=sys.stderr)
        if p.returncode != 0:
            raise RuntimeError("hipcc failed on " + src)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
