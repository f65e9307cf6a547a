"""Build libbridges.so (HIP for gfx950 + host C++) in the package directory."""
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SO = os.path.join(PKG, "libbridges.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include")]


def sources():
    c = os.path.join(PKG, "csrc")
    return sorted(glob.glob(os.path.join(c, "*.hip")) + glob.glob(os.path.join(c, "*.cpp")))


def build(verbose: bool = False) -> str:
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + sources() + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libbridges.so")
    if verbose:
        sys.stderr.write("\n".join(l for l in (r.stdout + r.stderr).splitlines()
                                   if "packed-fp32-ops" not in l) + "\n")
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
