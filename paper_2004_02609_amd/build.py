"""Build libvoxcap.so (HIP for gfx950) in-tree with hipcc."""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libvoxcap.so")
SOURCES = ["sandwich_f32_36.hip", "sandwich_f32_33.hip", "sandwich_f32_63.hip", "sandwich_f64_36.hip",
           "sandwich_f64_33.hip", "sandwich_f64_63.hip", "mvp_kernels.hip", "ypass_f32.hip", "ypass_f64.hip", "setup_kernels.hip",
           "solver_kernels.hip", "tucker_kernels.hip", "geometry.cpp", "setup.cpp", "apply.cpp", "tucker.cpp", "solver.cpp", "pack.cpp", "tuning.cpp",
           "toeplitz.cpp", "api.cpp", "noalloc.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=gfx950", "-Wall", "-Wno-unused-result",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")]


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"]
    cmd = [HIPCC] + FLAGS + lang + ["-c", os.path.join(SRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, r.returncode, r.stdout + r.stderr, cmd


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        for src, obj, rc, out, cmd in ex.map(_compile, SOURCES):
            if rc != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{' '.join(cmd)}\n{out}")
            if verbose and out.strip():
                print(out)
            objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
