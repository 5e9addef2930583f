"""Builds tests/host_check/host_check: the library's host code compiled with
AddressSanitizer and UndefinedBehaviorSanitizer (host pass only; the GPU code
is built as usual), linked with the check driver. Rebuilt only when a source
changed. Used by tests/test_host_sanitizers.py (CPU)."""
import concurrent.futures
import hashlib
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2303_16999_amd", "csrc")
OUT_DIR = os.path.join(HERE, "_build")
EXE = os.path.join(OUT_DIR, "host_check")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
# the sanitizer runtimes must be the compiler's own: clang's, as for the hipcc objects
CLANGXX = "/opt/rocm/llvm/bin/clang++" if os.path.exists("/opt/rocm/llvm/bin/clang++") else "clang++"
ARCH = os.environ.get("SPMM_OFFLOAD_ARCH", "gfx950")
# host files whose code the checks drive: sanitized on the host pass only
SANITIZED = {"runtime.cpp", "serve.cpp", "ell.cpp", "model.cpp", "group.cpp", "tune_cache.cpp", "train.cpp",
             "noalloc.cpp"}
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
COMMON = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"]


def _sources():
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))
    return srcs + [os.path.join(HERE, "host_check.cpp")]


def _digest():
    h = hashlib.sha256()
    for f in _sources() + [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".h")] + \
            [os.path.join(ROOT, "include", "spmm.h"), __file__]:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def _compile(src):
    obj = os.path.join(OUT_DIR, os.path.basename(src) + ".o")
    base = os.path.basename(src)
    if base == "host_check.cpp":
        cmd = [CLANGXX, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-fno-omit-frame-pointer", "-c", src, "-o", obj]
    else:
        cmd = [HIPCC] + COMMON + (HOST_SAN if base in SANITIZED else [])
        cmd += (["-x", "hip"] if src.endswith(".cpp") else []) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build():
    os.makedirs(OUT_DIR, exist_ok=True)
    stamp = os.path.join(OUT_DIR, "stamp")
    d = _digest()
    if os.path.exists(EXE) and os.path.exists(stamp) and open(stamp).read() == d:
        return EXE
    jobs = int(os.environ.get("MAX_JOBS", "8"))
    with concurrent.futures.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(_compile, _sources()))
    # the link names no GPU source (objects only); clang++ brings its sanitizer runtimes
    cmd = [CLANGXX, "-fsanitize=address,undefined", "-o", EXE] + objs + \
          ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-lrocblas", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    open(stamp, "w").write(d)
    return EXE


if __name__ == "__main__":
    print(build())
