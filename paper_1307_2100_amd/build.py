"""Builds the HIP library libtc.so for gfx950 in-tree (paper_1307_2100_amd/_lib/).

Every source under csrc/ is compiled with hipcc (one process per file, in
parallel) and linked into one shared library exposing the C ABI of
include/tc.h."""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
OUT = os.path.join(OUT_DIR, "libtc.so")
OBJ_DIR = os.path.join(HERE, "_build")
# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build of the same
# sources (the GPU code is built as usual): a CPU check of the planner and
# the C ABI's argument handling, loaded in place of libtc.so through
# TC_LIBRARY with clang's ASan runtime preloaded (tests/run_sanitized.py).
OUT_SANITIZED = os.path.join(OUT_DIR, "libtc_sanitized.so")
OBJ_DIR_SANITIZED = os.path.join(HERE, "_build_sanitized")
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]

ARCH = os.environ.get("TC_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src, sanitize=False):
    obj = os.path.join(OBJ_DIR_SANITIZED if sanitize else OBJ_DIR, os.path.basename(src) + ".o")
    cmd = ["hipcc"] + FLAGS + (SANITIZE_FLAGS if sanitize else []) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, out))
    return obj, out


def build(verbose=False, sanitize=False):
    os.makedirs(OUT_DIR, exist_ok=True)
    os.makedirs(OBJ_DIR_SANITIZED if sanitize else OBJ_DIR, exist_ok=True)
    srcs = sources()
    jobs = min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda f: _compile(f, sanitize), srcs))
    objs = []
    for obj, out in results:
        objs.append(obj)
        if verbose and out.strip():
            print(out)
    out = OUT_SANITIZED if sanitize else OUT
    tmp = out + ".tmp%d" % os.getpid()
    cmd = (["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH] + (SANITIZE_FLAGS if sanitize else []) + objs +
           ["-o", tmp])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
