"""Builds the C oracle (test infrastructure) into oracle/_build/libtc_oracle.so.

Plain gcc, OpenMP, -O2 with -ffp-contract=off so that the plain sum forms no
FMA (the compensated variant calls fma() explicitly)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tc_oracle.c")
OUT_DIR = os.path.join(HERE, "_build")
OUT = os.path.join(OUT_DIR, "libtc_oracle.so")
# AddressSanitizer + UndefinedBehaviorSanitizer build (clang, whose runtime the
# sanitized library run preloads), selected through TC_ORACLE_LIBRARY
OUT_SANITIZED = os.path.join(OUT_DIR, "libtc_oracle_sanitized.so")
CLANG = "/opt/rocm/llvm/bin/clang"


def build(force: bool = True) -> str:
    if not force and os.path.exists(OUT) and os.path.getmtime(OUT) >= os.path.getmtime(SRC):
        return OUT
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-std=c99", SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


def build_sanitized() -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = OUT_SANITIZED + ".tmp%d" % os.getpid()
    cmd = [CLANG, "-O1", "-g", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, OUT_SANITIZED)
    return OUT_SANITIZED


if __name__ == "__main__":
    print(build(force=True))
    sys.exit(0)
