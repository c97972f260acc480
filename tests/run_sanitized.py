"""Runs the CPU test suite (-m "not gpu") against host-sanitized builds of
the library and the oracle: AddressSanitizer + UndefinedBehaviorSanitizer on
the planner, the C ABI's argument handling and the C oracle (the GPU code is
built as usual and not run).  CPU only.

    python tests/run_sanitized.py [extra pytest arguments]

Builds paper_1307_2100_amd/_lib/libtc_sanitized.so and
oracle/_build/libtc_oracle_sanitized.so, then runs pytest in a child
process with clang's ASan runtime preloaded; any sanitizer report aborts the
run (UBSan without recovery), so the exit status is the verdict."""
import glob
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _load(name, rel):
    spec = importlib.util.spec_from_file_location(name, os.path.join(ROOT, rel))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def main():
    lib = _load("_tc_build", "paper_1307_2100_amd/build.py").build(sanitize=True)
    orc = _load("_oracle_build", "oracle/build_oracle.py").build_sanitized()
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        sys.exit("clang's ASan runtime is not installed")
    env = dict(os.environ, TC_LIBRARY=lib, TC_ORACLE_LIBRARY=orc, LD_PRELOAD=rt[-1],
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:allocator_may_return_null=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-q", "-m", "not gpu", "-p", "no:xdist"] + \
        sys.argv[1:]
    print("running:", " ".join(cmd), flush=True)
    sys.exit(subprocess.call(cmd, env=env, cwd=ROOT))


if __name__ == "__main__":
    main()
