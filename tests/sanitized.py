"""Runs the CPU test suite (-m "not gpu") under AddressSanitizer and
UndefinedBehaviorSanitizer: the oracle, the scene generator and the host side
of the HIP library (argument validation, workspace carving) are rebuilt with
clang's sanitizers into separate *_san.so files, which the packages load when
PG_SANITIZE=1; the sanitizer runtime is preloaded into the Python process.
Leak detection is off (the interpreter itself keeps memory until exit); any
other report aborts the run.

    python tests/sanitized.py [extra pytest arguments]
"""
import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def main() -> int:
    sys.path.insert(0, ROOT)
    import oracle
    import scenegen
    import paper_2404_11894_amd as pg

    oracle.build(sanitize=True)
    scenegen.build(sanitize=True)
    pg.build(sanitize=True)
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        print("no clang AddressSanitizer runtime under /opt/rocm/llvm", file=sys.stderr)
        return 2
    env = dict(os.environ, PG_SANITIZE="1", LD_PRELOAD=rt[-1],
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-m", "not gpu", "-q", "-p", "no:xdist",
           *sys.argv[1:]]
    return subprocess.run(cmd, cwd=ROOT, env=env).returncode


if __name__ == "__main__":
    sys.exit(main())
