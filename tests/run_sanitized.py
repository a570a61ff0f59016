"""The CPU test suite under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds the oracle (clang, fully instrumented) and libpic's host code
(libpic_san.so: the C ABI, tree builder, argument checks, scratch layout)
with both sanitizers, then runs ``pytest -m "not gpu"`` in a child process
that preloads clang's ASan runtime (the interpreter itself is not
instrumented) and loads those builds instead of the usual ones.  Any report
ends the run with a nonzero status.

    python tests/run_sanitized.py [extra pytest arguments]
"""
import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main(argv):
    import oracle
    from paper_1508_02435_amd import build as hip_build
    libpic = hip_build.build(sanitize=True)
    orc = oracle.build_sanitized(os.path.join(ROOT, "oracle", "_pic_oracle_san.so"))
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        raise SystemExit("clang's ASan runtime was not found")
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": rt[-1],
        # the interpreter and torch are not instrumented: their allocations
        # at exit are not this library's leaks
        "ASAN_OPTIONS": "detect_leaks=0:alloc_dealloc_mismatch=0:abort_on_error=1:halt_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
        "PIC_LIBPIC": libpic,
        "PIC_ORACLE_LIB": orc,
    })
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-m", "not gpu", "-q", "-x",
           "-p", "no:cacheprovider", *argv]
    return subprocess.call(cmd, env=env, cwd=ROOT)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
