"""The CPU test suite under AddressSanitizer and UndefinedBehaviorSanitizer.

Two passes, each with the sanitizer runtime of the compiler that built the
code it loads (the two runtimes cannot share a process):
  1. the oracle's C libraries built by gcc with -fsanitize=address,undefined
     (the oracle's own compiler: the complex-step tangent build must round
     its real parts exactly as the real build does, which gcc's complex
     arithmetic does and clang's does not at every operation), gcc's runtime
     preloaded, every CPU test except the ABI tests;
  2. the host side of libgodunov.so (argument checks, descriptor tables,
     dispatch; the device code as always) built by hipcc with the host-only
     sanitizer flags, clang's runtime preloaded, the ABI tests.
Any sanitizer report aborts its pass with a non-zero status.

    python tests/run_sanitized.py [extra pytest arguments]
"""
import glob
import os
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
GCC_SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer"]
OPTIONS = {
    # python and numpy are not instrumented: leaks at exit are theirs
    "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
    "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
}


def gcc_runtime():
    path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True, check=True).stdout.strip()
    if not os.path.isabs(path):
        raise SystemExit("gcc's ASan runtime was not found")
    return path


def clang_runtime():
    hits = glob.glob(os.path.join(ROCM, "llvm", "lib", "clang", "*", "lib", "linux",
                                  "libclang_rt.asan-x86_64.so"))
    if not hits:
        raise SystemExit("clang's ASan runtime was not found under " + ROCM)
    return hits[0]


def run(env_extra, args):
    env = dict(os.environ, **OPTIONS, **env_extra)
    env.setdefault("OMP_NUM_THREADS", "4")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
           *args]
    print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, env=env, cwd=ROOT).returncode


def main():
    sys.path.insert(0, ROOT)
    import oracle
    from paper_1412_0934_amd import build as gpu_build
    extra = sys.argv[1:]
    with tempfile.TemporaryDirectory() as tmp:
        print("pass 1: the oracle built with gcc's sanitizers", flush=True)
        oracle.build(out_dir=tmp, extra_flags=GCC_SAN)
        rc = run({"LD_PRELOAD": gcc_runtime(), "ORACLE_LIB_DIR": tmp},
                 [os.path.join(ROOT, "tests"), "--ignore", os.path.join(ROOT, "tests", "test_abi.py"),
                  *extra])
        if rc:
            return rc
        print("pass 2: libgodunov.so with its host code instrumented", flush=True)
        lib = gpu_build.build(sanitize=True, out=os.path.join(tmp, "libgodunov.so"))
        return run({"LD_PRELOAD": clang_runtime(), "GODUNOV_LIB": lib},
                   [os.path.join(ROOT, "tests", "test_abi.py"), *extra])


if __name__ == "__main__":
    sys.exit(main())
