"""CPU sanitizer builds of the oracle and of the library's host code.

AddressSanitizer + UndefinedBehaviorSanitizer, host code only (the kernels
are built as usual and never run here: there is no GPU on the build
machine).  The sanitized copies go to a scratch directory and are picked up
by the tests through PENT_ORACLE_LIB / PENTBATCH_LIB, with the matching
sanitizer runtime preloaded into the Python process that runs them:

    python -m tests.sanitize          # build both, run the CPU tests under them

Two runtimes cannot share one process, so the oracle (gcc, libasan) and the
library (hipcc's clang, libclang_rt.asan) run in separate processes.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

# every sanitizer flag sits directly after -Xarch_host: host code only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
ENV_RUN = {
    "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
    "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
}

# the tests each sanitized build runs (no GPU needed)
ORACLE_TESTS = ["tests/test_oracle_pins.py", "tests/test_oracle_cyclic.py",
                "tests/test_oracle_rewrite.py", "tests/test_oracle_workloads.py",
                "tests/test_oracle_mutants.py"]
LIB_TESTS = ["tests/test_abi.py"]


def build_oracle(outdir: str) -> str:
    import oracle
    out = os.path.join(outdir, "_pent_oracle_san.so")
    flags = [f for f in oracle.CFLAGS if f != "-O2"]
    subprocess.check_call(["gcc", "-O1", "-g", *flags, "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", out,
                           oracle._SRC, "-lm"])
    return out


def build_library(outdir: str) -> str:
    from paper_1807_07382_amd import build as hb
    srcs = hb.sources()

    def comp(src):
        obj = os.path.join(outdir, os.path.basename(src) + ".san.o")
        cmd = [HIPCC, *[f for f in hb.HIPFLAGS if f != "-O3"], "-O1", "-g", *HOST_SAN, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"sanitized compile failed for {src}:\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(comp, srcs))
    out = os.path.join(outdir, "libpentbatch_san.so")
    r = subprocess.run([HIPCC, f"--offload-arch={hb.ARCH}", "-shared", "-fPIC", "-o", out, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitized link failed:\n{r.stderr}")
    return out


def gcc_asan_runtime() -> str:
    return subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()


def clang_asan_runtime() -> str:
    hits = sorted(glob.glob(os.path.join(ROCM, "lib", "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise FileNotFoundError("clang's AddressSanitizer runtime is not installed")
    return hits[-1]


def run_tests(tests, preload: str, env_extra: dict) -> subprocess.CompletedProcess:
    env = dict(os.environ)
    env.update(ENV_RUN)
    env.update(env_extra)
    env["LD_PRELOAD"] = preload
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider", *tests]
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)


def main() -> int:
    with tempfile.TemporaryDirectory() as d:
        orc = build_oracle(d)
        r1 = run_tests(ORACLE_TESTS, gcc_asan_runtime(), {"PENT_ORACLE_LIB": orc})
        print(r1.stdout[-2000:], r1.stderr[-2000:])
        lib = build_library(d)
        r2 = run_tests(LIB_TESTS, clang_asan_runtime(), {"PENTBATCH_LIB": lib})
        print(r2.stdout[-2000:], r2.stderr[-2000:])
        return 0 if r1.returncode == 0 and r2.returncode == 0 else 1


if __name__ == "__main__":
    sys.exit(main())
