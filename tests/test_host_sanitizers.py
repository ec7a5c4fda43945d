"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Two builds made here, each exercised by the CPU tests that drive it, in a
child process with the matching ASan runtime preloaded (it must come first):

* the oracle (oracle.c) built by gcc with -fsanitize=address,undefined, run
  through the oracle's pin tests (ORACLE_LIB names the build);
* libjbfd.so with its host pass built by hipcc with the same sanitizers
  (each -fsanitize= behind -Xarch_host; the device code is unchanged), run
  through the C-ABI checks, which reach every entry point's host-side
  argument validation without a GPU (JBFD_LIB names the build).

Undefined behaviour aborts the child (-fno-sanitize-recover); leak checking
is off, the interpreter itself keeps memory until exit.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

ORACLE_TESTS = ["test_oracle_project.py", "test_oracle_filter.py",
                "test_oracle_grad.py", "test_oracle_heldout.py",
                "test_oracle_spread.py", "test_oracle_two_stage.py",
                "test_oracle_cloud.py", "test_oracle_afterimage.py"]


def _gcc_asan():
    if not shutil.which("gcc"):
        return None
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"],
                       capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _clang_asan():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/"
                            "libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def _imports_sanitizer(lib):
    names = subprocess.run(["nm", "-D", "--undefined-only", lib],
                           capture_output=True, text=True).stdout
    return "__asan_report" in names and "__ubsan_handle" in names


def _run_tests(files, runtime, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    # the ASan runtime has to be the first library loaded
    env["LD_PRELOAD"] = " ".join(x for x in (runtime, env.get("LD_PRELOAD"))
                                 if x)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=86"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p",
           "no:cacheprovider", "-m", "not gpu",
           *[os.path.join(ROOT, "tests", f) for f in files]]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True,
                         text=True, timeout=900)
    log = res.stdout + res.stderr
    assert res.returncode == 0, log[-4000:]
    for marker in ("runtime error:", "AddressSanitizer", "LeakSanitizer"):
        assert marker not in log, log[-4000:]
    return log


def test_oracle_under_asan_ubsan(tmp_path):
    runtime = _gcc_asan()
    if runtime is None:
        pytest.skip("gcc's ASan runtime is not installed")
    import oracle
    lib = str(tmp_path / "liboracle_san.so")
    flags = [f for f in oracle.GCC_FLAGS if not f.startswith("-O")]
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", *flags,
                    os.path.join(ROOT, "oracle", "oracle.c"), "-o", lib, "-lm"],
                   check=True)
    assert _imports_sanitizer(lib)
    log = _run_tests(ORACLE_TESTS, runtime, {"ORACLE_LIB": lib})
    assert " passed" in log


def test_abi_host_validation_under_asan_ubsan(tmp_path):
    runtime = _clang_asan()
    if runtime is None:
        pytest.skip("the ROCm compiler's ASan runtime is not installed")
    from paper_2601_01210_amd import build as B
    try:
        B.hipcc()
    except RuntimeError:
        pytest.skip("hipcc is not installed")
    lib = B.build(out=str(tmp_path / "libjbfd_san.so"),
                  extra_flags=B.HOST_SANITIZE_FLAGS)
    assert _imports_sanitizer(lib)
    log = _run_tests(["test_abi.py"], runtime, {"JBFD_LIB": lib})
    assert " passed" in log
