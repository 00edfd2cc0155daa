"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two builds are made into a temporary directory and exercised in child
processes (the sanitizer runtime has to be the first library loaded, so it is
preloaded into a fresh interpreter):

  oracle    every C source of the oracle, gcc -fsanitize=address,undefined;
            the oracle's own pin tests (those that finish in seconds) run on it
  C ABI     the library's host translation units (parameter validation,
            handle and error management, launch set-up) with host-only ASan
            and UBSan; the kernel objects are the ordinary ones.  The ABI tests
            run on it: every validation and error path that needs no GPU.

Any sanitizer report aborts the child (-fno-sanitize-recover=all), which fails
the test.  Leak checking is off: the interpreter itself does not free
everything at exit.  A first pair of children compiles a deliberate heap
overflow with the same flags and checks that the preloaded runtime reports it,
so a silently inactive sanitizer cannot pass for a clean run.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")

# oracle tests that finish within seconds (the long physics runs stay out)
ORACLE_TESTS = ["test_oracle_pins.py", "test_oracle_mlp.py", "test_oracle_rm.py", "test_oracle_d3q27.py"]
ABI_TESTS = ["test_abi.py"]

OVERFLOW_C = textwrap.dedent("""\
    #include <stdlib.h>
    #ifdef __cplusplus
    extern "C"
    #endif
    int overflow(int n) {
        int *a = (int *)malloc(sizeof(int) * n);
        for (int i = 0; i < n; ++i) a[i] = i;
        int s = a[n];  /* one past the end */
        free(a);
        return s;
    }
    """)


def gcc_asan_runtime():
    path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("gcc's libasan is not installed")
    return path


def child_env(preload, **extra):
    env = dict(os.environ)
    env.update(LD_PRELOAD=preload, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=23", PYTHONDONTWRITEBYTECODE="1")
    env.update(extra)
    return env


def run_child(args, env, timeout):
    r = subprocess.run([sys.executable] + args, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    return r.returncode, r.stdout + r.stderr


def expect_overflow_report(so, preload):
    code = ("import ctypes, sys\n"
            f"lib = ctypes.CDLL({so!r})\n"
            "lib.overflow(5)\n"
            "print('no report')\n")
    rc, out = run_child(["-c", code], child_env(preload), timeout=120)
    assert rc != 0 and "heap-buffer-overflow" in out, out[-2000:]


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    import oracle
    from paper_2010_01628_amd import build as B

    d = tmp_path_factory.mktemp("sanitized")
    gcc_rt = gcc_asan_runtime()
    clang_rt = B.asan_runtime()
    orc = oracle.build(out=str(d / "liboracle_san.so"), sanitize=True)
    abi = B.build_host_sanitized(str(d / "liblbm_san.so"))
    # the deliberate overflow, built with each toolchain's flags
    src = d / "overflow.c"
    src.write_text(OVERFLOW_C)
    gso = d / "overflow_gcc.so"
    subprocess.run(["gcc", "-shared", "-fPIC"] + oracle.SANITIZE + ["-o", str(gso), str(src)], check=True)
    cso = d / "overflow_clang.so"
    subprocess.run([B.HIPCC, "-shared", "-fPIC", f"--offload-arch={B.ARCH}", "-shared-libasan", "-g", "-O1"] +
                   B.HOST_SANITIZE + ["-x", "hip", "-o", str(cso), str(src)], check=True, capture_output=True)
    return dict(oracle=orc, abi=abi, gcc_rt=gcc_rt, clang_rt=clang_rt, gcc_probe=str(gso), clang_probe=str(cso))


def test_sanitizers_report_a_planted_overflow(sanitized):
    expect_overflow_report(sanitized["gcc_probe"], sanitized["gcc_rt"])
    expect_overflow_report(sanitized["clang_probe"], sanitized["clang_rt"])


def test_oracle_clean_under_asan_ubsan(sanitized):
    env = child_env(sanitized["gcc_rt"], ORACLE_LIBRARY=sanitized["oracle"], OMP_NUM_THREADS="4")
    args = ["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu and not slow"]
    args += [os.path.join(TESTS, t) for t in ORACLE_TESTS]
    code = ("import oracle\n"
            "oracle.lib()\n"
            f"assert oracle._SO == {sanitized['oracle']!r}\n"
            "maps = open('/proc/self/maps').read()\n"
            "assert 'liboracle_san.so' in maps and 'libasan' in maps\n")
    rc, out = run_child(["-c", code], env, timeout=120)
    assert rc == 0, out[-3000:]
    rc, out = run_child(args, env, timeout=600)
    assert rc == 0, out[-4000:]
    assert " passed" in out


def test_c_abi_clean_under_asan_ubsan(sanitized):
    env = child_env(sanitized["clang_rt"], LBM_LIBRARY=sanitized["abi"])
    probe = ("from paper_2010_01628_amd import lbm as L\n"
             "L.lib()\n"
             f"assert L.LIB_PATH == {sanitized['abi']!r}\n"
             "maps = open('/proc/self/maps').read()\n"
             "assert 'liblbm_san.so' in maps and 'libclang_rt.asan' in maps\n")
    rc, out = run_child(["-c", probe], env, timeout=300)
    assert rc == 0, out[-3000:]
    args = ["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"]
    args += [os.path.join(TESTS, t) for t in ABI_TESTS]
    rc, out = run_child(args, env, timeout=600)
    assert rc == 0, out[-4000:]
    assert " passed" in out
