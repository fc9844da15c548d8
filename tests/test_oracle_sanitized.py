"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is rebuilt with -fsanitize=address,undefined (every finding
fatal) and the CPU pin tests of its operators, time stepping, adjoint,
27-point stencil and rho/p run against that build in a child process, with
the gcc sanitizer runtimes preloaded into the uninstrumented interpreter.
Any out-of-bounds access, use after free or undefined arithmetic (signed
overflow, bad shifts, misaligned access) in the oracle fails the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_operators.py", "tests/test_oracle_evolution.py", "tests/test_oracle_adjoint.py",
        "tests/test_oracle_stencil27.py", "tests/test_oracle_rho_p.py", "tests/test_oracle_initial_state.py"]


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.timeout(900)
def test_oracle_pins_under_address_and_ub_sanitizers():
    import oracle
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = oracle.build(force=True, sanitize=True)
    env = dict(os.environ, LF_ORACLE_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    # the child loads the sanitizer build, with the runtime mapped
    probe = ("import oracle; oracle.lib(); maps = open('/proc/self/maps').read(); "
             "print(oracle.LIB, 'libasan' in maps, 'liblf_oracle_asan' in maps)")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.split()[-2:] == ["True", "True"], r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=850)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-3000:]
    assert r.returncode == 0, out[-3000:]
    assert " passed" in out
