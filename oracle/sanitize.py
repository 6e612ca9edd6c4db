"""Run the oracle's CPU pins against an AddressSanitizer + UndefinedBehaviorSanitizer build of
the oracle (test infrastructure; host code only).

    python -m oracle.sanitize

builds bdm_oracle.c with -fsanitize=address,undefined (no recovery: the first report aborts)
into a temporary directory, then runs the `-m "not gpu"` oracle tests in a child process that
preloads the sanitizer runtimes and loads that build through BDM_ORACLE_LIB.  Exits with the
test run's status.
"""
import os
import subprocess
import sys
import tempfile

from oracle.build import CFLAGS, SRC

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
TESTS = ["tests/test_oracle_rng.py", "tests/test_oracle_grid.py", "tests/test_oracle_mech.py",
         "tests/test_oracle_f32_law.py", "tests/test_oracle_spheroid.py", "tests/test_oracle_sir.py",
         "tests/test_oracle_oncology.py", "tests/test_oracle_diffusion.py", "tests/test_oracle_geometry.py",
         "tests/test_pretest_record.py"]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def runtime(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                          check=True).stdout.strip()


def main() -> int:
    with tempfile.TemporaryDirectory() as tmp:
        lib = os.path.join(tmp, "liboracle_san.so")
        cflags = [f for f in CFLAGS if f != "-O2"] + ["-O1"]
        subprocess.run(["gcc", *cflags, *SAN, SRC, "-o", lib, "-lm"], check=True)
        env = dict(os.environ)
        env["BDM_ORACLE_LIB"] = lib
        env["LD_PRELOAD"] = " ".join([runtime("libasan.so"), runtime("libubsan.so")])
        # Python itself is not instrumented: leak reports would list the interpreter's own
        env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
        env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
        cmd = [sys.executable, "-m", "pytest", "-q", "-m", "not gpu", "-p", "no:cacheprovider", *TESTS]
        return subprocess.run(cmd, cwd=ROOT, env=env).returncode


if __name__ == "__main__":
    sys.exit(main())
