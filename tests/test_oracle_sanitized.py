"""The oracle's pin suite under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is rebuilt with -fsanitize=address,undefined (every report aborts)
and the pins run against that build in a child process that preloads the
sanitizer runtimes.  The three longest convergence studies are left out: they
run the same code paths as the shorter pins on larger boxes.
"""
import os
import subprocess
import sys

import pytest

from oracle import build as oracle_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PIN_FILES = [
    "tests/test_oracle_kinetic.py",
    "tests/test_oracle_reconstruction.py",
    "tests/test_oracle_channel.py",
    "tests/test_oracle_scheme.py",
    "tests/test_oracle_dilatation.py",
    "tests/test_oracle_profiles.py",
]
LONG = ("test_density_wave_order_mode_z or test_tgv_early_decay_converges_to_the_viscous_rate or "
        "test_design_order_density_wave_along_x")


@pytest.mark.slow
def test_oracle_pins_pass_under_sanitizers():
    oracle_build.build(force=False, sanitize=True)
    env = dict(os.environ)
    env.update(
        HGKS_ORACLE_SANITIZED="1",
        LD_PRELOAD=":".join(oracle_build.sanitizer_runtimes()),
        ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
        UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
        OMP_NUM_THREADS="4",
    )
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-p", "no:xdist",
           "-m", "not slow and not gpu", "-k", f"not ({LONG})", *PIN_FILES]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout[-4000:] + "\n" + r.stderr[-4000:]).strip()
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
