"""CPU: the library's exact fp64 residue arithmetic (csrc/arith.hpp, built for
the host) swept against exact integer arithmetic.

The kernels compute every product modulo m of the transforms (Eqs. 2, 3) and of
the pointwise step with fused multiply-adds on residues held in doubles; the
results are exact only inside operand bounds that the kernels' range
bookkeeping keeps to.  tests/fp64_sweep.cpp checks each primitive at those
bounds, for both word policies, with uniform and adversarial operands (exact
quotients within 1/(2m) of a half-integer, operands at the ends of their
ranges), as congruences in 128-bit integers plus the stated bound on |r|."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "fp64_sweep.cpp")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def sweep(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not found")
    exe = str(tmp_path_factory.mktemp("fp64") / "fp64_sweep")
    # host code only (the routines are __host__ __device__)
    subprocess.run([HIPCC, "-x", "hip", "--cuda-host-only", "-O2", "-march=native", "-std=c++17", SRC, "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_fp64_residue_arithmetic_is_exact(sweep):
    r = subprocess.run([sweep, "1000000"], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith(" 0 failures"), r.stdout
    # checks per case: 5 for each of the 7 moduli of 32-bit words, 4 for each of the 3 of 64-bit words
    assert int(r.stdout.split()[0]) >= 1000000 * (7 * 5 + 3 * 4)


def test_sweep_detects_a_wrong_bound(tmp_path):
    # the harness itself: the same sweep with the twiddle operand pushed beyond
    # its exactness limit (|b| m >= 2^53) must report failures
    src = open(SRC).read()
    bad = src.replace("const int64_t bmax = 48 * m - 1 < bfit ? 48 * m - 1 : bfit",
                      "const int64_t bmax = 48 * m - 1")
    assert bad != src
    p = tmp_path / "fp64_sweep_bad.cpp"
    p.write_text(bad.replace('#include "../paper_1005_1497_amd/csrc/arith.hpp"',
                             '#include "%s"' % os.path.join(ROOT, "paper_1005_1497_amd", "csrc", "arith.hpp")))
    exe = str(tmp_path / "bad")
    subprocess.run([HIPCC, "-x", "hip", "--cuda-host-only", "-O2", "-march=native", "-std=c++17", str(p), "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe, "200000"], capture_output=True, text=True, timeout=600)
    assert r.returncode == 1 and "FAIL mulmod m=16777213" in r.stdout
