"""The oracle's C code and the kernels' host-side integer helper under
sanitizers (CPU only).

* `oracle/tmop_oracle.c` built with AddressSanitizer and
  UndefinedBehaviorSanitizer (gcc, stopping at the first report), loaded in a
  child process in place of the ordinary build, and driven through the
  oracle's Python API on small quad and hex meshes: energy, min det,
  gradient, Hessian action, diagonal, element and dense Hessians, the
  limiting term, and a few Newton steps.  Any out-of-bounds access, use of
  freed memory or undefined operation ends the child with an error; a
  planted one (an output array too short for the gradient, handed to the
  oracle's C entry point) is reported, which shows the check is live.
* the multiply-shift division that the kernels' host set-up uses
  (`make_fastdiv` / `fdiv` in `tmop_dev.hpp`) compiled for the host with
  UndefinedBehaviorSanitizer (no shift or overflow outside the defined range)
  and compared with plain division on random and edge pairs.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2205_12721_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DRIVER = r"""
import numpy as np
import oracle
from oracle import basis
from paper_2205_12721_amd import inputs

cases = [(2, (3, 2), 2, 4, "interior_jitter"), (2, (2, 2), 4, 6, "interior_jitter"),
         (3, (2, 2, 1), 2, 3, "smooth"), (3, (1, 2, 1), 3, 5, "smooth"),
         (3, (2, 2, 2), 2, 9, "smooth")]
for dim, ns, p, nq, recipe in cases:
    pb = oracle.Problem.box(dim, ns, p, nq)
    x, _ = inputs.perturbed_box(dim, ns, p, basis.gll_nodes(p), 1, recipe=recipe, amp=0.05,
                                is_valid=lambda x: pb.min_det(x) > 0)
    v = inputs.gaussian_vector(pb.ndof, 2, pb.ess)
    assert np.isfinite(pb.energy(x)) and pb.min_det(x) > 0
    g, y, d = pb.gradient(x), pb.hvp(x, v), pb.diag(x)
    assert np.all(np.isfinite(g)) and np.all(np.isfinite(y)) and np.all(np.isfinite(d))
    pb.element_hessian(x, 0)
    if pb.ndof <= 400:
        pb.dense_hessian(x)
    pb.set_limiting(x + 0.01, coef=0.5, delta=0.3)
    pb.energy(x), pb.gradient(x), pb.hvp(x, v), pb.diag(x)
    pb.set_limiting(None)
    oracle.newton_solve(pb, x, rel_grad_tol=1e-8, max_newton=2)
print("sanitized oracle ok")
"""

FASTDIV = r"""
#include "tmop_dev.hpp"
#include <cstdio>
#include <cstdint>

int main()
{
    uint64_t state = 0x243f6a8885a308d3ull;
    auto next31 = [&]() {
        uint64_t z = (state += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        z ^= z >> 31;
        return (int)(z >> 33);
    };
    long bad = 0;
    auto check = [&](int n, int d) {
        const tmop::FastDiv f = tmop::make_fastdiv(d);
        if (tmop::fdiv(n, f) != n / d) ++bad;
    };
    for (int d = 1; d <= 4096; ++d) {
        check(0, d);
        check(2147483647, d);
        check(d, d);
        check(d - 1, d);
    }
    for (int k = 0; k < 200000; ++k) {
        const int d = 1 + next31() % 2147483647, n = next31();
        check(n, d);
    }
    std::printf("%ld\n", bad);
    return bad != 0;
}
"""


def _gcc_ok():
    if shutil.which("gcc") is None:
        return False
    return os.path.exists(subprocess.run(["gcc", "-print-file-name=libasan.so"],
                                         capture_output=True, text=True).stdout.strip())


PLANTED = r"""
import ctypes
import numpy as np
import oracle
pb = oracle.Problem.box(2, (3, 2), 2, 4)
x = np.random.default_rng(0).uniform(size=pb.ndof)
out = np.zeros(pb.ndof // 2)  # too short for the gradient
oracle._lib().oracle_gradient(ctypes.byref(pb._pb), oracle._dp(x), oracle._dp(out))
print("not reported")
"""


def _sanitized_env(tmp_path):
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-fPIC",
                           "-shared", "-std=c11", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-o", str(lib),
                           os.path.join(ROOT, "oracle", "tmop_oracle.c"), "-lm"])
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    return dict(os.environ, TMOP_ORACLE_LIB=str(lib), LD_PRELOAD=asan, PYTHONPATH=ROOT,
                ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
                UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=24",
                OMP_NUM_THREADS="2")


@pytest.mark.skipif(not _gcc_ok(), reason="gcc with the AddressSanitizer runtime is needed")
def test_oracle_under_asan_ubsan(tmp_path):
    env = _sanitized_env(tmp_path)
    r = subprocess.run([sys.executable, "-c", PLANTED], env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 23 and "heap-buffer-overflow" in r.stderr, (r.stdout, r.stderr[-2000:])
    r = subprocess.run([sys.executable, "-c", DRIVER], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "sanitized oracle ok" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc is not installed")
def test_fastdiv_under_ubsan(tmp_path):
    src = tmp_path / "fastdiv_ubsan.cpp"
    src.write_text(FASTDIV)
    exe = tmp_path / "fastdiv_ubsan"
    cc = HIPCC if os.path.exists(HIPCC) else "hipcc"
    # host pass only is sanitized (the program has no device code to run)
    r = subprocess.run([cc, "-std=c++17", "-O1", "-I" + CSRC, "-Xarch_host",
                        "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all",
                        str(src), "-o", str(exe)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "0", (r.stdout, r.stderr[-3000:])
