"""CPU check of the multiply-shift division the kernels use for run-time
divisors fixed at set-up (grid rows, elements per row, polynomial order).

floor(n / d) = (n m) >> s with l = ceil(log2 d), m = ceil(2^(31+l) / d),
s = 31 + l is exact for 0 <= n < 2^31 (Granlund and Montgomery, 1994,
Thm. 4.2).  The header's own `make_fastdiv` / `fdiv` are compiled into a
host program and compared with plain integer division: exhaustively for
small divisors and numerators, on random pairs up to 2^31 - 1, and at the
edges (d = 1, powers of two and their neighbours, n = 2^31 - 1).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2205_12721_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = r"""
#include "tmop_dev.hpp"
#include <cstdio>
#include <cstdint>

static uint64_t state = 0x9e3779b97f4a7c15ull;
static uint32_t next31()
{
    // splitmix64, top 31 bits
    uint64_t z = (state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (uint32_t)(z >> 33);
}

int main()
{
    long bad = 0, checked = 0;
    auto check = [&](int n, int d) {
        const tmop::FastDiv f = tmop::make_fastdiv(d);
        ++checked;
        if (tmop::fdiv(n, f) != n / d) {
            if (bad < 5) std::printf("mismatch n=%d d=%d got %d\n", n, d, tmop::fdiv(n, f));
            ++bad;
        }
    };
    for (int d = 1; d <= 300; ++d)
        for (int n = 0; n < (1 << 16); ++n) check(n, d);
    for (int k = 0; k < 31; ++k) {
        const long long p = 1ll << k;
        for (long long d = p - 1; d <= p + 1; ++d) {
            if (d < 1 || d > 0x7fffffff) continue;
            check(0x7fffffff, (int)d);
            check(0x7ffffffe, (int)d);
            check((int)(d > 1 ? d - 1 : 0), (int)d);
            check((int)d, (int)d);
            for (int r = 0; r < 2000; ++r) check((int)next31(), (int)d);
        }
    }
    for (int r = 0; r < 2000000; ++r) {
        int d = (int)(next31() >> (next31() % 31));
        if (d < 1) d = 1;
        check((int)next31(), d);
    }
    std::printf("checked %ld bad %ld\n", checked, bad);
    return bad == 0 ? 0 : 1;
}
"""


def test_fastdiv_matches_integer_division(tmp_path):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc is not installed")
    src = tmp_path / "fastdiv.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "fastdiv"
    cc = HIPCC if os.path.exists(HIPCC) else "hipcc"
    r = subprocess.run([cc, "-std=c++17", "-O2", "-I" + CSRC, str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert " bad 0" in r.stdout
