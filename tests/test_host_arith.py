"""The traversal's integer arithmetic, compiled for the host from the
library's own header (paper_2402_13747_amd/csrc/internal.h) and checked on
the CPU against exact integer division.

span_div(x, m) with m = ceil(2^40 / span) replaces x / span in the DDA, the
key emission and the node links.  It must equal the quotient for every leaf
coordinate 0 <= x < 2^22 and span <= 2^18 (the grid's limits): exhaustively
for a few spans including both limits, and near every multiple (k span - 1,
k span, k span + 1) for every span up to 4096 and sampled spans up to 2^18.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

HARNESS = r'''
#include "internal.h"
#include <cstdio>
#include <cstdint>

static uint64_t magic(uint64_t s) { return ((uint64_t(1) << 40) + s - 1) / s; }

static long check(uint64_t s, int x) {
    const int q = pcrl::span_div(x, magic(s));
    if (q != (int)((uint64_t)x / s)) {
        std::printf("span %llu x %d: %d\n", (unsigned long long)s, x, q);
        return 1;
    }
    return 0;
}

int main() {
    const int X = 1 << 22;
    long bad = 0, n = 0;
    const uint64_t full[] = {1, 3, 7, 10, 100, 4095, (1u << 18) - 1, 1u << 18};
    for (uint64_t s : full)
        for (int x = 0; x < X; ++x, ++n) bad += check(s, x);
    for (uint64_t s = 1; s <= (1u << 18); s = s <= 4096 ? s + 1 : s * 17 / 16 + 1) {
        for (uint64_t k = 1; k * s < (uint64_t)X + s; ++k)
            for (int e = -1; e <= 1; ++e) {
                const int64_t x = (int64_t)(k * s) + e;
                if (x >= 0 && x < X) { bad += check(s, (int)x); ++n; }
            }
        bad += check(s, X - 1);
        ++n;
    }
    std::printf("checked %ld bad %ld\n", n, bad);
    return bad != 0;
}
'''


def test_span_div_is_exact(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not (os.path.exists(hipcc) or shutil.which(hipcc)):
        pytest.skip("no hipcc")
    src = tmp_path / "span_div.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "span_div"
    subprocess.run([hipcc, "--cuda-host-only", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I",
                    os.path.join(ROOT, "paper_2402_13747_amd", "csrc"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "bad 0" in r.stdout
    assert int(r.stdout.split("checked ")[1].split()[0]) > 40_000_000
