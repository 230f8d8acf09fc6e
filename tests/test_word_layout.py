"""Host-side check of the reduced-precision word storage (no GPU needed).

word_pos (paper_2004_10811_amd/csrc/smx_internal.h) places word w of element
(r, c) of an n_pad x n_pad group at word_pos(nw, n_pad, r, c) + 32 w.  The
products, conversions and the polish all index through it, so it must be a
bijection onto [0, nw n_pad^2) (no two values share a slot, no slot outside the
group), and one K step of 32 rows of a column (what the products load per
column) must be one contiguous nw * 32-word run.  The header is compiled for the
host with hipcc and the invariants are checked exhaustively for several
padded sizes and word counts.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = r"""
#include "smx_internal.h"
#include <cstdio>
#include <vector>
int main()
{
    const int lds[] = {32, 64, 96, 224, 864, 1056};
    for (int nw = 1; nw <= 3; nw++)
        for (int ld : lds) {
            const long long total = (long long)nw * ld * ld;
            std::vector<unsigned char> seen((size_t)total, 0);
            for (int c = 0; c < ld; c++)
                for (int r = 0; r < ld; r++)
                    for (int w = 0; w < nw; w++) {
                        const long long p = smx::word_pos(nw, ld, r, c) + 32 * w;
                        if (p < 0 || p >= total) { std::printf("out of range nw=%d ld=%d r=%d c=%d w=%d\n", nw, ld, r, c, w); return 1; }
                        if (seen[(size_t)p]++) { std::printf("collision nw=%d ld=%d r=%d c=%d w=%d\n", nw, ld, r, c, w); return 1; }
                    }
            // a K step of 32 rows of column c: words of rows k0 .. k0+31 fill
            // [word_pos(k0, c), word_pos(k0, c) + 32 nw) exactly
            for (int c = 0; c < ld; c += 7)
                for (int k0 = 0; k0 < ld; k0 += 32) {
                    const long long b = smx::word_pos(nw, ld, k0, c);
                    if (b != (long long)c * ld * nw + (long long)k0 * nw) { std::printf("block start nw=%d ld=%d\n", nw, ld); return 1; }
                    for (int i = 0; i < 32; i++)
                        for (int w = 0; w < nw; w++) {
                            const long long p = smx::word_pos(nw, ld, k0 + i, c) + 32 * w;
                            if (p != b + 32 * w + i) { std::printf("block layout nw=%d ld=%d\n", nw, ld); return 1; }
                        }
                }
        }
    std::printf("ok\n");
    return 0;
}
"""


def test_word_positions_are_a_bijection_with_contiguous_k_steps(tmp_path):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    src = tmp_path / "layout.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "paper_2004_10811_amd", "csrc")
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", f"-I{inc}", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
