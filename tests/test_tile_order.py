"""Host check of the products' grouped tile orders (csrc/tile_order.hpp): for
many grid shapes and band heights every index maps to a distinct tile of the
grid (or of its lower triangle), the tiles of one band come column by
column, and the renumbering of dispatch indices by XCD is a bijection.
Compiled with the host compiler; no GPU."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1907_01063_amd", "csrc")

HARNESS = r"""
#include <cstdio>
#include <set>
#include <utility>
#include "tile_order.hpp"
using namespace gpc;
int main() {
    long bad = 0, cases = 0;
    for (int64_t M = 1; M <= 40; ++M)
        for (int64_t G = 2; G <= 17; ++G) {
            for (int64_t N = 1; N <= 23; N += 3) {
                std::set<std::pair<int64_t, int64_t>> seen;
                int64_t prev_tn = 0, prev_band = -1;
                for (int64_t t = 0; t < M * N; ++t) {
                    int64_t tm, tn;
                    grouped_tile(t, M, N, G, tm, tn);
                    if (tm < 0 || tm >= M || tn < 0 || tn >= N) ++bad;
                    seen.insert({tm, tn});
                    const int64_t band = tm / G;
                    if (band == prev_band && tn < prev_tn) ++bad;     // columns never go back within a band
                    if (band < prev_band) ++bad;                     // bands in order
                    prev_band = band; prev_tn = tn;
                }
                if ((int64_t)seen.size() != M * N) ++bad;
                ++cases;
            }
            std::set<std::pair<int64_t, int64_t>> seen;
            int64_t prev_band = -1;
            const int64_t T = M * (M + 1) / 2;
            for (int64_t t = 0; t < T; ++t) {
                int64_t tm, tn, pm, pn;
                grouped_lower_tile(t, M, G, tm, tn);
                if (tn < 0 || tn > tm || tm >= M) ++bad;
                seen.insert({tm, tn});
                const int64_t band = tm / G;
                if (band < prev_band) ++bad;
                prev_band = band;
                lower_tile(t, pm, pn);
                if (pm / G != band) ++bad;                           // same band as in row-by-row order
            }
            if ((int64_t)seen.size() != T) ++bad;
            ++cases;
        }
    // the XCD renumbering is a bijection, each XCD's items contiguous
    for (int nwg = 1; nwg <= 700; ++nwg) {
        std::set<int> items;
        for (int w = 0; w < nwg; ++w) {
            const int u = xcd_item(w, nwg);
            if (u < 0 || u >= nwg) ++bad;
            items.insert(u);
            const int per = nwg / 8;
            if (w < per * 8 && u / per != w % 8) ++bad;   // XCD w mod 8 holds range w mod 8
        }
        if ((int)items.size() != nwg) ++bad;
        ++cases;
    }
    printf("%ld %ld\n", cases, bad);
    return bad != 0;
}
"""


def test_grouped_tile_orders_are_bijections(tmp_path):
    src = tmp_path / "h.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "h"
    r = subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stderr)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    cases, bad = map(int, out.stdout.split())
    assert cases > 1000 and bad == 0 and out.returncode == 0
