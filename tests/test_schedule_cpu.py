"""The round-robin order of the symmetric product's block pairs (host code,
built with g++ from the library's own header): every unordered pair of
distinct blocks meets once, every diagonal tile appears once, each block
takes part in exactly one tile per round, and the passes cover the rounds
within the slot limit."""
import os
import subprocess

import pytest

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1301_5885_amd", "csrc", "sym_schedule.h")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "sym_schedule.h"
int main() {
    std::vector<std::pair<int, int>> t;
    for (int nbk = 1; nbk <= 300; ++nbk) {
        std::vector<int> seen((size_t)nbk * nbk, 0);
        for (int r = 0; r < nbk; ++r) {
            gabi::sym_round(nbk, r, t);
            std::vector<int> use(nbk, 0);
            for (auto &p : t) {
                if (p.first < 0 || p.second >= nbk || p.first > p.second) {
                    printf("bad tile nbk=%d r=%d (%d,%d)\n", nbk, r, p.first, p.second);
                    return 1;
                }
                seen[(size_t)p.first * nbk + p.second]++;
                use[p.first]++;
                if (p.second != p.first) use[p.second]++;
            }
            for (int k = 0; k < nbk; ++k)
                if (use[k] != 1) {
                    printf("block %d used %d times in round %d of %d\n", k, use[k], r, nbk);
                    return 1;
                }
        }
        for (int a = 0; a < nbk; ++a)
            for (int b = a; b < nbk; ++b)
                if (seen[(size_t)a * nbk + b] != 1) {
                    printf("pair (%d,%d) of %d seen %d times\n", a, b, nbk,
                           seen[(size_t)a * nbk + b]);
                    return 1;
                }
        for (long long ms = 1; ms <= nbk + 2; ++ms) {
            int passes, slots;
            gabi::sym_passes(nbk, ms, passes, slots);
            if (slots > ms || slots < 1 || (long long)passes * slots < nbk ||
                (long long)(passes - 1) * slots >= nbk) {
                printf("passes nbk=%d ms=%lld: %d x %d\n", nbk, ms, passes, slots);
                return 1;
            }
        }
    }
    printf("ok\n");
    return 0;
}
"""


def test_round_robin_schedule(tmp_path):
    src = tmp_path / "sched.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "sched"
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", os.path.dirname(HDR), "-o", str(exe),
                    str(src)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"
