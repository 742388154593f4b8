"""The serving pool's range allocator (host logic, CPU only) against a
brute-force model: every allocation is a free range of the requested length,
no two live ranges overlap, freed ranges coalesce (the whole capacity is one
range again when everything is freed), and an allocation fails only when no
free run of that length exists."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HDR = os.path.join(os.path.dirname(HERE), "paper_1910_05971_amd", "csrc")

DRIVER = r'''
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "range_alloc.h"
using fsv::RangeAlloc;
static unsigned long long st = 88172645463325252ull;
static unsigned long long rnd() { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return st; }
int main(int argc, char **argv) {
    const long cap = atol(argv[1]);
    const int ops = atoi(argv[2]);
    st += atol(argv[3]);
    RangeAlloc a(cap);
    std::vector<char> used(cap, 0);
    std::vector<std::pair<long, long>> live;
    for (int k = 0; k < ops; ++k) {
        if (!live.empty() && (rnd() % 100) < 45) {
            size_t i = rnd() % live.size();
            auto r = live[i];
            live[i] = live.back();
            live.pop_back();
            for (long x = r.first; x < r.first + r.second; ++x) used[x] = 0;
            a.release(r.first, r.second);
        } else {
            long len = 1 + (long)(rnd() % (cap / 8 + 1));
            long s = a.alloc(len);
            // longest free run in the model
            long best = 0, run = 0;
            for (long x = 0; x < cap; ++x) { run = used[x] ? 0 : run + 1; if (run > best) best = run; }
            if (s < 0) {
                if (best >= len) { printf("FAIL missed fit len=%ld best=%ld\n", len, best); return 1; }
                continue;
            }
            if (s + len > cap) { printf("FAIL out of range\n"); return 1; }
            for (long x = s; x < s + len; ++x) {
                if (used[x]) { printf("FAIL overlap at %ld\n", x); return 1; }
                used[x] = 1;
            }
            live.push_back({s, len});
        }
    }
    for (auto &r : live) a.release(r.first, r.second);
    if (a.alloc(cap) != 0) { printf("FAIL no full coalesce\n"); return 1; }
    printf("OK\n");
    return 0;
}
'''


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("ra")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", HDR, str(src), "-o", str(exe)], check=True)
    return str(exe)


@pytest.mark.parametrize("cap,ops,seed", [(64, 4000, 1), (1000, 3000, 2), (5000, 2000, 3), (1, 50, 4)])
def test_range_alloc_matches_model(driver, cap, ops, seed):
    out = subprocess.run([driver, str(cap), str(ops), str(seed)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout
