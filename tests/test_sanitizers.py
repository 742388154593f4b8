"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The C oracle (oracle/oracle.c) and the serving pool's range allocator
(csrc/range_alloc.h) are compiled with -fsanitize=address,undefined by gcc/g++
into small driver programs that exercise every entry point on random and
degenerate graphs (n = 0, one vertex, edgeless, self loops, duplicates, a
capped run, traces shorter than the run) and random allocation sequences.
A sanitizer report makes the program exit non-zero."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE_C = os.path.join(ROOT, "oracle", "oracle.c")
CSRC = os.path.join(ROOT, "paper_1910_05971_amd", "csrc")

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

ORACLE_DRIVER = r'''
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
int32_t oracle_uf_labels(int32_t, const int32_t *, const int32_t *, int32_t *);
int32_t oracle_uf_labels_edges(int32_t, int64_t, const int32_t *, const int32_t *, int32_t *);
int32_t oracle_bfs_labels(int32_t, const int32_t *, const int32_t *, int32_t *);
int32_t oracle_fastsv_alg2(int32_t, const int32_t *, const int32_t *, int32_t, int32_t *, int32_t *, int64_t *, int32_t);
int32_t oracle_fastsv_alg3(int32_t, const int32_t *, const int32_t *, int32_t, const int32_t *, int32_t *, int32_t *,
                           int64_t *, int32_t);
int32_t oracle_sv_variant(int32_t, const int32_t *, const int32_t *, int32_t, int32_t, int32_t *, int32_t *, int64_t *,
                          int32_t);
int32_t oracle_fastsv_async(int32_t, const int32_t *, const int32_t *, int32_t, int32_t *);

static uint64_t st = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return (uint32_t)(st >> 11); }

/* symmetric CSR of m random pairs (loops and repeats kept) on n vertices */
static void build(int32_t n, int32_t m, int32_t **rp, int32_t **col, int32_t **src, int32_t **dst) {
    *src = malloc(sizeof(int32_t) * (m ? m : 1));
    *dst = malloc(sizeof(int32_t) * (m ? m : 1));
    *rp = calloc((size_t)n + 1, sizeof(int32_t));
    *col = malloc(sizeof(int32_t) * (2 * m ? 2 * m : 1));
    for (int32_t i = 0; i < m; ++i) { (*src)[i] = rnd() % n; (*dst)[i] = rnd() % n; }
    for (int32_t i = 0; i < m; ++i) { (*rp)[(*src)[i] + 1]++; (*rp)[(*dst)[i] + 1]++; }
    for (int32_t u = 0; u < n; ++u) (*rp)[u + 1] += (*rp)[u];
    int32_t *cur = malloc(sizeof(int32_t) * (n ? n : 1));
    for (int32_t u = 0; u < n; ++u) cur[u] = (*rp)[u];
    for (int32_t i = 0; i < m; ++i) {
        (*col)[cur[(*src)[i]]++] = (*dst)[i];
        (*col)[cur[(*dst)[i]]++] = (*src)[i];
    }
    free(cur);
}

static int check(int32_t n, int32_t m) {
    int32_t *rp, *col, *src, *dst;
    build(n, m, &rp, &col, &src, &dst);
    int32_t *a = malloc(sizeof(int32_t) * (n ? n : 1)), *b = malloc(sizeof(int32_t) * (n ? n : 1));
    int32_t *c = malloc(sizeof(int32_t) * (n ? n : 1)), *fi = malloc(sizeof(int32_t) * (n ? n : 1));
    const int32_t cap = 3;  /* traces shorter than most runs */
    int32_t *ft = malloc(sizeof(int32_t) * (size_t)(n ? n : 1) * cap);
    int64_t *ct = malloc(sizeof(int64_t) * cap);
    int bad = 0;
    oracle_uf_labels(n, rp, col, a);
    oracle_bfs_labels(n, rp, col, b);
    oracle_uf_labels_edges(n, m, src, dst, c);
    for (int32_t u = 0; u < n; ++u) bad |= a[u] != b[u] || a[u] != c[u];
    int32_t it = oracle_fastsv_alg2(n, rp, col, 0, c, ft, ct, cap);
    for (int32_t u = 0; u < n; ++u) bad |= c[u] != a[u];
    oracle_fastsv_alg2(n, rp, col, 1, c, NULL, NULL, 0);
    for (int32_t u = 0; u < n; ++u) fi[u] = a[u];  /* a valid start: the labels themselves */
    oracle_fastsv_alg3(n, rp, col, 0, NULL, c, ft, ct, cap);
    for (int32_t u = 0; u < n; ++u) bad |= c[u] != a[u];
    oracle_fastsv_alg3(n, rp, col, 0, fi, c, NULL, NULL, 0);
    for (int32_t u = 0; u < n; ++u) bad |= c[u] != a[u];
    for (int32_t fl = 0; fl < 16; ++fl) {
        oracle_sv_variant(n, rp, col, fl, 0, c, ft, ct, cap);
        for (int32_t u = 0; u < n; ++u) bad |= c[u] != a[u];
    }
    oracle_fastsv_async(n, rp, col, 0, c);
    for (int32_t u = 0; u < n; ++u) bad |= c[u] != a[u];
    (void)it;
    free(rp); free(col); free(src); free(dst); free(a); free(b); free(c); free(fi); free(ft); free(ct);
    return bad;
}

int main(void) {
    static const int32_t cases[][2] = {{0, 0}, {1, 0}, {1, 3}, {2, 1}, {7, 0}, {7, 3}, {50, 10}, {50, 200},
                                       {300, 150}, {1000, 3000}, {2000, 1500}};
    for (size_t i = 0; i < sizeof(cases) / sizeof(cases[0]); ++i) {
        const int32_t n = cases[i][0], m = n ? cases[i][1] : 0;
        if (check(n, m)) { printf("FAIL n=%d m=%d\n", n, m); return 1; }
    }
    printf("OK\n");
    return 0;
}
'''

RANGE_DRIVER = r'''
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "range_alloc.h"
using fsv::RangeAlloc;
static unsigned long long st = 88172645463325252ull;
static unsigned long long rnd() { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return st; }
int main() {
    for (long cap : {1L, 2L, 17L, 1000L, 65536L}) {
        RangeAlloc a(cap);
        std::vector<std::pair<long, long>> live;
        for (int k = 0; k < 20000; ++k) {
            if (!live.empty() && rnd() % 2) {
                size_t i = rnd() % live.size();
                a.release(live[i].first, live[i].second);
                live[i] = live.back();
                live.pop_back();
            } else {
                long len = 1 + (long)(rnd() % (cap / 4 + 1));
                long s = a.alloc(len);
                if (s >= 0) live.push_back({s, len});
            }
        }
        for (auto &r : live) a.release(r.first, r.second);
        a.reset(cap);
        if (a.alloc(cap) != 0) { std::printf("FAIL cap=%ld\n", cap); return 1; }
    }
    std::printf("OK\n");
    return 0;
}
'''


def _have_sanitizer_runtime(tmp):
    probe = tmp / "p.c"
    probe.write_text("int main(void){return 0;}\n")
    r = subprocess.run(["gcc", *SAN, str(probe), "-o", str(tmp / "p")], capture_output=True)
    return r.returncode == 0


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    return subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)


@pytest.fixture(scope="module")
def tmp(tmp_path_factory):
    if shutil.which("gcc") is None or shutil.which("g++") is None:
        pytest.skip("no host compiler")
    d = tmp_path_factory.mktemp("san")
    if not _have_sanitizer_runtime(d):
        pytest.skip("sanitizer runtime not available")
    return d


def test_oracle_under_asan_ubsan(tmp):
    src = tmp / "oracle_drv.c"
    src.write_text(ORACLE_DRIVER)
    exe = tmp / "oracle_drv"
    subprocess.run(["gcc", *SAN, "-std=c11", str(src), ORACLE_C, "-o", str(exe)], check=True)
    out = _run(str(exe))
    assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout + out.stderr[-4000:]


def test_range_alloc_under_asan_ubsan(tmp):
    src = tmp / "ra_drv.cpp"
    src.write_text(RANGE_DRIVER)
    exe = tmp / "ra_drv"
    subprocess.run(["g++", *SAN, "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    out = _run(str(exe))
    assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout + out.stderr[-4000:]
