"""The oracle's C source under AddressSanitizer and UndefinedBehaviorSanitizer (host code
only): a small driver links puffinn_oracle.c, builds indexes (independent, pooled and
cross-polytope functions) over seeded random points and runs searches under every stopping
rule, at B = 1, 12 and a segment larger than the table, with the filter on and off, k = 1
and k = n, recall 1 (linear scan), the stopping test after 1 to L groups of tables, and
the level trace; any invalid access, leak or
undefined operation aborts the run with a sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "puffinn_oracle.c")

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

uint64_t oracle_splitmix64(uint64_t seed, uint64_t s);
void oracle_hyperplanes(uint64_t seed, int64_t rows, int32_t d, float *out);
int64_t oracle_normalize(float *x, int64_t n, int32_t d);
int oracle_pool_select(uint64_t seed, int32_t pool, int32_t L, int32_t K, int32_t *sel);
void oracle_hash(const float *x, int64_t n, int32_t d, const float *hp, int32_t L, int32_t K, int32_t M,
                 const int32_t *sel, int32_t pool, uint32_t *codes, uint64_t *sketches);
void oracle_cp_hash(const float *x, int64_t n, int32_t d, uint64_t seed, int32_t L, int32_t K, uint32_t *codes);
void oracle_cp_table(uint64_t seed, int32_t d, int32_t R, double *tab);
int32_t oracle_cp_dims(int32_t d, int32_t *dprime, int32_t *ell);
int oracle_build_tables(const uint32_t *codes, int64_t n, int32_t L, int32_t K, uint32_t *tcode, uint32_t *tidx,
                        uint32_t *off);
void oracle_table_sketches(const uint32_t *tidx, const uint64_t *sketches, int64_t n, int32_t L, int32_t M,
                           uint64_t *tsk);
int oracle_search(const float *points, int64_t n, int32_t d, const float *hp, const uint32_t *tcode,
                  const uint32_t *tidx, const uint64_t *tsk, int32_t L, int32_t K, int32_t M, const int32_t *sel,
                  int32_t pool, const double *cptab, uint64_t cp_seed, const float *queries, int64_t m, int32_t k,
                  double recall, double eps, int32_t B, int32_t rule, int32_t filter_on, int32_t groups,
                  int32_t test_entries, int32_t *ids, float *ips,
                  double *ips64, int32_t *stop_level, int64_t *c_scan, int64_t *c_pass, int64_t *c_rerank,
                  int32_t *boundary, int64_t *trace, int64_t *ltrace);
int oracle_bruteforce(const float *points, int64_t n, int32_t d, const float *queries, int64_t m, int32_t k,
                      int32_t *ids, double *ips64);

static float *gauss(int64_t rows, int32_t d, uint64_t seed) {
    float *x = malloc((size_t)rows * d * sizeof(float));
    oracle_hyperplanes(seed, rows, d, x);
    if (oracle_normalize(x, rows, d) >= 0) exit(3);
    return x;
}

int main(void) {
    const int64_t n = 700, m = 9;
    const int32_t d = 19, M = 3;
    float *X = gauss(n, d, 11), *Q = gauss(m, d, 12);
    for (int variant = 0; variant < 3; ++variant) {
        const int32_t K = variant == 2 ? 16 : 24, L = 7, pool = variant == 1 ? 64 : 0;
        int32_t *sel = NULL;
        double *cptab = NULL;
        int64_t rows = (variant == 2 ? 0 : pool ? pool : (int64_t)L * K) + 64 * M;
        float *hp = malloc((size_t)rows * d * sizeof(float));
        oracle_hyperplanes(42, rows, d, hp);
        uint32_t *codes = malloc((size_t)L * n * 4);
        uint64_t *sk = malloc((size_t)M * n * 8);
        if (pool) {
            sel = malloc((size_t)L * K * 4);
            if (oracle_pool_select(42, pool, L, K, sel)) return 4;
        }
        if (variant == 2) {
            int32_t dp, ell;
            oracle_cp_dims(d, &dp, &ell);
            cptab = malloc(41 * (size_t)(ell + 1) * sizeof(double));
            oracle_cp_table(42, d, 50, cptab);
            oracle_cp_hash(X, n, d, 42, L, K, codes);
            oracle_hash(X, n, d, hp, 0, K, M, NULL, 0, NULL, sk);
        } else {
            oracle_hash(X, n, d, hp, L, K, M, sel, pool, codes, sk);
        }
        uint32_t *tcode = malloc((size_t)L * n * 4), *tidx = malloc((size_t)L * n * 4);
        uint32_t *off = malloc((size_t)L * ((1u << 13) + 1) * 4);
        uint64_t *tsk = malloc((size_t)L * n * 8);
        if (oracle_build_tables(codes, n, L, K, tcode, tidx, off)) return 5;
        oracle_table_sketches(tidx, sk, n, L, M, tsk);
        const int32_t kmax = (int32_t)n;
        int32_t *ids = malloc((size_t)m * kmax * 4), *stop = malloc(m * 4), *bd = malloc(m * 4);
        float *ips = malloc((size_t)m * kmax * 4);
        double *ip64 = malloc((size_t)m * kmax * 8);
        int64_t *cs = malloc(m * 8), *cp = malloc(m * 8), *cr = malloc(m * 8);
        int64_t *tr = malloc((size_t)(K + 1) * L * 4 * 8), *lt = malloc((size_t)(K + 1) * 8 * 8);
        const int32_t ks[] = {1, 10, kmax};
        const double recs[] = {0.5, 0.9, 1.0};
        const int32_t Bs[] = {1, 12, 100000};
        int runs = 0;
        for (int rule = 0; rule < 4; ++rule) {
            if (rule == 3 && !pool) continue;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    const int32_t k = ks[a];
                    const double rc = rule == 3 ? 0.5 : recs[b];
                    const int rc_ = oracle_search(X, n, d, hp, tcode, tidx, tsk, L, K, M, sel, pool, cptab, 42, Q, m,
                                                  k, rc, 0.1 * b, Bs[(a + b) % 3], rule, (a + b + rule) % 2 == 0,
                                                  1 + (a * 3 + b) % L, (a * 300 + b * 700) % 1200, ids, ips, ip64,
                                                  stop, cs, cp, cr, bd, tr, lt);
                    if (rc_) return 6;
                    ++runs;
                }
        }
        if (oracle_bruteforce(X, n, d, Q, m, 10, ids, ip64)) return 7;
        printf("variant %d: %d searches\n", variant, runs);
        free(hp); free(codes); free(sk); free(sel); free(cptab); free(tcode); free(tidx); free(off); free(tsk);
        free(ids); free(stop); free(bd); free(ips); free(ip64); free(cs); free(cp); free(cr); free(tr); free(lt);
    }
    free(X);
    free(Q);
    printf("sanitized oracle ok\n");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan(tmp_path):
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "oracle_san"
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-o", str(exe), str(drv), SRC, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized oracle ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
