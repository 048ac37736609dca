"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only) runs a search, a batch search and a generational solve with
restarts without a report: out-of-bounds accesses, use after free, leaks,
signed overflow and bad shifts in the checker itself would show here."""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "dabs_oracle.h"

int main(void) {
    const int n = 37, inst = 6;
    int32_t *W = calloc((size_t)n * n, sizeof(int32_t));
    uint32_t s = 12345u;
    for (int i = 0; i < n; i++)
        for (int j = i; j < n; j++) {
            s = s * 1664525u + 1013904223u;
            int v = (int)(s >> 24) - 128;
            W[i * n + j] = W[j * n + i] = v;
        }
    uint8_t x[37] = {0}, best[37], target[37];
    for (int k = 0; k < n; k++) target[k] = (uint8_t)(k % 3 == 0);
    int64_t delta[37], eb, e;
    int32_t trace[64];
    for (int rule = 0; rule < 8; rule++) {
        memset(x, 0, sizeof x);
        if (orc_search(W, n, rule, 40, 4, 7, 1, 2, 1000, x, target, best, &eb, &e, delta, trace, 64, 1) < 0) return 1;
    }
    uint32_t ph = 0;
    for (int rule = 2; rule <= 7; rule++)
        if (orc_batch_search(W, n, rule, 5, 2 * n, 4, 3, 0, &ph, 1000, x, target, best, &eb, &e, delta, trace, 64,
                             NULL, 0, NULL, 1) < 0) return 2;
    orc_ga_params g;
    memset(&g, 0, sizeof g);
    g.n_algos = 5;
    for (int a = 0; a < 5; a++) g.algos[a] = 2 + a;
    g.n_ops = 8;
    for (int o = 0; o < 8; o++) g.ops[o] = o;
    g.p_explore = 214748365u; g.p_mutation = g.p_zero = g.p_one = 1u << 29;
    g.crossover_kind = 1; g.capacity = 4; g.npools = 2; g.tau = 4; g.T = 4; g.Bn = n; g.greedy_cap = 1000;
    g.seed = 9; g.flags = ORC_GA_RESTART; g.merge_hamming = 10;
    uint8_t *pb = malloc((size_t)2 * 4 * n), *xo = malloc((size_t)inst * n), *tg = malloc((size_t)inst * n);
    int64_t pe[8], eo[6], pk[6], be, rb[5];
    int32_t pa[8], po[8], ins[5 * 6], nr;
    uint32_t pho[6];
    uint8_t bb[37];
    int64_t stt[50];
    if (orc_solve_ex(W, n, &g, inst, 5, pb, pe, pa, po, xo, eo, pho, ins, tg, pk, 1, NULL, NULL, bb, &be, &nr, rb, stt) < 0)
        return 3;
    free(W); free(pb); free(xo); free(tg);
    return 0;
}
"""


def test_oracle_under_asan_and_ubsan():
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "drv.c")
        with open(src, "w") as fh:
            fh.write(DRIVER)
        exe = os.path.join(d, "drv")
        cmd = ["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"), src,
               os.path.join(ROOT, "oracle", "dabs_oracle.c"), "-lm", "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
