"""Plants plausible mistakes in a copy of the oracle and checks that the pins
of test_oracle_pins.py catch each one (CPU only; the real oracle is untouched)."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "esg_oracle.c")

MUTATIONS = {
    # POST -> PRE: out-of-range neighbours never enter P
    "pre_instead_of_post": (
        "      list_insert(&P, c);                               /* P <- P u v */",
        "      if ((int64_t)v < x || (int64_t)v > y) continue; list_insert(&P, c);"),
    # stop test without the full-Q guard
    "stop_without_full_q": (
        "if (Q.len >= m && cand_less(Q.a[Q.len - 1], u)) break;",
        "if (Q.len > 0 && cand_less(Q.a[Q.len - 1], u)) break;"),
    # entry point always enters Q (ignores POST)
    "entry_always_in_q": (
        "if (x <= (int64_t)ep && (int64_t)ep <= y) list_insert(&Q, e);",
        "list_insert(&Q, e);"),
    # Q cut to m-1
    "q_off_by_one": ("if (Q.len > m) Q.len = m;", "if (Q.len > m - 1) Q.len = m - 1;"),
    # k-th feature taken one place too far down Q
    "feature_kth_index": ("double qk = kk > 0 ? (double)Q->a[kk - 1].dist : d_ep;",
                          "double qk = kk > 0 ? (double)Q->a[kk < Q->len ? kk : kk - 1].dist : d_ep;"),
    # in-range share counted against |V| + 1
    "feature_inrange_share": ("f[7] = (double)n_inr / (double)nv;",
                              "f[7] = (double)n_inr / (double)(nv + 1);"),
    # P's fill counted over the whole list instead of its live part
    "feature_p_fill_raw": ("f[5] = (double)live_count(P, Q, m) / (double)cap_p;",
                           "f[5] = (double)P->len / (double)cap_p;"),
    # switch taken although the search stops right at the end of the probe
    "switch_when_stopping": ("h == sw->switch_hop &&\n        !(Q.len >= m && cand_less(Q.a[Q.len - 1], P.a[0]))) {",
                             "h == sw->switch_hop) {"),
    # child boundaries rounded down (at fanout 2: the split point moves left)
    "child_start_floor": ("return a + (j * L + f - 1) / f;", "return a + (j * L) / f;"),
    # child numbering off by one
    "child_heap": ("(int64_t)s->fanout * (heap - 1) + 2 + j,", "(int64_t)s->fanout * (heap - 1) + 1 + j,"),
    # half-bounded index: prefix sizes halved with the division rounded down
    "chain_floor": ("    int64_t nx = (sp + base - 1) / base;\n    if (nx == sp || nx < rq + 1) break;",
                    "    int64_t nx = sp / base;\n    if (nx == sp || nx < rq + 1) break;"),
    # half-bounded index: the tie between the two sides goes to the suffix
    "chain_tie": ("else use_prefix = ss >= sp;", "else use_prefix = ss > sp;"),
    # strict elastic comparison
    "elastic_strict": ("return (int64_t)c_den * (y - x + 1) >= (b - a + 1);",
                       "return (int64_t)c_den * (y - x + 1) > (b - a + 1);"),
    # leaf test off by one
    "leaf_test_le": ("if (b - a < s->leaf) {", "if (b - a <= s->leaf) {"),
    # sign of the difference
    "delta_sign": ("float delta = dec(x, j, scale) - q[j];", "float delta = dec(x, j, scale) + q[j];"),
    # last dimension of each chunk dropped
    "chunk_tail_dropped": ("for (int32_t e = 0; e < w; e++) {", "for (int32_t e = 0; e < w - 1; e++) {"),
    # pair tree with halves instead of adjacent pairs
    "tree_halves": ("s[i] = s[2 * i] + s[2 * i + 1];", "s[i] = s[i] + s[i + width / 2];"),
    # chunks given to lanes in blocks instead of strided
    "chunks_blocked": ("for (int32_t c = t; c < chunks; c += g) {",
                       "for (int32_t c = t * ((chunks + g - 1) / g); c < chunks && c < (t + 1) * ((chunks + g - 1) / g); c++) {"),
    # ties broken by larger position
    "tie_reversed": ("return u.dist < v.dist || (u.dist == v.dist && u.pos < v.pos);\n}\n\n/* Sorted",
                     "return u.dist < v.dist || (u.dist == v.dist && u.pos > v.pos);\n}\n\n/* Sorted"),
    # brute force filter off by one at the right end
    "bruteforce_range": ("for (int64_t p = lq; p <= rq; p++) {\n    double s = 0.0;",
                         "for (int64_t p = lq; p < rq; p++) {\n    double s = 0.0;"),
    # fp8 exponent bias wrong
    "e4m3_bias": ("else v = ldexpf(1.0f + (float)m / 8.0f, e - 7);",
                  "else v = ldexpf(1.0f + (float)m / 8.0f, e - 8);"),
}


@pytest.fixture(scope="module")
def src_text():
    return open(SRC).read()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, src_text, tmp_path):
    old, new = MUTATIONS[name]
    assert src_text.count(old) == 1, f"mutation anchor not found once: {name}"
    mutated = tmp_path / "esg_oracle_mut.c"
    mutated.write_text(src_text.replace(old, new))
    so = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-shared",
                           "-fPIC", "-o", str(so), str(mutated), "-lm"])
    env = dict(os.environ, ESG_ORACLE_LIB=str(so), PYTHONPATH=ROOT)
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert p.returncode == 1, f"mutation {name} survived the pins:\n{p.stdout[-2000:]}"
