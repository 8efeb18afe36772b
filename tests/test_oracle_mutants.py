"""The oracle's pins catch planted mistakes: each mutant below is the
oracle's C source with one plausible mistake, compiled on its own; the pins
of the function it touches, run against it in a fresh interpreter, must
fail.  (Equivalent mutants, such as ones that differ only on self loops,
which valid graphs lack, are left out.)"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "centra_oracle.c")

MUTANTS = {
    "kpath_start_not_excluded": ("    if (x == s) return 1;\n", "    if (x == s && 0) return 1;\n",
                                 "tests/test_oracle_kpaths.py"),
    "kpath_length_off_by_one": ("const uint32_t l = 1 + (uint32_t)orc_bounded(&st, kappa);",
                                "const uint32_t l = (uint32_t)orc_bounded(&st, kappa);", "tests/test_oracle_kpaths.py"),
    "kpath_visited_counted": ("            if (on_walk(w, s, h, len)) continue;\n            if (r == 0) {",
                              "            if (r == 0) {", "tests/test_oracle_kpaths.py"),
    "vc_d1_floor_log2_b": ("    *d1 = j + 1;", "    *d1 = j;", "tests/test_oracle_vc.py"),
    "vc_union_k_plus_1": ("*dk_union = (uint64_t)floor((double)k * log2((double)n));",
                          "*dk_union = (uint64_t)floor((double)(k + 1) * log2((double)n));", "tests/test_oracle_vc.py"),
    "vc_lemma_factor": ("*dk_lemma = (uint64_t)floor(2.0 * (double)(*d1)", "*dk_lemma = (uint64_t)floor(1.0 * (double)(*d1)",
                        "tests/test_oracle_vc.py"),
    "triangles_b_below_a": ("        if (b <= a) continue;\n        for (uint64_t f = e + 1",
                            "        if (b >= a) continue;\n        for (uint64_t f = e + 1", "tests/test_oracle_triangles.py"),
    "triangles_c_from_row_start": ("        for (uint64_t f = e + 1; f < g->row_ptr[a + 1]; f++) {",
                                   "        for (uint64_t f = g->row_ptr[a]; f < g->row_ptr[a + 1]; f++) {",
                                   "tests/test_oracle_triangles.py"),
    "triangles_no_bc_edge": ("            if (!adjacent(g, b, c)) continue;", "            if (!adjacent(g, a, c)) continue;",
                             "tests/test_oracle_triangles.py"),
    "triangles_stream_tag": ("        orc_stream_init(&st, seed, first + i, instance, 5);",
                             "        orc_stream_init(&st, seed, first + i, instance, 4);", "tests/test_oracle_triangles.py"),
    "greedy_ties_highest_id": ("            if (gain[u] > gain[best]) best = u;", "            if (gain[u] >= gain[best]) best = u;",
                               "tests/test_oracle_cover_mcera.py"),
    "topk_negatives_kept": ("            if (x > 0) col[npos++] = x;", "            col[npos++] = x;",
                            "tests/test_oracle_cover_mcera.py"),
    "philox_round_constant": ("const uint64_t M0 = 0xD2E7470EE14C6C93ULL,", "const uint64_t M0 = 0xD2E7470EE14C6C95ULL,",
                              "tests/test_oracle_rng.py"),
    "lemire_no_rejection": ("        while (low < threshold) {", "        while (low < threshold && 0) {",
                            "tests/test_oracle_rng.py"),
    "pair_may_repeat_s": ("    uint32_t t = tp + (tp >= s ? 1u : 0u);", "    uint32_t t = tp + (tp > s ? 1u : 0u);",
                          "tests/test_oracle_sampler.py"),
    "counts_shift_one_short": ("        uint32_t shift = bl > c_bits ? bl - c_bits : 0;",
                               "        uint32_t shift = bl > c_bits + 1 ? bl - c_bits - 1 : 0;", "tests/test_oracle_sampler.py"),
    "count_bits_out_degree": ("    const uint32_t *ip = in_ptr(g);\n    uint64_t dmax = 0;",
                              "    const uint32_t *ip = g->row_ptr;\n    uint64_t dmax = 0;", "tests/test_oracle_sampler.py"),
    "graph_check_self_loops_allowed": ("            if (idx[e] == u) return -6;", "            if (idx[e] == u && 0) return -6;",
                                       "tests/test_oracle_sampler.py"),
    "graph_check_reverse_sources_unchecked": ("                if (!found) return -21;", "                if (!found && 0) return -21;",
                                              "tests/test_oracle_sampler.py"),
    "bidir_pair_may_repeat_s": ("    uint32_t t = tp >= s ? tp + 1u : tp;", "    uint32_t t = tp > s ? tp + 1u : tp;",
                                "tests/test_oracle_bidir.py"),
    "bidir_weight_forward_only": ("    return (unsigned __int128)F->sigma[v] * B->sigma[v];",
                                  "    return (unsigned __int128)F->sigma[v];", "tests/test_oracle_bidir.py"),
    "bidir_walk_wrong_side": ("            cur = walk_step(B, g->row_ptr, g->col_idx, cur, B->level[cur] - 1, &st);",
                              "            cur = walk_step(F, g->row_ptr, g->col_idx, cur, B->level[cur] - 1, &st);",
                              "tests/test_oracle_bidir.py"),
    "hedge_one_sided": ("    const double eta = sqrt((log(2.0) + orc_log_sets(n, k) + log(1.0 / delta_i)) / (2.0 * (double)m));",
                        "    const double eta = sqrt((orc_log_sets(n, k) + log(1.0 / delta_i)) / (2.0 * (double)m));",
                        "tests/test_oracle_bound.py"),
    "counts_no_clamp": ("            b->sigma[b->visited[q]] = x ? x : 1;", "            b->sigma[b->visited[q]] = x;",
                        "tests/test_oracle_sampler.py"),
    "schedule_root_term": ("const double inv_y = (sqrt(2.0 * L) + sqrt(2.0 * L + 4.0 * L * T / 3.0)) / (2.0 * T);",
                           "const double inv_y = (sqrt(2.0 * L) + sqrt(2.0 * L + 4.0 * L * T)) / (2.0 * T);",
                           "tests/test_oracle_schedule.py"),
    "bound_last_term_dropped": ("sqrt(2.0 * L * (nu + 4.0 * r) / md) + L / (3.0 * md);", "sqrt(2.0 * L * (nu + 4.0 * r) / md);",
                                "tests/test_oracle_bound.py"),
}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_fail_on_mutant(name, tmp_path):
    old, new, pins = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "the mutation site moved"
    c_file, lib = tmp_path / "mutant.c", tmp_path / "mutant.so"
    c_file.write_text(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-I", os.path.join(ROOT, "oracle"),
                           str(c_file), "-o", str(lib), "-lm"])
    code = ("import sys, oracle; oracle._LIB = sys.argv[1]; import pytest; "
            "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', sys.argv[2]]))")
    env = dict(os.environ, PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", code, str(lib), pins], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode not in (0, 5), f"{name} survived:\n{r.stdout[-2000:]}"
