"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check
that the pin suite rejects every one of them."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dc_oracle.c")

MUTANTS = {
    "own-community total keeps i": ("return two_m * e - ki * (own ? aX - ki : aX);",
                                    "return two_m * e - ki * aX;"),
    "ties to the larger label": ("(s == bs && X < best)", "(s == bs && X > best)"),
    "self-loop counted in e": ("    if (v == i) continue;\n    int32_t X = C[v];",
                               "    int32_t X = C[v];"),
    "numerator without 2m": ("return two_m * I - S;", "return I - S;"),
    "guard inverted": ("size[best] == 1 && best > c", "size[best] == 1 && best < c"),
    "no revert of a losing sweep": ("if (dN < 0) break; /* revert", "if (0) break; /* revert"),
    "level 0 ignores R": ("level == 0 ? active0 : all", "all"),
    "Alg. 2 without gain2 test": ("if (g1 >= g2 && g1 > 0) {", "if (g1 > 0) {"),
    "Alg. 2 forgets Gamma(i)": ("      R[jstar] = 1;\n      for (int64_t e = g->off[i]; e < g->off[i + 1]; ++e) R[g->col[e]] = 1;",
                                "      R[jstar] = 1;"),
    "Alg. 2 forgets C(j*)": ("      cflag[cj] = 1;", "      (void)cj;"),
    "coarsening drops the diagonal": ("          int32_t Y = rank[C[g->col[e]]];\n",
                                      "          int32_t Y = rank[C[g->col[e]]];\n          if (Y == r) continue;\n"),
    "deletion rule off": ("    if (d != C[i]) {\n      if (info) info->del_accepted++;",
                          "    if (0) {\n      if (info) info->del_accepted++;"),
}

# mistakes in the screener-sample code, caught by its own pins
SCREENER = "test_oracle_screener.py"
MUTANTS.update({
    "replaced pair counted twice": ("        if (p > 0 && pairs[p] == pairs[p - 1]) continue;\n", "", SCREENER),
    "labels from the screened set only": ("level_sweeps(g, two_m, Tthr, Cl, all,",
                                          "level_sweeps(g, two_m, Tthr, Cl, Rds,", SCREENER),
    "touched set misses neighbours": (
        "    T[v] = 1;\n    for (int64_t e = g->off[v]; e < g->off[v + 1]; ++e) T[g->col[e]] = 1;",
        "    T[v] = 1;", SCREENER),
    "degree feature scale": ("x[0] = (double)k / ((double)k + 16.0);",
                             "x[0] = (double)k / ((double)k + 8.0);", SCREENER),
    "gain feature not scaled by k": (
        "x[4] = (k > 0 && raw[4] != ORC_NO_GAIN) ? (double)raw[4] / (double)(two_m * k) : -3.0;",
        "x[4] = (k > 0 && raw[4] != ORC_NO_GAIN) ? (double)raw[4] / (double)two_m : -3.0;", SCREENER),
    "second best keeps the own community": ("      if (X == c) continue;\n      int64_t sc = score(two_m, ag->acc[X], k[i], a[X], 0);",
                                            "      int64_t sc = score(two_m, ag->acc[X], k[i], a[X], 0);", SCREENER),
})


# mistakes in the cascade-aware screening, caught by its pins
CASCADE = "test_oracle_cascade.py"
MUTANTS.update({
    "cascade candidates outside C(i)": ("      if (v != i && C[v] == C[i]) cand[v] = 1;",
                                         "      if (v != i && C[v] != C[i]) cand[v] = 1;", CASCADE),
    "cascade threshold flipped": ("    if (lhs >= rhs) {", "    if (lhs <= rhs) {", CASCADE),
    "cascade forgets Gamma(v)": (
        "      R[v] = 1;\n      for (int64_t e = g->off[v]; e < g->off[v + 1]; ++e) R[g->col[e]] = 1;\n    }\n  }\n  free(cand);",
        "      R[v] = 1;\n    }\n  }\n  free(cand);", CASCADE),
    "cascade best includes the own community": (
        "      if (X == c) continue;\n      int64_t sX = score(",
        "      int64_t sX = score(", CASCADE),
})


# mistakes in the smart local moving levels (dSLM), caught by their pins
SLM = "test_oracle_slm.py"
MUTANTS.update({
    "SLM refinement starts from the communities": (
        "    for (int32_t u = 0; u < cur.n; ++u) Rf[u] = u;\n",
        "    for (int32_t u = 0; u < cur.n; ++u) Rf[u] = C[u];\n", SLM),
    "SLM refinement crosses communities": (
        "      if (C[g->col[e]] == C[u]) nnz++;", "      nnz++;", SLM),
    "SLM refinement weights from the subgraph": (
        "(void)level_sweeps(&sub, two_m, T, Rf, all, opt, level, tr, &oom, k, 1);",
        "(void)level_sweeps(&sub, two_m, T, Rf, all, opt, level, tr, &oom, NULL, 1);", SLM),
    "SLM next level from singletons": (
        "    for (int32_t u = 0; u < cur.n; ++u) Cn[rank[Rf[u]]] = first[C[u]];",
        "    for (int32_t u = 0; u < cur.n; ++u) Cn[rank[Rf[u]]] = rank[Rf[u]];", SLM),
    "SLM compaction by the unrefined communities": (
        "    if (!coarsen(&cur, Rf, rank, &nxt)) {", "    if (!coarsen(&cur, C, rank, &nxt)) {", SLM),
    "SLM level 0 ignores R": ("    const uint8_t* act = (level > 0) ? all : active0;",
                              "    const uint8_t* act = all;", SLM),
})


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_planted_mistake(name, tmp_path):
    old, new, *target = MUTANTS[name]
    target = target[0] if target else "test_oracle_pins.py"
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name!r} not unique"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", "-I", os.path.join(ROOT, "oracle"),
                    "-o", str(so), str(mut)], check=True)
    env = dict(os.environ, DC_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", target)],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins did not catch mutant {name!r}:\n{r.stdout[-2000:]}"
