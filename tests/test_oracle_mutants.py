"""Plant plausible mistakes in a copy of the oracle and check the pins fail.

Each mutant is a one-line change to lsort_oracle.c (a dropped term, a wrong
sign or index, a transposed operand).  The copy is compiled to a temporary
library and the pin suite is run against it in a subprocess; every mutant
must make at least one pin fail.  CPU only.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lsort_oracle.c")

MUTANTS = {
    "knot_counts_own_copies": ("M->y[k] = (double)B / (double)M->mfin;",
                               "M->y[k] = (double)(B + d) / (double)M->mfin;"),
    "segment_starts_at_mid_rank": ("M->ylo[k] = (double)(2 * (B + d) - 1) / m2;", "M->ylo[k] = M->ym[k];"),
    "segment_upper_clamp_dropped": ("    if (F > M->yhi[j])\n        F = M->yhi[j];\n", ""),
    "slope_transposed": ("double sl = (yh - M->ylo[k]) / (Xh - M->X[k]);",
                         "double sl = (Xh - M->X[k]) / (yh - M->ylo[k]);"),
    "root_from_xmax": ("double t = (root_coord(x) - M->r0) * M->rs;",
                       "double t = (root_coord(x) - root_coord(M->xmax)) * M->rs;"),
    "knot_is_leaf_minimum": ("if (e - a > best[k]) {", "if (best[k] == 0) {"),
    "no_previous_knot": ("uint32_t j = (x >= M->X[k]) ? k : model_prev(M, k);", "uint32_t j = k;"),
    "level_offset_sign": ("int64_t q = (int64_t)v - B->offset;", "int64_t q = (int64_t)v + B->offset;"),
    "tail_flush_skips_last": ("for (uint32_t i = 0; i < f && rc == ORC_OK; ++i) {\n        uint32_t s = fsz[i];",
                              "for (uint32_t i = 0; i + 1 < f && rc == ORC_OK; ++i) {\n        uint32_t s = fsz[i];"),
    "defrag_cursor_not_advanced": ("        cur[b] += s;\n        r += s;", "        r += s;"),
    "sample_counter_off_by_one": ("uint64_t z = seed + (t + 1u) * 0x9e3779b97f4a7c15ull;",
                                  "uint64_t z = seed + t * 0x9e3779b97f4a7c15ull;"),
    "counting_sort_forward_walk": ("for (uint64_t k = n; k-- > 0;)\n        T[--K[P[k]]] = A[k];",
                                   "for (uint64_t k = 0; k < n; ++k)\n        T[--K[P[k]]] = A[k];"),
    "counting_sort_slot_from_parent": ("double v = (model_F(M, ord_value(A[k], dtype)) * scale - offset) * (double)n;",
                                       "double v = (model_F(M, ord_value(A[k], dtype)) * scale) * (double)n;"),
    "homogeneous_compares_neighbour_sign": ("if (A[k] != A[0])", "if ((A[k] >> 1) != (A[0] >> 1))"),
    "msd_digit_reversed": ("return (uint32_t)((o >> B->shift) & B->mask);",
                           "return (uint32_t)((~o >> B->shift) & B->mask);"),
    "msd_shift_one_too_high": ("B->shift = d + 1 - bits;", "B->shift = d + 2 - bits;"),
    "msd_shift_one_too_low": ("B->shift = d + 1 - bits;", "B->shift = d - bits;"),
    "msd_fallback_never_taken": ("if (rc == ORC_OK && 8 * biggest > 7 * n) {",
                                 "if (rc == ORC_OK && 8 * biggest > 8 * n) {"),
    "local_split_at_level1_scale": ("bucketer_t BM = {BK_MODEL, M, C->dtype, (double)C->f, 0, C->f, 0, 0};",
                                    "bucketer_t BM = {BK_MODEL, M, C->dtype, (double)C->f * C->f, 0, C->f, 0, 0};"),
    "local_split_buckets_reversed": ("        bucketer_t BM = {BK_MODEL, M, C->dtype, (double)C->f, 0, C->f, 0, 0};",
                                     "        bucketer_t BM = {BK_MODEL, M, C->dtype, -(double)C->f, -(int64_t)C->f + 1, C->f, 0, 0};"),
    "f64_ord_sign_flip": ("return (b >> 63) ? ~b : (b | 0x8000000000000000ull);",
                          "return (b >> 63) ? (b & 0x7fffffffffffffffull) : (b | 0x8000000000000000ull);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not found: " + name
    mut = tmp_path / "lsort_oracle.c"
    mut.write_text(src.replace(old, new))
    hdr = os.path.join(ROOT, "oracle", "lsort_oracle.h")
    (tmp_path / "lsort_oracle.h").write_text(open(hdr).read())
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o",
                    str(lib), str(mut), "-lm"], check=True)
    env = dict(os.environ, LSORT_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "--timeout", "120", os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "planted mistake %s survived every pin:\n%s" % (name, r.stdout[-2000:])
