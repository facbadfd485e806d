"""The oracle's pins must reject plausible mistakes. Each case plants one
mistake in a private copy of the oracle's C source (on the CPU, in a temporary
directory), builds it, and runs the pin suite against it in a child process;
the suite must fail for every mutant."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "spmm_oracle.c")

MUTANTS = {
    "drop_last_term": ("p < rowptr[i + 1]; ++p) {\n        double a = or_load(vals, p, vdt);\n        int64_t r",
                       "p + 1 < rowptr[i + 1]; ++p) {\n        double a = or_load(vals, p, vdt);\n        int64_t r"),
    "wrong_sign": ("if (absval) b = fabs(b);\n            out[c] += a * b;",
                   "if (absval) b = fabs(b);\n            out[c] -= a * b;"),
    "semiring_min_as_max": ("case 1: out[c] = fmin(out[c], a + b);", "case 1: out[c] = fmax(out[c], a + b);"),
    "semiring_identity": ("semiring == 1 ? INFINITY : -INFINITY", "semiring == 1 ? -INFINITY : -INFINITY"),
    "semiring_times_as_plus": ("default: out[c] = fmax(out[c], a * b);", "default: out[c] = fmax(out[c], a + b);"),
    "transposed_B": ("double b = or_load(B, r * ldb + c, bdt);\n            if (absval) b = fabs(b);\n            out[c]",
                     "double b = or_load(B, c * ldb + r, bdt);\n            if (absval) b = fabs(b);\n            out[c]"),
    "abs_dropped": ("if (absval) b = fabs(b);\n            out[c]", "out[c]"),
    "merge_tie_to_nnz": ("rowptr[i + 1] <= j)", "rowptr[i + 1] < j)"),
    "search_off_by_one": ("+ mid < d)", "+ mid <= d)"),
    "transpose_index": ("at_colind[q] = (int32_t)i;", "at_colind[q] = (int32_t)colind[p];"),
    "sddmm_row_index": ("double g = or_load(dC, i * ldc + c, cdt);\n                double b",
                        "double g = or_load(dC, r * ldc + c, cdt);\n                double b"),
    "spmm_t_target": ("double* dst = dB + (int64_t)colind[p] * n;", "double* dst = dB + i * n;"),
    "nz_search_strict": ("if ((int64_t)rowptr[mid + 1] <= j)", "if ((int64_t)rowptr[mid + 1] < j)"),
    "nz_first_piece_searched": ("for (int64_t p = 1; p <= P; ++p) {", "for (int64_t p = 0; p <= P; ++p) {"),
    "nz_parts_floor": ("int64_t P = (nnz + W - 1) / W;", "int64_t P = nnz / W;"),
    "heuristic_le": ("d < 9.35 ? 1 : 0", "d <= 9.35 ? 1 : 0"),
    "f16_exponent": ("e - 25", "e - 24"),
    "bf16_shift": ("<< 16;", "<< 15;"),
}

BATTERY = ["test_worked_example", "test_spmm_matches_dense_gemm", "test_identity_permutation",
           "test_row_sum", "test_transpose_vs_scipy", "test_merge_walk_invariants",
           "test_merge_closed_forms", "test_heuristic_table", "test_bf16_and_f16_decoders",
           "test_gradients_euler", "test_spmm_t_and_sddmm_vs_dense", "test_semirings_brute_force",
           "test_min_plus_bellman", "test_nz_partition"]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor for {name} not unique"
    src = tmp_path / "mutant.c"
    src.write_text(text.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    str(src), "-o", str(lib), "-lm"], check=True)
    env = dict(os.environ, ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py"), "-k", " or ".join(BATTERY)],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
