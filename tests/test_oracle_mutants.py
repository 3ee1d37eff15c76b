"""Plant plausible mistakes in copies of the oracle (on the CPU) and check that
each one fails at least one pin: the pins are chosen to catch a dropped term,
a wrong sign, a wrong index, a transposed operand or a wrong bit order."""

import os
import subprocess

import pytest

from oracle_pins import ALL_PINS

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "oracle.c")


def _energy_f64_body(src):
    a = src.index("double oracle_energy_f64(")
    b = src.index("int64_t oracle_energy_i64(")
    return a, b


def _in_energy_f64(old, new):
    def f(src):
        a, b = _energy_f64_body(src)
        body = src[a:b]
        assert old in body, old
        return src[:a] + body.replace(old, new) + src[b:]
    return f


def _first(old, new, nth=0):
    def f(src):
        idx = -1
        for _ in range(nth + 1):
            idx = src.index(old, idx + 1)
        return src[:idx] + new + src[idx + len(old):]
    return f


MUTANTS = {
    "drop_field_term": _in_energy_f64("e -= h[i] * si;", "(void)0;"),
    "drop_field_term_int": _first("e -= h[i] * si;", "(void)0;", nth=1),
    "coupling_sign": _in_energy_f64("e -= J[(size_t)i * N + j] * si * sj;",
                                    "e += J[(size_t)i * N + j] * si * sj;"),
    "field_sign": _in_energy_f64("e -= h[i] * si;", "e += h[i] * si;"),
    "transposed_J": _in_energy_f64("J[(size_t)i * N + j] * si * sj",
                                   "J[(size_t)j * N + i] * si * sj"),
    "reversed_bit_order": _in_energy_f64("(mask >> i)", "(mask >> (N - 1 - i))"),
    "spin_convention": _in_energy_f64("? 1.0 : -1.0", "? -1.0 : 1.0"),
    "diag_in_sum": _in_energy_f64("for (int j = i + 1; j < N; ++j) {",
                                  "for (int j = i; j < N; ++j) {"),
    "tie_break_reversed": _first("(x.e == y.e && x.m < y.m); }",
                                 "(x.e == y.e && x.m > y.m); }"),
    "heap_keeps_one_less": _first("if (*n < S) {", "if (*n < S - 1) {"),
    "thread_slice_gap": _first("uint64_t b = a + span / T + (t < (int)(span % T) ? 1 : 0);",
                               "uint64_t b = a + span / T - (t == 1 ? 1 : 0);"),
    "logz_missing_shift": _first("logz[b] = -beta[b] * e0 + log(Z);", "logz[b] = log(Z);"),
    "logz_weight_sign": _first("exp(-beta[b] * (e - e0))", "exp(-beta[b] * (e0 - e))"),
    "moment_sign": _first("ms[(size_t)b * N + i] += w * s[i];",
                          "ms[(size_t)b * N + i] -= w * s[i];"),
    "pair_moment_index": _first("mss[((size_t)b * N + i) * N + j] += w * s[i] * s[j];",
                                "mss[((size_t)b * N + i) * N + j] += w * s[i] * s[i];"),
    "grad_missing_beta": _first("g[b] * beta[b] * mss", "g[b] * mss"),
    "qubo_a_factor": _first("4.0 * J[(size_t)i * N + j]", "2.0 * J[(size_t)i * N + j]"),
    "dos_bin_offset": _first("int64_t k = oracle_energy_i64(N, J, h, m) - e_min;",
                             "int64_t k = oracle_energy_i64(N, J, h, m) - e_min + 1;"),
    "dos_thread_slice": _first("uint64_t b = a + span / T + (t < (int)(span % T) ? 1 : 0);",
                               "uint64_t b = a + span / T;", nth=2),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(orc, name, tmp_path):
    src = open(SRC).read()
    mutated = MUTANTS[name](src)
    assert mutated != src
    c = tmp_path / "oracle_mut.c"
    so = tmp_path / "liboracle_mut.so"
    c.write_text(mutated)
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-std=c11", "-o", str(so), str(c), "-lm"])
    failed = []
    with orc.swapped_library(str(so)):
        for pin in ALL_PINS:
            try:
                pin(orc)
            except Exception:  # noqa: BLE001 - any failure counts as caught
                failed.append(pin.__name__)
    assert failed, "planted mistake %r passed every pin" % name
