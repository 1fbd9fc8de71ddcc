"""Mutation check of the oracle's pins (CPU only).

Each mutant is a copy of oracle/hgp_oracle.cpp with one plausible slip built
in: a flipped sign, a wrong window, a reversed tie-break, the wrong pointer
moved.  The copy is compiled to a temporary library and the oracle's pin
tests are run against it in a child process (HGP_ORACLE_LIB selects the
library); every mutant must make at least one of them fail.  A mutant that
survives means a reading of the paper that nothing pins.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hgp_oracle.cpp")
PIN_TESTS = ["tests/test_oracle_readings.py", "tests/test_oracle_refine.py", "tests/test_oracle_coarsen.py",
             "tests/test_oracle_driver.py", "tests/test_oracle_eval.py", "tests/test_oracle_greedy.py"]

# name -> (exact text in the oracle, replacement); each text occurs once.
MUTANTS = {
    # chain rounds (Reading R16)
    "grade_penalty_sign": ("i64 G = mv[j].gain * 10000000LL -", "i64 G = mv[j].gain * 10000000LL +"),
    "grade_size_weight": ("(10 * std::llabs(nw[a] - nw[b]) + std::llabs((i64)nin[a] - nin[b]))",
                          "(std::llabs(nw[a] - nw[b]) + 10 * std::llabs((i64)nin[a] - nin[b]))"),
    "window_of_one": ("const int kWindow = 256,", "const int kWindow = 1,"),
    "window_of_257": ("const int kWindow = 256,", "const int kWindow = 257,"),
    "successor_tie_smaller_id": ("(G == bG && b > mv[bj].n)", "(G == bG && b < mv[bj].n)"),
    "window_keeps_linked_moves": ("                if (pred[j] != -1) continue;\n", ""),
    "acceptance_tie_smaller_id": ("(propG[i] == propG[a] && mv[i].n > mv[a].n)",
                                  "(propG[i] == propG[a] && mv[i].n < mv[a].n)"),
    # linearisation and ranking (Reading R17)
    "cycle_starts_at_largest": ("if (mv[cyc[q]].n < mv[cyc[at]].n) at = q;",
                                "if (mv[cyc[q]].n > mv[cyc[at]].n) at = q;"),
    "rank_ties_larger_first_id": ("return a.gain != b.gain ? a.gain > b.gain : a.first < b.first;",
                                  "return a.gain != b.gain ? a.gain > b.gain : a.first > b.first;"),
    # moves sort (Reading R15)
    "moves_sort_id_desc": ("        if (a.gain != b.gain) return a.gain > b.gain;\n        return a.n < b.n;",
                           "        if (a.gain != b.gain) return a.gain > b.gain;\n        return a.n > b.n;"),
    # isolated pairing (Reading R8)
    "isolated_skip_moves_i": ("        } else {\n            j--;\n        }", "        } else {\n            i++;\n        }"),
    # noise cap (Reading R3)
    "noise_cap_counts_single_pins": ("if (g.card(e) >= 2) { sum += tnorm(g, e); cnt += 1; }",
                                     "if (g.card(e) >= 1) { sum += tnorm(g, e); cnt += 1; }"),
    # k-way seating (Reading R21)
    "kway_heaviest_first": ("return pw[a] != pw[b] ? pw[a] < pw[b] : a < b;",
                            "return pw[a] != pw[b] ? pw[a] > pw[b] : a < b;"),
    # greedy matching of the ablation (Reading R28)
    "greedy_skips_root_pairs": ("        if (paired[r]) match[r] = target[r];\n", ""),
    "greedy_tie_smaller_id": ("(sc[c] == sc[bc] && c > bc)", "(sc[c] == sc[bc] && c < bc)"),
    "greedy_lowest_score": ("if (bc < 0 || sc[c] > sc[bc] ||", "if (bc < 0 || sc[c] < sc[bc] ||"),
    # early exit (Reading R25)
    "early_exit_leaves_level": ("                if (rep < prm.Theta / 2) rep = prm.Theta / 2 - 1;\n                else break;",
                                "                break;"),
}


def _build(name, tmpdir):
    with open(SRC) as f:
        text = f.read()
    old, new = MUTANTS[name]
    assert text.count(old) == 1, "mutation site of %s not found exactly once" % name
    src = os.path.join(tmpdir, name + ".cpp")
    lib = os.path.join(tmpdir, name + ".so")
    with open(src, "w") as f:
        f.write(text.replace(old, new))
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-o", lib, src])
    return lib


def _run_pins(lib):
    env = dict(os.environ, HGP_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
                       + PIN_TESTS, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def test_every_mutant_fails_a_pin(tmp_path):
    names = sorted(MUTANTS)
    with cf.ThreadPoolExecutor(4) as ex:
        libs = dict(zip(names, ex.map(lambda n: _build(n, str(tmp_path)), names)))
        results = dict(zip(names, ex.map(lambda n: _run_pins(libs[n]), names)))
    survivors = [n for n, (rc, _) in results.items() if rc == 0]
    errors = [n for n, (rc, out) in results.items() if rc not in (0, 1)]
    assert not errors, {n: results[n][1] for n in errors}
    assert not survivors, "mutants not caught by any pin: %s" % survivors


def test_unmutated_copy_passes(tmp_path):
    # The harness itself: the same build and run on the unchanged source pass.
    lib = os.path.join(str(tmp_path), "same.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-o", lib, SRC])
    rc, out = _run_pins(lib)
    assert rc == 0, out
