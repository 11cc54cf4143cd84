"""Plants plausible mistakes in copies of the oracle source and checks that the
pins catch every one of them (on the CPU; the real oracle is untouched)."""
import os
import subprocess

import pytest

import oracle
import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, original text, replacement, count) -- count = occurrences to replace (1 = first)
MUTANTS = [
    ("no_source_term", "const int64_t s = m + Ie[x] + Is[x];", "const int64_t s = m + Ie[x];", 1),
    ("no_relu", "out[x] = s > 0 ? s : 0;", "out[x] = s;", 1),
    ("pool_4_neighbourhood", "if (v > m) m = v;", "if (v > m && (dr == 0 || dc == 0)) m = v;", 1),
    ("padding_one", "? 0                       /* zero padding */", "? 1                       /* zero padding */", 1),
    ("start_from_zero", "memcpy(a, Is, sizeof(int64_t) * (size_t)N);", "memset(a, 0, sizeof(int64_t) * (size_t)N);", 1),
    ("one_layer_too_many", "for (n = 0; n < max_layers; ++n) {", "for (n = 0; n <= max_layers; ++n) {", 1),
    ("auto_one_past", "if (same_support(N, a, b)) break;",
     "if (same_support(N, a, b)) { int64_t *t = a; a = b; b = t; ++n; break; }", 1),
    ("obstacles_ignored", "Ie[i] = occ[i] ? -ORACLE_MAXINT : 0;", "Ie[i] = 0;", 1),
    ("obstacle_bias_small", "Ie[i] = occ[i] ? -ORACLE_MAXINT : 0;", "Ie[i] = occ[i] ? -1 : 0;", 1),
    ("bfs_4_neighbourhood", "if (occ[y] || dist[y] >= 0) continue;",
     "if (occ[y] || dist[y] >= 0 || (NB_DR[k] != 0 && NB_DC[k] != 0)) continue;", 1),
    ("bfs_step_two", "dist[y] = dist[x] + 1;", "dist[y] = dist[x] + 2;", 1),
    ("walk_last_max_wins", "if (O[y] > best_v) { best_v = O[y]; best = y; }",
     "if (O[y] >= best_v) { best_v = O[y]; best = y; }", 1),
    ("walk_reversed_order",
     "static const int NB_DR[8] = {-1, -1, -1, 0, 0, 1, 1, 1};\nstatic const int NB_DC[8] = {-1, 0, 1, -1, 1, -1, 0, 1};",
     "static const int NB_DR[8] = {1, 1, 1, 0, 0, -1, -1, -1};\nstatic const int NB_DC[8] = {1, 0, -1, 1, -1, 1, 0, -1};", 1),
    ("walk_column_major_order",
     "static const int NB_DR[8] = {-1, -1, -1, 0, 0, 1, 1, 1};\nstatic const int NB_DC[8] = {-1, 0, 1, -1, 1, -1, 0, 1};",
     "static const int NB_DR[8] = {-1, 0, 1, -1, 1, -1, 0, 1};\nstatic const int NB_DC[8] = {-1, -1, -1, 0, 0, 1, 1, 1};", 1),
    ("walk_drops_target_cell", "        cells[total++] = (int32_t)p;\n        while",
     "        while", 1),
    ("walk_zero_activity_allowed", "if (O[p] <= 0) { len[t] = -1; continue; }",
     "if (O[p] < 0) { len[t] = -1; continue; }", 1),
    ("random_ties_always_first", "p = cand[oracle_tie_hash(seed, (uint64_t)t, (uint64_t)steps) % (uint64_t)n_cand];",
     "p = cand[0];", 1),
    ("tie_hash_wrong_shift", "z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;", "z = (z ^ (z >> 26)) * 0x94d049bb133111ebULL;", 1),
    ("euclid_no_straightening", "if (dr == 1 && dc == 1) continue;   /* drop buf[i] */", "if (0) continue;", 1),
]


def _build_mutant(tmp_path, name, old, new, count):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutant {name}: pattern not found"
    mutated = src.replace(old, new, count)
    c = tmp_path / f"{name}.c"
    c.write_text(mutated)
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-o", str(so), str(c)])
    return oracle.Oracle(str(so))


@pytest.mark.parametrize("mutant", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(mutant, tmp_path):
    name, old, new, count = mutant
    o = _build_mutant(tmp_path, name, old, new, count)
    caught = []
    for check in pins.ALL_CHECKS:
        kwargs = {"four_by_four": False} if check is pins.check_bfs_exhaustive else {}
        try:
            check(o, **kwargs)
        except (AssertionError, RuntimeError, IndexError, ValueError):
            caught.append(check.__name__)
            break
    assert caught, f"no pin caught mutant {name}"
