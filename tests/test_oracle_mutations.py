"""The pins catch plausible mistakes: each case below plants one mistake in a
copy of the oracle's C source (on the CPU), builds it, and requires at least
one pin from test_oracle_pins.py to fail against it.  Each mutant runs in a
child process, because a planted indexing mistake may also write out of
bounds; a crash of the child counts as caught."""
import json
import os
import subprocess
import sys
import tempfile

import pytest

import oracle
import test_oracle_pins as pins

MUTANTS = {
    "tie_axis_order_x_first": ("{2, 1, 0}", "{0, 1, 2}"),
    "tie_axis_order_y_first": ("{2, 1, 0}", "{1, 2, 0}"),
    "tie_derivative_sign": ("s[f] = sgn64(d1[f] - d0[f]);", "s[f] = sgn64(d0[f] - d1[f]);"),
    "Db_rows_transposed": ("out[1] = det3(a, c, d);", "out[1] = det3(c, a, d);"),
    "Dc_uses_wrong_vertex": ("out[2] = det3(a, b, d);", "out[2] = det3(a, b, c);"),
    "det_cofactor_sign": ("- r0[1] * (r1[0]", "+ r0[1] * (r1[0]"),
    "det_cofactor_index": ("r1[0] * r2[2] - r1[2] * r2[0]", "r1[0] * r2[2] - r1[2] * r2[1]"),
    "pattern_sign_swapped": ("(s[0] > 0 && s[1] < 0 && s[2] > 0 && s[3] < 0)",
                             "(s[0] > 0 && s[1] < 0 && s[2] < 0 && s[3] < 0)"),
    "only_first_pattern": ("||\n           (s[0] < 0 && s[1] > 0 && s[2] < 0 && s[3] > 0)", "&& 1"),
    "box_low_bound": ("lo[a] = ceil_div(mn - S[a], 2 * S[a]);", "lo[a] = ceil_div(mn + S[a], 2 * S[a]);"),
    "box_high_short": ("hi[a] = floor_div(mx - S[a], 2 * S[a]);", "hi[a] = floor_div(mx - 3 * S[a], 2 * S[a]);"),
    # (excluding centers on the box's max faces would be an equivalent
    # mutant: the perturbation pushes such centers outside anyway)
    "box_low_strict": ("lo[a] = ceil_div(mn - S[a], 2 * S[a]);",
                       "lo[a] = ceil_div(mn - S[a] + 1, 2 * S[a]);"),
    "floor_div_negative": ("if ((a % b != 0) && (a < 0)) q -= 1;", "if (a < 0) q -= 1;"),
    "center_wrong_axis": ("(2 * k + 1) * S[2]", "(2 * k + 1) * S[1]"),
    "column_index_wrong_dim": ("int64_t col = i * J->n[1] + j;", "int64_t col = i * J->n[0] + j;"),
    "half_pitch_wrong": ("S[a] = (LATTICE / 2) / J->n[a];", "S[a] = LATTICE / J->n[a];"),
    # the multithreaded split and merge (meshes of 4096 tets and more)
    "thread_range_end_short": ("J->t1 = nt * (t + 1) / nthreads;", "J->t1 = nt * (t + 1) / nthreads - 1;"),
    "thread_range_start_late": ("J->t0 = nt * t / nthreads;", "J->t0 = nt * t / nthreads + (t > 0);"),
    "merge_skips_thread_1": ("        if (t > 0) {\n            for (int64_t w = 0;",
                             "        if (t > 1) {\n            for (int64_t w = 0;"),
    "merge_skips_last_word": ("for (int64_t w = 0; w < nwords; ++w) words[w] |= priv[t][w];",
                              "for (int64_t w = 0; w + 1 < nwords; ++w) words[w] |= priv[t][w];"),
    "status_of_thread_0_only": ("if (jobs[t].status != ORACLE_OK) status = jobs[t].status;",
                                "if (t == 0 && jobs[t].status != ORACLE_OK) status = jobs[t].status;"),
    "snap_round_away": ("double r = nearbyint(t);", "double r = round(t);"),
    "snap_scale": ("t = t * 65536.0;", "t = t * 65535.0;"),
    "snap_range": ("if (r < (double)Q_LO || r > (double)Q_HI)", "if (r < (double)Q_LO - 1 || r > (double)Q_HI)"),
}


def run_pins(mod):
    """Run a cross-section of the pins; return the names of those that fail."""
    checks = [
        ("predicate_small", lambda: pins.test_predicate_matches_exact_barycentric(mod, 3, 4, 300)),
        ("predicate_large", lambda: pins.test_predicate_matches_exact_barycentric(mod, 1 << 17, 1 << 17, 60)),
        ("identity", lambda: pins.test_theorem1_identity_and_cramer(mod)),
        ("corner", lambda: [pins.test_corner_tets_closed_form(mod, M) for M in (2, 5)]),
        ("aligned", lambda: pins.test_aligned_lattice_exact_cover(mod, 4, 4, 2, 32)),
        ("full_cube", lambda: pins.test_full_jittered_cube_is_all_ones(mod, 5, 0.4, (16, 32, 64), 12)),
        ("brute", lambda: pins.test_aabb_culling_matches_brute_force(mod)),
        ("rationals", lambda: pins.test_whole_mesh_against_exact_rationals(mod)),
        ("translation", lambda: pins.test_translation_by_one_voxel(mod)),
        ("mt_full_cube", lambda: [pins.test_full_cube_multithreaded_is_all_ones(mod, t) for t in (2, 3, 7)]),
        ("mt_partition", lambda: pins.test_kept_and_complement_partition_multithreaded(mod, 2)),
        ("mt_status", lambda: [pins.test_multithreaded_index_error_is_reported(mod, w)
                               for w in ("first", "middle", "last")]),
        ("snap_exact", lambda: pins.test_snap_exact_cases(mod)),
        ("snap_range", lambda: pins.test_snap_range_and_nan(mod)),
    ]
    failed = []
    for name, fn in checks:
        try:
            fn()
        except (AssertionError, oracle.OracleError, ValueError, IndexError, pytest.fail.Exception):
            failed.append(name)
    return failed


def run_pins_in_child(lib_path):
    """Run the pins against the library at lib_path in a child process.
    Returns (failed pin names, child exit code)."""
    here = os.path.dirname(os.path.abspath(__file__))
    code = (
        "import json, sys\n"
        f"sys.path[:0] = [{here!r}, {os.path.dirname(here)!r}]\n"
        "import oracle, test_oracle_mutations as m\n"
        f"oracle.use_library({lib_path!r})\n"
        "print('PINS', json.dumps(m.run_pins(oracle)))\n"
    )
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    for line in r.stdout.splitlines():
        if line.startswith("PINS "):
            return json.loads(line[5:]), r.returncode
    return None, r.returncode


@pytest.fixture(scope="module")
def mutant_dir():
    with tempfile.TemporaryDirectory() as d:
        yield d


def test_unmutated_copy_passes_every_check(oracle_mod, mutant_dir):
    out = oracle.build(oracle.SRC, os.path.join(mutant_dir, "clean.so"))
    failed, rc = run_pins_in_child(out)
    assert rc == 0 and failed == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(oracle_mod, mutant_dir, name):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    path = os.path.join(mutant_dir, f"{name}.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    out = oracle.build(path, os.path.join(mutant_dir, f"{name}.so"))
    failed, rc = run_pins_in_child(out)
    assert failed is None or failed, f"no pin caught the planted mistake {name}"
    if failed is None:
        assert rc != 0  # the child crashed: caught
