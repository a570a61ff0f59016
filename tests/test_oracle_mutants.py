"""Mutation check of the oracle pins.

Each mutant is a copy of the oracle's C source with one plausible slip planted
(a flipped sign, a dropped term, a swapped index or operand, a wrong tie
rule).  The copy is compiled on the CPU into a temporary library and the pins
of ``test_oracle_pins.py`` are run against it: at least one pin must fail for
every mutant.  This shows that the pins fix the oracle, rather than the
oracle fixing itself.
"""
import os
import subprocess
import tempfile

import pytest

import oracle
import test_oracle_paper_workload as PW
import test_oracle_pins as P
import test_oracle_stats as ST
import workloads as W

SRC = os.path.join(os.path.dirname(oracle.__file__), "pic_oracle.c")

MUTANTS = {
    "peano_parity_of_own_axis": ("int64_t e = (others % 2) ? 2 - digit : digit;",
                                 "int64_t e = (seen[k] % 2) ? 2 - digit : digit;"),
    "peano_never_complements": ("int64_t e = (others % 2) ? 2 - digit : digit;",
                                "int64_t e = digit;"),
    "child_slot_axes_swapped": ("slot += ((o->I[k] / p3) % 3) * m; m *= 3;",
                                "slot = slot * 3 + ((o->I[k] / p3) % 3); m *= 3;"),
    "owner_ties_round_down": ("if (2.0 * off >= (double)o->s) c |= 1 << k;",
                              "if (2.0 * off > (double)o->s) c |= 1 << k;"),
    "weights_f_g_swapped": ("double wc = (c & 1) ? f[0] : g[0];",
                            "double wc = (c & 1) ? g[0] : f[0];"),
    "weights_drop_axis1": ("for (int k = 1; k < t->dim; ++k) wc = wc *",
                           "for (int k = 2; k < t->dim; ++k) wc = wc *"),
    "gather_drops_corner1": ("for (int c = 1; c < nc; ++c) e = e + w[c] * Ej[vt[c]];",
                             "for (int c = 2; c < nc; ++c) e = e + w[c] * Ej[vt[c]];"),
    "gather_wrong_component": ("const double *Ej = E + (int64_t)j * t->n_vtx;",
                               "const double *Ej = E;"),
    "push_kick_sign": ("double vj = v[j * n + p] + qmdt * e;",
                       "double vj = v[j * n + p] - qmdt * e;"),
    "push_drift_old_velocity": ("qmdt * e;\n            double xj = x[j * n + p] + vj * dt;",
                                "qmdt * e;\n            double xj = x[j * n + p] + v[j * n + p] * dt;"),
    "wrap_keeps_one": ("if (xj == 1.0) xj = 0.0;\n            v[j * n + p] = vj;", "v[j * n + p] = vj;"),
    "rebin_arrivals_first": ("fill_stay[b] = acc;\n        fill_move[b] = acc + cnt_stay[b];",
                             "fill_move[b] = acc;\n        fill_stay[b] = acc + cnt_move[b];"),
    "deposit_corner_transposed": ("double term = qp * w[c];", "double term = qp * w[c ^ 1];"),
    "pidt_key_unshifted": ("J[k] = (b[k] * s + (t->S - 1) / 2) % t->S;",
                           "J[k] = (b[k] * s) % t->S;"),
    "leaf_key_span_one_axis": ("uint64_t span = (uint64_t)ipow3(t->dim * (t->L - n->level));",
                               "uint64_t span = (uint64_t)ipow3(t->L - n->level);"),
    "vertex_order_axis1_fastest": ("for (int k = 0; k < dim; ++k) { r += a[k] * m; m *= n; }",
                                   "for (int k = dim - 1; k >= 0; --k) { r += a[k] * m; m *= n; }"),
    "stats_lifts_from_new_level": ("const int lifts = l0 - m;", "const int lifts = l1 - m;"),
    "stats_dual_cells_unshifted": ("a[k] = (bk + (nl - 1) / 2) % nl;", "a[k] = bk % nl;"),
    "stats_tunnel_not_periodic": ("if (t->S - d < d) d = t->S - d;", ""),
    "reflect_at_zero_keeps_velocity": ("xj = -xj;\n                vj = -vj;", "xj = -xj;"),
    "reflect_at_one_wraps": ("xj = 2.0 - xj;", "xj = xj - 1.0;"),
    "landing_on_one_not_moved_inside": ("if (xj == 1.0) xj = nextafter(1.0, 0.0);", ""),
    "stream_drift_sign": ("double xj = x[j * n + p] + vj * dt;\n            if (boundary == 0) {",
                          "double xj = x[j * n + p] - vj * dt;\n            if (boundary == 0) {"),
}

# fast pins, cheapest first; a mutant must make at least one of them fail
PINS = [
    lambda: P.test_peano_matches_textbook_level1_order(),
    lambda: P.test_peano_is_a_face_continuous_bijection(2, 2),
    lambda: P.test_peano_prefix_property(2, 1),
    lambda: P.test_tree_tables_match_geometry(W.disc_tree(2, 2, 4)),
    lambda: P.test_dual_cells_nest_along_the_curve(2, 2),
    lambda: P.test_particle_on_a_vertex_sits_entirely_there(),
    lambda: P.test_push_kicks_against_the_field_for_negative_charge(),
    lambda: P.test_wrap_never_returns_one(),
    lambda: P.test_weights_exact_and_partition_of_unity(W.disc_tree(2, 2, 4)),
    lambda: P.test_gather_reproduces_constant_and_linear_fields(),
    lambda: P.test_deposit_exact_small_and_adjoint_to_gather(),
    lambda: P.test_free_streaming_matches_closed_form(),
    lambda: P.test_locate_matches_brute_force(W.disc_tree(2, 2, 4)),
    lambda: P.test_step_satisfies_theorems_and_order("small_adaptive", 0),
    lambda: P.test_step_satisfies_theorems_and_order("small_adaptive", 1),
    lambda: ST.test_hand_computed_lifts_on_a_9x9_tree(),
    lambda: ST.test_stats_match_the_lift_mechanism("disc2d_1_3", oracle.PIT, 4),
    lambda: ST.test_stats_match_the_lift_mechanism("reg2d_L2", oracle.PIDT, 4),
    lambda: PW.test_reflection_hand_cases(),
    lambda: PW.test_reflecting_stream_is_the_folded_straight_line(),
]


@pytest.fixture(scope="module")
def workdir():
    with tempfile.TemporaryDirectory() as d:
        yield d


def _compile(src_text, out):
    c = out + ".c"
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", out, c, "-lm"])


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, workdir):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    so = os.path.join(workdir, f"mut_{name}.so")
    _compile(src.replace(old, new), so)
    saved = oracle._lib
    oracle._lib = oracle.load(so)
    caught = None
    try:
        for i, pin in enumerate(PINS):
            try:
                pin()
            except (AssertionError, ValueError) as e:
                caught = (i, type(e).__name__)
                break
    finally:
        oracle._lib = saved
    assert caught is not None, f"no pin catches mutant {name}"


# Slips in the adaptation rule (Python): the function's source with one
# change, run against the adaptation pins.
ADAPT_MUTANTS = {
    "refine_at_ppc": ("count.get((l, a), 0) > ppc", "count.get((l, a), 0) >= ppc"),
    "coarsen_only_below_ppc": (") <= ppc:", ") < ppc:"),
    "root_coarsened": ("for l in range(1, L):", "for l in range(0, L):"),
    "no_level_cap": ("if l < max_level and count", "if count"),
    "coarsen_despite_refined_child": ("if any(kk in refined[l + 1] for kk in kids):\n                continue", ""),
}
ADAPT_PINS = [PW.test_overfull_leaf_is_refined_once, PW.test_underfull_children_are_coarsened,
              PW.test_cell_with_a_refined_child_is_not_coarsened,
              lambda adapt: PW.test_repeated_adaptation_reaches_the_ppc_fixed_point(2, "subbox", adapt=adapt)]


@pytest.mark.parametrize("name", sorted(ADAPT_MUTANTS))
def test_pins_catch_adapt_mutant(name):
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(oracle.adapt))
    old, new = ADAPT_MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    ns = dict(vars(oracle))
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), ns)
    caught = False
    for pin in ADAPT_PINS:
        try:
            pin(adapt=ns["adapt"])
        except (AssertionError, ValueError, pytest.fail.Exception):
            caught = True
            break
    assert caught, f"no pin catches mutant {name}"


VMAX_MUTANTS = {
    "pidt_from_own_leaf_only": ("per_leaf = per_bin[lv[\"pidt\"]].max(axis=1)", "np.maximum.at(per_leaf, leaf, speed)"),
    "leaves_only_no_ancestors": ("for up in range(l, -1, -1):", "for up in range(l, l - 1, -1):"),
    "predicate_strict": ("out[l] * dt <= 1.0 / 3 ** l", "out[l] * dt < 0.5 / 3 ** l"),
    "speed_from_axis0": ("speed = np.max(np.abs(np.asarray(v, np.float64)), axis=0)",
                         "speed = np.abs(np.asarray(v, np.float64))[0]"),
}


@pytest.mark.parametrize("name", sorted(VMAX_MUTANTS))
def test_pins_catch_vmax_mutant(name):
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(oracle.vmax_cells))
    old, new = VMAX_MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    ns = dict(vars(oracle))
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), ns)
    saved = oracle.vmax_cells
    oracle.vmax_cells = ns["vmax_cells"]
    caught = False
    try:
        for pin in (PW.test_vmax_hand_case, lambda: PW.test_vmax_of_a_cell_is_the_max_over_its_subtree_particles(0),
                    lambda: PW.test_vmax_of_a_cell_is_the_max_over_its_subtree_particles(1)):
            try:
                pin()
            except (AssertionError, ValueError):
                caught = True
                break
    finally:
        oracle.vmax_cells = saved
    assert caught, f"no pin catches mutant {name}"
