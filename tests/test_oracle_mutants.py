"""The oracle pins must catch plausible mistakes: each case below plants one
mistake in a private copy of oracle.c, builds it on the CPU and checks that
at least one pin fails on it."""

import os
import shutil
import subprocess
import tempfile

import pytest

import oracle
from tests import test_oracle as pins
from tests import test_oracle_terms as term_pins

ORACLE_SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

CANDIDATE_PINS = [
    pins.test_h1_rectified_stereo_is_1d_range_query,
    pins.test_h1_per_keypoint_tolerance,
    pins.test_closed_boundary_on_integer_grid,
    pins.test_h2_forward_motion_closed_form,
    pins.test_h3_wraparound_worked_case,
    pins.test_i1_noiseless_true_matches_are_candidates,
    pins.test_i3_scaling_and_sign_of_F,
]
MATCH_PINS = [
    pins.test_canonical_fp32_distance_is_exactly_rounded_chain,
    pins.test_selection_orders_by_distance_then_index,
    pins.test_ratio_test,
    pins.test_hamming_against_numpy_bitcount,
    pins.test_h5_eps_beyond_diagonal_is_brute_force,
]

TERM_PINS = [
    term_pins.test_point_line_dist_wraparound_hand_values,
    term_pins.test_terms_on_integer_lines_are_exact,
    term_pins.test_terms_scalar_and_per_keypoint_eps,
    term_pins.test_desc_dist_f64_hand_cases,
    term_pins.test_desc_dist_f64_within_its_rounding_bound,
]

MUTANTS = {
    "dropped_c_term": ("*a = F[0] * x + F[1] * y + F[2];", "*a = F[0] * x + F[1] * y;"),
    "transposed_F": ("*b = F[3] * x + F[4] * y + F[5];", "*b = F[1] * x + F[4] * y + F[7];"),
    "open_boundary": ("return num <= rhs;", "return num < rhs;"),
    "wrong_sign": ("double num = fabs(a * x + b * y + c);",
                   "double num = fabs(a * x - b * y + c);"),
    "no_sqrt": ("double rhs = eps * sqrt(a * a + b * b);", "double rhs = eps * (a * a + b * b);"),
    "wrong_norm": ("double rhs = eps * sqrt(a * a + b * b);",
                   "double rhs = eps * sqrt(a * a + a * a);"),
    "degenerate_not_empty": ("int degen = (a == 0.0 && b == 0.0);", "int degen = 0;"),
    "diff_as_sum": ("float t = a[k] - b[k];", "float t = a[k] + b[k];"),
    "no_fma": ("acc = fmaf(t, t, acc);", "acc = acc + t * t;"),
    "tie_to_higher_j": ("return (p->j > q->j) - (p->j < q->j);",
                        "return (p->j < q->j) - (p->j > q->j);"),
    "ratio_not_squared": ("float thr = c->ratio * c->ratio;", "float thr = c->ratio;"),
    "hamming_and": ("h += popcount32(a[w] ^ b[w]);", "h += popcount32(a[w] & b[w]);"),
    "second_is_worst": ("float sd = k > 1 ? buf[1].d : INFINITY;",
                        "float sd = k > 1 ? buf[k - 1].d : INFINITY;"),
    # listed-pair helpers (Eq. 3 distance, both sides of Eq. 3-4, FP64 distance)
    "dist_no_sqrt": ("out[t] = num / sqrt(a * a + b * b);", "out[t] = num / (a * a + b * b);"),
    "dist_swapped_xy": ("double num = fabs(a * (double)kp2[2 * j] + b * (double)kp2[2 * j + 1] + c);",
                        "double num = fabs(a * (double)kp2[2 * j + 1] + b * (double)kp2[2 * j] + c);"),
    "terms_wrong_norm": ("rhs[t] = eps * sqrt(a * a + b * b);", "rhs[t] = eps * sqrt(a * a + b * a);"),
    "terms_wrong_sign": ("num[t] = fabs(a * (double)kp2[2 * j] + b * (double)kp2[2 * j + 1] + c);",
                         "num[t] = fabs(a * (double)kp2[2 * j] + b * (double)kp2[2 * j + 1] - c);"),
    "terms_scalar_eps_ignored": ("double eps = (double)(eps2 ? eps2[j] : eps_scalar);",
                                 "double eps = (double)(eps2 ? eps2[j] : 1.0f);"),
    "f64_diff_as_sum": ("double t = (double)a[k] - (double)b[k];",
                        "double t = (double)a[k] + (double)b[k];"),
    "f64_term_in_f32": ("acc += t * t;", "acc += (float)(t * t);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    old, new = MUTANTS[name]
    src = open(ORACLE_SRC).read()
    assert src.count(old) == 1, name
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mutant.c")
        with open(path, "w") as fh:
            fh.write(src.replace(old, new))
        so = oracle.build(force=True, src=path, out=os.path.join(d, "libmutant.so"))
        mutant = oracle.OracleLib(so)
        caught = []
        for pin in CANDIDATE_PINS + MATCH_PINS + TERM_PINS:
            try:
                pin(mutant)
            except (AssertionError, IndexError, ValueError):
                caught.append(pin.__name__)
        assert caught, f"no pin caught mutant {name}"
