"""Planted mistakes in a copy of the oracle must be caught by the pins.

Each mutant is qw_oracle.c with one plausible error (a sign, an index, a
transposed operand, a dropped term, an off-by-one window), compiled into a
temporary library; the oracle module is pointed at it and a battery of the
pin tests runs.  At least one pin must fail for every mutant.  CPU only.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1003_3779_amd import inputs
from tests import test_oracle_pins as P
from tests import test_oracle_rbl as RB
from tests import test_oracle_graph as GR

SRC = os.path.join(os.path.dirname(oracle.__file__), "qw_oracle.c")

MUTANTS = {
    "shift_sign": ("int64_t sx = wrap(x - disp[2 * c], Lx);", "int64_t sx = wrap(x + disp[2 * c], Lx);"),
    "shift_y_index": ("int64_t sy = wrap(y - disp[2 * c + 1], Ly);", "int64_t sy = wrap(y - disp[2 * c], Ly);"),
    "coin_transposed": ("acc = c_add(acc, c_mul(C[c * d + cp], src[cp]));",
                        "acc = c_add(acc, c_mul(C[cp * d + c], src[cp]));"),
    "dropped_term": ("for (cp = 0; cp < d; cp++)\n                    acc = c_add(acc, c_mul(C[c * d + cp], src[cp]));",
                     "for (cp = 0; cp < d - 1; cp++)\n                    acc = c_add(acc, c_mul(C[c * d + cp], src[cp]));"),
    "cmul_sign": ("r.im = a.re * b.im + a.im * b.re;", "r.im = a.re * b.im - a.im * b.re;"),
    "su2_sign": ("C[2] = c_make(-ec.re * st, ec.im * st);", "C[2] = c_make(ec.re * st, ec.im * st);"),
    "su2_conj": ("C[3] = c_make(ep.re * ct, -ep.im * ct);", "C[3] = c_make(ep.re * ct, ep.im * ct);"),
    "grover_weight": ("C[a * d + b] = c_make(2.0 / d - (a == b ? 1.0 : 0.0), 0.0);",
                      "C[a * d + b] = c_make(1.0 / d - (a == b ? 1.0 : 0.0), 0.0);"),
    "hh_index": ("h[a >> 1][b >> 1] * h[a & 1][b & 1]", "h[a >> 1][b & 1] * h[a & 1][b >> 1]"),
    "prob_drops_imag": ("s += re * re + im * im;", "s += re * re;"),
    "window_radius": ("int64_t r = windowed ? t0 + s + 1 : -1;", "int64_t r = windowed ? t0 + s : -1;"),
    "inverse_no_conj": ("c_mul(c_conj(C[cp * d + c]), a[(sy * Lx + sx) * d + cp])",
                        "c_mul(C[cp * d + c], a[(sy * Lx + sx) * d + cp])"),
    "inverse_shift_sign": ("int64_t sx = wrap(x + disp[2 * cp], Lx);", "int64_t sx = wrap(x - disp[2 * cp], Lx);"),
    "bin_left_offset": ("int64_t offl = -(h - b) * w + k;", "int64_t offl = -(h - b) * w + k + 1;"),
    "rbl_link_owner": ("int64_t lx = positive[c] ? sx : x, ly = positive[c] ? sy : y;",
                       "int64_t lx = x, ly = y;"),
    "rbl_reflect_same_component": ("b[(y * Lx + x) * d + c] = phi[(y * Lx + x) * d + opp[c]];",
                                   "b[(y * Lx + x) * d + c] = phi[(y * Lx + x) * d + c];"),
    "philox_multiplier": ("const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;",
                          "const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D55u;"),
    "philox_key_schedule": ("if (r > 0) { k0 += W0; k1 += W1; }", "if (r > 1) { k0 += W0; k1 += W1; }"),
    "rbl_step_counter": ("link_broken(lx, ly, Lx, pair[c], (uint64_t)(step0 + s), realization, seed, thr)",
                         "link_broken(lx, ly, Lx, pair[c], (uint64_t)step0, realization, seed, thr)"),
    "rbl_pair_word": ("return (uint64_t)o[2 * (ay & 1) + pair] < thr;", "return (uint64_t)o[2 * (ay & 1)] < thr;"),
    "rbl_row_word": ("return (uint64_t)o[2 * (ay & 1) + pair] < thr;", "return (uint64_t)o[pair] < thr;"),
    "rbl_group_column": ("uint64_t g = (uint64_t)((ay >> 1) * Lx + ax);", "uint64_t g = (uint64_t)((ay >> 1) * Lx);"),
    "wall_edge_test": ("int edge = walls && (rx < 0 || rx >= Lx || ry < 0 || ry >= Ly);",
                       "int edge = walls && (rx < 0 || rx > Lx || ry < 0 || ry >= Ly);"),
    "graph_no_shift": ("b[rev[k0 + i]] = acc;   /* the shift: to the other end of the edge */",
                       "b[k0 + i] = acc;"),
    "graph_grover_weight": ("out[a * d + b] = c_make(2.0 / d - (a == b ? 1.0 : 0.0), 0.0);",
                            "out[a * d + b] = c_make(1.0 / d - (a == b ? 1.0 : 0.0), 0.0);"),
    "graph_fourier_sign": ("out[a * d + b] = c_make(s * cos(t), s * sin(t));",
                           "out[a * d + b] = c_make(s * cos(t), -s * sin(t));"),
    "graph_pairing": ("if (seen == occ) { found = j; break; }", "if (seen == 0) { found = j; break; }"),
    "graph_coin_transposed": ("for (j = 0; j < d; j++) acc = c_add(acc, c_mul(C[i * d + j], a[k0 + j]));",
                              "for (j = 0; j < d; j++) acc = c_add(acc, c_mul(C[j * d + i], a[k0 + j]));"),
    "wall_reflects_wrong_side": ("int64_t rx = x - disp[2 * c], ry = y - disp[2 * c + 1];",
                                 "int64_t rx = x + disp[2 * c], ry = y + disp[2 * c + 1];"),
}

ONE = lambda rng: inputs.haar_unitary(rng, 2)          # noqa: E731
FOUR = lambda rng: inputs.haar_unitary(rng, 4)         # noqa: E731

BATTERY = [
    lambda: P.test_dense_matrix_power_ring(5, "haar", ONE),
    lambda: P.test_dense_matrix_power_ring(8, "su2", P.COIN_CASES_1D[1][1]),
    lambda: P.test_dense_matrix_power_torus((4, 5), "PAIR", "haar", FOUR),
    lambda: P.test_dense_matrix_power_torus((4, 5), "DIAG", "grover", P.COIN_CASES_2D[0][1]),
    lambda: P.test_dense_matrix_power_torus((4, 5), "EQ8", "hh", P.COIN_CASES_2D[1][1]),
    lambda: P.test_dense_matrix_power_windowed_start(),
    lambda: P.test_path_sum_ring(5),
    lambda: P.test_hh_is_kron(),
    lambda: P.test_su2_is_unitary_and_special(),
    lambda: P.test_norm_conserved_torus(),
    lambda: P.test_site_parity_and_light_cone("PAIR"),
    lambda: P.test_exact_reversal("PAIR"),
    lambda: P.test_inverse_matches_matrix_inverse(),
    lambda: P.test_binning_symmetric_and_complete(),
    lambda: RB.test_philox_known_answers(),
    lambda: RB.test_no_broken_link_is_the_plain_walk("PAIR"),
    lambda: RB.test_every_link_broken_freezes_the_walker("EQ8"),
    lambda: RB.test_each_step_is_a_reflecting_shift("DIAG"),
    lambda: RB.test_each_step_is_a_reflecting_shift("RING"),
    lambda: RB.test_reflection_frequency_matches_p(),
    lambda: RB.test_steps_compose("PAIR"),
    lambda: RB.test_links_of_one_site_are_independent(),
    lambda: RB.test_links_of_neighbouring_sites_are_independent(),
    lambda: RB.test_walls_two_site_segment_by_hand(),
    lambda: RB.test_walls_segment_never_wraps(),
    lambda: RB.test_walls_reflect_exactly_at_the_edge("PAIR"),
    lambda: GR.test_dense_matrix_power_random_graphs(oracle.DENSE, 1),
    lambda: GR.test_dense_matrix_power_random_graphs(oracle.FOURIER, 2),
    lambda: GR.test_grover_keeps_the_uniform_arc_state(),
    lambda: GR.test_unitary_on_random_graphs_and_bad_input(),
]


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of {name} not found exactly once"
    c = tmp_path / f"{name}.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", "-std=c99", "-D_GNU_SOURCE", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                           str(c), "-o", str(so), "-lm"])
    return str(so)


def _failures():
    n = 0
    for check in BATTERY:
        try:
            check()
        except (AssertionError, ValueError, RuntimeError):
            n += 1
    return n


def test_unmutated_oracle_passes_the_battery():
    assert _failures() == 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    lib = oracle._open(_build(tmp_path, name, old, new))
    monkeypatch.setattr(oracle, "_lib", lib)
    assert _failures() >= 1, f"no pin caught the planted mistake {name}"
