"""Planted-mistake check of the oracle pins (CPU only).

Each case compiles a copy of the oracle's C source with one plausible mistake
planted (a dropped term, a wrong sign, index or scale) and asserts that at
least one of the pins in ``test_oracle_pins`` rejects it.  The shipped oracle
is never modified; the mutated copies live in a temporary directory.
"""
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "fdoracle.c")

MUTATIONS = {
    "drop_centre": ("double s = c[0] * at3(g, u, i0, i1, i2);", "double s = 0.0 * at3(g, u, i0, i1, i2);"),
    "neighbour_sign": ("s += c[k] * (at3", "s -= c[k] * (at3"),
    "wrong_axis_spacing": ("total += s / (g->h[a] * g->h[a]);", "total += s / (g->h[2] * g->h[2]);"),
    "weight_off_by_one": ("r *= (double)(M - k + j) / (double)(M + j);", "r *= (double)(M - k + j) / (double)(M + j + 1);"),
    "transposed_index": ("return u[(i0 * g->n[1] + i1) * g->n[2] + i2];", "return u[(i1 * g->n[0] + i0) * g->n[2] + i2];"),
    "update_centre_factor": ("+ 4.0 * m[i] * u_cur[i] +", "+ 2.0 * m[i] * u_cur[i] +"),
    "damping_sign": ("u_new[i] = ((tcse - 2.0 * m[i]) * u_prev[i]", "u_new[i] = ((-tcse - 2.0 * m[i]) * u_prev[i]"),
    "source_scale": ("spread(&w.sp[s], 2.0 * dt2 * amp[n * p->ns + s]", "spread(&w.sp[s], dt2 * amp[n * p->ns + s]"),
    "receiver_old_level": ("sample(&w.rp[r], u_new);", "sample(&w.rp[r], u_cur);"),
    "injection_unscaled": ("u[i] += s->w[j] * a / (dt * damp[i] + 2.0 * m[i]);", "u[i] += s->w[j] * a;"),
    "adjoint_source_sample_unscaled": ("= 2.0 * dt2 * sample(&w->sp[s], l0);", "= dt2 * sample(&w->sp[s], l0);"),
    "interp_fraction_swapped": ("w *= bit ? f[a] : 1.0 - f[a];", "w *= bit ? 1.0 - f[a] : f[a];"),
    "interp_sample_unweighted": ("acc += s->w[j] * u[s->idx[j]];", "acc += u[s->idx[j]];"),
    "interp_spread_unweighted": ("u[i] += s->w[j] * a / (dt * damp[i] + 2.0 * m[i]);", "u[i] += a / (dt * damp[i] + 2.0 * m[i]);"),
    "interp_cell_above": ("base[a + g->first] = i;", "base[a + g->first] = i > 0 ? i - 1 : i;"),
    "imaging_first_difference": ("(uk[i] - 2.0 * uk1[i] + uk2[i])", "(uk[i] - uk1[i])"),
    "born_source_sign": ("du[2][i] += -2.0 * dm[i] * (u[2][i]", "du[2][i] += 2.0 * dm[i] * (u[2][i]"),
    "born_first_difference": ("(u[2][i] - 2.0 * u[1][i] + u[0][i])", "(u[2][i] - u[1][i])"),
    "born_dm_power": ("dm[i] = -2.0 * dv[i] / (p->v[i] * p->v[i] * p->v[i]);", "dm[i] = -2.0 * dv[i] / (p->v[i] * p->v[i]);"),
    "sinc_window_radius": ("double t = d / (double)r;", "double t = d / (double)(r + 1);"),
    "sinc_node_shift": ("lo[ax] = i0 - r + 1;", "lo[ax] = i0 - r;"),
    "sinc_distance_sign": ("ksinc((double)node - x, r);", "ksinc(x - (double)node + 0.25, r);"),
    "sinc_bessel_term": ("term *= q / ((double)j * (double)j);", "term *= q / (double)j;"),
    "sponge_off_by_one": ("if (i < L) delta = (double)(L - i);", "if (i < L) delta = (double)(L - i - 1);"),
    "dt_squared_missing": ("double dt2 = dt * dt;\n#pragma omp parallel for schedule(static)\n    for (int64_t i0 = 0; i0 < g->n[0]; ++i0)\n        for (int64_t i1 = 0; i1 < g->n[1]; ++i1)\n            for (int64_t i2 = 0; i2 < g->n[2]; ++i2) {\n                int64_t i = (i0 * g->n[1] + i1) * g->n[2] + i2;\n                double tcse",
                           "double dt2 = dt;\n#pragma omp parallel for schedule(static)\n    for (int64_t i0 = 0; i0 < g->n[0]; ++i0)\n        for (int64_t i1 = 0; i1 < g->n[1]; ++i1)\n            for (int64_t i2 = 0; i2 < g->n[2]; ++i2) {\n                int64_t i = (i0 * g->n[1] + i1) * g->n[2] + i2;\n                double tcse"),
}


def _checks():
    """The pins run against a mutated library; each returns normally when it passes."""
    yield lambda: pins.test_weights_reproduce_paper_printed_constants()
    for so in (4, 8):
        yield lambda so=so: pins.test_weights_match_taylor_derivation(so)
    yield lambda: pins.test_laplacian_matches_dense_kronecker_sum((9, 6), 4)
    yield lambda: pins.test_laplacian_matches_dense_kronecker_sum((6, 5, 7), 8)
    yield lambda: pins.test_plane_wave_follows_discrete_dispersion((70, 64), 4, 9)
    yield lambda: pins.test_energy_balance_with_sponge()
    yield lambda: pins.test_sponge_reading_hand_values()
    for case in pins.CASES[1:3]:
        yield lambda case=case: pins.test_forward_and_adjoint_equal_dense_space_time_solve(*case)
    yield lambda: pins.test_gradient_equals_complex_step_of_dense_system((6, 5), 4, 6, 1)
    yield lambda: pins.test_first_step_injection_and_receiver_sampling()
    yield lambda: pins.test_offgrid_receivers_read_multilinear_fields_exactly(4)
    yield lambda: pins.test_offgrid_source_spreads_unit_mass_at_its_position((4.25, 5.5, 6.75))
    yield lambda: pins.test_offgrid_dot_product_fp64((40, 36))
    yield lambda: pins.test_born_is_the_derivative_of_the_forward_map(False)
    for r in (1, 4):
        yield lambda r=r: pins.test_sinc_weights_are_the_kaiser_windowed_sinc(r)
    yield lambda: pins.test_sinc_at_grid_nodes_is_the_node_itself(4)
    yield lambda: pins.test_sinc_receiver_reads_band_limited_waves(4, 3 * 1.2e-3)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_planted_mistake(name, tmp_path, monkeypatch):
    old, new = MUTATIONS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor for {name} not unique"
    src = tmp_path / "mut.c"
    src.write_text(text.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", str(lib), str(src), "-lm"])
    monkeypatch.setattr(oracle, "_LIB", str(lib))
    monkeypatch.setattr(oracle, "_SRC", str(src))
    monkeypatch.setattr(oracle, "_lib", None)
    caught = 0
    for chk in _checks():
        try:
            chk()
        except (AssertionError, ValueError, FloatingPointError):
            caught += 1
    monkeypatch.setattr(oracle, "_lib", None)
    assert caught > 0, f"no pin rejects the planted mistake {name}"
