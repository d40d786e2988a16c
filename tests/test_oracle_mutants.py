"""Planted mistakes in a copy of the oracle: every plausible slip in its
arithmetic (a dropped factor, a wrong exponent, a transposed operand, a
truncated series, a lost residual, a wrong charge or window bound) must make
at least one of the oracle's pins fail.

Each mutant is a text edit of ``adk_oracle.c`` written to a temporary folder,
compiled with the oracle's own build command and loaded as a separate copy of
the ``oracle`` module; the committed oracle and its library are not touched.
The pins run are the ones in ``test_oracle_rates.py``, ``test_oracle_chain.py``
and ``test_oracle_window.py``, called with fixed parameters.
"""
import importlib.util
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE_INIT = os.path.join(ROOT, "oracle", "__init__.py")
ORACLE_SRC = os.path.join(ROOT, "oracle", "adk_oracle.c")


def _load_path(name, path):
    spec = importlib.util.spec_from_file_location(name, path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


R = _load_path("pins_rates", os.path.join(HERE, "test_oracle_rates.py"))
C = _load_path("pins_chain", os.path.join(HERE, "test_oracle_chain.py"))
W = _load_path("pins_window", os.path.join(HERE, "test_oracle_window.py"))
A = _load_path("pins_adaptive", os.path.join(HERE, "test_oracle_adaptive.py"))

PINS = [
    ("hydrogen closed form", lambda o: R.test_hydrogen_closed_form(o, 100.0)),
    ("charge scaling law", lambda o: R.test_hydrogenic_scaling_law(o, 3, 1.7, 700.0)),
    ("projection ratio", lambda o: R.test_projection_ratio_closed_form(o, 2)),
    ("orbital factor", R.test_orbital_factor),
    ("field dependence", lambda o: R.test_field_dependence_at_noninteger_nstar(o, 40.74, 3, 1, 150.0, 900.0)),
    ("integer n* closed forms", lambda o: R.test_integer_nstar_closed_forms(o, 300.0)),
    ("hydrogen step", lambda o: R.test_hydrogen_step_closed_form(o, 100.0)),
    ("one level", lambda o: C.test_single_level_closed_form(o, 0.7)),
    ("two levels, Eq. (7)", lambda o: C.test_two_level_eq7(o, 0.4, 1.3)),
    ("brute-force expm", lambda o: C.test_mpmath_brute_force(o, 3)),
    ("chain invariants", lambda o: C.test_invariants(o, 3)),
    ("shift with fold", W.test_shift_folds_residual_and_moves_window),
    ("window = full chain", lambda o: W.test_window_equals_full_chain_when_it_covers_the_rest(o, 7, 7)),
    ("conservation over a pulse", W.test_conservation_and_nonnegativity_over_a_pulse),
    ("adaptive: zero tolerance = full chain", lambda o: A.test_zero_tolerance_is_the_full_chain(o, 7)),
    ("adaptive: fixed width = fixed window", lambda o: A.test_fixed_width_is_the_fixed_window(o, 3)),
    ("adaptive: leak bounds the full chain", lambda o: A.test_leak_bounds_what_the_full_chain_moves_past_the_top(o, 1e-6)),
    ("adaptive: leak closed forms", A.test_leak_closed_forms),
    ("adaptive: shift lowers the width", A.test_shift_lowers_the_width_and_keeps_the_top_level),
]

# (name, original text, planted text); the original must occur exactly once
MUTANTS = [
    ("power exponent without |m|", "2.0 * ns - am - 1.0", "2.0 * ns - 1.0"),
    ("tunnelling factor with (Q/n*)^2", "pow((double)Q / ns, 3.0)", "pow((double)Q / ns, 2.0)"),
    ("square-root factor without n*^3", "sqrt(3.0 * n3 * EL / (M_PI * Q3 * E_a))",
     "sqrt(3.0 * EL / (M_PI * Q3 * E_a))"),
    ("angular factor without n*", "(2.0 * M_PI * ns * pow(2.0, am)", "(2.0 * M_PI * pow(2.0, am)"),
    ("Q^2/(2 n*) instead of Q^2/(2 n*^2)", "(double)Q * Q / (2.0 * ns * ns)", "(double)Q * Q / (2.0 * ns)"),
    ("Stirling factor to the power n*", "pow(2.0 * M_E / ns, 2.0 * ns)", "pow(2.0 * M_E / ns, ns)"),
    ("Q instead of Q^2", "(double)Q * Q / (2.0 * ns * ns)", "(double)Q / (2.0 * ns * ns)"),
    ("e/n* instead of 2e/n*", "pow(2.0 * M_E / ns, 2.0 * ns)", "pow(M_E / ns, 2.0 * ns)"),
    ("l + 1 instead of 2l + 1", "(2.0 * l + 1.0) * orc_fact(l + am)", "(l + 1.0) * orc_fact(l + am)"),
    ("gain term transposed", "A[(i + 1) * n + i] = W[i] * dt;", "A[i * n + (i + 1)] = W[i] * dt;"),
    ("loss term sign", "A[i * n + i] = -W[i] * dt;", "A[i * n + i] = W[i] * dt;"),
    ("Taylor series cut at degree 3", "for (int k = 1; k <= 30; ++k)", "for (int k = 1; k <= 3; ++k)"),
    ("one squaring short", "for (int r = 0; r < s; ++r)", "for (int r = 1; r < s; ++r)"),
    ("shift drops the residual", "N[lo + 1] += N[lo];", "N[lo + 1] += 0.0;"),
    ("level k ionized at charge k", "W[k - lo] = orc_level_rate(U[k], k + 1,", "W[k - lo] = orc_level_rate(U[k], k + 2,"),
    ("window one level short", "const int top = lo + w < Z ? lo + w : Z;",
     "const int top = lo + w - 1 < Z ? lo + w - 1 : Z;"),
    ("adaptive: leak without the factorial", "L += term / orc_fact(t - s + 1);", "L += term;"),
    ("adaptive: leak misses the top rate", "for (int k = s; k <= t; ++k) term *= x[k];",
     "for (int k = s; k < t; ++k) term *= x[k];"),
    ("adaptive: widening test reversed", "while (top < room && !(orc_leak(N, x, top) <= tol)) ++top;",
     "while (top < room && (orc_leak(N, x, top) <= tol)) ++top;"),
    ("adaptive: width kept at a shift", "w = w > 0 ? w - 1 : 0;", "w = w > 0 ? w : 0;"),
    ("adaptive: top slot dropped", "pops[(int64_t)s * ncells + c] = s <= top ? N[s] : 0.0;",
     "pops[(int64_t)s * ncells + c] = s < top ? N[s] : 0.0;"),
]


def _mutant_oracle(tmpdir, idx, old, new):
    src = open(ORACLE_SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    csrc = os.path.join(tmpdir, f"mutant{idx}.c")
    with open(csrc, "w") as f:
        f.write(src.replace(old, new))
    mod = _load_path(f"oracle_mutant{idx}", ORACLE_INIT)
    mod._SRC = csrc
    mod._LIB = os.path.join(tmpdir, f"libmutant{idx}.so")
    mod._lib = None
    mod.build(force=True)
    return mod


def _failing_pins(orc):
    failed = []
    for name, pin in PINS:
        try:
            pin(orc)
        except AssertionError:
            failed.append(name)
    return failed


def test_unmutated_copy_passes_every_pin(tmp_path):
    """The harness itself: a copy with a no-op edit passes all pins, so a
    failure below comes from the planted mistake."""
    orc = _mutant_oracle(str(tmp_path), 0, "const double EL = fabs(E);", "const double EL = fabs(E) ;")
    assert _failing_pins(orc) == []


@pytest.mark.parametrize("name,old,new", MUTANTS)
def test_planted_mistake_is_caught(tmp_path, name, old, new):
    orc = _mutant_oracle(str(tmp_path), 1, old, new)
    failed = _failing_pins(orc)
    assert failed, f"no pin catches the planted mistake: {name}"


# The sub-cycled RK4 baseline's reference (oracle/subcycle.py), same idea:
# a mutated copy of the module text runs under the baseline's two pins.
SUBCYCLE_SRC = os.path.join(ROOT, "oracle", "subcycle.py")
S = _load_path("pins_subcycle", os.path.join(HERE, "test_oracle_subcycle.py"))

SUBCYCLE_MUTANTS = [
    ("RK4 weights 1, 1, 1, 1", "(h / 6.0) * (k1 + 2.0 * (k2 + k3) + k4)", "(h / 4.0) * (k1 + k2 + k3 + k4)"),
    ("second stage at the full substep", "y + 0.5 * h * k1", "y + h * k1"),
    ("top level leaks", "d[w] = x[w - 1] * y[w - 1]", "d[w] = x[w - 1] * y[w - 1] - x[w - 1] * y[w]"),
    ("rates not scaled by dt", "x[s, ok] = Wall[k[ok], np.nonzero(ok)[0]] * dt",
     "x[s, ok] = Wall[k[ok], np.nonzero(ok)[0]] * dt * 1.001"),
]


def _subcycle_copy(old, new):
    import types
    from oracle import mlp
    src = open(SUBCYCLE_SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    src = src.replace("from .mlp import window_shift\n", "").replace(old, new)
    mod = types.ModuleType("subcycle_mutant")
    mod.window_shift = mlp.window_shift
    exec(compile(src, "subcycle_mutant.py", "exec"), mod.__dict__)
    return mod


def _failing_subcycle_pins(orc, mod):
    saved = S.subcycle
    S.subcycle = mod
    failed = []
    try:
        for pin in (S.test_single_level_closed_form, S.test_conservation_and_fourth_order_convergence):
            try:
                pin(orc)
            except AssertionError:
                failed.append(pin.__name__)
    finally:
        S.subcycle = saved
    return failed


def test_unmutated_subcycle_copy_passes(orc):
    assert _failing_subcycle_pins(orc, _subcycle_copy("h = 1.0 / nsub", "h = 1.0 / nsub ")) == []


@pytest.mark.parametrize("name,old,new", SUBCYCLE_MUTANTS)
def test_planted_subcycle_mistake_is_caught(orc, name, old, new):
    assert _failing_subcycle_pins(orc, _subcycle_copy(old, new)), f"no pin catches: {name}"


# The surrogate network's reference (oracle/mlp.py) under its own pins.
MLP_SRC = os.path.join(ROOT, "oracle", "mlp.py")
M = _load_path("pins_mlp", os.path.join(HERE, "test_oracle_mlp.py"))

MLP_MUTANTS = [
    ("bfloat16 with 7 significant bits", "np.rint(m * 256.0) / 256.0", "np.rint(m * 128.0) / 128.0"),
    ("ReLU mask of the wrong layer", 'dz3 = (dz4 @ c["W4"]) * (c["h3"] > 0)', 'dz3 = (dz4 @ c["W4"]) * (c["h2"] > 0)'),
    ("weight gradient transposed", 'g["W2"] = dz2.T @ c["h1"]', 'g["W2"] = c["h1"].T @ dz2'),
    ("Adam without bias correction of m", "mh = m / (1.0 - beta1 ** t)", "mh = m"),
    ("band update drops the window top", "o[top] = N[top, c]", "o[top] = 0.0"),
    ("field feature not centred", "- 0.5 * (lE0 + lE1)) / (0.5 * (lE1 - lE0))", "- lE0) / (0.5 * (lE1 - lE0))"),
    ("stripped cells take the band", "use &= p < Z", "use &= p <= Z"),
    ("negligible-source test reversed", "negl = x[s] < NEGLIGIBLE_XDT if", "negl = x[s] > NEGLIGIBLE_XDT if"),
    ("field range open above", "(E <= rng.E_hi)", "(E <= 2 * rng.E_hi)"),
    ("band applied before the shift", "band = band_update(N, p, w, Z, cols, use)",
     "band = band_update(np.asarray(pops, np.float64), p, w, Z, cols, use)"),
]


def _mlp_copy(old, new):
    import sys
    import types
    src = open(MLP_SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    mod = types.ModuleType("mlp_mutant")
    sys.modules["mlp_mutant"] = mod  # dataclasses resolve annotations through sys.modules
    try:
        exec(compile(src.replace(old, new), "mlp_mutant.py", "exec"), mod.__dict__)
    finally:
        del sys.modules["mlp_mutant"]
    return mod


def _failing_mlp_pins(orc, mod):
    pins = [M.test_bf16_rounding, M.test_backward_matches_finite_differences,
            M.test_adam_first_step_and_bias_correction, M.test_softmax_invariants,
            lambda: M.test_weight_layout_out_in(True),
            lambda: M.test_band_update_with_exact_columns_is_the_step(orc, 3),
            M.test_features_map_the_trained_range_onto_the_unit_interval,
            lambda: M.test_surrogate_step_composition(orc)]
    saved = M.mlp
    M.mlp = mod
    failed = []
    try:
        for i, pin in enumerate(pins):
            try:
                pin()
            except AssertionError:
                failed.append(i)
    finally:
        M.mlp = saved
    return failed


def test_unmutated_mlp_copy_passes(orc):
    assert _failing_mlp_pins(orc, _mlp_copy("mh = m / (1.0 - beta1 ** t)", "mh = m / (1.0 - beta1 ** t) ")) == []


@pytest.mark.parametrize("name,old,new", MLP_MUTANTS)
def test_planted_mlp_mistake_is_caught(orc, name, old, new):
    assert _failing_mlp_pins(orc, _mlp_copy(old, new)), f"no pin catches: {name}"
