"""The oracle's pins catch plausible mistakes.  Each case plants one mistake
(a wrong sign or index, a dropped term, a transposed operand, a wrong
constant) in a copy of one oracle module's source, makes every oracle and
pin-test module use the mutant's functions, runs the pins of that part of
the oracle and requires at least one of them to fail.  CPU only; the
oracle's own files are never modified."""
import importlib
import sys

import pytest

import test_oracle_cell_ode as T_cell
import test_oracle_emrkc as T_emrkc
import test_oracle_fem as T_fem
import test_oracle_imexrl as T_imex
import test_oracle_models as T_models
import test_oracle_mrkc as T_mrkc
import test_oracle_powiter as T_pow
import test_oracle_rkc as T_rkc
import test_oracle_variants as T_var
from oracle.ionic import HH

# a planted mistake may overflow or divide by zero on its way to failing a pin
pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _mutant(modname, old, new, nth=None):
    """A fresh module built from `modname`'s source with `old` replaced by
    `new`: `old` must occur exactly once, or nth picks its occurrence."""
    mod = importlib.import_module(modname)
    src = open(mod.__file__).read()
    if nth is None:
        assert src.count(old) == 1, (modname, old)
        src = src.replace(old, new)
    else:
        at = -1
        for _ in range(nth + 1):
            at = src.index(old, at + 1)
        src = src[:at] + new + src[at + len(old):]
    m = type(mod)(modname)
    m.__package__ = mod.__package__
    m.__file__ = mod.__file__
    exec(compile(src, mod.__file__ + " [mutant]", "exec"), m.__dict__)
    return mod, m


def _install(monkeypatch, mod, mutant):
    """Every reference that an oracle or pin-test module holds to a function
    or class defined in `mod` now points at the mutant's."""
    originals = {name: obj for name, obj in vars(mod).items()
                 if callable(obj) and getattr(obj, "__module__", None) == mod.__name__}
    for m in list(sys.modules.values()):
        mn = getattr(m, "__name__", "") or ""
        if not (mn.startswith("oracle") or mn.startswith("test_oracle") or mn == "gpu_util"):
            continue
        for attr, val in list(vars(m).items()):
            for name, obj in originals.items():
                if val is obj:
                    monkeypatch.setattr(m, attr, getattr(mutant, name))


def _some_pin_fails(pins):
    failed = []
    for pin in pins:
        try:
            pin()
        except Exception as e:  # an assertion, or the mutant breaking outright
            failed.append((getattr(pin, "__name__", "pin"), type(e).__name__))
    return failed


# (id, module, text, planted mistake, pins of that part of the oracle)
CASES = [
    ("rkc_kappa_sign", "oracle.rkc", "kappa[j] = -b[j] / b[j - 2]", "kappa[j] = b[j] / b[j - 2]",
     [lambda: T_rkc.test_coeffs_against_closed_form_chebyshev(5), lambda: T_rkc.test_nu_plus_kappa_is_one(5)]),
    ("rkc_omega1_inverted", "oracle.rkc", "w1 = T[s] / dT[s]", "w1 = dT[s] / T[s]",
     [lambda: T_rkc.test_coeffs_against_closed_form_chebyshev(5),
      lambda: T_rkc.test_rkc_iteration_linear_is_chebyshev_polynomial(6)]),
    ("rkc_dT_dropped_term", "oracle.rkc", "dT[j] = 2.0 * T[j - 1] + 2.0 * x * dT[j - 1] - dT[j - 2]",
     "dT[j] = 2.0 * x * dT[j - 1] - dT[j - 2]",
     [lambda: T_rkc.test_coeffs_against_closed_form_chebyshev(5)]),
    ("rkc_stage_time_index", "oracle.rkc", "f(t + c[j - 1] * dt, g_prev)", "f(t + c[j] * dt, g_prev)",
     [T_rkc.test_rkc_stage_times]),
    ("rkc_stages_floor", "oracle.rkc", "int(math.ceil(math.sqrt(dt * rho / beta)))",
     "int(math.floor(math.sqrt(dt * rho / beta)))",
     [T_rkc.test_get_stages_random_bracket, lambda: T_rkc.test_get_stages_bracket(3)]),
    ("emrkc_exp_sign", "oracle.emrkc", "return y + np.expm1(eta * lam) * (y - yinf)",
     "return y + np.expm1(-eta * lam) * (y - yinf)",
     [T_emrkc.test_exponential_euler_exact_for_frozen_rates, T_emrkc.test_scalar_test_equation_closed_form]),
    ("emrkc_force_from_yE", "oracle.emrkc", "u_eta = rkc_iteration(t, yE, eta, f_u, m, eps)\n    return (u_eta - y) / eta",
     "u_eta = rkc_iteration(t, yE, eta, f_u, m, eps)\n    return (u_eta - yE) / eta",
     [T_emrkc.test_scalar_test_equation_closed_form, lambda: T_emrkc.test_linear_model_on_cosine_mode(1)]),
    ("emrkc_fS_frozen_at_y", "oracle.emrkc", "fS_frozen = prob.f_S(t, yE)", "fS_frozen = prob.f_S(t, y)",
     [T_emrkc.test_scalar_test_equation_closed_form]),
    ("emrkc_eta_factor", "oracle.emrkc", "eta = 2.0 * dt / ls", "eta = dt / ls",
     [T_emrkc.test_stage_counts_c1, T_emrkc.test_scalar_test_equation_closed_form]),
    ("fem_q1_axis_index", "oracle.fem", "dk = (1.0 if c[k] else -1.0) / h[k]", "dk = (1.0 if c[k] else -1.0) / h[0]",
     [lambda: T_fem.test_q1_invariants_and_tensor_form((5, 4), (0.25, 1 / 3), (0.1, 0.1))]),
    ("fem_p1_element_transposed_gradients", "oracle.fem", "G = np.vstack([-Binv.sum(axis=0), Binv])",
     "G = np.vstack([-Binv.T.sum(axis=0), Binv.T])",
     [T_fem.test_p1_single_reference_tet, T_fem.test_p1_skewed_tet_against_barycentric_interpolation]),
    ("fem_p1_assembly_transposed_gradients", "oracle.fem",
     "G = np.concatenate([-Binv.sum(axis=1, keepdims=True), Binv], axis=1)",
     "G = np.concatenate([-Binv.sum(axis=2, keepdims=True).transpose(0, 2, 1), Binv.transpose(0, 2, 1)], axis=1)",
     [T_fem.test_p1_mesh_invariants_and_patch_test, T_fem.test_p1_skewed_tet_against_barycentric_interpolation]),
    ("fem_p1_mass_constant", "oracle.fem", "Me = vol / 20.0 * (np.ones((4, 4)) + np.eye(4))",
     "Me = vol / 10.0 * (np.ones((4, 4)) + np.eye(4))",
     [T_fem.test_p1_single_reference_tet, T_fem.test_p1_mesh_invariants_and_patch_test]),
    ("monodomain_chi_dropped", "oracle.monodomain", "(self.A @ V) / (self.chi * self.Cm * self.ML)",
     "(self.A @ V) / (self.Cm * self.ML)",
     [T_pow.test_rho_F_converges_to_closed_form_max_eigenvalue, lambda: T_emrkc.test_linear_model_on_cosine_mode(1)]),
    ("monodomain_current_sign", "oracle.monodomain", "out[:self.N] = (self.I_stim(t) - I_ion) / self.Cm",
     "out[:self.N] = (I_ion - self.I_stim(t)) / self.Cm",
     [lambda: T_emrkc.test_linear_model_on_cosine_mode(1),
      lambda: T_emrkc.test_linear_model_matrix_function_brute_force((3, 3))]),
    ("ionic_zinf_sign", "oracle.ionic", "zinf = np.stack([a / (a + b) for a, b in rates])",
     "zinf = np.stack([-a / (a + b) for a, b in rates])",
     [T_models.test_hh_resting_gates_textbook_values]),
    ("ionic_rate_sum", "oracle.ionic", "lam = np.stack([-(a + b) for a, b in rates])",
     "lam = np.stack([-(a - b) for a, b in rates])",
     [T_models.test_hh_resting_gates_textbook_values, T_pow.test_rho_S_hh_closed_form,
      lambda: T_models.test_single_cell_action_potential_and_stiffness(HH(), "HH")]),
    ("powiter_step_inverted", "oracle.powiter", "        q = delta / nv\n        rho = nv / delta",
     "        q = nv / delta\n        rho = nv / delta",
     [T_pow.test_rho_F_converges_to_closed_form_max_eigenvalue, T_pow.test_rho_S_linear_model_is_a]),
    ("mrkc_gate_index", "oracle.mrkc", "self.gate = slice(N * (1 + stiff_gate), N * (2 + stiff_gate))",
     "self.gate = slice(N * stiff_gate, N * (1 + stiff_gate))",
     [T_mrkc.test_split_sums_to_the_full_right_hand_side]),
    ("cond_a_factor", "oracle.emrkc", "eta = (6.0 * dt / ls) * (m * m / (m * m - 1.0))",
     "eta = (2.0 * dt / ls) * (m * m / (m * m - 1.0))",
     [T_var.test_cond_a_stage_counts_definition, T_var.test_cond_a_scalar_closed_form]),
    ("progressive_forcing_sign", "oracle.emrkc", "forcing = prob.f_S(t, yE) + (yE - y) / eta",
     "forcing = prob.f_S(t, yE) - (yE - y) / eta",
     [T_var.test_progressive_scalar_closed_form, T_var.test_progressive_equals_standard_on_the_monodomain_split]),
    ("progressive_start_at_yE", "oracle.emrkc", "u_eta = rkc_iteration(t, y, eta, f_u, m, eps)",
     "u_eta = rkc_iteration(t, yE, eta, f_u, m, eps)",
     [T_var.test_progressive_scalar_closed_form, T_var.test_progressive_equals_standard_on_the_monodomain_split]),
    ("rho_every_at_step_zero", "oracle.emrkc", "if rho_every > 0 and n > 0 and n % rho_every == 0:",
     "if rho_every > 0 and n % rho_every == 0:",
     [T_var.test_rho_every_estimates_at_the_scheduled_states, T_var.test_rho_every_linear_model_warm_start]),
    ("rho_every_cold_start", "oracle.emrkc",
     'compute_rho(tn, y, prob.f_F, rho_state["vF"], rho_state["rF"])',
     'compute_rho(tn, y, prob.f_F, rho_state["vF"])',
     [T_var.test_rho_every_estimates_at_the_scheduled_states, T_var.test_rho_every_linear_model_warm_start]),
    ("mrkc_outer_count", "oracle.mrkc", "return rkc_iteration(tn, yn, dt, fbar, s, eps)",
     "return rkc_iteration(tn, yn, dt, fbar, m, eps)",
     [T_mrkc.test_scalar_test_equation_closed_form, lambda: T_mrkc.test_linear_model_matrix_function((3, 3))]),
    ("mrkc_slow_term_dropped", "oracle.mrkc", "return f_F(r, u) + fS_frozen", "return f_F(r, u)",
     [T_mrkc.test_scalar_test_equation_closed_form, lambda: T_mrkc.test_linear_model_matrix_function((3, 3))]),
    ("exexrl_gate_sign", "oracle.exexrl", "zE1 = zE + np.expm1(dt * LE) * (zE - zinf)",
     "zE1 = zE + np.expm1(dt * LE) * (zinf - zE)",
     [T_imex.test_first_order_convergence_against_exexrl], 0),
    ("exexrl_diffusion_dropped", "oracle.exexrl",
     "V1 = V + dt * (diff + (prob.I_stim(tn) - I_ion) / prob.Cm)",
     "V1 = V + dt * ((prob.I_stim(tn) - I_ion) / prob.Cm)",
     [T_imex.test_first_order_convergence_against_exexrl]),
    ("imexrl_gate_sign", "oracle.exexrl", "zE1 = zE + np.expm1(dt * LE) * (zE - zinf)",
     "zE1 = zE + np.expm1(dt * LE) * (zinf - zE)",
     [lambda: T_imex.test_linear_model_cosine_mode_closed_form(0.5)], 1),
    ("imexrl_explicit_sign", "oracle.exexrl", "return (sp.identity(prob.N, format=\"csr\") - dt * Fm).tocsc()",
     "return (sp.identity(prob.N, format=\"csr\") + dt * Fm).tocsc()",
     [lambda: T_imex.test_linear_model_cosine_mode_closed_form(0.5),
      T_imex.test_implicit_diffusion_is_bounded_at_large_steps]),
    # the V equation without the 1/Cm (invisible wherever Cm = 1)
    ("fS_membrane_capacitance", "oracle.monodomain", "out[:self.N] = (self.I_stim(t) - I_ion) / self.Cm",
     "out[:self.N] = self.I_stim(t) - I_ion",
     [lambda: T_cell.test_single_cell_converges_to_radau_solution(*T_cell.CASES[1])]),
    # the stimulus with the wrong sign
    ("fS_stimulus_sign", "oracle.monodomain", "out[:self.N] = (self.I_stim(t) - I_ion) / self.Cm",
     "out[:self.N] = (-self.I_stim(t) - I_ion) / self.Cm",
     [lambda: T_cell.test_single_cell_converges_to_radau_solution(*T_cell.CASES[0])]),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_planted_mistake_is_caught(monkeypatch, case):
    _, modname, old, new, pins = case[:5]
    mod, mutant = _mutant(modname, old, new, case[5] if len(case) > 5 else None)
    _install(monkeypatch, mod, mutant)
    failed = _some_pin_fails(pins)
    assert failed, "no pin caught the planted mistake %r -> %r in %s" % (old, new, modname)


def test_unmutated_oracle_passes_the_same_pins():
    """The pins used above pass on the oracle as it is (so a failure above
    is the planted mistake's doing)."""
    seen = set()
    for case in CASES:
        for pin in case[4]:
            if id(pin) not in seen:
                seen.add(id(pin))
                pin()
