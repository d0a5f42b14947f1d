"""The oracle's pins catch plausible mistakes in the oracle itself (CPU only).

Each case plants one slip in the oracle for the duration of the test (a dropped factor, a
raised index, a flipped sign or direction, an exponent or factorial off by one, a truncated
basis, a swapped table column) and
checks that at least one of the independent pins of the other ``test_oracle_*`` modules then
fails.  A pin that still passed with the slip planted would not be pinning that part of the
oracle.  The pins are the same functions the suite runs unmodified; nothing here touches the
HIP library.
"""

import inspect
import sys
import textwrap

import numpy as np
import pytest
import torch

import test_oracle_grad as PG
import test_oracle_quadrature as PQ
import test_oracle_sod as PD
import test_oracle_special as PS
import test_oracle_step as PT
from oracle import basis as bs
from oracle import grad as og
from oracle import lattice as L
from oracle import mj
from oracle import quadrature as qd
from oracle import sod


def _edit(mp, owner, name, old, new):
    """Replace ``owner.name`` by a copy compiled from its own source with the text ``old`` (which
    must occur exactly once) replaced by ``new``; the copy resolves globals as the original does."""
    fn = getattr(owner, name)
    src = textwrap.dedent(inspect.getsource(fn))
    assert src.count(old) == 1, (name, old)
    ns = dict(vars(sys.modules[fn.__module__]))
    exec(compile(src.replace(old, new), f"<{name} with a planted slip>", "exec"), ns)
    mp.setattr(owner, name, ns[name])


def _euclidean_metric(method):
    """The method run with eta replaced by the identity: an index that should be lowered is not."""
    def wrapped(self, *args):
        eta = self.eta
        self.eta = torch.eye(self.d + 1, dtype=torch.float64)
        try:
            return method(self, *args)
        finally:
            self.eta = eta
    return wrapped


def plant_landau_without_metric(mp):
    # Sec. 6.2 step 2: the eigenproblem of T^a_b taken as that of T^ab
    mp.setattr(L.Lattice, "landau", _euclidean_metric(L.Lattice.landau))


def plant_density_with_raised_index(mp):
    # Sec. 6.2 step 3: n = U^a N^a instead of U_a N^a
    mp.setattr(L.Lattice, "density", _euclidean_metric(L.Lattice.density))


def plant_omega_without_energy(mp):
    # Sec. 6.2 step 8: the 1/p^0 of the Anderson-Witting rate dropped
    orig = L.Lattice.omega

    def omega(self, U, tau):
        out = orig(self, U, tau)
        return out * self.p[:, 0].reshape((-1,) + (1,) * (out.dim() - 1))
    mp.setattr(L.Lattice, "omega", omega)


def plant_eos_wrong_dimension(mp):
    # Sec. 3: the (d+1)-dimensional equation of state on a d-dimensional lattice
    def temperature(self, eps, n):
        return mj.temperature_from_energy(eps / n, self.m, self.d + 1)
    mp.setattr(L.Lattice, "temperature", temperature)


def plant_stream_reversed(mp):
    # streaming reads f*(x + delta_i) instead of f*(x - delta_i)
    orig = L.Lattice.stream

    def stream(self, fstar):
        disp = self.disp
        self.disp = -disp
        try:
            return orig(self, fstar)
        finally:
            self.disp = disp
    mp.setattr(L.Lattice, "stream", stream)


def plant_force_sign(mp):
    # Sec. 5.4: the external-force term added instead of subtracted
    orig = L.Lattice.forcing
    mp.setattr(L.Lattice, "forcing", lambda self, T, U, feq: -orig(self, T, U, feq))


def plant_basis_truncated(mp):
    # Sec. 5.1: the generating monomials of the highest degree left out
    orig = bs.generating_set
    mp.setattr(bs, "generating_set", lambda d, order: orig(d, order - 1))


def plant_euclidean_mj_moments(mp):
    # App. B: eta^{ab} of the tensor moments taken as the identity
    mp.setattr(mj, "minkowski", lambda a, b: 1.0 if a == b else 0.0)


def plant_bessel_order_off_by_one(mp):
    # Sec. 3 / App. B: the ratio A_n/A_1 taken one order too high
    orig = mj.a_ratio
    mp.setattr(mj, "a_ratio", lambda n, zeta, d: orig(n + 1, zeta, d))


def plant_missing_direction(mp):
    # the product rule built over one direction too few
    mp.setattr(qd, "DIRS_2D", list(qd.DIRS_2D)[:-1])


def plant_ur_weight_columns_swapped(mp):
    # App. H.2: the weights of the (3, 4) and (5, 0) direction groups of the printed table exchanged
    mp.setattr(qd, "UR2D_W_34", qd.UR2D_W_50)
    mp.setattr(qd, "UR2D_W_50", qd.UR2D_W_34)


def plant_interpolation_weights_swapped(mp):
    # streaming: the weights of the two bracketing sites exchanged (frac <-> 1 - frac)
    _edit(mp, L.Lattice, "stream", "wgt *= frac[ax] if corner[ax] else 1.0 - frac[ax]",
          "wgt *= 1.0 - frac[ax] if corner[ax] else frac[ax]")


def plant_open_axis_wraps(mp):
    # an open axis read as periodic (upstream coordinates wrapped instead of clamped)
    _edit(mp, L.Lattice, "_gather", 'if self.bc[ax] == "periodic":', 'if self.bc[ax] != "wall":')


def plant_mj_alternating_sign_dropped(mp):
    # App. B.1: the (-1)^k of the pairing sum dropped
    _edit(mp, mj, "mj_tensor_moment", "total = total + (-1) ** k * a_ratio(r - k, zeta, d) * term",
          "total = total + a_ratio(r - k, zeta, d) * term")


def plant_mj_temperature_power(mp):
    # App. B.1: the rank-r moment scaled by T^r instead of T^(r-1)
    _edit(mp, mj, "mj_tensor_moment", "return n * T ** (r - 1) * total", "return n * T ** r * total")


def plant_wall_plane_off_by_one(mp):
    # Sec. 8.1: the far wall placed one plane inside the lattice
    _edit(mp, L.Lattice, "wall_mask", "idx[dim] = grid_shape[dim] - 1", "idx[dim] = grid_shape[dim] - 2")


def plant_product_momentum_slip(mp):
    # the product rule's |p| = sqrt(x^2 + 2 m x) with the factor 2 dropped
    _edit(mp, qd, "product_2d", "math.sqrt(x[j] * x[j] + 2.0 * m * x[j])", "math.sqrt(x[j] * x[j] + m * x[j])")


def plant_tau_law_inverted(mp):
    # Sec. 6.2 step 7 (constant eta/s): the relaxation time grown by tau_T T instead of tau_T / T
    _edit(mp, L.Lattice, "collide", 'tau = tau + self.tau_T / mac["T"]', 'tau = tau + self.tau_T * mac["T"]')


def plant_sphere_average_off_by_one(mp):
    # the sphere averages behind the 3D direction weights with (a+b+c-1)!! in the denominator
    _edit(mp, qd, "sphere_average", "dfact(a + b + c + 1)", "dfact(a + b + c - 1)")


def plant_massive_energy_power(mp):
    # Sec. 5.3: the moment system of the weights with the power of p^0 one too high
    _edit(mp, qd, "massive_group_weights", "A[r, g] = p0 ** row[0] *", "A[r, g] = p0 ** (row[0] + 1) *")


def plant_sod_fan_exponent(mp):
    # App. D: the rarefaction's pressure exponent without its factor 2
    _edit(mp, sod, "plateau_pressure", "k = 2.0 * math.sqrt(d) / (d + 1)", "k = math.sqrt(d) / (d + 1)")


def plant_sod_fan_density(mp):
    # App. D: the density in the fan with the exponent sqrt(d) instead of sqrt(d)/2
    _edit(mp, sod, "solution", "n[fan] = nL * ratio ** (sd / 2.0)", "n[fan] = nL * ratio ** sd")


def plant_adjoint_eigen_jacobian_sign(mp):
    # reverse mode: a sign slip in the Jacobian of the Landau eigenproblem
    _edit(mp, og, "landau_diff", "J[:, :D, D] = -u0", "J[:, :D, D] = u0")


def plant_adjoint_eos_newton_sign(mp):
    # reverse mode: the EOS inversion's Newton correction added instead of subtracted
    _edit(mp, og, "temperature_diff", "return T0 - (eT.detach() - e) / slope",
          "return T0 + (eT.detach() - e) / slope")


def plant_ce_shear_wrong_dimension(mp):
    # Sec. 4.1 / App. C: the Chapman-Enskog shear ratio of the (d+1)-dimensional gas
    orig = mj.ce_shear_ratio
    mp.setattr(mj, "ce_shear_ratio", lambda zeta, d: orig(zeta, d + 1))


# (slip, pins any one of which must fail with it planted)
CASES = {
    "landau_without_metric": (plant_landau_without_metric,
                              [(PT.test_landau_recovers_known_state, (2,))]),
    "density_with_raised_index": (plant_density_with_raised_index,
                                  [(PT.test_collision_invariants, ("p2m1",))]),
    "omega_without_energy": (plant_omega_without_energy,
                             [(PT.test_collision_invariants, ("p2m1",))]),
    "eos_wrong_dimension": (plant_eos_wrong_dimension,
                            [(PT.test_collision_invariants, ("p2m1",))]),
    "stream_reversed": (plant_stream_reversed,
                        [(PT.test_integer_streaming_is_a_shift, ())]),
    "force_sign": (plant_force_sign,
                   [(PT.test_force_term_moments, ("p2m1",))]),
    "basis_truncated": (plant_basis_truncated,
                        [(PQ.test_basis_orthonormal_and_dimension, ("p2",))]),
    "euclidean_mj_moments": (plant_euclidean_mj_moments,
                             [(PS.test_mj_moments_brute_force, (2, 1.0, 1.3, (0.3, -0.2)))]),
    "bessel_order_off_by_one": (plant_bessel_order_off_by_one,
                                [(PS.test_G_closed_forms_and_3d_identity, ())]),
    "missing_direction": (plant_missing_direction,
                          [(PQ.test_product_2d_exact_to_degree_7, (1.0,))]),
    "ur_weight_columns_swapped": (plant_ur_weight_columns_swapped,
                                  [(PQ.test_ur_rule_exact_to_degree_4_only, ())]),
    "interpolation_weights_swapped": (plant_interpolation_weights_swapped,
                                      [(PT.test_interpolated_streaming_conserves_each_population, ("p2m1",))]),
    "mj_alternating_sign_dropped": (plant_mj_alternating_sign_dropped,
                                    [(PS.test_mj_moments_brute_force, (2, 1.0, 1.3, (0.3, -0.2)))]),
    "mj_temperature_power": (plant_mj_temperature_power,
                             [(PS.test_mj_moments_brute_force, (2, 1.0, 1.3, (0.3, -0.2)))]),
    "wall_plane_off_by_one": (plant_wall_plane_off_by_one,
                              [(PT.test_force_accelerates_along_g_and_walls_hold_rest, ())]),
    "product_momentum_slip": (plant_product_momentum_slip,
                              [(PQ.test_product_2d_exact_to_degree_7, (1.0,))]),
    "open_axis_wraps": (plant_open_axis_wraps,
                        [(PT.test_open_axis_budget_of_an_integer_shift, ())]),
    "sphere_average_off_by_one": (plant_sphere_average_off_by_one,
                                  [(PQ.test_product_3d_exact_to_degree_7, (1.0,))]),
    "massive_energy_power": (plant_massive_energy_power,
                                 [(PQ.test_massive_solver_reproduces_printed_weights_and_window, ())]),
    "sod_fan_exponent": (plant_sod_fan_exponent,
                         [(PD.test_shock_jump_conditions, (2,)), (PD.test_rarefaction_fan, (2,))]),
    "sod_fan_density": (plant_sod_fan_density,
                        [(PD.test_rarefaction_fan, (2,)), (PD.test_global_conservation, (2,))]),
    "adjoint_eigen_jacobian_sign": (plant_adjoint_eigen_jacobian_sign,
                                    [(PG.test_gradient_matches_central_differences, (1,))]),
    "adjoint_eos_newton_sign": (plant_adjoint_eos_newton_sign,
                                [(PG.test_gradient_matches_central_differences, (1,))]),
    "ce_shear_wrong_dimension": (plant_ce_shear_wrong_dimension,
                                 [(PS.test_ce_shear_limits_and_table2, ())]),
    # the one pin of the tau law is the 300-step Sod run (about 30 s)
    "tau_law_inverted": (plant_tau_law_inverted,
                         [(PD.test_oracle_lattice_reproduces_app_d, ())]),
}

# pins too slow to run a second time unmodified here (their own module runs them)
SLOW_PINS = {PD.test_oracle_lattice_reproduces_app_d}


def _fails(pin, args):
    try:
        pin(*args)
    except AssertionError:
        return True
    return False


@pytest.mark.parametrize("slip", list(CASES))
def test_pins_pass_without_the_slip(slip):
    """The pins used below pass on the oracle as it is (so a failure below is the slip's)."""
    _, pins = CASES[slip]
    pins = [(pin, args) for pin, args in pins if pin not in SLOW_PINS]
    if not pins:
        pytest.skip("its pin runs unmodified in its own module")
    for pin, args in pins:
        pin(*args)


@pytest.mark.parametrize("slip", list(CASES))
def test_planted_slip_fails_a_pin(slip, monkeypatch):
    plant, pins = CASES[slip]
    plant(monkeypatch)
    with np.errstate(all="ignore"):
        failed = [pin.__name__ for pin, args in pins if _fails(pin, args)]
    assert failed, f"no pin caught the planted slip {slip!r}"
