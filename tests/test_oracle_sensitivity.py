"""The oracle's pins catch plausible mistakes in the oracle itself (CPU only).

Each case plants one slip in the oracle for the duration of the test (a dropped factor, a
raised index, a flipped sign or direction, a truncated basis, a swapped table column) and
checks that at least one of the independent pins of the other ``test_oracle_*`` modules then
fails.  A pin that still passed with the slip planted would not be pinning that part of the
oracle.  The pins are the same functions the suite runs unmodified; nothing here touches the
HIP library.
"""

import numpy as np
import pytest
import torch

import test_oracle_quadrature as PQ
import test_oracle_special as PS
import test_oracle_step as PT
from oracle import basis as bs
from oracle import lattice as L
from oracle import mj
from oracle import quadrature as qd


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
}


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
    for pin, args in pins:
        pin(*args)


@pytest.mark.parametrize("slip", list(CASES))
def test_planted_slip_fails_a_pin(slip, monkeypatch):
    plant, pins = CASES[slip]
    plant(monkeypatch)
    with np.errstate(all="ignore"):
        failed = [pin.__name__ for pin, args in pins if _fails(pin, args)]
    assert failed, f"no pin caught the planted slip {slip!r}"
