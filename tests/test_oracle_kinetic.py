"""The oracle's Monte Carlo ensemble against the kinetic equations of the
energy distributions (the validation case of Sec. 4, Eqs. 9-10): electrons of
gamma = 3000 in a uniform 7.48 MT field (chi_e ~ 5), every momentum
perpendicular to B.  Species numbers, energies and mean chi follow the
deterministic solution within the Monte Carlo's statistical error."""
import math

import numpy as np
import pytest

from oracle import kinetic as K
from oracle import oracle as O

GAMMA0, B_TESLA = 3000.0, 7.48e6
DT = 2 * math.pi / 100


def constant_b_mc_oracle(bt, n0: int, steps: int, checkpoints, seed=7):
    """Oracle Monte Carlo of the constant-B case; moments at the checkpoint steps."""
    u = O.units()
    Bh = B_TESLA / u["B_ref"]
    p0 = math.sqrt(GAMMA0 ** 2 - 1.0)
    e = {"x": np.zeros(n0), "y": np.zeros(n0), "z": np.zeros(n0), "ux": np.full(n0, p0),
         "uy": np.zeros(n0), "uz": np.zeros(n0), "w": np.ones(n0), "uid": np.arange(n0, dtype=np.uint64)}
    el = O.species_from(e, capacity=8 * n0)
    O.init_tau(el, seed)
    po = O.new_species(8 * n0)
    ph = O.new_species(200 * n0)
    un = [n0]
    tally = O.Tally()
    field = O.make_field(O.FIELD_UNIFORM, B=(0.0, 0.0, Bh))
    out = {}
    for n in range(steps):
        st = O.make_step(n * DT, DT, seed, rad_model=O.RAD_MC, chi_photon_push_min=0.0)
        n_ph0 = ph["n"]
        O.push_emit(bt, 0.8e-6, -1.0, el, field, ph, None, st, un, tally)
        O.push_emit(bt, 0.8e-6, +1.0, po, field, ph, None, st, un, tally)
        O.pair_create(bt, 0.8e-6, ph, field, el, po, st, un, tally, n_limit=n_ph0)
        if n + 1 in checkpoints:
            out[n + 1] = {"electrons": K.mc_moments(O.view(el), False, Bh, u["Es_hat"]),
                          "positrons": K.mc_moments(O.view(po), False, Bh, u["Es_hat"]),
                          "photons": K.mc_moments(O.view(ph), True, Bh, u["Es_hat"])}
    assert tally.as_dict()["N_overflow"] == 0
    return out


def kinetic_moments(bt, checkpoints):
    u = O.units()
    kin = K.Kinetic(bt, u, B_TESLA / u["B_ref"])
    kin.add_electrons(math.sqrt(GAMMA0 ** 2 - 1.0), 1.0)
    out = {}
    done = 0
    for s in sorted(checkpoints):
        kin.advance(s - done, DT)
        done = s
        out[s] = kin.moments()
    return out


def test_kinetic_solver_conserves_what_it_should(bound_tables):
    """Pair creation adds one electron and one positron; emission keeps the
    lepton number; the energy only drops by the sub-threshold photons."""
    u = O.units()
    kin = K.Kinetic(bound_tables, u, B_TESLA / u["B_ref"])
    kin.add_electrons(math.sqrt(GAMMA0 ** 2 - 1.0), 1.0)
    kin.advance(100, DT)
    m = kin.moments()
    assert m["electrons"]["n"] - m["positrons"]["n"] == pytest.approx(1.0, abs=1e-9)
    e_tot = m["electrons"]["energy"] + m["positrons"]["energy"] + m["photons"]["energy"]
    assert 0.98 * GAMMA0 < e_tot <= GAMMA0 * (1 + 1e-9)
    # the paper's qualitative picture: photons near gamma ~ 1e3 first, chi_gamma ~ 1 early
    kin2 = K.Kinetic(bound_tables, u, B_TESLA / u["B_ref"])
    kin2.add_electrons(math.sqrt(GAMMA0 ** 2 - 1.0), 1.0)
    kin2.advance(5, DT)
    m2 = kin2.moments()
    assert 0.3 < m2["photons"]["chi"] < 2.0


def test_oracle_mc_follows_kinetic_equations(bound_tables):
    checkpoints = (10, 25, 50, 100, 150)
    n0 = 1500
    mc = constant_b_mc_oracle(bound_tables, n0, max(checkpoints), checkpoints)
    kin = kinetic_moments(bound_tables, checkpoints)
    check(mc, kin, n0, checkpoints)


def check(mc, kin, n0, checkpoints):
    """Each moment within 4 / sqrt(particles of the species) + 2 % of the
    kinetic solution: the Monte Carlo's statistical error plus the solver's
    discretisation (grids, quantiles, sub-steps)."""
    for s in checkpoints:
        for sp in ("electrons", "positrons", "photons"):
            count = max(mc[s][sp]["n"], 1.0)
            tol = 4.0 / math.sqrt(count) + 0.02
            for q in ("n", "energy", "chi"):
                a = mc[s][sp][q] / (n0 if q != "chi" else 1.0)
                b = kin[s][sp][q]
                print(f"step {s} {sp} {q}: MC {a:.5g} kinetic {b:.5g} (tol {tol:.3f})")
                assert a == pytest.approx(b, rel=tol), (s, sp, q)
