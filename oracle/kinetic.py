"""Deterministic solution of the kinetic equations for the energy
distributions of electrons, positrons and photons in a uniform magnetic field:
the validation case of Sec. 4 (Eqs. 9-10), solved with the same rates and
inverse CDFs that the Monte Carlo step uses.

TEST INFRASTRUCTURE: only the tests and the validation script beside them use
this module; the product path never imports it.

Model (reading G18 of the equations).  With E = 0 and every momentum
perpendicular to B, a lepton keeps |u| between events and has
chi_e = |u| B / E_s; a photon emitted along u stays perpendicular to B with
chi_gamma = gamma_gamma B / E_s.
  * A lepton of momentum p (gamma = sqrt(1 + p^2)) emits at the rate
    W = A_hat h_rad(chi_e) / gamma (Eq. 6); the photon takes
    gamma_gamma = xi gamma with xi from the inverse CDF of Eq. 7, and the
    lepton keeps p' = max(p - gamma_gamma, 0) (Eq. 8).  Photons with
    gamma_gamma <= 2 are not created (Sec. 3); the lepton still recoils.
  * A photon decays at the rate A_hat h_pair(chi_gamma) / gamma_gamma (zero
    for gamma_gamma <= 2 or chi_gamma below the pair table) into an electron
    and a positron with gamma_- = 1 + (gamma_gamma - 2) eta and
    gamma_+ = 1 + (gamma_gamma - 2)(1 - eta), eta from the pair inverse CDF
    (reading G13).
The distributions live on grids of momentum (leptons, with a node at p = 0)
and of gamma_gamma (photons, with a node at 2).  Each transfer is deposited
on the two neighbouring nodes with weights that keep both the number and
the momentum (energy for photons) exact.  The spectra of the transfers use
n_quant equally spaced quantiles of the inverse CDFs.  Time advances in
explicit sub-steps within steps that follow the Monte Carlo step's timing
(see advance).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import sparse


def _cic(nodes: np.ndarray, v: float):
    """Two-node split of v on increasing nodes keeping count and first moment."""
    if v <= nodes[0]:
        return [(0, 1.0)]
    if v >= nodes[-1]:
        return [(len(nodes) - 1, 1.0)]
    j = int(np.searchsorted(nodes, v, side="right")) - 1
    a, b = nodes[j], nodes[j + 1]
    f = (v - a) / (b - a)
    return [(j, 1.0 - f), (j + 1, f)]


class Kinetic:
    def __init__(self, tabs, units: dict, B_hat: float, p_max: float = 1.2e4, per_decade: int = 200,
                 p_min: float = 1e-2, n_quant: int = 64, gamma_photon_min: float = 2.0,
                 pair_chi_min: float = 1e-2):
        self.es_inv = 1.0 / units["Es_hat"]
        self.A = units["A_hat"]
        self.B = B_hat
        nd = int(math.ceil(per_decade * math.log10(p_max / p_min)))
        self.p = np.concatenate([[0.0], np.geomspace(p_min, p_max, nd + 1)])
        kd = int(math.ceil(per_decade * math.log10(p_max / gamma_photon_min)))
        self.k = np.geomspace(gamma_photon_min, p_max, kd + 1)
        nl, nk = len(self.p), len(self.k)
        r = (np.arange(n_quant) + 0.5) / n_quant
        # emission: rate per lepton node and the transfer of one emission
        self.W = np.zeros(nl)
        lr, lc, lv, gr, gc, gv = [], [], [], [], [], []
        for j, p in enumerate(self.p):
            if p <= 0.0:
                continue
            gam = math.sqrt(1.0 + p * p)
            chi = p * self.B * self.es_inv
            self.W[j] = self.A * tabs.h_rad(chi) / gam
            for q in r:
                gg = tabs.sample_xi(chi, q) * gam
                p2 = max(p - gg, 0.0)
                for (i, w) in _cic(self.p, p2):
                    lr.append(j); lc.append(i); lv.append(w / n_quant)
                if gg > gamma_photon_min:
                    for (i, w) in _cic(self.k, gg):
                        gr.append(j); gc.append(i); gv.append(w / n_quant)
        self.T_lep = sparse.csr_matrix((lv, (lr, lc)), shape=(nl, nl))
        self.T_pho = sparse.csr_matrix((gv, (gr, gc)), shape=(nl, nk))
        # pair creation: rate per photon node and the leptons of one decay
        self.Wp = np.zeros(nk)
        er, ec, ev, pr, pc, pv = [], [], [], [], [], []
        for j, g in enumerate(self.k):
            chi = g * self.B * self.es_inv
            if not (g > 2.0 and chi >= pair_chi_min):
                continue
            self.Wp[j] = self.A * tabs.h_pair(chi) / g
            for q in r:
                eta = tabs.sample_eta(chi, q)
                gm = 1.0 + (g - 2.0) * eta
                gp = 1.0 + (g - 2.0) * (1.0 - eta)
                for (i, w) in _cic(self.p, math.sqrt(max(gm * gm - 1.0, 0.0))):
                    er.append(j); ec.append(i); ev.append(w / n_quant)
                for (i, w) in _cic(self.p, math.sqrt(max(gp * gp - 1.0, 0.0))):
                    pr.append(j); pc.append(i); pv.append(w / n_quant)
        self.P_ele = sparse.csr_matrix((ev, (er, ec)), shape=(nk, nl))
        self.P_pos = sparse.csr_matrix((pv, (pr, pc)), shape=(nk, nl))
        self.fe = np.zeros(nl)
        self.fp = np.zeros(nl)
        self.fg = np.zeros(nk)
        self.t = 0.0

    def add_electrons(self, p: float, n: float):
        for (i, w) in _cic(self.p, p):
            self.fe[i] += n * w

    def advance(self, steps: int, dt: float, n_sub: int = 8):
        """`steps` steps of length dt, each in n_sub explicit sub-steps, with the
        Monte Carlo step's timing: leptons emit all through the step (at their
        updated energy), photons alive at the start of the step decay during
        it, and the photons and pairs created in a step join their species at
        its end (they are stored at the next time level)."""
        h = dt / n_sub
        for _ in range(steps):
            ng = np.zeros_like(self.fg)
            ne = np.zeros_like(self.fe)
            np_ = np.zeros_like(self.fp)
            for _ in range(n_sub):
                oe = self.W * self.fe * h
                op = self.W * self.fp * h
                og = self.Wp * self.fg * h
                self.fe += self.T_lep.T @ oe - oe
                self.fp += self.T_lep.T @ op - op
                self.fg -= og
                ng += self.T_pho.T @ (oe + op)
                ne += self.P_ele.T @ og
                np_ += self.P_pos.T @ og
            self.fg += ng
            self.fe += ne
            self.fp += np_
            self.t += dt

    def moments(self) -> dict:
        """Number, energy (gamma, or gamma_gamma) and mean chi of each species."""
        gl = np.sqrt(1.0 + self.p ** 2)
        chil = self.p * self.B * self.es_inv
        chig = self.k * self.B * self.es_inv
        out = {}
        for name, f, e, c in (("electrons", self.fe, gl, chil), ("positrons", self.fp, gl, chil),
                              ("photons", self.fg, self.k, chig)):
            n = float(f.sum())
            out[name] = {"n": n, "energy": float(f @ e), "chi": float(f @ c) / n if n > 0 else 0.0}
        return out


def mc_moments(species: dict, photons: bool, B_hat: float, Es_hat: float) -> dict:
    """The same moments from Monte Carlo particles (dict of arrays, live entries only)."""
    u = np.sqrt(species["ux"].astype(np.float64) ** 2 + species["uy"].astype(np.float64) ** 2 +
                species["uz"].astype(np.float64) ** 2)
    w = species["w"].astype(np.float64)
    if photons:
        keep = ~np.isinf(species["tau"])
        u, w = u[keep], w[keep]
        e = u
    else:
        e = np.sqrt(1.0 + u * u)
    n = float(w.sum())
    return {"n": n, "energy": float(w @ e), "chi": float(w @ (u * B_hat / Es_hat)) / n if n > 0 else 0.0}
