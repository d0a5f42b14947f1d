"""Writes sod_eta002_300_profile.json: n, eps, T and beta = U^x / U^0 at every 8th site of the physical
half of the ultra-relativistic Sod tube after 300 steps, computed by the FP64 oracle alone: the
printed order-3 massless rule (App. H.2), 6400 x 5 sites with the mirror image of the left state
(T_L = 1, n_L = 1 for the first 1600 sites, P_L / P_R = 5.43, T_R = 0.475), tau = 1/2 + tau_T / T
for eta/s = 0.002 (Sec. 8.2, the inviscid test).  Run from the repository root:
    python tests/golden/make_sod_profile.py
It takes under a minute on the CPU."""
import json
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import lattice as OL                      # noqa: E402
from oracle import mj                                 # noqa: E402
from oracle import quadrature as qd                   # noqa: E402

NX, NY, SPLIT, STEPS, EVERY = 6400, 5, 1600, 300, 8


def main():
    PL, nL, TR = 1.0, 1.0, 0.475
    PR = 1.0 / 5.43
    nR = PR / TR
    k = np.arange(NX)
    left = np.where(k < NX // 2, k, NX - 1 - k) < SPLIT
    n = torch.tensor(np.where(left, nL, nR)[None, :] * np.ones((NY, 1)))
    T = torch.tensor(np.where(left, PL / nL, TR)[None, :] * np.ones((NY, 1)))
    u = torch.zeros((2, NY, NX), dtype=torch.float64)
    tau_T = 0.002 * 3 / mj.ce_shear_ratio(0.0, 2) * (197.327 / 400.0) / 0.01
    ol = OL.Lattice(qd.ur_onlattice_2d(3), 0.5, (NX, NY), tau_T=tau_T)
    fs = ol.collide(ol.init(n, T, u))      # the stored state f*_0 = C(f_0)
    for _ in range(STEPS):                 # f*_k = C(S(f*_{k-1}))
        fs = ol.collide(ol.stream(fs))
    mac = ol.macro(ol.stream(fs))          # the moments call's fields for f*_STEPS
    sites = list(range(0, NX // 2, EVERY))
    out = {"citation": "Sec. 8.2 (ultra-relativistic Sod tube, inviscid test, eta/s = 0.002) with the "
                       "printed order-3 massless rule of App. H.2; FP64 oracle only",
           "nx": NX, "ny": NY, "split": SPLIT, "steps": STEPS, "tau_T": tau_T, "sites": sites,
           "n": mac["n"][0, sites].tolist(), "eps": mac["eps"][0, sites].tolist(),
           "T": mac["T"][0, sites].tolist(), "beta": (mac["U"][1] / mac["U"][0])[0, sites].tolist()}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "sod_eta002_300_profile.json"), "w") as fh:
        json.dump(out, fh, indent=0)


if __name__ == "__main__":
    main()
