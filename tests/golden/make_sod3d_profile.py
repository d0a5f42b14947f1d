"""Writes sod3d_eta002_234_profile.json: n, eps, T and beta = U^x / U^0 at every 8th site of the physical
half of the ultra-relativistic Sod tube in (3+1) dimensions after 234 steps, computed by the FP64
oracle alone: the printed (3+1)-d order-3 massless rule (App. H.1, 288 populations, v0 = 1/sqrt(41)),
6400 x 1 x 1 sites (open y and z: the flow is one-dimensional) with the mirror image of the left
state (T_L = 1, n_L = 1 for the first 1600 sites, P_L / P_R = 5.43, T_R = 0.475), tau = 1/2 + tau_T / T
for eta/s = 0.002 (Sec. 8.2, the inviscid test; s = 4 n, c_eta = 4/5 for d = 3).  Light crosses
sqrt(41) sites per step, so dt = sqrt(41) * 0.002 fm/c and 234 steps reach t = 3.0 fm/c.  Run from
the repository root:
    python tests/golden/make_sod3d_profile.py
It takes a few minutes on the CPU."""
import json
import math
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import lattice as OL                      # noqa: E402
from oracle import mj                                 # noqa: E402
from oracle import quadrature as qd                   # noqa: E402

NX, SPLIT, STEPS, EVERY = 6400, 1600, 234, 8
DX = 0.002                                            # fm per site
HBARC_OVER_T0 = 197.327 / 400.0                       # fm


def main():
    d = 3
    PL, nL, TR = 1.0, 1.0, 0.475
    PR = 1.0 / 5.43
    nR = PR / TR
    k = np.arange(NX)
    left = np.where(k < NX // 2, k, NX - 1 - k) < SPLIT
    n = torch.tensor(np.where(left, nL, nR)[None, None, :])
    T = torch.tensor(np.where(left, PL / nL, TR)[None, None, :])
    u = torch.zeros((3, 1, 1, NX), dtype=torch.float64)
    dt = math.sqrt(41.0) * DX
    tau_T = 0.002 * (d + 1) / mj.ce_shear_ratio(0.0, d) * HBARC_OVER_T0 / dt
    ol = OL.Lattice(qd.ur_onlattice_3d(3), 0.5, (NX, 1, 1), bc=("periodic", "open", "open"), tau_T=tau_T)
    fs = ol.collide(ol.init(n, T, u))      # the stored state f*_0 = C(f_0)
    for s in range(STEPS):                 # f*_k = C(S(f*_{k-1}))
        fs = ol.collide(ol.stream(fs))
        if (s + 1) % 50 == 0:
            print("step", s + 1, flush=True)
    mac = ol.macro(ol.stream(fs))          # the moments call's fields for f*_STEPS
    sites = list(range(0, NX // 2, EVERY))
    out = {"citation": "Sec. 8.2 (ultra-relativistic Sod tube, inviscid test, eta/s = 0.002) in (3+1) "
                       "dimensions with the printed order-3 massless rule of App. H.1; FP64 oracle only",
           "nx": NX, "split": SPLIT, "steps": STEPS, "tau_T": tau_T, "sites": sites,
           "n": mac["n"][0, 0, sites].tolist(), "eps": mac["eps"][0, 0, sites].tolist(),
           "T": mac["T"][0, 0, sites].tolist(),
           "beta": (mac["U"][1] / mac["U"][0])[0, 0, sites].tolist()}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "sod3d_eta002_234_profile.json"), "w") as fh:
        json.dump(out, fh, indent=0)


if __name__ == "__main__":
    main()
