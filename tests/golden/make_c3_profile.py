"""Writes c3_tau08_2000_profile.json: the x-profiles of n, eps, T and U^x after 2000 steps of the 3D
shock tube (zeta = 1, N = 3 product rule, open x, tau = 0.8; left n = 8/3, T = 1.5 for x < 128,
right n = 1, T = 1, at rest), computed by the FP64 oracle alone on the equivalent 256 x 1 x 1
lattice (the state depends on x only).  Run from the repository root:
    python tests/golden/make_c3_profile.py
It takes a few minutes on the CPU."""
import json
import os
import sys

import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import workloads as W                                 # noqa: E402
from oracle import lattice as OL                      # noqa: E402
from oracle import quadrature as qd                   # noqa: E402

NX, STEPS, TAU = 256, 2000, 0.8


def main():
    n, T, u = (torch.tensor(a) for a in W.riemann_3d(NX, 1, 1, NX // 2, 8.0 / 3.0, 1.5, 1.0, 1.0))
    ol = OL.Lattice(qd.product_3d(1.0, 3), TAU, (NX, 1, 1), bc=("open", "periodic", "periodic"))
    fs = ol.collide(ol.init(n, T, u))      # the initial stored state f*_0 = C(f_0)
    for _ in range(STEPS):                 # f*_k = C(S(f*_{k-1}))
        fs = ol.collide(ol.stream(fs))
    mac = ol.macro(ol.stream(fs))          # what the moments call reports for f*_STEPS
    out = {"citation": "Shock tube of Sec. 7 with the (3+1)-d product rule of the 3D workload "
                       "(Riemann state n 8/3, T 1.5 | n 1, T 1 at rest; open x); FP64 oracle only",
           "nx": NX, "steps": STEPS, "tau": TAU, "zeta": 1.0, "order": 3,
           "n": mac["n"][0, 0].tolist(), "eps": mac["eps"][0, 0].tolist(), "T": mac["T"][0, 0].tolist(),
           "Ux": mac["U"][1, 0, 0].tolist()}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_tau08_2000_profile.json"), "w") as fh:
        json.dump(out, fh, indent=0)


if __name__ == "__main__":
    main()
