"""Writes c3_tau08_profiles.json: the x-profiles of n, eps, T and U^x of the 3D shock tube (zeta = 1,
N = 3 product rule, open x, tau = 0.8; left n = 8/3, T = 1.5 for x < 128, right n = 1, T = 1, at
rest) after 10, 100, 500, 1000 and 2000 steps, computed by the FP64 oracle alone on the equivalent
256 x 1 x 1 lattice (the state depends on x only).  Run from the repository root:
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

NX, TAU = 256, 0.8
CHECKPOINTS = (10, 100, 500, 1000, 2000)


def main():
    n, T, u = (torch.tensor(a) for a in W.riemann_3d(NX, 1, 1, NX // 2, 8.0 / 3.0, 1.5, 1.0, 1.0))
    ol = OL.Lattice(qd.product_3d(1.0, 3), TAU, (NX, 1, 1), bc=("open", "periodic", "periodic"))
    fs = ol.collide(ol.init(n, T, u))      # the initial stored state f*_0 = C(f_0)
    profiles = {}
    for s in range(1, CHECKPOINTS[-1] + 1):   # f*_k = C(S(f*_{k-1}))
        fs = ol.collide(ol.stream(fs))
        if s in CHECKPOINTS:
            mac = ol.macro(ol.stream(fs))  # what the moments call reports for f*_s
            profiles[str(s)] = {"n": mac["n"][0, 0].tolist(), "eps": mac["eps"][0, 0].tolist(),
                                "T": mac["T"][0, 0].tolist(), "Ux": mac["U"][1, 0, 0].tolist()}
            print("step", s, flush=True)
    out = {"citation": "Shock tube of Sec. 8.2 with the (3+1)-d product rule of the 3D workload "
                       "(Riemann state n 8/3, T 1.5 | n 1, T 1 at rest; open x); FP64 oracle only",
           "nx": NX, "tau": TAU, "zeta": 1.0, "order": 3, "checkpoints": list(CHECKPOINTS),
           "profiles": profiles}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_tau08_profiles.json"), "w") as fh:
        json.dump(out, fh, indent=0)


if __name__ == "__main__":
    main()
