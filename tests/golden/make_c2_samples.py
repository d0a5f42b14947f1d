"""Writes c2_samples.json: n, eps, T and U at 512 seeded sites of the 1024 x 1024 C2 workload
(zeta = 1, N = 3 product rule, tau = 0.8, Taylor-Green u0 = 0.1, T = 1, n = 1 + 1e-3 N(0, 1) with
seed 2, periodic) after 10, 100, 500 and 1000 steps, computed by the FP64 oracle alone.  Run from
the repository root (about an hour on 8 CPU cores):
    python tests/golden/make_c2_samples.py"""
import json
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import workloads as W                                 # noqa: E402
from oracle import lattice as OL                      # noqa: E402
from oracle import quadrature as qd                   # noqa: E402

L, K = 1024, 512
CHECKPOINTS = (10, 100, 500, 1000)


def main():
    n, T, u = (torch.tensor(a) for a in W.taylor_green_2d(L, L, 0.1, density_sigma=1e-3, seed=2))
    ol = OL.Lattice(qd.product_2d(1.0, 3), 0.8, (L, L))
    g = np.random.default_rng(12)
    ys, xs = g.integers(0, L, K), g.integers(0, L, K)
    fs = ol.collide(ol.init(n, T, u))      # the stored state f*_0 = C(f_0)
    samples = {}
    for s in range(1, CHECKPOINTS[-1] + 1):   # f*_k = C(S(f*_{k-1}))
        fs = ol.collide(ol.stream(fs))
        if s in CHECKPOINTS:
            mac = ol.macro(ol.stream(fs))  # the moments call's fields for f*_s
            samples[str(s)] = {"n": mac["n"][ys, xs].tolist(), "eps": mac["eps"][ys, xs].tolist(),
                               "T": mac["T"][ys, xs].tolist(), "U": mac["U"][:, ys, xs].tolist()}
            del mac
        if s % 100 == 0:
            print("step", s, flush=True)
    out = {"citation": "Taylor-Green workload of Sec. 7.1 on the (2+1)-d product rule, 1024^2; "
                       "FP64 oracle only",
           "L": L, "checkpoints": list(CHECKPOINTS), "ys": ys.tolist(), "xs": xs.tolist(), "samples": samples}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_samples.json"), "w") as fh:
        json.dump(out, fh, indent=0)


if __name__ == "__main__":
    main()
