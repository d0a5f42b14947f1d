"""Benchmark of the RLBM collide-and-stream update on one MI355X.

Workload (the 2D configuration the headline metric is quoted on): d = 2,
zeta = 1, order N = 3, off-lattice product quadrature (Q = 32), 1024 x 1024
periodic grid, relativistic Taylor-Green vortex u0 = 0.1, T = 1, density
1 + 1e-3 N(0,1) (seed 2), tau = 0.8, double storage.  A step is one fused
stream + collide over the whole lattice.

Prints one JSON line: MLUPS (10^6 site updates per second), the HBM roofline
of the step kernel (algorithmic bytes 2 Q s per site), variants (float
deviation storage), and the FP64 CPU oracle timed on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS and % HBM roofline (fwd, adjoint, batched) at stated error vs FP64 oracle"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the launch variant of the single-lattice legs (default: the library's default)")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-onlattice", action="store_true")
    ap.add_argument("--no-forcing", action="store_true")
    ap.add_argument("--no-staged-large", action="store_true")
    ap.add_argument("--size-3d", type=int, default=256)
    ap.add_argument("--only", default=None,
                    help="run the headline and this one optional leg (onlattice_ur, massive_onlattice, sod_ur, "
                         "calibrations, forcing_walls, shock_tube_3d, adjoint, batched, variants, staged_large)")
    a = ap.parse_args()
    if a.only is not None:
        a.no_variants = a.only != "variants"
        a.no_adjoint = a.only != "adjoint"
        a.no_3d = a.only != "shock_tube_3d"
        a.no_batch = a.only != "batched"
        a.no_forcing = a.only != "forcing_walls"
        a.no_staged_large = a.only != "staged_large"
        a.no_onlattice = a.only not in ("onlattice_ur", "massive_onlattice", "sod_ur", "calibrations")
    return a


def time_steps(lat, fa, fb, warmup, steps):
    """Average duration of one step, from HIP events on the launch stream around `steps` steps.

    The steps run as calls of `chunk` steps each, chunk the greatest common divisor of warmup and
    steps: the warmup calls capture the launch graph of a chunk on (fa, fb) and the timed calls
    replay it, so the timed region holds the `steps` steps and no graph capture.  (Each call steps
    from fa; with an odd chunk the result lands in fb each time.)"""
    import math
    import torch
    chunk = math.gcd(warmup, steps) if warmup > 0 else steps
    for _ in range(warmup // chunk):
        lat.step(fa, fb, chunk)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps // chunk):
        lat.step(fa, fb, chunk)
    e1.record(stream)
    torch.cuda.synchronize()
    lat.sync()
    return e0.elapsed_time(e1) / steps * 1e-3       # seconds per step


def make_lattice(L, storage, autotune=True):
    import torch
    import workloads as W
    from paper_1909_04502_amd import rlbm as R
    n, T, u = W.taylor_green_2d(L, L, 0.1, density_sigma=1e-3, seed=2)
    lat = R.Lattice(d=2, zeta=1.0, order=3, kind="product", extent=(L, L), storage=storage, tau=0.8)
    tune = lat.autotune(steps=10) if autotune else None
    fa = lat.init(torch.tensor(n), torch.tensor(T), torch.tensor(u))
    fb = lat.new_state()
    return lat, fa, fb, tune


def library_source_sha():
    import glob
    import hashlib
    files = []
    for pat in ("*.hip", "*.h", "*.cpp"):
        files += sorted(glob.glob(os.path.join(ROOT, "paper_1909_04502_amd", "csrc", pat)))
    h = hashlib.sha256()
    for f in files:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(name):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it matches this source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256_prefix") != library_source_sha():
        return None
    return rec["traffic_bytes"]


def copy_bandwidth(nbytes, planes=32, reps=20):
    """Device-to-device copies of nbytes (read + write bytes per second), the measured bandwidth
    references: torch's copy_, and the library's rlbm_copy_planes with the step kernel's access
    pattern (one site per thread, `planes` double planes) and as a flat 16-byte-vector copy, each with
    cached and non-temporal stores."""
    import torch
    from paper_1909_04502_amd import rlbm as R
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    kinds = {"torch_copy": lambda: b.copy_(a)}
    for mode in ("site", "flat"):
        for nt in (False, True):
            kinds[f"{mode}{'_nt' if nt else ''}"] = (lambda m=mode, t=nt: R.copy_planes(a, b, planes, m, t))
    out = {}
    for name, fn in kinds.items():
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / reps * 1e-3
        out[name] = round(2 * nbytes / t / 1e9, 1)
    assert torch.equal(a, b)
    del a, b
    torch.cuda.empty_cache()
    return out


def batched(count, warmup, steps, storage="f64", physics=False):
    """Many lattices (sides 64..512, tau in [0.6, 2], zeta in [0, 5], seed 4; Taylor-Green u0 = 0.05):
    one persistent launch per step (graph-replayed) against one launch per lattice per step."""
    import torch
    import workloads as W
    from paper_1909_04502_amd import rlbm as R
    specs = W.batch_specs(count, seed=4)
    b = R.Batch(specs, order=3, storage=storage)
    es = 8 if storage == "f64" else 4
    ns, Ts, us = [], [], []
    for i, sp in enumerate(specs):
        n, T, u = W.taylor_green_2d(*sp["extent"], 0.05, density_sigma=1e-3, seed=100 + i)
        ns.append(n), Ts.append(T), us.append(u)
    fa = b.init(ns, Ts, us)
    fb = b.new_state()
    del ns, Ts, us
    tune = b.autotune(fa, fb, steps=4)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    res = {}
    for graph in (True, False):
        b.step(fa, fb, warmup, graph=graph)
        b.step(fa, fb, steps, graph=graph)          # captures (graph) outside the timed region
        torch.cuda.synchronize()
        e0.record(stream)
        b.step(fa, fb, steps, graph=graph)
        e1.record(stream)
        torch.cuda.synchronize()
        res["graph" if graph else "eager"] = e0.elapsed_time(e1) / steps * 1e-3
    b.sync()
    # one launch per lattice per step, the same kernels' solo path
    views = [(m, b.view(fa, l), b.view(fb, l)) for l, m in enumerate(b.members)]
    ps = max(2, steps // 5)
    for m, va, vb in views:
        m.step(va, vb, 2)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(ps):
        for m, va, vb in views:
            m.step(va, vb, 1)
    e1.record(stream)
    torch.cuda.synchronize()
    t_solo = e0.elapsed_time(e1) / ps * 1e-3
    b.sync()
    # the configuration's whole run: 500 steps in one call (replays of the cached 256-step graph)
    run_steps = 500
    b.step(fa, fb, run_steps)
    torch.cuda.synchronize()
    e0.record(stream)
    b.step(fa, fb, run_steps)
    e1.record(stream)
    torch.cuda.synchronize()
    t_run = e0.elapsed_time(e1) / run_steps * 1e-3
    b.sync()
    sites = b.total_sites
    Q = b.Q
    t = res["graph"]
    out = {"lattices": count, "sites": sites, "MLUPS": round(sites / t / 1e6, 2), "ms_per_step": round(t * 1e3, 4),
           "eager_ms_per_step": round(res["eager"] * 1e3, 4),
           "per_lattice_launches_ms_per_step": round(t_solo * 1e3, 4),
           "speedup_vs_per_lattice": round(t_solo / t, 3),
           "achieved_GBs": round(2 * Q * es * sites / t / 1e9, 1),
           "frac": round(2 * Q * es * sites / t / 1e9 / HBM_PEAK_GBS, 4),
           "variant": b.variant, "autotune_ms": [round(x, 4) for x in tune],
           "run_500_steps_ms_per_step": round(t_run * 1e3, 4), "run_500_steps_MLUPS": round(sites / t_run / 1e6, 2),
           "workload": f"{count} lattices, sides U{{64..512}}, tau U[0.6,2], zeta U[0,5] (seed 4), N=3, {storage}"}
    if physics:
        out["shear_viscosity_fit"] = batch_viscosity_fit(b, specs)
    del b, fa, fb, views
    torch.cuda.empty_cache()
    return out


def batch_viscosity_fit(b, specs, steps=500, every=25, first=50):
    """The batched configuration's physics (untimed): a fresh Taylor-Green start run for its 500 steps,
    the amplitude of each lattice's mode (u_x projected on cos x sin y) every 25 steps, the decay rate
    gamma fitted from step 50 on, eta/P = gamma G_2(zeta) / (2 k^2) with G_2 = (zeta^2 + 3 zeta + 3) /
    (zeta + 1), and per zeta bin of width 1 the least-squares slope of eta/P against tau (with an
    intercept linear in zeta: interpolated streaming adds a tau-independent viscosity).  The tests
    compare each bin's slope with the Chapman-Enskog coefficient."""
    import numpy as np
    import torch
    import workloads as W
    ns, Ts, us = [], [], []
    for i, sp in enumerate(specs):
        n, T, u = W.taylor_green_2d(*sp["extent"], 0.05, density_sigma=1e-3, seed=100 + i)
        ns.append(n), Ts.append(T), us.append(u)
    fa = b.init(ns, Ts, us)
    fb = b.new_state()
    del ns, Ts, us
    modes = []
    for sp in specs:
        x = 2 * np.pi * np.arange(sp["extent"][0]) / sp["extent"][0]
        X, Y = np.meshgrid(x, x)
        modes.append(torch.tensor(np.cos(X) * np.sin(Y), device="cuda"))
    times = list(range(0, steps + 1, every))
    amps = np.zeros((len(specs), len(times)))
    for ti, t in enumerate(times):
        if t:
            r = b.step(fa, fb, every)
            if r is fb:
                fa, fb = fb, fa
        mom = b.moments(fa)
        amps[:, ti] = torch.stack([((m["U"][1] / m["U"][0]) * md).sum() / (md * md).sum()
                                   for m, md in zip(mom, modes)]).cpu().numpy()
    b.sync()
    sel = [i for i, t in enumerate(times) if t >= first]
    tt = np.array([times[i] for i in sel])
    tau = np.array([sp["tau"] for sp in specs])
    zeta = np.array([sp["zeta"] for sp in specs])
    gam = np.array([-np.polyfit(tt, np.log(np.abs(amps[l, sel])), 1)[0] for l in range(len(specs))])
    k = 2 * np.pi / np.array([sp["extent"][0] for sp in specs])
    y = gam * (zeta * zeta + 3 * zeta + 3) / (zeta + 1) / (2 * k * k)
    bins = []
    for lo in range(5):
        m = (zeta >= lo) & (zeta < lo + 1)
        A = np.stack([tau[m] - 0.5, np.ones(m.sum()), zeta[m] - zeta[m].mean()], 1)
        coef, *_ = np.linalg.lstsq(A, y[m], rcond=None)
        bins.append({"zeta_bin": [lo, lo + 1], "lattices": int(m.sum()), "mean_zeta": round(float(zeta[m].mean()), 4),
                     "eta_over_P_slope": round(float(coef[0]), 5)})
    return {"steps": steps, "fit_from_step": first, "per_zeta_bin": bins}


def adjoint_leg(L, warmup, steps):
    """Reverse step (rlbm_adjoint_step) against the forward step, 512 x 512 float-deviation storage with
    a tau field; algorithmic bytes of the reverse step: read B_{t-1} and lam_{t+1}, write lam_t (3 Q s per
    site) plus the dL/dtau accumulator (16 B per site)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1909_04502_amd import rlbm as R
    n, T, u = W.taylor_green_2d(L, L, 0.1, density_sigma=1e-3, seed=2)
    tau = torch.tensor(0.8 + 0.2 * np.random.default_rng(4).uniform(-1, 1, (L, L)))
    lat = R.Lattice(d=2, zeta=1.0, order=3, extent=(L, L), storage="f32dev", tau=0.8, tau_field=tau)
    fa = lat.init(torch.tensor(n), torch.tensor(T), torch.tensor(u))
    fb = lat.new_state()
    t_fwd = time_steps(lat, fa, fb, warmup, steps)
    lam_a = torch.randn_like(fa) * 1e-3
    lam_b = torch.empty_like(fa)
    dtau = torch.zeros((L, L), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        lat.adjoint_step(fa, lam_a, lam_b, dtau)
        lam_a, lam_b = lam_b, lam_a
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        lat.adjoint_step(fa, lam_a, lam_b, dtau)
        lam_a, lam_b = lam_b, lam_a
    e1.record(stream)
    torch.cuda.synchronize()
    lat.sync()
    t_adj = e0.elapsed_time(e1) / steps * 1e-3
    sites = L * L
    Q = lat.Q
    ab = (3 * Q * 4 + 16) * sites
    # the whole differentiable run: forward with checkpoints every 45 steps, then the backward pass
    # (segment recompute + reverse steps + the initial-condition VJP) through the autograd Function
    from paper_1909_04502_amd import adjoint as A
    nrun = 2000
    _, _, ut = W.taylor_green_2d(L, L, 0.08, phase=(0.3, -0.2))
    ut = torch.tensor(ut, device="cuda")
    n_t, T_t = torch.tensor(n), torch.tensor(T)
    for rep in range(2):                 # the first run captures the segment graphs; the second is timed
        taug = tau.clone().cuda().requires_grad_(True)
        u0g = torch.tensor(u).cuda().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U = A.run(lat, taug, u0g, n_t, T_t, nrun, every=45)
        loss = A.velocity_loss(U, ut)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    gt45, gu45 = taug.grad.clone(), u0g.grad.clone()
    # the same run with every state kept (2001 states of 33.5 MB, 67 GB of HBM): no segment recompute
    taug = tau.clone().cuda().requires_grad_(True)
    u0g = torch.tensor(u).cuda().requires_grad_(True)
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    U = A.run(lat, taug, u0g, n_t, T_t, nrun, every=1)
    loss = A.velocity_loss(U, ut)
    torch.cuda.synchronize()
    s1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    s2 = time.perf_counter()
    store_all = {"forward_ms_per_step": round((s1 - s0) / nrun * 1e3, 5),
                 "backward_ms_per_step": round((s2 - s1) / nrun * 1e3, 5),
                 "backward_over_forward_step": round((s2 - s1) / nrun / t_fwd, 3),
                 "state_GB": round((nrun + 1) * lat.Q * 4 * L * L / 1e9, 1),
                 "gradient_equals_checkpointed": bool(torch.equal(taug.grad, gt45) and torch.equal(u0g.grad, gu45))}
    del U, loss, taug, u0g, gt45, gu45
    torch.cuda.empty_cache()
    out = {"workload": f"{L}x{L} zeta=1 N=3 f32dev with tau field", "forward_ms": round(t_fwd * 1e3, 5),
           "run_steps": nrun, "run_checkpoint_every": 45,
           "run_forward_ms_per_step": round((t1 - t0) / nrun * 1e3, 5),
           "run_backward_ms_per_step": round((t2 - t1) / nrun * 1e3, 5),
           "run_backward_over_forward": round((t2 - t1) / (t1 - t0), 3),
           "run_forward_over_step_kernel": round((t1 - t0) / nrun / t_fwd, 3),
           "adjoint_ms": round(t_adj * 1e3, 5), "adjoint_over_forward": round(t_adj / t_fwd, 3),
           "adjoint_MLUPS": round(sites / t_adj / 1e6, 2), "adjoint_achieved_GBs": round(ab / t_adj / 1e9, 1),
           "adjoint_frac": round(ab / t_adj / 1e9 / HBM_PEAK_GBS, 4),
           "run_store_all_states": store_all}
    del lat, fa, fb, lam_a, lam_b
    torch.cuda.empty_cache()
    return out


def shock_tube_3d(L, warmup, steps, autotune=True, storage="f32dev"):
    """3D shock tube: zeta = 1, N = 3, Q = 104, L^3 with open x and periodic y, z, left state n = 8/3,
    T = 1.5 for x < L/2, right n = 1, T = 1, u = 0; float-deviation storage (832 B per site), updated
    in float (f32dev) or in double (f32dev_f64).  Timed at
    tau = 0.8, the set-up the 2000-step parity run validates: at tau = 0.6 the scheme itself (the FP64
    oracle on the same set-up) turns non-physical at step 113; the step costs the same at any tau."""
    import torch
    import workloads as W
    from paper_1909_04502_amd import rlbm as R
    n, T, u = W.riemann_3d(L, L, L, L // 2, 8.0 / 3.0, 1.5, 1.0, 1.0)
    lat = R.Lattice(d=3, zeta=1.0, order=3, extent=(L, L, L), bc=("open", "periodic", "periodic"),
                    storage=storage, tau=0.8)
    tune = lat.autotune(steps=3) if autotune else None
    fa = lat.init(torch.tensor(n), torch.tensor(T), torch.tensor(u))
    del n, T, u
    fb = lat.new_state()
    t = time_steps(lat, fa, fb, warmup, steps)
    sites = L ** 3
    b = 2 * lat.Q * 4 * sites
    out = {"workload": f"3D shock tube {L}^3, zeta=1 N=3 Q={lat.Q}, open x, tau=0.8 (the validated set-up; "
                       f"tau=0.6 turns non-physical at step 113 in the FP64 oracle itself), {storage}",
           "MLUPS": round(sites / t / 1e6, 2), "ms_per_step": round(t * 1e3, 4),
           "achieved_GBs": round(b / t / 1e9, 1), "frac": round(b / t / 1e9 / HBM_PEAK_GBS, 4),
           "variant": lat.variant, "autotune_ms": [round(x, 4) for x in tune] if tune else None}
    del lat, fa, fb
    torch.cuda.empty_cache()
    return out


def onlattice_leg(warmup, steps):
    """The printed ultra-relativistic on-lattice rule (d = 2, zeta = 0, N = 2, Q = 28, integer shifts), FP64:
    the 64 x 64 Taylor-Green configuration (u0 = 0.01, tau = 0.9, population noise 1e-6, seed 1; launch
    bound at this size) and the same rule on 1024 x 1024 (448 algorithmic bytes per site)."""
    import torch
    import workloads as W
    from paper_1909_04502_amd import rlbm as R
    out = {}
    for L in (64, 1024):
        n, T, u = W.taylor_green_2d(L, L, 0.01, seed=2)
        lat = R.Lattice(d=2, zeta=0.0, order=2, kind="ur_onlattice", extent=(L, L), tau=0.9)
        xi = torch.tensor(W.population_noise(lat.Q, (L, L), seed=1))
        fa = lat.init(torch.tensor(n), torch.tensor(T), torch.tensor(u), xi, 1e-6)
        fb = lat.new_state()
        t = time_steps(lat, fa, fb, warmup, steps)
        b = 2 * lat.Q * 8 * L * L
        out[f"{L}x{L}"] = {"MLUPS": round(L * L / t / 1e6, 2), "ms_per_step": round(t * 1e3, 5),
                           "achieved_GBs": round(b / t / 1e9, 1), "frac": round(b / t / 1e9 / HBM_PEAK_GBS, 4)}
        del lat, fa, fb
    torch.cuda.empty_cache()
    return out


def massive_leg(warmup, steps):
    """Massive on-lattice rules (Sec. 5.3) at zeta = 5, Taylor-Green start (u0 = 0.1, density noise 1e-3,
    seed 2), periodic, tau = 0.8, v0 the middle of the admissible window: the 45-vector order-3 stencil on
    the 512 x 512 lattice of the paper's GPU benchmark (FP64 and float deviations) and on 2048 x 2048
    (beyond the 256 MB last-level cache), the 29-vector order-2 stencil on 512 x 512, and the (3+1)-d
    143-vector stencil on the 192^3 lattice of the paper's 3D benchmark (3D Taylor-Green start; a tenth
    of the steps).  Algorithmic bytes per site: 2 Q x element size."""
    import torch
    import workloads as W
    from paper_1909_04502_amd import rlbm as R
    out = {}
    for name, d, order, L, storage in (("n3_512", 2, 3, 512, "f64"), ("n3_512_f32dev", 2, 3, 512, "f32dev"),
                                       ("n3_2048", 2, 3, 2048, "f64"), ("n2_512", 2, 2, 512, "f64"),
                                       ("d3_192", 3, 3, 192, "f64"), ("d3_192_f32dev", 3, 3, 192, "f32dev")):
        if d == 2:
            n, T, u = W.taylor_green_2d(L, L, 0.1, density_sigma=1e-3, seed=2)
        else:
            n, T, u = W.taylor_green_3d(L, L, L, 0.1, density_sigma=1e-3, seed=2)
        ext = (L,) * d
        lat = R.Lattice(d=d, zeta=5.0, order=order, kind="massive_onlattice", extent=ext, tau=0.8,
                        storage=storage)
        fa = lat.init(torch.tensor(n), torch.tensor(T), torch.tensor(u))
        fb = lat.new_state()
        k = steps if d == 2 else max(2, steps // 10)
        t = time_steps(lat, fa, fb, warmup if d == 2 else 2, k)
        sites = L ** d
        b = 2 * lat.Q * (8 if storage == "f64" else 4) * sites
        out[name] = {"Q": lat.Q, "v0": lat.v0, "MLUPS": round(sites / t / 1e6, 2), "ms_per_step": round(t * 1e3, 5),
                     "achieved_GBs": round(b / t / 1e9, 1), "frac": round(b / t / 1e9 / HBM_PEAK_GBS, 4)}
        del lat, fa, fb
        torch.cuda.empty_cache()
    torch.cuda.empty_cache()
    return out


def sod_leg(warmup, steps):
    """The ultra-relativistic Sod tube of the paper's inviscid test with the printed order-3 massless
    rule (Q = 44, integer shifts, FP64): 6400 x 5 sites (a mirror-periodic tube, uniform across the
    five rows), tau = 1/2 + tau_T / T for eta/s = 0.002, 300 steps to t = 3.0 fm/c (its agreement
    with App. D is checked by the tests); and the same rule on a 1024 x 1024 Taylor-Green lattice for
    throughput (704 algorithmic bytes per site)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1909_04502_amd import rlbm as R
    out = {}
    nx, ny, split, nsteps = 6400, 5, 1600, 300
    PL, PR, TR = 1.0, 1.0 / 5.43, 0.475
    nR = PR / TR
    k = np.arange(nx)
    left = np.where(k < nx // 2, k, nx - 1 - k) < split
    n = torch.tensor(np.where(left, 1.0, nR)[None, :] * np.ones((ny, 1)))
    T = torch.tensor(np.where(left, 1.0, TR)[None, :] * np.ones((ny, 1)))
    u = torch.zeros((2, ny, nx), dtype=torch.float64)
    tau_T = 0.002 * 3 / 0.75 * (197.327 / 400.0) / 0.01
    lat = R.Lattice(d=2, zeta=0.0, order=3, kind="ur_onlattice", extent=(nx, ny), tau=0.5, tau_T=tau_T)
    fa = lat.init(n, T, u)
    fb = lat.new_state()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    lat.step(fa, fb, nsteps)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3
    lat.sync()
    out["sod_6400x5"] = {"steps": nsteps, "ms_total": round(t * 1e3, 3), "MLUPS": round(nx * ny * nsteps / t / 1e6, 1)}
    del lat, fa, fb
    # the same tube in (3+1) dimensions: the printed order-3 rule of App. H.1 (288 populations), light
    # crossing sqrt(41) sites per step (234 steps to t = 3.0 fm/c), open y and z (one row)
    import math
    nsteps3 = 234
    n3 = torch.tensor(np.where(left, 1.0, nR)[None, None, :])
    T3 = torch.tensor(np.where(left, 1.0, TR)[None, None, :])
    u3 = torch.zeros((3, 1, 1, nx), dtype=torch.float64)
    tau_T3 = 0.002 * 4 / 0.8 * (197.327 / 400.0) / (math.sqrt(41.0) * 0.002)
    lat = R.Lattice(d=3, zeta=0.0, order=3, kind="ur_onlattice", extent=(nx, 1, 1), bc=("periodic", "open", "open"),
                    tau=0.5, tau_T=tau_T3)
    fa = lat.init(n3, T3, u3)
    fb = lat.new_state()
    lat.step(fa, fb, 2)
    torch.cuda.synchronize()
    e0.record()
    lat.step(fa, fb, nsteps3)
    e1.record()
    torch.cuda.synchronize()
    t3 = e0.elapsed_time(e1) * 1e-3
    lat.sync()
    out["sod3d_6400x1x1"] = {"Q": lat.Q, "steps": nsteps3, "ms_total": round(t3 * 1e3, 3),
                             "MLUPS": round(nx * nsteps3 / t3 / 1e6, 1)}
    del lat, fa, fb
    L = 1024
    n, T, u = W.taylor_green_2d(L, L, 0.01, seed=2)
    lat = R.Lattice(d=2, zeta=0.0, order=3, kind="ur_onlattice", extent=(L, L), tau=0.9)
    fa = lat.init(torch.tensor(n), torch.tensor(T), torch.tensor(u))
    fb = lat.new_state()
    t = time_steps(lat, fa, fb, warmup, steps)
    b = 2 * lat.Q * 8 * L * L
    out["ur3_1024x1024"] = {"MLUPS": round(L * L / t / 1e6, 2), "ms_per_step": round(t * 1e3, 5),
                            "achieved_GBs": round(b / t / 1e9, 1), "frac": round(b / t / 1e9 / HBM_PEAK_GBS, 4)}
    del lat, fa, fb
    torch.cuda.empty_cache()
    return out


def calibration_leg():
    """The transport calibrations on the 45-vector massive rule (zeta = 5, exact streaming), as the tests
    run them: the thermal conductivity lambda / (n tau) of a 200-site rod between plates at T = 1.005 and
    0.995 after 40,000 steps (steady Eckart heat flux over the interior) and the bulk viscosity
    mu / (P tau) of a 1600-site periodic sine wave (u0 = 1e-5) by least squares over half a sound
    period, both from pre-collision moments, tau = 1; with the wall-clock time of each run (the
    Chapman-Enskog values are 0.27832 and 0.0054534)."""
    import time
    import numpy as np
    import torch
    from paper_1909_04502_amd import rlbm as R
    out = {}
    p, w, disp = R.quadrature_build(2, 5.0, 3, "massive_onlattice")
    disp = disp.numpy()
    p = p.cuda()

    def streamed(lat, fs):
        return torch.stack([torch.roll(fs[i], shifts=(int(disp[i, 1]), int(disp[i, 0])), dims=(0, 1))
                            for i in range(lat.Q)])
    L, ny, tau = 200, 4, 1.0
    t0 = time.time()
    lat = R.Lattice(d=2, zeta=5.0, order=3, kind="massive_onlattice", extent=(L, ny), tau=tau,
                    bc=("wall", "periodic"), wall_T=((1.005, 0.995), (0.0, 0.0)))
    v0 = lat.v0
    ones = torch.ones((ny, L), dtype=torch.float64)
    fa = lat.init(ones, ones, torch.zeros((2, ny, L), dtype=torch.float64))
    fb = lat.new_state()
    lat.step(fa, fb, 40000)
    mac = lat.moments(fa)
    f = streamed(lat, fa)
    Nx = torch.einsum("i,i...->...", p[:, 1], f)
    h = (mac["eps"] + mac["n"] * mac["T"]) / mac["n"]
    qx = h * (mac["n"] * mac["U"][1] - Nx)
    dT = (torch.roll(mac["T"], -1, 1) - torch.roll(mac["T"], 1, 1)) / (2 * v0)
    inner = slice(10, L - 10)
    lam = -(qx[:, inner].mean() / dT[:, inner].mean()).item()
    out["thermal_conductivity"] = {"lambda_over_n_tau": round(lam / (mac["n"][:, inner].mean().item() * tau), 6),
                                   "steps": 40000, "seconds": round(time.time() - t0, 3)}
    del lat, fa, fb
    L, u0 = 1600, 1e-5
    t0 = time.time()
    lat = R.Lattice(d=2, zeta=5.0, order=3, kind="massive_onlattice", extent=(L, ny), tau=tau)
    u = np.zeros((2, ny, L))
    u[0] = u0 * np.sin(2 * np.pi * np.arange(L) / L)[None, :]
    ones = torch.ones((ny, L), dtype=torch.float64)
    fa = lat.init(ones, ones, torch.tensor(u))
    fb = lat.new_state()
    num = den = 0.0
    for s in range(10, 461, 10):
        lat.step(fa, fb, 10)
        if s < 40:
            continue
        mac = lat.moments(fa)
        f = streamed(lat, fa)
        P = mac["n"] * mac["T"]
        varpi = -(25.0 * f.sum(0) - (mac["eps"] - 2 * P)) / 2
        div = (torch.roll(mac["U"][1], -1, 1) - torch.roll(mac["U"][1], 1, 1)) / (2 * v0)
        num += -(varpi * div).sum().item() / P.mean().item()
        den += (div * div).sum().item()
    lat.sync()
    out["bulk_viscosity"] = {"mu_over_P_tau": round(num / den / tau, 7), "steps": 460,
                             "seconds": round(time.time() - t0, 3)}
    torch.cuda.empty_cache()
    return out


def staged_large_leg(warmup, steps, L=2048):
    """The 2D product rule (zeta = 1, N = 3) at L x L in each storage, where the two state buffers
    exceed 384 MiB: the default launch (the LDS-staged step) against the register kernel that is the
    default below that size.  Algorithmic bytes per site: 2 Q x element size."""
    import torch
    import workloads as W
    from paper_1909_04502_amd import rlbm as R
    n, T, u = (torch.tensor(a) for a in W.taylor_green_2d(L, L, 0.1, density_sigma=1e-3, seed=2))
    out = {"workload": f"2D zeta=1 N=3 Q=32 {L}x{L} periodic, Taylor-Green u0=0.1, tau=0.8"}
    for storage, reg in (("f64", 5), ("f32dev", 10), ("f32dev_f64", 9)):
        lat = R.Lattice(d=2, zeta=1.0, order=3, kind="product", extent=(L, L), storage=storage, tau=0.8)
        b = 2 * lat.Q * (8 if storage == "f64" else 4) * L * L
        row = {}
        for name, v in (("default", lat.variant), ("register", reg)):
            lat.variant = v
            fa = lat.init(n, T, u)
            fb = lat.new_state()
            t = time_steps(lat, fa, fb, warmup, steps)
            row[name] = {"variant": v, "ms_per_step": round(t * 1e3, 5), "MLUPS": round(L * L / t / 1e6, 2),
                         "frac": round(b / t / 1e9 / HBM_PEAK_GBS, 4)}
            del fa, fb
        out[storage] = row
        del lat
        torch.cuda.empty_cache()
    return out


def forcing_leg(L, warmup, steps):
    """The headline workload with the external force of Sec. 5.4 (scheme B, g = 1e-6 along y) and no-slip
    equilibrium walls on the x faces: the force/wall build of the step kernel."""
    import torch
    import workloads as W
    from paper_1909_04502_amd import rlbm as R
    n, T, u = W.taylor_green_2d(L, L, 0.1, density_sigma=1e-3, seed=2)
    lat = R.Lattice(d=2, zeta=1.0, order=3, extent=(L, L), bc=("wall", "periodic"), tau=0.8, force=(0.0, 1e-6))
    fa = lat.init(torch.tensor(n), torch.tensor(T), torch.tensor(u))
    fb = lat.new_state()
    t = time_steps(lat, fa, fb, warmup, steps)
    b = 2 * lat.Q * 8 * L * L
    out = {"workload": f"{L}x{L} zeta=1 N=3 f64, walls on x, g = 1e-6 along y", "MLUPS": round(L * L / t / 1e6, 2),
           "ms_per_step": round(t * 1e3, 5), "achieved_GBs": round(b / t / 1e9, 1),
           "frac": round(b / t / 1e9 / HBM_PEAK_GBS, 4)}
    del lat, fa, fb
    torch.cuda.empty_cache()
    return out


def cpu_baseline(seconds):
    """The FP64 oracle (as it stands) on a 128 x 128 lattice of the same workload, on this host's cores.
    The same leg states the error of the GPU path on that sample: the FP64 and float-deviation
    libraries' populations and moments after the oracle's first 10 steps, max-normalised."""
    import torch
    import workloads as W
    from oracle import lattice as OL
    from oracle import quadrature as qd
    from paper_1909_04502_amd import rlbm as R
    L, KERR = 128, 10
    n, T, u = (torch.tensor(a) for a in W.taylor_green_2d(L, L, 0.1, density_sigma=1e-3, seed=2))
    ol = OL.Lattice(qd.product_2d(1.0, 3), 0.8, (L, L))
    f = ol.collide(ol.init(n, T, u))
    for _ in range(KERR):                       # untimed: the reference for the error statement
        f = ol.collide(ol.stream(f))
    ref = (f.clone(), ol.macro(ol.stream(f)))
    def timed(budget, f):
        steps = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget or steps < 2:
            f = ol.collide(ol.stream(f))
            steps += 1
        return steps, time.perf_counter() - t0, f
    threads = torch.get_num_threads()
    steps, dt, f = timed(seconds, f)
    torch.set_num_threads(1)
    try:
        steps1, dt1, _ = timed(seconds / 3.0, f)
    finally:
        torch.set_num_threads(threads)
    errors = {"steps": KERR, "lattice": f"{L}x{L}"}
    for storage in ("f64", "f32dev", "f32dev_f64"):
        lat = R.Lattice(d=2, zeta=1.0, order=3, extent=(L, L), tau=0.8, storage=storage)
        res = lat.step(lat.init(n, T, u), lat.new_state(), KERR)
        mom = lat.moments(res)
        lat.sync()

        def rel(a, b):
            a = a.detach().cpu().to(torch.float64)
            return float((a - b).abs().max() / b.abs().max())
        e = {k: rel(mom[k], ref[1][k]) for k in ("n", "eps", "T")}
        e["U"] = rel(mom["U"][1:], ref[1]["U"][1:])
        if storage == "f64":
            e["f"] = rel(res, ref[0])
        errors[storage] = {k: float(f"{v:.2e}") for k, v in e.items()}
        del lat, res
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": L * L * steps / dt / 1e6, "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} steps of a {L}x{L} lattice of the same workload ({dt:.1f} s, torch float64 on CPU)",
            "one_core": {"value": L * L * steps1 / dt1 / 1e6, "unit": "MLUPS", "cores": 1,
                         "sample": f"{steps1} steps of the same {L}x{L} lattice ({dt1:.1f} s)"},
            "cpu": model, "host_cpus": os.cpu_count(), "gpu_error_vs_oracle": errors}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the lattice update runs "
              "on a single GPU", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    L = args.size
    Q = 32
    sites = L * L
    lat, fa, fb, tune = make_lattice(L, "f64", args.autotune)
    t = time_steps(lat, fa, fb, args.warmup, args.steps)
    mlups = sites / t / 1e6
    bytes_step = 2 * Q * 8 * sites
    achieved = bytes_step / t / 1e9
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D RLBM zeta=1 N=3 Q=32 off-lattice, {L}x{L} periodic, Taylor-Green u0=0.1, "
                               f"tau=0.8, density noise 1e-3 (seed 2)",
                   "sites": sites, "Q": Q, "storage": "f64"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("traffic_k_step_prod2d_f64_1024x1024.json"),
                     "algorithmic_bytes_per_site": 2 * Q * 8},
    }
    # launch variant 12 runs the LDS-staged kernel; the others the register kernel
    out["roofline"]["kernel"] = ("k_step_lds" if lat.variant == 12 else "k_step") + "<Stencil<PROD2D,4>,3,double>"
    if tune is not None:
        out["autotune"] = {"variant": lat.variant, "ms_per_step": [round(x, 5) for x in tune]}
    out["roofline"]["launch_variant"] = lat.variant
    out["roofline"]["stores"] = "nontemporal" if lat.nontemporal_stores else "cached"
    del lat, fa, fb
    torch.cuda.empty_cache()
    if not args.no_variants:
        lat, fa, fb, tune32 = make_lattice(L, "f32dev", args.autotune)
        t32 = time_steps(lat, fa, fb, args.warmup, args.steps)
        b32 = 2 * Q * 4 * sites
        out["variants"] = {"f32dev": {"MLUPS": round(sites / t32 / 1e6, 2), "ms_per_step": round(t32 * 1e3, 5),
                                      "achieved_GBs": round(b32 / t32 / 1e9, 1),
                                      "frac": round(b32 / t32 / 1e9 / HBM_PEAK_GBS, 4),
                                      "variant": lat.variant,
                                      "autotune_ms": [round(x, 5) for x in tune32] if tune32 else None}}
        del lat, fa, fb
        torch.cuda.empty_cache()
        # float storage, double arithmetic: float traffic, errors that do not grow with the run
        lat, fa, fb, tunem = make_lattice(L, "f32dev_f64", args.autotune)
        tm = time_steps(lat, fa, fb, args.warmup, args.steps)
        out["variants"]["f32dev_f64"] = {"MLUPS": round(sites / tm / 1e6, 2), "ms_per_step": round(tm * 1e3, 5),
                                         "achieved_GBs": round(b32 / tm / 1e9, 1),
                                         "frac": round(b32 / tm / 1e9 / HBM_PEAK_GBS, 4),
                                         "variant": lat.variant,
                                         "autotune_ms": [round(x, 5) for x in tunem] if tunem else None}
        del lat, fa, fb
        torch.cuda.empty_cache()
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(512, args.warmup, args.steps)
    if not args.no_3d:
        out["shock_tube_3d"] = shock_tube_3d(args.size_3d, max(2, args.warmup // 4), max(4, args.steps // 10),
                                             args.autotune)
        out["shock_tube_3d_f32dev_f64"] = shock_tube_3d(args.size_3d, max(2, args.warmup // 4),
                                                        max(4, args.steps // 10), args.autotune, "f32dev_f64")
    if not args.no_batch:
        out["batched"] = batched(args.batch_count, max(2, args.warmup // 4), max(4, args.steps // 10))
        out["batched_f32dev"] = batched(args.batch_count, max(2, args.warmup // 4), max(4, args.steps // 10),
                                        "f32dev", physics=True)
    if not args.no_onlattice:
        want = (lambda name: args.only in (None, name))
        if want("onlattice_ur"):
            out["onlattice_ur"] = onlattice_leg(args.warmup, args.steps)
        if want("massive_onlattice"):
            out["massive_onlattice"] = massive_leg(args.warmup, args.steps)
        if want("sod_ur"):
            out["sod_ur"] = sod_leg(args.warmup, args.steps)
        if want("calibrations"):
            out["calibrations"] = calibration_leg()
    if not args.no_forcing:
        out["forcing_walls"] = forcing_leg(L, args.warmup, args.steps)
    if not args.no_staged_large:
        out["staged_large"] = staged_large_leg(args.warmup, args.steps)
    if not args.no_copy:
        cb = copy_bandwidth(Q * 8 * sites, planes=Q)
        best = max(cb.values())
        out["roofline"]["copy_GBs"] = cb
        out["roofline"]["copy_ceiling_GBs"] = best
        out["roofline"]["frac_of_copy"] = round(achieved / best, 4)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
