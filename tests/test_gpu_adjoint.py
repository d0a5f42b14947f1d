"""GPU reverse mode: adjoint kernels against the oracle gradient and finite differences.

* the full gradient (dL/dtau field, dL/du0) of a run through the
  autograd.Function (checkpointed) vs the oracle's float64 autograd gradient;
* one adjoint step against central differences of one forward step
  (<J v, w> = <v, J^T w>);
* central differences of the GPU forward (h = 1e-4) along seeded directions;
* the float-deviation storage gradient against the double one.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import grad as OG
from oracle import lattice as OL
from oracle import quadrature as qd

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = a.detach().cpu().to(torch.float64)
    b = b.detach().cpu().to(torch.float64)
    return ((a - b).abs().max() / b.abs().max()).item()


def problem(nx, ny, zeta=1.0, order=3, seed=4):
    n, T, u = W.taylor_green_2d(nx, ny, 0.1, density_sigma=1e-3, seed=2)
    g = np.random.default_rng(seed)
    tau = 0.8 + 0.2 * g.uniform(-1, 1, (ny, nx))
    _, _, ut = W.taylor_green_2d(nx, ny, 0.08, phase=(0.3, -0.2))
    return [torch.tensor(a) for a in (n, T, u, tau, ut)]


def gpu_gradient(nx, ny, nsteps, every, storage="f64", zeta=1.0, order=3):
    from paper_1909_04502_amd import adjoint as A
    from paper_1909_04502_amd import rlbm as R
    n, T, u, tau, ut = problem(nx, ny, zeta, order)
    lat = R.Lattice(d=2, zeta=zeta, order=order, extent=(nx, ny), storage=storage, tau=0.8,
                    tau_field=tau.clone())
    taug = tau.clone().cuda().requires_grad_(True)
    u0g = u.clone().cuda().requires_grad_(True)
    U = A.run(lat, taug, u0g, n, T, nsteps, every=every)
    L = A.velocity_loss(U, ut.cuda())
    L.backward()
    return L.item(), taug.grad.detach(), u0g.grad.detach()


@pytest.mark.parametrize("nsteps,every", [(1, 1), (5, 2)])
def test_gradient_matches_oracle(nsteps, every):
    print(f"[case] adjoint vs oracle nsteps={nsteps}", flush=True)
    nx, ny = 24, 20
    L, gtau, gu0 = gpu_gradient(nx, ny, nsteps, every)
    n, T, u, tau, ut = problem(nx, ny)
    lat = OL.Lattice(qd.product_2d(1.0, 3), 0.8, (nx, ny))
    L0, gtau0, gu00 = OG.gradient(lat, n, T, u, tau, nsteps, ut)
    assert abs(L - L0.item()) / abs(L0.item()) < 1e-12
    print("dtau rel err", rel(gtau, gtau0), "du0 rel err", rel(gu0, gu00), flush=True)
    assert rel(gtau, gtau0) < 1e-10
    assert rel(gu0, gu00) < 1e-10


def test_single_adjoint_step_dot_product():
    """<w, (step(B + h v) - step(B - h v)) / 2h> == <v, adjoint(B, w)> (S^T and J_C^T together)."""
    from paper_1909_04502_amd import rlbm as R
    print("[case] adjoint dot product", flush=True)
    nx, ny = 20, 12
    n, T, u, tau, ut = problem(nx, ny)
    lat = R.Lattice(d=2, zeta=1.0, order=3, extent=(nx, ny), tau=0.8, tau_field=tau.clone())
    B = lat.init(n, T, u)
    g = np.random.default_rng(5)
    v = torch.tensor(g.normal(size=B.shape), device="cuda") * 1e-3 * B.abs().mean()
    w = torch.tensor(g.normal(size=B.shape), device="cuda")
    h = 1e-4
    Bp, Bm = lat.new_state(), lat.new_state()
    lat.step(B + h * v, Bp, 1)
    lat.step(B - h * v, Bm, 1)
    dB = (Bp - Bm) / (2 * h)
    lam = lat.adjoint_step(B, w)
    lat.sync()
    # lam = J_C(S B)^T S^T w is the adjoint of F_t -> F_{t+1}; with F_t = S B:
    # <lam, S v> = <w, S dB>  (streaming applied with the oracle's operator)
    ol = OL.Lattice(qd.product_2d(1.0, 3), 0.8, (nx, ny))
    lhs = (lam.cpu() * ol.stream(v.cpu())).sum().item()
    rhs = (w.cpu() * ol.stream(dB.cpu())).sum().item()
    assert abs(lhs - rhs) <= 1e-6 * abs(rhs)


def test_gradient_central_differences_gpu():
    """Directional central differences (h = 1e-4) of the GPU forward along seeded directions."""
    from paper_1909_04502_amd import adjoint as A
    from paper_1909_04502_amd import rlbm as R
    print("[case] adjoint vs FD", flush=True)
    nx, ny, nsteps = 32, 32, 20
    L, gtau, gu0 = gpu_gradient(nx, ny, nsteps, every=7)
    n, T, u, tau, ut = problem(nx, ny)
    lat = R.Lattice(d=2, zeta=1.0, order=3, extent=(nx, ny), tau=0.8, tau_field=tau.clone())

    def loss(tau_, u_):
        with torch.no_grad():
            U = A.run(lat, tau_.cuda(), u_.cuda(), n, T, nsteps, every=nsteps)
            return A.velocity_loss(U, ut.cuda()).item()

    g = np.random.default_rng(8)
    for _ in range(2):
        dt = torch.tensor(g.normal(size=tau.shape))
        du = torch.tensor(g.normal(size=u.shape)) * 0.05
        h = 1e-4
        fd = (loss(tau + h * dt, u + h * du) - loss(tau - h * dt, u - h * du)) / (2 * h)
        an = (gtau.cpu() * dt).sum().item() + (gu0.cpu() * du).sum().item()
        print("FD", fd, "adjoint", an, flush=True)
        assert abs(fd - an) <= 1e-6 * abs(an)


def test_float_deviation_gradient_vs_double():
    print("[case] adjoint f32dev", flush=True)
    nx, ny, nsteps = 32, 24, 10
    L64, gt64, gu64 = gpu_gradient(nx, ny, nsteps, every=4, storage="f64")
    L32, gt32, gu32 = gpu_gradient(nx, ny, nsteps, every=4, storage="f32dev")
    et, eu = rel(gt32, gt64), rel(gu32, gu64)
    print("f32dev gradient errors", et, eu, flush=True)
    assert abs(L32 - L64) / abs(L64) < 1e-4
    assert et < 2e-3 and eu < 2e-3


def test_reverse_mode_rejects_unsupported_lattices():
    from paper_1909_04502_amd import rlbm as R
    lat = R.Lattice(d=2, zeta=1.0, order=3, extent=(8, 8), bc=("open", "periodic"), tau=0.8)
    B = lat.new_state().zero_()
    with pytest.raises(R.RLBMError) as e:
        lat.adjoint_step(B, B.clone())
    assert e.value.status == R.ERR_UNSUPPORTED
