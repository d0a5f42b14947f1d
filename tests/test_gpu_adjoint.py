"""GPU reverse mode: adjoint kernels against the oracle gradient and finite differences.

* the full gradient (dL/dtau field, dL/du0) of a run through the
  autograd.Function (checkpointed) vs the oracle's float64 autograd gradient;
* one adjoint step against central differences of one forward step
  (<J v, w> = <v, J^T w>);
* central differences of the GPU forward (h = 1e-4) along seeded directions;
* the float-deviation storage gradient against the double one;
* one reverse step at C5's full size (512 x 512), sampled sites against the oracle's VJP.
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


def test_interleaved_runs_keep_their_own_tau():
    """Two differentiable runs on one lattice with different tau fields, then the backward of the
    first: its gradient equals that of a lone forward and backward (the second run overwrites the
    lattice's tau buffer and its work buffers in between)."""
    from paper_1909_04502_amd import adjoint as A
    from paper_1909_04502_amd import rlbm as R
    print("[case] interleaved runs", flush=True)
    nx, ny, nsteps, every = 24, 20, 6, 4
    n, T, u, tau, ut = problem(nx, ny)
    _, _, _, tau2, _ = problem(nx, ny, seed=11)
    lat = R.Lattice(d=2, zeta=1.0, order=3, extent=(nx, ny), tau=0.8, tau_field=tau.clone())
    grads = []
    for interleave in (False, True):
        taug = tau.clone().cuda().requires_grad_(True)
        u0g = u.clone().cuda().requires_grad_(True)
        L1 = A.velocity_loss(A.run(lat, taug, u0g, n, T, nsteps, every=every), ut.cuda())
        if interleave:
            t2 = tau2.clone().cuda().requires_grad_(True)
            u2 = (0.5 * u).clone().cuda().requires_grad_(True)
            L2 = A.velocity_loss(A.run(lat, t2, u2, n, T, nsteps, every=every), ut.cuda())
            assert abs(L2.item() - L1.item()) > 1e-9 * abs(L1.item())
        L1.backward()
        grads.append((L1.item(), taug.grad.detach().clone(), u0g.grad.detach().clone()))
    assert grads[0][0] == grads[1][0]
    assert rel(grads[1][1], grads[0][1]) == 0.0 and rel(grads[1][2], grads[0][2]) == 0.0


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
    # measured: 1.7e-6 (dL/dtau) and 7.6e-7 (dL/du0); against the oracle's gradient see
    # test_c5_segmentation_against_oracle
    assert abs(L32 - L64) / abs(L64) < 1e-6
    assert et < 1e-5 and eu < 1e-5


def test_reverse_mode_rejects_unsupported_lattices():
    from paper_1909_04502_amd import rlbm as R
    lat = R.Lattice(d=2, zeta=1.0, order=3, extent=(8, 8), bc=("open", "periodic"), tau=0.8)
    B = lat.new_state().zero_()
    with pytest.raises(R.RLBMError) as e:
        lat.adjoint_step(B, B.clone())
    assert e.value.status == R.ERR_UNSUPPORTED


def test_full_size_reverse_step_sampled():
    """C5's reverse step at full size, in the launch configuration the bench times: 512 x 512, float
    deviations, a tau field (0.8 +- 0.2, seed 4), zeta = 1, N = 3, from the state after 5 forward
    steps and a seeded lam_{t+1}.  lam_t and the dL/dtau increment at 256 sampled sites against the
    oracle: F_t(x) = S(B)(x) from B's 3 x 3 periodic neighbourhood, mu(x) = (S^T lam_{t+1})(x) from
    lam_{t+1}'s (the transposed pull reaches one site the other way, so a 3 x 3 window does not
    alias), and lam_t(x), dL/dtau(x) as the VJP of the oracle's collision at F_t(x) by autograd."""
    from paper_1909_04502_amd import rlbm as R
    print("[case] full-size reverse step", flush=True)
    L = 512
    n, T, u, tau, _ = problem(L, L)
    lat = R.Lattice(d=2, zeta=1.0, order=3, extent=(L, L), storage="f32dev", tau=0.8, tau_field=tau.clone())
    fa = lat.init(n, T, u)
    B = lat.step(fa, lat.new_state(), 5)
    g = np.random.default_rng(9)
    lam_next = torch.tensor(g.normal(size=tuple(B.shape)) * 1e-3, dtype=B.dtype, device="cuda")
    dtau = torch.zeros((L, L), dtype=torch.float64, device="cuda")
    lam = lat.adjoint_step(B, lam_next, dtau=dtau)
    lat.sync()
    q = qd.product_2d(1.0, 3)
    one = torch.ones(1, 1, dtype=torch.float64)
    fref = OL.Lattice(q, 0.8, (1, 1)).equilibrium(one, one, torch.tensor([1.0, 0.0, 0.0],
                                                                       dtype=torch.float64)[:, None, None])[:, 0, 0]
    tau32 = tau.to(torch.float32).to(torch.float64)          # the field the library holds
    K = 256
    ys, xs = g.integers(0, L, K), g.integers(0, L, K)
    ol3 = OL.Lattice(q, 0.8, (3, 3))
    Bc, lamc = B.cpu().to(torch.float64), lam_next.cpu().to(torch.float64)
    got_lam = lam.cpu().to(torch.float64)[:, ys, xs]
    got_dtau = dtau.cpu()[ys, xs]
    want_lam = torch.empty_like(got_lam)
    want_dtau = torch.empty_like(got_dtau)
    for k in range(K):
        iy = torch.tensor([(ys[k] + d) % L for d in (-1, 0, 1)])
        ix = torch.tensor([(xs[k] + d) % L for d in (-1, 0, 1)])
        Bw = Bc[:, iy][:, :, ix] + fref[:, None, None]
        Fc = ol3.stream(Bw)[:, 1:2, 1:2].clone().requires_grad_(True)
        G = torch.zeros((q.Q, 3, 3), dtype=torch.float64, requires_grad=True)
        (ol3.stream(G) * lamc[:, iy][:, :, ix]).sum().backward()
        mu = G.grad[:, 1:2, 1:2]
        tc = tau32[ys[k]:ys[k] + 1, xs[k]:xs[k] + 1].clone().requires_grad_(True)
        ol1 = OL.Lattice(q, 0.8, (1, 1))
        (OG.collide_diff(ol1, Fc, tc) * mu).sum().backward()
        want_lam[:, k] = Fc.grad[:, 0, 0]
        want_dtau[k] = tc.grad[0, 0]
    el, ed = rel(got_lam, want_lam), rel(got_dtau, want_dtau)
    print("full-size reverse step errors: lam", el, "dtau", ed, flush=True)
    # measured: lam 7.8e-8, dL/dtau 4.2e-6 (a sum over the populations of float products)
    assert el < 1e-5 and ed < 1e-5


@pytest.mark.parametrize("storage", ["f64", "f32dev", "f32dev_f64"])
def test_c5_segmentation_against_oracle(storage):
    """The adjoint configuration's segmentation on a lattice the oracle can differentiate: 16 x 16,
    100 steps checkpointed every 45 (segments of 45, 45 and 10 steps, each recomputed in the backward),
    a tau field 0.8 +- 0.2 and the L2 velocity loss against a shifted Taylor-Green target; the
    gradients dL/dtau(x) and dL/du0(x) against the oracle's reverse mode through all 100 steps.
    Double storage to 1e-10 (measured 4e-14); float deviations to 5e-6 (updated in float: measured
    6.3e-7 on dL/dtau, 1.2e-6 on dL/du0, 1.2e-7 on the loss)."""
    print(f"[case] C5 segmentation vs oracle {storage}", flush=True)
    nx, ny, nsteps, every = 16, 16, 100, 45
    L, gtau, gu0 = gpu_gradient(nx, ny, nsteps, every, storage=storage)
    n, T, u, tau, ut = problem(nx, ny)
    lat = OL.Lattice(qd.product_2d(1.0, 3), 0.8, (nx, ny))
    L0, gtau0, gu00 = OG.gradient(lat, n, T, u, tau, nsteps, ut)
    el, et, eu = abs(L - L0.item()) / abs(L0.item()), rel(gtau, gtau0), rel(gu0, gu00)
    print(f"C5 segmentation {storage}: loss {el:.2e}, dL/dtau {et:.2e}, dL/du0 {eu:.2e}", flush=True)
    if storage == "f64":
        assert el < 1e-12 and et < 1e-10 and eu < 1e-10
    else:
        assert el < 1e-6 and et < 5e-6 and eu < 5e-6


@pytest.mark.parametrize("storage", ["f64", "f32dev"])
def test_store_all_states_gives_the_checkpointed_gradient(storage):
    """every = 1 keeps every state instead of recomputing segments: the same kernels on the same
    states, so the loss and both gradients equal those of the run checkpointed every 45 steps bit for
    bit (24 x 20, 100 steps)."""
    print(f"[case] store-all gradient {storage}", flush=True)
    L45, gt45, gu45 = gpu_gradient(24, 20, 100, 45, storage=storage)
    L1, gt1, gu1 = gpu_gradient(24, 20, 100, 1, storage=storage)
    assert L1 == L45
    assert torch.equal(gt1, gt45) and torch.equal(gu1, gu45)


def test_c5_full_size_directional_differences_fp64():
    """C5's full size and length in double storage: 512 x 512, 2000 steps checkpointed every 45; the
    adjoint gradient along two seeded directions (tau field and initial velocity together) against
    central differences of the forward run with h = 1e-4."""
    from paper_1909_04502_amd import adjoint as A
    from paper_1909_04502_amd import rlbm as R
    print("[case] C5 full size FD (FP64)", flush=True)
    nx = ny = 512
    nsteps, every = 2000, 45
    L, gtau, gu0 = gpu_gradient(nx, ny, nsteps, every)
    n, T, u, tau, ut = problem(nx, ny)
    lat = R.Lattice(d=2, zeta=1.0, order=3, extent=(nx, ny), tau=0.8, tau_field=tau.clone())

    def loss(tau_, u_):
        with torch.no_grad():
            U = A.run(lat, tau_.cuda(), u_.cuda(), n, T, nsteps, every=every)
            return A.velocity_loss(U, ut.cuda()).item()

    assert abs(loss(tau, u) - L) <= 1e-12 * abs(L)
    g = np.random.default_rng(21)
    for _ in range(2):
        dt = torch.tensor(g.normal(size=tau.shape))
        du = torch.tensor(g.normal(size=u.shape)) * 0.05
        h = 1e-4
        fd = (loss(tau + h * dt, u + h * du) - loss(tau - h * dt, u - h * du)) / (2 * h)
        an = (gtau.cpu() * dt).sum().item() + (gu0.cpu() * du).sum().item()
        print("C5 full size: FD", fd, "adjoint", an, "rel", abs(fd - an) / abs(an), flush=True)
        assert abs(fd - an) <= 1e-6 * abs(an)
