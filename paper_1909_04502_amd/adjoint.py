"""Differentiable RLBM runs: a torch.autograd.Function over the C-ABI kernels.

Forward: f_0 from (n0, T0, u0), B_0 = C(f_0), B_t = C(S(B_{t-1})) for
t = 1..T, returning the four-velocity of F_{T+1} = S(B_T).  Every `every`
steps the state is checkpointed.  Backward: lam_{T+1} from rlbm_moments_vjp,
then segment by segment (last first) the states of the segment are
recomputed from its checkpoint and lam_t = rlbm_adjoint_step(B_{t-1},
lam_{t+1}) runs down to the segment start; finally rlbm_init_vjp gives
dL/du0.  dL/dtau(x) is accumulated by every reverse kernel.  Memory: the
checkpoints plus one segment of states.  every = 1 keeps every state (T + 1
state buffers: 67 GB for 2000 steps of a 512 x 512 float-deviation lattice, a
quarter of one GPU's HBM): each forward step writes a fresh buffer and the
backward recomputes nothing.  The tau field of the forward run is
kept and restored into the lattice before the backward recomputes, so other
runs on the same lattice between a forward and its backward do not change
the gradient.
"""
from __future__ import annotations

import torch

from .rlbm import Lattice


class _Run(torch.autograd.Function):
    @staticmethod
    def forward(ctx, tau_field, u0, lat, n0, T0, nsteps, every, noise, amp):
        if lat.tau_field is None:
            raise ValueError("the lattice must be created with a tau_field tensor")
        lat.tau_field.copy_(tau_field.detach().to(lat.tau_field.dtype))
        u0d = u0.detach().to(torch.float64)
        # the segments run in a buffer pair kept by the lattice: the library caches the launch
        # graph of a multi-step call per buffer pair, so every run replays the same graphs
        cur, nxt = _work_pair(lat)
        lat.init(n0, T0, u0d, noise, amp, out=cur)
        ckpt = {0: cur.clone()}
        if every == 1:
            # every state kept, in one allocation: B_t stepped from B_{t-1} straight into its slot
            store = torch.empty((nsteps + 1,) + tuple(cur.shape), dtype=cur.dtype, device=cur.device)
            store[0].copy_(cur)
            for t in range(1, nsteps + 1):
                lat.step(store[t - 1], store[t], 1)
            ckpt = {t: store[t] for t in range(nsteps)}
            final = store[nsteps]
        else:
            t = 0
            while t < nsteps:                              # one library call per checkpoint segment
                k = min(every, nsteps - t)
                res = lat.step(cur, nxt, k)
                if res is nxt:
                    cur, nxt = nxt, cur
                t += k
                if t < nsteps:
                    ckpt[t] = cur.clone()
            final = cur.clone()
        fields = lat.moments(final)
        ctx.lat, ctx.ckpt, ctx.final = lat, ckpt, final
        # the kernels read tau through the lattice's own buffer, which another run on the same
        # lattice may overwrite before this backward: keep this run's copy to restore there
        ctx.tau_saved = lat.tau_field.clone()
        ctx.args = (n0, T0, u0d, noise, amp, nsteps, every)
        ctx.tau_dtype = tau_field.dtype
        return fields["U"]

    @staticmethod
    def backward(ctx, gU):
        lat = ctx.lat
        n0, T0, u0d, noise, amp, nsteps, every = ctx.args
        lat.tau_field.copy_(ctx.tau_saved)
        lam = lat.moments_vjp(ctx.final, gU=gU.contiguous())
        lam_spare = torch.empty_like(lam)
        dtau = torch.zeros(lat.grid_shape, dtype=torch.float64, device="cuda")
        seg = [lat.new_state() for _ in range(max(0, min(every, nsteps) - 1))]
        for s in sorted(ctx.ckpt, reverse=True):
            e = min(s + every, nsteps)
            states = [ctx.ckpt[s]]
            for k in range(s + 1, e):                      # B_{s+1} .. B_{e-1}
                lat.step(states[-1], seg[k - s - 1], 1)
                states.append(seg[k - s - 1])
            for t in range(e, s, -1):                      # lam_t from B_{t-1} and lam_{t+1}
                out = lat.adjoint_step(states[t - 1 - s], lam, lam=lam_spare, dtau=dtau)
                lam_spare, lam = lam, out
            del states
        du0 = lat.init_vjp(n0, T0, u0d, lam, noise, amp, dtau=dtau)
        lat.sync()
        return dtau.to(ctx.tau_dtype), du0, None, None, None, None, None, None, None


def _work_pair(lat: Lattice):
    pair = getattr(lat, "_run_pair", None)
    if pair is None:
        pair = (lat.new_state(), lat.new_state())
        lat._run_pair = pair
    return pair


def run(lat: Lattice, tau_field, u0, n0, T0, nsteps: int, every: int = 45, noise=None, amp: float = 0.0):
    """Four-velocity U (d+1, grid) of the final state, differentiable in tau_field and u0."""
    return _Run.apply(tau_field, u0, lat, n0, T0, nsteps, every, noise, amp)


def velocity_loss(U, target_u):
    """L = 1/2 sum_x |u - u_target|^2 with the three-velocity u = U^a / U^0."""
    u = U[1:] / U[0]
    return 0.5 * ((u - target_u) ** 2).sum()
