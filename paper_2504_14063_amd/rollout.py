"""Differentiable multi-step rollout of the MPMC solver (torch.autograd.Function).

Forward: ``nsteps`` SSP-RK3 steps through the HIP library; dt and Gamma of
every step are recorded (from U^n as the step computes them, or given), and
the state is kept every ``every`` steps as a checkpoint.  Backward: for each
segment in reverse, the states of the segment are recomputed from its
checkpoint with the recorded dt and Gamma, then ``mpmc_adjoint_step`` carries
the cotangent back one step at a time.  Every limiter decision, min/max arm
and dt/Gamma is frozen as the forward took it; the WENO-Z weights are
differentiated.  All arithmetic runs in the library; this module only moves
tensors.
"""
import torch


class Rollout(torch.autograd.Function):
    """``U_K = Rollout.apply(U0, ctx, nsteps, every)``: U0 is a flat FP64 state
    [nv * cells] on the context's device; the result is a new tensor."""

    @staticmethod
    def forward(fctx, U0, mctx, nsteps, every=10, dts=None, gammas=None):
        nsteps = int(nsteps)
        every = max(1, int(every))
        U = U0.detach().clone()
        dt_rec = torch.empty(nsteps, dtype=torch.float64, device=U.device)
        g_rec = torch.empty(nsteps, dtype=torch.float64, device=U.device)
        ckpt = []
        for j in range(nsteps):
            if j % every == 0:
                ckpt.append(U.clone())
            if dts is not None:
                mctx.mpmc_rk3_step(U, dt_in=dts[j:j + 1], gamma_in=gammas[j:j + 1])
                dt_rec[j:j + 1].copy_(dts[j:j + 1])
                g_rec[j:j + 1].copy_(gammas[j:j + 1])
            else:
                mctx.mpmc_rk3_step(U, dt_out=dt_rec[j:j + 1], gamma_out=g_rec[j:j + 1])
        fctx.mctx = mctx
        fctx.nsteps = nsteps
        fctx.every = every
        fctx.ckpt = ckpt
        fctx.save_for_backward(dt_rec, g_rec)
        fctx.mark_non_differentiable(dt_rec, g_rec)
        return U, dt_rec, g_rec

    @staticmethod
    def backward(fctx, lam, _gdt=None, _gg=None):
        mctx = fctx.mctx
        dt_rec, g_rec = fctx.saved_tensors
        lam = lam.detach().to(torch.float64).contiguous().clone()
        out = torch.empty_like(lam)
        nseg = len(fctx.ckpt)
        for s in reversed(range(nseg)):
            j0 = s * fctx.every
            j1 = min(fctx.nsteps, j0 + fctx.every)
            # recompute the states U^{j0} .. U^{j1-1} of this segment
            states = [fctx.ckpt[s]]
            U = fctx.ckpt[s].clone()
            for j in range(j0, j1 - 1):
                mctx.mpmc_rk3_step(U, dt_in=dt_rec[j:j + 1], gamma_in=g_rec[j:j + 1])
                states.append(U.clone())
            for j in reversed(range(j0, j1)):
                mctx.mpmc_adjoint_step(states[j - j0], dt_rec[j:j + 1], g_rec[j:j + 1], lam, out)
                lam, out = out, lam
            del states
        return lam, None, None, None, None, None


def rollout(U0, mctx, nsteps, every=10, dts=None, gammas=None):
    """Run ``nsteps`` steps from U0; returns (U_K, dt per step, Gamma per step).
    Differentiable with respect to U0."""
    return Rollout.apply(U0, mctx, nsteps, every, dts, gammas)
