"""Differentiable multi-step rollout of the MPMC solver (torch.autograd.Function).

Forward: ``nsteps`` SSP-RK3 steps through the HIP library; dt and Gamma of
every step are recorded (from U^n as the step computes them, or given), and
the state is kept every ``every`` steps as a checkpoint.  Backward: for each
segment in reverse, the segment is recomputed from its checkpoint with the
recorded dt and Gamma, storing per step U^n, the two intermediate stage
states and the three stage decision masks (``mpmc_rk3_step_stages``); then
``mpmc_adjoint_step_stages`` carries the cotangent back one step at a time
from those records.  The recompute of the next segment runs on a second
context and stream while the current one is swept (two segments of records
are alive at a time).  With ``tape=False`` only U^n is stored and
``mpmc_adjoint_step`` recomputes the stages itself (a third of the memory,
about one more forward step per step).  Every limiter decision, min/max arm
and dt/Gamma is frozen as the forward took it; the WENO-Z weights are
differentiated.  All arithmetic runs in the library; this module only moves
tensors.
"""
import torch


class Rollout(torch.autograd.Function):
    """``U_K = Rollout.apply(U0, ctx, nsteps, every)``: U0 is a flat FP64 state
    [nv * cells] on the context's device; the result is a new tensor."""

    @staticmethod
    def forward(fctx, U0, mctx, nsteps, every=10, dts=None, gammas=None, tape=True):
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
        fctx.tape = bool(tape)
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
        if fctx.tape:
            lam = _backward_taped(fctx, mctx, dt_rec, g_rec, lam, out, nseg)
            return lam, None, None, None, None, None, None
        for s in reversed(range(nseg)):
            j0 = s * fctx.every
            j1 = min(fctx.nsteps, j0 + fctx.every)
            U = fctx.ckpt[s].clone()
            # recompute the states U^{j0} .. U^{j1-1} of this segment
            states = [fctx.ckpt[s]]
            for j in range(j0, j1 - 1):
                mctx.mpmc_rk3_step(U, dt_in=dt_rec[j:j + 1], gamma_in=g_rec[j:j + 1])
                states.append(U.clone())
            for j in reversed(range(j0, j1)):
                mctx.mpmc_adjoint_step(states[j - j0], dt_rec[j:j + 1], g_rec[j:j + 1], lam, out)
                lam, out = out, lam
            del states
        return lam, None, None, None, None, None, None


def _backward_taped(fctx, mctx, dt_rec, g_rec, lam, out, nseg):
    """Segments in reverse; each segment is recomputed (stage states and
    masks recorded, mpmc_rk3_step_stages) by a second context on a second
    stream while the adjoint sweeps the segment after it on the caller's
    stream, so the two overlap on the GPU.  The same kernels on the same
    inputs as one after the other: the same bits."""
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream(device=lam.device)
    twin = mctx.twin()
    ready = torch.cuda.Event()
    ready.record(main)  # checkpoints, dt and Gamma of the forward
    side.wait_event(ready)

    def recompute(s):
        j0 = s * fctx.every
        j1 = min(fctx.nsteps, j0 + fctx.every)
        recs = []
        with torch.cuda.stream(side):
            U = fctx.ckpt[s].clone()
            for j in range(j0, j1):
                Un = U.clone()
                S1, S2, M = torch.empty_like(U), torch.empty_like(U), twin.new_masks()
                twin.mpmc_rk3_step_stages(U, dt_rec[j:j + 1], g_rec[j:j + 1], S1, S2, M, stream=side)
                recs.append((Un, S1, S2, M))
            done = torch.cuda.Event()
            done.record(side)
        return j0, j1, recs, done

    pending = recompute(nseg - 1)
    for s in reversed(range(nseg)):
        j0, j1, recs, done = pending
        main.wait_event(done)
        for rec in recs:
            for t in rec:
                t.record_stream(main)  # freed only after the adjoint has read them
        if s > 0:
            pending = recompute(s - 1)
        for j in reversed(range(j0, j1)):
            Un, S1, S2, M = recs.pop()
            mctx.mpmc_adjoint_step_stages(Un, S1, S2, M, dt_rec[j:j + 1], g_rec[j:j + 1], lam, out,
                                          stream=main)
            lam, out = out, lam
            del Un, S1, S2, M
    return lam


def rollout(U0, mctx, nsteps, every=10, dts=None, gammas=None, tape=True):
    """Run ``nsteps`` steps from U0; returns (U_K, dt per step, Gamma per step).
    Differentiable with respect to U0.  ``tape``: store each recomputed
    segment's stage states and masks for the backward (default) or let each
    adjoint step recompute its stages."""
    return Rollout.apply(U0, mctx, nsteps, every, dts, gammas, tape)

