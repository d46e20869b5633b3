#!/usr/bin/env python
"""Benchmark of the four-equation MPMC hot path on one MI355X.

Workload: 3D three-component two-phase droplet in crossflow at 256^3 (liquid
stiffened-gas droplet, radius 32 cells with seeded centre jitter, in a
two-species ideal-gas mixture with seeded smooth composition noise,
crossflow 50 m/s, periodic, regularization and species diffusion on).  One
step = one SSP-RK3 step of the whole hot path.  Prints one JSON line.

Metric: cell-updates per second (cells x steps / wall time) with the state
resident in HBM; the FP64 form is `value`, the mixed form and the
adjoint/forward cost ratio are reported beside it.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per RK3 step, FP64 vs mixed at 256^3; adjoint/forward cost"
PEAK_FP64_FLOPS = 78.6e12  # MI355X FP64 vector, FMA = 2 flops (256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz)
PEAK_HBM = 8.0e12

# Algorithmic FP64 operations per face of one sweep (+ - * / sqrt log tanh
# each counted once), measured by the oracle's counting scalar on this
# workload (oracle/count_ops.py); per direction x, y, z.
OPS_PER_FACE = {"face_x": None, "face_y": None, "face_z": None}
OPS_FILE = os.path.join(ROOT, "oracle", "op_counts.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_ops():
    if os.path.exists(OPS_FILE):
        with open(OPS_FILE) as f:
            d = json.load(f)
        return d.get("droplet_crossflow_3d", {})
    return {}


PROFILE = os.path.join(ROOT, "profiles", "kernels_droplet_crossflow_3d_256.md")
KERNEL_SOURCES = ["mpmc_kernels.h", "mpmc_device.h", "mpmc_dual.h"]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, copy-calibrated); None when the
    kernel sources changed since the counters were taken."""
    import hashlib
    if not os.path.exists(PROFILE):
        return None
    src = b"".join(open(os.path.join(ROOT, "paper_2504_14063_amd", "csrc", f), "rb").read()
                   for f in KERNEL_SOURCES)
    sha = hashlib.sha1(src).hexdigest()[:16]
    rec, val = None, None
    with open(PROFILE) as f:
        for line in f:
            if line.startswith("SOURCE_SHA1 "):
                rec = line.split()[1]
            elif line.startswith("TRAFFIC ") and line[len("TRAFFIC "):].rsplit(" ", 1)[0] == kernel:
                val = float(line.rsplit(" ", 1)[1])
    return val if rec == sha else None


def time_forward(torch, ctx, U, steps, warmup, profile=True, dt_in=None):
    """Wall time of `steps` RK3 steps after `warmup` (dt from the CFL
    condition, or the device scalar dt_in; Gamma from the state)."""
    for _ in range(warmup):
        ctx.mpmc_rk3_step(U, dt_in=dt_in)
    torch.cuda.synchronize()
    if profile:
        ctx.mpmc_profile(True)
        ctx.mpmc_profile_read(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.mpmc_rk3_step(U, dt_in=dt_in)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = None
    if profile:
        prof = ctx.mpmc_profile_read(reset=True)
        ctx.mpmc_profile(False)
    return t1 - t0, prof


def paper_workloads(torch, steps, warmup, which="all"):
    """FP64 step rate of two of the paper's runs at their sizes: the Mach-100
    water column (held inlet, the paper's constant dt) and the air-water
    shock-droplet."""
    from paper_2504_14063_amd import inputs, mpmc
    res = {}
    for key, name, make in (("mach100", "mach100_water_column_2d 2048x1025 (held inlet, dt 7.5e-4 us)",
                             inputs.mach100_water_column_2d),
                            ("shock_droplet", "shock_droplet_air_water_2d 1024^2",
                             inputs.shock_droplet_air_water_2d)):
        if which not in ("all", key):
            continue
        wc = make()
        cw = mpmc.Context.from_case(wc)
        Uw = cw.init_state_from_case(wc)
        dt_w = None
        if "held" in wc.extra:
            cw.mpmc_set_held_cells(wc.extra["held"], inputs.held_values(wc, Uw.cpu().numpy()))
            dt_w = cw.scalar(wc.extra["dt"])
        ew, profw = time_forward(torch, cw, Uw, steps, warmup, dt_in=dt_w)
        vw = wc.ncell * steps / ew
        res[name] = dict(value=vw, unit="cell-updates/s", ms_per_step=1e3 * ew / steps,
                         kernels_ms={k: v[0] / max(v[1], 1) for k, v in profw.items() if v[1]})
        log(f"bench: {name} {vw:.4e} cell-updates/s")
        cw.close()
        del Uw
    return res


def cpu_baseline(case, target_s=12.0):
    """The oracle on the host cores: one step of the workload itself when that
    takes at most ~30 s, else K steps of a periodic sub-box of the same
    initial state; beside it one thread on a smaller box."""
    import numpy as np

    import oracle
    from paper_2504_14063_amd import inputs

    def box_case(m):
        c = inputs.droplet_crossflow_3d(n=case.n[0])
        sl = slice(0, m)
        off = [int(round(v)) - m // 2 for v in case.extra["center"]]
        idx = [(np.arange(m) + off[d]) % case.n[d] for d in range(3)]
        sub = lambda a: a[..., idx[2], :, :][..., :, idx[1], :][..., :, :, idx[0]]
        return inputs.Case("box", 3, (m, m, m), case.dx, (0, 0, 0), (0, 0, 0), case.materials, case.opts,
                           np.ascontiguousarray(sub(c.phi)), np.ascontiguousarray(sub(c.y)),
                           np.ascontiguousarray(sub(c.P)), np.ascontiguousarray(sub(c.T)),
                           np.ascontiguousarray(sub(c.vel)))

    def run(m, steps=1):
        bc = box_case(m)
        o = oracle.Oracle.from_case(bc)
        U = o.init_state(bc)
        t0 = time.perf_counter()
        for _ in range(steps):
            o.step(U)
        return time.perf_counter() - t0, m ** 3 * steps

    t, cells = run(24)
    rate = cells / t
    if case.ncell / rate <= 30.0:
        # one step of the workload itself, when it takes at most ~30 s
        o = oracle.Oracle.from_case(case)
        U = o.init_state(case)
        t0 = time.perf_counter()
        o.step(U)
        t, cells = time.perf_counter() - t0, case.ncell
        del U, o
        m, steps = case.n[0], 1
        sample = f"1 SSP-RK3 step of the whole {m}^3 workload ({t:.1f} s)"
    else:
        # a box of up to 128^3 around the droplet, and as many steps as bring
        # the sample to about target_s of CPU work
        m = int(max(24, min(128, round((target_s * rate) ** (1.0 / 3.0)))))
        steps = max(1, int(round(target_s * rate / m ** 3)))
        t, cells = run(m, steps)
        sample = (f"{steps} SSP-RK3 step(s) of a periodic {m}^3 sub-box centred on the droplet of the "
                  f"same {case.n[0]}^3 initial state ({t:.1f} s)")
    cores = oracle.num_threads()
    # the same on one thread, on a box 1/cores the size (about as long)
    oracle.set_num_threads(1)
    try:
        m1 = int(max(16, min(128, round(m / cores ** (1.0 / 3.0)))))
        t1, cells1 = run(m1, steps)
    finally:
        oracle.set_num_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=cells / t, unit="cell-updates/s", cores=cores, kind="oracle", sample=sample,
                one_thread=dict(value=cells1 / t1, sample=f"{steps} step(s) of a {m1}^3 sub-box ({t1:.1f} s)"),
                cpu_model=model)


def adjoint_cost(torch, n=512, steps=200, every=10, fd=True, floor=False):
    """Wall time of the checkpointed rollout backward (segment recompute +
    adjoint steps) over its forward, 2D shock-droplet, gradient of the final
    gas kinetic energy with respect to the initial state."""
    from paper_2504_14063_amd import inputs, mpmc
    from paper_2504_14063_amd.rollout import rollout
    case = inputs.shock_droplet_2d(n=n, steps=steps, floor=floor)
    ctx = mpmc.Context.from_case(case)
    ns, dim, nc = case.ns, case.dim, case.ncell
    gas = [k for k, m in enumerate(case.materials) if m.phase == inputs.GAS]
    U0 = ctx.init_state_from_case(case)

    def objective(U):
        Ur = U.view(ns + dim + 1, nc)
        rho = Ur[:ns].sum(0)
        rg = sum(Ur[k] for k in gas)
        return 0.5 * case.dx[0] * case.dx[1] * (rg * (Ur[ns:ns + dim] ** 2).sum(0) / (rho * rho)).sum()

    # warm-up (kernel loading, adjoint scratch allocation)
    Uw = U0.clone().requires_grad_(True)
    objective(rollout(Uw, ctx, 2, every)[0]).backward()
    torch.cuda.synchronize()
    Ux = U0.clone().requires_grad_(True)
    t0 = time.perf_counter()
    UK, _, _ = rollout(Ux, ctx, steps, every)
    J = objective(UK)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    grad = Ux.grad.detach()
    # per-kernel times from a separate, shorter profiled rollout (the event
    # pairs around every launch would inflate the timed backward above)
    Up = U0.clone().requires_grad_(True)
    Jp = objective(rollout(Up, ctx, 2 * every, every)[0])
    torch.cuda.synchronize()
    # the backward's recompute runs on the context's twin (second stream)
    for cx in (ctx, ctx.twin()):
        cx.mpmc_profile(True)
        cx.mpmc_profile_read(reset=True)
    Jp.backward()
    torch.cuda.synchronize()
    prof = {}
    for cx in (ctx, ctx.twin()):
        for k, (ms, nl) in cx.mpmc_profile_read(reset=True).items():
            a = prof.get(k, (0.0, 0))
            prof[k] = (a[0] + ms, a[1] + nl)
        cx.mpmc_profile(False)
    del Up, Jp
    # directional derivatives: the droplet radius R (cells; U0 is affine in
    # the liquid fraction at fixed P, T, y, u) and five seeded smooth shape
    # perturbations s_k(x, y) dU0/dR of the interface
    dirs = droplet_directions(torch, ctx, case)
    out = dict(workload=f"shock_droplet_2d {n}x{n}, {steps} steps, checkpoints every {every}",
               forward_s=t1 - t0, backward_s=t2 - t1, ratio=(t2 - t1) / (t1 - t0),
               backward_kernels_ms_per_launch={k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1]},
               grad_finite=bool(torch.isfinite(grad).all()),
               dJ_adjoint={name: float((grad * d).sum()) for name, d in dirs})
    ctx.close()
    if fd:
        out["fd_frozen"] = {f"{n}x{n}, 3 steps": frozen_fd(torch, n, 3, (1e-3, 1e-4, 1e-5)),
                            "64x64, 6 steps": frozen_fd(torch, 64, 6, (1e-4, 1e-5, 1e-6))}
    return out


def droplet_directions(torch, ctx, case):
    """[(name, dU0)]: dU0/dR of the shock-droplet and s_k dU0/dR, k = 0..4."""
    from paper_2504_14063_amd import inputs
    ns, dim, nc = case.ns, case.dim, case.ncell
    phi, y, P, T, vel = case.prim_arrays()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    one = np.zeros_like(phi)
    one[0] = 1.0
    U_l = ctx.mpmc_init_state(t(one), t(y), t(P), t(T), t(vel))
    U_g = ctx.mpmc_init_state(t(one[::-1].copy()), t(y), t(P), t(T), t(vel))
    dR = (U_l - U_g).view(ns + dim + 1, nc) * t(case.extra["dphil_dR"].reshape(-1))
    dirs = [("radius", dR.reshape(-1))]
    for k in range(5):
        s = t(inputs.smooth_field(case.n[0], case.n[1], 11 + k))
        dirs.append((f"shape{k}", (dR * s[None]).reshape(-1)))
    return dirs


def frozen_fd(torch, n, steps, hs):
    """Central differences of the frozen-decision map (mpmc_rk3_step_replay
    with the unperturbed run's dt, Gamma and face decisions) of the final
    gas kinetic energy along the droplet directions, against the adjoint:
    per direction and h the relative difference and the inadmissible cells
    the two replays met (no difference exists where they met any)."""
    from paper_2504_14063_amd import inputs, mpmc
    from paper_2504_14063_amd.rollout import rollout
    if n == 64:
        case = inputs.shock_droplet_2d(n=64, radius=8.0, shock_x=20.0, steps=steps)
    else:
        case = inputs.shock_droplet_2d(n=n, steps=steps)
    ctx = mpmc.Context.from_case(case, raise_inadmissible=False)
    ns, dim, nc = case.ns, case.dim, case.ncell
    gas = [k for k, m in enumerate(case.materials) if m.phase == inputs.GAS]

    def objective(U):
        Ur = U.view(ns + dim + 1, nc)
        rho = Ur[:ns].sum(0)
        rg = sum(Ur[k] for k in gas)
        return 0.5 * case.dx[0] * case.dx[1] * (rg * (Ur[ns:ns + dim] ** 2).sum(0) / (rho * rho)).sum()

    U0 = ctx.init_state_from_case(case)
    Ux = U0.clone().requires_grad_(True)
    UK, dts, gs = rollout(Ux, ctx, steps, 3)
    objective(UK).backward()
    grad = Ux.grad.detach()
    masks, U = [], U0.clone()
    for j in range(steps):
        m = ctx.new_masks()
        ctx.mpmc_rk3_step(U, dt_in=dts[j:j + 1], gamma_in=gs[j:j + 1], masks=m)
        masks.append(m)
    res = {}
    for name, d in droplet_directions(torch, ctx, case):
        ad = float((grad * d).sum())
        row = dict(adjoint=ad)
        for h in hs:
            vals, bad = [], 0
            for sg in (1.0, -1.0):
                V = U0 + sg * h * d
                ctx.mpmc_stats(reset=True)
                for j in range(steps):
                    ctx.mpmc_rk3_step_replay(V, dts[j:j + 1], gs[j:j + 1], masks[j])
                torch.cuda.synchronize()
                bad += ctx.mpmc_stats(reset=True)["inadmissible_cells"]
                vals.append(float(objective(V)))
            fdv = (vals[0] - vals[1]) / (2 * h)
            row[f"h={h:g}"] = dict(rel=abs(fdv - ad) / abs(ad) if bad == 0 else None, inadmissible_cells=bad)
        res[name] = row
    ctx.close()
    return res


def mixed_accuracy(n, steps):
    """Mixed form against FP64 on the n^3 droplet at matched steps (dt and
    Gamma of the FP64 run): relative L1 per field (partial densities over the
    density, momentum components over the momentum magnitude)."""
    import torch

    from paper_2504_14063_amd import inputs, mpmc
    case = inputs.droplet_crossflow_3d(n=n)
    log(f"mixed accuracy: droplet_crossflow_3d {n}^3, {steps} steps")
    ns, dim = case.ns, case.dim
    res = {}
    rate = {}
    for prec in (0, 1):
        ctx = mpmc.Context.from_case(case, precision=prec)
        U = ctx.init_state_from_case(case)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if prec == 0:
            dts = []
            for j in range(steps):
                dt, g = ctx.scalar(), ctx.scalar()
                ctx.mpmc_rk3_step(U, dt_out=dt, gamma_out=g)
                dts.append((dt, g))
                if j % 20 == 0:
                    log(f"  fp64 step {j}")
            ref = U
        else:
            for j in range(steps):
                ctx.mpmc_rk3_step(U, dt_in=dts[j][0], gamma_in=dts[j][1])
                if j % 20 == 0:
                    log(f"  mixed step {j}")
        torch.cuda.synchronize()
        rate["fp64" if prec == 0 else "mixed"] = case.ncell * steps / (time.perf_counter() - t0)
        if prec == 1:
            nv = ns + dim + 1
            a, b = U.view(nv, -1), ref.view(nv, -1)
            rho = b[:ns].abs().sum()
            mom = torch.sqrt((b[ns:ns + dim] ** 2).sum(0)).sum()
            den = [float(rho)] * ns + [float(mom)] * dim + [float(b[-1].abs().sum())]
            res = [float((a[v] - b[v]).abs().sum()) / den[v] for v in range(nv)]
            # velocity in the interface cells (liquid mass fraction in
            # [0.01, 0.99]) against the FP64 run, relative to the crossflow
            liq = [k for k, m in enumerate(case.materials) if m.phase == inputs.LIQUID]
            ra, rb = a[:ns].sum(0), b[:ns].sum(0)
            yl = sum(b[k] for k in liq) / rb
            itf = (yl > 0.01) & (yl < 0.99)
            du = ((a[ns:ns + dim] / ra - b[ns:ns + dim] / rb)[:, itf]).abs().max()
            u_interface = dict(cells=int(itf.sum()), max_abs_du_over_u0=float(du) / 50.0)
        st = ctx.mpmc_stats(reset=True)
        ctx.close()
        if prec == 1:
            del U
    return dict(workload=f"droplet_crossflow_3d {n}^3", steps=steps, rel_l1_per_field=res, max=max(res),
                interface_velocity=u_interface, unrecoverable_faces_mixed=st["unrecoverable"],
                cell_updates_per_s=rate, mixed_speedup=rate["mixed"] / rate["fp64"])


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-viscous", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--paper-workloads-only", choices=["all", "mach100", "shock_droplet"], default=None,
                    help="only time the Mach-100 water column and/or the air-water shock-droplet")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="form reported as `value` (profiling runs)")
    ap.add_argument("--step-layout", choices=["split", "fused"], default="split",
                    help="kernel split of the timed step (the same bits; split is the library's default)")
    ap.add_argument("--no-mixed-accuracy", action="store_true",
                    help="skip the mixed-vs-FP64 accuracy block (512^3, 100 steps) of the default run")
    ap.add_argument("--mixed-accuracy", type=int, default=0, metavar="N",
                    help="only compare the mixed form with FP64 on the N^3 droplet after --steps steps")
    ap.add_argument("--adjoint-only", type=int, default=0, metavar="STEPS",
                    help="only time the checkpointed adjoint of the 512^2 shock-droplet over STEPS steps "
                         "(no finite differences)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 3 plain device copies of MIB MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes_read=8 * n, copy_bytes_written=8 * n, launches=3)))
        return
    if args.adjoint_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(adjoint_cost(torch, steps=args.adjoint_only, fd=False)), flush=True)
        return
    if args.mixed_accuracy:
        print(json.dumps(mixed_accuracy(args.mixed_accuracy, args.steps)), flush=True)
        return
    if args.paper_workloads_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(paper_workloads(torch, args.steps, args.warmup, args.paper_workloads_only)), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} (WORLD_SIZE {world}) is not supported: "
              "the library has no multi-GPU path (one process drives one GPU).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2504_14063_amd import inputs, mpmc
    torch.cuda.set_device(0)
    case = inputs.droplet_crossflow_3d(n=args.n)
    cells = case.ncell
    log(f"bench: workload {case.name} {args.n}^3, {cells} cells, steps {args.steps}, warmup {args.warmup}")
    prec_main = 1 if args.precision == "mixed" else 0
    ctx = mpmc.Context.from_case(case, precision=prec_main, step_layout=1 if args.step_layout == "split" else 2)
    U0 = ctx.init_state_from_case(case)
    torch.cuda.synchronize()
    U = U0.clone()
    elapsed, prof = time_forward(torch, ctx, U, args.steps, args.warmup)
    st = ctx.mpmc_stats(reset=True)
    value = cells * args.steps / elapsed
    ms_step = 1e3 * elapsed / args.steps
    log(f"bench: {args.precision} {value:.4e} cell-updates/s, {ms_step:.2f} ms/step, limiter {st}")
    log("bench: kernel ms (sum, launches):", {k: (round(v[0], 3), v[1]) for k, v in prof.items()})

    # roofline of the dominant kernel (FP64 VALU binds: the counted
    # operations per face over the achieved launch time, HBM beside it)
    dom = max((k for k in prof if prof[k][1] > 0), key=lambda k: prof[k][0])
    ops = load_ops()
    roof = None
    if dom.startswith("face") and dom in ops:
        d = "xyz".index(dom[-1])
        faces = 1
        for k in range(3):
            faces *= case.n[k] + (1 if k == d else 0)
        avg_s = 1e-3 * prof[dom][0] / prof[dom][1]
        achieved = ops[dom] * faces / avg_s
        traffic = measured_traffic(f"k_face<3, 3, {d}, double, false, false, false>") \
            if args.step_layout == "split" and prec_main == 0 else None
        roof = dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_FP64_FLOPS / 1e12, unit="TFLOP/s",
                    frac=achieved / PEAK_FP64_FLOPS, traffic=traffic, kernel=dom,
                    avg_launch_ms=1e3 * avg_s, ops_per_face=ops[dom], faces_per_launch=faces,
                    hbm_achieved_GBps=None if traffic is None else traffic / avg_s / 1e9,
                    hbm_frac=None if traffic is None else traffic / avg_s / PEAK_HBM)

    out = dict(metric=METRIC, value=value, unit="cell-updates/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=ms_step, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f64" if prec_main == 0 else "f64+f32",
               data="synthetic (seeded generator, random-free physics ICs)",
               config=dict(workload=f"droplet_crossflow_3d {args.n}^3 (3 components, 2 phases, CDI + "
                                    f"diffusion, periodic)", cells=cells, precision=args.precision,
                           step_layout=args.step_layout),
               limiter=dict(fallback=st["fallback"], cdi_drop=st["cdi_drop"], faces=st["faces"],
                            unrecoverable=st["unrecoverable"]),
               kernels_ms={k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1]},
               roofline=roof)
    del U
    ctx.close()

    if not args.no_mixed and prec_main == 0:
        ctxm = mpmc.Context.from_case(case, precision=1)
        Um = U0.clone()
        em, profm = time_forward(torch, ctxm, Um, args.steps, args.warmup)
        vm = cells * args.steps / em
        out["mixed"] = dict(value=vm, ms_per_step=1e3 * em / args.steps, speedup=vm / value,
                            kernels_ms={k: v[0] / max(v[1], 1) for k, v in profm.items() if v[1]})
        log(f"bench: mixed {vm:.4e} cell-updates/s ({vm / value:.2f}x)")
        ctxm.close()
        del Um

    if not args.no_mixed and not args.no_mixed_accuracy and prec_main == 0:
        # the mixed form's accuracy at the 512^3 size of the same physics,
        # 100 steps at the FP64 run's dt and Gamma
        out["mixed_accuracy"] = mixed_accuracy(512, 100)
        log("bench: mixed accuracy", out["mixed_accuracy"])

    if not args.no_viscous and prec_main == 0:
        # the same workload with viscous stress and heat conduction on
        ctxv = mpmc.Context.from_case(case, viscous=1, prandtl=0.71)
        Uv = U0.clone()
        ev, profv = time_forward(torch, ctxv, Uv, args.steps, args.warmup)
        vv = cells * args.steps / ev
        out["viscous"] = dict(value=vv, ms_per_step=1e3 * ev / args.steps, relative=vv / value,
                              kernels_ms={k: v[0] / max(v[1], 1) for k, v in profv.items() if v[1]})
        log(f"bench: viscous {vv:.4e} cell-updates/s ({vv / value:.2f}x of the inviscid FP64 step)")
        ctxv.close()
        del Uv

    if not args.no_variants and prec_main == 0:
        # the same workload with the scheme variants in place of WENO5-Z,
        # with the five-equation interpolation basis (negative control), and
        # in the fused step layout (the same bits, another kernel split)
        for name, over in (("weno5js", dict(weno=1, weno_eps=1e-6, weno_p=2)),
                           ("teno5", dict(weno=2, weno_eps=1e-40)), ("teno6", dict(weno=3, weno_eps=1e-40)),
                           ("five_equation_basis", dict(basis=1, weno=0, weno_eps=1e-6, weno_p=2)),
                           ("fused_layout", dict(step_layout=2))):
            ctxs = mpmc.Context.from_case(case, **over)
            Us = U0.clone()
            es, profs = time_forward(torch, ctxs, Us, args.steps, args.warmup)
            vs = cells * args.steps / es
            out[name] = dict(value=vs, ms_per_step=1e3 * es / args.steps, relative=vs / value,
                             kernels_ms={k: v[0] / max(v[1], 1) for k, v in profs.items() if v[1]})
            log(f"bench: {name} {vs:.4e} cell-updates/s ({vs / value:.2f}x of the default step)")
            ctxs.close()
            del Us

    if not args.no_variants and prec_main == 0:
        # the cost of the iterative pressure (several distinct P_inf): the
        # same state with the second gas given a small stiffening pressure
        eos = case.eos_dict()
        eos["pinf"] = list(eos["pinf"])
        eos["pinf"][2] = 1e4
        ctxg = mpmc.Context(case.grid_dict(), eos, dict(case.opts))
        Ug = U0.clone()
        eg, profg = time_forward(torch, ctxg, Ug, args.steps, args.warmup)
        vg = cells * args.steps / eg
        out["general_eos"] = dict(value=vg, ms_per_step=1e3 * eg / args.steps, relative=vg / value,
                                  kernels_ms={k: v[0] / max(v[1], 1) for k, v in profg.items() if v[1]})
        log(f"bench: general_eos {vg:.4e} cell-updates/s ({vg / value:.2f}x of the default step)")
        ctxg.close()
        del Ug

    if not args.no_variants and prec_main == 0:
        # the same workload with characteristic (non-reflecting) boundaries on
        # both x sides in place of the periodic wrap, relaxed toward the
        # crossflow's far-field gas state (P, T of the initial condition, the
        # two gases at 0.7 / 0.3, u = 50 m/s)
        grid = case.grid_dict()
        grid["bc_lo"][0] = grid["bc_hi"][0] = 3
        ctxc = mpmc.Context(grid, case.eos_dict(), dict(case.opts))
        for side in (0, 1):
            ctxc.mpmc_set_boundary_target(0, side, 1e5, 300.0, [0.0, 0.7, 0.3], [50.0, 0.0, 0.0], 0.25)
        Uc = U0.clone()
        ec, profc = time_forward(torch, ctxc, Uc, args.steps, args.warmup)
        vc = cells * args.steps / ec
        out["characteristic_x"] = dict(value=vc, ms_per_step=1e3 * ec / args.steps, relative=vc / value,
                                       kernels_ms={k: v[0] / max(v[1], 1) for k, v in profc.items() if v[1]})
        log(f"bench: characteristic x boundaries {vc:.4e} cell-updates/s ({vc / value:.2f}x of the default step)")
        ctxc.close()
        del Uc

    if not args.no_variants and prec_main == 0:
        # the same workload with the configuration's plain logistic edges
        # (volume fractions not floored at phi_min): most faces then drop the
        # regularization flux, which changes the cost per face
        case_t = inputs.droplet_crossflow_3d(n=args.n, floor=False)
        ctxt = mpmc.Context.from_case(case_t, raise_inadmissible=False)
        Ut = ctxt.init_state_from_case(case_t)
        ctxt.mpmc_stats(reset=True)
        et, proft = time_forward(torch, ctxt, Ut, args.steps, args.warmup)
        stt = ctxt.mpmc_stats(reset=True)
        vt = cells * args.steps / et
        out["plain_logistic_ic"] = dict(value=vt, ms_per_step=1e3 * et / args.steps, relative=vt / value,
                                        limiter=dict(fallback=stt["fallback"], cdi_drop=stt["cdi_drop"],
                                                     faces=stt["faces"], unrecoverable=stt["unrecoverable"]),
                                        kernels_ms={k: v[0] / max(v[1], 1) for k, v in proft.items() if v[1]})
        log(f"bench: plain logistic edges {vt:.4e} cell-updates/s ({vt / value:.2f}x), limiter {stt}")
        ctxt.close()
        del Ut

    if not args.no_variants and prec_main == 0:
        # the same physics at smaller sizes: how far the step is from
        # filling the chip (the 512^3 rate is in mixed_accuracy)
        sweep = {}
        for m in (64, 128):
            case_m = inputs.droplet_crossflow_3d(n=m)
            ctxm_ = mpmc.Context.from_case(case_m)
            Um_ = ctxm_.init_state_from_case(case_m)
            em_, _ = time_forward(torch, ctxm_, Um_, args.steps, args.warmup, profile=False)
            sweep[f"{m}^3"] = dict(value=case_m.ncell * args.steps / em_, ms_per_step=1e3 * em_ / args.steps)
            ctxm_.close()
            del Um_
        sweep[f"{args.n}^3"] = dict(value=value, ms_per_step=ms_step)
        out["size_sweep"] = sweep
        log("bench: size sweep", sweep)

    if not args.no_variants and prec_main == 0:
        out["paper_workloads"] = paper_workloads(torch, args.steps, args.warmup)

    if not args.no_adjoint and prec_main == 0:
        out["adjoint"] = adjoint_cost(torch)
        log("bench: adjoint", out["adjoint"])

    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(case)
            log("bench: cpu baseline", out["cpu_baseline"])
        except Exception as e:  # the baseline is context only
            out["cpu_baseline"] = dict(error=str(e))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
