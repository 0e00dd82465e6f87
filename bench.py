"""Benchmark: the order-6 FP32 curvilinear layered workload on one GPU.

One step = five Runge-Kutta stages of the full semi-discrete right-hand side
(volume terms, boundary penalties, point source) fused with the stage update,
plus the receiver gather.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 2000] [--warmup 20] [--no-cpu]
    python bench.py --workload batched [--steps 100] [--warmup 5]

The metric is Mpts*stage/s (grid points times Runge-Kutta stages per
second).  A Runge-Kutta stage is the stage kernel over the tiled nodes (all
but the last q column and r row), the edge kernel over the rest, the
boundary-penalty kernel and the source kernel.  The roofline object reports
the stage kernel: algorithmic bytes of the nodes one launch computes over its
average launch duration, timed by the library's events around each launch
(sbp_set_profiling), against the 8 TB/s HBM peak and against the copy
ceiling a plain device copy reaches in the same run; `traffic` is the HBM
bytes per launch from the committed rocprofv3 counter summary when that was
taken on the current sources.  The same workload in double precision follows
as the `fp64` object.  cpu_baseline times the CPU oracle on a bounded sample
of the same workload.

`--workload batched` measures the batched-shots workload instead (32 cubes
of uneven size, orders 4 and 6, one sbp_step_batch call): shots per second
for `steps` steps per shot, beside the same shots stepped one after another.

`--workload surrogate` trains the spectral neural operator on solver-made
seismograms (64^3 Gaussian-random-field media, 64 receivers x 512 samples)
and reports its speedup over the solver on held-out media, with the
fallback to the solver for media outside its calibrated error budget.

`--workload orders` compares the interior orders 2-8 at marginal resolution
on the topography geometry against 2x refined runs of the same order.

`--workload adjoint` measures the material gradient (sbp_gradient): the
topo_layer block at 129^3, order 6, FP32, a model and a target model with 5 %
smooth perturbations of rho, lambda and mu, 64 receivers, 1500 steps with a
checkpoint every 100 steps; gradients per second, beside the forward run.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0  # dense BF16 matrix-core peak
# algorithmic words per node per stage: read Q_in (9) + 13 coefficients (the
# nine metric terms, J^-1, (rho J)^-1, lambda, mu), read the Runge-Kutta
# register (9, stages 2-5 only), write it (9) and Q_out (9): 40 words in the
# first stage, 49 in the others, 47.2 on average
WORDS_STAGE1 = 9 + 13 + 9 + 9
WORDS_STAGE = WORDS_STAGE1 + 9
WORDS_AVG = (WORDS_STAGE1 + 4 * WORDS_STAGE) / 5.0
# the library stores 12 coefficient words (J folded into lambda/J, mu/J and
# 1/(rho J)): 46.2 words on average, reported beside the figure above
WORDS_AVG_STORED = WORDS_AVG - 1.0
PROFILE = os.path.join(ROOT, "profiles", "stage_kernel_topo_layer_257x257x193.md")
CSRC = os.path.join(ROOT, "paper_2011_02600_amd", "csrc")


# sources that decide the stage kernel's code, launch shape and data layout
STAGE_SOURCES = ("api.cpp", "internal.hpp", "kernels.hip", "kernels.hpp", "penalty.hpp")


def kernel_sha():
    """sha256 (16 hex digits) of the library sources behind the stage kernel:
    its code, tiling and layout."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name in STAGE_SOURCES:
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def read_traffic(key="hbm_bytes_per_launch"):
    """HBM bytes per stage launch (`key`: hbm_bytes_per_launch for the
    single-precision kernel, hbm_bytes_per_launch_f64 for the double-precision
    one) from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source (else None)."""
    if not os.path.exists(PROFILE):
        return None
    vals = {}
    for line in open(PROFILE):
        line = line.strip().lstrip("-* ")
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256_16") != kernel_sha():
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def copy_ceiling(torch, dev, mib=1024, reps=10):
    """HBM bandwidth a plain device copy reaches on this GPU (read + write
    bytes over the time of `reps` copies of `mib` MiB, events on the current
    stream): the streaming ceiling the stage kernel is compared with."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * 4 * n * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    return gbs


def cpu_baseline(wl, order=6, nstages=5):
    """The CPU oracle as it stands, timed on the host: `nstages` Runge-Kutta
    stages (right-hand side + stage update; at most 5, one whole step) of the
    full workload."""
    import numpy as np
    from oracle import elastic as E
    from oracle import lsrk
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    blk = E.Block(wl["xyz"], order).set_material(wl["rho"], wl["cp"], wl["cs"])
    src = E.Source(blk, wl["src_xi"], wl["src_M"], E.STF_RICKER, wl["src_f0"], wl["src_t0"])
    Q = np.array(wl["Q0"], dtype=np.float64)
    dQ = np.zeros_like(Q)
    dt = wl["dt"]
    t0 = time.perf_counter()
    for k in range(nstages):
        dQ *= lsrk.A_F[k]
        dQ += dt * E.rhs(blk, Q, lsrk.C_F[k] * dt, wl["gamma"], sources=[src])
        Q += lsrk.B_F[k] * dQ
    el = time.perf_counter() - t0
    nodes = Q[0].size
    return {"value": nodes * nstages / el / 1e6, "unit": "Mpts*stage/s", "cores": cores, "kind": "oracle",
            "sample": "%d Runge-Kutta stages (RHS + update) of the full %dx%dx%d workload in float64 numpy, "
                      "%.1f s; mesh/metric setup excluded" % ((nstages,) + tuple(Q.shape[1:][::-1]) + (el,))}


def run_adjoint(args, W, sbp, torch, np, dev):
    """Misfit gradient of the 129^3 adjoint workload: the target traces and
    the model traces come from forward runs (untimed); the timed region is
    one sbp_gradient call (its checkpointed forward run, the block
    recomputations and the reverse sweep), beside one plain forward run."""
    steps, every = args.adjoint_steps, args.every
    print("bench: generating the adjoint workload", file=sys.stderr, flush=True)
    wl = W.adjoint_case()
    ns, nr, nq = wl["xyz"].shape[1:]
    s = sbp.Solver(wl["xyz"], order=6, dtype="f32", gamma=wl["gamma"], device=dev)
    s.add_source(wl["src_xi"], wl["src_M"], sbp.SBP_STF_RICKER, wl["src_f0"], wl["src_t0"])
    s.set_material(*wl["model"])
    ty, zc, _ = s.autotune()
    dt = wl["dt"]
    Q0 = torch.zeros((9, ns, nr, nq), dtype=torch.float32, device=dev)

    def forward(mat):
        s.set_material(*mat)
        s.set_state(Q0, 0.0)
        tr = s.record(wl["receivers"], steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps, dt)
        torch.cuda.synchronize()
        return tr.clone(), time.perf_counter() - t0

    target, _ = forward(wl["target"])
    traces, _ = forward(wl["model"])
    _, fwd_s = forward(wl["model"])
    res = traces - target
    misfit = 0.5 * float((res.double() ** 2).sum())
    for _ in range(args.warmup_grad):
        s.set_state(Q0, 0.0)
        s.gradient(min(steps, 2 * every), dt, res[:min(steps, 2 * every)], every)
    s.set_state(Q0, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grad = s.gradient(steps, dt, res, every)
    torch.cuda.synchronize()
    grad_s = time.perf_counter() - t0
    g = grad.double()
    if not bool(torch.isfinite(g).all()):
        raise RuntimeError("non-finite gradient")
    # the autograd path: a checkpointed forward run, then the reverse sweep alone
    s.set_state(Q0, 0.0)
    s.record(wl["receivers"], steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step_checkpointed(steps, dt, every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    grad2 = s.gradient_from_checkpoints(res)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fwd_ck_s, rev_s = t1 - t0, t2 - t1
    if not torch.equal(grad2, grad):
        raise RuntimeError("gradient from checkpoints differs from sbp_gradient")
    nbytes = sbp.sbp_adjoint_bytes(s.h, steps, every)
    print("bench: gradient of %d steps in %.3f s, forward %.3f s" % (steps, grad_s, fwd_s), file=sys.stderr,
          flush=True)
    s.close()
    out = {
        "metric": "gradients/s (d misfit / d (rho, lambda, mu), 129^3 order-6 FP32 curvilinear, %d steps)" % steps,
        "value": round(1.0 / grad_s, 4),
        "unit": "gradients/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup_grad,
        "ms_per_step": round(1e3 * grad_s / steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "adjoint: topo_layer block %dx%dx%d (order 6), model and target model = layered "
                               "medium x (1 + smooth seeded perturbations of rho, lambda, mu, max 5 %%), "
                               "64 surface receivers, Ricker moment source, CFL 0.5, misfit = 1/2 L2 of "
                               "the trace residual" % (nq, nr, ns),
                   "grid": [nq, nr, ns], "nodes": nq * nr * ns, "checkpoint_every": every, "dt": dt,
                   "launch": {"ty": ty, "zchunk": zc},
                   "adjoint_workspace_bytes": nbytes},
        "gradient_s": round(grad_s, 4),
        "forward_s": round(fwd_s, 4),
        "gradient_over_forward": round(grad_s / fwd_s, 3),
        "autograd_path": {"forward_checkpointed_s": round(fwd_ck_s, 4), "reverse_from_checkpoints_s": round(rev_s, 4),
                          "forward_plus_backward_over_forward": round((fwd_ck_s + rev_s) / fwd_s, 3)},
        "misfit": misfit,
        "grad_max_abs": [float(g[i].abs().max()) for i in range(3)],
    }
    print(json.dumps(out), flush=True)


def run_surrogate(args, W, sbp, torch, np, dev):
    """Learned surrogate: solver-made training data, GPU training, held-out
    evaluation with fallback; value = speedup of surrogate + fallback over
    the solver alone on the held-out media."""
    from paper_2011_02600_amd import nn
    from paper_2011_02600_amd import surrogate as SG
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    case = W.surrogate_case(T=args.sur_T, amp=args.sur_amp)
    ntr, nte = args.sur_train, args.sur_test
    nval = max(1, ntr // 10)
    log("surrogate: generating %d media" % (ntr + nte))
    fields = W.surrogate_fields(case, ntr + nte, seed=0)
    log("surrogate: solving %d shots" % (ntr + nte))
    y, gen_s = SG.solve_batch(sbp, torch, case, fields, dev, log=log)
    d = torch.tensor(np.stack(fields), dtype=torch.float32, device=dev)
    sur = SG.Surrogate(nn, torch, case, dev, members=args.sur_members)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = sur.train(d[:ntr - nval], y[:ntr - nval], epochs=args.sur_epochs, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    val_err, val_sc = sur.calibrate(d[ntr - nval:ntr], y[ntr - nval:ntr])
    # held-out media: the solver alone, then the surrogate (timed separately)
    log("surrogate: held-out solver run")
    y_test, solver_s = SG.solve_batch(sbp, torch, case, fields[ntr:], dev, log=log)
    dt_ = d[ntr:].contiguous()
    sur.predict(dt_[:8])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred, score = sur.predict_with_score(dt_)
    torch.cuda.synchronize()
    infer_s = time.perf_counter() - t0
    err = SG.Surrogate.rel_err(pred, y_test)
    err_mean_trace = SG.Surrogate.rel_err(sur.ymean.expand_as(y_test), y_test)
    acc = score <= sur.tau
    # the rejected media go to the solver (its batched time per shot)
    mixed_s = infer_s + solver_s * float(np.mean(~acc))
    # other error budgets: threshold from the calibration samples, then the
    # held-out acceptance and the combined speedup
    sweep = []
    for budget in (0.05, 0.10, 0.15, 0.20):
        tau = SG.Surrogate.threshold(val_err, val_sc, budget)
        ok = score <= tau
        sweep.append({"budget_p95": budget, "accepted": int(ok.sum()),
                      "accepted_rel_l2_p95": float(np.quantile(err[ok], 0.95)) if ok.any() else None,
                      "speedup": round(solver_s / (infer_s + solver_s * float(np.mean(~ok))), 3)})
    rank = lambda a: np.argsort(np.argsort(a))
    spearman = float(np.corrcoef(rank(score), rank(err))[0, 1])
    # the network's GEMMs over one training step (forward + backward, one
    # batch of 8 media, first member): flops, algorithmic bytes and time
    net = sur.nets[0]
    xb = sur._x(d[:8]).contiguous()
    net.forward(xb)
    torch.cuda.synchronize()
    nn.gemm_profile(True)
    out8 = net.forward(xb)
    _, dy8 = net.loss(out8, ((y[:8] - sur.ymean) / sur.yscale).contiguous(), scale=1.0 / 8)
    net.backward(dy8)
    torch.cuda.synchronize()
    gs = nn.gemm_profile_summary(nn.gemm_profile(False))
    ai = gs["flops"] / gs["bytes"]
    tflops = gs["flops"] / (gs["ms"] / 1e3) / 1e12
    gbs = gs["bytes"] / (gs["ms"] / 1e3) / 1e9
    bound = "hbm" if ai < PEAK_BF16_TFLOPS * 1e3 / PEAK_HBM_GBS else "mfma"
    out = {
        "metric": "speedup over the solver (surrogate with fallback, held-out media, <= 5 %% relative L2 "
                  "trace error on the accepted ones)",
        "value": round(solver_s / mixed_s, 3),
        "unit": "x",
        "n_gpus": 1,
        "steps": case["T"],
        "warmup": 1,
        "ms_per_step": round(1e3 * mixed_s / case["T"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 (network GEMMs, fp32 accumulation) / f32 (solver)",
        "data": "synthetic",
        "config": {"workload": "surrogate: %d^3 cube, order-%d FP32 solver, media = half-space x (1 + d), d a "
                               "Gaussian random field (correlation %d cells, max |d| = %g) on cp and cs, Ricker "
                               "source, %d receivers x %d samples of v_z; spectral operator (4 cosine-spectral "
                               "layers, width 32, 8^3 modes)" % (case["n"], case["order"], case["corr_cells"],
                                                                 case["amp"], len(case["receivers"]), case["T"]),
                   "train": ntr - nval, "calibration": nval, "test": nte, "epochs": args.sur_epochs,
                   "members": len(sur.nets)},
        "solver_s_per_shot": round(solver_s / nte, 5),
        "surrogate_s_per_shot": round(infer_s / nte, 6),
        "surrogate_only_speedup": round(solver_s / infer_s, 2),
        "test_rel_l2": {"mean": float(np.mean(err)), "median": float(np.median(err)),
                        "p95": float(np.quantile(err, 0.95)), "max": float(np.max(err))},
        "calibration_rel_l2_mean": float(np.mean(val_err)),
        "mean_trace_rel_l2_mean": float(np.mean(err_mean_trace)),
        "fallback": {"score": "relative L2 spread of the %d networks' predictions (a predicted error)"
                              % len(sur.nets),
                     "threshold": None if not np.isfinite(sur.tau) else float(sur.tau),
                     "spearman_score_vs_error": round(spearman, 3),
                     "accepted": int(acc.sum()), "rejected": int((~acc).sum()),
                     "accepted_rel_l2_mean": float(np.mean(err[acc])) if acc.any() else None,
                     "accepted_rel_l2_p95": float(np.quantile(err[acc], 0.95)) if acc.any() else None,
                     "accepted_rel_l2_max": float(np.max(err[acc])) if acc.any() else None,
                     "accepted_within_5pct": float(np.mean(err[acc] <= 0.05)) if acc.any() else None,
                     "rejected_rel_l2_mean": float(np.mean(err[~acc])) if (~acc).any() else None,
                     "budgets": sweep},
        "roofline": {"bound": bound, "kernel": "gemm_kernel (all GEMMs of one training step, 8 media)",
                     "achieved": round(gbs if bound == "hbm" else tflops, 1),
                     "peak": PEAK_HBM_GBS if bound == "hbm" else PEAK_BF16_TFLOPS,
                     "unit": "GB/s" if bound == "hbm" else "TFLOP/s",
                     "frac": round((gbs / PEAK_HBM_GBS) if bound == "hbm" else (tflops / PEAK_BF16_TFLOPS), 4),
                     "traffic": None, "gemm_calls": gs["calls"], "gemm_ms": round(gs["ms"], 3),
                     "flops": gs["flops"], "algorithmic_bytes": gs["bytes"], "flop_per_byte": round(ai, 2),
                     "tflops": round(tflops, 2), "gbs": round(gbs, 1)},
        "train_s": round(train_s, 2),
        "data_generation_s": round(gen_s, 2),
        "final_train_loss": hist[-1] if hist else None,
    }
    print(json.dumps(out), flush=True)


def run_orders(args, W, sbp, torch, np, dev):
    """Odd and even interior orders at marginal resolution on synthetic
    topography: the topo_layer geometry (seeded topography, free surface,
    moment source, 64 surface receivers) with a homogeneous half-space and a
    4 Hz Ricker wavelet, on a coarse 129 x 129 x 97 grid (8.7 points per S
    wavelength at the peak frequency, 3.5 at 2.5 f0) at CFL 0.25 (stable for
    every order) for every order the library runs, against the 2x
    refined grid (257 x 257 x 193, half the time step, same receivers) run
    with the same order.  Reports the relative L2 difference of the receiver
    traces per order."""
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    coarse = W.topo_layer(nq=129, nr=129, ns=97, nrec_side=8, cfl=0.25, f0=4.0)
    fine = W.topo_layer(nq=257, nr=257, ns=193, nrec_side=8, f0=4.0)
    assert np.array_equal(fine["receivers"][:, :2], 2 * coarse["receivers"][:, :2])
    # homogeneous half-space under the topography: a point-sampled layer
    # interface would add a first-order error that hides the operators'
    for wl in (coarse, fine):
        shape = wl["rho"].shape
        wl["rho"], wl["cp"], wl["cs"] = np.full(shape, 2.7), np.full(shape, 6.0), np.full(shape, 3.464)
    dt = coarse["dt"]
    tend = args.orders_time
    nc = int(round(tend / dt))

    def traces(wl, order, dtt, nsteps):
        s = sbp.Solver(wl["xyz"], order=order, dtype="f32", gamma=wl["gamma"], device=dev)
        s.set_material(wl["rho"], wl["cp"], wl["cs"])
        s.add_source(wl["src_xi"], wl["src_M"], sbp.SBP_STF_RICKER, wl["src_f0"], wl["src_t0"])
        tr = s.record(wl["receivers"], nsteps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(nsteps, dtt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out = tr.double().cpu().numpy()
        s.close()
        return out, el

    res = {}
    for order in (2, 3, 4, 5, 6, 7, 8):
        # reference: the same order on the refined grid (self-convergence,
        # the same yardstick for every order)
        ref, _ = traces(fine, order, dt / 2, 2 * nc)
        ref = ref[1::2]  # the fine steps that end at the coarse times
        tr, el = traces(coarse, order, dt, nc)
        err = float(np.linalg.norm(tr - ref) / np.linalg.norm(ref))
        res[str(order)] = {"rel_l2": round(err, 5), "s": round(el, 3)}
        log("orders: order %d: relative L2 trace difference to its 2x refined run %.4f (%.2f s)" % (order, err, el))
    out = {
        "metric": "relative L2 receiver-trace difference to the 2x refined run, per interior order (lower is better)",
        "value": res["6"]["rel_l2"],
        "unit": "relative L2",
        "n_gpus": 1,
        "steps": nc,
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "odd/even orders: topo_layer geometry, homogeneous half-space, on 129 x 129 x "
                               "97 (h = 100 m horizontally), 4 Hz Ricker, 64 surface receivers, %.1f s, CFL "
                               "0.25; reference: the same order on 257 x 257 x 193 with dt/2" % tend, "dt": dt},
        "per_order": res,
    }
    print(json.dumps(out), flush=True)


def run_batched(args, W, sbp, torch, np, dev):
    steps = args.steps if args.steps != 2000 else 100
    warm = args.warmup if args.warmup != 20 else 5
    print("bench: generating 32 shots", file=sys.stderr, flush=True)
    shots = W.batched_shots(32)
    solvers = []
    shapes = []
    for n, sh in enumerate(shots):
        s = sbp.Solver(sh["xyz"], order=sh["order"], dtype="f32", gamma=sh["gamma"], device=dev)
        s.set_material(sh["rho"], sh["cp"], sh["cs"])
        s.add_source(sh["src_xi"], sh["src_M"], sbp.SBP_STF_RICKER, sh["src_f0"], sh["src_t0"])
        s.record(sh["receivers"], 2 * (warm + steps))
        ty, zc, _ = s.autotune(3)
        shapes.append((ty, zc))
        solvers.append(s)
        print("bench: shot %d: %d^3 order %d, launch ty %d zchunk %d" % (n, sh["xyz"].shape[1], sh["order"], ty, zc),
              file=sys.stderr, flush=True)
    hs = [s.h for s in solvers]
    # the batch's own launch shape: s-chunk length of the persistent stage
    # launch over every shot's tiles
    batch_L, batch_stage_ms = sbp.sbp_autotune_batch(hs, 3)
    print("bench: batch autotune: s-chunk %d, %.3f ms per batched stage launch" % (batch_L, batch_stage_ms),
          file=sys.stderr, flush=True)
    dts = [sh["dt"] for sh in shots]
    stream = solvers[0].stream
    points = sum(int(np.prod(sh["xyz"].shape[1:])) for sh in shots)
    sbp.sbp_step_batch(hs, warm, dts)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sbp.sbp_step_batch(hs, steps, dts)
    e1.record(stream)
    torch.cuda.synchronize()
    batch_ms = e0.elapsed_time(e1)
    print("bench: batched %d steps in %.1f ms" % (steps, batch_ms), file=sys.stderr, flush=True)
    # the same shots one after another, each with its own sbp_step call
    e0.record(stream)
    for s, d in zip(solvers, dts):
        s.step(steps, d)
    e1.record(stream)
    torch.cuda.synchronize()
    seq_ms = e0.elapsed_time(e1)
    print("bench: one by one %d steps in %.1f ms" % (steps, seq_ms), file=sys.stderr, flush=True)
    for s in solvers:
        if not np.all(np.isfinite(s.traces.float().cpu().numpy())):
            raise RuntimeError("non-finite receiver traces")
        s.close()
    secs = batch_ms / 1e3
    bytes_stage = WORDS_AVG * 4 * points
    out = {
        "metric": "shots/s (batched shots, %d steps per shot)" % steps,
        "value": round(len(shots) / secs, 3),
        "unit": "shots/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(batch_ms / steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched_shots: 32 cubes of 65^3..193^3 points (seeded sizes), orders 4/6 "
                               "alternating, Gaussian-random-field media (10-cell correlation, +-10 %), "
                               "Ricker moment source, 16 surface receivers each, CFL 0.5",
                   "sizes": [int(sh["xyz"].shape[1]) for sh in shots],
                   "orders": [sh["order"] for sh in shots], "points": points,
                   "launch": "one stage launch per Runge-Kutta stage over a work list of the tiles and edge blocks of "
                             "all 32 shots (8-row tiles, s-chunk %d from the batch autotuner), steps replayed "
                             "from captured graphs" % batch_L,
                   "single_shot_launch": [{"ty": t, "zchunk": z} for t, z in shapes]},
        "batch_stage_launch_ms": round(batch_stage_ms, 4),
        "mpts_stage_per_s": round(points * 5 * steps / secs / 1e6, 1),
        "one_by_one": {"ms": round(seq_ms, 2), "shots_per_s": round(len(shots) / (seq_ms / 1e3), 3),
                       "batch_speedup": round(seq_ms / batch_ms, 3)},
        "stage_rate": {"scope": "whole Runge-Kutta stage of all shots (stage, edge and source kernels)",
                       "algorithmic_gbs": round(bytes_stage * 5 * steps / secs / 1e9, 1),
                       "frac_of_peak": round(bytes_stage * 5 * steps / secs / 1e9 / PEAK_HBM_GBS, 4)},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--kernel-steps", type=int, default=200,
                    help="steps of the stage-kernel-only timing region")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the double-precision run of the same workload (the fp64 object)")
    ap.add_argument("--ty", type=int, default=8)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"],
                    help="arithmetic of the topo_layer workload (f64: order 2 to 6)")
    ap.add_argument("--zchunk", type=int, default=0)
    ap.add_argument("--order", type=int, default=6, choices=[2, 3, 4, 5, 6, 7, 8],
                    help="interior order of the topo_layer run (the headline workload is order 6)")
    ap.add_argument("--workload", default="topo_layer",
                    choices=["topo_layer", "batched", "adjoint", "surrogate", "orders"])
    ap.add_argument("--orders-time", type=float, default=4.0, help="simulated seconds (orders workload)")
    ap.add_argument("--sur-train", type=int, default=2000, help="solver-made training media (surrogate workload)")
    ap.add_argument("--sur-test", type=int, default=200, help="held-out media (surrogate workload)")
    ap.add_argument("--sur-epochs", type=int, default=30, help="training epochs (surrogate workload)")
    ap.add_argument("--sur-T", type=int, default=512, help="time samples per trace (surrogate workload)")
    ap.add_argument("--sur-amp", type=float, default=0.02, help="max |d| of the media (surrogate workload)")
    ap.add_argument("--sur-members", type=int, default=2, help="networks in the ensemble (surrogate workload)")
    ap.add_argument("--adjoint-steps", type=int, default=1500, help="steps of the adjoint workload")
    ap.add_argument("--every", type=int, default=100, help="checkpoint interval of the adjoint workload")
    ap.add_argument("--warmup-grad", type=int, default=1, help="untimed short gradient runs (adjoint workload)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (x4) for HBM counter calibration")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver advances one block on one GPU "
              "(sharding across GPUs is not implemented).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2011_02600_amd import sbp

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read_per_copy": 4 * n, "copies": 4}))
        return
    if args.workload == "batched":
        run_batched(args, W, sbp, torch, np, dev)
        return
    if args.workload == "adjoint":
        run_adjoint(args, W, sbp, torch, np, dev)
        return
    if args.workload == "surrogate":
        run_surrogate(args, W, sbp, torch, np, dev)
        return
    if args.workload == "orders":
        run_orders(args, W, sbp, torch, np, dev)
        return
    print("bench: generating workload", file=sys.stderr, flush=True)
    # the interior symbols of orders 2 and 4 reach larger magnitudes than
    # order 6's (4 and 8/3 against 2.19), so the other orders run at CFL 0.25,
    # stable for all of them (the throughput does not depend on dt)
    wl = W.topo_layer() if args.order == 6 else W.topo_layer(cfl=0.25)
    ns, nr, nq = wl["xyz"].shape[1:]
    nodes = nq * nr * ns
    order = args.order
    m = measure_topo(args, wl, args.dtype, order, sbp, torch, np, dev)
    ceiling = copy_ceiling(torch, dev)
    traffic = read_traffic() if order == 6 and args.dtype == "f32" else None
    out = {
        "metric": "Mpts*stage/s (order-%d %s curvilinear RHS + LSRK4 stage update)"
                  % (order, {"f32": "FP32", "f64": "FP64"}[args.dtype]),
        "value": m["value"],
        "unit": "Mpts*stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "topo_layer: order-%d upwind SBP, curvilinear 257x257x193 (q,r,s) block under "
                               % order +
                               "seeded topography, 1 km layer over half-space, Ricker moment source, "
                               "64 surface receivers, CFL %.2g" % (0.5 if order == 6 else 0.25),
                   "grid": [nq, nr, ns], "nodes": nodes, "order": order, "dt": wl["dt"],
                   "launch": {"ty": args.ty, "zchunk": args.zchunk}},
        "roofline": dict(m["roofline"], traffic=None if traffic is None else int(traffic),
                         traffic_rate_gbs=None if traffic is None
                         else round(traffic / (m["roofline"]["avg_launch_ms"] / 1e3) / 1e9, 1),
                         copy_ceiling_gbs=round(ceiling, 1),
                         frac_of_copy_ceiling=round(m["roofline"]["achieved"] / ceiling, 4)),
    }
    if not args.no_fp64 and args.dtype == "f32":
        # the same workload in the paper's arithmetic (double precision)
        m64 = measure_topo(args, wl, "f64", order, sbp, torch, np, dev)
        t64 = read_traffic("hbm_bytes_per_launch_f64") if order == 6 else None
        r64 = dict(m64["roofline"], traffic=None if t64 is None else int(t64),
                   traffic_rate_gbs=None if t64 is None
                   else round(t64 / (m64["roofline"]["avg_launch_ms"] / 1e3) / 1e9, 1),
                   copy_ceiling_gbs=round(ceiling, 1),
                   frac_of_copy_ceiling=round(m64["roofline"]["achieved"] / ceiling, 4))
        out["fp64"] = {"value": m64["value"], "unit": "Mpts*stage/s", "ms_per_step": m64["ms_per_step"],
                       "steps": args.steps, "roofline": r64}
    if not args.no_cpu:
        print("bench: cpu oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, order)
    print(json.dumps(out), flush=True)


def measure_topo(args, wl, dtype, order, sbp, torch, np, dev):
    """Times the topo_layer workload in `dtype`: `args.steps` whole steps
    (stages, source, receivers) after `args.warmup` untimed ones, then the
    Runge-Kutta stage alone and the stage kernel's launches (library events
    on the solver's stream)."""
    ns, nr, nq = wl["xyz"].shape[1:]
    nodes = nq * nr * ns
    s = sbp.Solver(wl["xyz"], order=order, dtype=dtype, gamma=wl["gamma"], device=dev)
    s.set_material(wl["rho"], wl["cp"], wl["cs"])
    s.set_launch(args.ty, args.zchunk)
    s.add_source(wl["src_xi"], wl["src_M"], sbp.SBP_STF_RICKER, wl["src_f0"], wl["src_t0"])
    s.record(wl["receivers"], args.warmup + args.steps)
    stream = s.stream
    dt = wl["dt"]
    print("bench: %s warmup" % dtype, file=sys.stderr, flush=True)
    s.step(args.warmup, dt)
    torch.cuda.synchronize()

    # ---- timed region: the whole workload (stages + source + receivers)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    s.step(args.steps, dt)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1)
    secs = ms / 1e3
    value = nodes * 5 * args.steps / secs / 1e6
    traces = s.traces.float().cpu().numpy()
    if not np.all(np.isfinite(traces)):
        raise RuntimeError("non-finite receiver traces")
    print("bench: %s %d steps in %.3f s (events) / %.3f s (wall)" % (dtype, args.steps, secs, wall),
          file=sys.stderr, flush=True)

    # ---- the Runge-Kutta stage alone (same solver, no source, no receivers):
    # events on the solver's stream around the steps (stage + edge kernel per
    # stage), then the library's own events around every stage-kernel and
    # edge-kernel launch (sbp_set_profiling)
    sbp.sbp_record(s.h, 0, None, None, 0)
    sbp.sbp_clear_sources(s.h)
    k0 = torch.cuda.Event(enable_timing=True)
    k1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    k0.record(stream)
    s.step(args.kernel_steps, dt)
    k1.record(stream)
    torch.cuda.synchronize()
    rk_stage_ms = k0.elapsed_time(k1) / (5 * args.kernel_steps)
    s.set_profiling(True)
    s.step(args.kernel_steps // 4, dt)
    launch_ms, edge_ms, nprof, stage_nodes = s.profile()
    s.set_profiling(False)
    s.close()
    wbytes = 4 if dtype == "f32" else 8
    bytes_per_launch = WORDS_AVG * wbytes * stage_nodes
    achieved = bytes_per_launch / (launch_ms / 1e3) / 1e9
    achieved_stored = WORDS_AVG_STORED * wbytes * stage_nodes / (launch_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": None,
            "kernel": "stage_kernel<%s,%d,%d>" % ("float" if dtype == "f32" else "double", order, args.ty),
            "avg_launch_ms": round(launch_ms, 4),
            "launches_timed": nprof,
            "nodes_per_launch": stage_nodes,
            "algorithmic_bytes_per_launch": int(bytes_per_launch),
            "words_per_node": WORDS_AVG,
            "frac_stored_words": round(achieved_stored / PEAK_HBM_GBS, 4),
            "stored_words_per_node": WORDS_AVG_STORED,
            "edge_kernel_avg_launch_ms": round(edge_ms, 4),
            "rk_stage_ms": round(rk_stage_ms, 4)}
    return {"value": round(value, 2), "ms_per_step": round(ms / args.steps, 4), "roofline": roof}


if __name__ == "__main__":
    main()
