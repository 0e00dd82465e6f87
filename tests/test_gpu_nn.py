"""GPU checks of the surrogate kernels (include/sbp_nn.h): the BF16
matrix-core GEMM against a float64 product of the bf16-rounded operands
(strided, transposed, batched and ragged cases, each operand staged 16
bytes at a time along k, along its rows, or one element at a time), and the
spectral neural
operator's forward and backward passes against the float64 reference
network (oracle/fno.py) on the same parameters and inputs.

Bars: GEMM |C - C_ref| <= 2e-6 sum_k |a_ik b_kj| + 1e-30 per element (fp32
accumulation of exact bf16 products); network outputs and every parameter
gradient within 3e-2 relative L2 of the float64 reference (bf16 operands
through four layers; measured values are printed).
"""
import sys

import numpy as np
import pytest

from oracle import fno

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bf16(a):
    """Round to bfloat16 (nearest even), returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


GEMM_CASES = [
    # batch, M, N, K, a_trans, b_trans, beta
    (1, 70, 45, 37, False, False, 0.0),
    (1, 64, 64, 32, False, False, 0.0),
    (1, 33, 130, 70, True, False, 0.0),
    (1, 129, 17, 65, False, True, 1.0),
    (3, 40, 50, 31, True, True, 0.5),
    (5, 8, 8, 4097, False, True, 0.0),
    (2, 3000, 8, 64, False, False, 0.0),
    # 16-byte staging along k for both operands with a ragged K and ragged
    # rows; along the row index for both
    (2, 50, 36, 44, False, True, 0.0),
    (1, 52, 60, 40, True, False, 1.0),
]


@pytest.mark.parametrize("batch,M,N,K,at,bt,beta", GEMM_CASES)
def test_gemm_matches_bf16_reference(batch, M, N, K, at, bt, beta):
    say("case: gemm batch %d %dx%dx%d at=%s bt=%s beta=%g" % (batch, M, N, K, at, bt, beta))
    from paper_2011_02600_amd import nn
    rng = np.random.default_rng(M + N + K)
    A = rng.standard_normal((batch, K, M) if at else (batch, M, K)).astype(np.float32)
    B = rng.standard_normal((batch, N, K) if bt else (batch, K, N)).astype(np.float32)
    C0 = rng.standard_normal((batch, M, N)).astype(np.float32)
    dA, dB, dC = (torch.from_numpy(a).cuda() for a in (A, B, C0))
    sA = (K * M, 1, M) if at else (M * K, K, 1)
    sB = (N * K, 1, K) if bt else (K * N, N, 1)
    nn.gemm(dA, dB, dC, M, N, K, sA, sB, (M * N, N, 1), batch=batch, alpha=1.5, beta=beta)
    got = dC.cpu().numpy().astype(np.float64)
    Ab = bf16(A).transpose(0, 2, 1) if at else bf16(A)
    Bb = bf16(B).transpose(0, 2, 1) if bt else bf16(B)
    want = 1.5 * (Ab @ Bb) + beta * C0.astype(np.float64)
    bound = 2e-6 * (1.5 * (np.abs(Ab) @ np.abs(Bb)) + abs(beta) * np.abs(C0)) + 1e-30
    err = np.abs(got - want)
    say("  max |err| / bound = %.3f" % float((err / bound).max()))
    assert np.all(err <= bound)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_network_forward_backward_match_reference():
    say("case: spectral operator n=8 m=4 C=8 L=4 R=5 T=16 S=3")
    from paper_2011_02600_amd import nn
    n, m, C, L, R, Tn, S = 8, 4, 8, 4, 5, 16, 3
    rng = np.random.default_rng(3)
    pos = np.array([7 * 64 + 1 * 8 + 2, 7 * 64 + 4 * 8 + 4, 7 * 64 + 6 * 8 + 1, 3 * 64 + 2 * 8 + 5, 0])
    p = fno.init_params(n, m, C, L, R, Tn, seed=4)
    x = 0.3 * rng.standard_normal((S, n, n, n))
    target = rng.standard_normal((S, R, Tn))
    y_ref, cache = fno.forward(p, x, pos, m, L)
    g_ref = fno.backward(p, y_ref - target, cache)
    net = nn.SpectralOperator(n, m, C, L, pos, Tn)
    net.load_numpy(p)
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    y = net.forward(xd)
    loss, dy = net.loss(y, torch.tensor(target, dtype=torch.float32, device="cuda"))
    net.backward(dy)
    torch.cuda.synchronize()
    ey = rel_l2(y.cpu().numpy().astype(np.float64), y_ref)
    assert loss == pytest.approx(0.5 * np.sum((y_ref - target) ** 2), rel=3e-2)
    errs = {k: rel_l2(net.grads[k].cpu().numpy().astype(np.float64), g_ref[k]) for k in g_ref}
    say("  output rel L2 %.2e; gradients: %s" % (ey, ", ".join("%s %.1e" % kv for kv in errs.items())))
    assert ey <= 3e-2
    for k, e in errs.items():
        assert e <= 3e-2, k


def test_training_steps_reduce_the_loss():
    say("case: 30 Adam steps on a fixed batch")
    from paper_2011_02600_amd import nn
    n, m, C, L, R, Tn, S = 8, 4, 8, 4, 5, 16, 4
    rng = np.random.default_rng(5)
    pos = rng.choice(n ** 3, size=R, replace=False)
    net = nn.SpectralOperator(n, m, C, L, pos, Tn, seed=1)
    x = torch.tensor(0.3 * rng.standard_normal((S, n, n, n)), dtype=torch.float32, device="cuda")
    t = torch.tensor(rng.standard_normal((S, R, Tn)), dtype=torch.float32, device="cuda")
    losses = []
    for it in range(30):
        y = net.forward(x)
        loss, dy = net.loss(y, t)
        net.backward(dy)
        net.adam_step(1e-2)
        losses.append(loss)
    say("  loss %.4f -> %.4f" % (losses[0], losses[-1]))
    assert losses[-1] < 0.5 * losses[0]


def test_surrogate_pipeline_gains_over_the_mean_trace_and_the_solver():
    """End to end at a small size: solver-made training data (batched
    shots), GPU training, held-out evaluation.  The trained network must beat
    the method without it -- the mean training trace as the prediction --
    by a wide margin, and answer faster than the solver."""
    say("case: surrogate pipeline 16^3, 128 training / 16 held-out shots")
    import time
    import workloads as W
    from paper_2011_02600_amd import nn, sbp
    from paper_2011_02600_amd import surrogate as SG
    dev = torch.device("cuda:0")
    case = W.surrogate_case(n=16, T=96, amp=0.01, corr_cells=4, nrec_side=4)
    fields = W.surrogate_fields(case, 144, seed=3)
    y, _ = SG.solve_batch(sbp, torch, case, fields, dev)
    d = torch.tensor(np.stack(fields), dtype=torch.float32, device=dev)
    sur = SG.Surrogate(nn, torch, case, dev, modes=4, width=16)
    hist = sur.train(d[:128], y[:128], epochs=15, lr=3e-3)
    pred = sur.predict(d[128:])
    err = SG.Surrogate.rel_err(pred, y[128:])
    base = SG.Surrogate.rel_err(sur.ymean.expand_as(y[128:]), y[128:])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sur.predict(d[128:])
    torch.cuda.synchronize()
    t_net = time.perf_counter() - t0
    _, t_solver = SG.solve_batch(sbp, torch, case, fields[128:], dev)
    say("  loss %.2f -> %.2f; held-out rel L2 %.3f (mean trace %.3f); network %.4f s, solver %.4f s"
        % (hist[0], hist[-1], float(np.mean(err)), float(np.mean(base)), t_net, t_solver))
    assert np.mean(err) < 0.5 * np.mean(base)
    assert t_net < t_solver
    # the fallback score: the two networks' spread, finite and positive, and
    # a calibrated threshold that accepts a sample only within the budget
    _, score = sur.predict_with_score(d[128:])
    assert np.all(np.isfinite(score)) and np.all(score > 0)
    verr, vsc = sur.calibrate(d[112:128], y[112:128], budget=0.5)
    acc = vsc <= sur.tau
    assert acc.any() and np.quantile(verr[acc], 0.95) <= 0.5
