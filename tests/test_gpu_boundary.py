"""GPU tests of the library boundary: point sources at the block's faces,
inside the boundary closures, overlapping each other and given at a
physical position; graph replay against one-by-one launches; independence
from the contents of the scratch buffers; checkpoint identifiers; the
batched path and the full-size benchmark workload against the CPU oracle.

Bars as in test_gpu_parity: relative L2 per field <= 1e-12 (FP64) and
<= 2e-5 (FP32) after a run; single right-hand sides relative to each
field's largest value (1e-12 / 1e-5).
"""
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import elastic as E

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-5}
RHS_TOL = {"f64": 1e-12, "f32": 1e-5}
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "topo_layer_257x257x193_o6_100steps.npz")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sbp_mod():
    from paper_2011_02600_amd import sbp
    return sbp


def rel_l2(got, want):
    errs = []
    for f in range(want.shape[0]):
        nw = np.linalg.norm(want[f])
        ne = np.linalg.norm(got[f] - want[f])
        errs.append(ne / nw if nw > 0 else ne)
    return max(errs)


def rel_max(got, want):
    errs = []
    for f in range(want.shape[0]):
        nw = np.abs(want[f]).max()
        ne = np.abs(got[f] - want[f]).max()
        errs.append(ne / nw if nw > 0 else ne)
    return max(errs)


def solver(xyz, order, dtype, gamma, medium, variant=0):
    s = sbp_mod().Solver(xyz, order=order, dtype=dtype, gamma=gamma, sat_variant=variant)
    s.set_material(*medium)
    return s


# sources on faces (xi = 0 or 1 along some axis: the delta's window is
# clamped at the boundary), inside the closure rows, and two sources whose
# stencils overlap
SOURCE_SETS = {
    "faces": [((0.0, 0.45, 0.55), (0.3, -0.2, 0.1, 1.0, 0.4, -0.6)),
              ((0.6, 1.0, 0.3), (1.0, 0.5, -0.3, 0.2, 0.0, 0.7))],
    "corner_closure": [((0.02, 0.97, 0.04), (0.5, 0.5, 0.5, 0.3, -0.3, 0.2)),
                       ((1.0, 0.0, 1.0), (0.0, 1.0, 0.0, 0.0, 1.0, 0.0))],
    "overlap": [((0.41, 0.47, 0.52), (0.3, -0.1, 0.2, 1.0, -0.5, 0.25)),
                ((0.44, 0.49, 0.50), (-0.4, 0.6, 0.1, 0.2, 0.9, -0.3)),
                ((0.43, 0.46, 0.55), (0.1, 0.1, -0.8, 0.5, 0.0, 0.4))],
}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("which", sorted(SOURCE_SETS))
@pytest.mark.parametrize("order", [4, 6])
def test_sources_rhs_and_run(which, order, dtype):
    """Right-hand side and a 30-step run with the sources of each set on a
    warped mesh with a random medium, against the oracle."""
    say("case: sources %s order %d %s" % (which, order, dtype))
    shape = (23, 21, 25)
    ns, nr, nq = shape
    xyz = W.warped_mesh(nq, nr, ns, seed=11 + order)
    med = W.random_medium(shape, 4)
    gamma = [0.0, 1.0, 0.0, 0.5, 1.0, 0.0]
    s = solver(xyz, order, dtype, gamma, med)
    blk = E.Block(xyz, order).set_material(*med)
    srcs = []
    for xi, M in SOURCE_SETS[which]:
        s.add_source(xi, M, 0, 6.0, 0.05)
        srcs.append(E.Source(blk, xi, M, E.STF_RICKER, 6.0, 0.05))
    Q = W.random_state(shape, 8, smooth=True) * 1e-2
    s.set_state(Q)
    t = 0.031
    got = s.rhs(t).cpu().numpy().astype(np.float64)
    want = E.rhs(blk, Q, t, gamma, sources=srcs)
    err = rel_max(got, want)
    say("  rhs rel max = %.3e" % err)
    assert err <= RHS_TOL[dtype]
    dt = W.cfl_dt(xyz, med[1], 0.4)
    s.set_state(Q)
    s.step(30, dt)
    got = s.get_state().cpu().numpy().astype(np.float64)
    want, _, _ = E.run(blk, Q, 30, dt, gamma, sources=srcs)
    err = rel_l2(got, want)
    say("  30 steps rel L2 = %.3e" % err)
    assert err <= TOL[dtype]
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_source_at_physical_position(dtype):
    """sbp_add_source_at: the library's Newton inversion of the map agrees
    with the oracle's root finder, and the run with the located source
    matches the oracle's run with its own located source."""
    say("case: source at a physical position %s" % dtype)
    shape = (21, 23, 19)
    ns, nr, nq = shape
    xyz = W.warped_mesh(nq, nr, ns, seed=21)
    med = W.random_medium(shape, 6)
    gamma = [0.0, 0.0, 0.0, 0.0, 0.0, 1.0]
    s = solver(xyz, 6, dtype, gamma, med)
    blk = E.Block(xyz, 6).set_material(*med)
    M = (0.2, -0.4, 0.3, 1.0, 0.1, -0.2)
    # an interior point, a point in the closure rows, a point on the top face
    pts = [xyz[:, 9, 11, 8] * 0.6 + xyz[:, 10, 12, 9] * 0.4,
           xyz[:, 1, 2, nq - 2] * 0.5 + xyz[:, 2, 3, nq - 1] * 0.5,
           xyz[:, ns - 1, 7, 5] * 0.3 + xyz[:, ns - 1, 8, 6] * 0.7]
    srcs = []
    for x in pts:
        xi_lib = s.locate(x)
        xi_ora = E.locate(blk, x)
        say("  x = %s  xi lib %s  oracle %s" % (np.round(x, 4), np.round(xi_lib, 6), np.round(xi_ora, 6)))
        assert np.allclose(xi_lib, xi_ora, atol=1e-10, rtol=0)
        s.add_source_at(x, M, 0, 5.0, 0.1)
        srcs.append(E.Source(blk, xi_ora, M, E.STF_RICKER, 5.0, 0.1))
    with pytest.raises(sbp_mod().SBPError):
        s.add_source_at(xyz[:, 5, 5, 0] - np.array([0.05, 0.0, 0.0]), M, 0, 5.0, 0.1)
    dt = W.cfl_dt(xyz, med[1], 0.4)
    Q0 = np.zeros((9,) + shape)
    s.step(40, dt)
    got = s.get_state().cpu().numpy().astype(np.float64)
    want, _, _ = E.run(blk, Q0, 40, dt, gamma, sources=srcs)
    err = rel_l2(got, want)
    say("  40 steps rel L2 = %.3e" % err)
    assert err <= TOL[dtype]
    s.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_graph_replay_equals_eager_bitwise(dtype):
    """sbp_step replaying captured step graphs gives bitwise the state and
    receiver traces of one-by-one launches, also across re-captures (dt
    changed, a source added, receivers re-registered, launch shape changed)
    and over more than one source-time table chunk (600 steps)."""
    say("case: graph replay vs eager %s" % dtype)
    wl = W.topo_layer(nq=41, nr=37, ns=33, nrec_side=3)
    runs = []
    for graphs in (True, False):
        s = solver(wl["xyz"], 6, dtype, wl["gamma"], (wl["rho"], wl["cp"], wl["cs"]))
        s.set_graphs(graphs)
        s.add_source(wl["src_xi"], wl["src_M"], 0, 8.0, 0.1)
        tr = s.record(wl["receivers"], 700)
        s.step(13, wl["dt"])
        s.step(7, wl["dt"] * 0.9)
        s.add_source((0.3, 0.6, 0.5), (0, 0, 1.0, 0, 0, 0), 1, 0.05, 0.0)
        s.step(600, wl["dt"] * 0.9)
        s.set_launch(8, 11)
        s.step(5, wl["dt"] * 0.9)
        tr1 = tr.clone()
        tr2 = s.record(wl["receivers"][:4], 10)
        s.step(9, wl["dt"] * 0.9)
        torch.cuda.synchronize()
        runs.append((s.get_state().cpu().numpy(), tr1.cpu().numpy(), tr2.cpu().numpy(), s.time()))
        s.close()
    (qa, ta, ua, tma), (qb, tb, ub, tmb) = runs
    say("  max |graph - eager| state %.3e traces %.3e" % (np.abs(qa - qb).max(), np.abs(ta - tb).max()))
    assert np.isfinite(qa).all() and np.abs(qa).max() > 0
    assert np.array_equal(qa, qb)
    assert np.array_equal(ta, tb) and np.array_equal(ua, ub)
    assert tma == tmb


def test_batched_graph_replay_equals_eager_bitwise():
    """sbp_step_batch replaying captured step graphs (FP32 work list) gives
    bitwise the states and receiver traces of the same batch launched step
    by step (sbp_set_graphs(h, 0) on the first handle), over two calls and
    more than one source-time table chunk."""
    say("case: batched graph replay vs eager f32")
    sbp = sbp_mod()
    cases = [((19, 17, 21), 4), ((23, 21, 18), 6), ((17, 25, 19), 6)]
    runs = []
    for graphs in (True, False):
        ss, trs, dts = [], [], []
        for i, (shape, order) in enumerate(cases):
            ns, nr, nq = shape
            xyz = W.warped_mesh(nq, nr, ns, seed=60 + i)
            med = W.random_medium(shape, 70 + i)
            s = solver(xyz, order, "f32", [0.0, 0.0, 0.0, 0.0, 0.0, 1.0], med)
            s.add_source((0.4, 0.5, 0.45), (0.0, 0.0, 0.0, 1.0, 0.3, 0.0), 0, 6.0, 0.1)
            trs.append(s.record(np.array([[2, 3, ns - 1], [nq // 2, nr // 2, ns // 2]]), 600))
            s.set_state(W.random_state(shape, 80 + i, smooth=True) * 1e-3)
            dts.append(W.cfl_dt(xyz, med[1], 0.4))
            ss.append(s)
        ss[0].set_graphs(graphs)
        sbp.sbp_step_batch([s.h for s in ss], 17, dts)
        sbp.sbp_step_batch([s.h for s in ss], 560, dts)
        torch.cuda.synchronize()
        runs.append([(s.get_state().cpu().numpy(), t.cpu().numpy(), s.time()) for s, t in zip(ss, trs)])
        for s in ss:
            s.close()
    for (qa, ta, tma), (qb, tb, tmb) in zip(*runs):
        assert np.isfinite(qa).all() and np.abs(qa).max() > 0
        assert np.array_equal(qa, qb) and np.array_equal(ta, tb) and tma == tmb


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_scratch_contents_do_not_matter(dtype):
    """NaN in the next stage's output buffer and in the Runge-Kutta register
    before every step (and before a right-hand side) leaves the results
    bitwise unchanged and finite: every stage writes every node it later
    reads, the first stage does not read the register."""
    say("case: NaN-poisoned scratch %s" % dtype)
    for shape, order in (((33, 41, 65), 6), ((29, 37, 70), 4), ((14, 14, 14), 7 if dtype == "f32" else 5)):
        ns, nr, nq = shape
        xyz = W.warped_mesh(nq, nr, ns, seed=2)
        med = W.random_medium(shape, 9)
        gamma = [1.0, 0.0, -1.0, 0.4, 0.0, 1.0]
        Q = W.random_state(shape, 3, smooth=True)
        out = []
        for poison in (False, True):
            s = solver(xyz, order, dtype, gamma, med)
            s.add_source((0.4, 0.5, 0.6), (1, 0, 0, 0.5, 0, 0), 0, 6.0, 0.05)
            s.set_state(Q)
            if poison:
                s.fill_scratch(float("nan"))
            r = s.rhs(0.02).cpu().numpy()
            dt = W.cfl_dt(xyz, med[1], 0.4)
            for n in range(6):
                if poison:
                    s.fill_scratch(float("nan"))
                s.step(1, dt)
            out.append((r, s.get_state().cpu().numpy()))
            s.close()
        (r0, q0), (r1, q1) = out
        say("  shape %s order %d: finite %s" % (shape, order, np.isfinite(q1).all()))
        assert np.isfinite(r1).all() and np.isfinite(q1).all()
        assert np.array_equal(r0, r1) and np.array_equal(q0, q1)


def test_checkpoint_ids_and_two_forward_passes():
    """sbp_checkpoint_id names the checkpoints of the last forward run and
    drops to 0 once the handle is stepped or its receivers change; the
    autograd function gives each of two forward passes on one solver its own
    gradient (oracle gradient of each), whatever the order of backward."""
    from oracle import adjoint as A
    from paper_2011_02600_amd.autograd import Seismograms
    sbp = sbp_mod()
    say("case: checkpoint ids, two forward passes")
    shape = (13, 12, 14)
    ns, nr, nq = shape
    xyz = W.warped_mesh(nq, nr, ns, seed=4)
    rho, cp, cs = W.random_medium(shape, 2)
    mu = rho * cs ** 2
    lam = rho * cp ** 2 - 2 * mu
    gamma = [0.0, 0.0, 0.0, 0.0, 0.0, 1.0]
    s = sbp.Solver(xyz, order=4, dtype="f64", gamma=gamma)
    s.set_material(rho, cp, cs)
    s.add_source((0.5, 0.45, 0.4), (0, 0, 0, 1.0, 0, 0), 0, 4.0, 0.15)
    rec = np.array([[3, 4, ns - 1], [9, 7, ns - 1], [6, 10, ns - 1]], dtype=np.int32)
    dt = W.cfl_dt(xyz, cp, 0.4)
    nsteps = 6
    Q0 = torch.zeros((9,) + shape, dtype=torch.float64, device="cuda")
    s.record(rec, nsteps)
    s.step_checkpointed(nsteps, dt, 4)
    i1 = s.checkpoint_id()
    assert i1 > 0
    s.record(rec, nsteps)
    assert s.checkpoint_id() == 0
    s.set_state(Q0)
    s.record(rec, nsteps + 1)
    s.step_checkpointed(nsteps, dt, 4)
    i2 = s.checkpoint_id()
    assert i2 > i1
    s.step(1, dt)
    assert s.checkpoint_id() == 0
    # two forward passes (different media), one loss
    mats = []
    for f in (1.0, 1.03):
        mats.append([torch.tensor(a * f, device="cuda", requires_grad=True) for a in (rho, lam, mu)])
    data = [torch.tensor(np.random.default_rng(k).standard_normal((nsteps, 3, 3)) * 1e-3, device="cuda")
            for k in range(2)]
    for order_ in (0, 1):
        trs = [Seismograms.apply(*mats[k], s, Q0, rec, nsteps, dt, 4) for k in range(2)]
        losses = [0.5 * ((trs[k] - data[k]) ** 2).sum() for k in range(2)]
        for m in mats:
            for a in m:
                a.grad = None
        first, second = (0, 1) if order_ == 0 else (1, 0)
        losses[first].backward()
        losses[second].backward()
        for k in range(2):
            r, la, m = (a.detach().cpu().numpy() for a in mats[k])
            cpk, csk = np.sqrt((la + 2 * m) / r), np.sqrt(m / r)
            blk = E.Block(xyz, 4).set_material(r, cpk, csk)
            src = E.Source(blk, (0.5, 0.45, 0.4), (0, 0, 0, 1.0, 0, 0), E.STF_RICKER, 4.0, 0.15)
            _, g, _, _ = A.gradient(blk, np.zeros((9,) + shape), nsteps, dt, gamma, sources=[src], receivers=rec,
                                    target=data[k].cpu().numpy())
            for q in range(3):
                got = mats[k][q].grad.cpu().numpy()
                want = g[A.PARAMS[q]]
                err = np.linalg.norm(got - want) / np.linalg.norm(want)
                say("  backward order %d pass %d param %d rel L2 %.2e" % (order_, k, q, err))
                assert err < 1e-9
    s.close()


BATCH_ORACLE_CASES = {
    # (ns, nr, nq), order
    "worklist": [((19, 17, 21), 4), ((23, 21, 18), 6), ((17, 25, 19), 3), ((21, 19, 24), 5)],
    # an order-8 shot (not built into the work-list kernel) sends the whole
    # batch to one stage and one edge launch per order
    "grouped": [((19, 17, 21), 4), ((17, 18, 19), 8), ((17, 25, 19), 3)],
    # likewise order-7 and order-8 shots in double precision
    "grouped78": [((19, 17, 21), 4), ((17, 18, 19), 7), ((17, 25, 19), 3), ((18, 17, 17), 8)],
}


@pytest.mark.parametrize("dtype,kind", [("f64", "worklist"), ("f32", "worklist"), ("f32", "grouped"),
                                        ("f64", "grouped78")])
def test_batch_against_oracle(dtype, kind):
    """sbp_step_batch on shots of uneven size and mixed interior orders, each
    with its own random medium, source and receivers: 40 steps, every shot's
    state and traces against the oracle (work-list launches for orders 3-6,
    grouped launches when an order-8 shot, or in double precision an order-7
    or order-8 shot, is present)."""
    sbp = sbp_mod()
    cases = BATCH_ORACLE_CASES[kind]
    say("case: batch vs oracle %s %s" % (dtype, kind))
    ss, wants, trs = [], [], []
    for i, (shape, order) in enumerate(cases):
        ns, nr, nq = shape
        xyz = W.warped_mesh(nq, nr, ns, seed=30 + i)
        med = W.random_medium(shape, 40 + i)
        gamma = [0.0, 0.0, 0.0, 0.0, 0.0, 1.0]
        s = solver(xyz, order, dtype, gamma, med)
        xi = (0.35 + 0.05 * i, 0.5, 0.45)
        M = (0.0, 0.0, 0.0, 1.0, 0.2 * i, 0.0)
        s.add_source(xi, M, 0, 5.0 + i, 0.1)
        rec = np.array([[2 + i, 3, ns - 1], [nq - 3, nr - 4, ns - 1], [nq // 2, nr // 2, ns // 2]], dtype=np.int32)
        trs.append(s.record(rec, 40))
        Q0 = W.random_state(shape, 50 + i, smooth=True) * 1e-3
        s.set_state(Q0)
        dt = W.cfl_dt(xyz, med[1], 0.25 if order == 8 else 0.4)
        blk = E.Block(xyz, order).set_material(*med)
        src = E.Source(blk, xi, M, E.STF_RICKER, 5.0 + i, 0.1)
        wants.append((E.run(blk, Q0, 40, dt, gamma, sources=[src], receivers=rec), dt))
        ss.append(s)
    sbp.sbp_step_batch([s.h for s in ss], 40, [w[1] for w in wants])
    for i, s in enumerate(ss):
        got = s.get_state().cpu().numpy().astype(np.float64)
        (want, _, wtr), _ = wants[i]
        err = rel_l2(got, want)
        tr = trs[i].cpu().numpy().astype(np.float64)
        terr = np.linalg.norm(tr - wtr) / np.linalg.norm(wtr)
        say("  shot %d order %d: state %.3e traces %.3e" % (i, cases[i][1], err, terr))
        assert err <= TOL[dtype] and terr <= TOL[dtype]
        s.close()


def test_full_size_topo_layer_100_steps_against_stored_oracle():
    """The benchmark workload at full size (257 x 257 x 193, order 6, FP32,
    the benchmark's launch shape): 100 steps against values the oracle
    computed (tests/golden/make_topo_layer_golden.py): the 64 receiver traces
    and all nine fields at about 12 000 sample nodes (source support,
    receivers, corners, edges, the closure layers of every face, faces,
    interior) within relative L2 2e-5, and the whole-field L2 norms."""
    if not os.path.exists(GOLDEN):
        pytest.skip("stored oracle values not generated")
    g = np.load(GOLDEN)
    say("case: topo_layer 257x257x193 order 6 FP32, 100 steps vs stored oracle values")
    wl = W.topo_layer()
    s = solver(wl["xyz"], 6, "f32", wl["gamma"], (wl["rho"], wl["cp"], wl["cs"]))
    s.add_source(wl["src_xi"], wl["src_M"], 0, wl["src_f0"], wl["src_t0"])
    tr = s.record(wl["receivers"], 100)
    s.step(100, wl["dt"])
    Q = s.get_state()
    nodes = torch.tensor(g["nodes"].astype(np.int64), device=Q.device)
    vals = Q[:, nodes[:, 2], nodes[:, 1], nodes[:, 0]].cpu().numpy().astype(np.float64).T
    l2 = torch.linalg.vector_norm(Q.double().reshape(9, -1), dim=1).cpu().numpy()
    trs = tr.cpu().numpy().astype(np.float64)
    s.close()
    want = g["values"]
    ferr = [np.linalg.norm(vals[:, f] - want[:, f]) / np.linalg.norm(want[:, f]) for f in range(9)]
    terr = np.linalg.norm(trs - g["traces"]) / np.linalg.norm(g["traces"])
    cerr = [np.linalg.norm(trs[:, :, c] - g["traces"][:, :, c]) / np.linalg.norm(g["traces"][:, :, c])
            for c in range(3)]
    nerr = np.abs(l2 - g["field_l2"]) / g["field_l2"]
    say("  sample nodes rel L2 per field: %s" % " ".join("%.2e" % e for e in ferr))
    say("  traces rel L2 %.3e (per component %s); field norms max rel diff %.3e"
        % (terr, " ".join("%.2e" % e for e in cerr), nerr.max()))
    assert max(ferr) <= TOL["f32"]
    assert terr <= TOL["f32"] and max(cerr) <= TOL["f32"]
    assert nerr.max() <= TOL["f32"]
