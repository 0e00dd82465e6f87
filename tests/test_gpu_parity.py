"""GPU parity: the HIP library (called through its C ABI) against the CPU
oracle on the same seeded inputs.

Bars: relative L2 error per field <= 1e-12 in FP64 and <= 2e-5 in FP32 after
100 steps; single right-hand-side evaluations are compared field by field
relative to the field's largest value.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import elastic as E

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-5}


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


def make_solver(xyz, order, dtype, gamma, variant=0, medium=None):
    sbp = sbp_mod()
    s = sbp.Solver(xyz, order=order, dtype=dtype, gamma=gamma, sat_variant=variant)
    if medium is not None:
        s.set_material(*medium)
    return s


def test_cube_pulse_fp64_100_steps():
    """Cartesian unit cube 21^3, order 4, FP64, free surface on top and
    absorbing elsewhere, Gaussian pulse, CFL 0.5, 100 steps."""
    say("case: cube_pulse 21^3 order 4 f64 100 steps")
    wl = W.cube_pulse(n=21)
    s = make_solver(wl["xyz"], 4, "f64", wl["gamma"], medium=(wl["rho"], wl["cp"], wl["cs"]))
    s.set_state(wl["Q0"])
    e0 = s.energy()
    s.step(100, wl["dt"])
    got = s.get_state().cpu().numpy()
    e1 = s.energy()
    blk = E.Block(wl["xyz"], 4).set_material(wl["rho"], wl["cp"], wl["cs"])
    want, t, _ = E.run(blk, wl["Q0"], 100, wl["dt"], wl["gamma"])
    err = rel_l2(got, want)
    say("  rel L2 = %.3e" % err)
    assert err <= TOL["f64"]
    assert abs(e0 - E.energy(blk, wl["Q0"])) <= 1e-12 * e0
    assert abs(e1 - E.energy(blk, want)) <= 1e-12 * e0
    assert e1 < e0
    assert abs(s.time()[0] - 100 * wl["dt"]) < 1e-12
    s.close()


RHS_CASES = [
    # order, (ns, nr, nq), dtype, variant
    (2, (4, 4, 4), "f64", 0),
    (4, (8, 8, 8), "f64", 1),
    (6, (12, 12, 12), "f64", 0),
    (2, (11, 9, 70), "f64", 1),
    (4, (19, 23, 70), "f64", 0),
    (4, (19, 23, 70), "f32", 1),
    (6, (17, 13, 131), "f64", 0),
    (6, (17, 13, 131), "f32", 0),
    (6, (25, 21, 17), "f64", 1),
    (6, (13, 30, 65), "f32", 1),      # last q column by the edge kernel
    # sizes whose last q column and / or last r row go to the edge kernel
    # (n - 1 a multiple of the 128-byte line along q, of the tile height along r)
    (4, (13, 17, 65), "f64", 0),
    (6, (15, 25, 97), "f64", 1),
    (2, (9, 17, 40), "f32", 0),
    (6, (14, 33, 129), "f32", 0),
    # odd interior orders 3 and 5: minimum size, ragged multi-tile shapes,
    # edge-kernel shapes
    (3, (6, 6, 6), "f64", 0),
    (5, (10, 10, 10), "f64", 1),
    (3, (15, 19, 70), "f64", 1),
    (3, (13, 17, 65), "f32", 0),
    (5, (17, 13, 131), "f64", 0),
    (5, (17, 13, 131), "f32", 1),
    (5, (15, 25, 97), "f64", 0),
    (3, (14, 33, 129), "f64", 1),
    # interior order 7 (double precision: the s-flux ring with its newest
    # plane in registers)
    (7, (14, 14, 14), "f32", 0),
    (7, (17, 19, 70), "f32", 1),
    (7, (15, 25, 97), "f32", 0),
    (7, (14, 14, 14), "f64", 1),
    (7, (17, 19, 70), "f64", 0),
    (7, (15, 25, 97), "f64", 1),
    (7, (18, 21, 65), "f64", 0),
    # interior order 8: minimum size, ragged multi-tile shapes, edge-kernel
    # shape (double precision: three lead planes of the s-flux ring in
    # registers, no prefetch)
    (8, (16, 16, 16), "f32", 0),
    (8, (17, 19, 70), "f32", 1),
    (8, (18, 25, 97), "f32", 0),
    (8, (17, 17, 65), "f32", 1),
    (8, (16, 16, 16), "f64", 1),
    (8, (17, 19, 70), "f64", 0),
    (8, (18, 25, 97), "f64", 1),
    (8, (17, 17, 65), "f64", 0),
]


@pytest.mark.parametrize("order,shape,dtype,variant", RHS_CASES)
def test_rhs_parity(order, shape, dtype, variant):
    """One right-hand-side evaluation (volume terms, penalties on all six
    faces with mixed gamma, one source) on a warped mesh with a random medium.
    Shapes span several tiles with ragged tails and include the minimum size
    (2 m points per axis)."""
    say("case: rhs order %d shape %s %s variant %d" % (order, shape, dtype, variant))
    ns, nr, nq = shape
    xyz = W.warped_mesh(nq, nr, ns, seed=order + nq)
    med = W.random_medium(shape, 3)
    gamma = [1.0, 0.0, -1.0, 0.4, 0.0, 1.0]
    Q = W.random_state(shape, 5, smooth=(dtype == "f32"))
    s = make_solver(xyz, order, dtype, gamma, variant, med)
    Msrc = (0.3, -0.1, 0.2, 1.0, -0.5, 0.25)
    xi = (0.37, 0.52, 0.61)
    s.add_source(xi, Msrc, 0, 2.0, 0.1)
    s.set_state(Q)
    t = 0.13
    got = s.rhs(t).cpu().numpy().astype(np.float64)
    blk = E.Block(xyz, order).set_material(*med)
    src = E.Source(blk, xi, Msrc, E.STF_RICKER, 2.0, 0.1)
    want = E.rhs(blk, Q, t, gamma, variant, [src])
    err = rel_max(got, want)
    say("  rel max = %.3e" % err)
    assert err <= (1e-12 if dtype == "f64" else 1e-5)
    # the state is untouched by an RHS evaluation
    back = s.get_state().cpu().numpy()
    assert np.array_equal(back, Q.astype(back.dtype))
    s.close()


@pytest.mark.parametrize("dtype,order,size", [(d, o, sz) for d in ("f64", "f32")
                                              for o, sz in ((6, (49, 45, 37)), (6, (65, 41, 33)), (3, (65, 41, 33)),
                                                            (5, (49, 45, 37)), (7, (65, 41, 33)), (8, (65, 41, 33)))])
def test_topo_layer_small_100_steps(dtype, order, size):
    """The curvilinear layered workload (topography, transfinite mesh, soft
    layer over a half-space, Ricker moment source, surface receivers) at a
    reduced size: 100 steps, state and receiver traces against the oracle.
    The (65, 41, 33) size has its last q column and r row on the edge kernel,
    like the full-size workload."""
    nq, nr, ns = size
    say("case: topo_layer %dx%dx%d order %d %s 100 steps" % (nq, nr, ns, order, dtype))
    # order 8's closure has the largest spectral radius of the orders: CFL 0.25
    wl = W.topo_layer(nq=nq, nr=nr, ns=ns, nrec_side=4, cfl=0.25 if order == 8 else 0.5)
    s = make_solver(wl["xyz"], order, dtype, wl["gamma"], medium=(wl["rho"], wl["cp"], wl["cs"]))
    s.add_source(wl["src_xi"], wl["src_M"], 0, wl["src_f0"], wl["src_t0"])
    traces = s.record(wl["receivers"], 100)
    s.step(100, wl["dt"])
    got = s.get_state().cpu().numpy().astype(np.float64)
    tr = traces.cpu().numpy().astype(np.float64)
    blk = E.Block(wl["xyz"], order).set_material(wl["rho"], wl["cp"], wl["cs"])
    src = E.Source(blk, wl["src_xi"], wl["src_M"], E.STF_RICKER, wl["src_f0"], wl["src_t0"])
    want, _, wtr = E.run(blk, wl["Q0"], 100, wl["dt"], wl["gamma"], sources=[src], receivers=wl["receivers"])
    err = rel_l2(got, want)
    terr = np.linalg.norm(tr - wtr) / np.linalg.norm(wtr)
    say("  state rel L2 = %.3e, traces rel L2 = %.3e" % (err, terr))
    assert err <= TOL[dtype]
    assert terr <= TOL[dtype]
    s.close()


def test_full_size_sampled_rhs():
    """The 257 x 257 x 193 order-6 FP32 workload in the benchmark's launch
    configuration: the GPU right-hand side against the oracle evaluated node by
    node at sampled nodes (interior, closure planes, faces, edges, corners and
    the source support)."""
    say("case: full-size 257x257x193 order 6 f32 sampled rhs")
    wl = W.topo_layer()
    ns, nr, nq = wl["xyz"].shape[1:]
    Q = W.random_state((ns, nr, nq), 21, smooth=True)
    s = make_solver(wl["xyz"], 6, "f32", wl["gamma"], medium=(wl["rho"], wl["cp"], wl["cs"]))
    s.add_source(wl["src_xi"], wl["src_M"], 0, wl["src_f0"], wl["src_t0"])
    s.set_state(Q)
    t = 0.5
    got = s.rhs(t).cpu().numpy()
    s.close()
    blk = E.Block(wl["xyz"], 6).set_material(wl["rho"], wl["cp"], wl["cs"])
    src = E.Source(blk, wl["src_xi"], wl["src_M"], E.STF_RICKER, wl["src_f0"], wl["src_t0"])
    rng = np.random.default_rng(0)
    nodes = [tuple(int(rng.integers(0, n)) for n in (nq, nr, ns)) for _ in range(150)]
    for i in (0, 1, 5, 6, 7, nq // 2, nq - 7, nq - 6, nq - 1):
        for k in (0, 3, 5, 6, ns // 2, ns - 6, ns - 1):
            nodes.append((i, int(rng.integers(0, nr)), k))
    nodes += [(0, 0, 0), (nq - 1, nr - 1, ns - 1), (0, nr - 1, ns - 1), (nq - 1, 0, 0)]
    ks, js, is_ = src.sl
    nodes += [(is_.start + 3, js.start + 4, ks.start + 2), (is_.start, js.start, ks.start)]
    want = E.rhs_at(blk, Q, nodes, t, wl["gamma"], sources=[src])
    g = np.array([got[:, k, j, i] for i, j, k in nodes], dtype=np.float64)
    scale = np.abs(want).max(axis=0)
    err = (np.abs(g - want).max(axis=0) / scale).max()
    say("  sampled rel max = %.3e over %d nodes" % (err, len(nodes)))
    assert err <= 1e-5


def test_full_size_energy_decreases():
    """Property at full size: without sources the discrete energy never
    grows (Theorem for general boundary conditions, |gamma| <= 1), and the
    GPU energy equals the oracle's energy of the same state."""
    say("case: full-size 257x257x193 order 6 f32 energy over 10 steps")
    wl = W.topo_layer()
    shape = wl["xyz"].shape[1:]
    Q = W.random_state(shape, 8, smooth=True)
    s = make_solver(wl["xyz"], 6, "f32", wl["gamma"], medium=(wl["rho"], wl["cp"], wl["cs"]))
    s.set_state(Q)
    es = [s.energy()]
    for _ in range(10):
        s.step(1, wl["dt"])
        es.append(s.energy())
    last = s.get_state().cpu().numpy().astype(np.float64)
    s.close()
    say("  energies %s" % ["%.6e" % e for e in es])
    for a, b in zip(es[:-1], es[1:]):
        assert b <= a * (1 + 1e-6)
    blk = E.Block(wl["xyz"], 6).set_material(wl["rho"], wl["cp"], wl["cs"])
    eo = E.energy(blk, last)
    assert abs(eo - es[-1]) <= 1e-5 * eo


@pytest.mark.parametrize("size", [(70, 37, 29), (65, 33, 29)])
def test_launch_shapes_give_identical_results(size):
    """For a given tile height every node is computed by the same
    instructions whatever the s-chunking: results are bitwise identical across
    z-chunk sizes.  Different tile heights are different kernel instantiations
    (the compiler may contract or order operations differently), so across
    them the results agree to rounding.  The second size uses the edge
    kernel for its last q column and r row."""
    nq, nr, ns = size
    say("case: launch-shape invariance order 4 f32 %dx%dx%d" % size)
    xyz = W.warped_mesh(nq, nr, ns, seed=3)
    med = W.random_medium((ns, nr, nq), 4)
    Q = W.random_state((ns, nr, nq), 6, smooth=True)
    outs = {}
    for ty, zc in ((8, 0), (8, 5), (8, 1), (16, 29), (16, 3)):
        s = make_solver(xyz, 4, "f32", [0, 1, 0, 0, -1, 1], medium=med)
        s.set_launch(ty, zc)
        s.set_state(Q)
        s.step(3, 1e-3)
        outs[(ty, zc)] = s.get_state().cpu().numpy()
        s.close()
    for key, o in outs.items():
        ref = outs[(key[0], min(k[1] for k in outs if k[0] == key[0]))]
        assert np.array_equal(o, ref), key
    err = rel_max(outs[(16, 3)].astype(np.float64), outs[(8, 0)].astype(np.float64))
    say("  tile height 16 vs 8: rel max %.3e" % err)
    assert err < 1e-5


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_plain_pointer_addressing(dtype):
    """The plain-pointer stage kernel (the path grids with arrays of 4 GiB and
    more take) on a small grid, forced by sbp_set_addressing: 10 steps with
    sources agree with the buffer-addressed kernel to rounding, single and
    batched, and the state after them with the oracle."""
    nq, nr, ns = 65, 41, 33
    say("case: plain-pointer addressing order 6 %s %dx%dx%d" % (dtype, nq, nr, ns))
    sbp = sbp_mod()
    xyz = W.warped_mesh(nq, nr, ns, seed=5)
    med = W.random_medium((ns, nr, nq), 8)
    Q = W.random_state((ns, nr, nq), 9, smooth=True)
    gamma = [1, 0, 0.5, 0, -1, 1]
    src = ((0.4, 0.55, 0.5), (0.2, 0.1, -0.3, 1.0, 0.0, 0.4), 0, 8.0, 0.05)
    out = {}
    for mode in ("buffer", "plain", "plain batch"):
        s = make_solver(xyz, 6, dtype, gamma, medium=med)
        s.add_source(*src)
        s.set_state(Q)
        if mode != "buffer":
            s.set_addressing(1)
        if mode == "plain batch":
            sbp.sbp_step_batch([s.h], 10, [1e-3])
        else:
            s.step(10, 1e-3)
        out[mode] = s.get_state().cpu().numpy().astype(np.float64)
        s.close()
    tol = 1e-5 if dtype == "f32" else 1e-12
    e1 = rel_max(out["plain"], out["buffer"])
    e2 = rel_max(out["plain batch"], out["buffer"])
    blk = E.Block(xyz, 6).set_material(*med)
    osrc = E.Source(blk, src[0], src[1], E.STF_RICKER, src[3], src[4])
    want, _, _ = E.run(blk, Q, 10, 1e-3, gamma, sources=[osrc])
    e3 = rel_l2(out["plain"], want)
    say("  plain vs buffer %.2e, plain batched vs buffer %.2e, plain vs oracle %.2e" % (e1, e2, e3))
    assert e1 <= tol and e2 <= tol
    assert e3 <= TOL[dtype]
    with pytest.raises(sbp.SBPError):
        sbp.sbp_set_addressing(None, 1)


def test_resume_is_bitwise():
    say("case: resume 20 + 20 == 40 steps, order 6 f32")
    wl = W.topo_layer(nq=33, nr=29, ns=25)
    med = (wl["rho"], wl["cp"], wl["cs"])
    a = make_solver(wl["xyz"], 6, "f32", wl["gamma"], medium=med)
    a.add_source(wl["src_xi"], wl["src_M"], 0, wl["src_f0"], wl["src_t0"])
    a.step(40, wl["dt"])
    ref = a.get_state().cpu().numpy()
    a.close()
    b = make_solver(wl["xyz"], 6, "f32", wl["gamma"], medium=med)
    b.add_source(wl["src_xi"], wl["src_M"], 0, wl["src_f0"], wl["src_t0"])
    b.step(20, wl["dt"])
    mid = b.get_state()
    t_mid = b.time()[0]
    b.close()
    c = make_solver(wl["xyz"], 6, "f32", wl["gamma"], medium=med)
    c.add_source(wl["src_xi"], wl["src_M"], 0, wl["src_f0"], wl["src_t0"])
    c.set_state(mid, t_mid)
    c.step(20, wl["dt"])
    out = c.get_state().cpu().numpy()
    c.close()
    assert np.array_equal(out, ref)


def test_error_paths_on_device():
    say("case: error paths")
    sbp = sbp_mod()
    xyz = W.unit_cube(13, 13, 13)
    s = sbp.Solver(xyz, order=4, dtype="f32", gamma=[0] * 6)
    with pytest.raises(sbp.SBPError) as e:
        s.step(1, 1e-3)
    assert e.value.code == sbp.SBP_ESTATE
    s.set_material(2.7, 6.0, 3.464)
    with pytest.raises(sbp.SBPError) as e:
        s.add_source((0.5, 1.2, 0.5), (0, 0, 0, 1, 0, 0))
    assert e.value.code == sbp.SBP_EINVAL
    with pytest.raises(sbp.SBPError):
        s.set_material(2.7, 3.0, 3.464)  # lambda + 2/3 mu < 0
    s.record([(1, 2, 3)], 2)
    s.step(2, 1e-3)
    with pytest.raises(sbp.SBPError):
        s.step(1, 1e-3)  # receiver buffer full
    with pytest.raises(sbp.SBPError):
        s.record([(13, 0, 0)], 2)
    s.close()
    bad = xyz.copy()
    bad[0] = bad[0][:, :, ::-1]  # mirrored map: negative Jacobian
    with pytest.raises(sbp.SBPError) as e:
        sbp.Solver(bad, order=4, dtype="f32", gamma=[0] * 6)
    assert e.value.code == sbp.SBP_EINVAL


def test_degenerate_calls():
    """Zero steps (single or batched) change nothing: the state bitwise, the
    time and the step count; an empty handle list is SBP_EINVAL; an empty
    receiver list switches recording off and stepping goes on."""
    say("case: degenerate calls, order 4 f32 17x15x13")
    sbp = sbp_mod()
    nq, nr, ns = 17, 15, 13
    s = make_solver(W.warped_mesh(nq, nr, ns, seed=4), 4, "f32", [1, 0, 0, 0, 0, 1],
                    medium=W.random_medium((ns, nr, nq), 2))
    s.set_state(W.random_state((ns, nr, nq), 3, smooth=True))
    before = s.get_state().cpu().numpy()
    s.step(0, 1e-3)
    sbp.sbp_step_batch([s.h], 0, [1e-3])
    assert np.array_equal(s.get_state().cpu().numpy(), before)
    assert s.time() == (0.0, 0)
    with pytest.raises(sbp.SBPError) as e:
        sbp.sbp_step_batch([], 1, [])
    assert e.value.code == sbp.SBP_EINVAL
    s.record([(1, 2, 3)], 1)
    s.step(1, 1e-3)
    s.record(np.zeros((0, 3), dtype=np.int32), 1)
    s.step(3, 1e-3)
    assert s.time()[1] == 4
    assert np.all(np.isfinite(s.get_state().cpu().numpy()))
    s.close()


def test_profiling_changes_nothing():
    """sbp_set_profiling only times launches: the state after stepping with
    it on is bitwise the state without it, and the reported node count is
    the tiled part of the grid (all but the last q column, and the last r
    row when nr - 1 is a multiple of the tile height)."""
    say("case: profiling on/off, order 6 f32 65x41x29")
    nq, nr, ns = 65, 41, 29
    xyz = W.warped_mesh(nq, nr, ns, seed=9)
    med = W.random_medium((ns, nr, nq), 2)
    Q = W.random_state((ns, nr, nq), 4, smooth=True)
    outs = []
    for prof in (False, True):
        s = make_solver(xyz, 6, "f32", [1, 0, 0, 0, 0, 1], medium=med)
        s.set_state(Q)
        s.set_profiling(prof)
        s.step(3, 1e-3)
        outs.append(s.get_state().cpu().numpy())
        stage_ms, edge_ms, n, nodes = s.profile()
        if prof:
            assert n == 15 and stage_ms > 0 and edge_ms > 0
            assert nodes == (nq - 1) * (nr - 1) * ns
        else:
            assert n == 0
        s.close()
    assert np.array_equal(outs[0], outs[1])


BATCH_SHOTS = [
    # order, (nq, nr, ns), source, receivers
    (4, (33, 25, 21), True, True),
    (6, (49, 41, 37), True, False),
    (6, (29, 33, 24), False, True),
    (2, (40, 17, 30), False, False),
    (4, (65, 41, 19), True, True),
    (3, (37, 29, 22), True, True),
    (5, (45, 26, 27), False, True),
]


def _batch_solvers(dtype, io=True):
    out = []
    for n, (order, (nq, nr, ns), src, rec) in enumerate(BATCH_SHOTS):
        xyz = W.warped_mesh(nq, nr, ns, seed=30 + n)
        med = W.random_medium((ns, nr, nq), 40 + n)
        s = make_solver(xyz, order, dtype, [1, 0, 0.5, 0, -1, 0], medium=med)
        s.set_state(W.random_state((ns, nr, nq), 50 + n, smooth=True))
        if src and io:
            s.add_source((0.31 + 0.05 * n, 0.5, 0.47), (0.2, 0.1, -0.3, 1.0, 0.0, 0.4), 0, 8.0, 0.05)
        if rec and io:
            s.record(np.array([[1, 2, 3], [nq - 1, nr // 2, ns - 1], [nq // 2, 0, 0]]), 64)
        out.append(s)
    return out


@pytest.mark.parametrize("io", [False, True])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_equals_separate_steps(dtype, io):
    """sbp_step_batch over grids of uneven size and orders 2 to 6 (five
    launch groups), with (io) or without sources and receivers, for 40 steps
    (two chunks of per-step tables): states, times and receiver traces equal
    those of stepping every handle alone.  The batched launches run the same
    kernel bodies as sbp_step (instantiated with their arguments read from a
    device table instead of passed by value), so the results agree to
    rounding: relative max difference below 1e-5 (f32) / 1e-12 (f64)."""
    say("case: batch of %d shots %s io=%s, 40 steps" % (len(BATCH_SHOTS), dtype, io))
    sbp = sbp_mod()
    tol = 1e-5 if dtype == "f32" else 1e-12
    dts = [1.0e-3 * (1 + 0.1 * n) for n in range(len(BATCH_SHOTS))]
    alone = _batch_solvers(dtype, io)
    for s, d in zip(alone, dts):
        s.step(40, d)
    together = _batch_solvers(dtype, io)
    sbp.sbp_step_batch([s.h for s in together], 40, dts)
    report = []
    for n, (a, b) in enumerate(zip(alone, together)):
        x = a.get_state().cpu().numpy().astype(np.float64)
        y = b.get_state().cpu().numpy().astype(np.float64)
        es = rel_max(y, x)
        assert a.time() == b.time(), n
        et = 0.0
        if BATCH_SHOTS[n][3] and io:
            ta = a.traces.cpu().numpy().astype(np.float64)
            tb = b.traces.cpu().numpy().astype(np.float64)
            et = rel_max(tb, ta)
            if et > tol:
                rows = [int(r) for r in np.nonzero(np.abs(ta - tb).reshape(ta.shape[0], -1).max(axis=1))[0]]
                say("  shot %d traces differ at steps %s" % (n, rows[:12]))
        report.append((n, es, et))
    say("  (shot, state rel max, traces rel max): %s" % ["(%d, %.2e, %.2e)" % r for r in report])
    for n, es, et in report:
        assert es <= tol and et <= tol, n
    for s in alone + together:
        s.close()


def test_batch_error_paths():
    say("case: batch error paths")
    sbp = sbp_mod()
    a = _batch_solvers("f32")[:2]
    b = _batch_solvers("f64")[:1]
    with pytest.raises(RuntimeError):
        sbp.sbp_step_batch([a[0].h, b[0].h], 1, [1e-3, 1e-3])      # mixed dtype
    with pytest.raises(RuntimeError):
        sbp.sbp_step_batch([a[0].h, a[0].h], 1, [1e-3, 1e-3])      # same handle twice
    with pytest.raises(RuntimeError):
        sbp.sbp_step_batch([a[0].h, a[1].h], 1, [1e-3, -1.0])      # bad dt
    for s in a + b:
        s.close()


def test_autotune_keeps_state_and_picks_a_candidate():
    """sbp_autotune times launch shapes with right-hand-side evaluations: the
    state is unchanged, the chosen shape is one of the candidates, and
    stepping with it agrees with the default shape to rounding."""
    say("case: autotune order 4 f32 65x41x29")
    nq, nr, ns = 65, 41, 29
    xyz = W.warped_mesh(nq, nr, ns, seed=11)
    med = W.random_medium((ns, nr, nq), 3)
    Q = W.random_state((ns, nr, nq), 7, smooth=True)
    ref = make_solver(xyz, 4, "f32", [1, 0, 0, 0, 0, 1], medium=med)
    ref.set_state(Q)
    ref.step(5, 1e-3)
    want = ref.get_state().cpu().numpy().astype(np.float64)
    ref.close()
    s = make_solver(xyz, 4, "f32", [1, 0, 0, 0, 0, 1], medium=med)
    s.set_state(Q)
    ty, zc, ms = s.autotune(3)
    say("  chosen ty %d zchunk %d, %.4f ms per evaluation" % (ty, zc, ms))
    assert ty in (8, 16) and zc >= 1 and ms > 0
    assert np.array_equal(s.get_state().cpu().numpy(), Q.astype(np.float32))
    s.step(5, 1e-3)
    got = s.get_state().cpu().numpy().astype(np.float64)
    s.close()
    assert rel_max(got, want) < 1e-5


def test_order8_rhs_after_double_precision_kernels():
    """Window positions that the stage kernel reads with zero weights (order
    8's flux rows beyond r above the first tile) are cleared when a block
    starts: a single-precision order-8 right-hand side after double-precision
    kernels (whose data the LDS still holds, some of it NaN or Inf as
    single-precision words) equals the oracle's."""
    say("case: order 8 f32 rhs after f64 kernels")
    xyz = W.warped_mesh(65, 65, 49, seed=21)
    med = W.random_medium((49, 65, 65), 22)
    s64 = make_solver(xyz, 6, "f64", [1, 0, 0.5, 0, -1, 0], medium=med)
    s64.set_state(W.random_state((49, 65, 65), 23, smooth=True))
    s64.step(3, 1e-3)
    s64.close()
    ns, nr, nq = 17, 18, 19
    xyz = W.warped_mesh(nq, nr, ns, seed=24)
    med = W.random_medium((ns, nr, nq), 25)
    Q = W.random_state((ns, nr, nq), 26, smooth=True)
    gamma = [0, 0, 0, 0, 0, 1]
    s = make_solver(xyz, 8, "f32", gamma, medium=med)
    s.set_state(Q)
    got = s.rhs(0.0).cpu().numpy().astype(np.float64)
    s.close()
    blk = E.Block(xyz, 8).set_material(*med)
    want = E.rhs(blk, Q, 0.0, gamma, E.SAT_CHARACTERISTIC, [])
    err = rel_max(got, want)
    say("  rel max = %.3e" % err)
    assert np.isfinite(got).all() and err <= 1e-5
