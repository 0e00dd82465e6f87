"""Pins of the oracle's metric terms, free-stream preservation, point source,
source-time functions and the brute-force Kronecker assembly."""
import numpy as np
import pytest

import workloads as W
from oracle import elastic as E
from oracle import kron_form as K


def affine_mesh(shape, seed):
    rng = np.random.default_rng(seed)
    A = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    if np.linalg.det(A) < 0:
        A[:, 0] *= -1
    b = rng.standard_normal(3)
    ns, nr, nq = shape
    U = W.unit_cube(nq, nr, ns)
    X = np.einsum("ij,j...->i...", A, U) + b[:, None, None, None]
    return X, A


@pytest.mark.parametrize("order", [2, 3, 4, 5, 6, 7, 8])
def test_affine_map_metrics_exact(order):
    """For x = A xi + b: J = det A and M = J dxi/dx = J A^{-1} (Sec. 2.2)."""
    X, A = affine_mesh((17, 16, 18) if order > 6 else (13, 14, 12), order)
    blk = E.Block(X, order)
    J = np.linalg.det(A)
    Ainv = np.linalg.inv(A)
    assert np.allclose(blk.J, J, rtol=1e-12, atol=0)
    for xi in range(3):
        for c in range(3):
            assert np.allclose(blk.M[xi][c], J * Ainv[xi, c], rtol=0, atol=1e-11 * abs(J))


@pytest.mark.parametrize("order", [2, 3, 4, 5, 6, 7, 8])
def test_discrete_metric_identity(order):
    """sum_xi D-_xi M[xi][c] = 0 for the conservative cofactor metrics."""
    X = W.warped_mesh(16, 17, 16, seed=order)
    blk = E.Block(X, order)
    for c in range(3):
        s = sum(E.apply_along(blk.ops[xi]["Dm"], blk.M[xi][c], xi) for xi in range(3))
        assert np.abs(s).max() < 1e-11 * max(np.abs(blk.M[0][0]).max(), 1)


@pytest.mark.parametrize("order", [4, 6])
def test_free_stream_preserved_on_curvilinear_mesh(order):
    """Uniform stress, zero velocity, clamped faces (gamma = -1): the
    semi-discrete RHS vanishes to round-off on a warped mesh."""
    X = W.warped_mesh(14, 13, 15, seed=order + 1)
    blk = E.Block(X, order).set_material(*W.random_medium((15, 13, 14), 3))
    Q = np.zeros((9, 15, 13, 14))
    for k, val in enumerate([0.3, -1.2, 0.7, 0.25, -0.4, 0.9]):
        Q[3 + k] = val
    out = E.rhs(blk, Q, 0.0, [-1.0] * 6)
    assert np.abs(out).max() < 1e-10


@pytest.mark.parametrize("order", [4, 6])
def test_metrics_converge_to_analytic(order):
    """The discrete Jacobian on a smooth warped map converges to the analytic
    determinant, in the max norm at the boundary-closure order p of the
    derivative operators (Sec. 4.1)."""
    errs = []
    for n in (17, 33, 65):
        X = W.warped_mesh(n, n, n, seed=5)
        blk = E.Block(X, order)
        # exact derivatives of the seeded map (same draws as warped_mesh)
        rng = np.random.default_rng(5)
        ph = []
        amps = []
        for c in range(3):
            ph.append(rng.uniform(0, 2 * np.pi, size=3))
            amps.append(0.04 * rng.uniform(0.5, 1.0))
        s, r, q = np.meshgrid(*(np.linspace(0, 1, n),) * 3, indexing="ij")
        tw = 2 * np.pi
        Jm = np.zeros((3, 3) + q.shape)
        for c in range(3):
            a, (p0, p1, p2) = amps[c], ph[c]
            Jm[c, 0] = (c == 0) + a * tw * np.cos(tw * q + p0) * np.sin(tw * r + p1) * np.sin(tw * s + p2)
            Jm[c, 1] = (c == 1) + a * tw * np.sin(tw * q + p0) * np.cos(tw * r + p1) * np.sin(tw * s + p2)
            Jm[c, 2] = (c == 2) + a * tw * np.sin(tw * q + p0) * np.sin(tw * r + p1) * np.cos(tw * s + p2)
        Jex = np.linalg.det(np.moveaxis(Jm, (0, 1), (-2, -1)))
        errs.append(np.abs(blk.J - Jex).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > order // 2 - 0.3, rates


@pytest.mark.parametrize("order", [2, 3, 4, 5, 6, 7, 8])
def test_discrete_delta_moments(order):
    """sum_ijk H_ijk J_ijk delta_ijk f_ijk = f(x_s) for tensor polynomials of
    degree < 2(p+1) per reference axis, including near a boundary."""
    X = W.warped_mesh(19, 17, 21, seed=2)
    blk = E.Block(X, order)
    Hw = blk.norm_weights() * blk.J
    width = 2 * (order // 2 + 1)
    rng = np.random.default_rng(order)
    s, r, q = np.meshgrid(*(np.linspace(0, 1, n) for n in (21, 17, 19)), indexing="ij")
    for xi3 in [(0.43, 0.51, 0.37), (0.02, 0.97, 0.5), (1.0, 0.0, 0.111)]:
        sl, w = E.source_stencil(blk, xi3)
        for _ in range(4):
            e = rng.integers(0, width, size=3)
            f = q ** e[0] * r ** e[1] * s ** e[2]
            got = np.sum(Hw[sl] * w * f[sl])
            want = xi3[0] ** e[0] * xi3[1] ** e[1] * xi3[2] ** e[2]
            assert abs(got - want) < 1e-11 * (1 + abs(want))


def test_source_time_functions():
    f0, t0 = 2.0, 0.6
    assert abs(E.stf(E.STF_RICKER, t0, f0, t0) - 1.0) < 1e-15
    # Ricker zero crossings at t0 +- 1 / (pi f0 sqrt 2)
    tz = t0 + 1.0 / (np.pi * f0 * np.sqrt(2))
    assert abs(E.stf(E.STF_RICKER, tz, f0, t0)) < 1e-14
    T = 0.1
    assert abs(E.stf(E.STF_EXPT, T, T) - 1.0 / (T * np.e)) < 1e-13
    assert E.stf(E.STF_EXPT, -0.5, T) == 0.0
    # g = t/T^2 exp(-t/T) integrates to 1
    t = np.linspace(0, 5, 200001)
    g = E.stf(E.STF_EXPT, t, T)
    assert abs(np.sum(0.5 * (g[1:] + g[:-1]) * np.diff(t)) - 1.0) < 1e-6


@pytest.mark.parametrize("order,shape", [(2, (6, 5, 7)), (4, (9, 8, 10)), (6, (12, 13, 12))])
@pytest.mark.parametrize("variant", [E.SAT_CHARACTERISTIC, E.SAT_TRACTION])
def test_rhs_equals_kronecker_assembly(order, shape, variant):
    ns, nr, nq = shape
    blk = E.Block(W.warped_mesh(nq, nr, ns, seed=order), order)
    blk.set_material(*W.random_medium(shape, order + 1))
    gamma = [1.0, -1.0, 0.3, 0.0, -0.6, 1.0]
    Q = W.random_state(shape, order + 2)
    L = K.assemble(blk, gamma, variant)
    want = (L @ Q.ravel()).reshape(Q.shape)
    got = E.rhs(blk, Q, 0.0, gamma, variant)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("order", [4, 6])
def test_node_by_node_rhs_equals_whole_array(order):
    """The spot-check form used at full size agrees with the whole-array RHS
    (interior, face, edge, corner and source-support nodes)."""
    shape = (15, 13, 14)
    ns, nr, nq = shape
    blk = E.Block(W.warped_mesh(nq, nr, ns, seed=11), order)
    blk.set_material(*W.random_medium(shape, 12))
    src = E.Source(blk, (0.45, 0.5, 0.55), (0.1, -0.2, 0.3, 1.0, 0.5, -0.7), E.STF_RICKER, 2.0, 0.1)
    gamma = [0.0, 1.0, -0.5, 0.0, 0.25, 1.0]
    Q = W.random_state(shape, 13)
    full = E.rhs(blk, Q, 0.07, gamma, sources=[src])
    rng = np.random.default_rng(1)
    nodes = [(0, 0, 0), (nq - 1, nr - 1, ns - 1), (0, 5, 7), (6, 0, 3), (7, 6, ns - 1), (6, 6, 7)]
    nodes += [tuple(int(rng.integers(0, n)) for n in (nq, nr, ns)) for _ in range(20)]
    got = E.rhs_at(blk, Q, nodes, 0.07, gamma, sources=[src])
    want = np.array([full[:, k, j, i] for i, j, k in nodes])
    assert np.abs(got - want).max() <= 1e-12 * np.abs(full).max()


def _poly_map(U, V, Z):
    """A curvilinear map polynomial of degree <= 3 in each reference
    coordinate (exactly reproduced by Lagrange interpolation over 4 or more
    nodes per axis)."""
    x = U + 0.06 * U ** 2 * V - 0.03 * V * Z ** 3
    y = V + 0.05 * V * Z ** 2 + 0.02 * U ** 3
    z = Z + 0.04 * U * V * Z - 0.05 * Z ** 2 * V
    return np.stack([x, y, z])


@pytest.mark.parametrize("order", [2, 4, 6])
def test_locate_inverts_polynomial_map_exactly(order):
    """On a map that the interpolant reproduces exactly (degree < 2(p+1) per
    axis, p = order // 2 >= 1), locating X(xi*) returns xi* (random points,
    points in the boundary closures and on faces, corners)."""
    nq, nr, ns = 17, 15, 19
    ref = W.unit_cube(nq, nr, ns)
    X = _poly_map(ref[0], ref[1], ref[2])
    blk = E.Block(X, order)
    rng = np.random.default_rng(order)
    pts = [tuple(rng.uniform(0, 1, 3)) for _ in range(6)]
    pts += [(0.0, 0.3, 0.7), (1.0, 1.0, 0.0), (0.02, 0.97, 0.5), (0.51, 0.0, 1.0)]
    for xs in pts:
        x = _poly_map(*[np.array(v) for v in xs])
        got = E.locate(blk, x)
        assert np.allclose(got, xs, atol=1e-11, rtol=0), (xs, got)


def test_locate_nodes_and_outside():
    """A node's coordinates give that node's reference position; a point
    beyond a face is rejected."""
    xyz = W.warped_mesh(13, 14, 12, seed=5)
    blk = E.Block(xyz, 4)
    for (k, j, i) in [(0, 0, 0), (11, 13, 12), (4, 7, 2), (6, 0, 9)]:
        got = E.locate(blk, xyz[:, k, j, i])
        assert np.allclose(got, (i / 12, j / 13, k / 11), atol=1e-12)
    with pytest.raises(ValueError):
        E.locate(blk, xyz[:, 5, 5, 0] - np.array([0.05, 0.0, 0.0]))


def test_locate_topography_map():
    """On the transfinite topography mesh x = xi L, y = eta L, z = -D +
    zeta (z_top + D), locating a point returns xi and eta exactly (x and y
    are linear in them) and zeta to within the interpolation error of the
    surface (closed form zeta = (z + D) / (z_top + D))."""
    wl = W.topo_layer(nq=65, nr=65, ns=49)
    blk = E.Block(wl["xyz"], 6)
    L, D = 12.8, 9.6
    rng = np.random.default_rng(2)
    _, ztop = W.topo_mesh(5, 5, 5)
    for _ in range(4):
        xs, ys = rng.uniform(0.1, 0.9, 2) * L
        zt = float(ztop(np.array(xs), np.array(ys)))
        zeta = rng.uniform(0.1, 0.9)
        z = -D + zeta * (zt + D)
        got = E.locate(blk, (xs, ys, z))
        assert abs(got[0] - xs / L) < 1e-12 and abs(got[1] - ys / L) < 1e-12
        assert abs(got[2] - zeta) < 1e-6
