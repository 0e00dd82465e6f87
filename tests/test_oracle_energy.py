"""Energy-rate pins of the oracle RHS (Theorems of Sec. 4.2 and Sec. 5).

For random states, random heterogeneous media and a warped curvilinear mesh,
dE/dt = <Q, P~^{-1} dQ/dt>_H computed from the oracle RHS must equal the
boundary expressions the theorems give, evaluated here independently of the
oracle's SAT code (explicit rotated (n, m, l) frame, characteristic variables
and hat variables of App. A):

* volume terms only:   dE/dt = I(v^T T)  (surface term, eq. disc_boundary_term)
* characteristic SAT:  dE/dt = F_luc + I(v^_T T^)
                       = - sum_faces I_face( sum_eta (G_eta^2 + (1 - g^2) w_eta^2) / Z_eta )
  with w = q at xi = 0 and p at xi = 1 (eq. identity_pen, eq. identity_3_bc)
* traction SAT on all faces: dE/dt = 0.
A wrong sign, a swapped D+/D- or a dropped face term breaks these.
"""
import numpy as np
import pytest

import workloads as W
from oracle import elastic as E
from oracle.elastic import AXIS, FACES


def make_block(order, shape=None, seed=0, warped=True):
    # at least 2 m points per axis (m = order closure rows)
    shape = shape or ((13, 12, 14) if order <= 6 else ((15, 14, 16) if order == 7 else (17, 16, 18)))
    ns, nr, nq = shape
    xyz = W.warped_mesh(nq, nr, ns, seed) if warped else W.unit_cube(nq, nr, ns)
    blk = E.Block(xyz, order)
    blk.set_material(*W.random_medium(blk.shape, seed + 1))
    return blk


def energy_rate(blk, Q, dQ):
    """<Q, P~^{-1} dQ>_H with P~^{-1} = J diag(rho I, S)."""
    m = blk.mat
    w = blk.norm_weights() * blk.J
    kin = m["rho"] * (Q[0] * dQ[0] + Q[1] * dQ[1] + Q[2] * dQ[2])
    lam, mu = m["lam"], m["mu"]
    # S sigma-dot via the compliance written as a linear solve per node
    ns, nr, nq = blk.shape
    tot = np.sum(w * kin)
    for idx in np.ndindex(ns, nr, nq):
        C = np.zeros((6, 6))
        C[:3, :3] = lam[idx]
        for k in range(3):
            C[k, k] += 2 * mu[idx]
        for k in range(3, 6):
            C[k, k] = mu[idx]
        sd = np.linalg.solve(C, dQ[3:9][(slice(None),) + idx])
        tot += w[idx] * np.dot(Q[3:9][(slice(None),) + idx], sd)
    return tot


def face_nodes(blk, xi, side):
    ax = AXIS[xi]
    for idx in np.ndindex(*blk.shape):
        if idx[ax] == (0 if side == 0 else blk.shape[ax] - 1):
            yield idx


def transverse_weight(blk, xi, idx):
    w = 1.0
    for a in range(3):
        if a != xi:
            w *= blk.ops[a]["H"][idx[AXIS[a]]]
    return w


def local_frame(n):
    m0 = np.array([0.2, 0.9, -0.4])
    mm = m0 - np.dot(n, m0) * n
    mm /= np.linalg.norm(mm)
    return np.vstack([n, mm, np.cross(n, mm)])


def nodal(blk, Q, idx):
    v = np.array([Q[c][idx] for c in range(3)])
    sxx, syy, szz, sxy, sxz, syz = (Q[3 + k][idx] for k in range(6))
    sig = np.array([[sxx, sxy, sxz], [sxy, syy, syz], [sxz, syz, szz]])
    return v, sig


def surface_term(blk, Q):
    """I(v^T T): + on xi = 1 faces, - on xi = 0 faces."""
    tot = 0.0
    for xi, side in FACES:
        for idx in face_nodes(blk, xi, side):
            Mx = np.array([blk.M[xi][c][idx] for c in range(3)])
            nrm = np.linalg.norm(Mx)
            v, sig = nodal(blk, Q, idx)
            T = sig @ (Mx / nrm)
            tot += (1 if side else -1) * transverse_weight(blk, xi, idx) * nrm * np.dot(v, T)
    return tot


def sat_dissipation(blk, Q, gamma):
    tot = 0.0
    m = blk.mat
    for f, (xi, side) in enumerate(FACES):
        g = gamma[f]
        for idx in face_nodes(blk, xi, side):
            Mx = np.array([blk.M[xi][c][idx] for c in range(3)])
            nrm = np.linalg.norm(Mx)
            n = Mx / nrm
            R = local_frame(n)
            v, sig = nodal(blk, Q, idx)
            vl, Tl = R @ v, R @ (sig @ n)
            Z = np.array([m["Zp"][idx], m["Zs"][idx], m["Zs"][idx]])
            qc = 0.5 * (Z * vl + Tl)
            pc = 0.5 * (Z * vl - Tl)
            if side == 0:   # hat variables preserve q, satisfy the BC
                vh, Th = (1 + g) / Z * qc, (1 - g) * qc
                G = 0.5 * Z * (vl - vh) - 0.5 * (Tl - Th)
                wout = qc
            else:
                vh, Th = (1 + g) / Z * pc, -(1 - g) * pc
                G = 0.5 * Z * (vl - vh) + 0.5 * (Tl - Th)
                wout = pc
            tot -= transverse_weight(blk, xi, idx) * nrm * np.sum((G ** 2 + (1 - g * g) * wout ** 2) / Z)
    return tot


@pytest.mark.parametrize("order", [2, 3, 4, 5, 6, 7, 8])
def test_volume_terms_give_surface_term(order):
    blk = make_block(order, seed=order)
    Q = W.random_state(blk.shape, 10 + order)
    got = energy_rate(blk, Q, E.volume_rhs(blk, Q))
    want = surface_term(blk, Q)
    assert abs(got - want) <= 1e-11 * abs(want)


def test_negative_control_same_operator_breaks_identity():
    """Using D+ for the flux divergence as well (a plausible mistake) leaves a
    volume residual: the identity above is a real check."""
    blk = make_block(4, seed=3)
    Q = W.random_state(blk.shape, 4)
    for o in blk.ops:
        o["Dm_saved"] = o["Dm"]
        o["Dm"] = o["Dp"]
    try:
        got = energy_rate(blk, Q, E.volume_rhs(blk, Q))
    finally:
        for o in blk.ops:
            o["Dm"] = o.pop("Dm_saved")
    want = surface_term(blk, Q)
    assert abs(got - want) > 1e-3 * abs(want)


@pytest.mark.parametrize("order", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("gseed", [0, 1])
def test_characteristic_sat_energy_rate(order, gseed):
    blk = make_block(order, seed=20 + order)
    rng = np.random.default_rng(gseed)
    gamma = list(rng.uniform(-1, 1, size=6))
    gamma[gseed] = 1.0   # include exact free-surface and clamped faces
    gamma[5 - gseed] = -1.0
    Q = W.random_state(blk.shape, 30 + order)
    got = energy_rate(blk, Q, E.rhs(blk, Q, 0.0, gamma))
    want = sat_dissipation(blk, Q, gamma)
    assert want < 0
    assert abs(got - want) <= 1e-11 * abs(want)


@pytest.mark.parametrize("order", [4, 6])
def test_traction_sat_conserves_energy(order):
    blk = make_block(order, seed=40 + order)
    Q = W.random_state(blk.shape, 41)
    dQ = E.rhs(blk, Q, 0.0, [1.0] * 6, E.SAT_TRACTION)
    got = energy_rate(blk, Q, dQ)
    scale = abs(energy_rate(blk, Q, E.volume_rhs(blk, Q))) + 1.0
    assert abs(got) <= 1e-11 * scale


def test_hat_variables_closed_form():
    """Hat variables of App. A satisfy the boundary condition eq. BC_General2
    exactly, keep the outgoing characteristic and obey eq. identity_3_bc."""
    rng = np.random.default_rng(7)
    for _ in range(100):
        Z, v, T = rng.uniform(0.5, 3), rng.standard_normal(), rng.standard_normal()
        g = rng.uniform(-1, 1)
        q, p = 0.5 * (Z * v + T), 0.5 * (Z * v - T)
        vh, Th = (1 + g) / Z * q, (1 - g) * q          # xi = 0
        assert abs(0.5 * Z * (1 - g) * vh - 0.5 * (1 + g) * Th) < 1e-13
        assert abs(0.5 * (Z * vh + Th) - q) < 1e-13
        assert abs(Th * vh - (1 - g * g) / Z * q * q) < 1e-13
        vh, Th = (1 + g) / Z * p, -(1 - g) * p         # xi = 1
        assert abs(0.5 * Z * (1 - g) * vh + 0.5 * (1 + g) * Th) < 1e-13
        assert abs(0.5 * (Z * vh - Th) - p) < 1e-13
        assert abs(Th * vh + (1 - g * g) / Z * p * p) < 1e-13


def test_energy_decays_in_time_without_sources():
    """Fully discrete: LSRK4 at CFL 0.5 never increases the energy for the
    Cartesian pulse workload (21^3 reduced to 15^3 here for speed)."""
    wl = W.cube_pulse(n=15)
    blk = E.Block(wl["xyz"], wl["order"]).set_material(wl["rho"], wl["cp"], wl["cs"])
    Q = wl["Q0"].copy()
    e_prev = E.energy(blk, Q)
    for _ in range(10):
        Q, _, _ = E.run(blk, Q, 3, wl["dt"], wl["gamma"])
        e = E.energy(blk, Q)
        assert e <= e_prev * (1 + 1e-12)
        e_prev = e


def test_energy_function_is_the_weighted_norm():
    """elastic.energy equals 1/2 <Q, P~^{-1} Q>_H with the compliance applied
    as an explicit 6x6 solve per node (independent of the closed form used in
    elastic.energy)."""
    blk = make_block(4, shape=(9, 10, 11), seed=5)
    Q = W.random_state(blk.shape, 6)
    m = blk.mat
    w = blk.norm_weights() * blk.J
    want = 0.0
    for idx in np.ndindex(*blk.shape):
        C = np.zeros((6, 6))
        C[:3, :3] = m["lam"][idx]
        for k in range(3):
            C[k, k] += 2 * m["mu"][idx]
        for k in range(3, 6):
            C[k, k] = m["mu"][idx]
        sig = Q[3:9][(slice(None),) + idx]
        v = Q[0:3][(slice(None),) + idx]
        want += 0.5 * w[idx] * (m["rho"][idx] * v @ v + sig @ np.linalg.solve(C, sig))
    assert abs(E.energy(blk, Q) - want) <= 1e-12 * want


def test_run_records_receivers_and_matches_manual_stepping():
    wl = W.cube_pulse(n=9)
    blk = E.Block(wl["xyz"], 4).set_material(wl["rho"], wl["cp"], wl["cs"])
    rec = np.array([[1, 2, 3], [8, 0, 8], [4, 4, 4]])
    Q, t, tr = E.run(blk, wl["Q0"], 3, wl["dt"], wl["gamma"], receivers=rec)
    from oracle import lsrk
    Qm = wl["Q0"].copy()
    d = np.zeros_like(Qm)
    for n in range(3):
        lsrk.step(Qm, d, n * wl["dt"], wl["dt"], lambda q, tt: E.rhs(blk, q, tt, wl["gamma"]))
        for r, (i, j, k) in enumerate(rec):
            assert np.array_equal(tr[n, r], Qm[0:3, k, j, i])
    assert np.array_equal(Q, Qm)
    assert abs(t - 3 * wl["dt"]) < 1e-15
