"""Pins of the oracle's discrete adjoint (oracle/adjoint.py) against what
the mathematics fixes, independently of its own construction:

  * the material gradient against central finite differences of the misfit,
    the forward runs done by ``elastic.run`` (not by the adjoint module);
  * d chi / d Q0 against finite differences in the initial state;
  * the complex-step material derivatives of the right-hand side against
    central finite differences of ``elastic.rhs``;
  * the energy identity behind the library's adjoint (Theorem
    theo_sbp_sem_discrete with the penalties of Sec. 5): W L + L^T W, with W
    the energy weights H J diag(rho I_3, C^{-1}), couples boundary nodes only.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import adjoint as ADJ
from oracle import elastic as E
from oracle import kron_form

SHAPE = (8, 9, 10)  # (ns, nr, nq)


def setup(order=4, variant=E.SAT_CHARACTERISTIC, seed=0):
    ns, nr, nq = SHAPE
    xyz = W.warped_mesh(nq, nr, ns, seed=seed + 3, amp=0.03)
    rho, cp, cs = W.random_medium(SHAPE, seed + 5)
    blk = E.Block(xyz, order).set_material(rho, cp, cs)
    gamma = (1.0, 0.0, -1.0, 0.5, 0.0, 1.0)
    src = E.Source(blk, (0.42, 0.55, 0.47), (0.3, -0.2, 0.1, 1.0, 0.4, -0.3), E.STF_RICKER, 6.0, 0.12)
    rec = np.array([[2, 3, 7], [7, 4, 7], [5, 6, 3]])
    Q0 = 0.1 * W.random_state(SHAPE, seed + 7, smooth=True)
    dt = W.cfl_dt(xyz, cp, 0.3)
    return blk, gamma, src, rec, Q0, dt


def lame(blk):
    return blk.mat["rho"].copy(), blk.mat["lam"].copy(), blk.mat["mu"].copy()


def set_lame(blk, rho, lam, mu):
    blk.set_material(rho, np.sqrt((lam + 2 * mu) / rho), np.sqrt(mu / rho))


def run_misfit(blk, Q0, nsteps, dt, gamma, variant, src, rec, target):
    _, _, tr = E.run(blk, Q0, nsteps, dt, gamma, variant, sources=[src], receivers=rec)
    return ADJ.misfit(tr, target)


@pytest.mark.parametrize("order,variant", [(4, E.SAT_CHARACTERISTIC), (3, E.SAT_TRACTION)])
def test_material_gradient_matches_finite_differences(order, variant):
    blk, gamma, src, rec, Q0, dt = setup(order, variant)
    nsteps = 10
    rng = np.random.default_rng(11)
    target = 0.01 * rng.standard_normal((nsteps, rec.shape[0], 3))
    chi, g, _, tr = ADJ.gradient(blk, Q0, nsteps, dt, gamma, variant, [src], rec, target)
    assert chi == pytest.approx(run_misfit(blk, Q0, nsteps, dt, gamma, variant, src, rec, target), rel=1e-13)
    rho0, lam0, mu0 = lame(blk)
    base = dict(rho=rho0, lam=lam0, mu=mu0)
    for p in ADJ.PARAMS + ("all",):
        dirs = {q: np.zeros(SHAPE) for q in ADJ.PARAMS}
        for q in (ADJ.PARAMS if p == "all" else (p,)):
            dirs[q] = base[q] * rng.uniform(-1, 1, size=SHAPE)
        eps = 1e-5
        vals = []
        for s in (1, -1):
            set_lame(blk, *(base[q] + s * eps * dirs[q] for q in ADJ.PARAMS))
            vals.append(run_misfit(blk, Q0, nsteps, dt, gamma, variant, src, rec, target))
        set_lame(blk, rho0, lam0, mu0)
        fd = (vals[0] - vals[1]) / (2 * eps)
        ad = sum(float(np.sum(g[q] * dirs[q])) for q in ADJ.PARAMS)
        assert ad == pytest.approx(fd, rel=2e-6, abs=1e-12 * abs(chi)), (p, ad, fd)


def test_initial_state_gradient_matches_finite_differences():
    blk, gamma, src, rec, Q0, dt = setup()
    nsteps = 8
    rng = np.random.default_rng(12)
    target = 0.01 * rng.standard_normal((nsteps, rec.shape[0], 3))
    chi, _, Qb0, _ = ADJ.gradient(blk, Q0, nsteps, dt, gamma, E.SAT_CHARACTERISTIC, [src], rec, target)
    dQ = rng.standard_normal(Q0.shape) * 0.1
    eps = 1e-4
    fp = run_misfit(blk, Q0 + eps * dQ, nsteps, dt, gamma, E.SAT_CHARACTERISTIC, src, rec, target)
    fm = run_misfit(blk, Q0 - eps * dQ, nsteps, dt, gamma, E.SAT_CHARACTERISTIC, src, rec, target)
    # chi is quadratic in Q0: the central difference is exact up to rounding
    assert float(np.sum(Qb0 * dQ)) == pytest.approx((fp - fm) / (2 * eps), rel=1e-8)


def test_complex_step_derivatives_match_finite_differences():
    blk, gamma, _, _, _, _ = setup(6 if min(SHAPE) >= 12 else 4)
    Q = W.random_state(SHAPE, 21)
    der = ADJ.rhs_material_derivatives(blk, Q, gamma)
    rho0, lam0, mu0 = lame(blk)
    base = dict(rho=rho0, lam=lam0, mu=mu0)
    rng = np.random.default_rng(13)
    for p in ADJ.PARAMS:
        d = base[p] * rng.uniform(0.5, 1.0, size=SHAPE)
        eps = 1e-6
        out = []
        for s in (1, -1):
            m = dict(base)
            m[p] = base[p] + s * eps * d
            set_lame(blk, m["rho"], m["lam"], m["mu"])
            out.append(E.volume_rhs(blk, Q) + E.sat_rhs(blk, Q, gamma))
        set_lame(blk, rho0, lam0, mu0)
        fd = (out[0] - out[1]) / (2 * eps)
        want = der[p] * d
        assert np.max(np.abs(fd - want)) <= 1e-6 * np.max(np.abs(want)), p


def test_energy_weights_make_the_operator_skew_off_the_boundary():
    blk, gamma, _, _, _, _ = setup()
    L = kron_form.assemble(blk, gamma)
    m = blk.mat
    Nn = int(np.prod(SHAPE))
    w = (blk.norm_weights() * blk.J).ravel()
    rho, lam, mu = m["rho"].ravel(), m["lam"].ravel(), m["mu"].ravel()
    rows, cols, vals = [], [], []
    for node in range(Nn):
        for i in range(3):
            rows.append(i * Nn + node); cols.append(i * Nn + node); vals.append(w[node] * rho[node])
        Sinv = np.linalg.inv(kron_form.stiffness(lam[node], mu[node]))
        for a in range(6):
            for b in range(6):
                if Sinv[a, b] != 0.0:
                    rows.append((3 + a) * Nn + node); cols.append((3 + b) * Nn + node)
                    vals.append(w[node] * Sinv[a, b])
    Wm = sp.csr_matrix((vals, (rows, cols)), shape=(9 * Nn, 9 * Nn))
    K = (Wm @ L + L.T @ Wm).tocoo()
    ns, nr, nq = SHAPE
    k, j, i = np.unravel_index(K.row % Nn, SHAPE)
    big = np.abs(K.data) > 1e-12 * np.abs(Wm @ L).max()
    onb = (i == 0) | (i == nq - 1) | (j == 0) | (j == nr - 1) | (k == 0) | (k == ns - 1)
    assert np.all(onb[big])
    kc, jc, ic = np.unravel_index(K.col % Nn, SHAPE)
    onbc = (ic == 0) | (ic == nq - 1) | (jc == 0) | (jc == nr - 1) | (kc == 0) | (kc == ns - 1)
    assert np.all(onbc[big])
    assert np.any(big)  # the boundary terms are there
