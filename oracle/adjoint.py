"""Discrete adjoint of the fully discrete scheme and the gradient of a
receiver misfit with respect to the nodal material (oracle side; test
infrastructure only).

The paper does not treat adjoints; this is an extension built on its scheme.
What is differentiated is the fully discrete method exactly as the rest of
the oracle runs it: the semi-discrete operator of eq.
gen_hyp_transformed_discrete_SAT (with sources, eq. momententor_pointsource)
advanced by the five-stage 2N-storage Runge-Kutta scheme of Sec. 7, receivers
sampling v after every step.  The misfit is

    chi = 1/2 sum_n sum_r |v(x_r, t_{n+1}) - d_{n r}|^2 .

Definitions written out (the chain rule, nothing more):
  * each stage reads  dQ_k = A_k dQ_{k-1} + dt (L Q_{k-1} + f_k),
                      Q_k  = Q_{k-1} + B_k dQ_k ;
    its adjoint, run backwards over the stages of a step with the adjoint
    state Qb and register dQb, is
                      dQb += B_k Qb
                      Qb  += dt L^T dQb
                      g   += dt (d(L Q_{k-1}) / dm)^T dQb
                      dQb  = A_k dQb ,
    and before the reverse pass over step n the misfit adds (v - d) of the
    receivers of step n to the velocity part of Qb;
  * L^T is the explicit transpose of the sparse operator assembled by
    ``kron_form.assemble`` (an independent assembly of the same operator);
  * the right-hand side at a node depends on the material of that node only
    (pointwise coefficients rho, lambda, mu after the derivatives; the
    penalties of the node's faces), so d(L Q)/d rho is diagonal and one
    complex-step evaluation of ``elastic.rhs`` per parameter (rho, lambda and
    mu perturbed by i h at every node at once) gives all of it to rounding.
The sources do not depend on the state or the material and drop out of the
adjoint.  Pinned by central finite differences of the misfit computed with
``elastic.run`` (tests/test_oracle_adjoint.py).
"""
import numpy as np

from . import elastic as E
from . import kron_form
from . import lsrk

PARAMS = ("rho", "lam", "mu")


def misfit(traces, target):
    """chi = 1/2 sum |traces - target|^2."""
    r = np.asarray(traces) - np.asarray(target)
    return 0.5 * float(np.sum(r * r))


def forward_stage_inputs(blk, Q0, nsteps, dt, gamma, variant=E.SAT_CHARACTERISTIC, sources=(), receivers=(),
                         t0=0.0):
    """Run the scheme as ``elastic.run`` does, keeping every stage input.
    Returns (stage inputs [n][k] (9, ns, nr, nq), traces [nsteps, nrec, 3])."""
    rec = np.asarray(receivers, dtype=np.int64).reshape(-1, 3)
    Q = np.array(Q0, dtype=np.float64, copy=True)
    dQ = np.zeros_like(Q)
    stages = []
    traces = np.zeros((nsteps, rec.shape[0], 3))
    for n in range(nsteps):
        t = t0 + n * dt
        ins = []
        for k in range(lsrk.NSTAGE):
            ins.append(Q.copy())
            dQ *= lsrk.A_F[k]
            dQ += dt * E.rhs(blk, Q, t + lsrk.C_F[k] * dt, gamma, variant, sources)
            Q += lsrk.B_F[k] * dQ
        stages.append(ins)
        for c in range(3):
            traces[n, :, c] = Q[c][rec[:, 2], rec[:, 1], rec[:, 0]]
    return stages, traces


def rhs_material_derivatives(blk, Q, gamma, variant=E.SAT_CHARACTERISTIC, h=1e-30):
    """d rhs(Q)_node / d m_node for m in (rho, lambda, mu): a dict of
    (9, ns, nr, nq) arrays, by the complex step Im(rhs(Q; m + i h)) / h
    (sources omitted: they do not depend on the material)."""
    base = blk.mat
    Qc = np.asarray(Q, dtype=np.complex128)
    out = {}
    try:
        for p in PARAMS:
            rho = base["rho"].astype(np.complex128)
            lam = base["lam"].astype(np.complex128)
            mu = base["mu"].astype(np.complex128)
            if p == "rho":
                rho = rho + 1j * h
            elif p == "lam":
                lam = lam + 1j * h
            else:
                mu = mu + 1j * h
            # Z_p = rho c_p = sqrt(rho (lambda + 2 mu)), Z_s = rho c_s = sqrt(rho mu)
            blk.mat = dict(base, rho=rho, lam=lam, mu=mu, Zp=np.sqrt(rho * (lam + 2 * mu)), Zs=np.sqrt(rho * mu))
            r = E.volume_rhs(blk, Qc) + E.sat_rhs(blk, Qc, gamma, variant)
            out[p] = r.imag / h
    finally:
        blk.mat = base
    return out


def adjoint_operator(blk, gamma, variant=E.SAT_CHARACTERISTIC):
    """L^T as a sparse matrix on the flattened (field-major) state."""
    return kron_form.assemble(blk, gamma, variant).T.tocsr()


def adjoint_rhs(blk, lam, gamma, variant=E.SAT_CHARACTERISTIC, LT=None):
    """L^T applied to an adjoint state lam of shape (9, ns, nr, nq)."""
    if LT is None:
        LT = adjoint_operator(blk, gamma, variant)
    lam = np.asarray(lam, dtype=np.float64)
    return (LT @ lam.ravel()).reshape(lam.shape)


def gradient(blk, Q0, nsteps, dt, gamma, variant=E.SAT_CHARACTERISTIC, sources=(), receivers=(), target=None,
             t0=0.0):
    """Misfit chi and its gradient.

    Returns (chi, g, Qb0, traces): g is a dict of d chi / d m (ns, nr, nq)
    for m in (rho, lambda, mu) at every node, Qb0 = d chi / d Q0 (9, ns, nr,
    nq), traces the forward receiver traces."""
    rec = np.asarray(receivers, dtype=np.int64).reshape(-1, 3)
    stages, traces = forward_stage_inputs(blk, Q0, nsteps, dt, gamma, variant, sources, rec, t0)
    target = np.zeros_like(traces) if target is None else np.asarray(target, dtype=np.float64)
    chi = misfit(traces, target)
    res = traces - target
    LT = adjoint_operator(blk, gamma, variant)
    Qb = np.zeros_like(np.asarray(Q0, dtype=np.float64))
    g = {p: np.zeros(blk.shape) for p in PARAMS}
    for n in range(nsteps - 1, -1, -1):
        # the misfit reads v after step n
        for r in range(rec.shape[0]):
            i, j, k = rec[r]
            for c in range(3):
                Qb[c, k, j, i] += res[n, r, c]
        dQb = np.zeros_like(Qb)
        for k in range(lsrk.NSTAGE - 1, -1, -1):
            dQb += lsrk.B_F[k] * Qb
            Qb += dt * (LT @ dQb.ravel()).reshape(Qb.shape)
            der = rhs_material_derivatives(blk, stages[n][k], gamma, variant)
            for p in PARAMS:
                g[p] += dt * np.sum(der[p] * dQb, axis=0)
            dQb *= lsrk.A_F[k]
    return chi, g, Qb, traces
