"""The semi-discrete operator of eq. gen_hyp_transformed_discrete_SAT
assembled literally as one sparse matrix (oracle side; test infrastructure
only).  Used as a brute-force pin of ``elastic.rhs`` on tiny grids.

Differences from ``elastic`` on purpose:
  * derivatives are the Kronecker products D_{eta xi} of Sec. 4.1 acting on
    the flattened grid functions;
  * the stiffness C and P~ = J^{-1} P are applied as explicit 6x6 / 9x9
    matrices (eq. S matrix);
  * boundary penalties use the rotated frame R = (n; m; l) of eq.
    velocity_traction_rotation with an explicit m = normalised (m0 - (n.m0) n),
    the characteristics of eq. characteristics, the hat variables of
    eq. data_hat and the penalty vectors SAT_0 / SAT_n, each face node's 9x9
    penalty block being obtained by applying those formulas to the nine unit
    vectors.
"""
import numpy as np
import scipy.sparse as sp

from .elastic import AXIS, FACES, SAT_TRACTION


def _axis_op(blk, D, xi):
    """D_{eta xi} = I x ... x D x ... x I in the flattening of (ns, nr, nq)."""
    nq, nr, ns = blk.npts
    Iq, Ir, Is = sp.identity(nq), sp.identity(nr), sp.identity(ns)
    Dsp = sp.csr_matrix(D)
    if xi == 0:
        return sp.kron(Is, sp.kron(Ir, Dsp))
    if xi == 1:
        return sp.kron(Is, sp.kron(Dsp, Iq))
    return sp.kron(Dsp, sp.kron(Ir, Iq))


def stiffness(lam, mu):
    """eq. S matrix."""
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    for k in range(3):
        C[k, k] = lam + 2 * mu
    for k in range(3, 6):
        C[k, k] = mu
    return C


def _penalty_block(n, Zp, Zs, rho, lam, mu, g, side, variant):
    """9x9 matrix mapping the nodal state to the 9-vector the face adds to
    P~^{-1} dQ/dt before the factor -H^{-1} e J|grad xi| (characteristic) or
    +- H^{-1} e J |grad xi| (traction).  Built column by column."""
    m0 = np.array([0.3, -0.7, 0.65])  # any vector not parallel to n
    if abs(np.dot(m0, n)) > 0.9 * np.linalg.norm(m0):
        m0 = np.array([0.8, 0.2, -0.4])
    mvec = m0 - np.dot(n, m0) * n
    mvec /= np.linalg.norm(mvec)
    lvec = np.cross(n, mvec)
    R = np.vstack([n, mvec, lvec])
    Z = np.array([Zp, Zs, Zs])
    out = np.zeros((9, 9))
    for col in range(9):
        Q = np.zeros(9)
        Q[col] = 1.0
        v = Q[:3]
        sxx, syy, szz, sxy, sxz, syz = Q[3:]
        sig = np.array([[sxx, sxy, sxz], [sxy, syy, syz], [sxz, syz, szz]])
        T = sig @ n
        if variant == SAT_TRACTION and g == 1.0:
            sat = np.concatenate([T, np.zeros(6)])
            # eq. SAT_free_surface: + at xi = 0, - at xi = 1 ; report with the
            # same leading "-" convention as the characteristic SAT
            out[:, col] = -sat if side == 0 else sat
            continue
        vl = R @ v
        Tl = R @ T
        qc = 0.5 * (Z * vl + Tl)
        pc = 0.5 * (Z * vl - Tl)
        if side == 0:
            vhat = (1 + g) / Z * qc
            That = (1 - g) * qc
            Gl = 0.5 * Z * (vl - vhat) - 0.5 * (Tl - That)
        else:
            vhat = (1 + g) / Z * pc
            That = -(1 - g) * pc
            Gl = 0.5 * Z * (vl - vhat) + 0.5 * (Tl - That)
        Gx = R.T @ Gl
        Gt = R.T @ (Gl / Z)
        sgn = -1.0 if side == 0 else 1.0
        sym = np.array([n[0] * Gt[0], n[1] * Gt[1], n[2] * Gt[2],
                        n[1] * Gt[0] + n[0] * Gt[1],
                        n[2] * Gt[0] + n[0] * Gt[2],
                        n[2] * Gt[1] + n[1] * Gt[2]])
        out[:, col] = np.concatenate([Gx, sgn * sym])
    return out


def assemble(blk, gamma, variant=0):
    """Sparse L with dQ/dt = L Q (flattened state, field-major)."""
    Nn = int(np.prod(blk.shape))
    m = blk.mat
    M = [[blk.M[xi][c].ravel() for c in range(3)] for xi in range(3)]
    Dp = [_axis_op(blk, blk.ops[xi]["Dp"], xi) for xi in range(3)]
    Dm = [_axis_op(blk, blk.ops[xi]["Dm"], xi) for xi in range(3)]
    dg = sp.diags
    Z0 = sp.csr_matrix((Nn, Nn))
    # stress components sigma_{ic} -> field index
    sidx = [[3, 6, 7], [6, 4, 8], [7, 8, 5]]
    blocks = [[Z0] * 9 for _ in range(9)]

    def add(r, c, mat):
        blocks[r][c] = blocks[r][c] + mat

    # divergence of the conservative flux (velocity rows)
    for i in range(3):
        for xi in range(3):
            for c in range(3):
                add(i, sidx[i][c], Dm[xi] @ dg(M[xi][c]))
    # non-conservative terms B_xi(grad_{D+} Q) (stress rows, eq. split_form)
    for xi in range(3):
        ex, ey, ez = (dg(M[xi][c]) for c in range(3))
        add(3, 0, ex @ Dp[xi])
        add(4, 1, ey @ Dp[xi])
        add(5, 2, ez @ Dp[xi])
        add(6, 0, ey @ Dp[xi]); add(6, 1, ex @ Dp[xi])
        add(7, 0, ez @ Dp[xi]); add(7, 2, ex @ Dp[xi])
        add(8, 1, ez @ Dp[xi]); add(8, 2, ey @ Dp[xi])
    Lvol = sp.bmat(blocks, format="csr")

    # boundary penalties, node by node (dense 9x9 blocks, summed over faces)
    rows, cols, vals = [], [], []
    shape = blk.shape
    for f, (xi, side) in enumerate(FACES):
        ax = AXIS[xi]
        hw0 = blk.ops[xi]["H"][0]
        it = np.ndindex(*shape)
        for node in it:
            if node[ax] != (0 if side == 0 else shape[ax] - 1):
                continue
            flat = np.ravel_multi_index(node, shape)
            Mx = np.array([blk.M[xi][c][node] for c in range(3)])
            nrm = np.linalg.norm(Mx)
            n = Mx / nrm
            blkm = _penalty_block(n, m["Zp"][node], m["Zs"][node], m["rho"][node],
                                  m["lam"][node], m["mu"][node], float(gamma[f]), side, variant)
            # SAT_{xi,i} = -H_xi^{-1} e J|grad xi| SAT_i, J|grad xi| = |M_xi|
            blkm = -(nrm / hw0) * blkm
            for a in range(9):
                for b in range(9):
                    if blkm[a, b] != 0.0:
                        rows.append(a * Nn + flat)
                        cols.append(b * Nn + flat)
                        vals.append(blkm[a, b])
    Lsat = sp.csr_matrix((vals, (rows, cols)), shape=(9 * Nn, 9 * Nn))
    # P~ = J^{-1} P, P = diag(rho^{-1} I_3, C)
    Jinv = 1.0 / blk.J.ravel()
    Pt_rows, Pt_cols, Pt_vals = [], [], []
    lam, mu, rho = m["lam"].ravel(), m["mu"].ravel(), m["rho"].ravel()
    for node in range(Nn):
        for i in range(3):
            Pt_rows.append(i * Nn + node); Pt_cols.append(i * Nn + node)
            Pt_vals.append(Jinv[node] / rho[node])
        C = stiffness(lam[node], mu[node])
        for a in range(6):
            for b in range(6):
                if C[a, b] != 0.0:
                    Pt_rows.append((3 + a) * Nn + node); Pt_cols.append((3 + b) * Nn + node)
                    Pt_vals.append(Jinv[node] * C[a, b])
    Pt = sp.csr_matrix((Pt_vals, (Pt_rows, Pt_cols)), shape=(9 * Nn, 9 * Nn))
    return Pt @ (Lvol + Lsat)
