"""Semi-discrete upwind-SBP elastic solver on one curvilinear block, FP64,
CPU (oracle side; test infrastructure only).

Every function follows a passage of the paper; readings of silent or garbled
passages are marked "reading".  Grid functions have shape (ns, nr, nq); the
state Q has shape (9, ns, nr, nq) with fields (vx, vy, vz, sxx, syy, szz, sxy,
sxz, syz) (eq. elastic_sys).  Face order everywhere: (q0, q1, r0, r1, s0, s1).
"""
import numpy as np

from . import lsrk
from . import sbp_operators as sbp

# reference axis xi in (q, r, s) -> numpy axis of a grid function
AXIS = (2, 1, 0)
FACES = ((0, 0), (0, 1), (1, 0), (1, 1), (2, 0), (2, 1))  # (xi, side)
SAT_CHARACTERISTIC = 0
SAT_TRACTION = 1
STF_RICKER = 0
STF_EXPT = 1


def apply_along(D, f, xi):
    """(D applied along reference axis xi) f, with D a dense 1D operator: the
    tensor-product operator of Sec. 4.1 (I x ... x D x ... x I)."""
    ax = AXIS[xi]
    return np.moveaxis(np.tensordot(D, f, axes=([1], [ax])), 0, ax)


def stress_tensor(sig6):
    """Symmetric 3x3 stress from (sxx, syy, szz, sxy, sxz, syz)."""
    sxx, syy, szz, sxy, sxz, syz = sig6
    return [[sxx, sxy, sxz], [sxy, syy, syz], [sxz, syz, szz]]


class Block:
    """One curvilinear block: operators, metric terms and material.

    xyz   : (3, ns, nr, nq) physical node coordinates (x, y, z).
    order : interior order of the upwind SBP pair (2, 4 or 6).
    """

    def __init__(self, xyz, order):
        xyz = np.asarray(xyz, dtype=np.float64)
        if xyz.ndim != 4 or xyz.shape[0] != 3:
            raise ValueError("xyz must have shape (3, ns, nr, nq)")
        self.order = order
        self.shape = xyz.shape[1:]
        ns, nr, nq = self.shape
        self.npts = (nq, nr, ns)  # points along q, r, s
        self.ops = [sbp.operators(order, n) for n in self.npts]
        self.xyz = xyz
        self._metrics()
        self.mat = None

    # ---- Sec. 2.2 curvilinear transform; metric discretisation is a reading
    def _metrics(self):
        """Coordinate derivatives x_{c,xi} = D0_xi x_c with D0 = (D+ + D-)/2
        (reading: the paper does not say how metrics are discretised).
        J = det[x_{c,xi}] (Jacobian formula of Sec. 2.2).
        M[xi][c] = J * d(xi)/d(x_c) in the conservative cofactor form
            M[xi][c] = D-_zeta(e * D0_eta d) - D-_eta(e * D0_zeta d)
        with (xi, eta, zeta) and (c, d, e) cyclic (reading), which makes
        sum_xi D-_xi M[xi][c] = 0 to round-off (discrete metric identity)."""
        X = self.xyz
        d = [[apply_along(self.ops[xi]["D0"], X[c], xi) for xi in range(3)] for c in range(3)]
        self.dxdxi = d
        # J = x_q (y_r z_s - z_r y_s) - y_q (x_r z_s - z_r x_s) + z_q (x_r y_s - y_r x_s)
        xq, xr, xs = d[0]
        yq, yr, ys = d[1]
        zq, zr, zs = d[2]
        J = xq * (yr * zs - zr * ys) - yq * (xr * zs - zr * xs) + zq * (xr * ys - yr * xs)
        if np.any(J <= 0):
            raise ValueError("non-positive Jacobian")
        self.J = J
        M = [[None] * 3 for _ in range(3)]
        for xi in range(3):
            eta, zeta = (xi + 1) % 3, (xi + 2) % 3
            for c in range(3):
                dd, e = (c + 1) % 3, (c + 2) % 3
                M[xi][c] = (apply_along(self.ops[zeta]["Dm"], X[e] * apply_along(self.ops[eta]["D0"], X[dd], eta), zeta)
                            - apply_along(self.ops[eta]["Dm"], X[e] * apply_along(self.ops[zeta]["D0"], X[dd], zeta), eta))
        self.M = M

    # ---- eq. S matrix: isotropic stiffness from rho, cp, cs
    def set_material(self, rho, cp, cs):
        rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), self.shape).copy()
        cp = np.broadcast_to(np.asarray(cp, dtype=np.float64), self.shape).copy()
        cs = np.broadcast_to(np.asarray(cs, dtype=np.float64), self.shape).copy()
        mu = rho * cs ** 2
        lam = rho * cp ** 2 - 2.0 * mu
        if np.any(rho <= 0) or np.any(mu <= 0) or np.any(3 * lam + 2 * mu <= 0):
            raise ValueError("material is not positive definite")
        self.mat = dict(rho=rho, cp=cp, cs=cs, mu=mu, lam=lam, Zp=rho * cp, Zs=rho * cs)
        return self

    def norm_weights(self):
        """Diagonal of the 3D norm H = H_q x H_r x H_s (Sec. 4.1)."""
        hq, hr, hs = (o["H"] for o in self.ops)
        return hs[:, None, None] * hr[None, :, None] * hq[None, None, :]


def volume_rhs(blk, Q):
    """dQ/dt from eq. gen_hyp_transformed_discrete: D- on the conservative
    stress flux F_xi = M_xi . sigma (eq. split_form rows read as e_xi . sigma_i,
    reading of the garbled transformed flux), D+ on the velocities in the
    non-conservative term B_xi, both scaled by P~ = J^{-1} P (eq.
    transformedEQ, eq. S matrix)."""
    m = blk.mat
    v = Q[0:3]
    S = stress_tensor(Q[3:9])
    M = blk.M
    Jinv = 1.0 / blk.J
    out = np.zeros_like(Q)
    # B terms: u[xi][i] = D+_xi v_i ; G[c][i] = sum_xi M[xi][c] u[xi][i]
    u = [[apply_along(blk.ops[xi]["Dp"], v[i], xi) for i in range(3)] for xi in range(3)]
    G = [[sum(M[xi][c] * u[xi][i] for xi in range(3)) for i in range(3)] for c in range(3)]
    lam, mu = m["lam"], m["mu"]
    div = G[0][0] + G[1][1] + G[2][2]
    out[3] = Jinv * (lam * div + 2.0 * mu * G[0][0])
    out[4] = Jinv * (lam * div + 2.0 * mu * G[1][1])
    out[5] = Jinv * (lam * div + 2.0 * mu * G[2][2])
    out[6] = Jinv * mu * (G[1][0] + G[0][1])
    out[7] = Jinv * mu * (G[2][0] + G[0][2])
    out[8] = Jinv * mu * (G[2][1] + G[1][2])
    # conservative flux: F[xi][i] = sum_c M[xi][c] sigma_{ic}
    rJinv = Jinv / m["rho"]
    for i in range(3):
        acc = 0.0
        for xi in range(3):
            F = sum(M[xi][c] * S[i][c] for c in range(3))
            acc = acc + apply_along(blk.ops[xi]["Dm"], F, xi)
        out[i] = rJinv * acc
    return out


def _face_index(blk, xi, side):
    ax = AXIS[xi]
    n = blk.shape[ax]
    idx = [slice(None)] * 3
    idx[ax] = 0 if side == 0 else n - 1
    return tuple(idx)


def sat_rhs(blk, Q, gamma, variant=SAT_CHARACTERISTIC):
    """Boundary penalties added to dQ/dt on the six faces.

    Characteristic variant (eq. penalty_terms, eq. rotate_back_forth,
    eq. SAT_General and the hat variables eq. data_hat of App. A):
      G_eta = p_eta - gamma q_eta at xi = 0, q_eta - gamma p_eta at xi = 1, so
      G_eta = 1/2 [(1-gamma) Z_eta v_eta + eps (1+gamma) T_eta], eps = -1 / +1.
    The tangential frame (m, l) enters only through the projection onto the
    tangent plane because Z_m = Z_l = Z_s and gamma_m = gamma_l (reading: one
    gamma per face), so no explicit m_0 is needed.
    With P~ = J^{-1} P and kappa = |M_xi| / (J h_xi w_0):
      dv/dt     -= kappa / rho * G
      dsigma/dt -= eps * kappa * C . sym(n (x) G~),   G~ = G_n/Z_p n + G_t/Z_s.
    Traction variant (eq. SAT_free_surface), used on faces with gamma == 1:
      dv/dt     -= eps * kappa / rho * T.
    Penalties of all faces a node belongs to are summed."""
    gamma = [float(g) for g in gamma]
    if len(gamma) != 6 or any(abs(g) > 1 for g in gamma):
        raise ValueError("gamma must hold 6 values in [-1, 1]")
    m = blk.mat
    out = np.zeros_like(Q)
    for f, (xi, side) in enumerate(FACES):
        g = gamma[f]
        eps = -1.0 if side == 0 else 1.0
        ix = _face_index(blk, xi, side)
        Mx = [blk.M[xi][c][ix] for c in range(3)]
        nrm = np.sqrt(Mx[0] ** 2 + Mx[1] ** 2 + Mx[2] ** 2)
        n = [Mx[c] / nrm for c in range(3)]
        J = blk.J[ix]
        hw0 = blk.ops[xi]["H"][0]
        kappa = nrm / (J * hw0)
        rho, lam, mu = m["rho"][ix], m["lam"][ix], m["mu"][ix]
        Zp, Zs = m["Zp"][ix], m["Zs"][ix]
        v = [Q[i][ix] for i in range(3)]
        S = stress_tensor([Q[3 + k][ix] for k in range(6)])
        T = [sum(S[i][c] * n[c] for c in range(3)) for i in range(3)]
        dv = [None] * 3
        ds = None
        if variant == SAT_TRACTION and g == 1.0:
            for i in range(3):
                dv[i] = -eps * kappa / rho * T[i]
        else:
            vn = sum(v[c] * n[c] for c in range(3))
            Tn = sum(T[c] * n[c] for c in range(3))
            vt = [v[c] - vn * n[c] for c in range(3)]
            Tt = [T[c] - Tn * n[c] for c in range(3)]
            Gn = 0.5 * ((1 - g) * Zp * vn + eps * (1 + g) * Tn)
            Gt = [0.5 * ((1 - g) * Zs * vt[c] + eps * (1 + g) * Tt[c]) for c in range(3)]
            G = [Gn * n[c] + Gt[c] for c in range(3)]
            Gtil = [Gn / Zp * n[c] + Gt[c] / Zs for c in range(3)]
            for i in range(3):
                dv[i] = -kappa / rho * G[i]
            s = [n[0] * Gtil[0], n[1] * Gtil[1], n[2] * Gtil[2],
                 n[1] * Gtil[0] + n[0] * Gtil[1],
                 n[2] * Gtil[0] + n[0] * Gtil[2],
                 n[2] * Gtil[1] + n[1] * Gtil[2]]
            tr = s[0] + s[1] + s[2]
            Cs = [lam * tr + 2 * mu * s[0], lam * tr + 2 * mu * s[1], lam * tr + 2 * mu * s[2],
                  mu * s[3], mu * s[4], mu * s[5]]
            ds = [-eps * kappa * c for c in Cs]
        for i in range(3):
            out[i][ix] += dv[i]
        if ds is not None:
            for k in range(6):
                out[3 + k][ix] += ds[k]
    return out


# ---- point moment-tensor source, eq. momententor_pointsource ---------------

def stf(kind, t, f0_or_T, t0=0.0):
    """Source-time functions: Ricker (workload choice) and the paper's
    g(t) = t / T^2 exp(-t / T) for t >= 0 (eq. momententor_pointsource)."""
    t = np.asarray(t, dtype=np.float64)
    if kind == STF_RICKER:
        a = (np.pi * f0_or_T * (t - t0)) ** 2
        return (1.0 - 2.0 * a) * np.exp(-a)
    if kind == STF_EXPT:
        T = f0_or_T
        tt = t - t0
        return np.where(tt >= 0, tt / T ** 2 * np.exp(-tt / T), 0.0)
    raise ValueError("unknown source-time function")


def delta_1d(npts, H, xi, width):
    """One-dimensional discrete delta at reference coordinate xi in [0, 1]
    (reading; the paper defers to Petersson et al. 2016): Lagrange weights over
    the `width` nodes nearest to xi, divided by the norm weight H_i, so that
    sum_i H_i d_i f_i reproduces f(xi) for polynomials of degree < width.
    Returns (first node index, weights)."""
    u = xi * (npts - 1)
    start = int(np.floor(u)) - width // 2 + 1
    start = min(max(start, 0), npts - width)
    nodes = np.arange(start, start + width, dtype=np.float64)
    phi = np.empty(width)
    for a in range(width):
        num = 1.0
        den = 1.0
        for b in range(width):
            if b != a:
                num *= (u - nodes[b])
                den *= (nodes[a] - nodes[b])
        phi[a] = num / den
    return start, phi / H[start:start + width]


def source_stencil(blk, xi3):
    """Tensor-product discrete delta delta_ijk = d_i d_j d_k / J_ijk at the
    reference point xi3 = (xi_q, xi_r, xi_s) (reading).  Width 2(p+1) per axis
    for interior order 2p.  Returns (slices, weights[ks, kr, kq])."""
    width = 2 * (blk.order // 2 + 1)
    if any(x < 0 or x > 1 for x in xi3):
        raise ValueError("source outside the block")
    parts = [delta_1d(blk.npts[a], blk.ops[a]["H"], xi3[a], width) for a in range(3)]
    (sq, dq), (sr, dr), (ss, ds) = parts
    sl = (slice(ss, ss + width), slice(sr, sr + width), slice(sq, sq + width))
    w = ds[:, None, None] * dr[None, :, None] * dq[None, None, :] / blk.J[sl]
    return sl, w


def _interp_map(blk, u):
    """Node coordinates interpolated at u = (u_q, u_r, u_s) in node units:
    tensor product of Lagrange polynomials over the 2(p+1) nodes nearest to u
    per axis (the window of the discrete delta, ``delta_1d``)."""
    width = 2 * (blk.order // 2 + 1)
    bases = []
    for a in range(3):
        n = blk.npts[a]
        start = min(max(int(np.floor(u[a])) - width // 2 + 1, 0), n - width)
        nodes = start + np.arange(width)
        L = np.ones(width)
        for i in range(width):
            for j in range(width):
                if j != i:
                    L[i] *= (u[a] - nodes[j]) / (nodes[i] - nodes[j])
        bases.append((start, L))
    (sq, Lq), (sr, Lr), (ss, Ls) = bases
    sub = blk.xyz[:, ss:ss + width, sr:sr + width, sq:sq + width]
    return np.einsum("ckji,k,j,i->c", sub, Ls, Lr, Lq)


def locate(blk, x):
    """Reference coordinates (q, r, s), each in [0, 1], of the physical point x
    (reading: eq. momententor_pointsource places the source at a physical
    point; between nodes the map is the Lagrange interpolant of the node
    coordinates over the window of the discrete delta).  The root of
    X(u) - x is found by scipy's fsolve from the nearest node; a root outside
    the block raises ValueError."""
    from scipy.optimize import fsolve
    x = np.asarray(x, dtype=np.float64)
    d2 = sum((blk.xyz[c] - x[c]) ** 2 for c in range(3))
    k, j, i = np.unravel_index(np.argmin(d2), d2.shape)
    u0 = np.array([i, j, k], dtype=np.float64)
    u, info, ier, msg = fsolve(lambda u: _interp_map(blk, u) - x, u0, xtol=1e-14, full_output=True)
    if ier != 1 and np.linalg.norm(_interp_map(blk, u) - x) > 1e-11 * np.ptp(blk.xyz):
        raise ValueError("map not inverted: %s" % msg)
    npm1 = np.array(blk.npts, dtype=np.float64) - 1
    if np.any(u < -1e-9) or np.any(u > npm1 + 1e-9):
        raise ValueError("point outside the block")
    return tuple(np.clip(u, 0, npm1) / npm1)


class Source:
    """sigma_dot += M g(t) delta_h (reading: added to the stress rates as
    printed, no stiffness factor)."""

    def __init__(self, blk, xi3, Mvec, kind, f0_or_T, t0=0.0):
        self.sl, self.w = source_stencil(blk, xi3)
        self.M = np.asarray(Mvec, dtype=np.float64)
        self.kind, self.f0, self.t0 = kind, f0_or_T, t0

    def add(self, out, t):
        g = float(stf(self.kind, t, self.f0, self.t0))
        for k in range(6):
            out[3 + k][self.sl] += self.M[k] * g * self.w
        return out


# ---- full RHS, energy, stepping ----------------------------------------------

def rhs(blk, Q, t=0.0, gamma=(0, 0, 0, 0, 0, 0), variant=SAT_CHARACTERISTIC, sources=()):
    """Right-hand side of eq. gen_hyp_transformed_discrete_SAT plus sources."""
    out = volume_rhs(blk, Q) + sat_rhs(blk, Q, gamma, variant)
    for s in sources:
        s.add(out, t)
    return out


def energy(blk, Q):
    """Discrete energy 1/2 <Q, P~^{-1} Q>_H with P~^{-1} = J P^{-1} (reading
    of eq. physical_energy_discrete on a curvilinear grid):
    E = 1/2 sum H_ijk J (rho |v|^2 + sigma^T S sigma), S = C^{-1}."""
    m = blk.mat
    w = blk.norm_weights() * blk.J
    kin = m["rho"] * (Q[0] ** 2 + Q[1] ** 2 + Q[2] ** 2)
    lam, mu = m["lam"], m["mu"]
    sxx, syy, szz, sxy, sxz, syz = Q[3:9]
    tr = sxx + syy + szz
    # isotropic compliance: normal block (1/(2mu)) (I - lam/(3 lam + 2 mu) 11^T), shear 1/mu
    strain = (sxx ** 2 + syy ** 2 + szz ** 2 - lam / (3 * lam + 2 * mu) * tr ** 2) / (2 * mu) \
        + (sxy ** 2 + sxz ** 2 + syz ** 2) / mu
    return 0.5 * float(np.sum(w * (kin + strain)))


def run(blk, Q0, nsteps, dt, gamma, variant=SAT_CHARACTERISTIC, sources=(), receivers=None, t0=0.0):
    """Integrate nsteps LSRK4 steps from Q0.  receivers: int array (nrec, 3)
    of node indices (i, j, k) = (q, r, s); v is recorded after every step.
    Returns (Q, t, traces[nsteps, nrec, 3] or None)."""
    Q = np.array(Q0, dtype=np.float64, copy=True)
    dQ = np.zeros_like(Q)
    t = t0
    f = lambda QQ, tt: rhs(blk, QQ, tt, gamma, variant, sources)
    traces = None
    if receivers is not None:
        rec = np.asarray(receivers, dtype=np.int64).reshape(-1, 3)
        traces = np.zeros((nsteps, rec.shape[0], 3))
    for n in range(nsteps):
        lsrk.step(Q, dQ, t, dt, f)
        t = t0 + (n + 1) * dt
        if traces is not None:
            for c in range(3):
                traces[n, :, c] = Q[c][rec[:, 2], rec[:, 1], rec[:, 0]]
    return Q, t, traces


def rhs_at(blk, Q, nodes, t=0.0, gamma=(0, 0, 0, 0, 0, 0), variant=SAT_CHARACTERISTIC, sources=()):
    """The same right-hand side as ``rhs`` evaluated node by node, for
    spot checks on grids too large for the whole-array form: each node needs
    only the three grid lines through it.  nodes: int array (n, 3) of
    (i, j, k) = (q, r, s) indices.  Returns (n, 9)."""
    nodes = np.asarray(nodes, dtype=np.int64).reshape(-1, 3)
    m = blk.mat
    out = np.zeros((nodes.shape[0], 9))
    sidx = [[3, 6, 7], [6, 4, 8], [7, 8, 5]]
    for n, (i, j, k) in enumerate(nodes):
        node = (k, j, i)
        pos = (i, j, k)  # position along q, r, s
        lines = []
        for xi in range(3):
            sl = [k, j, i]
            sl[AXIS[xi]] = slice(None)
            lines.append(tuple(sl))
        u = [[float(blk.ops[xi]["Dp"][pos[xi]] @ Q[c][lines[xi]]) for c in range(3)] for xi in range(3)]
        G = [[sum(blk.M[xi][c][node] * u[xi][ii] for xi in range(3)) for ii in range(3)] for c in range(3)]
        Jinv = 1.0 / blk.J[node]
        lam, mu, rho = m["lam"][node], m["mu"][node], m["rho"][node]
        div = G[0][0] + G[1][1] + G[2][2]
        r = np.zeros(9)
        r[3] = Jinv * (lam * div + 2 * mu * G[0][0])
        r[4] = Jinv * (lam * div + 2 * mu * G[1][1])
        r[5] = Jinv * (lam * div + 2 * mu * G[2][2])
        r[6] = Jinv * mu * (G[1][0] + G[0][1])
        r[7] = Jinv * mu * (G[2][0] + G[0][2])
        r[8] = Jinv * mu * (G[2][1] + G[1][2])
        for ii in range(3):
            acc = 0.0
            for xi in range(3):
                F = sum(blk.M[xi][c][lines[xi]] * Q[sidx[ii][c]][lines[xi]] for c in range(3))
                acc += float(blk.ops[xi]["Dm"][pos[xi]] @ F)
            r[ii] = Jinv / rho * acc
        out[n] = r
    # boundary penalties (only on face nodes; computed face-wise) and sources
    on_face = [any(p in (0, blk.npts[a] - 1) for a, p in enumerate((i, j, k))) for i, j, k in nodes]
    if any(on_face):
        sat = sat_rhs(blk, Q, gamma, variant)
        for n, (i, j, k) in enumerate(nodes):
            if on_face[n]:
                out[n] += sat[:, k, j, i]
    for s in sources:
        ks, js, is_ = s.sl
        g = float(stf(s.kind, t, s.f0, s.t0))
        for n, (i, j, k) in enumerate(nodes):
            if ks.start <= k < ks.stop and js.start <= j < js.stop and is_.start <= i < is_.stop:
                for c in range(6):
                    out[n, 3 + c] += s.M[c] * g * s.w[k - ks.start, j - js.start, i - is_.start]
    return out
