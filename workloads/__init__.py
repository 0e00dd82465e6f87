"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark: meshes, media, initial states, source and receiver placement.

This module holds none of the method's arithmetic (no operators, metrics,
penalties or time stepping); it only produces the data a user would hand to
the solver.  Both the CPU oracle and the HIP library are fed from here.

Workloads (stand-ins for the paper's LOH1 and Zugspitze runs, whose data are
not available):

* ``cube_pulse``  Cartesian unit cube, homogeneous rho=2.7, cp=6.0, cs=3.464
  (the Zugspitze medium of Sec. 7.2), free surface on top (s = 1), absorbing
  elsewhere, Gaussian velocity pulse (sigma = 0.1, seed-placed centre),
  LSRK4 at CFL 0.5.
* ``topo_layer``  curvilinear block under a free-surface topography
  z_top = 0.1 sin(2 pi x / L) cos(2 pi y / L) + seeded Gaussian hills
  (each at most 5 % of the depth), transfinite mesh, a 1 km low-velocity
  layer over a half-space (LOH1-like, Sec. 7.1), a point moment-tensor
  source with a Ricker wavelet and 64 surface receivers.
* ``batched_shots``  32 independent cubes of uneven size (65^3 .. 193^3),
  orders 4 and 6 alternating, FP32, each over its own Gaussian-random-field
  medium (correlation length 10 cells, at most +-10 % around the half-space
  values), a Ricker moment source and 16 surface receivers.

Array convention: grid functions have shape (ns, nr, nq), q fastest; node
coordinates are returned as xyz with shape (3, ns, nr, nq).
"""
import numpy as np

FACE_NAMES = ("q0", "q1", "r0", "r1", "s0", "s1")


def unit_cube(nq, nr, ns):
    """Node coordinates of the uniformly meshed unit cube (identity map)."""
    q = np.linspace(0.0, 1.0, nq)
    r = np.linspace(0.0, 1.0, nr)
    s = np.linspace(0.0, 1.0, ns)
    S, R, Qg = np.meshgrid(s, r, q, indexing="ij")
    return np.stack([Qg, R, S])


def gaussian_pulse(xyz, seed, width=0.1, lo=0.3, hi=0.7):
    """Velocity pulse v = d exp(-|x - x_c|^2 / (2 width^2)), stresses zero.
    x_c ~ U[lo, hi]^3 and d = normalised N(0, I_3), both from `seed`."""
    rng = np.random.default_rng(seed)
    xc = rng.uniform(lo, hi, size=3)
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    r2 = sum((xyz[c] - xc[c]) ** 2 for c in range(3))
    g = np.exp(-r2 / (2 * width ** 2))
    Q = np.zeros((9,) + xyz.shape[1:])
    for c in range(3):
        Q[c] = d[c] * g
    return Q


def cfl_dt(xyz, cp, cfl):
    """dt = cfl * h_min / max(cp), h_min the smallest physical distance between
    grid-adjacent nodes."""
    hmin = np.inf
    for ax in range(3):
        dx = np.diff(xyz, axis=ax + 1)
        hmin = min(hmin, float(np.sqrt((dx ** 2).sum(axis=0)).min()))
    return cfl * hmin / float(np.max(cp))


def cube_pulse(n=21, seed=0, cfl=0.5):
    """Cartesian unit cube n^3, homogeneous medium, Gaussian pulse."""
    xyz = unit_cube(n, n, n)
    shape = xyz.shape[1:]
    rho = np.full(shape, 2.7)
    cp = np.full(shape, 6.0)
    cs = np.full(shape, 3.464)
    Q0 = gaussian_pulse(xyz, seed)
    return dict(xyz=xyz, rho=rho, cp=cp, cs=cs, Q0=Q0, gamma=(0.0, 0.0, 0.0, 0.0, 0.0, 1.0),
                dt=cfl_dt(xyz, cp, cfl), order=4)


def _topography(L, D, seed, nhills=8):
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.0, 0.05 * D, size=nhills)
    cen = rng.uniform(0.0, L, size=(nhills, 2))
    wid = rng.uniform(0.5, 2.0, size=nhills)

    def ztop(x, y):
        z = 0.1 * np.sin(2 * np.pi * x / L) * np.cos(2 * np.pi * y / L)
        for a, (cx, cy), w in zip(amp, cen, wid):
            z = z + a * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * w ** 2))
        return z
    return ztop


def topo_mesh(nq, nr, ns, seed=0, L=12.8, D=9.6):
    """Transfinite mesh x = xi L, y = eta L, z = -D + zeta (z_top(x, y) + D).
    Returns (xyz, ztop callable)."""
    ztop = _topography(L, D, seed)
    q = np.linspace(0.0, 1.0, nq)
    r = np.linspace(0.0, 1.0, nr)
    s = np.linspace(0.0, 1.0, ns)
    S, R, Qg = np.meshgrid(s, r, q, indexing="ij")
    x = Qg * L
    y = R * L
    zt = ztop(x, y)
    z = -D + S * (zt + D)
    return np.stack([x, y, z]), ztop


def layered_medium(xyz, ztop, layer=1.0):
    """1 km soft layer (cs 2.0, cp 4.0, rho 2.6) over a half-space
    (cs 3.464, cp 6.0, rho 2.7), point-sampled at the nodes."""
    depth = ztop(xyz[0], xyz[1]) - xyz[2]
    soft = depth <= layer
    rho = np.where(soft, 2.6, 2.7)
    cp = np.where(soft, 4.0, 6.0)
    cs = np.where(soft, 2.0, 3.464)
    return rho, cp, cs


def topo_layer(nq=257, nr=257, ns=193, seed=0, cfl=0.5, L=12.8, D=9.6, src_depth=2.0,
               f0=2.0, nrec_side=8):
    """Curvilinear layered workload (order 6).  Sizes default to 257 x 257 x 193
    (q, r, s).  The source sits at (L/2, L/2) +- a seeded 1 km horizontal
    offset, src_depth below the local surface, with a strike-slip moment
    M = (0, 0, 0, 1, 0, 0) (sxy) and a Ricker wavelet f0, t0 = 1.2 / f0.
    Receivers: nrec_side^2 surface nodes evenly spread over the top face."""
    xyz, ztop = topo_mesh(nq, nr, ns, seed, L, D)
    rho, cp, cs = layered_medium(xyz, ztop)
    rng = np.random.default_rng(seed + 1)
    off = rng.uniform(-1.0, 1.0, size=2)
    xs, ys = L / 2 + off[0], L / 2 + off[1]
    zt = float(ztop(np.array(xs), np.array(ys)))
    zs = zt - src_depth
    # the transfinite map is invertible in closed form
    src_xi = (xs / L, ys / L, (zs + D) / (zt + D))
    step_q = (nq - 1) / nrec_side
    step_r = (nr - 1) / nrec_side
    rec = [(int(round(step_q * (a + 0.5))), int(round(step_r * (b + 0.5))), ns - 1)
           for b in range(nrec_side) for a in range(nrec_side)]
    Q0 = np.zeros((9, ns, nr, nq))
    return dict(xyz=xyz, rho=rho, cp=cp, cs=cs, Q0=Q0, gamma=(0.0, 0.0, 0.0, 0.0, 0.0, 1.0),
                dt=cfl_dt(xyz, cp, cfl), order=6, src_xi=src_xi,
                src_M=(0.0, 0.0, 0.0, 1.0, 0.0, 0.0), src_f0=f0, src_t0=1.2 / f0,
                receivers=np.array(rec, dtype=np.int32))


def random_state(shape, seed, smooth=False):
    """Seeded random 9-field state; smooth=True gives a low-wavenumber field
    (sum of a few random sinusoids) for tests that need bounded derivatives."""
    rng = np.random.default_rng(seed)
    if not smooth:
        return rng.standard_normal((9,) + tuple(shape))
    ns, nr, nq = shape
    q = np.linspace(0, 1, nq)
    r = np.linspace(0, 1, nr)
    s = np.linspace(0, 1, ns)
    Q = np.zeros((9,) + tuple(shape))
    for f in range(9):
        for _ in range(3):
            k = rng.uniform(0.5, 3.0, size=3)
            ph = rng.uniform(0, 2 * np.pi, size=3)
            a = rng.standard_normal()
            cq = np.cos(2 * np.pi * k[0] * q + ph[0])
            cr = np.cos(2 * np.pi * k[1] * r + ph[1])
            cs = np.cos(2 * np.pi * k[2] * s + ph[2])
            Q[f] += a * cs[:, None, None] * cr[None, :, None] * cq[None, None, :]
    return Q


def random_medium(shape, seed, rho=(2.0, 3.0), cs=(1.5, 3.5), ratio=(1.6, 2.0)):
    """Seeded heterogeneous medium with cp = ratio * cs (positive definite)."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(*rho, size=shape)
    s = rng.uniform(*cs, size=shape)
    p = s * rng.uniform(*ratio, size=shape)
    return r, p, s


def warped_mesh(nq, nr, ns, seed, amp=0.04):
    """Smooth seeded curvilinear map of the unit cube (for tests): every
    coordinate is perturbed by a product of low-wavenumber sines that vanish
    nowhere in particular; small enough that the Jacobian stays positive."""
    rng = np.random.default_rng(seed)
    X = unit_cube(nq, nr, ns)
    q, r, s = X[0], X[1], X[2]
    out = X.copy()
    for c in range(3):
        ph = rng.uniform(0, 2 * np.pi, size=3)
        a = amp * rng.uniform(0.5, 1.0)
        out[c] = X[c] + a * np.sin(2 * np.pi * q + ph[0]) * np.sin(2 * np.pi * r + ph[1]) \
            * np.sin(2 * np.pi * s + ph[2])
    return out


def grf(shape, corr_cells, seed, amp=0.1):
    """Gaussian random field: white noise filtered in Fourier space by
    exp(-|k|^2 l^2 / 2), l = corr_cells grid spacings, scaled so that its
    largest magnitude is `amp`."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    k = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(n) for n in shape], indexing="ij", sparse=True)
    k2 = sum(kk ** 2 for kk in k)
    f = np.fft.ifftn(np.fft.fftn(w) * np.exp(-0.5 * k2 * corr_cells ** 2)).real
    return amp * f / np.abs(f).max()


def batched_shots(nshots=32, seed=0, h=0.05, cfl=0.5, corr_cells=10, amp=0.1, f0=4.0, nrec_side=4):
    """Independent shots for batched stepping: cube i has n_i points per axis,
    n_i drawn from {65, 69, ..., 193} with `seed`, interior order 4 for even i
    and 6 for odd i, spacing h (km).  Medium: the half-space values
    (cs 3.464, cp 6.0, rho 2.7) times 1 + delta, one random field (grf) for
    cp and cs together (their ratio stays fixed) and one for rho.  Free
    surface on top, absorbing elsewhere; a Ricker moment source (M = sxy,
    f0, t0 = 1.2 / f0) at a seeded point of the central region; nrec_side^2
    receivers on the top face."""
    rng = np.random.default_rng(seed)
    sizes = 65 + 4 * rng.integers(0, 33, size=nshots)
    shots = []
    for i, n in enumerate(sizes):
        n = int(n)
        xyz = unit_cube(n, n, n) * (h * (n - 1))
        shape = (n, n, n)
        dv = grf(shape, corr_cells, 1000 * seed + 2 * i, amp)
        dr = grf(shape, corr_cells, 1000 * seed + 2 * i + 1, amp)
        cs = 3.464 * (1 + dv)
        cp = 6.0 * (1 + dv)
        rho = 2.7 * (1 + dr)
        src = tuple(rng.uniform(0.35, 0.65, size=3))
        step = (n - 1) / nrec_side
        rec = [(int(round(step * (a + 0.5))), int(round(step * (b + 0.5))), n - 1)
               for b in range(nrec_side) for a in range(nrec_side)]
        shots.append(dict(xyz=xyz, rho=rho, cp=cp, cs=cs, order=4 if i % 2 == 0 else 6,
                          gamma=(0.0, 0.0, 0.0, 0.0, 0.0, 1.0), dt=cfl_dt(xyz, cp, cfl),
                          src_xi=src, src_M=(0.0, 0.0, 0.0, 1.0, 0.0, 0.0), src_f0=f0, src_t0=1.2 / f0,
                          receivers=np.array(rec, dtype=np.int32)))
    return shots


def adjoint_case(n=129, seed=0, amp=0.05, corr_cells=10, cfl=0.5, nrec_side=8):
    """Material-gradient workload: the topo_layer block at n^3 points (order
    6), a model and a target model that are the layered medium times 1 + d,
    with separate smooth seeded perturbations d (grf, max |d| = amp) of rho,
    lambda and mu in each; nrec_side^2 surface receivers, the Ricker moment
    source of topo_layer, zero initial state.  dt from the larger cp of the
    two models.  Returns the topo_layer dict with model=(rho, cp, cs) and
    target=(rho, cp, cs)."""
    wl = topo_layer(nq=n, nr=n, ns=n, seed=seed, cfl=cfl, nrec_side=nrec_side)
    rho0, cp0, cs0 = wl["rho"], wl["cp"], wl["cs"]
    mu0 = rho0 * cs0 ** 2
    lam0 = rho0 * cp0 ** 2 - 2 * mu0
    shape = rho0.shape

    def perturbed(s):
        rho = rho0 * (1 + grf(shape, corr_cells, s, amp))
        lam = lam0 * (1 + grf(shape, corr_cells, s + 1, amp))
        mu = mu0 * (1 + grf(shape, corr_cells, s + 2, amp))
        return rho, np.sqrt((lam + 2 * mu) / rho), np.sqrt(mu / rho)

    model = perturbed(1000 * seed + 11)
    target = perturbed(1000 * seed + 21)
    wl.update(model=model, target=target, dt=cfl_dt(wl["xyz"], np.maximum(model[1], target[1]), cfl))
    return wl


def surrogate_case(n=64, h=0.05, T=512, amp=0.02, corr_cells=16, f0=6.0, cfl=0.5, nrec_side=8, order=4):
    """Fixed geometry of the surrogate workload: an n^3 cube with spacing h
    (km), half-space background (cs 3.464, cp 6.0, rho 2.7), free surface on
    top and absorbing elsewhere, a Ricker moment source (M = sxy, f0) at
    reference point (0.5, 0.5, 0.4), nrec_side^2 receivers on the top face,
    T steps at the dt of CFL `cfl` for the fastest medium the perturbations
    allow (cp (1 + amp)).  Perturbations come from surrogate_fields."""
    xyz = unit_cube(n, n, n) * (h * (n - 1))
    shape = (n, n, n)
    cp = np.full(shape, 6.0)
    cs = np.full(shape, 3.464)
    rho = np.full(shape, 2.7)
    step = (n - 1) / nrec_side
    rec = [(int(round(step * (a + 0.5))), int(round(step * (b + 0.5))), n - 1)
           for b in range(nrec_side) for a in range(nrec_side)]
    return dict(n=n, xyz=xyz, rho=rho, cp=cp, cs=cs, order=order, gamma=(0.0, 0.0, 0.0, 0.0, 0.0, 1.0),
                dt=cfl_dt(xyz, cp * (1 + amp), cfl), T=T, amp=amp, corr_cells=corr_cells,
                src_xi=(0.5, 0.5, 0.4), src_M=(0.0, 0.0, 0.0, 1.0, 0.0, 0.0), src_f0=f0, src_t0=1.2 / f0,
                receivers=np.array(rec, dtype=np.int32))


def surrogate_fields(case, count, seed):
    """`count` seeded perturbation fields d (grf, max |d| = amp each)."""
    n = case["n"]
    return [grf((n, n, n), case["corr_cells"], 100000 * seed + i, case["amp"]) for i in range(count)]
