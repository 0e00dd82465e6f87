"""Writes the stored expected values of the full-size topography benchmark
workload: 257 x 257 x 193 nodes, interior order 6, curvilinear block under
the seeded topography, 1 km layer over a half-space, Ricker moment source,
64 surface receivers, free surface on top and absorbing faces elsewhere,
100 LSRK4 steps at CFL 0.5 from rest.

Only the CPU oracle (``oracle/``) and the seeded input generators
(``workloads``) are called.  The result file holds, after 100 steps:

* ``traces``        (100, 64, 3)  v at the receivers after every step;
* ``nodes``         (n, 3)        sample nodes (i, j, k) = (q, r, s);
* ``values``        (n, 9)        the 9 fields at the sample nodes;
* ``field_l2``      (9,)          L2 norm of each whole field;
* ``field_absmax``  (9,)          largest magnitude of each whole field;
* ``meta``                        grid, order, steps, dt, seeds (JSON text).

Sample nodes (seeded): the whole source support, the receivers, every node
of the 12 edges' first two layers at a seeded subset of positions, the 8
corners, nodes of the closure layers next to each of the 6 faces, nodes on
each face, and interior nodes, about 12 000 in all.

    python tests/golden/make_topo_layer_golden.py [--steps 100] [--out FILE]

Takes about half an hour on 8 cores (numpy with threaded BLAS).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import elastic as E  # noqa: E402
from oracle import lsrk  # noqa: E402

DEFAULT_OUT = os.path.join(HERE, "topo_layer_257x257x193_o6_100steps.npz")


def sample_nodes(shape, src_sl, receivers, seed=7):
    """Seeded sample nodes, (i, j, k) rows, without repeats."""
    ns, nr, nq = shape
    rng = np.random.default_rng(seed)
    pts = []
    ks, js, is_ = src_sl
    for k in range(ks.start, ks.stop):
        for j in range(js.start, js.stop):
            for i in range(is_.start, is_.stop):
                pts.append((i, j, k))
    pts += [tuple(int(x) for x in r) for r in receivers]
    N = (nq, nr, ns)
    # corners
    for c in range(8):
        pts.append(tuple((N[a] - 1) if (c >> a) & 1 else 0 for a in range(3)))
    # edges: two axes pinned at 0/1 or n-2/n-1, the third axis random
    for ax in range(3):
        o1, o2 = [a for a in range(3) if a != ax]
        for p1 in (0, 1, N[o1] - 2, N[o1] - 1):
            for p2 in (0, 1, N[o2] - 2, N[o2] - 1):
                for t in rng.integers(0, N[ax], size=12):
                    p = [0, 0, 0]
                    p[ax], p[o1], p[o2] = int(t), p1, p2
                    pts.append(tuple(p))
    # closure layers (distance 0..6 from each face) and faces
    for ax in range(3):
        for side in (0, 1):
            for d in range(7):
                cnt = 150 if d == 0 else 60
                for _ in range(cnt):
                    p = [int(rng.integers(0, N[a])) for a in range(3)]
                    p[ax] = d if side == 0 else N[ax] - 1 - d
                    pts.append(tuple(p))
    # interior
    for _ in range(4000):
        pts.append(tuple(int(rng.integers(0, N[a])) for a in range(3)))
    # a box of nodes around the source support (where the field is largest)
    cq, cr, cs = (is_.start + is_.stop) // 2, (js.start + js.stop) // 2, (ks.start + ks.stop) // 2
    for _ in range(2000):
        p = (int(np.clip(cq + rng.integers(-40, 41), 0, nq - 1)),
             int(np.clip(cr + rng.integers(-40, 41), 0, nr - 1)),
             int(np.clip(cs + rng.integers(-40, 41), 0, ns - 1)))
        pts.append(p)
    seen = set()
    out = []
    for p in pts:
        if p not in seen:
            seen.add(p)
            out.append(p)
    return np.array(out, dtype=np.int32)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--nq", type=int, default=257)
    ap.add_argument("--nr", type=int, default=257)
    ap.add_argument("--ns", type=int, default=193)
    args = ap.parse_args()
    wl = W.topo_layer(nq=args.nq, nr=args.nr, ns=args.ns)
    order = wl["order"]
    t0 = time.time()
    blk = E.Block(wl["xyz"], order).set_material(wl["rho"], wl["cp"], wl["cs"])
    src = E.Source(blk, wl["src_xi"], wl["src_M"], E.STF_RICKER, wl["src_f0"], wl["src_t0"])
    print("set-up %.1f s" % (time.time() - t0), flush=True)
    rec = np.asarray(wl["receivers"], dtype=np.int64)
    Q = np.array(wl["Q0"], dtype=np.float64)
    dQ = np.zeros_like(Q)
    dt = wl["dt"]
    traces = np.zeros((args.steps, rec.shape[0], 3))
    f = lambda QQ, tt: E.rhs(blk, QQ, tt, wl["gamma"], E.SAT_CHARACTERISTIC, [src])
    for n in range(args.steps):
        lsrk.step(Q, dQ, n * dt, dt, f)
        for c in range(3):
            traces[n, :, c] = Q[c][rec[:, 2], rec[:, 1], rec[:, 0]]
        print("step %d/%d  %.0f s" % (n + 1, args.steps, time.time() - t0), flush=True)
    nodes = sample_nodes(Q.shape[1:], src.sl, rec)
    values = np.stack([Q[f][nodes[:, 2], nodes[:, 1], nodes[:, 0]] for f in range(9)], axis=1)
    meta = dict(grid=[args.nq, args.nr, args.ns], order=order, steps=args.steps, dt=dt, cfl=0.5,
                workload="topo_layer(seed=0)", sample_seed=7,
                note="written by tests/golden/make_topo_layer_golden.py from oracle/ only")
    np.savez_compressed(args.out, traces=traces, nodes=nodes, values=values,
                        field_l2=np.array([np.linalg.norm(Q[f]) for f in range(9)]),
                        field_absmax=np.array([np.abs(Q[f]).max() for f in range(9)]),
                        meta=np.array(json.dumps(meta)))
    print("wrote %s (%d sample nodes) in %.0f s" % (args.out, nodes.shape[0], time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
