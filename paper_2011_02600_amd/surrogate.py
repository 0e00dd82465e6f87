"""Surrogate pipeline: training data from the solver, training of the
spectral neural operator (nn.SpectralOperator), and prediction with a
fallback to the solver.

The solver produces every sample: for a material perturbation field d on an
n^3 grid (cp and cs scaled by 1 + d, rho fixed), sbp_step_batch runs the
shots and the receivers record v_z after every step.  An ensemble of
networks (same data, different initialisations and sample orders) maps d
(scaled to unit amplitude) to the normalised traces; the prediction is
their mean.  The fallback score of a sample is a predicted error: the
relative spread of the ensemble's predictions.  A sample is answered by the
ensemble when its score lies at or below a threshold calibrated on held-out
training samples so that the accepted ones stay within the error budget;
otherwise the solver runs.  Orchestration only: the solver and the
networks run in the HIP library.
"""
import time

import numpy as np


def solve_batch(sbp, torch, case, fields, dev, nmax=64, log=None):
    """Traces v_z (len(fields), R, T) for the media of `fields` (host float64
    arrays (n, n, n)), by sbp_step_batch over groups of up to nmax shots.
    Returns (traces tensor on dev, solver seconds: the stepping alone)."""
    n, T = case["n"], case["T"]
    rec = case["receivers"]
    out = torch.empty((len(fields), len(rec), T), dtype=torch.float32, device=dev)
    zero = torch.zeros((9, n, n, n), dtype=torch.float32, device=dev)
    solvers = []
    secs = 0.0
    for g0 in range(0, len(fields), nmax):
        grp = fields[g0:g0 + nmax]
        t0 = time.perf_counter()
        while len(solvers) < len(grp):
            s = sbp.Solver(case["xyz"], order=case["order"], dtype="f32", gamma=case["gamma"], device=dev)
            s.add_source(case["src_xi"], case["src_M"], sbp.SBP_STF_RICKER, case["src_f0"], case["src_t0"])
            solvers.append(s)
            if log and len(solvers) % 16 == 0:
                log("surrogate: %d solvers ready (%.1f s)" % (len(solvers), time.perf_counter() - t0))
        t1 = time.perf_counter()
        for s, d in zip(solvers, grp):
            s.set_material(case["rho"], case["cp"] * (1 + d), case["cs"] * (1 + d))
            s.set_state(zero, 0.0)
            s.record(rec, T)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        sbp.sbp_step_batch([s.h for s in solvers[:len(grp)]], T, [case["dt"]] * len(grp))
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        secs += t3 - t2
        for i, s in enumerate(solvers[:len(grp)]):
            out[g0 + i] = s.traces[:, :, 2].transpose(0, 1)
        if log:
            log("surrogate: shots %d-%d: set-up %.2f s, media %.2f s, stepping %.2f s"
                % (g0, g0 + len(grp) - 1, t1 - t0, t2 - t1, t3 - t2))
    for s in solvers:
        s.close()
    return out, secs


class Surrogate:
    """An ensemble of spectral operators + normalisation + fallback
    threshold on the ensemble's spread."""

    def __init__(self, nn, torch, case, dev, modes=8, width=32, layers=4, seed=0, members=2):
        self.torch, self.case, self.dev = torch, case, dev
        n = case["n"]
        pos = [k * n * n + j * n + i for (i, j, k) in case["receivers"]]
        self.nets = [nn.SpectralOperator(n, modes, width, layers, pos, case["T"], device=dev, seed=seed + 101 * e)
                     for e in range(members)]
        self.net = self.nets[0]
        self.xscale = 1.0 / case["amp"]
        self.yscale = 1.0
        self.ymean = 0.0
        self.tau = -np.inf

    def _x(self, d):
        return d * self.xscale

    def train(self, d, y, epochs=20, batch=8, lr=2e-3, log=None):
        """d: (N, n, n, n) device tensor of perturbations; y: (N, R, T) traces.
        Every member sees every sample each epoch, in its own order."""
        torch = self.torch
        N = d.shape[0]
        # the networks predict the deviation from the mean training trace
        self.ymean = y.mean(dim=0)
        self.yscale = float((y - self.ymean).std())
        yn = (y - self.ymean) / self.yscale
        steps = epochs * (N // batch)
        hist = []
        for e, net in enumerate(self.nets):
            rng = np.random.default_rng(1000 + e)
            k = 0
            for ep in range(epochs):
                order = rng.permutation(N)
                tot = 0.0
                for b0 in range(0, N - batch + 1, batch):
                    idx = torch.tensor(order[b0:b0 + batch], device=self.dev)
                    x = self._x(d[idx]).contiguous()
                    t = yn[idx].contiguous()
                    out = net.forward(x)
                    loss, dy = net.loss(out, t, scale=1.0 / batch)
                    net.backward(dy)
                    # cosine learning-rate decay
                    net.adam_step(lr * 0.5 * (1 + np.cos(np.pi * k / steps)))
                    tot += loss
                    k += 1
                if e == 0:
                    hist.append(tot / (N // batch))
                if log:
                    log("surrogate: member %d epoch %d loss %.5f" % (e, ep, tot / (N // batch)))
        return hist

    def _members(self, d, batch=8):
        """Each member's denormalised prediction: (members, N, R, T)."""
        torch = self.torch
        outs = []
        for net in self.nets:
            parts = []
            for b0 in range(0, d.shape[0], batch):
                x = self._x(d[b0:b0 + batch]).contiguous()
                parts.append(net.forward(x).clone())
            outs.append(torch.cat(parts) * self.yscale + self.ymean)
        return torch.stack(outs)

    def predict_with_score(self, d, batch=8):
        """(ensemble mean prediction, fallback score per sample): the score is
        the relative L2 spread of the members around their mean."""
        p = self._members(d, batch)
        mean = p.mean(dim=0)
        spread = ((p - mean) ** 2).sum(dim=(2, 3)).mean(dim=0).sqrt()
        score = (spread / (mean ** 2).sum(dim=(1, 2)).sqrt()).double().cpu().numpy()
        return mean, score

    def predict(self, d, batch=8):
        return self.predict_with_score(d, batch)[0]

    @staticmethod
    def rel_err(pred, true):
        num = ((pred - true) ** 2).sum(dim=(1, 2)).sqrt()
        return (num / (true ** 2).sum(dim=(1, 2)).sqrt()).double().cpu().numpy()

    @staticmethod
    def threshold(err, sc, budget=0.05, quantile=0.95):
        """Largest score threshold whose accepted samples (score <= threshold)
        keep the `quantile` of their relative errors within `budget`; -inf if
        none does."""
        order = np.argsort(sc)
        tau = -np.inf
        for i in range(1, len(order) + 1):
            if np.quantile(err[order[:i]], quantile) <= budget:
                tau = sc[order[i - 1]]
        return tau

    def calibrate(self, d_val, y_val, budget=0.05, quantile=0.95):
        """Sets the threshold from validation samples (see threshold);
        returns their errors and scores."""
        pred, sc = self.predict_with_score(d_val)
        err = self.rel_err(pred, y_val)
        self.tau = self.threshold(err, sc, budget, quantile)
        return err, sc
