"""Training driver for the learned P^(e) initial guess.

Samples come from the method itself: for every seeded training mesh the
library builds a hierarchy with the plain initial guess and 10 projected-CG
energy-minimisation iterations; the sample holds the level-0 features, the
plain initial values and the final P^(e)_0 values (the target).  Training runs
the library's forward, backward and Adam kernels (hcurl_mpnn_train_step).

Default recipe (the learned-guess workload): 200 meshes with N ~ U{24..48}
hexes per side, node jitter ~ U[0, 0.2] h, lognormal sigma with s ~ U[0, 3],
seeds 1000..1199.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def init_params(seed: int, zero_head: bool = False) -> np.ndarray:
    """Glorot-uniform weights (numpy PCG64), zero biases; flat FP32 array in
    the library's parameter order."""
    rng = np.random.default_rng(seed)

    def glorot(a, b):
        lim = np.sqrt(6.0 / (a + b))
        return rng.uniform(-lim, lim, size=(a, b))

    parts = [glorot(16, 64).ravel(), np.zeros(64)]
    for _ in range(3):
        parts += [glorot(192, 64).ravel(), np.zeros(64)]
    w_out = np.zeros(64) if zero_head else glorot(64, 1)[:, 0] * 0.1
    parts += [w_out, np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def mesh_specs(n: int, seed0: int = 1000, nmin: int = 24, nmax: int = 48):
    rng = np.random.default_rng(seed0)
    out = []
    for k in range(n):
        out.append(dict(N=int(rng.integers(nmin, nmax + 1)), jitter=float(rng.uniform(0.0, 0.2)),
                        jitter_seed=seed0 + 2 * k, sigma=("lognormal", seed0 + 2 * k + 1, float(rng.uniform(0.0, 3.0))),
                        f_seed=seed0 + k))
    return out


def build_sample(spec, stream=None):
    import synth
    import paper_2506_08284_amd as P
    pr = synth.problem(**spec)
    m = pr["mesh"]["n"] ** 3
    H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), pr["aggregates"], n_nodes=m,
                    coords=pr["coords"], stream=stream)
    s = H.mpnn_sample()
    H.close()
    return s


def train(net, samples, steps: int, lr: float = 1e-3, seed: int = 0, log_every: int = 0, lr_final: float | None = None):
    import paper_2506_08284_amd as P
    rng = np.random.default_rng(seed)
    losses = []
    for step in range(1, steps + 1):
        s = samples[int(rng.integers(len(samples)))]
        lr_t = lr if lr_final is None else lr * (lr_final / lr) ** ((step - 1) / max(1, steps - 1))
        losses.append(P.hcurl_mpnn_train_step(net.h, s, lr_t, step))
        if log_every and step % log_every == 0:
            print("step %d loss %.3e" % (step, np.mean(losses[-log_every:])), flush=True)
    return losses


def evaluate(net, spec, stream=None, emin_plain: int = 10, emin_learned: int = 3):
    """Plain start + emin_plain CG iterations against the learned start +
    emin_learned: final level-0 energy, PCG iterations and setup seconds."""
    import synth
    import paper_2506_08284_amd as P
    pr = synth.problem(**spec)
    m = pr["mesh"]["n"] ** 3
    n = pr["A"][0].shape[0] - 1
    out = {}
    for name, opts in (("plain", dict(emin_iters=emin_plain)),
                       ("plain_short", dict(emin_iters=emin_learned)),
                       ("learned", dict(init_guess=2, mpnn=net, emin_iters_given=emin_learned))):
        t0 = time.time()
        H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), pr["aggregates"], n_nodes=m,
                        coords=pr["coords"], record_energy=1, stream=stream, **opts)
        t1 = time.time()
        E = H.export_vec(0, "energy")
        it, rel, rc = H.solve(pr["f"], np.empty(n))
        out[name] = dict(energy=float(E[-1]), energy_start=float(E[0]), iters=it, relres=rel, setup_s=t1 - t0)
        H.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--meshes", type=int, default=200)
    ap.add_argument("--nmin", type=int, default=24)
    ap.add_argument("--nmax", type=int, default=48)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default="mpnn_weights.npy")
    ap.add_argument("--eval-n", type=int, default=0, help="evaluate on an N^3 held-out mesh after training")
    args = ap.parse_args()
    import paper_2506_08284_amd as P
    t0 = time.time()
    samples = []
    for k, spec in enumerate(mesh_specs(args.meshes, nmin=args.nmin, nmax=args.nmax)):
        samples.append(build_sample(spec))
        if (k + 1) % 20 == 0:
            print("built %d samples (%.0f s)" % (k + 1, time.time() - t0), flush=True)
    net = P.Network(init_params(7))
    losses = train(net, samples, args.steps, args.lr, log_every=100, lr_final=args.lr * 0.1)
    np.save(args.out, net.params())
    print("trained %d steps in %.0f s, final loss %.3e" % (args.steps, time.time() - t0, np.mean(losses[-100:])),
          flush=True)
    for s in samples:
        P.hcurl_mpnn_sample_destroy(s)
    if args.eval_n:
        spec = dict(N=args.eval_n, jitter=0.1, jitter_seed=404, sigma=("lognormal", 405, 2.0), f_seed=104)
        res = evaluate(net, spec)
        for k, v in res.items():
            print("eval %d^3 %-12s energy %.6g (from %.6g)  PCG its %d relres %.1e  setup %.2f s" % (
                args.eval_n, k, v["energy"], v["energy_start"], v["iters"], v["relres"], v["setup_s"]), flush=True)


if __name__ == "__main__":
    main()
