"""Write the stored oracle trajectories the GPU parity tests compare against.

    python tests/golden/make_golden.py [medium] [large]

Calls only the FP64 oracle and the synth input generator.  Outputs:
  medium_block_clip.npz  -- the 256^2 / 256 views x 512 bins / 100 energies
      workload, Poisson counts (seed of synth.problem("medium")), MOCCA with
      block-diagonal SPC and clipped curvature, lambda = 3e-7, from f = 0:
      maps f after 100 iterations (float32 [3, 256, 256]) and D_TPL every 10
      iterations (float64).
  large_block_clip.npz   -- the 512^2 / 720 views x 1024 bins / 120 energies
      workload (the benchmark's scan), Poisson counts from the oracle's
      counts model at the phantom (seed of synth.problem("large")), MOCCA with
      block-diagonal SPC and clipped curvature, lambda = 2e-8, from f = 0:
      the counts themselves (int32 [4, 720, 1024]: building the oracle's X for
      this scan takes minutes, too long for a GPU test), maps f after 100
      iterations (float32 [3, 512, 512]) and D_TPL every 10 iterations.  About
      15 minutes and 30 GB of host memory on one core.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import model, mocca, projector  # noqa: E402

MEDIUM = dict(name="medium", lam=3e-7, precond="block", curvature="clip", n_iter=100, every=10)
LARGE = dict(name="large", lam=2e-8, precond="block", curvature="clip", n_iter=100, every=10)


def workload_inputs(name):
    pr = synth.problem(name)
    X = projector.system_matrix(pr.geom)
    chat = model.counts_model(X @ pr.f_true.reshape(3, -1).T, pr.spec)
    c = synth.poisson_counts(chat, pr.seed)
    return pr, X, c


def medium_inputs():
    return workload_inputs("medium")


def run(cfg, store_counts):
    t0 = time.time()
    pr, X, c = workload_inputs(cfg["name"])
    print(f"{cfg['name']}: X built ({X.nnz} nonzeros) in {time.time() - t0:.0f}s", flush=True)

    def progress(it, st):
        if (it + 1) % 10 == 0:
            print(f"  iteration {it + 1} at {time.time() - t0:.0f}s", flush=True)

    st, hist = mocca.mocca(X, c, pr.spec, cfg["lam"], cfg["n_iter"], cfg["precond"], cfg["curvature"],
                           dtpl_every=cfg["every"], callback=progress)
    g = pr.geom
    extra = {}
    if store_counts:
        assert c.max() < 2 ** 31
        extra["counts"] = c.T.reshape(4, g.n_views, g.n_bins).astype(np.int32)
    out = os.path.join(HERE, f"{cfg['name']}_block_clip.npz")
    np.savez_compressed(out, f=st.f.reshape(3, g.n, g.n).astype(np.float32),
                        dtpl=np.array([h[1] for h in hist]), iters=np.array([h[0] for h in hist]),
                        lam=cfg["lam"], n_iter=cfg["n_iter"], **extra)
    print(f"wrote {out} in {time.time() - t0:.0f}s; D_TPL {[f'{h[1]:.4e}' for h in hist]}", flush=True)


def main(argv):
    names = argv or ["medium"]
    for name in names:
        if name == "medium":
            run(MEDIUM, store_counts=False)
        elif name == "large":
            run(LARGE, store_counts=True)
        else:
            raise SystemExit(f"unknown workload {name}")


if __name__ == "__main__":
    main(sys.argv[1:])
