"""Write the stored oracle trajectories the GPU parity tests compare against.

    python tests/golden/make_golden.py

Calls only the FP64 oracle and the synth input generator.  Output:
  medium_block_clip.npz  -- the 256^2 / 256 views x 512 bins / 100 energies
      workload, Poisson counts (seed of synth.problem("medium")), MOCCA with
      block-diagonal SPC and clipped curvature, lambda = 3e-7, from f = 0:
      maps f after 100 iterations (float32 [3, 256, 256]) and D_TPL every 10
      iterations (float64).
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


def medium_inputs():
    pr = synth.problem("medium")
    X = projector.system_matrix(pr.geom)
    chat = model.counts_model(X @ pr.f_true.reshape(3, -1).T, pr.spec)
    c = synth.poisson_counts(chat, pr.seed)
    return pr, X, c


def main():
    t0 = time.time()
    pr, X, c = medium_inputs()
    cfg = MEDIUM
    st, hist = mocca.mocca(X, c, pr.spec, cfg["lam"], cfg["n_iter"], cfg["precond"], cfg["curvature"],
                           dtpl_every=cfg["every"])
    out = os.path.join(HERE, "medium_block_clip.npz")
    np.savez_compressed(out, f=st.f.reshape(3, pr.geom.n, pr.geom.n).astype(np.float32),
                        dtpl=np.array([h[1] for h in hist]), iters=np.array([h[0] for h in hist]),
                        lam=cfg["lam"], n_iter=cfg["n_iter"])
    print(f"wrote {out} in {time.time() - t0:.0f}s; D_TPL {[f'{h[1]:.4e}' for h in hist]}")


if __name__ == "__main__":
    main()
