"""Small seeded problems shared by the tests (inputs only, no method arithmetic)."""
import numpy as np

import synth


def micro_problem(n=16, views=16, bins=32, e_step=5, i0=1e5):
    """16^2 image over 20 cm, 16 views x 32 bins, 20 energies 20..115 keV."""
    geom = synth.make_geometry(n, 20.0, views, bins)
    spec = synth.make_spectral(20, 119, 120.0, i0, e_step=e_step)
    f_true = synth.inserts_phantom(n, 20.0)
    return geom, spec, f_true


def rotation(seed=0):
    """A random 3x3 orthogonal matrix."""
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    return q * np.sign(np.diag(r))[None, :]
