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


def dev(a):
    """numpy -> float32 CUDA tensor."""
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    """CUDA tensor -> float64 numpy (synchronising)."""
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def normwise(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def sino(a_lw, n_views, n_bins):
    """oracle ray-major [L, W] -> library [W, V, D]."""
    return np.ascontiguousarray(np.asarray(a_lw).T.reshape(-1, n_views, n_bins))


UPPER = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
