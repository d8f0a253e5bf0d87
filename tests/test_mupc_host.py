"""The library's host-side mu-PC basis (osscir_mu_pc_basis, no device work)
against the oracle's Gram-Schmidt (two independent implementations of the
same reading), and its error path."""
import os

import numpy as np
import pytest

import synth
from oracle import mupc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1801_06263_amd", "libosscir.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libosscir.so not built")


@pytest.mark.parametrize("kvp,hi", [(120.0, 119), (140.0, 139)])
def test_library_basis_matches_oracle(kvp, hi):
    from paper_1801_06263_amd.osscir import mu_pc_basis
    spec = synth.make_spectral(20, hi, kvp, 1e5)
    B, mu_t = mu_pc_basis(spec)
    B_ref, Q_ref = mupc.mu_pc_basis(spec)
    np.testing.assert_allclose(B, B_ref, rtol=1e-12, atol=1e-12 * np.abs(B_ref).max())
    np.testing.assert_allclose(mu_t, Q_ref, rtol=0, atol=1e-12 * np.abs(Q_ref).max())


def test_dependent_rows_are_rejected():
    from paper_1801_06263_amd.osscir import OsscirError, mu_pc_basis
    spec = synth.make_spectral(20, 119, 120.0, 1e5)
    mu = spec.mu.copy()
    mu[2] = 2.0 * mu[0]
    with pytest.raises(OsscirError):
        mu_pc_basis(synth.Spectral(mu=mu, s=spec.s, n0=spec.n0))
