"""Pin of the Poisson wavenumber solves through the projection step.

After the spanwise FFT, the per-wavenumber wall-normal solves (PPT, k = 0
gauge pinned) and the inverse FFT, the gradient-corrected velocity must be
discretely divergence free to round-off (fractional step of Sec. 2.2).  A
wrong coefficient index, sign, wavenumber or gauge choice leaves an O(1)
divergence.
"""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("P,method", [(4, "PPT"), (1, "EXACT"), (8, "PPT")])
def test_projection_divergence_free(orc, P, method):
    from oracle import projection
    Nz, Ny, Nx = 24, 32, 3
    rng = np.random.default_rng(2024)
    dy = np.diff(W.tanh_faces(Ny))
    dz = 1.0 / Nz
    v = rng.standard_normal((Nz, Ny + 1, Nx))
    v[:, 0, :] = 0.0
    v[:, Ny, :] = 0.0
    w = rng.standard_normal((Nz, Ny, Nx))
    div0 = np.max(np.abs(projection.divergence(v, w, dy, dz)))
    v1, w1, phi = projection.project(v, w, dy, dz, P=P, method=getattr(orc, method))
    div1 = np.max(np.abs(projection.divergence(v1, w1, dy, dz)))
    assert div0 > 10.0
    assert div1 <= 1e-13 * div0, (div1, div0)
    # walls untouched, k = 0 compatibility of the discrete divergence
    assert np.all(v1[:, 0, :] == 0) and np.all(v1[:, Ny, :] == 0)
    D = projection.divergence(v, w, dy, dz)
    assert abs(np.sum(D * dy[None, :, None])) < 1e-11 * np.sum(np.abs(D) * dy[None, :, None])


def test_projection_pdd_fails_at_low_k(orc):
    """The same projection with PDD (P = 4) leaves a visible divergence: the low
    wavenumber systems are too weakly dominant for the truncated Z."""
    from oracle import projection
    Nz, Ny, Nx = 24, 64, 2
    rng = np.random.default_rng(9)
    dy = np.diff(W.tanh_faces(Ny))
    dz = 1.0 / Nz
    v = rng.standard_normal((Nz, Ny + 1, Nx))
    v[:, 0, :] = v[:, Ny, :] = 0.0
    w = rng.standard_normal((Nz, Ny, Nx))
    div0 = np.max(np.abs(projection.divergence(v, w, dy, dz)))
    v1, w1, _ = projection.project(v, w, dy, dz, P=4, method=orc.PDD)
    assert np.max(np.abs(projection.divergence(v1, w1, dy, dz))) > 1e-6 * div0
