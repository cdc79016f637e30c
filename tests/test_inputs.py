"""The seeded input generators: the paper's hidden-layer initialisation
(sec. 4.1, eq. init_be) mapped to the library's local coordinates."""
import math

import numpy as np

from paper_2503_10032_amd import inputs as I


def test_paper_initialisation_in_local_coordinates():
    """w ~ U([-l, l]^2) with l = c M^{1/2} / diam(B_r) and diam(B_r) =
    2 diam(Omega_i); b = -w . xi with xi in the closed r-neighbourhood B_r,
    r = diam(Omega_i)/2.  In local coordinates xi_loc = (x - centre)/half the
    neuron reads (w * half) . xi_loc + w . (centre - xi), so the hyperplane of
    every neuron lies within diam(Omega_i)/2 + r = diam(Omega_i) of the centre."""
    nx, ny, M, c = 3, 2, 400, 0.75
    W, b = I.paper_hidden_params(nx, ny, M, c, seed=4)
    assert W.shape == (nx * ny, M, 2) and b.shape == (nx * ny, M)
    hx, hy = 1.0 / nx, 1.0 / ny
    diam = math.hypot(hx, hy)
    ell = c * math.sqrt(M) / (2.0 * diam)
    half = 0.5 * np.array([hx, hy])
    for i in range(nx * ny):
        w = W[i] / half                              # weights acting on global coordinates
        assert np.all(np.abs(w) <= ell * (1 + 1e-12))
        assert np.abs(w).max() > 0.95 * ell
        dist = np.abs(b[i]) / np.linalg.norm(w, axis=1)    # centre to the neuron's hyperplane
        assert np.all(dist <= diam * (1 + 1e-12))
        assert dist.max() > 0.5 * diam               # the hyperplanes reach beyond the box itself
    W2, b2 = I.paper_hidden_params(nx, ny, M, c, seed=4)
    np.testing.assert_array_equal(W, W2)
    np.testing.assert_array_equal(b, b2)
