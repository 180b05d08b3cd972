"""Pins of the differentiable-workload oracle: L = sum_k w_k |(F x)_k|^2 and
its gradient 2 F^H (w . F x), against FP64 central finite differences."""
import numpy as np

import oracle


def test_gradient_matches_central_differences():
    n, batch = 64, 3
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, (batch, n)) + 1j * rng.uniform(-1, 1, (batch, n))
    w = rng.uniform(0, 1, n)
    L0, g = oracle.weighted_power_loss(x, w)
    h = 1e-6
    picks = rng.integers(0, batch * n, 24)
    xf = x.reshape(-1)
    for idx in picks:
        for part, unit in (("re", 1.0), ("im", 1j)):
            xp, xm = xf.copy(), xf.copy()
            xp[idx] += h * unit
            xm[idx] -= h * unit
            fd = (oracle.weighted_power_loss(xp.reshape(batch, n), w, want_grad=False)[0]
                  - oracle.weighted_power_loss(xm.reshape(batch, n), w, want_grad=False)[0]) / (2 * h)
            an = g.reshape(-1)[idx].real if part == "re" else g.reshape(-1)[idx].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (idx, part, fd, an)


def test_loss_closed_form():
    # x = delta_0 gives X = ones, so L = sum_k w_k.
    n = 128
    w = np.linspace(0, 1, n)
    d = np.zeros(n, complex)
    d[0] = 1
    L, g = oracle.weighted_power_loss(d, w)
    assert abs(L - w.sum()) < 1e-12
    # gradient: 2 F^H w = 2 * (inverse-sign DFT of w)
    assert np.allclose(g, 2 * np.fft.ifft(w) * n, atol=1e-12)
