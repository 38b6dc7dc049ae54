"""Pins of the FP64 network oracle: the forward pass against a network
written out by hand, backward against central finite differences of that
forward, the SiLU derivative against its definition, the first Adam step
against its closed form, and the lbml symbols."""
import re
import os

import numpy as np
import pytest

from oracle import mlp

DIMS = [5, 16, 12, 7]


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    n = sum(DIMS[i] * DIMS[i + 1] + DIMS[i + 1] for i in range(len(DIMS) - 1))
    p = 0.5 * rng.standard_normal(n)
    x = rng.standard_normal((9, DIMS[0]))
    t = rng.standard_normal((9, DIMS[-1]))
    loss, g = mlp.loss_and_grad(p, DIMS, x, t)
    h = 1e-6
    idx = rng.choice(n, 120, replace=False)
    for i in idx:
        e = np.zeros(n)
        e[i] = h
        fd = (mlp.loss_and_grad(p + e, DIMS, x, t)[0] - mlp.loss_and_grad(p - e, DIMS, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9


def test_forward_hand_computed():
    """Forward pass of a 2-2-1 network written out by hand: layer 0 is
    z_j = sum_k W0[j][k] x_k + b0[j] with SiLU(z) = z / (1 + e^-z), the
    output layer is linear. W0 is square and not symmetric, so a transposed
    weight matrix, a missing bias, a swapped row order or SiLU on the output
    each change the numbers."""
    import math
    W0 = [[1.0, -2.0], [0.5, 3.0]]
    b0 = [0.1, -0.2]
    W1 = [[2.0, -1.0]]
    b1 = [0.3]
    p = np.array([W0[0][0], W0[0][1], W0[1][0], W0[1][1], b0[0], b0[1], W1[0][0], W1[0][1], b1[0]])
    x = np.array([[1.0, 2.0], [-0.7, 0.4]])

    def silu(z):
        return z / (1.0 + math.exp(-z))

    want = []
    for row in x:
        z0 = row[0] * W0[0][0] + row[1] * W0[0][1] + b0[0]
        z1 = row[0] * W0[1][0] + row[1] * W0[1][1] + b0[1]
        want.append(W1[0][0] * silu(z0) + W1[0][1] * silu(z1) + b1[0])
    y, _ = mlp.forward(p, [2, 2, 1], x)
    assert y.shape == (2, 1)
    assert np.allclose(y[:, 0], want, rtol=1e-15, atol=0)
    # first row by hand: z = (-2.9, 6.3)
    assert y[0, 0] == pytest.approx(2 * (-2.9 / (1 + math.exp(2.9))) - 6.3 / (1 + math.exp(-6.3)) + 0.3,
                                    rel=1e-15)


def test_silu_derivative():
    z = np.linspace(-8, 8, 101)
    s = mlp.sigmoid(z)
    d = s * (1 + z * (1 - s))
    h = 1e-6
    fd = ((z + h) * mlp.sigmoid(z + h) - (z - h) * mlp.sigmoid(z - h)) / (2 * h)
    assert np.allclose(d, fd, atol=1e-8)


def test_first_adam_step_is_signed_lr():
    """With zero moments, the bias-corrected first step is -lr g/(|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p, m, v = mlp.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=1e-2, eps=1e-8)
    assert np.allclose(p, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_lbml_symbols_exported():
    from paper_1310_7450_amd import lbnlm
    from paper_1310_7450_amd.mlp import LBML_FUNCTIONS
    if not os.path.exists(lbnlm.LIB_PATH):
        pytest.skip("liblbnlm.so not built")
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lbml.h")).read()
    declared = set(re.findall(r"^\s*(?:lbml_status|const char \*)\s*(lbml_\w+)\s*\(", hdr, re.M))
    assert declared == set(LBML_FUNCTIONS)
    L = lbnlm.load_library()
    for n in declared:
        assert hasattr(L, n)
    from paper_1310_7450_amd import mlp as gmlp
    assert gmlp.param_count([5, 256, 256, 256, 192]) == 182464
