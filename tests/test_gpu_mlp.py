"""GPU network kernels against the FP64 numpy oracle (BF16 operands, FP32
accumulation).

Element by element: every output and every gradient entry equals the
oracle's network evaluated at BF16 operands (both factors of every product
rounded to BF16, the precision the network is specified in; sums in FP64)
within 2^-8 of the absolute product sums of the GEMM that produced it. As
norms against the plain FP64 oracle: forward and gradients within 2e-2
relative L2, cosine >= 0.999; Adam within FP32 round-off of the oracle's
update applied to the GPU's own gradients."""
import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

DIMS = [5, 256, 256, 256, 192]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_1310_7450_amd import mlp
    rng = np.random.default_rng(1)
    B = 100  # not a multiple of 16: ragged tiles
    x = rng.standard_normal((B, DIMS[0])).astype(np.float32)
    t = (0.3 * rng.standard_normal((B, DIMS[-1]))).astype(np.float32)
    p = mlp.init_params(DIMS, seed=3)
    net = mlp.Net(DIMS, max_batch=256)
    net.set_params(p)
    xd = torch.from_numpy(x).cuda()
    td = torch.from_numpy(t).cuda()
    return net, p, x, t, xd, td


def bf16(a):
    """FP32 -> BF16 -> FP64 with round to nearest, ties to even: keep the top
    16 bits of the FP32 pattern after adding half an ulp of the kept part
    (0x7fff plus the kept part's lowest bit)."""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_rounding_helper():
    """The test's BF16 rounding: exact values stay, halfway cases go to the
    even neighbour, others to the nearest (BF16 keeps 8 significant bits)."""
    assert bf16(np.float32(1.0)) == 1.0
    assert bf16(np.float32(1.0 + 2.0 ** -8)) == 1.0                 # tie, to even
    assert bf16(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6  # tie, to even (up)
    assert bf16(np.float32(1.0 + 2.0 ** -8 + 2.0 ** -20)) == 1.0 + 2.0 ** -7
    assert bf16(np.float32(-3.0)) == -3.0


@pytest.fixture(scope="module")
def setup_bias():
    """The network with random biases (zero biases would hide a bias added to
    the wrong column) and a ragged batch of 77 rows."""
    import torch
    from paper_1310_7450_amd import mlp
    rng = np.random.default_rng(11)
    B = 77
    x = rng.standard_normal((B, DIMS[0])).astype(np.float32)
    p = mlp.init_params(DIMS, seed=4).astype(np.float64)
    o = 0
    for l in range(len(DIMS) - 1):
        o += DIMS[l] * DIMS[l + 1]
        p[o:o + DIMS[l + 1]] = rng.uniform(-0.5, 0.5, DIMS[l + 1])
        o += DIMS[l + 1]
    p = p.astype(np.float32)
    net = mlp.Net(DIMS, max_batch=256)
    net.set_params(p)
    return net, p, x, torch.from_numpy(x).cuda()


# Element-wise tolerance against the oracle at BF16 operands: one BF16 unit
# roundoff (2^-8) of the absolute product sum sum_k |a_ik b_kj| of the GEMM
# that produced the entry. What separates the two is FP32 accumulation (at
# most K 2^-24 of that sum, 1.5e-5 at K = 256) and operands that round to the
# other BF16 neighbour on one side: an activation or a back-propagated dZ
# whose FP32 value differs from the oracle's by the accumulation error can
# cross a rounding midpoint, which changes that term by one BF16 ulp (2^-7 of
# itself). Back-propagated dZ come from sums with much cancellation, so such
# crossings are common there, and a weight gradient sums only the 77 rows of
# the batch. A wrong tile, row or bias gives errors of the size of the
# entries themselves.
TOL_ABS_SUM = 2.0 ** -8


def test_forward_elementwise(setup_bias):
    """Every output of the 5-256-256-256-192 network on a ragged batch of 77
    rows equals the oracle evaluated at BF16 operands within 2^-8 of the
    last layer's absolute product sums; against the FP64 oracle the outputs
    agree within 2e-2 relative L2."""
    import torch
    net, p, x, xd = setup_bias
    y = net.forward(xd)
    torch.cuda.synchronize()
    yg = y.cpu().numpy().astype(np.float64)
    p64, x64 = p.astype(np.float64), x.astype(np.float64)
    yb, cache = omlp.forward(p64, DIMS, x64, operand=bf16)
    W_last = omlp.unpack(p64, DIMS)[-1][0]
    absum = np.abs(bf16(cache[-1][0])) @ np.abs(bf16(W_last)).T
    ratio = np.abs(yg - yb) / (TOL_ABS_SUM * absum)
    y64 = omlp.forward(p64, DIMS, x64)[0]
    print(f"forward: max |err| / tol {ratio.max():.3e}; tol / |y| median "
          f"{np.median(TOL_ABS_SUM * absum / np.abs(yb)):.2e}; vs FP64 rel L2 {rel(yg, y64):.2e}", flush=True)
    assert ratio.max() <= 1.0
    assert rel(yg, y64) < 2e-2


def test_gradients_elementwise(setup_bias):
    """From the oracle's dL/dy (mean squared error against a seeded target),
    every weight gradient dW_l = dZ_l^T H_(l-1) and bias gradient sum_rows dZ_l
    of every layer, through the hidden layers' dZ = (dZ W) * SiLU'(z) path,
    equals the oracle's backward at BF16 operands within 2^-8 of the
    absolute product (or row) sums; against the FP64 oracle the gradients
    agree within 2e-2 relative L2 with cosine > 0.999."""
    import torch
    net, p, x, xd = setup_bias
    rng = np.random.default_rng(12)
    t = 0.3 * rng.standard_normal((x.shape[0], DIMS[-1]))
    p64, x64 = p.astype(np.float64), x.astype(np.float64)
    yb, cache = omlp.forward(p64, DIMS, x64, operand=bf16)
    _, dy = omlp.mse(yb, t)
    dy = dy.astype(np.float32).astype(np.float64)
    gb = omlp.backward(p64, DIMS, cache, dy, operand=bf16)
    net.forward(xd)
    net.backward(torch.from_numpy(dy.astype(np.float32)).cuda())
    g = net.get_grads().astype(np.float64)
    # absolute sums of every gradient entry, from the oracle's own dZ
    layers = omlp.unpack(p64, DIMS)
    dz = dy
    sums = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        h, _ = cache[l]
        sums[l] = (np.abs(bf16(dz)).T @ np.abs(bf16(h)), np.abs(dz).sum(axis=0))
        if l > 0:
            z = cache[l - 1][1]
            s = 1.0 / (1.0 + np.exp(-z))
            dz = (bf16(dz) @ bf16(layers[l][0])) * (s * (1.0 + z * (1.0 - s)))
    absum = np.concatenate([np.concatenate([a.ravel(), c]) for a, c in sums])
    ratio = np.abs(g - gb) / (TOL_ABS_SUM * absum)
    o = 0
    for l in range(len(DIMS) - 1):
        nW, nb = DIMS[l] * DIMS[l + 1], DIMS[l + 1]
        print(f"layer {l}: dW max |err| / tol {ratio[o:o + nW].max():.3e}, "
              f"db {ratio[o + nW:o + nW + nb].max():.3e}", flush=True)
        o += nW + nb
    go = omlp.backward(p64, DIMS, omlp.forward(p64, DIMS, x64)[1], dy)
    cos = float(g @ go / np.linalg.norm(g) / np.linalg.norm(go))
    print(f"gradients vs FP64: rel L2 {rel(g, go):.2e}, cos {cos:.6f}", flush=True)
    assert ratio.max() <= 1.0
    assert cos > 0.999 and rel(g, go) < 2e-2


def test_forward_matches_oracle(setup):
    import torch
    net, p, x, t, xd, td = setup
    y = net.forward(xd)
    torch.cuda.synchronize()
    yo, _ = omlp.forward(p.astype(np.float64), DIMS, x)
    e = rel(y.cpu().numpy(), yo)
    print(f"forward rel L2 {e:.3e}", flush=True)
    assert e < 2e-2


def test_gradients_match_oracle(setup):
    import torch
    net, p, x, t, xd, td = setup
    y = net.forward(xd)
    dy = torch.empty_like(y)
    loss = net.mse(y, td, dy)
    net.backward(dy)
    g = net.get_grads()
    lo, go = omlp.loss_and_grad(p.astype(np.float64), DIMS, x, t)
    cos = float(g @ go / np.linalg.norm(g) / np.linalg.norm(go))
    e = rel(g, go)
    print(f"loss {loss:.6e} vs {lo:.6e}; grad rel L2 {e:.3e} cos {cos:.6f}", flush=True)
    assert abs(loss - lo) / lo < 2e-2
    assert cos > 0.999 and e < 2e-2


def test_adam_matches_oracle(setup):
    import torch
    from paper_1310_7450_amd import mlp
    net, p, x, t, xd, td = setup
    net2 = mlp.Net(DIMS, max_batch=256)
    net2.set_params(p)
    y = net2.forward(xd)
    dy = torch.empty_like(y)
    net2.mse(y, td, dy)
    net2.backward(dy)
    g = net2.get_grads().astype(np.float64)
    net2.adam_step(lr=1e-3)
    p1 = net2.get_params()
    po, m, v = omlp.adam(p.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, lr=1e-3)
    assert np.abs(p1 - po).max() < 1e-6


def test_training_reduces_loss():
    """A smooth synthetic regression (outputs are fixed sinusoids of the
    inputs): 300 Adam steps on the GPU cut the loss by more than 10x."""
    import torch
    from paper_1310_7450_amd import mlp
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, (256, 5)).astype(np.float32)
    A = rng.standard_normal((5, 192))
    t = np.sin(x @ A).astype(np.float32)
    net = mlp.Net(DIMS, max_batch=256)
    net.set_params(mlp.init_params(DIMS, seed=0))
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    dy = torch.empty_like(td)
    first = None
    for it in range(300):
        y = net.forward(xd)
        loss = net.mse(y, td, dy, want_loss=(it % 50 == 0 or it == 299))
        if first is None:
            first = loss
        net.backward(dy)
        net.adam_step(lr=2e-3)
    print(f"loss {first:.4e} -> {loss:.4e}", flush=True)
    assert loss < first / 10


def test_train_step_equals_separate_calls():
    """lbml_train_step (rows gathered on the device, one call) gives the same
    loss, gradients and updated parameters, bit for bit, as forward, mse,
    backward and adam_step on the same rows gathered by torch; two steps in a
    row, the second with a smaller batch."""
    import torch
    from paper_1310_7450_amd import mlp
    rng = np.random.default_rng(21)
    X = torch.from_numpy(rng.standard_normal((300, DIMS[0])).astype(np.float32)).cuda()
    Y = torch.from_numpy((0.3 * rng.standard_normal((300, DIMS[-1]))).astype(np.float32)).cuda()
    p0 = mlp.init_params(DIMS, seed=6)
    a, b = mlp.Net(DIMS, max_batch=128), mlp.Net(DIMS, max_batch=128)
    a.set_params(p0)
    b.set_params(p0)
    for batch in (100, 37):
        idx = torch.from_numpy(rng.choice(300, batch, replace=False).astype(np.int32)).cuda()
        la = a.train_step(X, Y, idx, lr=1e-3, want_loss=True)
        xb = X.index_select(0, idx.long()).contiguous()
        yb = Y.index_select(0, idx.long()).contiguous()
        y = b.forward(xb)
        dy = torch.empty_like(y)
        lb = b.mse(y, yb, dy, want_loss=True)
        b.backward(dy)
        b.adam_step(lr=1e-3)
        torch.cuda.synchronize()
        print(f"batch {batch}: loss {la:.6e} vs {lb:.6e}", flush=True)
        assert la == lb
        assert np.array_equal(a.get_grads(), b.get_grads())
        assert np.array_equal(a.get_params(), b.get_params())
