"""Pins of the CNN and random-number oracles (CPU only).

Each layer of ``oracle.cnn`` is checked against a library routine or a
closed form it reduces to (scipy correlation, numpy Kronecker products,
block means), its gradients against central finite differences (the loss is
linear in each argument, so the difference quotient is exact up to
rounding), the whole U-Net's gradient against finite differences on a tiny
grid, and Adam against its closed-form first step.  ``oracle.rng`` is
pinned to the published Philox known-answer vectors, its small-mean Poisson
branch to scipy's inverse CDF, and both branches to the Poisson law by
moments and a chi-square test.
"""

import os

import numpy as np
import pytest
from scipy import ndimage, signal, stats

from oracle import cnn, rng

HERE = os.path.dirname(__file__)


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


# ---- bfloat16 rounding -------------------------------------------------------------

def test_round_bf16_matches_torch_cast():
    torch = pytest.importorskip("torch")
    r = np.random.default_rng(0)
    x = np.concatenate([r.standard_normal(20000) * 10.0 ** r.integers(-30, 30, 20000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, 1e-40]])
    # exact ties: 1 + 2^-8 (tie, even below) and 1 + 3 * 2^-8 (tie, even above)
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.round_bf16(x), ref)


# ---- single layers ------------------------------------------------------------------

def test_k3_single_channel_is_scipy_correlate():
    x = _rand((1, 5, 6, 7, 1), 1)
    W = _rand((1, 3, 3, 3, 1), 2)
    y = cnn.conv("k3", x, W)
    ref = ndimage.correlate(x[0, ..., 0], W[0, ..., 0], mode="constant", cval=0.0)
    np.testing.assert_allclose(y[0, ..., 0], ref, rtol=1e-13, atol=1e-13)


def test_k3_multichannel_sums_single_channel_correlations():
    x = _rand((2, 4, 5, 3, 3), 3)
    W = _rand((4, 3, 3, 3, 3), 4)
    b = _rand(4, 5)
    y = cnn.conv("k3", x, W, b)
    for n in range(2):
        for o in range(4):
            ref = sum(ndimage.correlate(x[n, ..., c], W[o, ..., c], mode="constant") for c in range(3)) + b[o]
            np.testing.assert_allclose(y[n, ..., o], ref, rtol=1e-12, atol=1e-12)


def test_dn_is_strided_valid_correlation_and_block_mean():
    x = _rand((1, 6, 4, 8, 2), 6)
    W = _rand((3, 2, 2, 2, 2), 7)
    y = cnn.conv("dn", x, W)
    assert y.shape == (1, 3, 2, 4, 3)
    for o in range(3):
        ref = sum(signal.correlate(x[0, ..., c], W[o, ..., c], mode="valid")[::2, ::2, ::2] for c in range(2))
        np.testing.assert_allclose(y[0, ..., o], ref, rtol=1e-12, atol=1e-12)
    mean = cnn.conv("dn", x[..., :1], np.full((1, 2, 2, 2, 1), 0.125))
    blocks = x[0, ..., 0].reshape(3, 2, 2, 2, 4, 2).mean(axis=(1, 3, 5))
    np.testing.assert_allclose(mean[0, ..., 0], blocks, rtol=1e-13)


def test_up_is_kronecker_product_and_adjoint_of_dn():
    x = _rand((1, 3, 2, 4, 2), 8)
    W = _rand((2, 2, 2, 3, 2), 9)
    y = cnn.conv("up", x, W)
    assert y.shape == (1, 6, 4, 8, 3)
    for o in range(3):
        ref = sum(np.kron(x[0, ..., c], W[..., o, c]) for c in range(2))
        np.testing.assert_allclose(y[0, ..., o], ref, rtol=1e-12, atol=1e-12)
    # <dn_V(a), b> = <a, up_W(b)> with W[i,j,k,c,o] = V[o,i,j,k,c]
    V = _rand((3, 2, 2, 2, 2), 10)
    a = _rand((2, 4, 6, 2, 2), 11)
    bb = _rand((2, 2, 3, 1, 3), 12)
    Wt = np.transpose(V, (1, 2, 3, 4, 0))
    lhs = np.vdot(cnn.conv("dn", a, V), bb)
    rhs = np.vdot(a, cnn.conv("up", bb, Wt))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_k1_identity_and_mixing():
    x = _rand((2, 2, 3, 4, 5), 13)
    np.testing.assert_array_equal(cnn.conv("k1", x, np.eye(5)), x)
    W = _rand((3, 5), 14)
    y = cnn.conv("k1", x, W)
    np.testing.assert_allclose(y[1, 1, 2, 3], W @ x[1, 1, 2, 3], rtol=1e-13)


@pytest.mark.parametrize("kind,xs,co", [("k3", (2, 3, 4, 5, 3), 2), ("dn", (1, 4, 2, 6, 2), 3),
                                        ("up", (2, 2, 1, 3, 3), 2), ("k1", (1, 2, 3, 2, 4), 3)])
def test_layer_gradients_match_finite_differences(kind, xs, co):
    x = _rand(xs, 20)
    W = _rand(cnn.weight_shape(kind, co, xs[-1]), 21)
    b = _rand(co, 22)
    R = _rand(cnn.conv(kind, x, W, b).shape, 23)

    def loss(x_, W_, b_):
        return float(np.vdot(cnn.conv(kind, x_, W_, b_), R))

    dx, dW, db = cnn.conv_backward(kind, x, W, R)
    h = 1e-3
    for arr, grad, which in ((x, dx, 0), (W, dW, 1), (b, db, 2)):
        flat = arr.reshape(-1)
        for idx in np.random.default_rng(24).choice(flat.size, min(flat.size, 25), replace=False):
            args = [x.copy(), W.copy(), b.copy()]
            a = args[which].reshape(-1)
            a[idx] += h
            lp = loss(*args)
            a[idx] -= 2 * h
            lm = loss(*args)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grad.reshape(-1)[idx]) <= 1e-9 * (1 + abs(fd)), (which, idx)


# ---- U-Net ---------------------------------------------------------------------------

CH = (2, 3, 4, 4)


def _tiny_net(seed=30):
    P = cnn.init_params(CH, seed)
    r = np.random.default_rng(seed + 1)
    for k in P:
        if k.endswith(".b"):
            P[k] = r.uniform(0.05, 0.2, P[k].shape)
    return P


def test_unet_layer_list_and_shapes():
    names = [n for n, *_ in cnn.unet_layers()]
    assert len(names) == 21 and names[0] == "e1a" and names[-1] == "head"
    kinds = {k for _, k, _, _ in cnn.unet_layers()}
    assert kinds == set(cnn.KINDS)
    P = _tiny_net()
    y, acts = cnn.unet_forward(P, _rand((1, 8, 8, 16, 1), 31), CH)
    assert y.shape == (1, 8, 8, 16, 1) and (y >= 0).all()
    assert acts["m4b"].shape == (1, 1, 1, 2, 4)
    assert acts["cat1"].shape == (1, 8, 8, 16, 4)


def test_unet_gradient_matches_finite_differences():
    P = _tiny_net()
    x = np.abs(_rand((1, 8, 8, 8, 1), 32))
    R = _rand((1, 8, 8, 8, 1), 33)
    _, acts = cnn.unet_forward(P, x, CH)
    G = cnn.unet_backward(P, acts, R, CH)
    assert set(G) == set(P)
    r = np.random.default_rng(34)
    h = 1e-6
    worst = 0.0
    for k in sorted(P):
        flat = P[k].reshape(-1)
        for idx in r.choice(flat.size, min(flat.size, 3), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = float(np.vdot(cnn.unet_forward(P, x, CH)[0], R))
            flat[idx] = old - h
            lm = float(np.vdot(cnn.unet_forward(P, x, CH)[0], R))
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            g = G[k].reshape(-1)[idx]
            err = abs(fd - g) / (1e-6 + abs(fd) + abs(g))
            worst = max(worst, err)
            assert err <= 1e-5, (k, idx, fd, g)
    print("worst relative FD mismatch", worst)


def test_unet_rounded_storage_stays_close():
    P = _tiny_net()
    x = np.abs(_rand((1, 8, 8, 8, 1), 35))
    y, _ = cnn.unet_forward(P, x, CH)
    yb, _ = cnn.unet_forward(P, x, CH, store=cnn.round_bf16)
    assert np.linalg.norm(yb - y) <= 2e-2 * np.linalg.norm(y)


def test_mse_and_adam_closed_forms():
    y, t = _rand(50, 40), _rand(50, 41)
    L, g = cnn.mse(y, t)
    assert L == pytest.approx(np.sum((y - t) ** 2) / 50, rel=1e-14)
    h = 1e-6
    yp = y.copy()
    yp[7] += h
    assert (cnn.mse(yp, t)[0] - L) / h == pytest.approx(g[7], rel=1e-5)
    # first step from zero moments: w - lr g / (|g| + eps) (bias correction
    # makes m_hat = g, v_hat = g^2); with a constant gradient every step is
    # the same
    w0 = _rand(20, 42)
    gr = _rand(20, 43)
    w1, m, v = cnn.adam_step(w0, gr, np.zeros(20), np.zeros(20), 1, lr=0.01)
    np.testing.assert_allclose(w1, w0 - 0.01 * gr / (np.abs(gr) + 1e-8), rtol=1e-12)
    w2, _, _ = cnn.adam_step(w1, gr, m, v, 2, lr=0.01)
    np.testing.assert_allclose(w2 - w1, w1 - w0, rtol=1e-10)


# ---- random numbers -------------------------------------------------------------------

def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(v, 16) for v in line.split()])
    return rows


def test_philox_known_answer_vectors():
    rows = _kat()
    assert len(rows) == 3
    for r in rows:
        out = rng.philox4x32_10(*[np.array([v], dtype=np.uint32) for v in r[:4]], np.uint32(r[4]),
                                np.uint32(r[5]))
        assert [int(o[0]) for o in out] == r[6:]


def test_uniform53_range_and_resolution():
    assert rng.uniform53(0, 0) == 0.0
    top = rng.uniform53(0xFFFFFFFF, 0xFFFFFFFF)
    assert top < 1.0 and top == 1.0 - 2.0 ** -53
    w = rng.philox_words(7, np.arange(200000))
    u = rng.uniform53(w[0], w[1])
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / u.size)
    assert stats.kstest(u, "uniform").pvalue > 1e-4


def test_small_mean_poisson_is_inverse_cdf():
    lam = np.random.default_rng(50).uniform(0.0, 9.99, 20000)
    k = rng.poisson_sample(lam, seed=11, stream=3)
    w = rng.philox_words(11, np.arange(lam.size), 3, 0)
    u = rng.uniform53(w[0], w[1])
    ref = stats.poisson.ppf(u, lam)
    assert np.mean(k == ref) > 0.9999


@pytest.mark.parametrize("lam", [0.3, 4.0, 9.9, 10.0, 37.5, 1.0e3, 2.5e5])
def test_poisson_law(lam):
    n = 200000
    k = rng.poisson_sample(np.full(n, lam), seed=99, stream=int(lam * 10) % 1000)
    se_mean = np.sqrt(lam / n)
    assert abs(k.mean() - lam) < 5 * se_mean
    # variance of the sample variance of a Poisson law: (lam + 2 lam^2 (n/(n-1))) / n
    se_var = np.sqrt((lam + 2 * lam * lam) / n)
    assert abs(k.var(ddof=1) - lam) < 5 * se_var
    lo, hi = stats.poisson.ppf([1e-4, 1 - 1e-4], lam)
    edges = np.unique(np.linspace(lo, hi + 1, 40).astype(np.int64))
    obs = np.histogram(np.clip(k, edges[0], edges[-1] - 1), bins=edges)[0]
    cdf = stats.poisson.cdf(edges - 1, lam)
    cdf[0], cdf[-1] = 0.0, 1.0
    exp = np.diff(cdf) * n
    keep = exp > 5
    chi2 = np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep])
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4


def test_noisy_histogram_scaling():
    m = np.abs(_rand(5000, 60)).astype(np.float32)
    d = rng.noisy_histogram(m, 1e4, seed=5)
    s = 1e4 / float(m.max())
    counts = d.astype(np.float64) * s
    assert np.allclose(counts, np.round(counts), atol=1e-3)
    assert abs(d.sum() / m.sum() - 1) < 5 / np.sqrt(m.sum() * s)
