"""Pins of the warm-start network oracle (oracle/unet.py), on the CPU: each check comes from
outside the oracle (explicit loops, finite differences, closed forms, hand-worked bit patterns)."""
import numpy as np
import pytest
import torch

from oracle import unet as U
from paper_2012_14707_amd import geometry as G


def _loop_conv(x, w, b, periodic=False):
    """Explicit-loop 'same' convolution of one image x (H, W, cin) with w [k*k][cout][cin]."""
    H, W, _ = x.shape
    taps, cout, _ = w.shape
    k = int(round(taps ** 0.5))
    out = np.zeros((H, W, cout))
    for y in range(H):
        for xx in range(W):
            acc = np.array(b, dtype=float)
            for ky in range(k):
                for kx in range(k):
                    sy, sx = y + ky - k // 2, xx + kx - k // 2
                    if periodic:
                        sy, sx = sy % H, sx % W
                    if 0 <= sy < H and 0 <= sx < W:
                        acc = acc + w[ky * k + kx] @ x[sy, sx]
            out[y, xx] = acc
    return out


@pytest.mark.parametrize("k", [1, 3])
@pytest.mark.parametrize("periodic", [False, True])
def test_conv_matches_explicit_loops(k, periodic):
    rng = np.random.default_rng(k)
    x = rng.normal(size=(2, 5, 7, 6))
    w = rng.normal(size=(k * k, 4, 6))
    b = rng.normal(size=4)
    got = U.conv(torch.tensor(x).permute(0, 3, 1, 2), torch.tensor(w), torch.tensor(b),
                 periodic).permute(0, 2, 3, 1).numpy()
    for n in range(2):
        assert np.allclose(got[n], _loop_conv(x[n], w, b, periodic), rtol=1e-13, atol=1e-13)
    if periodic and k == 3:
        # a periodic convolution commutes with periodic shifts of the image
        sh = U.conv(torch.tensor(np.roll(x, (2, 3), (1, 2))).permute(0, 3, 1, 2), torch.tensor(w), torch.tensor(b),
                    True).permute(0, 2, 3, 1).numpy()
        assert np.allclose(sh, np.roll(got, (2, 3), (1, 2)), rtol=1e-13, atol=1e-13)


def _loop_forward(x, flat, L, base, cin, cout, periodic=False):
    """The network of include/lbm.h written loop by loop, with its own reading of the layout."""
    cin0 = (cin + 7) // 8 * 8
    off = [0]

    def take(taps, ci, co):
        w = flat[off[0]:off[0] + taps * co * ci].reshape(taps, co, ci)
        off[0] += taps * co * ci
        b = flat[off[0]:off[0] + co]
        off[0] += co
        return w, b

    enc = []
    for l in range(L):
        c = base * 2 ** l
        enc.append((take(9, cin0 if l == 0 else c // 2, c), take(9, c, c)))
    dec = {}
    for l in range(L - 2, -1, -1):
        c = base * 2 ** l
        dec[l] = (take(9, 3 * c, c), take(9, c, c))
    wo, bo = take(1, base, 8)
    assert off[0] == flat.size
    outs = []
    for img in x:
        h = img
        skips = []
        for l in range(L):
            h = np.maximum(_loop_conv(h, *enc[l][0], periodic), 0)
            h = np.maximum(_loop_conv(h, *enc[l][1], periodic), 0)
            if l < L - 1:
                skips.append(h)
                H, W, C = h.shape
                p = np.zeros((H // 2, W // 2, C))
                for y in range(H // 2):
                    for xx in range(W // 2):
                        p[y, xx] = (h[2 * y, 2 * xx] + h[2 * y + 1, 2 * xx] + h[2 * y, 2 * xx + 1]
                                    + h[2 * y + 1, 2 * xx + 1]) / 4
                h = p
        for l in range(L - 2, -1, -1):
            H, W, C = h.shape
            up = np.zeros((2 * H, 2 * W, C))
            for y in range(2 * H):
                for xx in range(2 * W):
                    up[y, xx] = h[y // 2, xx // 2]
            h = np.concatenate([up, skips[l]], axis=-1)
            h = np.maximum(_loop_conv(h, *dec[l][0], periodic), 0)
            h = np.maximum(_loop_conv(h, *dec[l][1], periodic), 0)
        outs.append(_loop_conv(h, wo, bo)[..., :cout])
    return np.array(outs)


@pytest.mark.parametrize("periodic", [False, True])
def test_forward_matches_loop_network(periodic):
    L, base, cin, cout = 3, 8, 5, 3
    rng = np.random.default_rng(7)
    flat = rng.normal(scale=0.3, size=U.param_count(L, base, cin, cout))
    x = rng.normal(size=(2, 8, 12, 8))
    got = U.forward(x, flat, L, base, cin, cout, periodic=periodic).numpy()
    want = _loop_forward(x, flat, L, base, cin, cout, periodic)
    assert np.abs(want).max() > 0.1
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12)


def test_param_count_closed_form():
    # 5 levels, 32 base channels, 12 inputs (16 stored), 3 outputs (8 stored)
    c = 32
    enc = (9 * 16 * c + c) + sum(9 * (c << (l - 1)) * (c << l) + (c << l) for l in range(1, 5)) \
        + sum(9 * (c << l) ** 2 + (c << l) for l in range(5))
    dec = sum(9 * 3 * (c << l) * (c << l) + (c << l) + 9 * (c << l) ** 2 + (c << l) for l in range(4))
    total = enc + dec + c * 8 + 8
    assert U.param_count(5, 32, 12, 3) == total
    assert 7.8e6 < total < 7.9e6


@pytest.mark.parametrize("periodic", [False, True])
def test_gradients_match_finite_differences(periodic):
    L, base, cin, cout = 2, 8, 3, 2
    rng = np.random.default_rng(3)
    n_p = U.param_count(L, base, cin, cout)
    flat = rng.normal(scale=0.4, size=n_p)
    x = np.zeros((2, 8, 8, 8))
    x[..., :cin] = rng.normal(size=(2, 8, 8, cin))
    target = rng.normal(size=(2, 8, 8, cout))
    mask = rng.random((2, 8, 8)) < 0.7
    loss, grad = U.loss_and_grad(x, flat, target, mask, L, base, cin, cout, periodic=periodic)
    assert np.isfinite(loss) and loss > 0

    def f(p):
        return float(U.loss(U.forward(x, p, L, base, cin, cout, periodic=periodic), target, mask))

    idx = rng.choice(n_p, 60, replace=False)
    # include the first conv, the bottleneck, the decoder and the output layer's bias
    idx = np.concatenate([idx, [0, n_p // 2, n_p - 9, n_p - 7]])
    h = 1e-6
    for i in idx:
        e = np.zeros(n_p)
        e[i] = h
        fd = (f(flat + e) - f(flat - e)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * (abs(grad[i]) + 1e-3 * np.abs(grad).max()), (i, fd, grad[i])
    # dead output rows (>= out_channels) get no gradient
    w_out_off = n_p - (base * 8 + 8)
    rows = grad[w_out_off:w_out_off + base * 8].reshape(8, base)
    assert np.all(rows[cout:] == 0)


def test_loss_definition():
    y = torch.tensor(np.arange(8.0).reshape(1, 2, 2, 2))
    t = np.zeros((1, 2, 2, 2))
    mask = np.array([[[1, 0], [0, 1]]])
    # pixels 0 and 3: (0^2 + 1^2 + 6^2 + 7^2) / (2 pixels * 2 channels)
    assert float(U.loss(y, t, mask)) == pytest.approx(86 / 4)


def test_adam_first_step_moves_by_lr_sign():
    rng = np.random.default_rng(0)
    g = rng.normal(size=100)
    w = rng.normal(size=100)
    w1, m1, v1 = U.adam(w, np.zeros(100), np.zeros(100), g, 1, lr=1e-3)
    assert np.allclose(w1 - w, -1e-3 * np.sign(g), rtol=0, atol=1e-3 * 1e-8 / np.abs(g).min() + 1e-15)
    # second step with the same gradient moves again by lr sign(g)
    w2, _, _ = U.adam(w1, m1, v1, g, 2, lr=1e-3)
    assert np.allclose(w2 - w1, -1e-3 * np.sign(g), atol=1e-9)


def test_bf16_rounding_bit_patterns():
    one = 1.0
    ulp = 2.0 ** -7
    vals = np.array([one, one + ulp / 2, one + 1.5 * ulp, one + ulp / 2 + 2.0 ** -20, -3.0, 0.0,
                     2.0 ** -130], dtype=np.float32)
    want = np.array([one, one, one + 2 * ulp, one + ulp, -3.0, 0.0, 2.0 ** -130], dtype=np.float32)
    got = U.bf16_round(vals)
    assert np.array_equal(got[:6], want[:6])
    rng = np.random.default_rng(1)
    r = rng.normal(size=10000).astype(np.float32) * 10.0 ** rng.integers(-5, 5, 10000)
    assert np.array_equal(U.bf16_round(r), torch.tensor(r).to(torch.bfloat16).to(torch.float32).numpy())


def test_features_of_poiseuille_channel():
    pb = G.poiseuille_config1()
    f = U.features(pb["solid"], pb["links"], 0.5, 1.0, 0.0)
    solid = pb["solid"] != 0
    assert np.all(f[solid][:, :9] == 0)
    fl = ~solid
    assert np.all(f[..., 0][fl] == 1)
    rows = np.where(fl.any(axis=1))[0]
    top, bot = rows.max(), rows.min()
    # the wall above the top fluid row and below the bottom one sit at q = 0.3 along N/NE/NW
    # and S/SE/SW; every other direction and every interior node has no link (1)
    for d in (2, 5, 6):
        assert np.allclose(f[top, :, d], 0.3)
        assert np.all(f[bot, :, d] == 1)
    for d in (4, 7, 8):
        assert np.allclose(f[bot, :, d], 0.3)
    for d in (1, 3):
        assert np.all(f[fl][:, d] == 1)
    assert np.all(f[rows[1:-1]][:, :, 1:9] == 1)
    assert np.all(f[..., 9] == 0.5) and np.all(f[..., 10] == 1.0) and np.all(f[..., 11] == 0.0)
    assert np.all(f[..., 12:] == 0)


def test_fields_keep_rest_mass():
    rng = np.random.default_rng(2)
    solid = (rng.random((9, 11)) < 0.3).astype(np.uint8)
    pred = rng.normal(size=(9, 11, 3))
    rho, ux, uy = U.fields(pred, solid, 1e-3, 2e-4, 1.0)
    fl = solid == 0
    assert rho[fl].sum() == pytest.approx(fl.sum(), rel=1e-15)
    assert np.all(rho[~fl] == 1.0) and np.all(ux[~fl] == 0) and np.all(uy[~fl] == 0)
    assert np.allclose(ux[fl], 1e-3 * pred[..., 0][fl]) and np.allclose(uy[fl], 1e-3 * pred[..., 1][fl])
    const = np.ones((9, 11, 3))
    rho_c, _, _ = U.fields(const, solid, 1.0, 1.0, 1.0)
    assert np.all(rho_c == 1.0)


@pytest.mark.parametrize("periodic", [False, True])
def test_conv_grads_match_finite_differences(periodic):
    rng = np.random.default_rng(5)
    x = rng.normal(size=(1, 4, 5, 3))
    w = rng.normal(size=(9, 2, 3))
    d = rng.normal(size=(1, 4, 5, 2))
    gx, gw, gb = U.conv_grads(x, w, d, periodic)

    def f(xx, ww):
        return float((U.conv(torch.tensor(xx).permute(0, 3, 1, 2), torch.tensor(ww), None,
                             periodic).permute(0, 2, 3, 1).numpy() * d).sum())

    h = 1e-6
    for i in range(x.size):
        e = np.zeros(x.size)
        e[i] = h
        e = e.reshape(x.shape)
        assert (f(x + e, w) - f(x - e, w)) / (2 * h) == pytest.approx(gx.reshape(-1)[i], abs=1e-7)
    for i in range(w.size):
        e = np.zeros(w.size)
        e[i] = h
        e = e.reshape(w.shape)
        assert (f(x, w + e) - f(x, w - e)) / (2 * h) == pytest.approx(gw.reshape(-1)[i], abs=1e-7)
    assert np.allclose(gb, d.sum(axis=(0, 1, 2)))


def test_smoothing_definition():
    # a constant field on the fluid stays constant; solid sites are 0
    solid = np.zeros((5, 6), np.uint8)
    solid[2, 1:4] = 1
    c = [np.full((5, 6), 2.5), np.full((5, 6), -1.0)]
    out = U.smooth(c, solid, True)
    assert np.all(out[0][solid == 0] == 2.5) and np.all(out[1][solid == 0] == -1.0) and np.all(out[0][solid == 1] == 0)
    # hand-worked corner of a bounded 3 x 3 image with one solid site: the corner (0, 0) averages
    # its fluid neighbours (0,0), (0,1), (1,0) ((1,1) is solid)
    solid = np.zeros((3, 3), np.uint8)
    solid[1, 1] = 1
    v = np.arange(9.0).reshape(3, 3)
    got = U.smooth([v], solid, False)[0]
    assert got[0, 0] == pytest.approx((0 + 1 + 3) / 3)
    assert got[0, 1] == pytest.approx((0 + 1 + 2 + 3 + 5) / 5)
    # periodic: the same corner also sees the wrapped row 2 and column 2
    got = U.smooth([v], solid, True)[0]
    assert got[0, 0] == pytest.approx((0 + 1 + 2 + 3 + 5 + 6 + 7 + 8) / 8)
    # against a vectorised masked box filter on a random periodic case
    rng = np.random.default_rng(0)
    solid = (rng.random((7, 9)) < 0.3).astype(np.uint8)
    u = rng.normal(size=(7, 9)) * (solid == 0)
    w = (solid == 0).astype(float)
    sm = sum(np.roll(np.roll(u, a, 0), b, 1) for a in (-1, 0, 1) for b in (-1, 0, 1))
    cn = sum(np.roll(np.roll(w, a, 0), b, 1) for a in (-1, 0, 1) for b in (-1, 0, 1))
    want = np.where(solid == 0, sm / np.maximum(cn, 1), 0)
    assert np.allclose(U.smooth([u], solid, True)[0], want, rtol=1e-14, atol=1e-15)


def test_fields_smoothing_keeps_rest_mass():
    rng = np.random.default_rng(3)
    solid = (rng.random((8, 10)) < 0.3).astype(np.uint8)
    pred = rng.normal(size=(8, 10, 3))
    rho, ux, uy = U.fields(pred, solid, 1e-3, 2e-4, 1.0, smooth_iters=3, periodic=True)
    fl = solid == 0
    assert rho[fl].sum() == pytest.approx(fl.sum(), rel=1e-15)
    # three passes shrink the spread of a noise field
    assert ux[fl].std() < 0.6 * 1e-3 * pred[..., 0][fl].std()
