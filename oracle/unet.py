"""CPU oracle of the learned warm start (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
module.  It is written from the network's definition (the encoder-decoder, its parameter
vector layout, the masked squared-error loss, Adam, the input features and the initial fields)
in plain float64 torch CPU operations, with autograd for gradients; it shares no code with the
HIP library.  The network is not part of the paper: it only supplies the initial state of the
lattice, whose steady solution does not depend on it.

Tensor conventions: images are NHWC numpy arrays; a convolution's weights are stored as
[k*k][cout][cin] with tap index ky*k + kx and offset (ky - k//2, kx - k//2).

Pins (tests/test_oracle_nn.py): the convolution against explicit loops, the whole forward
pass against a loop-by-loop implementation on a tiny network, every gradient against central
finite differences, the parameter count against its closed form, Adam's first step against its
closed form (each parameter moves by lr * sign(g)), bf16 rounding against hand-worked bit
patterns, and the features and fields against hand-built cases.
"""
import numpy as np
import torch
import torch.nn.functional as F

OUT_PAD = 8  # the output convolution always has 8 rows; rows >= out_channels are zero


def bf16_round(a):
    """Round-to-nearest-even of float32 values to bfloat16 (the top 16 bits), returned as float32."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).reshape(a32.shape)


def layer_shapes(levels, base, in_channels, out_channels):
    """(taps, cin, cout) of every convolution in parameter-vector order: encoder levels
    0..L-1 (two convolutions each), decoder levels L-2..0 (two each), then the 1x1 output."""
    cin0 = (in_channels + 7) // 8 * 8
    shapes = []
    for l in range(levels):
        c = base << l
        shapes.append((9, cin0 if l == 0 else base << (l - 1), c))
        shapes.append((9, c, c))
    for l in range(levels - 2, -1, -1):
        c = base << l
        shapes.append((9, (base << (l + 1)) + c, c))
        shapes.append((9, c, c))
    shapes.append((1, base, OUT_PAD))
    return shapes


def param_count(levels, base, in_channels, out_channels):
    return sum(t * ci * co + co for t, ci, co in layer_shapes(levels, base, in_channels, out_channels))


def unpack(flat, levels, base, in_channels, out_channels):
    """List of (w [taps][cout][cin], b [cout]) float64 torch tensors from the flat vector."""
    flat = flat if isinstance(flat, torch.Tensor) else torch.as_tensor(np.asarray(flat, dtype=np.float64))
    out, off = [], 0
    for t, ci, co in layer_shapes(levels, base, in_channels, out_channels):
        w = flat[off:off + t * co * ci].reshape(t, co, ci)
        off += t * co * ci
        b = flat[off:off + co]
        off += co
        out.append((w, b))
    assert off == flat.numel()
    return out


def conv(x, w, b, periodic=False):
    """'Same' convolution of x (N, C, H, W) with w [k*k][cout][cin]: out[co](y, x) =
    b[co] + sum_{ky,kx,ci} in[ci](y + ky - k//2, x + kx - k//2) w[ky*k+kx][co][ci], where in[] is
    zero outside the image, or (periodic) indices are taken modulo the image size."""
    taps, co, ci = w.shape
    k = int(round(taps ** 0.5))
    weight = w.reshape(k, k, co, ci).permute(2, 3, 0, 1)
    if periodic and k > 1:
        return F.conv2d(F.pad(x, (k // 2,) * 4, mode="circular"), weight, b)
    return F.conv2d(x, weight, b, padding=k // 2)


def conv_grads(x_nhwc, w, dout_nhwc, periodic=False):
    """Gradients of sum(conv(x, w, 0) * dout) with respect to x (NHWC) and to w ([k*k][cout][cin]),
    and the bias gradient (sum of dout over pixels); float64 numpy."""
    x = torch.tensor(np.asarray(x_nhwc, dtype=np.float64)).permute(0, 3, 1, 2).requires_grad_(True)
    wt = torch.tensor(np.asarray(w, dtype=np.float64), requires_grad=True)
    d = torch.tensor(np.asarray(dout_nhwc, dtype=np.float64)).permute(0, 3, 1, 2)
    (conv(x, wt, None, periodic) * d).sum().backward()
    return (x.grad.permute(0, 2, 3, 1).numpy().copy(), wt.grad.numpy().copy(),
            np.asarray(dout_nhwc, dtype=np.float64).sum(axis=(0, 1, 2)))


def forward(x_nhwc, flat, levels, base, in_channels, out_channels, emulate_bf16=False, periodic=False):
    """Network output (N, H, W, out_channels) as a float64 torch tensor.

    emulate_bf16: round the input, the weights and every stored activation (convolution outputs
    after ReLU, pooled tensors) to bf16 as the device stores them; accumulation stays float64 and
    gradients pass through the roundings unchanged.  periodic: every convolution wraps around."""
    def rnd(t):
        if not emulate_bf16:
            return t
        r = torch.as_tensor(bf16_round(t.detach().numpy()), dtype=torch.float64)
        return t + (r - t).detach()  # rounded value; the gradient passes straight through
    params = unpack(flat, levels, base, in_channels, out_channels)
    if emulate_bf16:
        params = [(rnd(w), b) for w, b in params]
    x = torch.as_tensor(np.asarray(x_nhwc, dtype=np.float64)).permute(0, 3, 1, 2)
    h = rnd(x)
    skips = []
    i = 0
    for l in range(levels):
        h = rnd(F.relu(conv(h, *params[i], periodic)))
        h = rnd(F.relu(conv(h, *params[i + 1], periodic)))
        i += 2
        if l < levels - 1:
            skips.append(h)
            h = rnd(F.avg_pool2d(h, 2))
    for l in range(levels - 2, -1, -1):
        up = F.interpolate(h, scale_factor=2, mode="nearest")
        h = torch.cat([up, skips[l]], dim=1)
        h = rnd(F.relu(conv(h, *params[i], periodic)))
        h = rnd(F.relu(conv(h, *params[i + 1], periodic)))
        i += 2
    y = conv(h, *params[i])
    return y.permute(0, 2, 3, 1)[..., :out_channels]


def loss(y, target, mask):
    """sum over mask pixels and channels of (y - target)^2 / (mask count * channels)."""
    m = torch.as_tensor(np.asarray(mask) != 0)
    t = torch.as_tensor(np.asarray(target, dtype=np.float64))
    d = (y - t)[m]
    return (d * d).sum() / (max(int(m.sum()), 1) * y.shape[-1])


def loss_and_grad(x_nhwc, flat, target, mask, levels, base, in_channels, out_channels, emulate_bf16=False,
                  periodic=False):
    """Loss and its gradient with respect to the flat parameter vector (float64; with
    emulate_bf16 the forward values are rounded as in forward(), gradients are not)."""
    p = torch.tensor(np.asarray(flat, dtype=np.float64), requires_grad=True)
    y = forward(x_nhwc, p, levels, base, in_channels, out_channels, emulate_bf16=emulate_bf16, periodic=periodic)
    L = loss(y, target, mask)
    L.backward()
    return float(L), p.grad.numpy().copy()


def adam(w, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam step (step count t >= 1); returns new (w, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def features(solid, links, kn_feature, ax_feature, ay_feature, channels=16):
    """Input features of one lattice (ny, nx, channels): channel 0 the fluid indicator, 1..8
    the distance ratio q of the wall link in each D2Q9 direction (1 where there is none, 0 on
    solid sites), 9..11 the three scalar features, the rest zero."""
    solid = np.asarray(solid) != 0
    ny, nx = solid.shape
    f = np.zeros((ny, nx, channels))
    fluid = (~solid).astype(float)
    f[..., 0] = fluid
    for d in range(1, 9):
        f[..., d] = fluid
    f[..., 9], f[..., 10], f[..., 11] = kn_feature, ax_feature, ay_feature
    for x, y, d, q in zip(links["x"], links["y"], links["dir"], links["q"]):
        if not solid[y, x]:
            f[y, x, d] = q
    return f


def smooth(planes, solid, periodic):
    """One pass of the masked 3 x 3 mean: at each fluid site, the mean of every plane over the fluid
    sites of its neighbourhood (indices modulo the image size if periodic, else inside the image);
    0 on solid sites.  planes: list of (ny, nx) arrays."""
    solid = np.asarray(solid) != 0
    ny, nx = solid.shape
    out = [np.zeros((ny, nx)) for _ in planes]
    for y in range(ny):
        for x in range(nx):
            if solid[y, x]:
                continue
            acc = [0.0] * len(planes)
            cnt = 0
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    yy, xx = y + dy, x + dx
                    if periodic:
                        yy, xx = yy % ny, xx % nx
                    if not (0 <= yy < ny and 0 <= xx < nx) or solid[yy, xx]:
                        continue
                    cnt += 1
                    for c, p in enumerate(planes):
                        acc[c] += p[yy, xx]
            for c in range(len(planes)):
                out[c][y, x] = acc[c] / cnt
    return out


def fields(pred, solid, u_scale, rho_scale, rho0, smooth_iters=0, periodic=False):
    """Initial (rho, ux, uy) from one predicted image (ny, nx, 3): the three channels on fluid
    sites, smoothed smooth_iters times (see smooth), then u = u_scale (t0, t1) and
    rho = rho0 + rho_scale (t2 - its fluid mean) on fluid sites; rho0 and 0 on solid sites."""
    solid = np.asarray(solid) != 0
    pred = np.asarray(pred, dtype=np.float64)
    fl = ~solid
    t = [np.where(fl, pred[..., c], 0.0) for c in range(3)]
    for _ in range(smooth_iters):
        t = smooth(t, solid, periodic)
    mean = t[2][fl].mean() if fl.any() else 0.0
    rho = np.where(fl, rho0 + rho_scale * (t[2] - mean), rho0)
    ux = np.where(fl, u_scale * t[0], 0.0)
    uy = np.where(fl, u_scale * t[1], 0.0)
    return rho, ux, uy
