"""Warm-start network kernels (lbm_conv2d_*, lbm_nn_*) against the CPU oracle (oracle/unet.py).

Inputs are seeded and rounded to bf16 on the host before upload, so both sides see the same
values.  Tolerances:
  * fp32 outputs of one convolution: max |got - ref| <= 1e-5 max |ref| (fp32 accumulation of at
    most 9 * 512 products of bf16 values against fp64);
  * bf16 outputs: the correctly rounded value, or one bf16 unit off when the fp32 sum sits within
    fp32 rounding of a bf16 tie (|got - ref| <= 2^-8 |ref| + 1e-6 max |ref|);
  * the whole network stores each of its ~20 activations in bf16 (relative rounding <= 2^-9);
    against the oracle with the same roundings emulated in fp64 the output differs by
    <= 1e-2 max |ref|, against the exact fp64 network by <= 5e-2 (relative L2);
  * parameter gradients: against the oracle gradient taken through the same bf16 forward
    roundings (straight-through), the only difference left is the bf16 storage of the ~20
    back-propagated gradient tensors: cosine >= 0.9999 and relative L2 <= 2e-2 for every
    convolution.  Against the exact fp64 gradient the forward roundings add to that; first-layer
    weight gradients are sums with much cancellation, so only cosine >= 0.998 is asked there.
"""
import ctypes as C
import sys

import numpy as np
import pytest

from oracle import unet as U
from paper_2012_14707_amd import geometry as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev_bf16(a):
    import torch
    return torch.tensor(U.bf16_round(a), dtype=torch.float32).to(torch.bfloat16).cuda().contiguous()


def _host(t):
    import torch
    return t.to(torch.float32).cpu().numpy().astype(np.float64)


CONV_CASES = [
    # n, h, w, cin, cout, k: ragged pixel tails, several M/N tiles, partial K steps
    (2, 13, 21, 24, 40, 3),
    (1, 64, 64, 64, 128, 3),
    (3, 7, 5, 8, 8, 3),
    (2, 16, 16, 512, 64, 3),
    (2, 19, 11, 96, 32, 1),
    (1, 32, 32, 32, 8, 1),
    # 3x3 halo tiles: 8 x 32 x 32 with one chunk, with a short last chunk and three channel tiles;
    # 8 x 16 x 64 with a short single chunk; 8 x 32 x 64 (enough blocks at batch 4)
    (2, 32, 64, 32, 32, 3),
    (1, 16, 32, 48, 96, 3),
    (2, 16, 64, 16, 64, 3),
    (4, 128, 128, 32, 64, 3),
    # tiles over several chunks: two LDS stages below 512 blocks (8 x 32 x 32 with a short last
    # chunk; two chunks per split of two), one reloaded stage from 512 blocks on (8 x 32 x 32 with
    # three chunks and with a short last chunk, 8 x 32 x 64, 8 x 16 x 64)
    (4, 64, 256, 40, 32, 3),
    (2, 64, 256, 96, 32, 3),
    (8, 64, 256, 96, 32, 3),
    (8, 64, 256, 40, 32, 3),
    (8, 64, 256, 64, 64, 3),
    (8, 64, 144, 64, 64, 3),
    # partial tiles: 40 output channels over 32-channel tiles (and 16-channel weight-gradient
    # groups) with a 24-channel input; 192 output channels over 8 x 16 x 64 tiles with a short last
    # chunk of a 40-channel input
    (1, 16, 32, 24, 40, 3),
    (1, 8, 16, 40, 192, 3),
]


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("case", CONV_CASES)
def test_conv_forward(case, periodic):
    import torch
    from paper_2012_14707_amd import lbm
    n, h, w, cin, cout, k = case
    _say(f"[conv fwd] {case} periodic {periodic}")
    rng = np.random.default_rng(hash(case) % 2 ** 32)
    x = U.bf16_round(rng.normal(size=(n, h, w, cin)))
    wt = U.bf16_round(rng.normal(scale=1 / np.sqrt(k * k * cin), size=(k * k, cout, cin)))
    b = rng.normal(size=cout).astype(np.float32)
    for relu in (False, True):
        out = torch.empty((n, h, w, cout), dtype=torch.bfloat16, device="cuda")
        out32 = torch.empty((n, h, w, cout), dtype=torch.float32, device="cuda")
        lbm.conv2d_forward(_dev_bf16(x), _dev_bf16(wt), torch.tensor(b).cuda(), out, out32, relu=relu,
                           periodic=periodic)
        torch.cuda.synchronize()
        ref = U.conv(torch.tensor(x.astype(np.float64)).permute(0, 3, 1, 2), torch.tensor(wt.astype(np.float64)),
                     torch.tensor(b.astype(np.float64)), periodic).permute(0, 2, 3, 1).numpy()
        if relu:
            ref = np.maximum(ref, 0)
        scale = np.abs(ref).max()
        got32 = out32.cpu().numpy()
        assert np.abs(got32 - ref).max() <= 1e-5 * scale, (case, relu)
        got = _host(out)
        assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-6 * scale), (case, relu)


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("case", CONV_CASES)
def test_conv_gradients(case, periodic):
    import torch
    from paper_2012_14707_amd import lbm
    n, h, w, cin, cout, k = case
    _say(f"[conv grads] {case} periodic {periodic}")
    rng = np.random.default_rng(hash(case) % 2 ** 32 + 1)
    x = U.bf16_round(rng.normal(size=(n, h, w, cin)))
    wt = U.bf16_round(rng.normal(scale=1 / np.sqrt(k * k * cin), size=(k * k, cout, cin)))
    d = U.bf16_round(rng.normal(size=(n, h, w, cout)))
    gx_ref, gw_ref, gb_ref = U.conv_grads(x, wt, d, periodic)
    din = torch.empty((n, h, w, cin), dtype=torch.bfloat16, device="cuda")
    lbm.conv2d_dgrad(_dev_bf16(d), _dev_bf16(wt), din, periodic=periodic)
    dw = torch.empty((k * k, cout, cin), dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    lbm.conv2d_wgrad(_dev_bf16(x), _dev_bf16(d), dw, db, periodic=periodic)
    torch.cuda.synchronize()
    gx = _host(din)
    s = np.abs(gx_ref).max()
    assert np.all(np.abs(gx - gx_ref) <= 2.0 ** -8 * np.abs(gx_ref) + 1e-6 * s), case
    # fp32 sums over n h w pixels (up to 4096 per split) of bf16 products
    assert np.abs(dw.cpu().numpy() - gw_ref).max() <= 1e-5 * np.abs(gw_ref).max(), case
    assert np.abs(db.cpu().numpy() - gb_ref).max() <= 1e-5 * np.abs(gb_ref).max(), case


def test_conv_wgrad_deterministic_and_workspace_checked():
    import torch
    from paper_2012_14707_amd import lbm
    rng = np.random.default_rng(9)
    x = _dev_bf16(rng.normal(size=(4, 64, 64, 32)))
    d = _dev_bf16(rng.normal(size=(4, 64, 64, 32)))
    outs = []
    for _ in range(2):
        dw = torch.empty((9, 32, 32), dtype=torch.float32, device="cuda")
        lbm.conv2d_wgrad(x, d, dw)
        outs.append(dw.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    lib = lbm.load()
    need = C.c_int64()
    assert lib.lbm_conv2d_wgrad_workspace(4, 64, 64, 32, 32, 3, C.byref(need)) == 0
    work = torch.empty(int(need.value) - 1, dtype=torch.float32, device="cuda")
    st = lib.lbm_conv2d_wgrad(C.c_void_p(x.data_ptr()), C.c_void_p(d.data_ptr()), C.c_void_p(dw.data_ptr()), None,
                              C.c_void_p(work.data_ptr()), int(need.value) - 1, 4, 64, 64, 32, 32, 3, 0, None)
    assert st == -1 and "workspace" in lib.lbm_last_error().decode()


def _net_inputs(rng, n, h, w, cin, cout):
    x = np.zeros((n, h, w, (cin + 7) // 8 * 8))
    x[..., :cin] = U.bf16_round(rng.normal(size=(n, h, w, cin)))
    target = rng.normal(size=(n, h, w, cout)).astype(np.float32)
    mask = (rng.random((n, h, w)) < 0.7).astype(np.uint8)
    return x, target, mask


def _seeded_net(rng, L, base, cin, cout, h, w, max_batch, periodic):
    """A network with the device's seeded weights and random non-zero biases (so that they are
    exercised); returns it with its parameters as the oracle takes them."""
    from paper_2012_14707_amd import lbm
    net = lbm.Net(levels=L, base_channels=base, in_channels=cin, out_channels=cout, height=h, width=w,
                  max_batch=max_batch, periodic=periodic, seed=5)
    assert net.n_params == U.param_count(L, base, cin, cout)
    flat = net.get_params().astype(np.float64)
    # the device's seeded initialisation: padded input columns and output rows are zero
    ws = U.unpack(flat, L, base, cin, cout)
    assert np.all(ws[0][0].numpy()[:, :, cin:] == 0) and np.all(ws[-1][0].numpy()[:, cout:, :] == 0)
    off = 0
    for t, ci, co in U.layer_shapes(L, base, cin, cout):
        off += t * ci * co
        flat[off:off + co] = rng.normal(scale=0.05, size=co) * (np.arange(co) < (cout if co == 8 and t == 1 else co))
        off += co
    net.set_params(flat.astype(np.float32))
    return net, flat.astype(np.float32).astype(np.float64)


# (levels, base channels, in, out, batch, height, width, periodic).  The 256^2 network at batch 1
# splits K in most deep layers (pooling and upsampling then take their separate passes below level
# 0); at batch 4 levels 1 and 2 run unsplit with the pooling fused into the convolutions, here with
# zero padding.
@pytest.mark.parametrize("shape", [(3, 16, 12, 3, 2, 32, 48, False), (3, 16, 12, 3, 2, 32, 48, True),
                                   (5, 32, 12, 3, 1, 256, 256, True), (5, 32, 12, 3, 4, 256, 256, False)])
def test_network_forward_and_gradients(shape):
    import torch
    from paper_2012_14707_amd import lbm
    L, base, cin, cout, n, h, w, periodic = shape
    _say(f"[net] {shape}")
    rng = np.random.default_rng(L * 100 + base)
    net, flat = _seeded_net(rng, L, base, cin, cout, h, w, max(n, 2), periodic)
    x, target, mask = _net_inputs(rng, n, h, w, cin, cout)
    y = torch.empty((n, h, w, cout), dtype=torch.float32, device="cuda")
    net.forward(_dev_bf16(x), y)
    loss = net.backward(torch.tensor(target).cuda(), torch.tensor(mask).cuda())
    got = y.cpu().numpy().astype(np.float64)
    emu = U.forward(x, flat, L, base, cin, cout, emulate_bf16=True, periodic=periodic).numpy()
    exact = U.forward(x, flat, L, base, cin, cout, periodic=periodic).numpy()
    e_emu = np.abs(got - emu).max() / np.abs(emu).max()
    e_ex = np.linalg.norm(got - exact) / np.linalg.norm(exact)
    ref_loss, ref_grad = U.loss_and_grad(x, flat, target, mask, L, base, cin, cout, periodic=periodic)
    _, emu_grad = U.loss_and_grad(x, flat, target, mask, L, base, cin, cout, emulate_bf16=True, periodic=periodic)
    grad = net.get_grads().astype(np.float64)
    _say(f"[net] {shape}: forward err vs emulated {e_emu:.2e}, vs exact {e_ex:.2e}; loss {loss:.6e} vs {ref_loss:.6e}")
    off = 0
    worst = 1.0
    stats = []
    for i, (t, ci, co) in enumerate(U.layer_shapes(L, base, cin, cout)):
        m = t * ci * co + co
        g, r, re = grad[off:off + m], ref_grad[off:off + m], emu_grad[off:off + m]
        off += m
        if np.linalg.norm(r) == 0:
            stats.append((i, None))
            continue
        cos = g @ r / (np.linalg.norm(g) * np.linalg.norm(r))
        rel = np.linalg.norm(g - r) / np.linalg.norm(r)
        cos_e = g @ re / (np.linalg.norm(g) * np.linalg.norm(re))
        rel_e = np.linalg.norm(g - re) / np.linalg.norm(re)
        worst = min(worst, cos)
        stats.append((i, round(cos, 6), round(rel, 4), round(cos_e, 6), round(rel_e, 4)))
    for st in stats:
        _say(f"[net] {shape} layer {st}")
    assert e_emu <= 1e-2 and e_ex <= 5e-2
    assert loss == pytest.approx(ref_loss, rel=5e-2)
    for st in stats:
        assert st[1] is None or (st[3] >= 0.9999 and st[4] <= 2e-2 and st[1] >= 0.998), st
    _say(f"[net] {shape}: worst gradient cosine {worst:.6f}")
    net.close()


def test_network_forward_at_the_benchmark_batch():
    """The warm-start network's shape at batch 8, the configuration the benchmark times (its plans
    differ from smaller batches: one reloaded LDS stage at 256^2 and 128^2, no K splits above the
    deepest level), against the oracle network."""
    import torch
    from paper_2012_14707_amd import warmstart as W
    shape = W.NET_SHAPE
    L, base, cin, cout = shape["levels"], shape["base_channels"], shape["in_channels"], shape["out_channels"]
    n, h, w, periodic = 8, W.SIDE, W.SIDE, True
    rng = np.random.default_rng(8)
    net, flat = _seeded_net(rng, L, base, cin, cout, h, w, n, periodic)
    x, _, _ = _net_inputs(rng, n, h, w, cin, cout)
    y = torch.empty((n, h, w, cout), dtype=torch.float32, device="cuda")
    net.forward(_dev_bf16(x), y)
    got = y.cpu().numpy().astype(np.float64)
    emu = U.forward(x, flat, L, base, cin, cout, emulate_bf16=True, periodic=periodic).numpy()
    exact = U.forward(x, flat, L, base, cin, cout, periodic=periodic).numpy()
    e_emu = np.abs(got - emu).max() / np.abs(emu).max()
    e_ex = np.linalg.norm(got - exact) / np.linalg.norm(exact)
    _say(f"[net] batch {n}: forward err vs emulated {e_emu:.2e}, vs exact {e_ex:.2e}")
    assert e_emu <= 1e-2 and e_ex <= 5e-2
    net.close()


def test_adam_step_matches_oracle():
    import torch
    from paper_2012_14707_amd import lbm
    L, base, cin, cout, n, h, w = 2, 8, 3, 2, 2, 16, 16
    rng = np.random.default_rng(4)
    net = lbm.Net(levels=L, base_channels=base, in_channels=cin, out_channels=cout, height=h, width=w, max_batch=2,
                  seed=1)
    x, target, mask = _net_inputs(rng, n, h, w, cin, cout)
    wv = net.get_params().astype(np.float64)
    m = np.zeros_like(wv)
    v = np.zeros_like(wv)
    for t in (1, 2, 3):
        net.forward(_dev_bf16(x))
        net.backward(torch.tensor(target).cuda(), torch.tensor(mask).cuda())
        g = net.get_grads().astype(np.float64)
        net.adam_step(1e-3, 0.9, 0.999, 1e-8)
        wv, m, v = U.adam(wv, m, v, g, t, 1e-3)
        got = net.get_params().astype(np.float64)
        assert np.abs(got - wv).max() <= 1e-6 * max(np.abs(wv).max(), 1.0), t
        wv = got  # continue from the device's fp32 values


def test_training_overfits_one_batch():
    import torch
    from paper_2012_14707_amd import lbm
    rng = np.random.default_rng(8)
    net = lbm.Net(levels=3, base_channels=16, in_channels=12, out_channels=3, height=32, width=32, max_batch=2,
                  seed=2)
    x, _, mask = _net_inputs(rng, 2, 32, 32, 12, 3)
    yy, xx = np.mgrid[0:32, 0:32] / 32.0
    target = np.stack([np.sin(2 * np.pi * yy), np.cos(2 * np.pi * xx), yy * xx], -1)[None].repeat(2, 0)
    target = target.astype(np.float32)
    xd, td, md = _dev_bf16(x), torch.tensor(target).cuda(), torch.tensor(mask).cuda()
    losses = []
    for it in range(300):
        net.forward(xd)
        losses.append(net.backward(td, md))
        net.adam_step(2e-3)
    _say(f"[overfit] loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert np.isfinite(losses).all() and losses[-1] < 0.05 * losses[0]


def _links_dev(links):
    import torch
    from paper_2012_14707_amd import lbm
    arr, n = lbm.make_links(links)
    raw = np.frombuffer(C.string_at(C.addressof(arr), C.sizeof(arr)), dtype=np.uint8).copy()
    return torch.tensor(raw).cuda(), n


def test_features_match_oracle():
    import torch
    from paper_2012_14707_amd import lbm
    for pb in (G.poiseuille_config1(), G.random_cylinders(n=64, porosity=0.75, rmin=4, rmax=9, seed=3, kn=0.05,
                                                          h=26.0, ax=1e-6)):
        solid = np.ascontiguousarray(pb["solid"], np.uint8)
        ny, nx = solid.shape
        links, nl = _links_dev(pb["links"])
        out = torch.full((ny, nx, 16), 7.0, dtype=torch.bfloat16, device="cuda")
        lbm.nn_features(torch.tensor(solid).cuda(), links, nx, ny, -0.25, 0.8, -0.6, out)
        torch.cuda.synchronize()
        ref = U.bf16_round(U.features(solid, pb["links"], -0.25, 0.8, -0.6).astype(np.float32))
        assert np.array_equal(out.to(torch.float32).cpu().numpy(), ref)


@pytest.mark.parametrize("smooth_iters,periodic", [(0, False), (3, True), (2, False)])
def test_fields_match_oracle(smooth_iters, periodic):
    import torch
    from paper_2012_14707_amd import lbm
    rng = np.random.default_rng(6)
    solid = (rng.random((37, 53)) < 0.35).astype(np.uint8)
    pred = rng.normal(size=(37, 53, 3)).astype(np.float32)
    rho, ux, uy = (torch.empty(37 * 53, dtype=torch.float64, device="cuda") for _ in range(3))
    bad = lbm.nn_fields(torch.tensor(pred).cuda(), torch.tensor(solid).cuda(), 53, 37, 2e-3, 5e-4, 1.0, rho, ux, uy,
                        smooth_iters=smooth_iters, periodic=periodic)
    assert bad == 0
    r_ref, ux_ref, uy_ref = U.fields(pred, solid, 2e-3, 5e-4, 1.0, smooth_iters, periodic)
    # fp64 sums in the same order; the mean over fluid sites is reduced in another order
    assert np.allclose(rho.cpu().numpy().reshape(37, 53), r_ref, rtol=0, atol=1e-15)
    assert np.allclose(ux.cpu().numpy().reshape(37, 53), ux_ref, rtol=1e-14, atol=0)
    assert np.allclose(uy.cpu().numpy().reshape(37, 53), uy_ref, rtol=1e-14, atol=0)
    pred[3, 4, 1] = np.nan
    pred[5, 6, 2] = np.inf
    solid[3, 4] = 0
    solid[5, 6] = 0
    bad = lbm.nn_fields(torch.tensor(pred).cuda(), torch.tensor(solid).cuda(), 53, 37, 2e-3, 5e-4, 1.0, rho, ux, uy,
                        smooth_iters=smooth_iters, periodic=periodic)
    assert bad >= 2
