"""Learned warm start for steady porous-media flow (not part of the paper).

A convolutional encoder-decoder (lbm.Net, liblbm's lbm_nn_* kernels) predicts the steady
velocity and density deviation of a 256 x 256 random-cylinder lattice from its problem statement
(mask, distance ratios q, Kn, force direction).  The lattice starts from f^eq(rho, u) of the
prediction instead of rest and then runs the unchanged method to the same residual, so the
converged field is the lattice's own; the rest start is both the fallback (non-finite prediction,
non-finite or growing residual) and the yardstick.

Workload: random non-overlapping cylinders on a doubly periodic 256^2 lattice, porosity
U[0.6, 0.9], radii U[6, 20] lu, Kn log-uniform in [0.005, 0.1], H = 26, body force a_x
log-uniform in [1e-6, 1e-5] along x; training seeds 1000-2999, test seeds 9000-9199.

Normalisation: Stokes flow is linear in the force and, by Darcy's law, proportional to the
permeability, so velocities are divided by a K / nu and density deviations by 3 a sqrt(K), with K a
Kozeny-Carman estimate from the mask and the link table; each is then divided by a gain fixed on
the training set so that the network's targets have unit RMS over fluid sites.  The network
convolutions wrap around (the domains are doubly periodic).

Run ``python -m paper_2012_14707_amd.warmstart --help`` for the command line (data generation,
training, evaluation).
"""
import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

from . import geometry as G
from . import lbm

SIDE = 256
H_REF = 26.0
IN_CHANNELS = 12
IN_PAD = 16
OUT_CHANNELS = 3
NET_SHAPE = dict(levels=5, base_channels=32, in_channels=IN_CHANNELS, out_channels=OUT_CHANNELS, height=SIDE,
                 width=SIDE, periodic=True)
TRAIN_SEEDS = range(1000, 3000)
TEST_SEEDS = range(9000, 9200)
# Passes of the masked 3 x 3 mean applied to the prediction before it initialises the lattice: the
# network's pixel-scale error (and the bf16 rounding of its activations) would otherwise excite
# grid-scale oscillations of the populations that keep the step-to-step residual up.
SMOOTH_ITERS = 4
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(HERE, "weights", "warmstart_256.npz")


def instance(seed):
    """One warm-start problem: parameters drawn from a stream of its own, placement from `seed`."""
    rng = np.random.default_rng([int(seed), 5])
    porosity = rng.uniform(0.6, 0.9)
    kn = math.exp(rng.uniform(math.log(0.005), math.log(0.1)))
    ax = math.exp(rng.uniform(math.log(1e-6), math.log(1e-5)))
    pb = G.random_cylinders(n=SIDE, porosity=porosity, rmin=6.0, rmax=20.0, seed=int(seed), kn=kn, h=H_REF, ax=ax)
    pb["meta"] = {"kind": "warmstart", "seed": int(seed), "porosity": float(pb["meta"]["porosity"]), "kn": kn,
                  "ax": ax}
    return pb


def instances(seeds, workers=8):
    seeds = list(seeds)
    if workers <= 1 or len(seeds) < 8:
        return [instance(s) for s in seeds]
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(instance, seeds, chunksize=8)


def force(pb):
    p = pb["params"]
    return float(p.get("ax", 0.0)), float(p.get("ay", 0.0))


def feature_scalars(pb):
    """(kn feature, ax feature, ay feature): log10(Kn) + 2 and the unit force direction."""
    ax, ay = force(pb)
    a = math.hypot(ax, ay)
    return math.log10(pb["params"]["kn"]) + 2.0, (ax / a if a else 0.0), (ay / a if a else 0.0)


# Wall links per unit length of wall: a circle of radius R has about 19.3 R links (D2Q9, all
# eight directions) against its perimeter 2 pi R.
LINKS_PER_WALL_LENGTH = 19.3 / (2.0 * math.pi)
KOZENY_CONSTANT = 5.0


def permeability_estimate(pb):
    """Kozeny-Carman permeability phi^3 / (c S^2) from the mask (porosity phi) and the link table
    (wall length per unit area S)."""
    solid = np.asarray(pb["solid"]) != 0
    phi = 1.0 - solid.mean()
    s = len(pb["links"]["q"]) / LINKS_PER_WALL_LENGTH / solid.size
    return phi ** 3 / (KOZENY_CONSTANT * max(s, 1e-12) ** 2)


def reference_scales(pb, nu):
    """(velocity scale a K / nu, density scale 3 a sqrt(K)) of a problem, K the Kozeny-Carman
    permeability estimate: Darcy's law for the velocity and the force balance over a pore for
    the pressure, whose deviation is c_s^2 = 1/3 times the density's."""
    a = math.hypot(*force(pb))
    k = permeability_estimate(pb)
    return a * k / nu, 3.0 * a * math.sqrt(k)


def _links_device(pb):
    import ctypes as C
    import torch
    arr, n = lbm.make_links(pb["links"])
    if n == 0:
        return None
    raw = np.frombuffer(C.string_at(C.addressof(arr), n * C.sizeof(lbm.Link)), dtype=np.uint8)
    return torch.from_numpy(raw.copy()).cuda()


def features_into(pb, out):
    """Rasterises one problem's features into out (bf16 device [SIDE, SIDE, IN_PAD]) with lbm_nn_features."""
    import torch
    solid = torch.from_numpy(np.ascontiguousarray(pb["solid"], np.uint8)).cuda()
    ny, nx = pb["solid"].shape
    lbm.nn_features(solid, _links_device(pb), nx, ny, *feature_scalars(pb), out)
    return solid


class Model:
    """Trained network plus its output gains."""

    def __init__(self, net, u_gain=1.0, rho_gain=1.0):
        self.net = net
        self.u_gain = float(u_gain)
        self.rho_gain = float(rho_gain)

    @classmethod
    def create(cls, max_batch=8, seed=0):
        return cls(lbm.Net(**NET_SHAPE, max_batch=max_batch, seed=seed))

    def save(self, path):
        """Weights are stored in bf16 (the precision the forward pass uses), biases in fp32."""
        p = self.net.get_params()
        is_bias = _bias_mask(self.net.n_params)
        bits = p.view(np.uint32)
        rounded = ((bits.astype(np.uint64) + 0x7FFF + ((bits >> 16) & 1)) >> 16).astype(np.uint16)
        np.savez(path, weights_bf16=rounded[~is_bias], biases=p[is_bias], u_gain=self.u_gain,
                 rho_gain=self.rho_gain, shape=json.dumps(NET_SHAPE))

    @classmethod
    def load(cls, path=DEFAULT_MODEL, max_batch=1):
        z = np.load(path, allow_pickle=False)
        if json.loads(str(z["shape"])) != NET_SHAPE:
            raise ValueError(f"{path}: network shape differs from {NET_SHAPE}")
        net = lbm.Net(**NET_SHAPE, max_batch=max_batch)
        is_bias = _bias_mask(net.n_params)
        p = np.zeros(net.n_params, np.float32)
        p[~is_bias] = (z["weights_bf16"].astype(np.uint32) << 16).view(np.float32)
        p[is_bias] = z["biases"]
        net.set_params(p)
        return cls(net, float(z["u_gain"]), float(z["rho_gain"]))

    def predict(self, pb, nu, rho0=1.0):
        """Initial (rho, ux, uy) float64 device tensors [ny, nx] and the count of non-finite
        predictions (the caller falls back to rest when it is non-zero)."""
        import torch
        x = torch.empty((1, SIDE, SIDE, IN_PAD), dtype=torch.bfloat16, device="cuda")
        solid = features_into(pb, x[0])
        y = torch.empty((1, SIDE, SIDE, OUT_CHANNELS), dtype=torch.float32, device="cuda")
        self.net.forward(x, y)
        us, rs = reference_scales(pb, nu)
        rho, ux, uy = (torch.empty((SIDE, SIDE), dtype=torch.float64, device="cuda") for _ in range(3))
        bad = lbm.nn_fields(y, solid, SIDE, SIDE, us * self.u_gain, rs * self.rho_gain, rho0, rho, ux, uy,
                            smooth_iters=SMOOTH_ITERS, periodic=True)
        return rho, ux, uy, bad


def _bias_mask(n_params):
    """True at the bias entries of the parameter vector (layout of lbm_nn_create)."""
    m = np.zeros(n_params, bool)
    off = 0
    c = NET_SHAPE["base_channels"]
    L = NET_SHAPE["levels"]
    shapes = []
    for l in range(L):
        shapes += [(9, IN_PAD if l == 0 else c << (l - 1), c << l), (9, c << l, c << l)]
    for l in range(L - 2, -1, -1):
        shapes += [(9, (c << (l + 1)) + (c << l), c << l), (9, c << l, c << l)]
    shapes.append((1, c, 8))
    for t, ci, co in shapes:
        off += t * ci * co
        m[off:off + co] = True
        off += co
    assert off == n_params
    return m


def forward_flops(shape=None, batch=1):
    """Multiply-add count x 2 of one forward pass (padded channels included, as computed)."""
    shape = shape or NET_SHAPE
    c, L = shape["base_channels"], shape["levels"]
    cin0 = (shape["in_channels"] + 7) // 8 * 8
    total = 0
    for l in range(L):
        px = (shape["height"] >> l) * (shape["width"] >> l)
        total += 2 * px * 9 * ((cin0 if l == 0 else c << (l - 1)) + (c << l)) * (c << l)
        if l < L - 1:
            total += 2 * px * 9 * ((c << (l + 1)) + 2 * (c << l)) * (c << l)
    total += 2 * shape["height"] * shape["width"] * c * 8
    return total * batch


# ------------------------------------------------------------------------------------ data

def generate(problems, tol=1e-8, check_every=100, max_steps=400_000, chunk=128, precision="fp64", log=print):
    """Steady fields of every problem from the batched solver (rest start, residual <= tol).

    Returns dict with device tensors x (bf16 features [N, SIDE, SIDE, IN_PAD]), t (fp32
    normalised targets [N, SIDE, SIDE, 3], before the gains), m (uint8 fluid masks [N, SIDE, SIDE]) and
    host lists status / steps / nu."""
    import torch
    n = len(problems)
    x = torch.empty((n, SIDE, SIDE, IN_PAD), dtype=torch.bfloat16, device="cuda")
    t = torch.empty((n, SIDE, SIDE, OUT_CHANNELS), dtype=torch.float32, device="cuda")
    m = torch.empty((n, SIDE, SIDE), dtype=torch.uint8, device="cuda")
    status, steps, nus = [], [], []
    t0 = time.perf_counter()
    for c0 in range(0, n, chunk):
        pbs = problems[c0:c0 + chunk]
        b = lbm.Batch(pbs, precision=precision)
        b.set_launch(block=256, graph_steps=50, blocks_per_cu=4)
        st, sp, _ = b.solve(tol, check_every=check_every, max_steps=max_steps)
        for i, pb in enumerate(pbs):
            k = c0 + i
            rho, ux, uy = b.moments_host(i)
            nu = b.info(i)["nu"]
            us, rs = reference_scales(pb, nu)
            fl = pb["solid"] == 0
            drho = np.where(fl, rho - pb["params"].get("rho0", 1.0), 0.0)
            drho = np.where(fl, drho - drho[fl].mean(), 0.0)
            tgt = np.stack([ux / us, uy / us, drho / rs], -1).astype(np.float32)
            t[k] = torch.from_numpy(tgt)
            m[k] = torch.from_numpy(fl.astype(np.uint8))
            features_into(pb, x[k])
            status.append(st[i])
            steps.append(int(sp[i]))
            nus.append(nu)
        b.close()
        log(f"[data] {min(c0 + chunk, n)}/{n} solved ({time.perf_counter() - t0:.1f} s); chunk steps "
            f"min {int(sp.min())} median {int(np.median(sp))} max {int(sp.max())}; "
            f"statuses {dict((s, st.count(s)) for s in set(st))}")
    return dict(x=x, t=t, m=m, status=status, steps=steps, nu=nus)


def target_gains(data):
    """RMS over fluid sites of the normalised velocity and density targets."""
    t, m = data["t"], data["m"].bool()
    u = t[..., :2][m]
    r = t[..., 2][m]
    return float(u.pow(2).mean().sqrt()), float(r.pow(2).mean().sqrt())


def _masked_mse(y, t, m):
    mm = m.bool()
    d = (y - t)[mm]
    return float(d.pow(2).mean())


# Mirrors of the feature channels: y -> -y swaps the link directions N<->S, NE<->SE, NW<->SW;
# x -> -x swaps E<->W, NE<->NW, SE<->SW.
_YFLIP_CHANNELS = [0, 1, 4, 3, 2, 8, 7, 6, 5, 9, 10, 11, 12, 13, 14, 15]
_XFLIP_CHANNELS = [0, 3, 2, 1, 4, 6, 5, 8, 7, 9, 10, 11, 12, 13, 14, 15]


def augment(x, t, m, rng, xflip=True):
    """A random symmetry of the doubly periodic problem class applied to a batch: a periodic
    shift; with probability 1/2 the mirror y -> -y (u_y and a_y change sign); and, if xflip,
    with probability 1/2 the mirror x -> -x combined with reversing the force, which by the
    linearity of creeping flow leaves a_x and u_x as they are and changes the sign of u_y and
    of the density deviation (exact for Stokes flow, approximate at the small Reynolds numbers
    of the workload)."""
    import torch
    dy, dx = (int(v) for v in rng.integers(0, SIDE, 2))
    x, t, m = (torch.roll(a, shifts=(dy, dx), dims=(1, 2)) for a in (x, t, m))
    if rng.random() < 0.5:
        idx = torch.tensor(_YFLIP_CHANNELS, device=x.device)
        x = torch.flip(x, dims=(1,)).index_select(3, idx)
        x[..., 11] = -x[..., 11]
        t = torch.flip(t, dims=(1,)) * torch.tensor([1.0, -1.0, 1.0], device=t.device)
        m = torch.flip(m, dims=(1,))
    if xflip and rng.random() < 0.5:
        idx = torch.tensor(_XFLIP_CHANNELS, device=x.device)
        x = torch.flip(x, dims=(2,)).index_select(3, idx)
        x[..., 11] = -x[..., 11]
        t = torch.flip(t, dims=(2,)) * torch.tensor([1.0, -1.0, -1.0], device=t.device)
        m = torch.flip(m, dims=(2,))
    return x.contiguous(), t.contiguous(), m.contiguous()


def train(data, test=None, epochs=30, batch=8, lr=1e-3, lr_final=2e-5, seed=0, augment_data=True, xflip=True,
          log=print):
    """Adam on the masked squared error of the gain-normalised targets; cosine learning-rate decay."""
    import torch
    model = Model.create(max_batch=batch, seed=seed)
    model.u_gain, model.rho_gain = target_gains(data)
    gain = torch.tensor([model.u_gain, model.u_gain, model.rho_gain], device="cuda")
    n = data["x"].shape[0]
    iters = epochs * (n // batch)
    rng = np.random.default_rng(seed)
    it = 0
    t0 = time.perf_counter()
    history = []
    for ep in range(epochs):
        order = rng.permutation(n)
        losses = []
        for b0 in range(0, n - batch + 1, batch):
            idx = torch.from_numpy(order[b0:b0 + batch]).cuda()
            xb = data["x"].index_select(0, idx)
            tb = (data["t"].index_select(0, idx) / gain).contiguous()
            mb = data["m"].index_select(0, idx)
            if augment_data:
                xb, tb, mb = augment(xb, tb, mb, rng, xflip)
            model.net.forward(xb)
            losses.append(model.net.backward(tb, mb))
            cur = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * it / max(iters, 1)))
            model.net.adam_step(cur)
            it += 1
        rec = dict(epoch=ep + 1, train_loss=float(np.mean(losses)), seconds=time.perf_counter() - t0)
        if test is not None:
            rec["test_loss"] = evaluate_loss(model, test)
        history.append(rec)
        log(f"[train] epoch {ep + 1}/{epochs} " + " ".join(f"{k} {v:.4g}" for k, v in rec.items() if k != "epoch"))
    return model, history


def evaluate_loss(model, data, batch=None):
    """Masked MSE of the gain-normalised prediction over a dataset (no parameter change)."""
    import torch
    batch = batch or model.net.cfg.max_batch
    gain = torch.tensor([model.u_gain, model.u_gain, model.rho_gain], device="cuda")
    n = data["x"].shape[0]
    tot, cnt = 0.0, 0
    for b0 in range(0, n, batch):
        xb = data["x"][b0:b0 + batch].contiguous()
        y = torch.empty((xb.shape[0], SIDE, SIDE, OUT_CHANNELS), dtype=torch.float32, device="cuda")
        model.net.forward(xb, y)
        mm = data["m"][b0:b0 + batch].bool()
        d = (y - data["t"][b0:b0 + batch] / gain)[mm]
        tot += float(d.pow(2).sum())
        cnt += int(d.numel())
    return tot / max(cnt, 1)


# ------------------------------------------------------------------------------------ solve

def solve(pb, model=None, tol=1e-8, check_every=100, max_steps=1_000_000, precision="fp64", growth=10.0,
          lattice=None, neq=True):
    """Runs one problem to residual <= tol from rest (model None) or from the model's prediction.

    The predicted (rho, u) become f^eq plus, with neq, the first-order non-equilibrium stress of the
    predicted velocity gradients (lbm_init_fields_neq), which a steady flow carries.

    Wall time covers everything after the lattice exists: for a warm start the upload of mask and
    links, features, the forward pass, the fields, the initialisation, and every step and residual
    check.  Fallback to rest (then counted in the same wall time and steps): a non-finite
    prediction, a non-finite residual, or a residual more than `growth` times above the first
    one after the warm start.  Returns (dict of results, lattice)."""
    import torch
    lat = lattice or lbm.Lattice(pb, precision=precision)
    rho0 = float(pb["params"].get("rho0", 1.0))
    nu = lat.info["nu"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fallback = None
    warm = model is not None
    if warm:
        rho, ux, uy, bad = model.predict(pb, nu, rho0)
        if bad:
            fallback = "non-finite prediction"
            warm = False
            lat.init_rest()
        else:
            lat.init_fields(rho, ux, uy, neq=neq)
    else:
        lat.init_rest()
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    steps = 0
    first = None
    res = math.inf
    while steps < max_steps:
        lat.step(check_every)
        steps += check_every
        res, _ = lat.residual(raise_unstable=False)
        if warm and (not math.isfinite(res) or (first is not None and res > growth * first)):
            fallback = "non-finite residual" if not math.isfinite(res) else "growing residual"
            warm = False
            lat.init_rest()
            first = None
            continue
        if warm and first is None:
            first = res
        if not math.isfinite(res):
            break
        if res <= tol:
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return dict(steps=steps, wall=wall, init=t_init, residual=res, fallback=fallback, converged=res <= tol), lat


def compare(pb, model, tol=1e-8, check_every=100, max_steps=1_000_000, precision="fp64", neq=True, also_feq=False):
    """Rest and warm solves of one problem, and the difference of their converged velocities.
    With also_feq, a third solve starts from the prediction's f^eq alone (warm_feq_* entries)."""
    rest, lat = solve(pb, None, tol, check_every, max_steps, precision)
    _, ux_r, uy_r = lat.moments_host()
    extra = {}
    if also_feq:
        feq, lat = solve(pb, model, tol, check_every, max_steps, precision, lattice=lat, neq=False)
        extra = dict(warm_feq_steps=feq["steps"], warm_feq_wall=feq["wall"])
    warm, lat = solve(pb, model, tol, check_every, max_steps, precision, lattice=lat, neq=neq)
    _, ux_w, uy_w = lat.moments_host()
    lat.close()
    umax = max(np.abs(ux_r).max(), np.abs(uy_r).max())
    diff = max(np.abs(ux_w - ux_r).max(), np.abs(uy_w - uy_r).max()) / umax
    return dict(seed=pb["meta"].get("seed"), kn=pb["params"]["kn"], porosity=pb["meta"].get("porosity"),
                rest_steps=rest["steps"], rest_wall=rest["wall"], warm_steps=warm["steps"], warm_wall=warm["wall"],
                warm_init=warm["init"], fallback=warm["fallback"], converged=rest["converged"] and warm["converged"],
                u_rel_diff=diff, **extra)


def summarize(rows):
    rs = np.array([r["rest_steps"] for r in rows], float)
    ws = np.array([r["warm_steps"] for r in rows], float)
    rw = np.array([r["rest_wall"] for r in rows])
    ww = np.array([r["warm_wall"] for r in rows])
    ratio = ws / rs
    wr = ww / rw
    out = dict(n=len(rows), rest_steps_median=float(np.median(rs)), warm_steps_median=float(np.median(ws)),
               warm_init_ms_median=float(np.median([r.get("warm_init", 0.0) for r in rows]) * 1e3),
               step_ratio_median=float(np.median(ratio)), step_ratio_mean=float(ratio.mean()),
               step_ratio_worst=float(ratio.max()), wall_ratio_median=float(np.median(wr)),
               wall_ratio_mean=float(wr.mean()), wall_ratio_worst=float(wr.max()),
               rest_wall_total=float(rw.sum()), warm_wall_total=float(ww.sum()),
               fallbacks=sum(r["fallback"] is not None for r in rows),
               all_converged=all(r["converged"] for r in rows),
               u_rel_diff_max=float(max(r["u_rel_diff"] for r in rows)))
    if all("warm_feq_steps" in r for r in rows):
        fr = np.array([r["warm_feq_steps"] for r in rows], float) / rs
        out.update(feq_init_step_ratio_median=float(np.median(fr)), feq_init_step_ratio_worst=float(fr.max()))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="warm-start data generation, training and evaluation")
    ap.add_argument("--train", type=int, default=len(TRAIN_SEEDS), help="training instances (seeds from 1000)")
    ap.add_argument("--test", type=int, default=len(TEST_SEEDS), help="test instances (seeds from 9000)")
    ap.add_argument("--eval", type=int, default=None, help="test instances solved warm vs rest (default: --test)")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-steps", type=int, default=400_000)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--model", default=None, help="load this model instead of training")
    ap.add_argument("--out", default="gpurun_out/warmstart", help="output folder")
    args = ap.parse_args(argv)

    import torch
    os.makedirs(args.out, exist_ok=True)

    def log(*a):
        print(*a, flush=True)

    t0 = time.perf_counter()
    test_pbs = instances(TEST_SEEDS[:args.test], args.workers)
    log(f"[ws] {len(test_pbs)} test problems built ({time.perf_counter() - t0:.1f} s)")
    report = dict(config=dict(vars(args)))
    if args.model:
        model = Model.load(args.model, max_batch=args.batch)
        test = generate(test_pbs, args.tol, max_steps=args.max_steps, log=log) if args.test else None
    else:
        train_pbs = instances(TRAIN_SEEDS[:args.train], args.workers)
        log(f"[ws] {len(train_pbs)} training problems built ({time.perf_counter() - t0:.1f} s)")
        data = generate(train_pbs, args.tol, max_steps=args.max_steps, log=log)
        del train_pbs
        test = generate(test_pbs, args.tol, max_steps=args.max_steps, log=log) if args.test else None
        report["data"] = dict(train_steps_median=float(np.median(data["steps"])),
                              train_statuses={s: data["status"].count(s) for s in set(data["status"])},
                              seconds=time.perf_counter() - t0)
        model, hist = train(data, test, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
        report["train"] = hist
        model.save(os.path.join(args.out, "warmstart_256.npz"))
        log(f"[ws] model saved; gains u {model.u_gain:.4g} rho {model.rho_gain:.4g}")
        del data
        torch.cuda.empty_cache()
    if test is not None:
        report["test_loss"] = evaluate_loss(model, test)
        report["test_loss_zero_prediction"] = evaluate_loss(_ZeroModel(model), test)
        log(f"[ws] test loss {report['test_loss']:.4g} (zero prediction {report['test_loss_zero_prediction']:.4g})")
        del test
    rows = []
    n_eval = args.test if args.eval is None else args.eval
    model1 = model
    for k, pb in enumerate(test_pbs[:n_eval]):
        r = compare(pb, model1, args.tol, max_steps=args.max_steps)
        rows.append(r)
        log(f"[eval] {k + 1}/{n_eval} seed {r['seed']} Kn {r['kn']:.4f} rest {r['rest_steps']} steps "
            f"{r['rest_wall']:.3f} s, warm {r['warm_steps']} steps {r['warm_wall']:.3f} s, fallback {r['fallback']}, "
            f"du {r['u_rel_diff']:.1e}")
    if rows:
        report["eval"] = summarize(rows)
        report["rows"] = rows
        log("[ws] " + json.dumps(report["eval"]))
    with open(os.path.join(args.out, "report.json"), "w") as f:
        json.dump(report, f, indent=1)
    return report


class _ZeroModel:
    """Baseline for the test loss: predicts zero everywhere (what the rest start amounts to)."""

    def __init__(self, model):
        self.u_gain, self.rho_gain = model.u_gain, model.rho_gain

        class _N:
            cfg = model.net.cfg

            @staticmethod
            def forward(x, y):
                y.zero_()
        self.net = _N()


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
