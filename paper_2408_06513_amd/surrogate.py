"""The learned surrogate of the iterated regularisation.

A five-level convolutional U-Net (channels 32/64/128/256/256, two 3x3
convolutions with ReLU per level, 2x2 average pooling, nearest upsampling,
concatenated skips, a 1x1 output convolution) maps the smoothed density of a
point set to the displacement that `iters` iterations of the method on a
res x res raster give the texel centres of a net_res x net_res lattice (the
composite map of Sec. 4.3 minus the identity, in 1/64 of the unit square).
The samples are then moved by one bilinear advection of that field.  With
net_res < res the network sees a coarser raster than the method (its
Gaussian radius scaled by net_res / res): the composite map is smooth on the
scale of the method's Gaussian, a coarse field captures it at a sixteenth
of the work for res / net_res = 4, and bilinear interpolation of a
fold-free coarse lattice of convex cells cannot fold between its nodes.
It is trained on fields that the method itself computes, and the method
remains the reference and the fallback: a prediction whose deformed
lattice folds, or that does not make the samples more uniform, is replaced by
the plain regularisation.

Every layer runs in the HIP kernels of libinim.so (BF16 matrix-core
convolutions with FP32 accumulation; include/inim_nn.h); PyTorch only holds
the device memory.  Weights are kept in FP32 (updated by Adam) with BF16
copies for the convolutions.
"""
from __future__ import annotations

import math
import os
import time

import numpy as np
import torch

from . import capi, datagen, nn

# The trained network of the 256 x 256, 8-iteration configuration (5 levels,
# 32-256 channels, first-step input, 64 x 64 output lattice; bfloat16 weights),
# written by UNet.save after 10,000 Adam steps of 16 on 50,000 method-labelled
# point sets (seeds 0..49999 of datagen.surrogate_mixture).
C5_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "surrogate_256_field64.npz")
C5_TRAINING = {"train_sets": 50000, "train_steps": 10000, "batch": 16, "lr": 1e-3}

BF16, F32 = torch.bfloat16, torch.float32
CIN, COUT = 8, 8  # input channel 0 = relative density; output channels 0, 1 = displacement


def conv_shapes(chans=(32, 64, 128, 256, 256), out_level: int = 0):
    """(name, cin, cout, ks) of every convolution in forward order.  The
    decoder climbs back to level `out_level` (0: the input's resolution;
    2: a quarter of it along each axis), where the 1x1 head sits."""
    out, prev = [], CIN
    for lvl, c in enumerate(chans):
        out += [(f"e{lvl}a", prev, c, 3), (f"e{lvl}b", c, c, 3)]
        prev = c
    for lvl in range(len(chans) - 2, out_level - 1, -1):
        c = chans[lvl]
        out += [(f"d{lvl}a", prev + c, c, 3), (f"d{lvl}b", c, c, 3)]
        prev = c
    out.append(("head", prev, COUT, 1))
    return out


class Conv:
    def __init__(self, name, cin, cout, ks, w32: torch.Tensor, dev):
        self.name, self.cin, self.cout, self.ks = name, cin, cout, ks
        self.w = w32.to(dev).contiguous()
        self.b = torch.zeros(cout, dtype=F32, device=dev)
        self.w16 = torch.empty(self.w.shape, dtype=BF16, device=dev)
        self.wT = torch.empty((cin, ks * ks, cout), dtype=BF16, device=dev)
        self.gw, self.gb = torch.zeros_like(self.w), torch.zeros_like(self.b)
        self.mw, self.vw = torch.zeros_like(self.w), torch.zeros_like(self.w)
        self.mb, self.vb = torch.zeros_like(self.b), torch.zeros_like(self.b)
        self.refresh()

    def refresh(self):
        nn.to_bf16(self.w, self.w16)
        nn.weight_transpose(self.w16, self.wT)

    def step(self, t, lr):
        nn.adam(self.w, self.gw, self.mw, self.vw, t, lr=lr, w16=self.w16)
        nn.adam(self.b, self.gb, self.mb, self.vb, t, lr=lr)
        nn.weight_transpose(self.w16, self.wT)


class UNet:
    """The network on one device; forward() keeps what backward() needs.
    out_level > 0 ends the decoder at level out_level: the output then has
    1 / 2^out_level of the input's resolution along each axis."""

    def __init__(self, dev, seed: int = 0, chans=(32, 64, 128, 256, 256), out_level: int = 0,
                 first_step: bool = False):
        if not 0 <= out_level < len(chans):
            raise ValueError("out_level must name a level of the network")
        self.dev, self.chans, self.levels, self.out_level = dev, tuple(chans), len(chans), int(out_level)
        # first_step: the input also holds the displacement of one iteration of
        # the method on the network's raster (channels 1 and 2)
        self.first_step = bool(first_step)
        g = np.random.Generator(np.random.PCG64(seed))
        self.convs = {}
        for name, ci, co, ks in conv_shapes(chans, out_level):
            std = math.sqrt((2.0 if name != "head" else 1.0) / (ci * ks * ks))
            w = torch.tensor(g.standard_normal((co, ks * ks, ci)) * std, dtype=F32)
            self.convs[name] = Conv(name, ci, co, ks, w, dev)
        self.t = 0
        self._work = None

    def params_f64(self) -> dict:
        """The FP32 master weights as FP64 CPU tensors (for the oracle)."""
        out = {}
        for k, c in self.convs.items():
            out[k + ".w"] = c.w.detach().double().cpu()
            out[k + ".b"] = c.b.detach().double().cpu()
        return out

    # ------------------------------------------------------------------ forward
    def _work_for(self, c: Conv, n, h, w):
        need = nn.conv_workspace(n, h, w, c.cin, c.cout, c.ks)
        if self._work is None or self._work.numel() < need:
            self._work = torch.empty(need, dtype=torch.uint8, device=self.dev)
        return self._work

    def _conv(self, name, x, relu=True, out32=False):
        c = self.convs[name]
        n, h, w, _ = x.shape
        work = self._work_for(c, n, h, w)
        if out32:
            y = torch.empty((n, h, w, c.cout), dtype=F32, device=self.dev)
            nn.conv_forward(x, c.w16, c.b, relu, y32=y, work=work)
        else:
            y = torch.empty((n, h, w, c.cout), dtype=BF16, device=self.dev)
            nn.conv_forward(x, c.w16, c.b, relu, y16=y, work=work)
        return y

    def forward(self, x16: torch.Tensor) -> torch.Tensor:
        """x16 [n, H, W, 8] bf16 -> [n, H / 2^out_level, W / 2^out_level, 8] f32
        (H, W divisible by 2^(levels - 1))."""
        L = self.levels
        self.inp, self.mid, self.out = {}, {}, {}
        h = x16
        for lvl in range(L):
            if lvl:
                n, hh, ww, c = h.shape
                p = torch.empty((n, hh // 2, ww // 2, c), dtype=BF16, device=self.dev)
                h = nn.pool2(h, p)
            self.inp[f"e{lvl}"] = h
            a = self._conv(f"e{lvl}a", h)
            b = self._conv(f"e{lvl}b", a)
            self.mid[f"e{lvl}"], self.out[f"e{lvl}"] = a, b
            h = b
        for lvl in range(L - 2, self.out_level - 1, -1):
            skip = self.out[f"e{lvl}"]
            n, hh, ww, cs = skip.shape
            cu = h.shape[3]
            cat = torch.empty((n, hh, ww, cu + cs), dtype=BF16, device=self.dev)
            nn.concat_up2(h, skip, cat)
            self.inp[f"d{lvl}"] = cat
            a = self._conv(f"d{lvl}a", cat)
            b = self._conv(f"d{lvl}b", a)
            self.mid[f"d{lvl}"], self.out[f"d{lvl}"] = a, b
            h = b
        self.inp["head"] = h
        return self._conv("head", h, relu=False, out32=True)

    # ------------------------------------------------------------------ backward
    def _wgrad(self, c: Conv, gz16, x16):
        n, h, w, _ = x16.shape
        nn.conv_backward_weight(gz16, x16, c.ks, c.gw, c.gb, self._work_for(c, n, h, w))

    def _dgrad(self, c: Conv, gz16):
        n, h, w, _ = gz16.shape
        dx = torch.empty((n, h, w, c.cin), dtype=F32, device=self.dev)
        return nn.conv_backward_data(gz16, c.wT, dx, self._work_for(c, n, h, w))

    def _relu_back(self, g32, act16):
        g16 = torch.empty(g32.shape, dtype=BF16, device=self.dev)
        return nn.relu_backward(g32, act16, g16)

    def backward(self, gy16: torch.Tensor, record: dict | None = None):
        """gy16: gradient of the loss w.r.t. the forward output, bf16 [n, H, W, 8].
        With `record`, every convolution's name maps to what its backward
        consumed and produced: "g" the FP32 gradient of its ReLU output (absent
        for the head), "gz" the masked BF16 gradient of its pre-activation, and
        "dx" the FP32 gradient of its input (absent for the first convolution)."""
        L = self.levels

        def keep(name, **t):
            if record is not None:
                record.setdefault(name, {}).update(t)

        c = self.convs["head"]
        self._wgrad(c, gy16, self.inp["head"])
        g = self._dgrad(c, gy16)  # d loss / d (output of the last decoder level)
        keep("head", gz=gy16, dx=g)
        skip_grad = {}
        for lvl in range(self.out_level, L - 1):  # decoder levels, top first
            a, b, cat = self.mid[f"d{lvl}"], self.out[f"d{lvl}"], self.inp[f"d{lvl}"]
            gz = self._relu_back(g, b)
            keep(f"d{lvl}b", g=g, gz=gz)
            cb = self.convs[f"d{lvl}b"]
            self._wgrad(cb, gz, a)
            g = self._dgrad(cb, gz)
            keep(f"d{lvl}b", dx=g)
            gz = self._relu_back(g, a)
            keep(f"d{lvl}a", g=g, gz=gz)
            ca = self.convs[f"d{lvl}a"]
            self._wgrad(ca, gz, cat)
            gcat = self._dgrad(ca, gz)
            keep(f"d{lvl}a", dx=gcat)
            n, hh, ww, ct = gcat.shape
            cs = self.out[f"e{lvl}"].shape[3]
            cu = ct - cs
            sg = torch.empty((n, hh, ww, cs), dtype=F32, device=self.dev)
            skip_grad[lvl] = nn.take_channels(gcat, cu, sg)
            g = torch.empty((n, hh // 2, ww // 2, cu), dtype=F32, device=self.dev)
            nn.upsample2_backward(gcat, g)
        for lvl in range(L - 1, -1, -1):  # encoder, bottom first
            a, b, x = self.mid[f"e{lvl}"], self.out[f"e{lvl}"], self.inp[f"e{lvl}"]
            gz = self._relu_back(g, b)
            keep(f"e{lvl}b", g=g, gz=gz)
            cb = self.convs[f"e{lvl}b"]
            self._wgrad(cb, gz, a)
            g = self._dgrad(cb, gz)
            keep(f"e{lvl}b", dx=g)
            gz = self._relu_back(g, a)
            keep(f"e{lvl}a", g=g, gz=gz)
            ca = self.convs[f"e{lvl}a"]
            self._wgrad(ca, gz, x)
            if lvl == 0:
                break
            gx = self._dgrad(ca, gz)  # gradient of the pooled input
            keep(f"e{lvl}a", dx=gx)
            if lvl - 1 in skip_grad:  # the level below also feeds a decoder level
                g = nn.pool2_backward(gx, skip_grad[lvl - 1], accumulate=True)
            else:
                n, hh, ww, c = self.out[f"e{lvl - 1}"].shape
                g = nn.pool2_backward(gx, torch.empty((n, hh, ww, c), dtype=F32, device=self.dev))

    def step(self, lr: float):
        self.t += 1
        for c in self.convs.values():
            c.step(self.t, lr)

    # ------------------------------------------------------------------ checkpoints
    def save(self, path: str, optimizer: bool = True, bf16: bool = False) -> None:
        """Writes the network to `path` as a .npz archive of plain arrays (no
        pickled objects): the FP32 master weights and biases, the step count
        and the shape (channels, output level, input channels), and with
        `optimizer` Adam's moments (needed to resume training, not to
        predict).  bf16=True (without the optimizer) stores the weights as the
        bfloat16 bit patterns the convolutions use: the same predictions from
        half the bytes."""
        if bf16 and optimizer:
            raise ValueError("bfloat16 weights are for prediction only: save without the optimizer")
        arrays = {"meta_bf16": np.array([int(bf16)], dtype=np.int64),
                  "meta_chans": np.array(self.chans, dtype=np.int64),
                  "meta_out_level": np.array([self.out_level], dtype=np.int64),
                  "meta_first_step": np.array([int(self.first_step)], dtype=np.int64),
                  "meta_t": np.array([self.t], dtype=np.int64)}
        parts = ("w", "b", "mw", "vw", "mb", "vb") if optimizer else ("w", "b")
        for k, c in self.convs.items():
            for part in parts:
                if bf16 and part == "w":
                    arrays[f"{k}.w"] = c.w16.detach().cpu().view(torch.int16).numpy().view(np.uint16)
                else:
                    arrays[f"{k}.{part}"] = getattr(c, part).detach().cpu().numpy()
        with open(path, "wb") as f:
            np.savez(f, **arrays)

    @classmethod
    def load(cls, path: str, dev) -> "UNet":
        """The network saved by save(), on `dev`, ready to predict or to train on."""
        with np.load(path, allow_pickle=False) as z:
            first = bool(z["meta_first_step"][0]) if "meta_first_step" in z.files else False
            as_bf16 = "meta_bf16" in z.files and bool(z["meta_bf16"][0])
            net = cls(dev, chans=tuple(int(v) for v in z["meta_chans"]), out_level=int(z["meta_out_level"][0]),
                      first_step=first)
            net.t = int(z["meta_t"][0])
            for k, c in net.convs.items():
                for part in ("w", "b", "mw", "vw", "mb", "vb"):
                    if f"{k}.{part}" not in z.files and part not in ("w", "b"):
                        continue  # saved without the optimizer: moments stay zero
                    a = z[f"{k}.{part}"]
                    if as_bf16 and part == "w":  # bfloat16 bit patterns -> float32 values
                        a = (a.astype(np.uint32) << 16).view(np.float32)
                    dst = getattr(c, part)
                    if tuple(a.shape) != tuple(dst.shape):
                        raise ValueError(f"{k}.{part}: shape {a.shape} in the file, {tuple(dst.shape)} expected")
                    dst.copy_(torch.from_numpy(a))
                c.refresh()
        return net


# ------------------------------------------------------------------ data
def net_radius(radius: int, res: int, net_res: int) -> int:
    """The method's Gaussian radius on the network's coarser raster."""
    return max(1, round(radius * net_res / res))


class FirstStep:
    """The workspace of one iteration of the method on the network's raster:
    the deformation field of a density (inim_deform_density: its integral
    images and map fused, the kernels of the method's own iteration)."""

    def __init__(self, res: int, dev):
        self.res = res
        self.ws = capi.workspace(capi.deform_density_workspace_size(res), dev)

    def field(self, dens: torch.Tensor, n: int, out: torch.Tensor) -> torch.Tensor:
        """The deformation field [res, res, 2] of density `dens` of n samples
        (background n / res^2, the method's default)."""
        return capi.deform_density(dens, n / (self.res * self.res), field=out, ws=self.ws)


def density_input(xy: torch.Tensor, net_res: int, radius: int, out16: torch.Tensor, counts=None, dens=None,
                  ws=None, check: bool = True, first: FirstStep | None = None, field1=None):
    """The network's input: the smoothed density on the net_res raster
    divided by its mean in channel 0 (bf16 [net_res, net_res, 8]); with
    `first`, the displacement of one iteration of the method on that raster
    (times 64) in channels 1 and 2 (field1: its [net_res, net_res, 2] buffer);
    other channels 0.  check: as for capi.rasterize (False under graph
    capture)."""
    if counts is None:
        counts = torch.empty((net_res, net_res), dtype=torch.uint32, device=xy.device)
    if dens is None:
        dens = torch.empty((net_res, net_res), dtype=F32, device=xy.device)
    capi.rasterize(xy, net_res, radius=radius, counts=counts, density=dens, ws=ws, check=check)
    scale = net_res * net_res / xy.shape[0]
    if first is None:
        return nn.pack_density(dens, scale, out16)
    if field1 is None:
        field1 = torch.empty((net_res, net_res, 2), dtype=F32, device=xy.device)
    first.field(dens, xy.shape[0], field1)
    nn.pack_input_many(dens[None], field1[None], [scale], out16[None])
    return out16


def pack_many(net: "UNet", dens: torch.Tensor, ns, x16: torch.Tensor, first: FirstStep | None = None,
              field1: torch.Tensor | None = None) -> torch.Tensor:
    """The network's inputs for a stack of densities [k, R, R] of sets of
    ns[q] samples (with the method's first step when the network takes it;
    field1, if given, receives those first-step fields [k, R, R, 2])."""
    R = dens.shape[-1]
    scales = [R * R / max(1, int(n)) for n in ns]
    if not net.first_step:
        return nn.pack_density_many(dens, scales, x16)
    first = first or FirstStep(R, dens.device)
    f1 = field1 if field1 is not None else torch.empty((dens.shape[0], R, R, 2), dtype=F32, device=dens.device)
    for q in range(dens.shape[0]):
        first.field(dens[q], max(1, int(ns[q])), f1[q])
    return nn.pack_input_many(dens, f1, scales, x16)


def example(xy_np: np.ndarray, res: int, iters: int, dev, radius: int = 8, net_res: int | None = None,
            out_level: int = 0, first_step: bool = False):
    """Input [net_res, net_res, 8] bf16 and target [f, f, 2] f32 with
    f = net_res / 2^out_level: the displacement by `iters` iterations of the
    method on a res x res raster, at the texel centres of the f x f lattice,
    of one point set."""
    net_res = net_res or res
    fres = net_res >> out_level
    xy = torch.from_numpy(xy_np).to(dev)
    x16 = torch.empty((net_res, net_res, CIN), dtype=BF16, device=dev)
    density_input(xy, net_res, net_radius(radius, res, net_res), x16,
                  first=FirstStep(net_res, dev) if first_step else None)
    lat = torch.from_numpy(datagen.lattice_points(fres)).to(dev)
    capi.regularize_probes(xy.clone(), lat, res, iters, radius=radius)
    tgt = torch.empty((fres, fres, 2), dtype=F32, device=dev)
    nn.displacement(lat, fres, tgt)
    return x16, tgt


def dataset(seeds, res: int, iters: int, dev, n_hi: int = 500_000, net_res: int | None = None,
            out_level: int = 0, first_step: bool = False):
    xs, ts = [], []
    for s in seeds:
        x, t = example(datagen.surrogate_mixture(s, n_hi=n_hi), res, iters, dev, net_res=net_res,
                       out_level=out_level, first_step=first_step)
        xs.append(x)
        ts.append(t)
    return torch.stack(xs), torch.stack(ts)


class Compact:
    """A training set kept compact on the device: the smoothed densities
    (float32 [k, R, R]) with their scales (R^2 / n), packed into the
    network's 8-channel bfloat16 input batch by batch, and the target
    displacements [k, f, f, 2]."""

    def __init__(self, dens: torch.Tensor, scales: np.ndarray, targets: torch.Tensor, field1=None):
        self.dens, self.scales, self.targets = dens, np.asarray(scales, dtype=np.float64), targets
        self.field1 = field1  # [k, R, R, 2]: the method's first step, or None
        self.shape = (dens.shape[0],)

    def batch(self, idx: np.ndarray):
        dev = self.dens.device
        it = torch.from_numpy(idx).to(dev)
        d = self.dens[it].contiguous()
        x16 = torch.empty((len(idx), d.shape[1], d.shape[2], CIN), dtype=BF16, device=dev)
        sc = [float(self.scales[i]) for i in idx]
        if self.field1 is None:
            nn.pack_density_many(d, sc, x16)
        else:
            nn.pack_input_many(d, self.field1[it].contiguous(), sc, x16)
        return x16, self.targets[it].contiguous()


def dataset_compact(seeds, res: int, iters: int, dev, n_hi: int = 500_000, net_res: int | None = None,
                    out_levels=(0,), radius: int = 8, workers: int = 0, log=None, first_step: bool = False) -> dict:
    """The training set of `seeds` as Compact sets, one per output level:
    point sets drawn by `workers` processes (0: in this process), each
    rasterised on the device once and labelled by one run of the method with
    the texel centres of every requested f x f lattice (f = net_res /
    2^out_level) as probes (its composite map there)."""
    import concurrent.futures as cf
    import functools
    import multiprocessing as mp
    net_res = net_res or res
    fr = [net_res >> lv for lv in out_levels]
    seeds = list(seeds)
    k = len(seeds)
    dens = torch.empty((k, net_res, net_res), dtype=F32, device=dev)
    tgt = [torch.empty((k, f, f, 2), dtype=F32, device=dev) for f in fr]
    scales = np.empty(k)
    lat0 = torch.from_numpy(np.concatenate([datagen.lattice_points(f) for f in fr])).to(dev)
    lat = torch.empty_like(lat0)
    offs = np.cumsum([0] + [f * f for f in fr])
    counts = torch.empty((net_res, net_res), dtype=torch.uint32, device=dev)
    r = net_radius(radius, res, net_res)
    f1 = torch.empty((k, net_res, net_res, 2), dtype=F32, device=dev) if first_step else None
    first = FirstStep(net_res, dev) if first_step else None
    draw = functools.partial(datagen.surrogate_mixture, n_hi=n_hi)
    pool = cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) if workers > 0 else None
    try:
        it = pool.map(draw, seeds, chunksize=16) if pool else map(draw, seeds)
        for q, xy_np in enumerate(it):
            xy = torch.from_numpy(xy_np).to(dev)
            capi.rasterize(xy, net_res, radius=r, counts=counts, density=dens[q], check=False)
            scales[q] = net_res * net_res / xy.shape[0]
            if first is not None:
                first.field(dens[q], xy.shape[0], f1[q])
            lat.copy_(lat0)
            capi.regularize_probes(xy, lat, res, iters, radius=radius, check=False)
            for i, f in enumerate(fr):
                nn.displacement(lat[offs[i]:offs[i + 1]], f, tgt[i][q])
            if log and q % 4096 == 0:
                log(f"labels {q}/{k}")
    finally:
        if pool:
            pool.shutdown()
    torch.cuda.synchronize(dev)
    return {lv: Compact(dens, scales, t, f1) for lv, t in zip(out_levels, tgt)}


def train(net: UNet, X, T, steps: int, batch: int, lr: float = 1e-3, seed: int = 0, log=None) -> list:
    """Adam on mini-batches drawn (seeded) from X, T (or from the Compact set
    X, with T None); returns the losses."""
    g = np.random.Generator(np.random.PCG64(seed))
    loss = torch.zeros(1, dtype=F32, device=net.dev)
    losses = []
    for s in range(steps):
        pick = g.choice(X.shape[0], size=batch, replace=False)
        if T is None:
            x, t = X.batch(pick)
        else:
            idx = torch.from_numpy(pick).to(net.dev)
            x, t = X[idx].contiguous(), T[idx].contiguous()
        y = net.forward(x)
        gy = torch.empty(y.shape, dtype=BF16, device=net.dev)
        nn.mse(y, t, loss, gy)
        net.backward(gy)
        cur = lr * 0.5 * (1.0 + math.cos(math.pi * s / steps))  # cosine decay
        net.step(cur)
        losses.append(float(loss.item()) / t.numel())
        if log and (s % 50 == 0 or s == steps - 1):
            log(f"step {s} loss {losses[-1]:.4f}")
    return losses


# ------------------------------------------------------------------ use
def bin_std(xy: torch.Tensor, res: int, bin_px: int = 4) -> float:
    """Standard deviation of the sample counts over bin x bin texel blocks."""
    counts = torch.empty((res, res), dtype=torch.uint32, device=xy.device)
    capi.rasterize(xy, res, radius=0, counts=counts, want_density=False)
    mom = torch.zeros(2, dtype=torch.float64, device=xy.device)
    nn.bin_moments(counts, res, bin_px, mom)
    s1, s2 = mom.tolist()
    k = (res // bin_px) ** 2
    return math.sqrt(max(s2 / k - (s1 / k) ** 2, 0.0))


# Smoothing radius of the predicted displacement: the composite map is
# smooth on the scale of the density's Gaussian, while the network's error is
# not, and smoothing removes the part of it that folds the lattice: 2 texels
# at 64 x 64, res / 16 above (16 at 256 x 256, the largest radius).
def field_radius(res: int) -> int:
    return 2 if res <= 64 else min(16, res // 16)


def predict_field(net: UNet, xy: torch.Tensor, res: int, radius: int = 8, net_res: int | None = None,
                  return_first: bool = False):
    """The predicted composite map (absolute positions) on the output lattice
    (net_res / 2^out_level texels a side); with return_first, also the
    method's first-step field on the network's raster (None if the network
    does not read it)."""
    net_res = net_res or res
    fres = net_res >> net.out_level
    x16 = torch.empty((1, net_res, net_res, CIN), dtype=BF16, device=xy.device)
    f1 = torch.empty((net_res, net_res, 2), dtype=F32, device=xy.device) if net.first_step else None
    density_input(xy, net_res, net_radius(radius, res, net_res), x16[0],
                  first=FirstStep(net_res, xy.device) if net.first_step else None, field1=f1)
    y = net.forward(x16)
    field = torch.empty((fres, fres, 2), dtype=F32, device=xy.device)
    field = nn.field(y[0], fres, field, field_radius(fres))
    return (field, f1) if return_first else field


def regularize_many(net: UNet, xys, res: int, radius: int = 8, net_res: int | None = None,
                    check: bool = True) -> list:
    """The surrogate's move of several point sets at once, in place and
    without the gate: their densities, fields and moves each in shared
    launches (up to 64 sets a launch) around one batched forward pass.
    A NaN or out-of-range sample in a group of 64 sets leaves that group
    unmoved; check=True synchronises and raises DomainError then (pass
    False under graph capture and check the returned status workspaces)."""
    net_res = net_res or res
    k = len(xys)
    r = net_radius(radius, res, net_res)
    first = FirstStep(net_res, net.dev) if net.first_step else None
    wss = []
    for q0 in range(0, k, 64):
        part = xys[q0:q0 + 64]
        m = len(part)
        x16 = torch.empty((m, net_res, net_res, CIN), dtype=BF16, device=net.dev)
        _, dens, ws = capi.rasterize_many(part, net_res, radius=r, check=False)
        pack_many(net, dens, [xy.shape[0] for xy in part], x16, first)
        y = net.forward(x16)
        fres = net_res >> net.out_level
        field = torch.empty((m, fres, fres, 2), dtype=F32, device=net.dev)
        nn.field_many(y, fres, field, field_radius(fres))
        capi.advect_many(field, part, ws=ws, check=False)
        wss.append(ws)
    if check:
        check_status(wss)
    return wss


def check_status(wss) -> None:
    """Synchronises and raises DomainError if a call that used one of these
    status workspaces met a NaN or out-of-range sample."""
    for ws in wss:
        capi._check(capi.sync_status(ws))


class SurrogateGraph:
    """The surrogate's move of n samples (density on the net_res raster,
    forward pass, field, advection) captured once as a HIP graph and replayed,
    for callers that repeat it on sets of the same size.  Every buffer is
    allocated before the capture; the library's kernels clear their own
    status words, so nothing in the graph is a memset.  Same results as
    predict_field + advect, without the gate.  With `xy` given, the graph
    moves that tensor itself (call it without an argument); otherwise it moves
    a private copy of the argument of each call."""

    def __init__(self, net: UNet, n: int, res: int, net_res: int | None = None, radius: int = 8,
                 xy: torch.Tensor | None = None):
        self.net, self.res, self.net_res = net, res, net_res or res
        dev = net.dev
        r = self.net_res
        self.radius = net_radius(radius, res, r)
        self.own = xy is None
        saved = None if self.own else xy.clone()
        self.xy = torch.zeros((n, 2), dtype=F32, device=dev) + 0.5 if self.own else xy
        self.x16 = torch.empty((1, r, r, CIN), dtype=BF16, device=dev)
        self.counts = torch.empty((r, r), dtype=torch.uint32, device=dev)
        self.dens = torch.empty((r, r), dtype=F32, device=dev)
        self.first = FirstStep(r, dev) if net.first_step else None
        self.field1 = torch.empty((r, r, 2), dtype=F32, device=dev) if net.first_step else None
        self.fres = r >> net.out_level
        self.field = torch.empty((self.fres, self.fres, 2), dtype=F32, device=dev)
        self.fwork = torch.empty_like(self.field)
        self.ws = capi.workspace(256, dev)
        self._run()  # sizes the network's work buffer outside the capture
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._run()
        torch.cuda.synchronize(dev)
        if saved is not None:  # the warm-up run moved the caller's samples
            self.xy.copy_(saved)

    def _run(self):
        density_input(self.xy, self.net_res, self.radius, self.x16[0], self.counts, self.dens, ws=self.ws,
                      check=False, first=self.first, field1=self.field1)
        y = self.net.forward(self.x16)
        nn.field(y[0], self.fres, self.field, field_radius(self.fres), work=self.fwork)
        capi.advect(self.field, self.xy, ws=self.ws, check=False)

    def __call__(self, xy: torch.Tensor | None = None, check: bool = False) -> torch.Tensor:
        """Moves xy (same n) in place, or the tensor given at construction;
        returns it.  check=True synchronises after the replay and raises
        DomainError if a sample was NaN or outside the unit square (the
        samples are then unmoved)."""
        if xy is None or not self.own:
            if xy is not None and xy is not self.xy:
                raise ValueError("this graph moves the tensor it was built on")
            self.graph.replay()
            if check:
                check_status([self.ws])
            return self.xy
        self.xy.copy_(xy)
        self.graph.replay()
        if check:
            check_status([self.ws])
        xy.copy_(self.xy)
        return xy


class SurrogateManyGraph:
    """regularize_many on a fixed list of point sets (at most 64), captured
    once as a HIP graph: each replay moves those same tensors in place.  All
    buffers are allocated before or inside the capture; nothing in the graph
    is a memset."""

    def __init__(self, net: UNet, xys, res: int, net_res: int | None = None, radius: int = 8):
        if not 1 <= len(xys) <= 64:
            raise ValueError("1 to 64 point sets")
        self.net, self.xys, self.res, self.net_res, self.radius = net, list(xys), res, net_res or res, radius
        dev = net.dev
        saved = [x.clone() for x in self.xys]
        self._run()  # sizes the network's work buffer outside the capture
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.wss = self._run()
        torch.cuda.synchronize(dev)
        for x, x0 in zip(self.xys, saved):  # the warm-up run moved them
            x.copy_(x0)

    def _run(self):
        return regularize_many(self.net, self.xys, self.res, self.radius, self.net_res, check=False)

    def __call__(self, check: bool = False):
        """One replay; check=True synchronises and raises DomainError if a
        sample was NaN or outside the unit square (the sets are then unmoved)."""
        self.graph.replay()
        if check:
            check_status(self.wss)
        return self.xys


def calibrate_gate(res: int, iters: int, dev, seeds=range(200_000, 200_016), slack: float = 1.05,
                   n_hi: int = 500_000) -> float:
    """The gate's ratio: over point sets of the training distribution (seeds
    neither training nor evaluation draw), the largest ratio of the 4 x 4-bin
    standard deviation after `iters` iterations of the method to the one
    after its first iteration, times `slack`.  A prediction must bring its
    set at least that far beyond the method's own first step."""
    worst = 0.0
    for s in seeds:
        x0 = torch.from_numpy(datagen.surrogate_mixture(s, n_hi=n_hi)).to(dev)
        x1, xk = x0.clone(), x0.clone()
        capi.regularize(x1, res, 1)
        capi.regularize(xk, res, iters)
        worst = max(worst, bin_std(xk, res) / max(bin_std(x1, res), 1e-12))
    return worst * slack


def _gate_reference(net: UNet, xy: torch.Tensor, res: int, net_res: int, f1, ratio, min_gain: float) -> float:
    """The bin standard deviation a prediction must reach: `ratio` times the
    one after the method's first step on this set (networks that read it, on
    the method's own raster), else (1 - min_gain) times the input's."""
    if ratio is not None and f1 is not None and net_res == res:
        first = xy.clone()
        capi.advect(f1, first)
        return ratio * bin_std(first, res)
    return (1.0 - min_gain) * bin_std(xy, res)


def regularize(net: UNet, xy: torch.Tensor, res: int, iters: int, min_gain: float = 0.2,
               net_res: int | None = None, ratio: float | None = None):
    """Moves xy (in place) by the surrogate's field when its deformed lattice
    has no fold and its bin standard deviation reaches the gate's reference
    (_gate_reference: `ratio` times the method's own first step, from
    calibrate_gate, or a relative gain `min_gain`); otherwise runs the plain
    method.  Returns 'surrogate' or 'fallback'."""
    net_res = net_res or res
    field, f1 = predict_field(net, xy, res, net_res=net_res, return_first=True)
    ref = _gate_reference(net, xy, res, net_res, f1, ratio, min_gain)
    folds = torch.zeros(1, dtype=torch.uint32, device=xy.device)
    nn.count_folds(field, net_res >> net.out_level, folds)
    moved = xy.clone()
    capi.advect(field, moved)
    if int(folds.item()) == 0 and bin_std(moved, res) <= ref:
        xy.copy_(moved)
        return "surrogate"
    capi.regularize(xy, res, iters)
    return "fallback"


def _bin_moments_into(xy: torch.Tensor, res: int, out: torch.Tensor, counts: torch.Tensor, ws: torch.Tensor):
    """Enqueues the 4 x 4-bin count moments of xy into out (float64 [2],
    cleared first); no synchronisation."""
    capi.rasterize(xy, res, radius=0, counts=counts, want_density=False, ws=ws, check=False)
    out.zero_()
    nn.bin_moments(counts, res, 4, out)


def _std_from_moments(m, res: int, bin_px: int = 4) -> float:
    k = (res // bin_px) ** 2
    return math.sqrt(max(m[1] / k - (m[0] / k) ** 2, 0.0))


class SurrogateGatedGraph:
    """regularize() on one fixed tensor of samples, its GPU work captured once
    as a HIP graph: the prediction, the fold count, the move of a copy, the
    method's first step on another copy (the gate's reference, when the
    network reads it) and the three bin moments.  A call replays the graph,
    reads the fold count and the moments back once, and then either copies
    the moved samples into the tensor or runs the method on it (its own
    captured graph).  Same decisions and results as regularize(); nothing in
    either graph is a memset."""

    def __init__(self, net: UNet, xy: torch.Tensor, res: int, iters: int, net_res: int | None = None,
                 ratio: float | None = None, min_gain: float = 0.2):
        self.net, self.xy, self.res, self.iters = net, xy, res, iters
        self.net_res = net_res or res
        self.ratio, self.min_gain = ratio, min_gain
        dev = xy.device
        r = self.net_res
        self.by_first = ratio is not None and net.first_step and self.net_res == res
        self.radius = net_radius(8, res, r)
        self.x16 = torch.empty((1, r, r, CIN), dtype=BF16, device=dev)
        self.counts_r = torch.empty((r, r), dtype=torch.uint32, device=dev)
        self.dens = torch.empty((r, r), dtype=F32, device=dev)
        self.first = FirstStep(r, dev) if net.first_step else None
        self.field1 = torch.empty((r, r, 2), dtype=F32, device=dev) if net.first_step else None
        self.fres = r >> net.out_level
        self.field = torch.empty((self.fres, self.fres, 2), dtype=F32, device=dev)
        self.fwork = torch.empty_like(self.field)
        self.folds = torch.zeros(1, dtype=torch.uint32, device=dev)
        self.mom = torch.zeros((3, 2), dtype=torch.float64, device=dev)  # input, moved, after the first step
        self.counts = torch.empty((res, res), dtype=torch.uint32, device=dev)
        self.moved = torch.empty_like(xy)
        self.firsts = torch.empty_like(xy)
        self.ws = capi.workspace(256, dev)
        self.ws_m = capi.workspace(256, dev)
        self.ws_reg = capi.workspace(capi.workspace_size(res, xy.shape[0]), dev)
        self.method = capi.Graph()
        self._run()  # sizes the network's work buffer outside the capture
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._run()
        torch.cuda.synchronize(dev)

    def _run(self):
        xy = self.xy
        density_input(xy, self.net_res, self.radius, self.x16[0], self.counts_r, self.dens, ws=self.ws,
                      check=False, first=self.first, field1=self.field1)
        y = self.net.forward(self.x16)
        nn.field(y[0], self.fres, self.field, field_radius(self.fres), work=self.fwork)
        self.folds.zero_()
        nn.count_folds(self.field, self.fres, self.folds)
        if not self.by_first:  # the relative-gain gate measures the input
            _bin_moments_into(xy, self.res, self.mom[0], self.counts, self.ws_m)
        if self.by_first:
            torch.mul(xy, 1.0, out=self.firsts)  # a copy kernel (x * 1 is exact, -0 included)
            capi.advect(self.field1, self.firsts, ws=self.ws_m, check=False)
            _bin_moments_into(self.firsts, self.res, self.mom[2], self.counts, self.ws_m)
        torch.mul(xy, 1.0, out=self.moved)
        capi.advect(self.field, self.moved, ws=self.ws_m, check=False)
        _bin_moments_into(self.moved, self.res, self.mom[1], self.counts, self.ws_m)

    def __call__(self) -> str:
        """Moves the tensor given at construction; returns 'surrogate' or
        'fallback'.  Raises DomainError (samples unmoved) for a NaN or
        out-of-range sample."""
        self.graph.replay()
        check_status([self.ws, self.ws_m])
        mh = self.mom.cpu().numpy()  # one readback: the stream is idle after the status check
        folds = int(self.folds.cpu().item())
        ref = (self.ratio * _std_from_moments(mh[2], self.res) if self.by_first
               else (1.0 - self.min_gain) * _std_from_moments(mh[0], self.res))
        if folds == 0 and _std_from_moments(mh[1], self.res) <= ref:
            self.xy.copy_(self.moved)
            return "surrogate"
        capi.regularize_graph(self.xy, self.res, self.iters, self.method, self.ws_reg)
        return "fallback"


def regularize_many_gated(net: UNet, xys, res: int, iters: int, min_gain: float = 0.2,
                          net_res: int | None = None, ws_batch: torch.Tensor | None = None,
                          ratio: float | None = None) -> list:
    """The surrogate's batched move (regularize_many) under the gate of
    regularize(): a set whose predicted lattice folds, or whose bin standard
    deviation falls by less than `min_gain`, is regularised by the method
    instead -- all such sets in one batched call of the method.  The fields,
    folds, moves and uniformity measures are enqueued for every set first and
    read back once.  The gate is regularize()'s (`ratio` times the method's
    first step when the network reads it, else `min_gain`).  Returns the
    decisions ('surrogate' / 'fallback')."""
    net_res = net_res or res
    k = len(xys)
    if k == 0:
        return []
    dev = xys[0].device
    fres = net_res >> net.out_level
    counts = torch.empty((res, res), dtype=torch.uint32, device=dev)
    mom = torch.zeros((3, k, 2), dtype=torch.float64, device=dev)  # input, moved, after the first step
    by_first = ratio is not None and net.first_step and net_res == res
    folds = torch.zeros(k, dtype=torch.uint32, device=dev)
    ws = capi.workspace(256, dev)
    for q, x in enumerate(xys):
        _bin_moments_into(x, res, mom[0, q], counts, ws)
    moved = [x.clone() for x in xys]
    r = net_radius(8, res, net_res)
    fields = []
    for q0 in range(0, k, 64):
        part = moved[q0:q0 + 64]
        m = len(part)
        x16 = torch.empty((m, net_res, net_res, CIN), dtype=BF16, device=dev)
        _, dens, wsp = capi.rasterize_many(part, net_res, radius=r, check=False)
        f1 = torch.empty((m, net_res, net_res, 2), dtype=F32, device=dev) if by_first else None
        pack_many(net, dens, [x.shape[0] for x in part], x16, field1=f1)
        y = net.forward(x16)
        field = torch.empty((m, fres, fres, 2), dtype=F32, device=dev)
        nn.field_many(y, fres, field, field_radius(fres))
        for q in range(m):
            nn.count_folds(field[q], fres, folds[q0 + q:q0 + q + 1])
        if by_first:  # the method's first step on copies, for the gate's reference
            firsts = [xys[q0 + q].clone() for q in range(m)]
            capi.advect_many(f1, firsts, ws=wsp, check=False)
            for q in range(m):
                _bin_moments_into(firsts[q], res, mom[2, q0 + q], counts, ws)
        capi.advect_many(field, part, ws=wsp, check=False)
        fields.append(wsp)
    for q, x in enumerate(moved):
        _bin_moments_into(x, res, mom[1, q], counts, ws)
    check_status(fields + [ws])
    mh, fh = mom.cpu().numpy(), folds.cpu().numpy()
    decisions, rejected = [], []
    for q in range(k):
        ref = (ratio * _std_from_moments(mh[2, q], res) if by_first
               else (1.0 - min_gain) * _std_from_moments(mh[0, q], res))
        ok = int(fh[q]) == 0 and _std_from_moments(mh[1, q], res) <= ref
        decisions.append("surrogate" if ok else "fallback")
        if ok:
            xys[q].copy_(moved[q])
        else:
            rejected.append(xys[q])
    if rejected:
        capi.regularize_batch(rejected, [res] * len(rejected), iters, ws=ws_batch)
    return decisions


def evaluate(net: UNet, seeds, res: int, iters: int, dev, n_hi: int = 500_000, min_gain: float = 0.2,
             net_res: int | None = None, ratio: float | None = None) -> dict:
    """Held-out comparison on fresh point sets: bin standard deviation (4 x 4
    texel bins) before, after the plain method, after its first iteration,
    after the surrogate's field;
    folds of the surrogate's deformed lattice; how often the gate (ratio /
    min_gain as in regularize) falls back, and how many accepted predictions
    end more than 5% less uniform than the method; the displacement error
    against the method's own field."""
    rows = []
    for s in seeds:
        xy_np = datagen.surrogate_mixture(s, n_hi=n_hi)
        xy = torch.from_numpy(xy_np).to(dev)
        before = bin_std(xy, res)
        plain = xy.clone()
        capi.regularize(plain, res, iters)
        one = xy.clone()
        capi.regularize(one, res, 1)
        field = predict_field(net, xy, res, net_res=net_res)
        folds = torch.zeros(1, dtype=torch.uint32, device=dev)
        nn.count_folds(field, (net_res or res) >> net.out_level, folds)
        sur = xy.clone()
        capi.advect(field, sur)
        x16, tgt = example(xy_np, res, iters, dev, net_res=net_res, out_level=net.out_level,
                           first_step=net.first_step)
        y = net.forward(x16[None].contiguous())
        loss = torch.zeros(1, dtype=F32, device=dev)
        nn.mse(y, tgt[None].contiguous(), loss)
        zero = torch.zeros_like(y)
        base = torch.zeros(1, dtype=F32, device=dev)
        nn.mse(zero, tgt[None].contiguous(), base)
        gated = xy.clone()
        which = regularize(net, gated, res, iters, min_gain, net_res=net_res, ratio=ratio)
        rows.append({"n": int(xy.shape[0]), "before": before, "plain": bin_std(plain, res),
                     "first": bin_std(one, res), "surrogate": bin_std(sur, res), "folds": int(folds.item()), "gate": which,
                     "mse": float(loss.item()), "mse_zero": float(base.item())})
    acc = [r for r in rows if r["gate"] == "surrogate"]
    return {"rows": rows,
            "accepted_short_of_method": int(sum(r["surrogate"] > 1.05 * r["plain"] for r in acc)),
            "plain_gain": float(np.mean([1 - r["plain"] / r["before"] for r in rows])),
            "surrogate_gain": float(np.mean([1 - r["surrogate"] / r["before"] for r in rows])),
            "explained": float(1 - sum(r["mse"] for r in rows) / sum(r["mse_zero"] for r in rows)),
            "folds": int(sum(r["folds"] for r in rows)),
            "fallbacks": int(sum(r["gate"] == "fallback" for r in rows))}
