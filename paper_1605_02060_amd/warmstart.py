"""Learned warm start for masked LDDMM: a 3-D conv encoder-decoder that maps the
mask pair (M0, M1) to an initial velocity, trained on registrations the library
itself computes, then refined by the plain gradient descent.

The paper registers from v = 0 (Methods, Registration); the descent it uses
stays the judge here: the network only proposes v_init, and lddmm_register
refines it.  Every tensor operation of training and inference runs in the
library's HIP kernels (paper_1605_02060_amd.cnn): convolutions on the bf16
matrix cores, FP32 master weights with Adam, FP64 losses.  PyTorch provides
device memory only.

Network (channels-last, bf16 activations, FP32 accumulation):
  enc0  2 -> 16   stride 1, ReLU     (full resolution)
  enc1 16 -> 32   stride 2, ReLU     (1/2)
  enc2 32 -> 64   stride 2, ReLU     (1/4)
  enc3 64 -> 128  stride 2, ReLU     (1/8)
  dec  [up2(enc3), enc2] 192 -> 64, ReLU   (1/4)
  head 64 -> 3T   (1/4, FP32 output)
The output is the time-varying velocity in voxels per unit time at a quarter
of the resolution, channel 3j + component; lddmm_cnn_expand_velocity scales it
by the spacing and upsamples it twice (cell-centred trilinear) to v_init.
"""

from __future__ import annotations

import json
import os
import math
import time

import numpy as np
import torch

from . import cnn as G
from . import lddmm as L

WIDTH = (16, 32, 64, 128)


def layer_specs(T, width=WIDTH):
    """(name, c_in, c_out, stride, relu) of every convolution, in order."""
    c0, c1, c2, c3 = width
    return [("enc0", 2, c0, 1, True), ("enc1", c0, c1, 2, True), ("enc2", c1, c2, 2, True),
            ("enc3", c2, c3, 2, True), ("dec", c3 + c2, c2, 1, True),
            ("head", c2, 3 * T, 1, False)]


def _round64(n):
    return (n + 63) // 64 * 64


class WarmStartNet:
    """Parameters live in one flat FP32 buffer (so one Adam launch updates all of
    them) with a bf16 copy for the convolutions and transposed bf16 weights for
    the input gradients.  Segments are 64-element aligned (16-byte vector loads)."""

    def __init__(self, T=10, width=WIDTH, seed=0, device="cuda"):
        self.T, self.width, self.device = T, tuple(width), device
        self.specs = layer_specs(T, width)
        self.off = {}
        n = 0
        for name, ci, co, s, relu in self.specs:
            self.off[name] = (n, n + _round64(co * 27 * ci))     # weight segment, bias segment
            n += _round64(co * 27 * ci) + _round64(co)
        self.count = n
        rng = np.random.default_rng(seed)
        p = np.zeros(n, dtype=np.float32)
        for name, ci, co, s, relu in self.specs:
            w0, b0 = self.off[name]
            std = math.sqrt(2.0 / (27 * ci)) if relu else math.sqrt(1.0 / (27 * ci))
            p[w0:w0 + co * 27 * ci] = rng.normal(0.0, std, co * 27 * ci)
        self.p = torch.as_tensor(p, device=device)
        self.g = torch.zeros_like(self.p)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.pb = torch.empty(n, dtype=torch.bfloat16, device=device)
        self.wt = {name: torch.empty((ci, 27 * co), dtype=torch.bfloat16, device=device)
                   for name, ci, co, s, relu in self.specs}
        self.step_count = 0
        self.label_scale = 1.0          # label = pooled v / spacing (voxels per unit time)
        self._ws = None
        self._refresh()

    # views ------------------------------------------------------------------
    def w(self, name, buf=None):
        buf = self.pb if buf is None else buf
        ci, co = self._io(name)
        w0, _ = self.off[name]
        return buf[w0:w0 + co * 27 * ci].view(co, 3, 3, 3, ci)

    def b(self, name, buf=None):
        buf = self.p if buf is None else buf
        ci, co = self._io(name)
        _, b0 = self.off[name]
        return buf[b0:b0 + co]

    def _io(self, name):
        for n_, ci, co, s, relu in self.specs:
            if n_ == name:
                return ci, co
        raise KeyError(name)

    def _refresh(self):
        G.to_bf16(self.p, out=self.pb)
        self._transpose()

    def _transpose(self):
        for name, ci, co, s, relu in self.specs:
            G.transpose_weight(self.w(name), out=self.wt[name])

    # forward / backward -----------------------------------------------------
    def forward(self, x, keep=False):
        """x [B, D, H, W, 2] bf16 -> out [B, D/4, H/4, W/4, 3T] FP32."""
        a = {"in": x}
        h = x
        for name, ci, co, s, relu in self.specs[:4]:
            h = G.conv3d_forward(h, self.w(name), self.b(name), s, relu)
            a[name] = h
        a["cat"] = G.upcat(a["enc3"], a["enc2"])
        a["dec"] = G.conv3d_forward(a["cat"], self.w("dec"), self.b("dec"), 1, True)
        out = G.conv3d_forward(a["dec"], self.w("head"), self.b("head"), 1, False,
                               out_dtype=torch.float32)
        if keep:
            self._acts = a
        return out

    def backward(self, dout):
        """dout [B, D/4, H/4, W/4, 3T] bf16 -> parameter gradients in self.g."""
        a = self._acts
        self._wgrad_into(dout, a["dec"], "head", 1)
        d = G.conv3d_backward_data(dout, tuple(a["dec"].shape), self.wt["head"], 1, mask=a["dec"])
        self._wgrad_into(d, a["cat"], "dec", 1)
        dcat = G.conv3d_backward_data(d, tuple(a["cat"].shape), self.wt["dec"], 1, mask=a["cat"])
        d = G.upcat_backward(dcat, tuple(a["enc3"].shape))
        self._wgrad_into(d, a["enc2"], "enc3", 2)
        c3 = a["enc3"].shape[-1]
        d = G.conv3d_backward_data(d, tuple(a["enc2"].shape), self.wt["enc3"], 2, mask=a["enc2"],
                                   add=dcat, add_off=c3)
        self._wgrad_into(d, a["enc1"], "enc2", 2)
        d = G.conv3d_backward_data(d, tuple(a["enc1"].shape), self.wt["enc2"], 2, mask=a["enc1"])
        self._wgrad_into(d, a["enc0"], "enc1", 2)
        d = G.conv3d_backward_data(d, tuple(a["enc0"].shape), self.wt["enc1"], 2, mask=a["enc0"])
        self._wgrad_into(d, a["in"], "enc0", 1)

    def _wgrad_into(self, dy, x, name, stride):
        need = G.wgrad_workspace_bytes(tuple(x.shape), dy.shape[-1], stride)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        G.conv3d_backward_weight(dy, x, stride, ws=self._ws, dw=self.w(name, self.g),
                                 db=self.b(name, self.g))

    def adam_step(self, lr):
        self.step_count += 1
        G.adam(self.p, self.g, self.m, self.v, self.step_count, lr, p_bf16=self.pb)
        self._transpose()

    def train_step(self, x, target, lr):
        """One Adam step on the mean squared error; returns the loss (device FP64)."""
        out = self.forward(x, keep=True)
        loss, dout = G.mse(out, target)
        self.backward(dout)
        self.adam_step(lr)
        self._acts = None
        return loss

    # inference --------------------------------------------------------------
    def predict_velocity(self, M0, M1, spacing, v=None):
        """Initial velocity [T, 3, D, H, W] for one mask pair [D, H, W] (float32,
        D, H, W multiples of 8)."""
        x = G.pack_masks(M0, M1).unsqueeze(0)
        out = self.forward(x)[0]
        return G.expand_velocity(out.contiguous(), self.T, spacing * self.label_scale, v=v)

    # persistence ------------------------------------------------------------
    def state(self):
        meta = {"T": self.T, "width": list(self.width), "label_scale": self.label_scale,
                "steps": self.step_count}
        return {"params": self.p.detach().cpu().numpy()}, meta

    def save(self, path, extra=None):
        from safetensors.numpy import save_file
        tensors, meta = self.state()
        if extra:
            meta.update(extra)
        save_file(tensors, path, metadata={"meta": json.dumps(meta)})

    @classmethod
    def load(cls, path, device="cuda"):
        from safetensors import safe_open
        with safe_open(path, framework="np") as f:
            meta = json.loads(f.metadata()["meta"])
            params = f.get_tensor("params")
        net = cls(T=meta["T"], width=tuple(meta["width"]), device=device)
        if params.shape[0] != net.count:
            raise ValueError("weights file does not match the network layout")
        net.p.copy_(torch.as_tensor(params, device=device))
        net.label_scale = meta.get("label_scale", 1.0)
        net.step_count = meta.get("steps", 0)
        net.meta = meta
        net._refresh()
        return net


# ---------------------------------------------------------------- data ----

def plain_params(T=10, iters=200, step=0.02):
    """The plain method the network learns from and is judged against: one level,
    fixed-step descent, alpha = 0.02, gamma = sigma = 1."""
    return L.Params(alpha=0.02, gamma=1.0, sigma=1.0, T=T, n_levels=1, iters=(iters,),
                    step=step, guard=False, weight=(1.0, 0.0))


def make_dataset(seeds, spacing=0.05, T=10, iters=200, chunk=32, device="cuda", log=print):
    """Register every pair (masks from synth.warmstart_masks_device) with the plain
    method in batched launches; returns (X [N, 96, 96, 96, 2] bf16, Y [N, 24, 24, 24, 3T]
    FP32 labels = pooled v / spacing)."""
    from . import synth
    n = len(seeds)
    X = torch.empty((n, 96, 96, 96, 2), dtype=torch.bfloat16, device=device)
    Y = torch.empty((n, 24, 24, 24, 3 * T), dtype=torch.float32, device=device)
    prm = plain_params(T, iters)
    wss = None
    t0 = time.perf_counter()
    for c0 in range(0, n, chunk):
        idx = list(range(c0, min(n, c0 + chunk)))
        pairs = []
        for i in idx:
            M0, M1 = synth.warmstart_masks_device(int(seeds[i]), device)
            pairs.append({"M0": M0, "M1": M1, "spacing": spacing})
            G.pack_masks(M0, M1, out=X[i])
        if wss is None or len(wss) < len(pairs):
            wss = [L.workspace((96, 96, 96), prm, spacing, device) for _ in pairs]
        res, code = L.lddmm_register_batched(pairs, prm, wss=wss[:len(pairs)], want_phi=False)
        for i, r in zip(idx, res):
            G.pool_velocity(r["v"], 1.0 / spacing, out=Y[i])
        torch.cuda.synchronize()
        log(f"dataset {min(n, c0 + chunk)}/{n} pairs, {time.perf_counter() - t0:.1f} s")
    return X, Y


def train(net, X, Y, epochs=20, batch=8, lr=1e-3, seed=0, log=print, lr_final=1e-4):
    """Adam on the mean squared error, cosine learning-rate decay from lr to lr_final."""
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    steps = epochs * (n // batch)
    k = 0
    t0 = time.perf_counter()
    hist = []
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(n), device=X.device)
        losses = []
        for b0 in range(0, n - batch + 1, batch):
            ib = perm[b0:b0 + batch]
            x = X.index_select(0, ib).contiguous()
            y = Y.index_select(0, ib).contiguous()
            cur = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * k / max(steps, 1)))
            losses.append(net.train_step(x, y, cur))
            k += 1
        ep_loss = float(torch.stack(losses).mean())
        hist.append(ep_loss)
        log(f"epoch {ep + 1}/{epochs} loss {ep_loss:.5f} ({time.perf_counter() - t0:.1f} s)")
    return hist


# ----------------------------------------------------------- evaluation ----

def first_reaching(D, target):
    """Index of the first trace row whose masked SSD is <= target (None if never)."""
    hit = np.nonzero(np.asarray(D) <= target)[0]
    return int(hit[0]) if hit.size else None


def _batched_runs(masks, prm, spacing, chunk, device, net=None):
    """Register all pairs in batched launches (from v = 0, or from the network's
    v_init); returns (masked-SSD traces, wall seconds, seconds spent in the network)."""
    T = prm.T
    m = min(chunk, len(masks))
    wss = [L.workspace((96, 96, 96), prm, spacing, device) for _ in range(m)]
    vs = [torch.zeros((T, 3, 96, 96, 96), dtype=torch.float32, device=device) for _ in range(m)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_net = 0.0
    traces = []
    for c0 in range(0, len(masks), chunk):
        part = masks[c0:c0 + chunk]
        ta = time.perf_counter()
        for k, (M0, M1) in enumerate(part):
            if net is None:
                vs[k].zero_()
            else:
                net.predict_velocity(M0, M1, spacing, v=vs[k])
        if net is not None:
            torch.cuda.synchronize()
            t_net += time.perf_counter() - ta
        res, code = L.lddmm_register_batched(
            [{"M0": M0, "M1": M1, "spacing": spacing} for M0, M1 in part], prm,
            vs=vs[:len(part)], wss=wss[:len(part)], want_phi=False)
        traces += [r["trace"][:, 2].cpu().numpy() for r in res]
    torch.cuda.synchronize()
    return traces, time.perf_counter() - t0, t_net


def iterations_to_target(D_plain, D_warm):
    """Per pair: the first iteration at which the plain and the warm-started descent
    reach the plain method's final masked SSD D* (the last entry of D_plain).  A
    warm-started run that never reaches it within its iterations is censored at
    len(trace) (one more than it ran).  Returns (plain, warm, reached) arrays."""
    kp, kw, hit = [], [], []
    for dp, dw in zip(D_plain, D_warm):
        target = dp[-1]
        kp.append(first_reaching(dp, target))
        k = first_reaching(dw, target)
        hit.append(k is not None)
        kw.append(k if k is not None else len(dw))
    return np.array(kp), np.array(kw), np.array(hit)


def evaluate(net, seeds, spacing=0.05, plain_iters=200, warm_iters=50, chunk=32, device="cuda",
             log=print):
    """Held-out comparison of the plain method (v = 0, plain_iters iterations; its final
    masked SSD is the per-pair target D*) with the network's v_init refined by the same
    descent, both in batched launches, on every pair.

    Wall seconds, inputs in HBM:
      plain_seq_s         one lddmm_register call per pair (context only)
      plain_batched_s     the plain registrations in batched launches
      warm_batched_s      network on every pair + batched refinement of warm_iters
      warm_batched_long_s network + batched refinement of plain_iters
    Iterations to D*: the first trace row at or below D*, from the plain_iters runs;
    a warm-started pair that does not reach D* in plain_iters iterations is censored
    at plain_iters + 1 and stays in every median (none is dropped).  Time to D* per
    pair = network time per pair + iterations x the batched time per iteration."""
    from . import synth
    n = len(seeds)
    masks = [synth.warmstart_masks_device(int(s), device) for s in seeds]
    pp = plain_params(net.T, plain_iters)
    pw = plain_params(net.T, warm_iters)
    ws = L.workspace((96, 96, 96), pp, spacing, device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for M0, M1 in masks:
        L.lddmm_register(M0, M1, params=pp, spacing=spacing, ws=ws, want_phi=False)
    torch.cuda.synchronize()
    t_plain_seq = time.perf_counter() - t0
    log(f"plain sequential: {n} pairs x {plain_iters} iterations in {t_plain_seq:.2f} s")
    D_plain, t_plain_batch, _ = _batched_runs(masks, pp, spacing, chunk, device)
    log(f"plain batched: {t_plain_batch:.2f} s")
    D_warm, t_warm_batch, t_net = _batched_runs(masks, pw, spacing, chunk, device, net)
    log(f"warm + batched ({warm_iters} iterations): {t_warm_batch:.2f} s, network {t_net:.2f} s")
    D_warm_long, t_warm_long, t_net_long = _batched_runs(masks, pp, spacing, chunk, device, net)
    D_star = np.array([d[-1] for d in D_plain])
    kp, kw, hit = iterations_to_target(D_plain, D_warm_long)
    t_iter = t_plain_batch / (n * plain_iters)                  # batched, per pair and iteration
    t_iter_w = (t_warm_long - t_net_long) / (n * plain_iters)
    t_plain_to = kp * t_iter
    t_warm_to = t_net_long / n + kw * t_iter_w
    t_warm_to_c = np.where(hit, t_warm_to, np.inf)               # censored: never reached
    saving = kp - kw                                             # censored pairs: <= -1
    within = [first_reaching(d, ds) for d, ds in zip(D_warm, D_star)]
    return {
        "pairs": n, "plain_iters": plain_iters, "warm_iters": warm_iters,
        "plain_seq_s": t_plain_seq, "plain_batched_s": t_plain_batch,
        "warm_batched_s": t_warm_batch, "warm_batched_long_s": t_warm_long,
        "network_s": t_net,
        "reached_Dstar_within_warm_iters": int(sum(k is not None for k in within)),
        "reached_Dstar_within_plain_iters": int(hit.sum()),
        "iters_to_Dstar_plain": kp.tolist(),
        "iters_to_Dstar_warm": [int(k) if h else -1 for k, h in zip(kw, hit)],
        "iters_to_Dstar_plain_median": float(np.median(kp)),
        "iters_to_Dstar_warm_median_censored": float(np.median(np.where(hit, kw, np.inf))),
        "iters_saving_median_censored": float(np.median(saving)),
        "iters_saving_mean_reached": float(saving[hit].mean()) if hit.any() else None,
        "time_to_Dstar_plain_batched_per_pair_s_median": float(np.median(t_plain_to)),
        "time_to_Dstar_warm_batched_per_pair_s_median_censored": float(np.median(t_warm_to_c)),
        "time_to_Dstar_plain_batched_total_s": float(t_plain_to.sum()),
        "time_to_Dstar_warm_batched_total_s_reached_pairs": float(t_warm_to[hit].sum()),
        "time_to_Dstar_plain_batched_total_s_same_pairs": float(t_plain_to[hit].sum()),
        "D_zero_mean": float(np.mean([d[0] for d in D_plain])),
        "D_plain_at_warm_iters_mean": float(np.mean([d[warm_iters] for d in D_plain])),
        "D_star_mean": float(D_star.mean()),
        "D_warm_init_mean": float(np.mean([d[0] for d in D_warm])),
        "D_warm_at_warm_iters_mean": float(np.mean([d[-1] for d in D_warm])),
        "D_warm_at_plain_iters_mean": float(np.mean([d[-1] for d in D_warm_long])),
    }


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="train the warm-start network on registrations "
                                             "computed by the plain method, then evaluate it")
    ap.add_argument("--pairs", type=int, default=2000)
    ap.add_argument("--first-seed", type=int, default=10000)
    ap.add_argument("--eval-pairs", type=int, default=100)
    ap.add_argument("--eval-seed", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=None, help="where to save the trained weights")
    ap.add_argument("--eval-only", default=None, metavar="WEIGHTS",
                    help="skip training: evaluate these saved weights")
    ap.add_argument("--report", default=None)
    args = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    L.load()
    if args.eval_only:
        net = WarmStartNet.load(args.eval_only)
        ev = evaluate(net, np.arange(args.eval_seed, args.eval_seed + args.eval_pairs), log=log)
        report = {"weights": os.path.basename(args.eval_only), "evaluation": ev}
        log(json.dumps(report))
        if args.report:
            with open(args.report, "w") as f:
                json.dump(report, f, indent=1)
        return
    if not args.out:
        ap.error("--out is required for training")
    seeds = np.arange(args.first_seed, args.first_seed + args.pairs)
    t0 = time.perf_counter()
    X, Y = make_dataset(seeds, log=log)
    t_data = time.perf_counter() - t0
    net = WarmStartNet(T=10, seed=0)
    t0 = time.perf_counter()
    hist = train(net, X, Y, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del X, Y
    info = {"train_pairs": args.pairs, "first_seed": args.first_seed, "epochs": args.epochs,
            "batch": args.batch, "lr": args.lr, "loss_history": hist,
            "data_s": t_data, "train_s": t_train}
    net.save(args.out, extra={"training": info})
    log(f"saved {args.out}")
    ev = evaluate(net, np.arange(args.eval_seed, args.eval_seed + args.eval_pairs), log=log)
    report = {"training": info, "evaluation": ev}
    log(json.dumps(report))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)


if __name__ == "__main__":
    main()
