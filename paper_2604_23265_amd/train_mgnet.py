"""Offline training of MgNet weights for a family of 2D problems.

The preconditioner z = M(v) of the library -- the V-cycle of Sec. 3.3 with
the CoeffNet fields of Sec. 3.2, in the reading the library implements
(input scaling by diag(L), 1x1 lift, smoothing steps
u <- u + B * (a^{-1} (.) (f - A * u - a (.) u)), stride-2 restriction and
transposed-conv prolongation, 1x1 projection plus the diagonal skip) -- is
written here in PyTorch so it can be differentiated.  Training minimises the
residual loss E ||b - L M(b)||^2 / ||b||^2 over seeded media of the family
and random right-hand sides: the unsupervised loss of Sec. 3.4, taken on the
discrete operator L of Sec. 2.1 (step-upwind streaming, eq. (DORTE_2d)) that
the solver preconditions.  Optimiser: AdamW with a cosine schedule (the
paper's choice), from the seeded initial weights.  The result is an MGN1
blob that mgnet_load reads.

Usage (on a machine with a GPU):
    python -m paper_2604_23265_amd.train_mgnet --family c2 --steps 1500 --out c2.mgn1
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from rte_inputs import configs, media
from rte_inputs import weights as W


def _torch():
    import torch
    return torch


# ------------------------------------------------------------ operator ---

class Medium:
    """Tensors of a batch of problems sharing grid and directions.  S is one
    scattering matrix [N, N] for all of them or one per problem [B, N, N]."""

    def __init__(self, probs, S, device, dtype):
        torch = _torch()
        p0 = probs[0]
        assert p0["dim"] == 2, "training covers 2D families"
        nx, ny, _ = p0["n"]
        self.nx, self.ny = nx, ny
        self.N = p0["dirs"].shape[0]
        h = 1.0 / nx
        dirs = np.asarray(p0["dirs"], float)
        st = np.stack([np.asarray(p["sigma_t"], float).reshape(ny, nx) for p in probs])
        sa = np.stack([np.asarray(p["sigma_a"], float).reshape(ny, nx) for p in probs])
        eps = np.stack([np.broadcast_to(np.asarray(p["eps"], float), (ny, nx)) for p in probs])
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)
        # diffusive scaling of eq. (RTE)
        self.sT = t(st / eps)[:, None]
        self.sA = t(eps * sa)[:, None]
        S = np.asarray(S, float)
        S = np.broadcast_to(S.reshape(-1, self.N, self.N), (len(probs), self.N, self.N))
        self.S = t(S)
        self.dcx = t(np.abs(dirs[:, 0]) / h)[None, :, None, None]
        self.dcy = t(np.abs(dirs[:, 1]) / h)[None, :, None, None]
        self.sgx = t(np.sign(dirs[:, 0]))[None, :, None, None]
        self.sgy = t(np.sign(dirs[:, 1]))[None, :, None, None]
        sS = self.sT - self.sA
        self.diag = self.dcx + self.dcy + self.sT - sS * torch.diagonal(self.S, dim1=1, dim2=2)[:, :, None, None]
        # CoeffNet input [log sT, sA / sT, log eps]
        self.X = torch.cat([torch.log(self.sT), self.sA / self.sT, t(np.log(eps))[:, None]], dim=1)


def apply_L(psi, md):
    """L psi for psi [B, N, ny, nx] (zero upwind values outside the grid)."""
    torch = _torch()
    F = torch.nn.functional
    left = F.pad(psi, (1, 0))[..., :-1]      # value at i - 1
    right = F.pad(psi, (0, 1))[..., 1:]      # value at i + 1
    down = F.pad(psi, (0, 0, 1, 0))[..., :-1, :]
    up = F.pad(psi, (0, 0, 0, 1))[..., 1:, :]
    zero = torch.zeros_like(psi)
    nbx = torch.where(md.sgx > 0, left, torch.where(md.sgx < 0, right, zero))
    nby = torch.where(md.sgy > 0, down, torch.where(md.sgy < 0, up, zero))
    Spsi = torch.einsum("bmn,bnyx->bmyx", md.S, psi)
    return md.dcx * (psi - nbx) + md.dcy * (psi - nby) + md.sT * (psi - Spsi) + md.sA * Spsi


# ------------------------------------------------------------- network ---

class MgNet:
    """Trainable MgNet + CoeffNet holding the MGN1 tensors by tag."""

    def __init__(self, hdr, tensors, device, dtype):
        torch = _torch()
        self.hdr = dict(hdr)
        self.L = hdr["levels"]
        self.p = {k: torch.nn.Parameter(torch.as_tensor(np.asarray(v, np.float64), dtype=dtype, device=device))
                  for k, v in tensors.items()}

    def params(self):
        return list(self.p.values())

    def g(self, kind, level=0, index=0):
        return self.p[W.tag(kind, level, index)]

    def coeffnet(self, X):
        torch = _torch()
        F = torch.nn.functional
        a, ainv = [], []
        Fm = X
        for l in range(self.L):
            Fm = torch.relu(F.conv2d(Fm, self.g(W.K_CW, l), self.g(W.K_CB, l), stride=1 if l == 0 else 2,
                                     padding=1))
            a.append(torch.einsum("Cc,bcyx->bCyx", self.g(W.K_HAW, l), Fm) + self.g(W.K_HAB, l)[None, :, None, None])
            ainv.append(torch.einsum("Cc,bcyx->bCyx", self.g(W.K_HIW, l), Fm)
                        + self.g(W.K_HIB, l)[None, :, None, None])
        return a, ainv

    def __call__(self, v, md, fields):
        """z = M(v) for v [B, N, ny, nx]."""
        torch = _torch()
        F = torch.nn.functional
        a, ainv = fields
        L = self.L
        vt = v / md.diag
        f = [None] * L
        u = [None] * L
        f[0] = torch.einsum("cn,bnyx->bcyx", self.g(W.K_WIN), vt)

        def residual(l):
            return f[l] - F.conv2d(u[l], self.g(W.K_A, l), padding=1) - a[l] * u[l]

        def smooth(l, B):
            u[l] = u[l] + F.conv2d(ainv[l] * residual(l), B, padding=1)

        for l in range(L - 1):
            u[l] = torch.zeros_like(f[l])
            for i in range(self.hdr["nu_pre"]):
                smooth(l, self.g(W.K_BPRE, l, i))
            f[l + 1] = F.conv2d(residual(l), self.g(W.K_R, l), stride=2, padding=1)
        u[L - 1] = torch.zeros_like(f[L - 1])
        for i in range(self.hdr["nu_coarse"]):
            smooth(L - 1, self.g(W.K_BC, L - 1, i))
        for l in range(L - 2, -1, -1):
            u[l] = u[l] + F.conv_transpose2d(u[l + 1], self.g(W.K_PR, l), stride=2, padding=1)
            for i in range(self.hdr["nu_post"]):
                smooth(l, self.g(W.K_BPOST, l, i))
        return self.g(W.K_S)[0] * vt + torch.einsum("nc,bcyx->bnyx", self.g(W.K_WOUT), u[0])

    def blob(self):
        t = {k: v.detach().double().cpu().numpy().astype(np.float32) for k, v in self.p.items()}
        return W.pack_mgn1(self.hdr, t)


# ------------------------------------------------------------ training ---

FAMILIES = {
    # media of the C2 family with seeds disjoint from the benchmark's (2000 + s, s < 10)
    "c2": lambda s: configs.c2(10000 + s),
    # the serving stream's family (grids 64/128/256, log-uniform eps in [1e-3, 1],
    # g in [0, 0.8]) for one direction count, seeds disjoint from the stream's
    # (3000 + r, r < 4096)
    "c3_n16": lambda s: configs.c3_request(100000 + s, ndir_choices=(16,)),
    "c3_n32": lambda s: configs.c3_request(100000 + s, ndir_choices=(32,)),
}
# batch per grid size (a step's cost grows with the grid)
BATCH_OF_GRID = {64: 16, 128: 8, 256: 2, 512: 1}


def rhs_pool(count, N, ny, nx, rng):
    """Right-hand sides mixing white noise with smooth fields: an isotropic
    multiscale Gaussian random field (the slow modes of the diffusive regime)
    and per-direction combinations of smooth fields, each normalised, with
    random weights.  Returned as a float array [count, N, ny, nx]."""
    out = np.empty((count, N, ny, nx), dtype=np.float32)
    for b in range(count):
        white = rng.standard_normal((N, ny, nx))
        iso = media.gaussian_random_field((ny, nx), 1.0, rng.uniform(0.03, 0.3), rng)[None]
        aniso = np.stack([media.gaussian_random_field((ny, nx), 1.0, rng.uniform(0.05, 0.3), rng)
                          for _ in range(2)])
        mix = rng.standard_normal((N, 2)) @ aniso.reshape(2, -1)
        parts = [white, np.broadcast_to(iso, (N, ny, nx)), mix.reshape(N, ny, nx)]
        wts = rng.dirichlet([1.0, 1.0, 1.0])
        out[b] = sum(w * p / np.linalg.norm(p) for w, p in zip(wts, parts))
    return out


class BestKeeper:
    """Guards a long run against late divergence: every `window` steps the mean loss of the
    window is compared with the best so far and the parameters of the best window are kept;
    at the end they are restored when the last window is worse by more than `slack` (or the
    loss stopped being finite)."""

    def __init__(self, window=200, slack=1.5):
        self.window, self.slack = window, slack
        self.best, self.params, self.step = math.inf, None, -1

    def update(self, it, hist, params):
        if (it + 1) % self.window:
            return
        w = float(np.mean(hist[-self.window:]))
        if math.isfinite(w) and w < self.best:
            self.best, self.step = w, it
            self.params = [q.detach().clone() for q in params]

    def finish(self, hist, params):
        """Restores the best window's parameters if needed; returns (step kept, its loss)."""
        last = float(np.mean(hist[-self.window:])) if hist else math.inf
        if self.params is None or (math.isfinite(last) and last <= self.slack * self.best):
            return len(hist) - 1, last
        with _torch().no_grad():
            for q, b in zip(params, self.params):
                q.copy_(b)
        return self.step, self.best


def train(family, scatter, steps, batch, lr, seed, log, device="cuda", media_pool=64, rhs_count=256):
    """scatter(prob) -> S [N, N] of a problem (the library's matrix)."""
    torch = _torch()
    dtype = torch.float32
    probs = [FAMILIES[family](s) for s in range(media_pool)]
    hdr, t = configs.problem_weights(probs[0])
    net = MgNet(hdr, t, device, dtype)
    opt = torch.optim.AdamW(net.params(), lr=lr, weight_decay=1e-5)
    rng = np.random.default_rng(seed)
    by_grid = {}
    for p in probs:
        by_grid.setdefault(p["n"][0], []).append(p)
    groups, pools = [], {}
    for n, ps in sorted(by_grid.items()):
        bsz = batch if len(by_grid) == 1 else BATCH_OF_GRID.get(n, 1)
        for i in range(0, len(ps), bsz):
            chunk = ps[i:i + bsz]
            groups.append(Medium(chunk, np.stack([scatter(p) for p in chunk]), device, dtype))
        N = ps[0]["dirs"].shape[0]
        log("building %d right-hand sides on %dx%d" % (rhs_count, n, n))
        pools[n] = torch.as_tensor(rhs_pool(rhs_count, N, n, n, rng), device=device)
    log("%d media in %d groups" % (len(probs), len(groups)))
    hist = []
    keeper = BestKeeper()
    t0 = time.time()
    for it in range(steps):
        lr_t = lr * 0.5 * (1 + math.cos(math.pi * it / steps))
        for gp in opt.param_groups:
            gp["lr"] = lr_t
        md = groups[int(rng.integers(0, len(groups)))]
        pool = pools[md.nx]
        B = md.sT.shape[0]
        i = torch.as_tensor(rng.integers(0, rhs_count, (2, B)), device=device)
        c = torch.as_tensor(rng.standard_normal((2, B)), dtype=dtype, device=device)
        b = c[0, :, None, None, None] * pool[i[0]] + c[1, :, None, None, None] * pool[i[1]]
        fields = net.coeffnet(md.X)
        r = b - apply_L(net(b, md, fields), md)
        loss = ((r ** 2).sum(dim=(1, 2, 3)) / (b ** 2).sum(dim=(1, 2, 3))).mean()
        opt.zero_grad()
        loss.backward()
        torch.nn.utils.clip_grad_norm_(net.params(), 1.0)
        opt.step()
        hist.append(float(loss.detach()))
        keeper.update(it, hist, net.params())
        if it % 50 == 0 or it == steps - 1:
            log("step %d loss %.4f lr %.2e (%.0f s)" % (it, hist[-1], lr_t, time.time() - t0))
        if not math.isfinite(hist[-1]):
            log("step %d: loss is not finite, stopping" % it)
            break
    kept, kept_loss = keeper.finish(hist, net.params())
    if kept != len(hist) - 1:
        log("final loss %.3g against %.3g at step %d: keeping the parameters of step %d"
            % (float(np.mean(hist[-keeper.window:])), kept_loss, kept, kept))
    net.kept_step, net.kept_loss = kept, kept_loss
    return net, hist


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--family", default="c2", choices=sorted(FAMILIES))
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--media", type=int, default=64, help="seeded media in the training pool")
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    torch = _torch()
    from . import api
    from . import _lib as L

    def log(*a):
        print(*a, flush=True)

    torch.cuda.set_device(0)
    # scattering matrices are the library's (HG kernel and normalisation of Sec. 2.1)
    cache = {}

    def scatter(p):
        # S depends on the directions, weights, g and kernel only: a small grid suffices
        key = (p["dirs"].shape[0], float(p["g"]))
        if key not in cache:
            small = configs._problem("S", 2, (4, 4, 1), p["dirs"], p["weights"], p["g"], p.get("kernel", "auto"),
                                     np.ones((4, 4)), np.zeros((4, 4)), np.ones((4, 4)), 1.0, None, None, None)
            op = api.Operator(small)
            cache[key] = op.array(L.ARR_SCATTER).cpu().numpy().reshape(p["dirs"].shape[0], -1)
            op.close()
        return cache[key]

    net, hist = train(args.family, scatter, args.steps, args.batch, args.lr, args.seed, log, media_pool=args.media)
    blob = net.blob()
    with open(args.out, "wb") as fh:
        fh.write(blob)
    rec = {"family": args.family, "steps": args.steps, "batch": args.batch, "lr": args.lr, "seed": args.seed,
           "media": args.media,
           "loss_first": hist[0], "loss_last": float(np.mean(hist[-50:])), "blob_bytes": len(blob),
           "kept_step": net.kept_step, "kept_window_loss": net.kept_loss}
    with open(args.out + ".json", "w") as fh:
        json.dump(rec, fh, indent=1)
    log(json.dumps(rec))


if __name__ == "__main__":
    sys.exit(main())
