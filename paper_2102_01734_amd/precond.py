"""Learned ALI correction: weight-blob format, the training model and the
trainer (offline tool; inference runs in the library's HIP kernels).

The network (include/rt3d.h, rt_set_preconditioner) maps per-voxel features
(r / max|r|, log10 chi / 4, log10 eps / 3 + 1), r = (J_fs - J) / J the
formal-solution residual of the iterate before an ALI update, to a relative
correction c of the ALI iterate: J <- J (1 + clamp(max|r| c, -1/2, 1)).
Training pairs come from the solver itself: for synthetic fields, plain
Ng-ALI iterates J_k, their residuals r_k, the updated iterates J_{k+1}, and
the converged J*; the target is (J*/J_{k+1} - 1) / max|r_k|.

PyTorch is used here for autograd only.  The model mirrors the kernels:
3x3x3 convolutions periodic in x, y and zero-padded in z, stride-2
convolutions down, linear (align-corners) 2x upsampling then a convolution
up, additive skips, ReLU after every convolution but the 1x1 head.
"""
from __future__ import annotations

import struct
from typing import List, Sequence

import numpy as np

MAGIC = b"RTUN"
VERSION = 1


def conv_shapes(C: Sequence[int]):
    """(c_in, c_out, taps) of every convolution in blob order."""
    L = len(C)
    out = [(3, C[0], 27), (C[0], C[0], 27)]
    for l in range(1, L):
        out += [(C[l - 1], C[l], 27), (C[l], C[l], 27)]
    for l in range(L - 1, 0, -1):
        out += [(C[l], C[l - 1], 27), (C[l - 1], C[l - 1], 27)]
    out.append((C[0], 1, 1))
    return out


def pack_blob(C: Sequence[int], convs: Sequence) -> bytes:
    """convs: [(W [taps][c_out][c_in], b [c_out]), ...] in blob order (float32)."""
    shapes = conv_shapes(C)
    if len(convs) != len(shapes):
        raise ValueError(f"expected {len(shapes)} convolutions, got {len(convs)}")
    parts = [MAGIC, struct.pack("<II", VERSION, len(C)), struct.pack(f"<{len(C)}I", *C)]
    for (ci, co, taps), (W, b) in zip(shapes, convs):
        W = np.ascontiguousarray(W, dtype="<f4")
        b = np.ascontiguousarray(b, dtype="<f4")
        if W.shape != (taps, co, ci) or b.shape != (co,):
            raise ValueError(f"bad shapes {W.shape} {b.shape} for ({taps}, {co}, {ci})")
        parts += [W.tobytes(), b.tobytes()]
    return b"".join(parts)


def unpack_blob(blob: bytes):
    if blob[:4] != MAGIC:
        raise ValueError("not a network blob")
    ver, L = struct.unpack_from("<II", blob, 4)
    C = list(struct.unpack_from(f"<{L}I", blob, 12))
    off = 12 + 4 * L
    convs = []
    for ci, co, taps in conv_shapes(C):
        n = taps * co * ci
        W = np.frombuffer(blob, "<f4", n, off).reshape(taps, co, ci).copy()
        off += 4 * n
        b = np.frombuffer(blob, "<f4", co, off).copy()
        off += 4 * co
        convs.append((W, b))
    return C, convs


def random_blob(C: Sequence[int], seed: int = 0, scale: float = 1.0) -> bytes:
    """He-initialised weights (for tests)."""
    rng = np.random.default_rng(seed)
    convs = []
    for ci, co, taps in conv_shapes(C):
        W = rng.standard_normal((taps, co, ci)) * scale * np.sqrt(2.0 / (taps * ci))
        b = rng.standard_normal(co) * 0.05 * scale
        convs.append((W, b))
    return pack_blob(C, convs)


# ---------------------------------------------------------------------------
# PyTorch model for training
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def build_model(C: Sequence[int]):
    """The network as a torch module on one channels-last volume [Z][Y][X][3]
    -> [Z][Y][X].  Each 3x3x3 convolution is the sum over its 27 taps of a
    shifted slice times the tap's [c_in, c_out] matrix (plain GEMMs), with the
    parameters held exactly as the blob stores them."""
    torch = _torch()
    nn = torch.nn

    def pad(x):
        x = torch.cat([x[:, -1:], x, x[:, :1]], dim=1)          # y periodic
        x = torch.cat([x[:, :, -1:], x, x[:, :, :1]], dim=2)    # x periodic
        return torch.nn.functional.pad(x, (0, 0, 0, 0, 0, 0, 1, 1))  # z zero

    def conv(x, W, b, stride=1):
        Z, Y, X = x.shape[:3]
        if stride == 2:
            Z, Y, X = (Z + 1) // 2, (Y + 1) // 2, (X + 1) // 2
        xp = pad(x)
        out = b
        for dz in range(3):
            for dy in range(3):
                for dx in range(3):
                    sl = xp[dz:dz + stride * (Z - 1) + 1:stride, dy:dy + stride * (Y - 1) + 1:stride,
                            dx:dx + stride * (X - 1) + 1:stride]
                    out = out + torch.matmul(sl, W[(dz * 3 + dy) * 3 + dx].t())
        return out

    def up2(x, shape):
        for ax, (n_f, periodic) in zip((0, 1, 2), ((shape[0], False), (shape[1], True), (shape[2], True))):
            n_c = x.shape[ax]
            o = torch.arange(n_f, device=x.device)
            i1 = (o + 1) // 2
            i1 = i1 % n_c if periodic else torch.clamp(i1, max=n_c - 1)
            x = 0.5 * (x.index_select(ax, o // 2) + x.index_select(ax, i1))
        return x

    class Net(nn.Module):
        def __init__(self):
            super().__init__()
            self.C = list(C)
            self.L = len(C)
            ws, bs = [], []
            for ci, co, taps in conv_shapes(C):
                ws.append(nn.Parameter(torch.randn(taps, co, ci) * np.sqrt(2.0 / (taps * ci))))
                bs.append(nn.Parameter(torch.zeros(co)))
            self.W = nn.ParameterList(ws)
            self.b = nn.ParameterList(bs)

        def forward(self, f):
            relu = torch.relu
            k = iter(range(len(self.W)))

            def nxt(x, stride=1):
                i = next(k)
                return conv(x, self.W[i], self.b[i], stride)

            h = [None] * self.L
            x = relu(nxt(f))
            h[0] = relu(nxt(x))
            for l in range(1, self.L):
                x = relu(nxt(h[l - 1], 2))
                h[l] = relu(nxt(x))
            for l in range(self.L - 1, 0, -1):
                u = up2(h[l], h[l - 1].shape[:3])
                x = relu(nxt(u)) + h[l - 1]
                h[l - 1] = relu(nxt(x))
            i = next(k)
            return torch.matmul(h[0], self.W[i][0].t())[..., 0] + self.b[i][0]

    return Net()


def export_blob(model) -> bytes:
    convs = [(W.detach().cpu().numpy().astype(np.float32), b.detach().cpu().numpy().astype(np.float32))
             for W, b in zip(model.W, model.b)]
    return pack_blob(model.C, convs)


def load_into(model, blob: bytes):
    torch = _torch()
    C, convs = unpack_blob(blob)
    assert list(C) == list(model.C)
    with torch.no_grad():
        for W, b, (Wn, bn) in zip(model.W, model.b, convs):
            W.copy_(torch.from_numpy(Wn))
            b.copy_(torch.from_numpy(bn))


def features_torch(r, scale, chi, eps):
    """The network's input features, as the library forms them ([Z][Y][X][3])."""
    torch = _torch()
    f0 = r / scale
    f1 = torch.log10(torch.clamp(chi, min=1e-30)) * 0.25
    f2 = torch.log10(torch.clamp(eps, min=1e-30)) / 3.0 + 1.0
    return torch.stack([f0, f1, f2], dim=-1)


# ---------------------------------------------------------------------------
# training data from the solver
# ---------------------------------------------------------------------------
def trajectory_samples(case, n_steps: int, every: int = 1, tol_star: float = 1e-9, max_iter: int = 400,
                       prec: str = "f64", log=None) -> List[dict]:
    """Runs plain Ng-ALI on `case` (one wavelength) through the library and returns
    training samples (features on the GPU, target) for steps 1..n_steps."""
    torch = _torch()
    from . import rt3d
    dev = "cuda"
    dt = torch.float64 if prec == "f64" else torch.float32
    g = rt3d.Grid(case.Nx, case.Ny, case.Nz, case.n_mu, case.n_phi, prec, 1)
    chi = torch.tensor(case.chi, dtype=dt, device=dev)
    eps = torch.tensor(case.eps, dtype=dt, device=dev)
    B = torch.tensor(case.B, dtype=dt, device=dev)
    Ib = torch.tensor(case.I_bc, dtype=dt, device=dev)
    # converged solution
    st = g.new_state(chi, eps, B, Ib)
    status, rep = g.solve(st, g.opts(tol=tol_star, max_iter=max_iter))
    if log:
        log(f"reference solve: status {status}, {rep.iters} steps, last change {rep.max_rel_change:.2e}")
    Jstar = g.state_tensors(st)["J"].clone()
    # replay the plain trajectory step by step
    st = g.new_state(chi, eps, B, Ib)
    opts = g.opts(tol=1e-300, max_iter=1)
    out = []
    for k in range(1, n_steps + 1):
        t = g.state_tensors(st)
        Jk = t["J"].clone()
        Sk = t["S"].clone() if k > 1 else None
        g.ali_step(st, opts)
        t = g.state_tensors(st)
        Jn = t["J"]
        if k % every or Sk is None:
            continue
        Jfs, _ = g.formal_solution(chi, Sk.to(dt), Ib)
        # keep only steps whose formal solution ran on J_k itself (no Ng extrapolation first)
        den = torch.clamp(1.0 - (1.0 - eps.double()) * t["lstar"].double(), min=1e-12)
        Jpred = Jk + (Jfs.double() - Jk) / den
        if float(((Jpred - Jn).abs() / Jn.abs()).max()) > 1e-6:
            continue
        r = (Jfs.double() - Jk) / Jk
        s = float(r.abs().max())
        if not s > 0:
            continue
        target = (Jstar / Jn - 1.0) / s
        f = features_torch(r[0].float(), s, chi[0].float(), eps[0].float())
        out.append(dict(f=f, target=target[0].float(), s=s, step=k))
    g.close()
    return out


def train(samples: List[dict], C=(16, 32, 32), iters: int = 1500, lr: float = 2e-3, seed: int = 0, crop: int = 48,
          margin: int = 6, log=print):
    """Adam on random crops (crop^3, loss on the interior away from the crop's
    artificial borders) of the samples."""
    import time
    torch = _torch()
    torch.manual_seed(seed)
    model = build_model(C).cuda()
    opt = torch.optim.Adam(model.parameters(), lr=lr)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, iters)
    rng = np.random.default_rng(seed)
    t0 = time.time()
    m = margin
    for it in range(iters):
        smp = samples[int(rng.integers(len(samples)))]
        f, tg = smp["f"], smp["target"]
        o = [int(rng.integers(0, max(n - crop, 0) + 1)) for n in tg.shape]
        sl = tuple(slice(a, a + crop) for a in o)
        pred = model(f[sl])
        d = (pred - tg[sl])[m:-m, m:-m, m:-m]
        loss = torch.mean(d * d)
        opt.zero_grad()
        loss.backward()
        opt.step()
        sched.step()
        if it % 100 == 0 or it == iters - 1:
            log(f"train iter {it} loss {float(loss.detach()):.4e} ({time.time() - t0:.1f} s)")
    return model


def main(argv=None):
    """Trains a network on plain Ng-ALI trajectories of synthetic stratified x
    log-normal boxes (seeds disjoint from the benchmark's) and writes the blob."""
    import argparse
    import time

    import synthetic as sy
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--out", required=True)
    ap.add_argument("--N", type=int, default=129)
    ap.add_argument("--n-mu", type=int, default=8)
    ap.add_argument("--n-phi", type=int, default=16)
    ap.add_argument("--trajectories", type=int, default=16)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--seed0", type=int, default=1000)
    ap.add_argument("--channels", default="16,32,32")
    ap.add_argument("--iters", type=int, default=1500)
    ap.add_argument("--lr", type=float, default=2e-3)
    a = ap.parse_args(argv)
    t0 = time.time()
    samples = []
    for k in range(a.trajectories):
        seed = a.seed0 + k
        case = sy.box_lognormal(N=a.N, n_mu=a.n_mu, n_phi=a.n_phi, field_seed=seed, eps_seed=seed + 100000,
                                dtype="f64")
        smp = trajectory_samples(case, a.steps, log=lambda m: print(m, flush=True))
        samples += smp
        print(f"trajectory {k} (seed {seed}): {len(smp)} samples, {time.time() - t0:.1f} s", flush=True)
    C = tuple(int(c) for c in a.channels.split(","))
    model = train(samples, C=C, iters=a.iters, lr=a.lr, log=lambda m: print(m, flush=True))
    blob = export_blob(model)
    with open(a.out, "wb") as f:
        f.write(blob)
    print(f"wrote {a.out} ({len(blob)} bytes) after {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
