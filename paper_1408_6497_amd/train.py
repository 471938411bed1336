"""Training of the learned smoother on the GPU, through the C ABI.

Pairs (r, e): for a Gaussian-random-field source f (power spectrum |k|^-alpha,
alpha ~ U[2, 4]) on the finest level, b = M f - mean, and the residuals
r_0 = b, r_{k+1} = r_k - A V r_k of plain FP64 V-cycles (k < cycles).  Cycle k
of a plain FP32 V-cycle on right side r_k gives two pairs, one at each position
that a learned correction takes in a learned cycle:
  pre   u = 0, one degree-3 Chebyshev application, r = r_k - A u;
  post  nu_pre applications, coarse-grid correction (restriction, V-cycle on
        the next level, prolongation), one more application, r = r_k - A u;
and, for the energy loss, e = A^+ r from a plain FP64 solve to 1e-10.  With
e~ = s N(D^-1 r / s) the loss is
  energy    ||e - e~||_A^2 / ||e||_A^2, or
  residual  ||r - A e~||_2^2 / ||r||_2^2 (the contraction the fallback test measures;
            needs no solve),
minimized by Adam in batches of 8.  Every step -- load vector, smoothing, residual, solve, net forward and
backward, loss gradient, Adam -- runs in libgmg's kernels; torch only holds the
buffers and the random-field generator.

Checkpoint file (little endian):
  magic b"GMGW", uint32 version, int32 depth, int32 order, int32 n,
  int64 step, int64 count (7776), float32 master[count], uint16 bf16[count];
  version 2 adds float32 adam_m[count], float32 adam_v[count], then uint32 length
  and that many bytes of UTF-8 JSON: the training configuration and the position
  in the pair stream (source, cycle, position), so a run can stop and resume and
  end on the same bits as an uninterrupted one.

  python -m paper_1408_6497_amd.train --n 64 --sources 10000 --out weights.gmgw
  python -m paper_1408_6497_amd.train --n 64 --depth 2 --sources 10000 --out q2_depth2.gmgw
  python -m paper_1408_6497_amd.train --resume weights.gmgw --out weights.gmgw

The net of depth d (d levels below the finest) is trained on the level at depth d of the
n-element training hierarchy: the finest level of the mesh with n / 2^d elements, whose
cycles are that hierarchy's cycles below depth d.  The file records d.
"""
import argparse
import json
import os
import struct
import sys
import time

import numpy as np

MAGIC = b"GMGW"
VERSION = 2
NW = 7776


def he_init(seed):
    """Seeded He-normal initialization (std sqrt(2 / fan_in)); the output layer scaled by 0.1."""
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal(432) * np.sqrt(2.0 / 27.0)
    w2 = rng.standard_normal(6912) * np.sqrt(2.0 / (16.0 * 27.0))
    w3 = rng.standard_normal(432) * np.sqrt(2.0 / (16.0 * 27.0)) * 0.1
    return np.concatenate([w1, w2, w3]).astype(np.float32)


def bf16_bits(w):
    """Round-to-nearest-even BF16 bit patterns of FP32 values."""
    u = np.ascontiguousarray(w, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def save(path, w, depth, order, n, step, m=None, v=None, extra=None):
    """Write a checkpoint: version 2 when the Adam moments are given, else version 1."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    version = 2 if m is not None else 1
    with open(path + ".tmp", "wb") as fh:
        fh.write(MAGIC + struct.pack("<Iiiiqq", version, depth, order, n, step, NW))
        fh.write(w.tobytes())
        fh.write(bf16_bits(w).tobytes())
        if version == 2:
            fh.write(np.ascontiguousarray(m, dtype=np.float32).tobytes())
            fh.write(np.ascontiguousarray(v, dtype=np.float32).tobytes())
            blob = json.dumps(extra or {}).encode()
            fh.write(struct.pack("<I", len(blob)) + blob)
    os.replace(path + ".tmp", path)


def load(path):
    with open(path, "rb") as fh:
        head = fh.read(4 + struct.calcsize("<Iiiiqq"))
        if head[:4] != MAGIC:
            raise ValueError(f"{path}: not a weights file")
        version, depth, order, n, step, count = struct.unpack("<Iiiiqq", head[4:])
        if version not in (1, 2) or count != NW:
            raise ValueError(f"{path}: unsupported version {version} / count {count}")
        w = np.frombuffer(fh.read(4 * NW), dtype=np.float32).copy()
        wb = np.frombuffer(fh.read(2 * NW), dtype=np.uint16).copy()
        out = {"w": w, "bf16": wb, "depth": depth, "order": order, "n": n, "step": step, "version": version,
               "m": None, "v": None, "extra": None}
        if version == 2:
            out["m"] = np.frombuffer(fh.read(4 * NW), dtype=np.float32).copy()
            out["v"] = np.frombuffer(fh.read(4 * NW), dtype=np.float32).copy()
            (ln,) = struct.unpack("<I", fh.read(4))
            out["extra"] = json.loads(fh.read(ln).decode())
    return out


class PairMaker:
    """(r, e) pairs on the finest level of `ctx` (a plain FP64 context)."""

    def __init__(self, ctx, cctx=None, nu_pre=2):
        """cctx: a context on the next coarser mesh (same order, same options), whose
        finest-level V-cycle is the coarse-grid correction of ctx's V-cycle; needed
        for pairs at the post-smoothing position."""
        import torch
        self.torch = torch
        self.ctx = ctx
        self.cctx = cctx
        self.nu_pre = nu_pre
        n = ctx.num_dofs()
        self.N = ctx.lattice()
        dev = "cuda"
        if cctx is not None:
            nc = cctx.num_dofs()
            if nc != ctx.num_dofs(ctx.levels - 2):
                raise ValueError("cctx is not the next coarser mesh")
            self.rc32 = torch.empty(nc, dtype=torch.float32, device=dev)
            self.ec32 = torch.empty(nc, dtype=torch.float32, device=dev)
        self.b64 = torch.empty(n, dtype=torch.float64, device=dev)
        self.b32 = torch.empty(n, dtype=torch.float32, device=dev)
        self.u32 = torch.empty(n, dtype=torch.float32, device=dev)
        self.r32 = torch.empty(n, dtype=torch.float32, device=dev)
        self.r64 = torch.empty(n, dtype=torch.float64, device=dev)
        self.e64 = torch.empty(n, dtype=torch.float64, device=dev)
        self.e32 = torch.empty(n, dtype=torch.float32, device=dev)

    def source(self, seed):
        """b = load vector of the seeded random field (the right side of cycle 0)."""
        from workloads import grf
        f, _ = grf(self.N, seed, device="cuda")
        self.ctx.rhs(f, self.b64)

    def next_cycle(self):
        """b <- b - A V b: the residual after one more plain FP64 V-cycle."""
        self.ctx.vcycle(self.b64, self.e64)
        self.ctx.residual(-1, self.b64, self.e64, self.r64)
        self.b64.copy_(self.r64)

    def pair(self, position="pre", need_e=True):
        """(r, e) at a replaced smoother's position of the cycle whose right side is b."""
        c = self.ctx
        self.b32.copy_(self.b64)
        self.u32.zero_()
        if position == "pre":
            c.smooth(-1, self.b32, self.u32, 1)
        else:
            c.smooth(-1, self.b32, self.u32, self.nu_pre)
            c.residual(-1, self.b32, self.u32, self.r32)
            c.restrict(-1, self.r32, self.rc32)
            self.cctx.vcycle(self.rc32, self.ec32)
            c.prolong(-1, self.ec32, self.u32)
            c.smooth(-1, self.b32, self.u32, 1)
        c.residual(-1, self.b32, self.u32, self.r32)
        if not need_e:
            return self.r32, None
        self.r64.copy_(self.r32)
        self.ctx.solve_rhs(self.r64, self.e64, 1e-10)
        self.e32.copy_(self.e64)
        return self.r32, self.e32

    def make(self, seed, cycle=0, position="pre", need_e=True):
        self.source(seed)
        for _ in range(cycle):
            self.next_cycle()
        return self.pair(position, need_e)


def chebyshev_loss(ctx, r32, e32, tmp, kind):
    """The same loss for the polynomial application the net replaces: e~ = S(r) from zero."""
    from paper_1408_6497_amd import LOSS_ENERGY
    et, d = tmp
    et.zero_()
    ctx.smooth(-1, r32, et, 1)
    ctx.residual(-1, r32, et, d)
    if kind == LOSS_ENERGY:
        er = ctx.dot(e32, r32)
        return (ctx.dot(e32, d) - ctx.dot(et, d)) / er
    return ctx.dot(d, d) / ctx.dot(r32, r32)


def validate(ctx, pm, cache, seeds, kind, with_cheb=False, cycles=1, positions=("pre",)):
    """Mean loss over the validation sources; source i is taken at cycle i mod cycles
    and position (i div cycles) mod len(positions)."""
    import torch
    from paper_1408_6497_amd import LOSS_ENERGY
    losses, cheb = [], []
    tmp = (torch.empty_like(pm.r32), torch.empty_like(pm.r32))
    for i, s in enumerate(seeds):
        r, e = pm.make(s, i % cycles, positions[(i // cycles) % len(positions)], kind == LOSS_ENERGY)
        losses.append(ctx.net_loss_grad(0, r, e, cache, kind=kind))
        if with_cheb:
            cheb.append(chebyshev_loss(ctx, r, e, tmp, kind))
    return float(np.mean(losses)), (float(np.mean(cheb)) if with_cheb else None)


def train(n=64, sources=10000, batch=8, lr=1e-3, val=100, init_seed=12345, out=None, log=print,
          train_seed0=0, val_seed0=20000, cycles=2, positions=("pre", "post"), loss="residual",
          stop_after=None, resume=None, depth=0):
    """Adam on the net of one depth (trained on the finest level of the n / 2^depth-element mesh);
    stop_after ends the run early (a checkpoint to resume from), resume continues a version-2
    checkpoint with its own configuration."""
    import torch
    from paper_1408_6497_amd import Context, GMG_FP64, LOSS_ENERGY, LOSS_RESIDUAL
    ck = None
    if resume:
        ck = load(resume)
        if ck["version"] < 2:
            raise ValueError(f"{resume}: version 1 checkpoints hold no optimizer state")
        cfg = ck["extra"]["config"]
        n, sources, batch, lr, val = cfg["n"], cfg["sources"], cfg["batch"], cfg["lr"], cfg["val"]
        init_seed, train_seed0, val_seed0 = cfg["init_seed"], cfg["train_seed0"], cfg["val_seed0"]
        cycles, positions, loss = cfg["cycles"], tuple(cfg["positions"]), cfg["loss"]
        depth = cfg.get("depth", 0)
    config = {"n": n, "sources": sources, "batch": batch, "lr": lr, "val": val, "init_seed": init_seed,
              "train_seed0": train_seed0, "val_seed0": val_seed0, "cycles": cycles, "positions": list(positions),
              "loss": loss, "depth": depth}
    nd = n >> depth
    if nd < 8 or nd << depth != n:
        raise ValueError(f"depth {depth} leaves {n / 2 ** depth} elements of the {n}-element mesh (8 at least)")
    kind = {"energy": LOSS_ENERGY, "residual": LOSS_RESIDUAL}[loss]
    ctx = Context(2, nd, 0, seed=0, vcycle_prec=GMG_FP64)
    cctx = Context(2, nd // 2, 0, seed=0, vcycle_prec=GMG_FP64) if "post" in positions else None
    pm = PairMaker(ctx, cctx)
    if ck:
        ctx.net_set_state(0, ck["w"], ck["m"], ck["v"])
    else:
        ctx.net_set_weights(0, he_init(init_seed))
    cache = ctx.net_cache(0)
    gw = torch.zeros(NW, dtype=torch.float32, device="cuda")
    vseeds = range(val_seed0, val_seed0 + val)
    v0, vcheb = validate(ctx, pm, cache, vseeds, kind, with_cheb=True, cycles=cycles, positions=positions)
    log(f"[train] validation before: loss {v0:.4f}  (Chebyshev application it replaces: {vcheb:.4f})")
    # each source contributes cycles x positions consecutive pairs
    state = dict(ck["extra"]["stream"]) if ck else {"src": 0, "cyc": 0, "pos": 0}
    if state["cyc"] > 0 or state["pos"] > 0:
        # rebuild the right side the next pair starts from
        pm.source(train_seed0 + state["src"])
        for _ in range(state["cyc"] - (1 if state["pos"] == 0 else 0)):
            pm.next_cycle()

    def next_pair():
        if state["pos"] == 0:
            if state["cyc"] == 0:
                pm.source(train_seed0 + state["src"])
            else:
                pm.next_cycle()
        r, e = pm.pair(positions[state["pos"]], kind == LOSS_ENERGY)
        state["pos"] += 1
        if state["pos"] == len(positions):
            state["pos"], state["cyc"] = 0, state["cyc"] + 1
            if state["cyc"] == cycles:
                state["src"], state["cyc"] = state["src"] + 1, 0
        return r, e

    steps = sources * cycles * len(positions) // batch
    step0 = ck["step"] if ck else 0
    last = steps if stop_after is None else min(steps, step0 + stop_after)
    t0 = time.perf_counter()
    hist = []
    for step in range(step0 + 1, last + 1):
        gw.zero_()
        tot = 0.0
        for k in range(batch):
            r, e = next_pair()
            tot += ctx.net_loss_grad(0, r, e, cache, gw, scale=1.0 / batch, kind=kind)
        ctx.adam_step(0, gw, lr, step)
        hist.append(tot / batch)
        if step % max(1, steps // 20) == 0 or step == steps:
            log(f"[train] step {step}/{steps} loss {np.mean(hist[-50:]):.4f} ({time.perf_counter() - t0:.1f} s)")
    w, m, v = ctx.net_get_state(0)
    if out:
        save(out, w, depth, 2, nd, last, m, v, {"config": config, "stream": state})
    v1, _ = validate(ctx, pm, cache, vseeds, kind, cycles=cycles, positions=positions)
    log(f"[train] validation after: loss {v1:.4f}")
    return {"w": w, "val_before": v0, "val_after": v1, "val_chebyshev": vcheb, "steps": last - step0,
            "step": last, "seconds": time.perf_counter() - t0, "loss_history": hist}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64, help="Q2 elements per direction of the training grid")
    ap.add_argument("--sources", type=int, default=10000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--val", type=int, default=100)
    ap.add_argument("--cycles", type=int, default=2, help="cycles 0 .. cycles-1 of each source give pairs")
    ap.add_argument("--positions", default="pre,post", help="pair positions in the cycle: pre, post or both")
    ap.add_argument("--loss", default="residual", choices=("residual", "energy"))
    ap.add_argument("--out", default=None)
    ap.add_argument("--stop-after", type=int, default=None, help="stop after this many Adam steps (checkpoint)")
    ap.add_argument("--resume", default=None, help="continue a version-2 checkpoint")
    ap.add_argument("--depth", type=int, default=0, help="the net's depth below the finest level")
    a = ap.parse_args()
    res = train(a.n, a.sources, a.batch, a.lr, a.val, out=a.out, log=lambda *m: print(*m, flush=True),
                cycles=a.cycles, positions=tuple(a.positions.split(",")), loss=a.loss,
                stop_after=a.stop_after, resume=a.resume, depth=a.depth)
    print(f"[train] done: {res['steps']} steps in {res['seconds']:.1f} s; validation {res['val_before']:.4f} -> "
          f"{res['val_after']:.4f} (Chebyshev {res['val_chebyshev']:.4f})", flush=True)


if __name__ == "__main__":
    ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    main()
