"""Out-of-core-shaped hierarchical solve: bricks streamed through a device pool.

The fine volume and its seed labels stay in host memory; the device holds
the LOD levels, the coarse solution, the fine seed map (for the brick
classification) and a fixed pool of brick sub-volumes.  Steps (every one a
librw.so call; this module only moves buffers and sequences calls):

1. level 1 from the fine volume brick by brick: pinned host staging buffer
   -> async H2D on a copy stream -> rw_downsample of the brick -> placed
   into the device level-1 volume; level 2 = rw_downsample(level 1);
2. whole solve of level 2 (rw_solve);
3. rw_classify_bricks on the fine brick grid;
4. uncertain bricks in batches of `pool` slots: each brick with its
   one-voxel halo (clipped to the volume) copied H2D into its slot while the
   previous batch is being solved (two pools, double-buffered), then one
   rw_solve_bricks over the batch's sub-volumes, then D2H of the brick
   probabilities into the host output;
5. certain bricks: rw_fill_bricks of the upsampled coarse probabilities into
   a device brick buffer, D2H.

Output: float32 probabilities [K][nz][ny][nx] and/or the uint8 label map
(rw_argmax on the device, only labels cross PCIe) in host memory.  The PCIe
traffic is reported separately from the solves.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import rw


def _brick_grid(shape, brick):
    out = []
    for z in range(0, shape[0], brick[0]):
        for y in range(0, shape[1], brick[1]):
            for x in range(0, shape[2], brick[2]):
                out.append(((z, y, x), (min(brick[0], shape[0] - z), min(brick[1], shape[1] - y),
                                        min(brick[2], shape[2] - x))))
    return out


def streamed_solve(vol_host, lab_host, K, beta, brick=(128, 128, 128), pool=16, tol=1e-6,
                   levels=2, lo=None, hi=None, lo_thr=0.02, hi_thr=0.98, precision="mixed",
                   out=None, labels_out=None, ctx=None, update_delta=None):
    """vol_host: uint16 or float32 numpy [nz][ny][nx]; lab_host: uint8 numpy.

    Brick sizes must be even (level-1 blocks must not straddle bricks).
    lo, hi: the normalisation g = (v - lo) / (hi - lo); None takes 0 and
    65535 for uint16 volumes and the volume's own minimum and maximum for
    float32 ones.
    out: float32 [K][...] host array for the probabilities; labels_out: uint8
    [...] host array for the label map.  With neither given, probabilities
    are returned.  update_delta: the brick solves' float64 refresh threshold
    (None: the brick default).  Returns (out, info dict with timings and
    counts).
    """
    if not all(b % 2 == 0 for b in brick):
        raise ValueError("brick sizes must be even")
    ctx = ctx or rw.default_context()
    if vol_host.dtype == np.uint16:
        lo = 0.0 if lo is None else float(lo)
        hi = 65535.0 if hi is None else float(hi)
    elif vol_host.dtype == np.float32:
        # min-max normalisation over the whole level-0 volume
        lo = float(np.min(vol_host)) if lo is None else float(lo)
        hi = float(np.max(vol_host)) if hi is None else float(hi)
    else:
        raise TypeError(f"streamed volumes are uint16 or float32, not {vol_host.dtype}")
    dev = torch.device("cuda")
    shape = tuple(int(s) for s in vol_host.shape)
    tdt = torch.from_numpy(vol_host[:1, :1, :1].copy()).dtype
    copy = torch.cuda.Stream()
    main = torch.cuda.current_stream()
    info = dict(h2d_bytes=0, d2h_bytes=0)
    t_all = time.perf_counter()

    # ---- level 1 brick by brick, fine seed map kept on the device
    l1_shape = tuple((s + 1) // 2 for s in shape)
    g1 = torch.empty(l1_shape, dtype=torch.float32, device=dev)
    l1 = torch.empty(l1_shape, dtype=torch.uint8, device=dev)
    lab_dev = torch.empty(shape, dtype=torch.uint8, device=dev)
    grid = _brick_grid(shape, brick)
    stage_v = [torch.empty(brick, dtype=tdt).pin_memory() for _ in range(2)]
    stage_l = [torch.empty(brick, dtype=torch.uint8).pin_memory() for _ in range(2)]
    dbuf_v = [torch.empty(brick, dtype=tdt, device=dev) for _ in range(2)]
    dbuf_l = [torch.empty(brick, dtype=torch.uint8, device=dev) for _ in range(2)]
    done = [torch.cuda.Event() for _ in range(2)]
    ready = [torch.cuda.Event() for _ in range(2)]
    t0 = time.perf_counter()
    for i, (o, s) in enumerate(grid):
        k = i & 1
        done[k].synchronize()  # slot k's previous brick has been consumed
        sv = stage_v[k][:s[0], :s[1], :s[2]]
        sl = stage_l[k][:s[0], :s[1], :s[2]]
        sv.copy_(torch.from_numpy(vol_host[o[0]:o[0] + s[0], o[1]:o[1] + s[1], o[2]:o[2] + s[2]]))
        sl.copy_(torch.from_numpy(lab_host[o[0]:o[0] + s[0], o[1]:o[1] + s[1], o[2]:o[2] + s[2]]))
        dv = dbuf_v[k][:s[0], :s[1], :s[2]]
        dl = dbuf_l[k][:s[0], :s[1], :s[2]]
        with torch.cuda.stream(copy):
            dv.copy_(sv, non_blocking=True)
            dl.copy_(sl, non_blocking=True)
            ready[k].record(copy)
        main.wait_event(ready[k])
        dvc, dlc = dv.contiguous(), dl.contiguous()
        gb, lb = rw.downsample(dvc, dlc, lo=lo, hi=hi, out_dtype=torch.float32, ctx=ctx)
        c = tuple(v // 2 for v in o)
        g1[c[0]:c[0] + gb.shape[0], c[1]:c[1] + gb.shape[1], c[2]:c[2] + gb.shape[2]] = gb
        l1[c[0]:c[0] + gb.shape[0], c[1]:c[1] + gb.shape[1], c[2]:c[2] + gb.shape[2]] = lb
        lab_dev[o[0]:o[0] + s[0], o[1]:o[1] + s[1], o[2]:o[2] + s[2]] = dlc
        done[k].record(main)
        info["h2d_bytes"] += sv.numel() * sv.element_size() + sl.numel()
    torch.cuda.synchronize()
    info["lod_s"] = time.perf_counter() - t0
    g, lab = g1, l1
    for _ in range(levels - 1):
        g, lab = rw.downsample(g, lab, lo=0.0, hi=1.0, out_dtype=torch.float32, ctx=ctx)

    # ---- coarse solve and classification
    t0 = time.perf_counter()
    coarse, _, cst = rw.solve(g, lab, K, beta, tol=tol, precision=precision, lo=0.0, hi=1.0,
                              argmax=False, ctx=ctx, return_stats=True)
    f = 2 ** levels
    cands, active = rw.classify_bricks(coarse, lab_dev, f, brick, (0, 0, 0), lo_thr, hi_thr,
                                       ctx=ctx)
    torch.cuda.synchronize()
    info["coarse_s"] = time.perf_counter() - t0
    info["coarse_iters"] = cst["iters"]
    info["coarse"] = coarse
    act = [b for b, a in zip(cands, active) if a]
    ina = [b for b, a in zip(cands, active) if not a]
    info["bricks"] = len(cands)
    info["active_bricks"] = len(act)
    if out is None and labels_out is None:
        out = np.empty((K,) + shape, dtype=np.float32)

    # ---- certain bricks: upsampled coarse probabilities (labels only are streamed)
    t0 = time.perf_counter()
    bvox = int(np.prod(brick))
    nfill = max(1, min(pool, len(ina)))
    fl = torch.zeros((1, 1, nfill * bvox), dtype=torch.uint8, device=dev)
    fp = torch.empty((K, 1, 1, nfill * bvox), dtype=torch.float32, device=dev)
    for i0 in range(0, len(ina), nfill):
        chunk = ina[i0:i0 + nfill]
        subs, local = [], []
        for j, (o, s) in enumerate(chunk):
            n = int(np.prod(s))
            fl.view(-1)[j * bvox:j * bvox + n] = lab_dev[o[0]:o[0] + s[0], o[1]:o[1] + s[1],
                                                         o[2]:o[2] + s[2]].reshape(-1)
            subs.append((j * bvox, s, o))
            local.append(((0, 0, 0), s))
        rw.fill_bricks(coarse, fl, f, local, fp, subvols=subs, ctx=ctx)
        fv = fp.view(K, -1)
        am = rw.argmax(fv, ctx=ctx) if labels_out is not None else None
        for j, (o, s) in enumerate(chunk):
            n = int(np.prod(s))
            sl = (slice(o[0], o[0] + s[0]), slice(o[1], o[1] + s[1]), slice(o[2], o[2] + s[2]))
            if out is not None:
                out[(slice(None),) + sl] = fv[:, j * bvox:j * bvox + n].reshape(
                    (K,) + tuple(s)).cpu().numpy()
                info["d2h_bytes"] += K * n * 4
            if am is not None:
                labels_out[sl] = am[j * bvox:j * bvox + n].reshape(tuple(s)).cpu().numpy()
                info["d2h_bytes"] += n
    torch.cuda.synchronize()
    info["fill_s"] = time.perf_counter() - t0

    # ---- uncertain bricks through the pool
    t0 = time.perf_counter()
    hal = tuple(b + 2 for b in brick)
    slot = int(np.prod(hal))
    pools = [dict(v=torch.empty((1, 1, pool * slot), dtype=tdt, device=dev),
                  l=torch.zeros((1, 1, pool * slot), dtype=torch.uint8, device=dev),
                  p=torch.empty((K, 1, 1, pool * slot), dtype=torch.float32, device=dev),
                  sv=torch.empty((pool * slot,), dtype=tdt).pin_memory(),
                  sl=torch.empty((pool * slot,), dtype=torch.uint8).pin_memory(),
                  ev=torch.cuda.Event(), done=torch.cuda.Event()) for _ in range(2)]
    batches = [act[i:i + pool] for i in range(0, len(act), pool)]
    meta = []

    def stage(bi):
        P = pools[bi & 1]
        P["done"].synchronize()
        subs, bricks_local = [], []
        off = 0
        for o, s in batches[bi]:
            lo_ = [max(o[a] - 1, 0) for a in range(3)]
            hi_ = [min(o[a] + s[a] + 1, shape[a]) for a in range(3)]
            dims = tuple(hi_[a] - lo_[a] for a in range(3))
            n = int(np.prod(dims))
            P["sv"][off:off + n].copy_(torch.from_numpy(
                np.ascontiguousarray(vol_host[lo_[0]:hi_[0], lo_[1]:hi_[1], lo_[2]:hi_[2]]).ravel()))
            P["sl"][off:off + n].copy_(torch.from_numpy(
                np.ascontiguousarray(lab_host[lo_[0]:hi_[0], lo_[1]:hi_[1], lo_[2]:hi_[2]]).ravel()))
            subs.append((off, dims, tuple(lo_)))
            bricks_local.append((tuple(o[a] - lo_[a] for a in range(3)), s))
            off += n
        with torch.cuda.stream(copy):
            P["v"].view(-1)[:off].copy_(P["sv"][:off], non_blocking=True)
            P["l"].view(-1)[:off].copy_(P["sl"][:off], non_blocking=True)
            P["ev"].record(copy)
        info["h2d_bytes"] += off * (P["sv"].element_size() + 1)
        return subs, bricks_local

    pending = stage(0) if batches else None
    solve_s = 0.0
    iters_all = []
    for bi in range(len(batches)):
        P = pools[bi & 1]
        subs, bricks_local = pending
        main.wait_event(P["ev"])
        if bi + 1 < len(batches):
            pending = stage(bi + 1)  # overlaps the solve below
        ts = time.perf_counter()
        _, iters, bst = rw.solve_bricks(P["v"], P["l"], K, beta, coarse, f, bricks_local,
                                        prob_out=P["p"], tol=tol, precision=precision, lo=lo,
                                        hi=hi, ctx=ctx, return_stats=True, subvols=subs,
                                        update_delta=update_delta)
        solve_s += time.perf_counter() - ts
        iters_all += iters
        meta.append(bst)
        # brick interiors back to the host
        pv = P["p"].view(K, -1)
        am = rw.argmax(pv, ctx=ctx) if labels_out is not None else None
        for (off, dims, lo_), (ob, s) in zip(subs, bricks_local):
            n = int(np.prod(dims))
            g0 = tuple(lo_[a] + ob[a] for a in range(3))
            dst = (slice(g0[0], g0[0] + s[0]), slice(g0[1], g0[1] + s[1]),
                   slice(g0[2], g0[2] + s[2]))
            src = (slice(ob[0], ob[0] + s[0]), slice(ob[1], ob[1] + s[1]),
                   slice(ob[2], ob[2] + s[2]))
            if out is not None:
                inner = pv[:, off:off + n].view((K,) + dims)[(slice(None),) + src]
                out[(slice(None),) + dst] = inner.cpu().numpy()
                info["d2h_bytes"] += inner.numel() * 4
            if am is not None:
                inner = am[off:off + n].view(dims)[src]
                labels_out[dst] = inner.cpu().numpy()
                info["d2h_bytes"] += inner.numel()
        P["done"].record(main)
    torch.cuda.synchronize()
    info["bricks_s"] = time.perf_counter() - t0
    info["brick_solve_s"] = solve_s
    info["brick_iters"] = iters_all
    info["brick_stats"] = meta
    info["total_s"] = time.perf_counter() - t_all
    return (out if out is not None else labels_out), info


