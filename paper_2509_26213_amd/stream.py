"""Out-of-core-shaped hierarchical solve: bricks streamed through a device pool.

The fine volume and its seed labels stay in host memory; the device holds
the LOD levels, the coarse solution, the list of seeds (flat index and
label, a few bytes per seed) and two fixed pools of brick sub-volumes, so
only the bricks being solved are resident.  Steps (every one a librw.so
call; this module only moves buffers and sequences calls):

1. level 1 from the fine volume brick by brick: pinned host staging buffer
   -> async H2D on a copy stream -> rw_downsample of the brick -> placed
   into the device level-1 volume; the brick's seeds are appended to the
   seed list; level 2 = rw_downsample(level 1);
2. whole solve of level 2 (rw_solve);
3. rw_classify_bricks_sparse on the fine brick grid (the seed rule from the
   seed list);
4. certain bricks: their labels streamed in, rw_fill_bricks of the
   upsampled coarse probabilities, results back;
5. uncertain bricks in batches of `pool` slots: each brick with its
   one-voxel halo (clipped to the volume) copied H2D into its slot while the
   previous batch is being solved (two pools), then one rw_solve_bricks over
   the batch's sub-volumes, then an async D2H of the batch's results into a
   pinned buffer.  A worker thread stages the next batch into pinned memory
   and scatters the previous batch's results into the host output while the
   main thread waits in the (blocking) solve.

Output: float32 probabilities [K][nz][ny][nx] and/or the uint8 label map
(rw_argmax on the device, only labels cross PCIe) in host memory.  The PCIe
traffic is reported separately from the solves.
"""
from __future__ import annotations

import time
from concurrent.futures import ThreadPoolExecutor

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


def _box(a, o, s):
    return a[o[0]:o[0] + s[0], o[1]:o[1] + s[1], o[2]:o[2] + s[2]]


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

    # ---- level 1 brick by brick; the seeds into a list
    l1_shape = tuple((s + 1) // 2 for s in shape)
    g1 = torch.empty(l1_shape, dtype=torch.float32, device=dev)
    l1 = torch.empty(l1_shape, dtype=torch.uint8, device=dev)
    grid = _brick_grid(shape, brick)
    stage_v = [torch.empty(brick, dtype=tdt).pin_memory() for _ in range(2)]
    stage_l = [torch.empty(brick, dtype=torch.uint8).pin_memory() for _ in range(2)]
    dbuf_v = [torch.empty(brick, dtype=tdt, device=dev) for _ in range(2)]
    dbuf_l = [torch.empty(brick, dtype=torch.uint8, device=dev) for _ in range(2)]
    done = [torch.cuda.Event() for _ in range(2)]
    ready = [torch.cuda.Event() for _ in range(2)]
    seed_idx, seed_lab = [], []
    t0 = time.perf_counter()
    for i, (o, s) in enumerate(grid):
        k = i & 1
        done[k].synchronize()  # slot k's previous brick has been consumed
        n = int(np.prod(s))
        sv = stage_v[k].view(-1)[:n].view(s)   # contiguous staging of this brick
        sl = stage_l[k].view(-1)[:n].view(s)
        sv.copy_(torch.from_numpy(_box(vol_host, o, s)))
        sl.copy_(torch.from_numpy(_box(lab_host, o, s)))
        dv = dbuf_v[k].view(-1)[:n].view(s)
        dl = dbuf_l[k].view(-1)[:n].view(s)
        with torch.cuda.stream(copy):
            dv.copy_(sv, non_blocking=True)
            dl.copy_(sl, non_blocking=True)
            ready[k].record(copy)
        # this brick's seeds: flat indices of the fine grid and labels
        lf = sl.numpy().reshape(-1)
        loc = np.flatnonzero(lf)
        if loc.size:
            z, r = np.divmod(loc, s[1] * s[2])
            y, x = np.divmod(r, s[2])
            seed_idx.append(((z + o[0]) * shape[1] + (y + o[1])) * shape[2] + (x + o[2]))
            seed_lab.append(lf[loc])
        main.wait_event(ready[k])
        gb, lbd = rw.downsample(dv, dl, lo=lo, hi=hi, out_dtype=torch.float32, ctx=ctx)
        c = tuple(v // 2 for v in o)
        g1[c[0]:c[0] + gb.shape[0], c[1]:c[1] + gb.shape[1], c[2]:c[2] + gb.shape[2]] = gb
        l1[c[0]:c[0] + gb.shape[0], c[1]:c[1] + gb.shape[1], c[2]:c[2] + gb.shape[2]] = lbd
        done[k].record(main)
        info["h2d_bytes"] += sv.numel() * sv.element_size() + sl.numel()
    torch.cuda.synchronize()
    info["lod_s"] = time.perf_counter() - t0
    sidx = torch.from_numpy(np.concatenate(seed_idx).astype(np.int64) if seed_idx
                            else np.zeros(0, np.int64)).to(dev)
    slab = torch.from_numpy(np.concatenate(seed_lab) if seed_lab
                            else np.zeros(0, np.uint8)).to(dev)
    info["seeds"] = int(sidx.numel())
    del stage_v, stage_l, dbuf_v, dbuf_l
    g, lab = g1, l1
    for _ in range(levels - 1):
        g, lab = rw.downsample(g, lab, lo=0.0, hi=1.0, out_dtype=torch.float32, ctx=ctx)

    # ---- coarse solve and classification
    t0 = time.perf_counter()
    coarse, _, cst = rw.solve(g, lab, K, beta, tol=tol, precision=precision, lo=0.0, hi=1.0,
                              argmax=False, ctx=ctx, return_stats=True)
    f = 2 ** levels
    cands, active = rw.classify_bricks_sparse(coarse, sidx, slab, shape, f, brick, (0, 0, 0),
                                              lo_thr, hi_thr, ctx=ctx)
    torch.cuda.synchronize()
    info["coarse_s"] = time.perf_counter() - t0
    info["coarse_iters"] = cst["iters"]
    info["coarse"] = coarse
    del g1, l1, g, lab, sidx, slab
    act = [b for b, a in zip(cands, active) if a]
    ina = [b for b, a in zip(cands, active) if not a]
    info["bricks"] = len(cands)
    info["active_bricks"] = len(act)
    if out is None and labels_out is None:
        out = np.empty((K,) + shape, dtype=np.float32)
    want_p, want_l = out is not None, labels_out is not None
    worker = ThreadPoolExecutor(max_workers=1)

    def scatter(pin_p, pin_l, ev, items):
        """Copy a batch's results from its pinned buffers into the outputs
        once their D2H copy has completed (runs on the worker thread)."""
        ev.synchronize()
        hp = pin_p.numpy() if want_p else None
        hl = pin_l.numpy() if want_l else None
        nbytes = 0
        for off, dims, src, dst in items:
            n = int(np.prod(dims))
            if want_p:
                out[(slice(None),) + dst] = hp[:, off:off + n].reshape((K,) + dims)[
                    (slice(None),) + src]
                nbytes += K * n * 4
            if want_l:
                labels_out[dst] = hl[off:off + n].reshape(dims)[src]
                nbytes += n
        return nbytes

    def fetch(pv, pa, n_used, pin_p, pin_l):
        """Async D2H of a batch's outputs (the first n_used pool voxels) on
        the copy stream after the main stream's work; returns the event."""
        ev_main = torch.cuda.Event()
        ev_main.record(main)
        ev = torch.cuda.Event()
        with torch.cuda.stream(copy):
            copy.wait_event(ev_main)
            if want_p:
                pin_p[:, :n_used].copy_(pv[:, :n_used], non_blocking=True)
            if want_l:
                pin_l[:n_used].copy_(pa[:n_used], non_blocking=True)
            ev.record(copy)
        return ev

    # ---- certain bricks: labels streamed in, upsampled coarse probabilities out
    t0 = time.perf_counter()
    bvox = int(np.prod(brick))
    nfill = max(1, min(pool, len(ina)))
    fl = torch.zeros((1, 1, nfill * bvox), dtype=torch.uint8, device=dev)
    fl_pin = torch.zeros((nfill * bvox,), dtype=torch.uint8).pin_memory()
    fp = torch.empty((K, 1, 1, nfill * bvox), dtype=torch.float32, device=dev)
    fa = torch.empty((nfill * bvox,), dtype=torch.uint8, device=dev)
    fpin_p = torch.empty((K, nfill * bvox), dtype=torch.float32).pin_memory() if want_p else None
    fpin_l = torch.empty((nfill * bvox,), dtype=torch.uint8).pin_memory() if want_l else None
    for i0 in range(0, len(ina), nfill):
        chunk = ina[i0:i0 + nfill]
        subs, local, items = [], [], []
        for j, (o, s) in enumerate(chunk):
            n = int(np.prod(s))
            fl_pin[j * bvox:j * bvox + n].copy_(torch.from_numpy(
                np.ascontiguousarray(_box(lab_host, o, s)).reshape(-1)))
            subs.append((j * bvox, s, o))
            local.append(((0, 0, 0), s))
            full = (slice(None),) * 3
            items.append((j * bvox, tuple(s), full,
                          (slice(o[0], o[0] + s[0]), slice(o[1], o[1] + s[1]),
                           slice(o[2], o[2] + s[2]))))
        used = len(chunk) * bvox
        fl.view(-1)[:used].copy_(fl_pin[:used], non_blocking=True)
        info["h2d_bytes"] += used
        rw.fill_bricks(coarse, fl, f, local, fp, subvols=subs, ctx=ctx)
        fv = fp.view(K, -1)
        if want_l:
            rw.argmax(fv, out=fa, ctx=ctx)
        ev = fetch(fv, fa, used, fpin_p, fpin_l)
        info["d2h_bytes"] += scatter(fpin_p, fpin_l, ev, items)
    torch.cuda.synchronize()
    info["fill_s"] = time.perf_counter() - t0

    # ---- uncertain bricks through the pools
    t0 = time.perf_counter()
    hal = tuple(b + 2 for b in brick)
    slot = int(np.prod(hal))

    def make_pool():
        return dict(v=torch.empty((1, 1, pool * slot), dtype=tdt, device=dev),
                    l=torch.zeros((1, 1, pool * slot), dtype=torch.uint8, device=dev),
                    p=torch.empty((K, 1, 1, pool * slot), dtype=torch.float32, device=dev),
                    a=torch.empty((pool * slot,), dtype=torch.uint8, device=dev),
                    sv=torch.empty((pool * slot,), dtype=tdt).pin_memory(),
                    sl=torch.empty((pool * slot,), dtype=torch.uint8).pin_memory(),
                    op=(torch.empty((K, pool * slot), dtype=torch.float32).pin_memory()
                        if want_p else None),
                    ol=torch.empty((pool * slot,), dtype=torch.uint8).pin_memory() if want_l
                    else None,
                    ev=torch.cuda.Event(), done=torch.cuda.Event(), fetched=None, scat=None)

    pools = [make_pool() for _ in range(2 if len(act) > pool else 1)]
    batches = [act[i:i + pool] for i in range(0, len(act), pool)]

    def stage(bi):
        """Fill pool bi % 2's pinned staging from the host volume and queue
        its H2D copies (runs on the worker thread while the main thread
        solves the previous batch)."""
        P = pools[bi % len(pools)]
        P["done"].synchronize()  # the pool's previous batch has been solved
        if P["scat"] is not None:
            P["scat"].result()  # and its results scattered (its pinned output reused later)
        subs, bricks_local, items = [], [], []
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
            ob = tuple(o[a] - lo_[a] for a in range(3))
            subs.append((off, dims, tuple(lo_)))
            bricks_local.append((ob, s))
            items.append((off, dims,
                          (slice(ob[0], ob[0] + s[0]), slice(ob[1], ob[1] + s[1]),
                           slice(ob[2], ob[2] + s[2])),
                          (slice(o[0], o[0] + s[0]), slice(o[1], o[1] + s[1]),
                           slice(o[2], o[2] + s[2]))))
            off += n
        with torch.cuda.stream(copy):
            P["v"].view(-1)[:off].copy_(P["sv"][:off], non_blocking=True)
            P["l"].view(-1)[:off].copy_(P["sl"][:off], non_blocking=True)
            P["ev"].record(copy)
        return subs, bricks_local, items, off, off * (P["sv"].element_size() + 1)

    pending = worker.submit(stage, 0) if batches else None
    solve_s = 0.0
    iters_all = []
    meta = []
    scatters = []
    for bi in range(len(batches)):
        P = pools[bi % len(pools)]
        subs, bricks_local, items, used, h2d = pending.result()
        info["h2d_bytes"] += h2d
        if bi + 1 < len(batches):
            # staged on the worker while this thread solves batch bi; the
            # worker runs tasks in order, so batch bi-1's results (same pool)
            # are scattered before its staging is overwritten
            pending = worker.submit(stage, bi + 1)
        main.wait_event(P["ev"])
        ts = time.perf_counter()
        _, iters, bst = rw.solve_bricks(P["v"], P["l"], K, beta, coarse, f, bricks_local,
                                        prob_out=P["p"], tol=tol, precision=precision, lo=lo,
                                        hi=hi, ctx=ctx, return_stats=True, subvols=subs,
                                        update_delta=update_delta,
                                        brick_voxels=int(brick[0]) * brick[1] * brick[2])
        solve_s += time.perf_counter() - ts
        iters_all += iters
        meta.append(bst)
        pv = P["p"].view(K, -1)
        if want_l:
            rw.argmax(pv, out=P["a"], ctx=ctx)
        ev = fetch(pv, P["a"], used, P["op"], P["ol"])
        P["done"].record(main)
        # results of this batch: scattered on the worker thread; the next
        # batch is staged there too, both while this thread solves
        P["scat"] = worker.submit(scatter, P["op"], P["ol"], ev, items)
        scatters.append(P["scat"])
    for sc in scatters:
        info["d2h_bytes"] += sc.result()
    worker.shutdown()
    torch.cuda.synchronize()
    info["bricks_s"] = time.perf_counter() - t0
    info["brick_solve_s"] = solve_s
    info["brick_iters"] = iters_all
    info["brick_stats"] = meta
    info["total_s"] = time.perf_counter() - t_all
    return (out if out is not None else labels_out), info
