"""Shared test helpers: device transfer and the parity bar."""
import numpy as np


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def top_two_gap(prob):
    s = np.sort(prob, axis=0)
    return s[-1] - s[-2]


def assert_parity(prob_gpu, prob_ref, atol=1e-5, gap=1e-4, what=""):
    """Max-abs probability error <= atol and identical argmax labels wherever
    the reference's top-two gap is >= gap (ties excluded)."""
    prob_gpu = np.asarray(prob_gpu, dtype=np.float64)
    prob_ref = np.asarray(prob_ref, dtype=np.float64)
    err = np.max(np.abs(prob_gpu - prob_ref))
    assert err <= atol, f"{what}: max-abs error {err:.3e} > {atol:.1e}"
    clear = top_two_gap(prob_ref) >= gap
    am_g = np.argmax(prob_gpu, axis=0)
    am_r = np.argmax(prob_ref, axis=0)
    bad = np.count_nonzero((am_g != am_r) & clear)
    assert bad == 0, f"{what}: {bad} argmax mismatches away from ties"
    return err, int(np.count_nonzero(~clear))



def near_threshold(coarse, labels, f, origin, size, lo_thr=0.02, hi_thr=0.98, eps=1e-4):
    """Whether a brick's activity decision is within eps of flipping (the
    only bricks two correct implementations may classify differently).  The
    decision is "some upsampled probability of the brick or its face shell
    lies strictly inside (lo_thr, hi_thr), or a seed of the brick is not the
    upsampled argmax"; it is marginal unless moving every probability by eps
    cannot change it.  coarse: the reference's coarse probabilities."""
    from oracle import rw_oracle as O
    o = np.array(origin)
    s = np.array(size)
    shape = labels.shape
    P = np.stack([O.upsample_trilinear(coarse[k], shape, f, (tuple(o - 1), tuple(s + 2)))
                  for k in range(coarse.shape[0])])
    inner = P[:, 1:-1, 1:-1, 1:-1]
    zz, yy, xx = O._shell_mask(shape, origin, size)
    vals = np.concatenate([inner.reshape(-1), P[:, zz - o[0] + 1, yy - o[1] + 1,
                                                xx - o[2] + 1].reshape(-1)])
    depth = np.max(np.minimum(vals - lo_thr, hi_thr - vals))   # > 0: some value inside
    lab = labels[o[0]:o[0] + s[0], o[1]:o[1] + s[1], o[2]:o[2] + s[2]]
    seeded = lab > 0
    if seeded.any():
        ps = inner[:, seeded]
        own = ps[lab[seeded] - 1, np.arange(ps.shape[1])]
        others = ps.copy()
        others[lab[seeded] - 1, np.arange(ps.shape[1])] = -np.inf
        wrong = np.max(np.max(others, axis=0) - own)           # > 0: some seed not the argmax
    else:
        wrong = -np.inf
    if depth > eps or wrong > eps:
        return False                                           # robustly active
    return depth >= -eps or wrong >= -eps                      # else robustly inactive


def c_brick_solver(g, labels, beta, tol, labels_solved):
    """Brick solves for the oracle's hierarchical pipeline by the C oracle
    (single-threaded: the bricks are small): (origin, size, P_frame) ->
    (x [len(labels_solved)][brick], info), shell values and x0 from the
    upsampled frame P_frame [K][frame]."""
    from oracle import c_oracle

    def solve(origin, size, P_frame):
        xs, info = [], []
        for s in labels_solved:
            x, it, st, _ = c_oracle.solve_box(g, labels, s, beta, tol=tol,
                                              box=(tuple(origin), tuple(size)),
                                              shell=P_frame[s - 1],
                                              x0=P_frame[s - 1][1:-1, 1:-1, 1:-1], nthreads=1)
            assert st >= 0, st
            xs.append(x)
            info.append(dict(label=s, iters=it, status=st))
        return np.stack(xs), info
    return solve


def progress(request, msg):
    """A progress line on the real terminal, past pytest's output capture
    (long oracle computations otherwise run silent for minutes)."""
    import sys
    capman = request.config.pluginmanager.getplugin("capturemanager")
    if capman is None:
        print(msg, flush=True)
        return
    with capman.global_and_fixture_disabled():
        sys.stdout.write(msg + "\n")
        sys.stdout.flush()
