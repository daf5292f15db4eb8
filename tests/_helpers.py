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
