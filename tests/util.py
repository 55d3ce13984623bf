"""Helpers shared by the GPU tests: device copies of workload fields and tolerance checks."""
import numpy as np


def to_device(f, theta_row=0):
    import torch
    dev = torch.device("cuda:0")
    locs = torch.from_numpy(np.ascontiguousarray(f.locs)).to(dev)
    z = torch.from_numpy(np.ascontiguousarray(f.z)).to(dev)
    nbr = torch.from_numpy(np.ascontiguousarray(f.nbr)).to(dev) if f.m > 0 else None
    theta = torch.from_numpy(np.ascontiguousarray(f.thetas[theta_row])).to(dev)
    return locs, z, nbr, theta


def assert_total_close(got, ref, rel, what=""):
    err = abs(got - ref)
    assert err <= rel * abs(ref), f"{what}: got {got!r} ref {ref!r} rel err {err / abs(ref):.3e} > {rel:.0e}"


def assert_grad_close(got, ref, gterms_abs_sum, rel, what=""):
    """Per component: |got - ref| <= rel * max(|ref|, 1e-3 * sum_i |g_i|).

    The floor covers components that cancel to near zero.  With rel = 1e-9 it
    is an absolute bound of 1e-12 * sum_i |g_i|: the per-term gradients must
    agree to about 1e-12 of their magnitude on average, the agreement of two
    FP64 evaluations of well-conditioned terms; summing n terms in another
    order moves the total by about n * eps * sum_i |g_i|, far below that."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.maximum(np.abs(ref), 1e-3 * np.asarray(gterms_abs_sum))
    err = np.abs(got - ref)
    assert np.all(err <= rel * scale), f"{what}: got {got} ref {ref} err/scale {err / scale}"
