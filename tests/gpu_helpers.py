"""Shared helpers of the GPU parity tests: device copies of synthetic problems and the error
measures the tolerances are stated in."""
import numpy as np
import torch


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def problem_tensors(p, idx=None):
    """Device tensors (float32) of a synthetic problem, restricted to views idx."""
    angles, w = (p.angles, p.w) if idx is None else p.views(idx)
    return dict(coef=dev(p.coef), mu=dev(p.mu), scale=dev(p.scale), quat=dev(p.quat),
                rho=dev(p.rho), angles=dev(angles), w=dev(w))


def oracle_inputs(p, idx=None):
    angles, w = (p.angles, p.w) if idx is None else p.views(idx)
    return (p.coef, p.mu, p.scale, p.quat, p.rho, angles, w)


def max_rel_to_max(got, ref):
    """max |got - ref| / max |ref| (the per-pixel measure, relative to the image's maximum)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def norm_rel(got, ref):
    """||got - ref|| / ||ref|| (norm-wise relative error)."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def elem_rel(got, ref):
    """max |got - ref| / max |ref| over the elements of one parameter group."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)) if ref.size else 0.0


GRAD_NORM_BAR = 1e-4   # ||got - ref|| / ||ref|| per parameter group
GRAD_ELEM_BAR = 1e-3   # max |got - ref| / max |ref| per parameter group


def _host(x):
    return x.double().cpu().numpy() if isinstance(x, torch.Tensor) else np.asarray(x, np.float64)


def check_grads(got: dict, ref: dict, norm_bar=GRAD_NORM_BAR, elem_bar=GRAD_ELEM_BAR):
    """Gradients against a reference, every group (dL/dw included) both norm-wise and
    element-wise; prints the measured figures and returns them."""
    errs = {}
    for k in ref:
        g, r = _host(got[k]), _host(ref[k])
        assert g.shape == r.shape, (k, g.shape, r.shape)
        errs[k] = (norm_rel(g, r), elem_rel(g, r))
    print({k: "norm %.2e elem %.2e" % e for k, e in errs.items()}, flush=True)
    for k, (nr, er) in errs.items():
        assert nr <= norm_bar, (k, "norm-wise", nr)
        assert er <= elem_bar, (k, "element-wise", er)
    return errs
