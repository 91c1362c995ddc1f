"""Shared test helpers: case construction and error metrics (no method arithmetic)."""
import numpy as np

from paper_2604_22718_amd import workloads as wl


def split_cores(flat, bond):
    out, off = [], 0
    for k in range(len(bond) - 1):
        a, b = int(bond[k]), int(bond[k + 1])
        out.append(flat[off:off + 2 * a * b].reshape(2, a, b).copy())
        off += 2 * a * b
    return out


def device_cores(psi, bond, n_terms=1):
    """The quantised cores exactly as the library uses them."""
    if n_terms == 1:
        return split_cores(psi.core_values(bond, 0), bond)
    return [split_cores(psi.core_values(bond, t), bond) for t in range(n_terms)]


def check_ratios(lr_gpu, sg_gpu, r_ref, kappa, tol, k0=10.0):
    """Per-ratio bound |Delta log|r_j|| <= tol * max(1, kappa_j / k0).

    kappa_j = max(kappa(s), kappa(s^j)) is the oracle's cancellation measure
    (condition_numbers); a floating-point evaluation of psi has relative
    error ~ gamma * kappa, so the tolerance holds as stated for
    well-conditioned ratios (kappa <= k0) and grows linearly beyond.  Signs
    must agree wherever the allowed error is below 1/2.  Returns a summary."""
    r_ref = np.asarray(r_ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        dlog = np.abs(np.asarray(lr_gpu) - np.log(np.abs(r_ref)))
    allow = tol * np.maximum(1.0, np.asarray(kappa) / k0)
    nz = r_ref != 0
    bad = nz & ~(dlog <= allow)
    sign_bad = nz & (allow < 0.5) & (np.sign(r_ref) != np.asarray(sg_gpu))
    well = nz & (np.asarray(kappa) <= k0)
    return {
        "n": int(nz.sum()), "n_well": int(well.sum()),
        "max_well": float(dlog[well].max()) if well.any() else 0.0,
        "max_all": float(dlog[nz].max()), "p999_all": float(np.quantile(dlog[nz], 0.999)),
        "median": float(np.median(dlog[nz])),
        "n_bad": int(bad.sum()), "n_sign_bad": int(sign_bad.sum()),
        "worst_ratio_to_allow": float((dlog[nz] / allow[nz]).max()),
    }


def ratio_errors(lr_gpu, sg_gpu, r_ref):
    """Errors of GPU log-ratios against reference ratios r_ref (W, N).

    rel: |Delta log|r_j|| (the relative error of r_j) where |r_j| is at least
    1e-3 of the walker's median |r|; tiny ratios are compared in absolute
    terms relative to that median instead (they carry no weight in E_loc)."""
    r_ref = np.asarray(r_ref)
    a = np.abs(r_ref)
    med = np.median(a, axis=1, keepdims=True)
    big = a >= 1e-3 * med
    with np.errstate(divide="ignore", invalid="ignore"):
        dlog = np.abs(lr_gpu - np.log(a))
    r_gpu = sg_gpu * np.exp(lr_gpu)
    absrel = np.abs(r_gpu - r_ref) / med
    sign_ok = np.all((np.sign(r_ref) == sg_gpu) | ~big)
    return dlog[big], absrel[~big], sign_ok


def case(N, R, chi, path="perm", seed=0, bond=None):
    if path == "repeat":
        pi = wl.path_repeat(N, R)
    elif path == "perm":
        pi = wl.path_site_plus_perms(N, R, seed + 5)
    else:
        pi = np.asarray(path, dtype=np.int32)
    L = len(pi)
    if bond is None:
        bond = wl.open_bonds(L, chi)
    cores = wl.gaussian_cores(bond, seed + 11)
    return pi, np.asarray(bond), cores
