import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU check")


def read_golden(name):
    """Rows of integers/floats from a golden fixture; '#' starts a comment."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(t) if ("." in t or "e" in t) else int(t) for t in line.split()])
    return rows


def gpu_binding():
    """The HIP binding, or skip when this machine has no GPU.  A missing
    library is an error, never a skip."""
    import pytest
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU on this machine")
    from paper_1302_4018_amd import binding
    return binding


def to_dev(a):
    import torch
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()


import numpy as np  # noqa: E402  (used by to_dev)


def gradient_entry_bounds(g_mass_ref, g_coup_ref, tol, V, lam_lb, scale_slack=1e-13):
    """Per-entry bounds on |g_gpu - g_oracle| for dT/dm and dT/dw when both
    sides solve every right-hand side to a true relative residual <= tol.

    Each solution carries an error d = A^-1 r with ||d|| <= tol ||b|| / lambda_min
    = eps (||b||^2 = V for the unit-modulus diluted probes), so two solutions of
    one system differ by delta <= 2 eps.  An entry is -(1/s) sum_j f_j with
    f_j = ||x_j(y)||^2 (mass) or ||x_j(y) - U x_j(y+mu)||^2 (coupling), and
    |f_j(x + delta) - f_j(x)| <= delta_j (2 a_j + delta_j) with a_j the
    oracle's norm at the entry (delta_j <= 2 eps for a site, 4 eps for an
    edge).  Cauchy-Schwarz over j with sum_j a_j^2 = s |g(y)| gives
        |dg(y)| <= 2 D sqrt(|g(y)|) + D^2,   D = 2 eps (mass) or 4 eps (coupling),
    plus a rounding slack relative to the largest entry."""
    eps = tol * np.sqrt(V) / lam_lb
    bm = 2 * (2 * eps) * np.sqrt(np.abs(g_mass_ref)) + (2 * eps) ** 2
    bw = 2 * (4 * eps) * np.sqrt(np.abs(g_coup_ref)) + (4 * eps) ** 2
    bm = bm + scale_slack * np.abs(g_mass_ref).max()
    bw = bw + scale_slack * np.abs(g_coup_ref).max()
    return bm, bw


def assert_gradient_entries(gm, gw, gm_ref, gw_ref, tol, V, lam_lb):
    """Every entry of the mass and coupling gradients within its bound."""
    bm, bw = gradient_entry_bounds(gm_ref, gw_ref, tol, V, lam_lb)
    dm = np.abs(gm - gm_ref)
    dw = np.abs(gw - gw_ref)
    im, iw = int(np.argmax(dm - bm)), int(np.argmax((dw - bw).ravel()))
    assert np.all(dm <= bm), f"mass gradient entry {im}: |diff| {dm[im]:.3e} > bound {bm[im]:.3e}"
    assert np.all(dw <= bw), (f"coupling gradient entry {np.unravel_index(iw, dw.shape)}: |diff| "
                              f"{dw.ravel()[iw]:.3e} > bound {bw.ravel()[iw]:.3e}")


def read_quadratures(name):
    """Stored oracle quadratures (tests/golden/make_quadratures.py): label ->
    complex array indexed by probe m."""
    rows = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            label, m, re, im = line.split()
            rows.setdefault(label, {})[int(m)] = complex(float(re), float(im))
    return {k: np.array([v[m] for m in range(len(v))]) for k, v in rows.items()}
