"""Shared checks of GPU results against the CPU oracle (test helpers only).

Not a test module (pytest collects test_*.py): the GPU test files import these
so that every comparison with the oracle uses the same definitions of error,
sampling and probing.
"""

from __future__ import annotations

import numpy as np

import oracle as O
from hs_inputs import cn

# Bounds stated for the two arithmetic forms: complex FP64 (4-product and 3M)
# and the split-precision forms.
TOL_FP64 = 1e-12
TOL_SPLIT = 1e-9
MODE_TOL = {0: TOL_FP64, 1: TOL_SPLIT, 2: TOL_SPLIT, 3: TOL_FP64, 4: TOL_SPLIT, 5: TOL_SPLIT}
MODE_NAME = {0: "fp64", 1: "split_f16", 2: "split_i8", 3: "fp64_3m", 4: "split_bf16",
             5: "split_i8_crt"}


def rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def expected_info(p):
    info = np.zeros(p.N_A, np.int32)
    for a in p.failing:
        info[a] = 1
    for a, piv in p.planted.items():
        info[a] = piv
    return info


def sample_columns(n_g, seed=1, n_random=6):
    """Both ends, a tile edge, the middle and seeded random columns."""
    rng = np.random.default_rng(seed)
    fixed = [0, 1, 127, 128, n_g // 2, n_g - 1]
    return sorted({c for c in fixed + rng.integers(0, n_g, n_random).tolist() if 0 <= c < n_g})


def check_full(p, H, S, info, tol):
    """Every element: relative Frobenius error of H and of S, exact
    Hermiticity with a real diagonal, exact Cholesky flags."""
    Hr = O.hamiltonian(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.nl)
    Sr = O.overlap(p.A, p.B, p.U, p.nl)
    eh, es = rel(H, Hr), rel(S, Sr)
    print(f"  rel err H {eh:.2e} S {es:.2e}", flush=True)
    assert eh <= tol and es <= tol, (eh, es)
    assert np.array_equal(H, H.conj().T) and np.array_equal(S, S.conj().T)
    assert np.all(H.diagonal().imag == 0) and np.all(S.diagonal().imag == 0)
    assert np.array_equal(info, expected_info(p))
    return eh, es


def check_columns_and_probes(A, B, T_AA, T_AB, T_BB, U, nl, Hd, Sd, cols, tol, n_probe=2,
                             probe_seed=0):
    """Host copies Hd, Sd of a large result: each sampled column within `tol`
    (relative) of the oracle's column, exact Hermiticity, and bilinear probes
    y^H H x, y^H S x within tol * ||.||_F ||x|| ||y|| of the oracle's
    per-atom evaluation (which never forms H or S)."""
    n_g = Hd.shape[0]
    Hr = O.hamiltonian_columns(A, B, T_AA, T_AB, T_BB, nl, cols)
    Sr = O.overlap_columns(A, B, U, nl, cols)
    worst = 0.0
    for j, g in enumerate(cols):
        eh = np.linalg.norm(Hd[:, g] - Hr[:, j]) / np.linalg.norm(Hr[:, j])
        es = np.linalg.norm(Sd[:, g] - Sr[:, j]) / np.linalg.norm(Sr[:, j])
        assert eh <= tol and es <= tol, (g, eh, es)
        worst = max(worst, eh, es)
    assert np.array_equal(Hd, Hd.conj().T) and np.array_equal(Sd, Sd.conj().T)
    fro_h, fro_s = np.linalg.norm(Hd), np.linalg.norm(Sd)
    rng = np.random.default_rng(probe_seed)
    for _ in range(n_probe):
        x, y = cn(rng, (n_g,)), cn(rng, (n_g,))
        h, s = O.bilinear(A, B, T_AA, T_AB, T_BB, U, nl, x, y)
        nx, ny = np.linalg.norm(x), np.linalg.norm(y)
        assert abs(y.conj() @ (Hd @ x) - h) <= tol * fro_h * nx * ny
        assert abs(y.conj() @ (Sd @ x) - s) <= tol * fro_s * nx * ny
    print(f"  sampled columns {len(cols)}: worst rel err {worst:.2e}", flush=True)
    return worst


def check_sampled(p, run, cols, tol, n_probe=2):
    """check_columns_and_probes on a DeviceBuild's outputs, plus exact flags."""
    Hd = run.H.cpu().numpy()
    Sd = run.S.cpu().numpy()
    worst = check_columns_and_probes(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.U, p.nl, Hd, Sd, cols,
                                     tol, n_probe)
    assert np.array_equal(run.info.cpu().numpy(), expected_info(p))
    return worst
