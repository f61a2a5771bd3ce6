"""Flop accounting for one H/S build.

Two counts are kept apart:

* `paper_step_flops` - the per-step counts printed beside the steps of
  Alg. 1 (complex double, 8 real flops per complex multiply-add), keyed by
  step: zgemm/zhemm of the first loop 8 N_L^2 N_G each, zher2k
  8 N_A N_L N_G^2, each zherk of S 4 N_A N_L N_G^2, the U scaling
  2 N_A N_L N_G, zpotrf 4/3 N_L^3, ztrmm 4 N_L^2 N_G, zhemm 8 N_L^2 N_G, the
  failure-branch zgemm 8 N_notHPD N_L N_G^2 and the HPD zherk
  4 N_HPD N_L N_G^2.
* `algorithmic_flops` - what the build must compute, used for the reported
  TFLOP/s: the same counts, except that the failure branch's product
  A_notHPD^H X_notHPD is counted as a Hermitian (triangular) contribution,
  4 N_L N_G^2 per failing atom, like the HPD zherk. With K = sum_a N_L(a) the
  large reductions then total 20 K N_G^2.
"""

from __future__ import annotations

import numpy as np


def paper_step_flops(nl, n_g, info):
    """Dict of Alg. 1 step -> flops, from the per-step formulas of Alg. 1."""
    nl = np.asarray(nl, dtype=np.float64)
    ok = np.asarray(info) == 0
    n_g = float(n_g)
    K = nl.sum()
    K_hpd = nl[ok].sum()
    K_fail = nl[~ok].sum()
    return {
        "loop1_zgemm_TBA_A": float(8 * (nl ** 2).sum() * n_g),
        "loop1_zhemm_TBB_B": float(8 * (nl ** 2).sum() * n_g),
        "H_zher2k_Z_B": float(8 * K * n_g ** 2),
        "S_zherk_A": float(4 * K * n_g ** 2),
        "S_scale_B_by_U": float(2 * K * n_g),
        "S_zherk_UB": float(4 * K * n_g ** 2),
        "loop2_zpotrf": float(4.0 / 3.0 * (nl ** 3).sum()),
        "loop2_ztrmm_Y": float(4 * (nl[ok] ** 2).sum() * n_g),
        "loop2_zhemm_X": float(8 * (nl[~ok] ** 2).sum() * n_g),
        "H_zgemm_A_X": float(8 * K_fail * n_g ** 2),
        "H_zherk_Y": float(4 * K_hpd * n_g ** 2),
    }


def algorithmic_flops(nl, n_g, info):
    """F_alg of one build (see module docstring)."""
    f = paper_step_flops(nl, n_g, info)
    nl = np.asarray(nl, dtype=np.float64)
    ok = np.asarray(info) == 0
    f["H_zgemm_A_X"] = float(4 * nl[~ok].sum() * float(n_g) ** 2)
    return float(sum(f.values()))


def reduction_flops(nl, n_g):
    """Flops of the two large lower-triangle reductions alone: 20 K N_G^2."""
    return 20.0 * float(np.sum(nl)) * float(n_g) ** 2
