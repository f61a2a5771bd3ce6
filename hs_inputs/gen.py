"""Seeded generators for the synthetic H/S workloads.

The paper's own inputs (the NaCl and AuAg FLEUR systems, Sec. 4 and Tab. 1)
are not available, so every workload here is synthetic with the shapes the
paper gives (Sec. 2: N_A ~ 100, N_G ~ 10^3..10^4, N_L ~ 100).

Distributions (one independent child stream per array, so an array does not
depend on the order in which the others are drawn):
  * CN(0,1) = (x + i y)/sqrt(2), x, y iid N(0,1), so E|z|^2 = 1
  * A_a, B_a       CN(0,1)/sqrt(N_G)
  * T_AA,a         herm(M M^H / N_L + I), M ~ CN(0,1)^{N_L x N_L}
  * T_AB,a         CN(0,1)/N_L
  * T_BB,a         (X + X^H) / (2 N_L),   X ~ CN(0,1)^{N_L x N_L}
  * U_a            real uniform [0.5, 2] stored as complex; with complex_u,
                   the same moduli times e^{i phi}, phi uniform in [0, 2 pi)
                   (its own child stream), so |u|^2 differs from Re(u)^2
  * failing atoms  T_AA,a <- T_AA,a - 2 lambda_max(T_AA,a) I (fails at pivot 1)
where herm(T) = (T + T^H)/2, which is exactly Hermitian in IEEE arithmetic
(the diagonal's imaginary part is exactly zero and mirrored entries are exact
conjugates), so a reader that uses only the lower triangle and one that uses
the whole matrix see the same operator.

No arithmetic of the H/S build lives here.
"""

from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence

import numpy as np

# Named child streams, in a fixed order.
_STREAMS = ("A", "B", "T_AA", "T_AB", "T_BB", "U", "fail", "plant", "U_phase")


def cn(rng: np.random.Generator, shape) -> np.ndarray:
    """Complex standard normal CN(0,1): (x + i y)/sqrt(2)."""
    z = rng.standard_normal(tuple(shape) + (2,))
    z *= np.sqrt(0.5)
    return z.view(np.complex128).reshape(shape)


def _herm(t: np.ndarray) -> np.ndarray:
    return (t + t.conj().T) * 0.5


@dataclasses.dataclass
class Problem:
    """One k-point's inputs in the ABI layout (see the package docstring)."""

    A: np.ndarray
    B: np.ndarray
    T_AA: np.ndarray
    T_AB: np.ndarray
    T_BB: np.ndarray
    U: np.ndarray
    nl: np.ndarray
    N_G: int
    seed: int
    failing: List[int]
    planted: Dict[int, int]
    name: str = "custom"

    @property
    def N_A(self) -> int:
        return int(self.nl.shape[0])

    @property
    def K(self) -> int:
        return int(self.nl.sum())

    @property
    def uniform_nl(self) -> Optional[int]:
        return int(self.nl[0]) if np.all(self.nl == self.nl[0]) else None

    def row_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.nl)]).astype(np.int64)

    def t_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.nl.astype(np.int64) ** 2)])

    def t_block(self, which: str, a: int) -> np.ndarray:
        t = getattr(self, which)
        off = self.t_offsets()
        n = int(self.nl[a])
        return t[off[a]:off[a + 1]].reshape(n, n)

    def set_t_block(self, which: str, a: int, value: np.ndarray) -> None:
        t = getattr(self, which)
        off = self.t_offsets()
        t[off[a]:off[a + 1]] = np.asarray(value, dtype=np.complex128).reshape(-1)

    def copy(self) -> "Problem":
        return dataclasses.replace(
            self,
            A=self.A.copy(), B=self.B.copy(), T_AA=self.T_AA.copy(),
            T_AB=self.T_AB.copy(), T_BB=self.T_BB.copy(), U=self.U.copy(),
            nl=self.nl.copy(), failing=list(self.failing), planted=dict(self.planted),
        )


def _hpd_block(rng: np.random.Generator, n: int) -> np.ndarray:
    m = cn(rng, (n, n))
    return _herm(m @ m.conj().T / n + np.eye(n))


def _planted_block(rng: np.random.Generator, n: int, pivot: int) -> np.ndarray:
    """Hermitian block whose Cholesky fails first at 1-based pivot `pivot`.

    Built as T = C C^H from a lower-triangular C with a positive diagonal, so
    the exact pivots are C_jj^2; the diagonal entry at `pivot` is then lowered
    by 1.5 C_pp^2, which leaves the leading minors before it positive definite
    and makes that pivot -0.5 C_pp^2 (a clear margin).
    """
    c = np.tril(cn(rng, (n, n)) / np.sqrt(n), -1)
    c[np.diag_indices(n)] = 1.0 + np.abs(rng.standard_normal(n))
    t = _herm(c @ c.conj().T)
    p = pivot - 1
    t[p, p] = t[p, p].real - 1.5 * c[p, p].real ** 2
    return t


def make_problem(
    N_A: int,
    N_L,
    N_G: int,
    seed: int = 0,
    n_fail: int = 0,
    fail_atoms: Optional[Sequence[int]] = None,
    planted: Optional[Dict[int, int]] = None,
    name: str = "custom",
    complex_u: bool = False,
) -> Problem:
    """Draw one problem.

    N_L is an int (all atoms alike) or a sequence of N_A ints (mixed types).
    n_fail atoms (seeded choice without replacement), or the explicit
    fail_atoms, get the -2 lambda_max shift. `planted` maps atom -> 1-based
    pivot at which that atom's T_AA is built to fail. complex_u gives every
    U entry a seeded phase (the moduli are the same draws as without it).
    """
    if np.isscalar(N_L):
        nl = np.full(N_A, int(N_L), dtype=np.int32)
    else:
        nl = np.asarray(N_L, dtype=np.int32)
        assert nl.shape == (N_A,)
    K = int(nl.sum())
    kids = dict(zip(_STREAMS, np.random.SeedSequence(seed).spawn(len(_STREAMS))))
    rng = {k: np.random.Generator(np.random.PCG64(v)) for k, v in kids.items()}

    scale = 1.0 / np.sqrt(N_G)
    A = cn(rng["A"], (K, N_G))
    A *= scale
    B = cn(rng["B"], (K, N_G))
    B *= scale

    t_aa, t_ab, t_bb = [], [], []
    for n in nl:
        n = int(n)
        t_aa.append(_hpd_block(rng["T_AA"], n).reshape(-1))
        t_ab.append((cn(rng["T_AB"], (n, n)) / n).reshape(-1))
        x = cn(rng["T_BB"], (n, n))
        t_bb.append(((x + x.conj().T) / (2 * n)).reshape(-1))
    U = rng["U"].uniform(0.5, 2.0, size=K).astype(np.complex128)
    if complex_u:
        U *= np.exp(1j * rng["U_phase"].uniform(0.0, 2.0 * np.pi, size=K))

    prob = Problem(
        A=A, B=B,
        T_AA=np.concatenate(t_aa), T_AB=np.concatenate(t_ab), T_BB=np.concatenate(t_bb),
        U=U, nl=nl, N_G=int(N_G), seed=int(seed), failing=[], planted={}, name=name,
    )

    if fail_atoms is None and n_fail > 0:
        fail_atoms = sorted(int(a) for a in rng["fail"].choice(N_A, size=n_fail, replace=False))
    for a in fail_atoms or []:
        t = prob.t_block("T_AA", a)
        lam = float(np.linalg.eigvalsh(t).max())
        t = t.copy()
        t[np.diag_indices(t.shape[0])] -= 2.0 * lam
        prob.set_t_block("T_AA", a, t)
        prob.failing.append(int(a))
    for a, piv in sorted((planted or {}).items()):
        prob.set_t_block("T_AA", a, _planted_block(rng["plant"], int(nl[a]), int(piv)))
        prob.planted[int(a)] = int(piv)
    return prob


# The five workloads. Sizes follow the paper's typical ranges (Sec. 2, Tab. 1).
CONFIGS = {
    # tiny plain case, small enough for the entrywise oracle
    "plain_tiny": dict(N_A=4, N_L=16, N_G=256, n_fail=0),
    # plain case with three atoms taking the Cholesky-failure branch
    "plain_gpu": dict(N_A=32, N_L=49, N_G=2000, n_fail=3),
    # large case (N_G = 8000) used for the FP64 / split-precision comparison
    "precision": dict(N_A=100, N_L=81, N_G=8000, n_fail=0),
    # four atom types of different l_max, 5% of atoms failing (round(6.4) = 6)
    "batching": dict(N_A=128, N_L=[16] * 32 + [49] * 32 + [81] * 32 + [121] * 32,
                     N_G=6000, n_fail=6),
    # the paper's two test systems at K_max = 4.0 (Tab. 1), synthetic values of
    # the same shapes: NaCl (512 atoms, l_max 6) and AuAg (108 atoms, l_max 10)
    "nacl_kmax4": dict(N_A=512, N_L=49, N_G=9273, n_fail=0),
    "auag_kmax4": dict(N_A=108, N_L=121, N_G=13379, n_fail=0),
}

# Serving workload: one resident atom set, a stream of k-point requests.
SERVING = dict(N_A=64, N_L=64, n_requests=64, ng_lo=1500, ng_hi=9000)


def make_config(name: str, seed: int = 0) -> Problem:
    cfg = dict(CONFIGS[name])
    return make_problem(name=name, seed=seed, **cfg)


def serving_requests(seed: int = 0, n_requests: int = SERVING["n_requests"],
                     ng_lo: int = SERVING["ng_lo"], ng_hi: int = SERVING["ng_hi"]):
    """Sizes of the serving stream: N_G of each request, integer-uniform inclusive."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0xC5])))
    return rng.integers(ng_lo, ng_hi + 1, size=n_requests)


def serving_arrivals(seed: int, n: int, rate: float) -> np.ndarray:
    """Poisson arrival times (seconds from 0) at `rate` requests per second."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0xA7])))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def serving_atoms(seed: int = 0) -> Problem:
    """The resident atom data (T, U) of the serving workload, with a 1-column A/B stub."""
    return make_problem(SERVING["N_A"], SERVING["N_L"], 1, seed=seed, name="serving_atoms")


def serving_request_ab(seed: int, r: int, n_g: int, K: int):
    """Fresh A, B of request r (CN(0,1)/sqrt(N_G))."""
    ss = np.random.SeedSequence([seed, 0x5E, r]).spawn(2)
    ra, rb = (np.random.Generator(np.random.PCG64(s)) for s in ss)
    A = cn(ra, (K, n_g))
    A *= 1.0 / np.sqrt(n_g)
    B = cn(rb, (K, n_g))
    B *= 1.0 / np.sqrt(n_g)
    return A, B
