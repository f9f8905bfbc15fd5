"""Synthetic workloads shared by the tests, the smoke check and the benchmark.

This module holds inputs only -- physical parameters, sizes, seeds and the
synthetic PDF table -- and none of the integrand's arithmetic.  Both the CPU
oracle and the GPU library receive the very same arrays from here.

The paper (Sec. 3) runs LO hadronic processes at sqrt(s) = 13 TeV with a real
PDF set that it does not name; the PDF table below is a smooth synthetic
stand-in with the shape of a gluon density, tabulated on a grid of the kind
PDFFlow interpolates (log-spaced in x and Q^2).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

SQRT_S = 13000.0          # GeV, hadronic centre-of-mass energy (Sec. 3)
M_TOP = 173.0             # GeV
W_TOP = 1.5               # GeV
ALPHA_S = 0.118           # fixed
MU_F = 173.0              # GeV, factorisation scale, held fixed
N_BINS = 50               # VEGAS bins per dimension
ALPHA_DAMP = 1.5          # VEGAS damping exponent

PROCESS_NG = {"gg_ttx": 2, "gg_ttxg": 3, "gg_ttxgg": 4, "gg_ttxggg": 5, "pp_ttx": 2}


@dataclass(frozen=True)
class PdfTable:
    log_x: np.ndarray      # [n_x] ascending ln x
    log_q2: np.ndarray     # [n_q2] ascending ln Q^2
    xf: np.ndarray         # [n_q2, n_x] x g(x, Q^2), C-contiguous float64
    xq: np.ndarray | None = None   # [4, n_q2, n_x] x q(x, Q^2) for u, ubar, d, dbar, or None


def synthetic_pdf(n_x: int = 100, n_q2: int = 50, A: float = 1.0, quarks: bool = False) -> PdfTable:
    """x g(x, Q^2) = A x^-0.2 (1 - x)^5 (1 + 0.1 ln Q^2) on log-spaced knots:
    x in [1e-7, 1] (100 knots, the last one x = 1), Q^2 in [10, 1e8] GeV^2.

    With quarks=True also proton-like quark tables for the q qbar channels,
    valence plus sea, the same Q^2 factor:
      x ubar = 0.09 x^-0.2 (1 - x)^7,   x u = 1.6 x^0.55 (1 - x)^3.2 + x ubar,
      x dbar = 0.11 x^-0.2 (1 - x)^7,   x d = 0.85 x^0.55 (1 - x)^4 + x dbar."""
    x = 10.0 ** (-7.0 + 7.0 * np.arange(n_x) / (n_x - 1))
    q2 = 10.0 ** (1.0 + 7.0 * np.arange(n_q2) / (n_q2 - 1))
    fq = 1.0 + 0.1 * np.log(q2)
    xg = A * x ** -0.2 * (1.0 - x) ** 5
    table = np.outer(fq, xg)
    xq = None
    if quarks:
        ubar = 0.09 * x ** -0.2 * (1.0 - x) ** 7
        dbar = 0.11 * x ** -0.2 * (1.0 - x) ** 7
        u = 1.6 * x ** 0.55 * (1.0 - x) ** 3.2 + ubar
        d = 0.85 * x ** 0.55 * (1.0 - x) ** 4 + dbar
        xq = np.ascontiguousarray(np.stack([np.outer(fq, f) for f in (u, ubar, d, dbar)]), dtype=np.float64)
    return PdfTable(np.ascontiguousarray(np.log(x)), np.ascontiguousarray(np.log(q2)),
                    np.ascontiguousarray(table, dtype=np.float64), xq)


@dataclass(frozen=True)
class Workload:
    name: str
    process: str
    n_g: int
    n_events: int
    n_iter: int
    seeds: tuple
    ptmin_g: float = 0.0
    etamax_g: float = 0.0
    drmin_gg: float = 0.0
    precision: str = "fp64"
    m_top: float = M_TOP
    w_top: float = W_TOP
    alpha_s: float = ALPHA_S
    mu_f: float = MU_F
    extra: dict = field(default_factory=dict)

    @property
    def n_dims(self) -> int:
        return 2 + 3 * self.n_g - 4


# The five workload configurations: LO g g -> t tbar (+ 0, 1, 2 gluons).
WORKLOADS = {
    "ttx": Workload("ttx", "gg_ttx", 2, 100_000, 5, (0,)),
    "ttxg": Workload("ttxg", "gg_ttxg", 3, 10_000_000, 10, (0, 1, 2, 3, 4),
                     ptmin_g=20.0, etamax_g=2.5),
    "ttxgg": Workload("ttxgg", "gg_ttxgg", 4, 10_000_000, 10, (0,),
                      ptmin_g=20.0, drmin_gg=0.4),
    "ttx_grad": Workload("ttx_grad", "gg_ttx", 2, 10_000_000, 10, (0,),
                         extra={"m_top_scan": (170.0, 173.0, 176.0)}),
    "ttxgg_fp32": Workload("ttxgg_fp32", "gg_ttxgg", 4, 100_000_000, 10, (0,),
                           ptmin_g=20.0, drmin_gg=0.4, precision="fp32_kahan"),
}


def random_uniforms(n: int, dims: int, seed: int) -> np.ndarray:
    """Seeded uniforms in [0, 1) for tests that feed explicit random inputs."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.random((n, dims)))
