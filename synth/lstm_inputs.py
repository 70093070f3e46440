"""Seeded synthetic inputs of the MDHP-LSTM layer (no layer arithmetic).

One case holds a batch of B sequences of L inputs of width D, layer weights
for hidden width H drawn from U(-1/sqrt(H), 1/sqrt(H)) (torch.nn.LSTM's
initialisation), Hawkes-gate weights [A | B | C] from U(-8/sqrt(Kf),
8/sqrt(Kf)) over their Kf columns (so that hks spreads over most of
(-1, 1) rather than staying near 0), and per-sequence MDHP parameters of M dimensions on the
scale the layer is fed after standardisation: alpha in [0, 0.5/M] per
entry, beta in [0.5, 2], window lengths T_span in [0.5, 2], baselines theta
in [0.1, 1].  The upstream gradient dh is standard normal.  Everything is
float32 (the layer's precision), drawn from numpy's PCG64 with the seed.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class LstmCase:
    x: np.ndarray
    W: np.ndarray
    U: np.ndarray
    bias: np.ndarray
    Whks: np.ndarray
    alpha: np.ndarray
    beta: np.ndarray
    T_span: np.ndarray
    theta: np.ndarray
    dh: np.ndarray

    @property
    def dims(self):
        B, L, D = self.x.shape
        return B, L, D, self.U.shape[1], self.alpha.shape[1]

    def split_whks(self):
        """(A, B, C) blocks of Whks = [A | B | C]."""
        M = self.alpha.shape[1]
        Kb = 1 if self.beta.ndim == 1 else M * M
        return (self.Whks[:, :M * M], self.Whks[:, M * M:M * M + Kb],
                self.Whks[:, M * M + Kb:])


def case(seed: int, B: int, L: int, D: int, H: int, M: int, pair: bool = False) -> LstmCase:
    g = np.random.default_rng(seed)
    k = 1.0 / np.sqrt(H)
    Kb = M * M if pair else 1
    f = np.float32
    return LstmCase(
        x=g.standard_normal((B, L, D)).astype(f),
        W=g.uniform(-k, k, (4 * H, D)).astype(f),
        U=g.uniform(-k, k, (4 * H, H)).astype(f),
        bias=g.uniform(-k, k, 4 * H).astype(f),
        Whks=g.uniform(-1.0, 1.0, (H, M * M + Kb + M)).astype(f) * f(8.0 / np.sqrt(M * M + Kb + M)),
        alpha=g.uniform(0.0, 0.5 / M, (B, M, M)).astype(f),
        beta=g.uniform(0.5, 2.0, (B, M, M) if pair else B).astype(f),
        T_span=g.uniform(0.5, 2.0, B).astype(f),
        theta=g.uniform(0.1, 1.0, (B, M)).astype(f),
        dh=g.standard_normal((B, L, H)).astype(f))
