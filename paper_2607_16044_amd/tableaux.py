"""ARS IMEX tableau pairs in the padded layout of Sec. 4.2.2 (Tab. butcher_tableau_sidebyside).

The paper adopts the Ascher-Ruuth-Spiteri (1997) schemes without printing
their constants; they are restated here from that reference.  ARS(2,2,2) is
FSAL and stiffly accurate; ARS(3,4,3) is stiffly accurate only.  For
ARS(3,4,3) the published 10-digit decimals are kept and the first entry of
each explicit row is set so that the row sums equal the stage times exactly.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Pair:
    name: str
    s: int
    Ae: np.ndarray    # (s+1, s+1) explicit, strictly lower triangular
    be: np.ndarray    # (s+1,)
    Ai: np.ndarray    # (s, s) implicit (SDIRK)
    bi: np.ndarray    # (s,)

    @property
    def fsal(self) -> bool:
        return bool(np.array_equal(self.be, self.Ae[-1]))

    @property
    def stiffly_accurate(self) -> bool:
        return bool(np.array_equal(self.bi, self.Ai[-1]))

    def to_ctypes(self, cls):
        t = cls()
        t.s = self.s
        for i in range(self.s + 1):
            for j in range(self.s + 1):
                t.Ae[4 * i + j] = self.Ae[i, j]
            t.be[i] = self.be[i]
        for i in range(self.s):
            for j in range(self.s):
                t.Ai[3 * i + j] = self.Ai[i, j]
            t.bi[i] = self.bi[i]
        t.fsal = int(self.fsal)
        t.stiffly_accurate = int(self.stiffly_accurate)
        return t


def ars222() -> Pair:
    gam = (2.0 - math.sqrt(2.0)) / 2.0
    dl = -math.sqrt(2.0) / 2.0          # 1 - 1/(2 gamma)
    Ae = np.array([[0.0, 0.0, 0.0], [gam, 0.0, 0.0], [dl, 1.0 - dl, 0.0]])
    return Pair("ARS222", 2, Ae, Ae[2].copy(), np.array([[gam, 0.0], [1.0 - gam, gam]]),
                np.array([1.0 - gam, gam]))


def ars343() -> Pair:
    # gamma: root of 6 g^3 - 18 g^2 + 9 g - 1 in (0, 1), by bisection
    lo, hi = 0.4, 0.5
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if (6 * mid ** 3 - 18 * mid ** 2 + 9 * mid - 1) > 0:
            lo = mid
        else:
            hi = mid
    gam = 0.5 * (lo + hi)
    b1 = -1.5 * gam * gam + 4.0 * gam - 0.25
    b2 = 1.5 * gam * gam - 5.0 * gam + 1.25
    a32, a42, a43 = 0.3966543747, 0.5529291479, 0.5529291479
    Ae = np.zeros((4, 4))
    Ae[1, 0] = gam
    Ae[2, 1] = a32
    Ae[2, 0] = 0.5 * (1.0 + gam) - a32
    Ae[3, 1] = a42
    Ae[3, 2] = a43
    Ae[3, 0] = 1.0 - a42 - a43
    be = np.array([0.0, b1, b2, gam])
    Ai = np.array([[gam, 0.0, 0.0], [0.5 * (1.0 - gam), gam, 0.0], [b1, b2, gam]])
    return Pair("ARS343", 3, Ae, be, Ai, np.array([b1, b2, gam]))


def get(name: str) -> Pair:
    return {"ARS222": ars222, "ARS343": ars343}[name]()
