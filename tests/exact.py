"""Exact references for the 2D q-state Potts model on small periodic lattices.

These are the independent results the oracle is pinned to; they share nothing
with the oracle or the GPU library.

* :func:`dos_transfer` -- density of states g(b), b = number of satisfied bonds
  (E = -b, eq. (3) with J = 1), by a row-to-row transfer matrix.
* :func:`dos_brute` -- the same by enumerating every configuration.
* :func:`ising_lnZ_kaufman` -- Kaufman's (1949) closed form for the Ising
  partition function on an m x n torus, in the form given by Beale (1996).
* :func:`potts_q2_lnZ` -- q = 2 Potts from Ising: delta(s,s') = (1 + sigma sigma')/2
  gives Z_Potts(beta) = exp(beta N) Z_Ising(K = beta/2) on a lattice with 2N bonds.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def _row_states(L: int, q: int) -> np.ndarray:
    """All q^L rows as an array [q^L, L] of spins."""
    return np.array(list(itertools.product(range(q), repeat=L)), dtype=np.int64)


def dos_transfer(L: int, q: int) -> np.ndarray:
    """g[b] for b = 0..2N: number of configurations with b satisfied bonds.

    Bonds: every site to its right and to its lower neighbour, periodic (2N
    bonds; on L = 2 each nearest-neighbour pair is bonded twice).

    The generating polynomial sum_b g[b] z^b equals trace(T(z)^L) for the
    row-to-row transfer matrix T(z)[a, b] = z^(vertical bonds(a, b) +
    horizontal bonds(b)).  It is evaluated at the 2N+1 roots of unity and the
    integer coefficients are recovered by an inverse DFT (exact after rounding
    while q^N is far below 2^53)."""
    N = L * L
    if q ** N >= 2 ** 50:
        raise ValueError("too large for exact recovery in double precision")
    rows = _row_states(L, q)
    horiz = (rows == np.roll(rows, -1, axis=1)).sum(axis=1)
    vert = (rows[:, None, :] == rows[None, :, :]).sum(axis=2)
    w = vert + horiz[None, :]
    D = 2 * N + 1
    vals = np.empty(D, dtype=np.complex128)
    for k in range(D):
        z = np.exp(2j * np.pi * k / D)
        T = z ** w
        vals[k] = np.trace(np.linalg.matrix_power(T, L))
    # vals[k] = sum_b g_b exp(2 pi i k b / D), so the forward DFT returns D g_b
    coef = np.fft.fft(vals) / D
    return np.rint(coef.real).astype(np.int64)


def dos_brute(L: int, q: int, energy=None) -> np.ndarray:
    """g[b] by enumerating all q^N configurations.  ``energy`` (optional) maps a
    configuration array [N] (uint8) to E; by default bonds are counted here."""
    N = L * L
    g = np.zeros(2 * N + 1, dtype=np.int64)
    if energy is not None:
        for conf in itertools.product(range(q), repeat=N):
            E = energy(np.array(conf, dtype=np.uint8))
            g[-E] += 1
        return g
    idx = np.arange(N).reshape(L, L)
    right = np.roll(idx, -1, axis=1).ravel()
    down = np.roll(idx, -1, axis=0).ravel()
    chunk_digits = min(N, 10)
    low = np.array(list(itertools.product(range(q), repeat=chunk_digits)), dtype=np.int8)
    for high in itertools.product(range(q), repeat=N - chunk_digits):
        conf = np.empty((len(low), N), dtype=np.int8)
        conf[:, : N - chunk_digits] = np.array(high, dtype=np.int8)
        conf[:, N - chunk_digits:] = low
        b = (conf == conf[:, right]).sum(axis=1) + (conf == conf[:, down]).sum(axis=1)
        g += np.bincount(b, minlength=2 * N + 1)
    return g


def lnZ_from_dos(g: np.ndarray, beta: float) -> float:
    """ln sum_b g[b] exp(beta b)  (E = -b)."""
    b = np.nonzero(g)[0]
    terms = np.log(g[b].astype(np.float64)) + beta * b
    m = terms.max()
    return float(m + math.log(np.exp(terms - m).sum()))


def mean_E_from_dos(g: np.ndarray, beta: float) -> float:
    b = np.nonzero(g)[0]
    terms = np.log(g[b].astype(np.float64)) + beta * b
    p = np.exp(terms - terms.max())
    p /= p.sum()
    return float(-(p * b).sum())


def var_E_from_dos(g: np.ndarray, beta: float) -> float:
    b = np.nonzero(g)[0]
    terms = np.log(g[b].astype(np.float64)) + beta * b
    p = np.exp(terms - terms.max())
    p /= p.sum()
    m = (p * b).sum()
    return float((p * (b - m) ** 2).sum())


def ising_lnZ_kaufman(m: int, n: int, K: float) -> float:
    """ln Z of the Ising model H = -sum sigma_i sigma_j on an m x n torus at
    coupling K = beta J (Kaufman 1949; Beale, PRL 76 (1996) 78):

        Z = 1/2 (2 sinh 2K)^{mn/2} (Z1 + Z2 + Z3 + Z4),
        Z1 = prod_{r<n} 2 cosh(m g_{2r+1}/2),  Z2 = prod 2 sinh(m g_{2r+1}/2),
        Z3 = prod_{r<n} 2 cosh(m g_{2r}/2),    Z4 = prod 2 sinh(m g_{2r}/2),
        cosh g_k = cosh 2K coth 2K - cos(pi k / n),   g_0 = 2K + ln tanh K.
    """
    c = math.cosh(2 * K) / math.tanh(2 * K)

    def gamma(k: int) -> float:
        if k == 0:
            return 2 * K + math.log(math.tanh(K))
        return math.acosh(c - math.cos(math.pi * k / n))

    logs, signs = [], []
    for odd, fn in ((1, "cosh"), (1, "sinh"), (0, "cosh"), (0, "sinh")):
        lg, sg = 0.0, 1
        for r in range(n):
            x = m * gamma(2 * r + odd) / 2
            v = 2 * (math.cosh(x) if fn == "cosh" else math.sinh(x))
            if v == 0.0:
                lg, sg = -math.inf, 0
                break
            lg += math.log(abs(v))
            sg *= 1 if v > 0 else -1
        logs.append(lg)
        signs.append(sg)
    top = max(l for l in logs if l != -math.inf)
    s = sum(sg * math.exp(l - top) for l, sg in zip(logs, signs) if sg != 0)
    return math.log(0.5) + (m * n / 2) * math.log(2 * math.sinh(2 * K)) + top + math.log(s)


def potts_q2_lnZ(L: int, beta: float) -> float:
    N = L * L
    return beta * N + ising_lnZ_kaufman(L, L, beta / 2)


def one_sweep_matrix_L2(q: int, beta: float) -> tuple[np.ndarray, np.ndarray]:
    """Exact transition matrix of one checkerboard Metropolis sweep on the
    2 x 2 periodic lattice, and the energies of its q^4 configurations.

    Configuration index a = s0 q^3 + s1 q^2 + s2 q + s3 with sites
    0 = (0,0), 1 = (0,1), 2 = (1,0), 3 = (1,1) (row-major).  Colour 0 =
    {0, 3}, colour 1 = {1, 2}; a half-sweep updates the sites of one colour,
    each seeing only the other colour.  Each site's left and right neighbours
    are the same site, as are its upper and lower ones, so each counts twice.
    Per site: a proposal uniform over the q - 1 other states, accepted with
    probability 1 when dE <= 0, else T(dE) / 2^32 with the integer threshold
    T(dE) = floor(2^32 exp(-beta dE)) (w uniform over 2^32 words, accepted when
    w < T).  The sweep is colour 0, then colour 1: P = P0 @ P1."""
    confs = np.array(list(itertools.product(range(q), repeat=4)), dtype=np.int64)
    nb = {0: (1, 2), 1: (0, 3), 2: (3, 0), 3: (2, 1)}   # (horizontal, vertical) neighbour

    def energy(c):
        return -sum(2 * int(c[n] == c[nb[n][0]]) + 2 * int(c[n] == c[nb[n][1]]) for n in range(4)) // 2

    E = np.array([energy(c) for c in confs], dtype=np.int64)
    acc = {d: (1.0 if d <= 0 else math.floor(math.ldexp(math.exp(-beta * d), 32)) / 2.0 ** 32)
           for d in range(-8, 9)}

    def site_kernel(c, n):
        """Distribution of the new spin of site n given configuration c."""
        s = int(c[n])
        h, v = c[nb[n][0]], c[nb[n][1]]
        neigh = (h, h, v, v)
        p = np.zeros(q)
        stay = 1.0
        for t in range(q):
            if t == s:
                continue
            dE = sum(int(x == s) for x in neigh) - sum(int(x == t) for x in neigh)
            pt = acc[dE] / (q - 1)
            p[t] = pt
            stay -= pt
        p[s] += stay
        return p

    def half_matrix(sites):
        M = np.zeros((len(confs), len(confs)))
        for a, c in enumerate(confs):
            pa_, pb_ = site_kernel(c, sites[0]), site_kernel(c, sites[1])
            for ta in range(q):
                for tb in range(q):
                    d = c.copy()
                    d[sites[0]], d[sites[1]] = ta, tb
                    M[a, int(d[0] * q ** 3 + d[1] * q ** 2 + d[2] * q + d[3])] += pa_[ta] * pb_[tb]
        return M

    return half_matrix((0, 3)) @ half_matrix((1, 2)), E
