"""Oracle of the ensemble sampler and the prior reweighting (Sec. II D:
sampling in the Delta e coordinates; Sec. III A: importance weights
p_target / p_sampled).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy, exact
32-bit integer arithmetic for the random numbers.

Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC 2011), key = the seed's two 32-bit
words, counter = (walker, step mod 2^32, (step / 2^32 mod 2^31) | half << 31,
call).  Uniforms u = ((a >> 5) 2^26 + (b >> 6) + 1/2) 2^-53 from each pair of
output words.

Moves: differential-evolution Metropolis (ter Braak, Stat. Comput. 16, 2006)
over the two halves of the ensemble: walker i of a half proposes
Y = X_i + g (X_j - X_k), j != k from the other half, g = gamma (1 + 0.01 n)
or 1 with probability p_jump; the angles alpha, psi, phi wrap (periods 2 pi,
pi, 2 pi, differences taken the shorter way round).  Accept with probability
min(1, posterior ratio), ln L weighted by beta = beta0^(1 - step / anneal)
during an annealed start.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .physics import theta_to_phys

MASK = 0xFFFFFFFF
PERIODS = {4: 2.0 * math.pi, 6: math.pi, 8: 2.0 * math.pi}


def philox4x32_10(ctr, key):
    """ctr: 4 arrays (or ints) of 32-bit words, key: 2; returns 4 uint64
    arrays holding the 32-bit outputs.  Each of the 10 rounds multiplies
    words 0 and 2 by 0xD2511F53 and 0xCD9E8D57 (full 64-bit products) and
    mixes the halves with the other words and the round key; the key grows by
    0x9E3779B9 and 0xBB67AE85 per round."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & MASK for v in ctr)
    k0 = np.uint64(key[0] & MASK)
    k1 = np.uint64(key[1] & MASK)
    m0, m1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
    for _ in range(10):
        p0 = c0 * m0            # < 2^64: exact in uint64
        p1 = c2 * m1
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + np.uint64(0x9E3779B9)) & np.uint64(MASK)
        k1 = (k1 + np.uint64(0xBB67AE85)) & np.uint64(MASK)
    return c0, c1, c2, c3


def u01(a, b):
    m = ((a >> np.uint64(5)) << np.uint64(26)) | (b >> np.uint64(6))
    return (m.astype(np.float64) + 0.5) * 2.0 ** -53


def uniform_pair(seed: int, walker, step: int, half: int, call: int):
    """Two uniforms per walker from one Philox block."""
    walker = np.asarray(walker, dtype=np.uint64)
    ctr = (walker, np.full_like(walker, step & MASK), np.full_like(walker, ((step >> 32) & 0x7FFFFFFF) | (half << 31)),
           np.full_like(walker, call))
    o = philox4x32_10(ctr, (seed & MASK, (seed >> 32) & MASK))
    return u01(o[0], o[1]), u01(o[2], o[3])


@dataclass
class Prior:
    t_lo: float
    t_hi: float
    d_lo: float
    d_hi: float
    d_exp: float = 0.0


def log_prior(frame, f0: float, chi_max: float, prior: Prior, P: np.ndarray) -> np.ndarray:
    """P: [11][n].  Uniform in Delta e inside the unit ball and the physical
    region; isotropic sky (density cos dec) and orientation (sin iota);
    alpha, psi, phi uniform; t_c uniform; d_L density d^d_exp."""
    x = P[0:4].T / frame.semi[None, :]
    inside = np.sum(x * x, axis=1) <= 1.0
    th = frame.theta_c[None, :] + P[0:4].T @ frame.vecs.T
    m1, m2, c1, c2, eta = theta_to_phys(th.T, f0)
    with np.errstate(invalid="ignore"):
        phys = (eta <= 0.25) & (np.abs(c1) <= chi_max) & (np.abs(c2) <= chi_max) & np.isfinite(c1 + c2)
        dec, iota, tc, dl = P[5], P[7], P[9], P[10]
        ok = inside & phys & (dec > -math.pi / 2) & (dec < math.pi / 2) & (iota > 0) & (iota < math.pi)
        ok &= (tc >= prior.t_lo) & (tc <= prior.t_hi) & (dl >= prior.d_lo) & (dl <= prior.d_hi)
        val = np.log(np.cos(dec)) + np.log(np.sin(iota)) + prior.d_exp * np.log(dl)
    return np.where(ok, val, -np.inf)


def init_walkers(frame, f0: float, chi_max: float, prior: Prior, seed: int, W: int):
    """Walkers from the prior (counter step 2^63 - 1, half 1): Delta e by
    rejection from the cube to the unit ball and the physical region (up to
    4096 tries, else the centre), then alpha = 2 pi u, dec = asin(2u - 1),
    psi = pi u, iota = acos(2u - 1), phi = 2 pi u, t_c uniform, d_L by the
    inverse of its cumulative distribution."""
    step, half = 0x7FFFFFFFFFFFFFFF, 1
    X = np.zeros((11, W))
    for w in range(W):
        t = 0
        found = False
        for _ in range(4096):
            a0, a1 = uniform_pair(seed, [w], step, half, t)
            a2, a3 = uniform_pair(seed, [w], step, half, t + 1)
            t += 2
            u = np.array([a0[0], a1[0], a2[0], a3[0]])
            x = 2.0 * u - 1.0
            if np.sum(x * x) > 1.0:
                continue
            de = x * frame.semi
            th = frame.theta_c + frame.vecs @ de
            m1, m2, c1, c2, eta = theta_to_phys(th, f0)
            if eta <= 0.25 and abs(c1) <= chi_max and abs(c2) <= chi_max and np.isfinite(c1 + c2):
                X[0:4, w] = de
                found = True
                break
        if not found:
            X[0:4, w] = 0.0
        u = []
        for k in range(4):
            p, q = uniform_pair(seed, [w], step, half, t + k)
            u += [p[0], q[0]]
        X[4, w] = 2.0 * math.pi * u[0]
        X[5, w] = math.asin(2.0 * u[1] - 1.0)
        X[6, w] = math.pi * u[2]
        X[7, w] = math.acos(2.0 * u[3] - 1.0)
        X[8, w] = 2.0 * math.pi * u[4]
        X[9, w] = prior.t_lo + (prior.t_hi - prior.t_lo) * u[5]
        e = prior.d_exp + 1.0
        a, b = prior.d_lo ** e, prior.d_hi ** e
        X[10, w] = (a + (b - a) * u[6]) ** (1.0 / e)
    return X


def de_half_step(X, lnl_x, lp_x, seed: int, step: int, half: int, gamma: float, p_jump: float, lnl_fn, lp_fn,
                 beta: float = 1.0):
    """One half-step in place.  X: [11][W]; lnl_fn / lp_fn map proposals
    [11][M] to ln L / log prior; beta weights ln L in the acceptance (an
    annealed start).  Returns (proposals, accepted mask)."""
    W = X.shape[1]
    M = W // 2
    gi = half * M + np.arange(M)
    other = (1 - half) * M
    u0, u1 = uniform_pair(seed, gi, step, half, 0)
    u2, u3 = uniform_pair(seed, gi, step, half, 1)
    u4, _ = uniform_pair(seed, gi, step, half, 3)
    j = np.minimum((u0 * M).astype(np.int64), M - 1)
    k = np.minimum((u1 * (M - 1)).astype(np.int64), M - 2)
    k = np.where(k >= j, k + 1, k)
    g = gamma * (1.0 + 0.01 * np.sqrt(-2.0 * np.log(u2)) * np.cos(2.0 * math.pi * u3))
    g = np.where(u4 < p_jump, 1.0, g)
    Y = np.empty((11, M))
    for m in range(11):
        d = X[m, other + j] - X[m, other + k]
        P = PERIODS.get(m, 0.0)
        if P:
            d = d - P * np.rint(d / P)
        y = X[m, gi] + g * d
        if P:
            y = np.mod(y, P)
        Y[m] = y
    lpy = lp_fn(Y)
    ly = np.asarray(lnl_fn(Y), dtype=np.float64)
    ly = np.where(np.isnan(ly), -np.inf, ly)
    ua, _ = uniform_pair(seed, gi, step, half, 2)
    cur = lnl_x[gi] + lp_x[gi]
    prop = ly + lpy
    with np.errstate(invalid="ignore"):
        ratio = beta * (ly - lnl_x[gi]) + (lpy - lp_x[gi])
        take = np.isfinite(prop) & (~np.isfinite(cur) | (np.log(ua) < ratio))
    X[:, gi[take]] = Y[:, take]
    lnl_x[gi[take]] = ly[take]
    lp_x[gi[take]] = lpy[take]
    return Y, take


def anneal_beta(step: int, anneal_steps: int, beta0: float) -> float:
    return beta0 ** (1.0 - step / anneal_steps) if step < anneal_steps else 1.0


def log_prior_weights(frame, f0: float, params: np.ndarray, box, d_exp: float) -> np.ndarray:
    """log w = log |det d(m1, m2, chi1, chi2) / d Delta e| + d_exp log d_L
    (-inf outside box): importance weights from the prior uniform in Delta e
    to one uniform in the component masses and spins.  The Jacobian
    d phys / d Theta by the complex step through the closed-form inverse of
    Eq. metric_coords (V orthonormal: |det V| = 1)."""
    n = params.shape[1]
    th = frame.theta_c[None, :] + params[0:4].T @ frame.vecs.T
    m1, m2, c1, c2, _ = theta_to_phys(th.T, f0)
    phys = np.stack([m1, m2, c1, c2], axis=1)
    out = np.full(n, -np.inf)
    lo = np.asarray(box[0::2], dtype=np.float64)
    hi = np.asarray(box[1::2], dtype=np.float64)
    for i in range(n):
        p = phys[i]
        if not (np.all(np.isfinite(p)) and np.all(p >= lo) and np.all(p <= hi)):
            continue
        J = np.empty((4, 4))
        for m in range(4):
            tc = th[i].astype(np.complex128)
            h = 1e-20 * abs(th[i, m])
            tc[m] += 1j * h
            q = theta_to_phys(tc, f0)
            J[:, m] = np.imag(np.array(q[:4])) / h                 # d phys / d Theta_m
        out[i] = math.log(abs(np.linalg.det(J))) + d_exp * math.log(params[10, i])
    return out


def smc_stage(lnl: np.ndarray, beta: float, ess_frac: float, seed: int, stage: int):
    """One stage of the tempered sequential Monte Carlo start (Del Moral,
    Doucet and Jasra 2006): the increment db in (0, 1 - beta] that brings
    the effective sample size of the weights w = L^db to ess_frac W (the
    whole remainder if it stays above), found by bisection (60 halvings);
    the log evidence increment log mean w; and systematic resampling
    indices, position (u + i) / W with u from Philox (walker 2^32 - 1, step
    = stage, half 1, call 4).  Walkers with ln L = -inf get weight 0."""
    W = lnl.size
    fin = np.isfinite(lnl)
    m = np.max(lnl[fin])
    d = np.where(fin, lnl - m, -np.inf)

    def ess(db):
        w = np.exp(db * d)
        return math.fsum(w) ** 2 / math.fsum(w * w)

    rem = 1.0 - beta
    if ess(rem) >= ess_frac * W:
        db = rem
    else:
        lo, hi = 0.0, rem
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if ess(mid) >= ess_frac * W:
                lo = mid
            else:
                hi = mid
        db = lo
    w = np.exp(db * d)
    logz = db * m + math.log(math.fsum(w) / W)
    c = np.cumsum(w)
    c /= c[-1]
    u, _ = uniform_pair(seed, [0xFFFFFFFF], stage, 1, 4)
    pos = (u[0] + np.arange(W)) / W
    idx = np.minimum(np.searchsorted(c, pos, side="right"), W - 1)
    return db, idx, logz
