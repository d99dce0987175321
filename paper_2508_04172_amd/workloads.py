"""Seeded synthetic workloads shared by the library's callers and the oracle.

This module holds configuration constants and seeded random draws only: no
waveform, no PSD, no inner product and no other step of the likelihood
method.  Everything that depends on the method (colouring the noise, the
injection, the ellipsoid frame, the reference distance) is computed by each
consumer on its own side.

Workload shapes follow the paper's simulated-signal study (Sec. III A: NSBH
systems, three-detector network, Table I priors) and its third-generation
case (Sec. III A, ET paragraph), scaled to synthetic stand-ins: an analytic
aLIGO-like PSD and a TaylorF2-like multimode waveform family.

Seeds: 0 noise, 1 queries, 2 injection extrinsics, 3 ragged event generator,
4 MLP initialisation, 5 surrogate training points, 6 held-out points.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Tuple

import numpy as np

EARTH_RADIUS_LS = 6371.0e3 / 299792458.0  # Earth radius in light-seconds

ALL_MODES: Tuple[Tuple[int, int], ...] = ((2, 2), (2, 1), (3, 3), (3, 2), (4, 4))

# Three synthetic ground sites: latitude, longitude, x-arm azimuth (from
# north toward east), arm opening angle, distance from the geocentre.
_DEG = math.pi / 180.0
SITES_HLV = (
    (46.5 * _DEG, -119.4 * _DEG, 36.0 * _DEG, 90.0 * _DEG, EARTH_RADIUS_LS),
    (30.6 * _DEG, -90.8 * _DEG, 108.0 * _DEG, 90.0 * _DEG, EARTH_RADIUS_LS),
    (43.6 * _DEG, 10.5 * _DEG, 71.0 * _DEG, 90.0 * _DEG, EARTH_RADIUS_LS),
)
# A single detector placed at the geocentre (zero light-travel delay).
SITE_GEOCENTRE = ((0.8, -2.0, 0.3, 90.0 * _DEG, 0.0),)
# Co-located triangle: three 60-degree interferometers rotated by 120 degrees.
SITES_TRIANGLE = tuple((40.5 * _DEG, 9.4 * _DEG, a * _DEG, 60.0 * _DEG, EARTH_RADIUS_LS)
                       for a in (0.0, 120.0, 240.0))


@dataclass(frozen=True)
class Config:
    """One workload: detector network, signal, interpolant and query shape."""
    name: str
    fs: float
    seg_len: float
    f_low: float
    modes: Tuple[Tuple[int, int], ...]
    sites: Tuple[Tuple[float, float, float, float, float], ...]
    psd_scale: float
    inj_phys: Tuple[float, float, float, float]   # m1, m2 [Msun], chi1z, chi2z
    inj_snr: float
    match: float
    n_nodes: int
    q: int
    eps: float
    poly_degree: int
    half_window: float
    n_queries: int
    tc_span: float                                # queries: t_c offset in +-tc_span [s]
    random_sky: bool                              # queries draw sky/psi/iota (else injected)
    noise_seed: int = 0
    query_seed: int = 1
    inj_seed: int = 2
    chi_max: float = 1.0
    center_node: bool = False
    f_ref: float = 0.0                            # template time/phase reference [Hz]; 0 = automatic, < 0 = coalescence
    squeeze: bool = False                         # contract the longest ellipsoid axis to the true-match crossing
    optimise_centre: bool = False                 # move the centre to the network-SNR optimum first
    centre_offset: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 0.0)   # seed = injection + offset
    earth_rate: float = 0.0                       # Earth rotation [rad/s] in the exact model and the injection
    n_bands: int = 1                              # time bands of the antenna patterns in the meshfree model (1: frozen)

    @property
    def n_det(self) -> int:
        return len(self.sites)

    @property
    def n_samples(self) -> int:
        return int(round(self.fs * self.seg_len))

    @property
    def n_freq(self) -> int:
        return self.n_samples // 2 + 1

    @property
    def t_trig(self) -> float:
        """Trigger (injection merger) time: on the sample grid, 2 s before the end."""
        return self.seg_len - 2.0

    @property
    def n_poly(self) -> int:
        return math.comb(self.poly_degree + 4, 4)

    @property
    def n_out(self) -> int:
        """Interpolated real outputs per query: per detector (and time band) 2q
        per mode + n^2 overlap reals."""
        n = len(self.modes)
        return self.n_det * max(1, self.n_bands) * (2 * self.q * n + n * n)

    @property
    def seed_phys(self) -> Tuple[float, float, float, float]:
        """The ellipsoid centre handed to the start-up: the injection plus
        centre_offset (a seed template off the injection, as a search's best
        match would be)."""
        return tuple(a + b for a, b in zip(self.inj_phys, self.centre_offset))

    def with_(self, **kw) -> "Config":
        return replace(self, **kw)


CFG1 = Config(name="cfg1_single_det_22", fs=2048.0, seg_len=16.0, f_low=20.0,
              modes=((2, 2),), sites=SITE_GEOCENTRE, psd_scale=1.0,
              inj_phys=(8.0, 1.4, 0.3, 0.0), inj_snr=20.0, match=0.97,
              n_nodes=200, q=20, eps=1.0, poly_degree=1, half_window=0.05,
              n_queries=10_000, tc_span=0.047, random_sky=False)

CFG2 = Config(name="cfg2_hlv_5mode", fs=4096.0, seg_len=64.0, f_low=20.0,
              modes=ALL_MODES, sites=SITES_HLV, psd_scale=1.0,
              inj_phys=(8.0, 1.4, 0.3, 0.0), inj_snr=20.0, match=0.97,
              n_nodes=800, q=40, eps=2.0, poly_degree=1, half_window=0.05,
              n_queries=1_000_000, tc_span=0.027, random_sky=True)

CFG3 = Config(name="cfg3_mixed_cubic", fs=2048.0, seg_len=256.0, f_low=10.0,
              modes=((2, 2),), sites=SITE_GEOCENTRE, psd_scale=1.0,
              inj_phys=(8.0, 1.4, 0.3, 0.0), inj_snr=20.0, match=0.97,
              n_nodes=1500, q=60, eps=3.0, poly_degree=3, half_window=0.05,
              n_queries=4_000_000, tc_span=0.047, random_sky=False)

CFG5 = Config(name="cfg5_triangle_snr200", fs=4096.0, seg_len=2048.0, f_low=5.0,
              modes=ALL_MODES, sites=SITES_TRIANGLE, psd_scale=0.1,
              inj_phys=(8.0, 1.4, 0.3, 0.0), inj_snr=200.0, match=0.97,
              n_nodes=3000, q=80, eps=3.0, poly_degree=1, half_window=0.05,
              n_queries=10_000_000, tc_span=0.027, random_sky=True)

# Reduced cases that the oracle finishes in seconds, used for element-wise parity.
SMALL_MULTI = CFG2.with_(name="small_hlv_3mode", fs=2048.0, seg_len=8.0,
                         modes=ALL_MODES[:3], n_nodes=150, q=12, n_queries=3000,
                         tc_span=0.027)

# Long signals on a rotating Earth: the source's Earth-fixed longitude drifts
# during the signal.  The small case turns the Earth fast (2e-2 rad/s, 0.1 rad
# over its 5.6 s signal) so that a few time bands matter at 8 s of data; the
# third-generation case rotates at the sidereal rate over its 1694 s signal.
SIDEREAL = 7.2921150e-5
SMALL_BANDED = SMALL_MULTI.with_(name="small_hlv_banded", earth_rate=2e-2, n_bands=4)
CFG5_ROTATING = CFG5.with_(name="cfg5_triangle_rotating", earth_rate=SIDEREAL)

CONFIGS = {c.name: c for c in (CFG1, CFG2, CFG3, CFG5, SMALL_MULTI, SMALL_BANDED, CFG5_ROTATING)}


# ----------------------------------------------------------------------------
# seeded draws
# ----------------------------------------------------------------------------

def white_noise(cfg: Config) -> np.ndarray:
    """Standard normal deviates, shape [n_det][n_freq][2] (re, im); seed cfg.noise_seed."""
    rng = np.random.default_rng(cfg.noise_seed)
    return rng.standard_normal((cfg.n_det, cfg.n_freq, 2))


def injection_extrinsics(cfg: Config) -> np.ndarray:
    """(alpha, dec, psi, iota, phi) of the injection, seed cfg.inj_seed (Table I shapes)."""
    rng = np.random.default_rng(cfg.inj_seed)
    alpha = rng.uniform(0.0, 2 * math.pi)
    dec = math.asin(rng.uniform(-1.0, 1.0))
    psi = rng.uniform(0.0, math.pi)
    iota = math.acos(rng.uniform(-1.0, 1.0))
    phi = rng.uniform(0.0, 2 * math.pi)
    return np.array([alpha, dec, psi, iota, phi])


def uniform_ball(rng: np.random.Generator, n: int, dim: int = 4) -> np.ndarray:
    """n points uniform in the unit dim-ball, shape [n][dim]."""
    g = rng.standard_normal((n, dim))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    r = rng.uniform(0.0, 1.0, n) ** (1.0 / dim)
    return g * r[:, None]


@dataclass
class QueryDraw:
    """Queries in normalised form.

    x: [n][4] displacement along the ellipsoid eigen-axes in units of each
    semi-axis (uniform in the unit ball); ext: [n][5] (alpha, dec, psi, iota,
    phi); dt: [n] t_c offset from the trigger [s]; dist_ratio: [n] d_L over
    the reference (injection) distance, uniform in volume over [1/2, 2].
    The caller turns these into the paper's coordinates with its own frame:
    delta_e = semi_axes * x, t_c = t_trig + dt, d_L = d_ref * dist_ratio.
    """
    x: np.ndarray
    ext: np.ndarray
    dt: np.ndarray
    dist_ratio: np.ndarray

    def subset(self, idx) -> "QueryDraw":
        return QueryDraw(self.x[idx], self.ext[idx], self.dt[idx], self.dist_ratio[idx])

    def near_nodes(self, nodes: np.ndarray, node_idx: np.ndarray, jitter: np.ndarray) -> "QueryDraw":
        """Copy with x = nodes[node_idx] + jitter (rescaled into the unit ball)."""
        x = nodes[node_idx] + jitter
        x /= np.maximum(1.0, np.linalg.norm(x, axis=1) / 0.999999)[:, None]
        return QueryDraw(x, self.ext, self.dt, self.dist_ratio)

    def __len__(self) -> int:
        return self.x.shape[0]


def queries(cfg: Config, n: int | None = None, seed: int | None = None,
            inj_ext: np.ndarray | None = None, clustered: float = 0.0) -> QueryDraw:
    """Seeded query draw.  With cfg.random_sky False the sky, polarisation and
    inclination stay at the injected values (the paper's Fig. 3 protocol) and
    only phase, distance, t_c and the intrinsic point vary.  clustered > 0
    draws x from a Gaussian of that width about the centre instead (a
    converged sampler step) and t_c within +-2 ms."""
    n = cfg.n_queries if n is None else n
    rng = np.random.default_rng(cfg.query_seed if seed is None else seed)
    if clustered > 0.0:
        x = rng.standard_normal((n, 4)) * clustered
        x /= np.maximum(1.0, np.linalg.norm(x, axis=1) / 0.999)[:, None]
        dt = rng.uniform(-0.002, 0.002, n)
    else:
        x = uniform_ball(rng, n)
        dt = rng.uniform(-cfg.tc_span, cfg.tc_span, n)
    if inj_ext is None:
        inj_ext = injection_extrinsics(cfg)
    ext = np.empty((n, 5))
    if cfg.random_sky:
        ext[:, 0] = rng.uniform(0.0, 2 * math.pi, n)
        ext[:, 1] = np.arcsin(rng.uniform(-1.0, 1.0, n))
        ext[:, 2] = rng.uniform(0.0, math.pi, n)
        ext[:, 3] = np.arccos(rng.uniform(-1.0, 1.0, n))
    else:
        ext[:, 0:4] = inj_ext[0:4]
    ext[:, 4] = rng.uniform(0.0, 2 * math.pi, n)
    lo, hi = 0.5 ** 3, 2.0 ** 3
    dist_ratio = (lo + (hi - lo) * rng.uniform(0.0, 1.0, n)) ** (1.0 / 3.0)
    return QueryDraw(x=x, ext=ext, dt=dt, dist_ratio=dist_ratio)


def node_jitter(n: int, n_nodes: int, sigma: float = 0.03, seed: int = 7):
    """Seeded (node index, jitter) pairs for proposals near the interpolation
    nodes, i.e. inside the physical part of the ellipsoid where a sampler's
    proposals concentrate; resolve with QueryDraw.near_nodes(own_nodes, ...)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, n_nodes, n), rng.standard_normal((n, 4)) * sigma


def mlp_normals(n_params: int, seed: int = 4) -> np.ndarray:
    """Standard normal deviates for the surrogate network's initial weights."""
    return np.random.default_rng(seed).standard_normal(n_params)


def ragged_events(n_events: int = 64, seed: int = 3, walkers: int = 1024,
                  base: Config = CFG2, seg_range=(8.0, 512.0), node_range=(200, 1500),
                  q_range=(20, 60)) -> List[Config]:
    """Uneven events for the multi-event batch: segment length log-uniform in
    [8, 512] s, m1 ~ U[5, 20], m2 ~ U[1, 3] with m1 / m2 <= 10,
    chi1 ~ U[-0.998, 0.998], chi2 ~ U[-0.05, 0.05] (the paper's NSBH injection
    ranges, Sec. III A and Table I), 1-5 modes,
    200-1500 nodes, q in 20-60.  f_low is raised above 20 Hz where needed so
    that the Newtonian chirp time fits in 90% of the segment."""
    rng = np.random.default_rng(seed)
    out = []
    msun_s = 4.925490947641267e-06
    for e in range(n_events):
        seg = float(round(math.exp(rng.uniform(math.log(seg_range[0]), math.log(seg_range[1])))))
        m1 = rng.uniform(5.0, 20.0)
        m2 = rng.uniform(1.0, 3.0)
        while m1 > 10.0 * m2:              # Table I keeps the mass ratio within [1, 10]
            m1 = rng.uniform(5.0, 20.0)
            m2 = rng.uniform(1.0, 3.0)
        c1 = rng.uniform(-0.998, 0.998)
        c2 = rng.uniform(-0.05, 0.05)
        n_modes = int(rng.integers(1, 6))
        n_nodes = int(rng.integers(node_range[0], node_range[1] + 1))
        q = int(rng.integers(q_range[0], q_range[1] + 1))
        mc = (m1 * m2) ** 0.6 / (m1 + m2) ** 0.2 * msun_s
        # Newtonian chirp time from f: (5/256) (pi f)^(-8/3) Mc^(-5/3)
        f_low = 20.0
        while (5.0 / 256.0) * (math.pi * f_low) ** (-8.0 / 3.0) * mc ** (-5.0 / 3.0) > 0.9 * seg:
            f_low += 1.0
        eps = 0.0       # chosen by each side from its RBF system (smallest integer with cond <= 1e12)
        out.append(base.with_(name=f"event{e:02d}", seg_len=seg, f_low=f_low,
                              modes=ALL_MODES[:n_modes], inj_phys=(m1, m2, c1, c2),
                              n_nodes=n_nodes, q=q, eps=eps, n_queries=walkers,
                              noise_seed=1000 + e, inj_seed=2000 + e, query_seed=3000 + e))
    return out
