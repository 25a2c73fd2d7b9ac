"""Seeded stand-ins for the paper's populations, and the subspace list.

Sources of the shapes:

* The paper's catalogue (Sec. 2.1, Tab. 1) has |D| = 31,693 objects and 15
  features, every one min-max normalised to [0, 1] before any join
  (Sec. 3.3).  Every subset of 2..15 features is a feature space, which
  makes 32,752 spaces (Eq. 1).
* The catalogue itself is not available, so a SNAPShot1-shaped population
  is drawn with the distributions below (one column per feature, column f is
  bit f of a subspace mask):

  ====  ==========================================  =========================
  col   distribution                                role
  ====  ==========================================  =========================
  0     LogNormal(mu = ln 8 h, sigma = 1)           rotation period
  1     Gamma(shape 2, scale 0.15)                  light-curve amplitude
  2     Normal(15, 1.5)                             absolute magnitude H
  3..6  Normal(0.4, 0.1), pairwise rho = 0.6        four colour-like features
  7     Uniform(2.1, 3.3)                           semi-major axis (AU)
  8     Beta(2, 12)                                 eccentricity
  9     Rayleigh(sigma = 0.12 rad)                  inclination
  10..  Normal(0, 1)                                five further features
  ====  ==========================================  =========================

  0.5 % of the objects are tail outliers: 1-3 random features of each are
  moved to mu +/- U(6, 10) sigma of that feature with a random sign (for the
  log-normal column the shift is applied in log space).
* The LSST-scale set of Sec. 2.2 (5M objects) is drawn from the same
  generator at N = 5,000,000.

Every draw is seeded from ``SeedSequence(240520176)``; one child per
workload, and grandchildren per job or request.  The normalisation below is
the input precondition of Sec. 3.3 (per feature, over the whole population,
computed in float64 and rounded to float32; a constant feature maps to 0).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field
from typing import Iterator, List, Tuple

import numpy as np

ROOT_SEED = 240520176
N_FEATURES = 15
FEATURE_NAMES = (
    "rotper_h", "lcamp", "h_mag", "col0", "col1", "col2", "col3",
    "a_au", "ecc", "inc_rad", "z0", "z1", "z2", "z3", "z4",
)
TABLE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tables")

# Workload indices of the five configurations.
C0, C1, C2, C3, C4 = range(5)


def config_seeds() -> List[np.random.SeedSequence]:
    """One SeedSequence per workload, in the order C0..C4."""
    return np.random.SeedSequence(ROOT_SEED).spawn(5)


def _rng(cfg: int) -> np.random.Generator:
    return np.random.default_rng(config_seeds()[cfg])


# ---------------------------------------------------------------- ingest ---

def normalize_minmax(raw: np.ndarray, lo=None, hi=None):
    """Min-max normalise each column of ``raw`` (rows = objects) to [0, 1].

    Computed in float64 and rounded to float32.  ``lo``/``hi`` default to the
    column minima/maxima of ``raw``; passing a population's bounds maps new
    objects (alerts) into that population's frame, where they may fall
    outside [0, 1].  Returns ``(x32, lo, hi)``.
    """
    r = np.asarray(raw, dtype=np.float64)
    if lo is None:
        lo = r.min(axis=0)
    if hi is None:
        hi = r.max(axis=0)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    span = hi - lo
    safe = np.where(span > 0, span, 1.0)
    x = (r - lo) / safe
    x = np.where(span > 0, x, 0.0)
    return x.astype(np.float32), lo, hi


# ------------------------------------------------------------- subspaces ---

def all_masks(n_features: int = N_FEATURES, dmin: int = 2, dmax: int | None = None) -> np.ndarray:
    """Every feature subset with dmin <= |S| <= dmax as a bit mask, ordered
    by (|S|, mask).  For 15 features and 2..15 this is the 32,752 spaces of
    Eq. 1."""
    if dmax is None:
        dmax = n_features
    masks = [m for m in range(1, 1 << n_features) if dmin <= bin(m).count("1") <= dmax]
    masks.sort(key=lambda m: (bin(m).count("1"), m))
    return np.asarray(masks, dtype=np.uint32)


def mask_features(mask: int) -> List[int]:
    """Column indices (ascending) of the features in ``mask``."""
    return [f for f in range(32) if (int(mask) >> f) & 1]


# --------------------------------------------------------- C0 (tiny run) ---

def gen_c0(n: int = 2000):
    """Tiny plain run: n objects in one 3-feature space.

    97 % from a 3-component isotropic Gaussian mixture (equal weights, means
    U[0.2, 0.8]^3, sigma_c U[0.05, 0.15]), 3 % uniform in [0, 1]^3, then
    normalised.  Returns ``(x32 [n, 3], k)`` with k = 5.
    """
    rng = _rng(C0)
    n_out = int(round(0.03 * n))
    n_in = n - n_out
    means = rng.uniform(0.2, 0.8, size=(3, 3))
    sig = rng.uniform(0.05, 0.15, size=3)
    comp = rng.integers(0, 3, size=n_in)
    pts = means[comp] + rng.standard_normal((n_in, 3)) * sig[comp, None]
    iso = rng.uniform(0.0, 1.0, size=(n_out, 3))
    raw = np.concatenate([pts, iso], axis=0)
    raw = raw[rng.permutation(n)]
    x, _, _ = normalize_minmax(raw)
    return x, 5


def gen_isolated_fixture(n_cluster: int = 600, m_corner: int = 5, seed_offset: int = 0):
    """Three tight clusters (sigma 0.02, means in [0.3, 0.7]^3) plus
    ``m_corner`` points on corners of the unit cube.  Corner (0,0,0) and
    (1,1,1) are always included so that normalisation keeps the corners on
    the corners.  Returns ``(x32, corner_ids)``."""
    ss = config_seeds()[C0].spawn(8 + seed_offset)[-1]
    rng = np.random.default_rng(ss)
    means = rng.uniform(0.3, 0.7, size=(3, 3))
    comp = np.repeat(np.arange(3), n_cluster // 3 + 1)[:n_cluster]
    pts = means[comp] + rng.standard_normal((n_cluster, 3)) * 0.02
    corners_all = np.array([[(c >> 2) & 1, (c >> 1) & 1, c & 1] for c in range(8)], dtype=np.float64)
    others = rng.choice(np.arange(1, 7), size=m_corner - 2, replace=False)
    corners = corners_all[np.concatenate([[0, 7], others])]
    raw = np.concatenate([pts, corners], axis=0)
    perm = rng.permutation(raw.shape[0])
    raw = raw[perm]
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    corner_ids = np.sort(inv[n_cluster:])
    x, _, _ = normalize_minmax(raw)
    return x, corner_ids


# ------------------------------------------- SNAPShot1-shaped population ---

# (mu, sigma) of each column's distribution, used to place tail outliers.
_LOGNORM_MU, _LOGNORM_SIG = math.log(8.0), 1.0
_COL_MOMENTS = [
    (_LOGNORM_MU, _LOGNORM_SIG),                       # in log space
    (2 * 0.15, math.sqrt(2) * 0.15),                   # Gamma(2, 0.15)
    (15.0, 1.5),
    (0.4, 0.1), (0.4, 0.1), (0.4, 0.1), (0.4, 0.1),
    (2.7, 1.2 / math.sqrt(12.0)),                      # U(2.1, 3.3)
    (2.0 / 14.0, math.sqrt(2.0 * 12.0 / (14.0 ** 2 * 15.0))),   # Beta(2, 12)
    (0.12 * math.sqrt(math.pi / 2), 0.12 * math.sqrt((4 - math.pi) / 2)),  # Rayleigh
    (0.0, 1.0), (0.0, 1.0), (0.0, 1.0), (0.0, 1.0), (0.0, 1.0),
]


def snapshot1_like_raw(rng: np.random.Generator, n: int, outlier_frac: float = 0.005) -> np.ndarray:
    """Raw (un-normalised) SNAPShot1-shaped features, float64 [n, 15]."""
    out = np.empty((n, N_FEATURES), dtype=np.float64)
    log_per = rng.normal(_LOGNORM_MU, _LOGNORM_SIG, size=n)
    out[:, 1] = rng.gamma(2.0, 0.15, size=n)
    out[:, 2] = rng.normal(15.0, 1.5, size=n)
    cov = np.full((4, 4), 0.6) + 0.4 * np.eye(4)
    chol = np.linalg.cholesky(cov)
    out[:, 3:7] = 0.4 + 0.1 * (rng.standard_normal((n, 4)) @ chol.T)
    out[:, 7] = rng.uniform(2.1, 3.3, size=n)
    out[:, 8] = rng.beta(2.0, 12.0, size=n)
    out[:, 9] = rng.rayleigh(0.12, size=n)
    out[:, 10:15] = rng.standard_normal((n, 5))
    n_out = int(round(outlier_frac * n))
    if n_out:
        rows = rng.choice(n, size=n_out, replace=False)
        for r in rows:
            nf = int(rng.integers(1, 4))
            feats = rng.choice(N_FEATURES, size=nf, replace=False)
            for f in feats:
                mu, sg = _COL_MOMENTS[f]
                v = mu + (1.0 if rng.random() < 0.5 else -1.0) * rng.uniform(6.0, 10.0) * sg
                if f == 0:
                    log_per[r] = v
                else:
                    out[r, f] = v
    out[:, 0] = np.exp(log_per)
    return out


C1_N = 31693


def gen_c1(n: int = C1_N):
    """SNAPShot1-shaped full run: normalised float32 [n, 15] population and
    the (|S|, mask)-ordered list of all 32,752 subspaces; k = 10."""
    raw = snapshot1_like_raw(_rng(C1), n)
    x, _, _ = normalize_minmax(raw)
    return x, all_masks(), 10


def load_c1_eps(path: str | None = None):
    """The stored float32 epsilon per C1 subspace (target mean count 10),
    aligned with :func:`all_masks`.  Written by ``make_eps_tables.py``."""
    path = path or os.path.join(TABLE_DIR, "c1_eps.npz")
    z = np.load(path, allow_pickle=False)
    masks, eps = z["masks"], z["eps"]
    if not np.array_equal(masks, all_masks()):
        raise ValueError("epsilon table does not match the subspace order")
    return eps.astype(np.float32)


# ----------------------------------------------------------- C2 (LSST) ---

def gen_c2(n: int = 5_000_000):
    """LSST-scale population (Sec. 2.2 stand-in): normalised float32
    [n, 15]; spaces = the full 15-feature space plus the 105 two-feature
    spaces; k = 10; epsilon target mean count 20."""
    raw = snapshot1_like_raw(_rng(C2), n)
    x, _, _ = normalize_minmax(raw)
    del raw
    masks = np.concatenate([[np.uint32((1 << N_FEATURES) - 1)], all_masks(dmin=2, dmax=2)])
    return x, masks.astype(np.uint32), 10, 20


def load_c2_eps(path: str | None = None):
    """The stored float32 epsilon of every C2 space (target mean count 20),
    aligned with the masks of :func:`gen_c2`.  Written by
    ``make_eps_tables.py c2``."""
    path = path or os.path.join(TABLE_DIR, "c2_eps.npz")
    z = np.load(path, allow_pickle=False)
    masks = np.concatenate([[np.uint32((1 << N_FEATURES) - 1)], all_masks(dmin=2, dmax=2)]).astype(np.uint32)
    if not np.array_equal(z["masks"], masks):
        raise ValueError("C2 epsilon table does not match the space order")
    return z["eps"].astype(np.float32)


# --------------------------------------------------- C3 (batched uneven) ---

@dataclass
class C3Job:
    index: int
    n: int
    mask: int
    k: int
    seed: np.random.SeedSequence = field(repr=False)


def gen_c3_jobs(n_jobs: int = 4096) -> List[C3Job]:
    """Batched uneven jobs: N log-uniform in [1e4, 5e5], |S| uniform in
    2..15 with a seeded feature subset, k in {5, 10, 20}; each job owns its
    own population (drawn lazily by :func:`gen_c3_population`)."""
    ss = config_seeds()[C3]
    rng = np.random.default_rng(ss)
    kids = ss.spawn(n_jobs)
    jobs = []
    for j in range(n_jobs):
        n = int(round(math.exp(rng.uniform(math.log(1e4), math.log(5e5)))))
        d = int(rng.integers(2, 16))
        feats = rng.choice(N_FEATURES, size=d, replace=False)
        mask = int(sum(1 << int(f) for f in feats))
        k = int(rng.choice([5, 10, 20]))
        jobs.append(C3Job(j, n, mask, k, kids[j]))
    return jobs


def gen_c3_population(job: C3Job, n: int | None = None) -> np.ndarray:
    """Normalised float32 [n, 15] population of one C3 job (``n`` overrides
    the job's size for scaled-down tests)."""
    rng = np.random.default_rng(job.seed)
    raw = snapshot1_like_raw(rng, job.n if n is None else n)
    x, _, _ = normalize_minmax(raw)
    return x


def gen_c3_projected(job: C3Job, n: int | None = None) -> np.ndarray:
    """The job's population in its own subspace: normalised float32 [n, d],
    the subspace's features in ascending order -- all a job reads of its
    population.  Only those d features are drawn, each from a stream of its
    own (spawned from the job's seed), with the distributions of
    :func:`snapshot1_like_raw`: the four colour-like features are drawn
    jointly (correlated) whenever one of them is in the subspace, and the
    0.5 % tail outliers (1-3 of the 15 features each, moved to mean +/-
    U(6, 10) sigma; the rotation period in log space) come from one more
    stream, so that every job sees the same outlier rows and features
    whatever its subspace.  Normalisation is per feature over the
    population, as for the other workloads."""
    n = job.n if n is None else n
    feats = mask_features(job.mask)
    kids = job.seed.spawn(N_FEATURES + 1)
    raw = np.empty((n, len(feats)), dtype=np.float64)
    colour = None
    for c, f in enumerate(feats):
        if 3 <= f <= 6:
            if colour is None:
                cov = np.full((4, 4), 0.6) + 0.4 * np.eye(4)
                colour = 0.4 + 0.1 * (np.random.default_rng(kids[3]).standard_normal((n, 4)) @
                                      np.linalg.cholesky(cov).T)
            raw[:, c] = colour[:, f - 3]
            continue
        rng = np.random.default_rng(kids[f])
        if f == 0:
            raw[:, c] = rng.normal(_LOGNORM_MU, _LOGNORM_SIG, size=n)      # log period; exp below
        elif f == 1:
            raw[:, c] = rng.gamma(2.0, 0.15, size=n)
        elif f == 2:
            raw[:, c] = rng.normal(15.0, 1.5, size=n)
        elif f == 7:
            raw[:, c] = rng.uniform(2.1, 3.3, size=n)
        elif f == 8:
            raw[:, c] = rng.beta(2.0, 12.0, size=n)
        elif f == 9:
            raw[:, c] = rng.rayleigh(0.12, size=n)
        else:
            raw[:, c] = rng.standard_normal(n)
    rng = np.random.default_rng(kids[N_FEATURES])
    n_out = int(round(0.005 * n))
    if n_out:
        rows = rng.choice(n, size=n_out, replace=False)
        nf = rng.integers(1, 4, size=n_out)
        which = np.argsort(rng.random((n_out, N_FEATURES)), axis=1)[:, :3]
        sign = np.where(rng.random((n_out, 3)) < 0.5, 1.0, -1.0)
        mag = rng.uniform(6.0, 10.0, size=(n_out, 3))
        col_of = {f: c for c, f in enumerate(feats)}
        for t in range(3):
            for r, f, sg, mg, keep in zip(rows, which[:, t], sign[:, t], mag[:, t], t < nf):
                if keep and int(f) in col_of:
                    mu, sd = _COL_MOMENTS[int(f)]
                    raw[r, col_of[int(f)]] = mu + sg * mg * sd
    if 0 in feats:
        raw[:, 0] = np.exp(raw[:, 0])
    x, _, _ = normalize_minmax(raw)
    return x


def load_c3_eps(path: str | None = None):
    """The stored float32 epsilon of every C3 job (sampler target = the job's
    k), aligned with :func:`gen_c3_jobs`.  Written by ``make_eps_tables.py
    c3``."""
    path = path or os.path.join(TABLE_DIR, "c3_eps.npz")
    z = np.load(path, allow_pickle=False)
    jobs = gen_c3_jobs(len(z["eps"]))
    if not (np.array_equal(z["masks"], [j.mask for j in jobs]) and np.array_equal(z["n"], [j.n for j in jobs])):
        raise ValueError("C3 epsilon table does not match the job list")
    return z["eps"].astype(np.float32)


# ------------------------------------------------------------ C4 (serve) ---

@dataclass
class C4Request:
    rid: int
    arrival_s: float
    pop: int
    space: int           # index into that population's served-space list
    n_alerts: int
    seed: np.random.SeedSequence = field(repr=False)


@dataclass
class C4Workload:
    n_pop: int
    pop_n: int
    spaces: List[np.ndarray]          # per population: uint32 masks
    k: int
    rate_hz: float
    seeds: List[np.random.SeedSequence] = field(repr=False)

    def population(self, p: int):
        """Normalised float32 [pop_n, 15] population p and its raw bounds."""
        rng = np.random.default_rng(self.seeds[p])
        raw = snapshot1_like_raw(rng, self.pop_n)
        x, lo, hi = normalize_minmax(raw)
        return x, lo, hi

    def requests(self, duration_s: float, max_alerts: int = 10_000, start_s: float = 0.0) -> Iterator[C4Request]:
        """Open-loop Poisson arrivals (exponential gaps at ``rate_hz``);
        alerts per request log-uniform in [1, max_alerts]."""
        ss = self.seeds[-1]
        rng = np.random.default_rng(ss)
        t = start_s
        rid = 0
        while True:
            t += rng.exponential(1.0 / self.rate_hz)
            if t >= start_s + duration_s:
                return
            p = int(rng.integers(0, self.n_pop))
            s = int(rng.integers(0, len(self.spaces[p])))
            na = int(math.floor(math.exp(rng.uniform(0.0, math.log(max_alerts + 1)))))
            na = max(1, min(max_alerts, na))
            yield C4Request(rid, t, p, s, na, np.random.SeedSequence(entropy=ROOT_SEED, spawn_key=(4, 1000, rid)))
            rid += 1

    def alerts(self, req: C4Request, lo, hi) -> np.ndarray:
        """Alert objects of a request, drawn from the same generator and
        mapped with the population's bounds: float32 [n_alerts, 15]."""
        rng = np.random.default_rng(req.seed)
        raw = snapshot1_like_raw(rng, req.n_alerts, outlier_frac=0.005)
        x, _, _ = normalize_minmax(raw, lo, hi)
        return x


def load_c4_eps(path: str | None = None):
    """Stored float32 eps of the first served subspaces of every serving
    population: (masks [n_pop, s], eps [n_pop, s]).  Written by
    ``make_eps_tables.py c4``."""
    path = path or os.path.join(TABLE_DIR, "c4_eps.npz")
    z = np.load(path, allow_pickle=False)
    return z["masks"], z["eps"].astype(np.float32)


def gen_c4(n_pop: int = 4, pop_n: int = 1_000_000, spaces_per_pop: int = 64,
           rate_hz: float = 200.0, k: int = 10) -> C4Workload:
    """Serving workload: ``n_pop`` resident populations, each with a seeded
    catalogue of served subspaces (|S| uniform in 2..15)."""
    ss = config_seeds()[C4]
    kids = ss.spawn(n_pop + 2)
    rng = np.random.default_rng(kids[n_pop])
    spaces = []
    for _ in range(n_pop):
        ms = []
        while len(ms) < spaces_per_pop:
            d = int(rng.integers(2, 16))
            feats = rng.choice(N_FEATURES, size=d, replace=False)
            m = int(sum(1 << int(f) for f in feats))
            if m not in ms:
                ms.append(m)
        spaces.append(np.asarray(ms, dtype=np.uint32))
    return C4Workload(n_pop, pop_n, spaces, k, rate_hz, list(kids[:n_pop]) + [kids[n_pop + 1]])


def to_soa(x: np.ndarray, ld: int | None = None) -> Tuple[np.ndarray, int]:
    """Row-major [n, F] float32 -> column-major SoA [F, ld] float32 with the
    leading dimension rounded up to a multiple of 64 (zero padding)."""
    n, f = x.shape
    if ld is None:
        ld = (n + 63) // 64 * 64
    out = np.zeros((f, ld), dtype=np.float32)
    out[:, :n] = x.T
    return out, ld
