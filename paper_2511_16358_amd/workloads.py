"""Seeded synthetic inputs for iFCTN tensor completion workloads.

This module holds random draws and data-shaping only: it never evaluates an
iFCTN reconstruction, a factor update or any other step of the completion
method.  A planted low-rank tensor is returned as *factor draws*; the caller
assembles the planted tensor with whatever implementation it is testing or
timing (the CPU oracle in tests, the HIP library in benchmarks) and hands the
result back to :func:`finish`, which adds the non-iFCTN structure (bumps,
textures, outliers, noise), normalises to [0, 1] and draws the sampling mask
and the initial factors.

Conventions shared by every consumer (layout only, no arithmetic):

* modes are 0-based, tensors are row-major (last mode fastest);
* the factor ``G[(k, i)]`` (the paper's cherry factor G_{k,i}) has shape
  ``(R_ki, I_k)``; the packed order is k ascending, then i ascending (i != k),
  each factor row-major;
* ranks are an N x N symmetric integer matrix with an unused diagonal.

The recipes follow the workload descriptions of the paper's experiments
(multispectral images 256x256x31, traffic 214x61x144; Sec. 5) with synthetic
stand-ins for the datasets, which are not available.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Dict, Tuple

import numpy as np

FactorDict = Dict[Tuple[int, int], np.ndarray]


# --------------------------------------------------------------------------
# layout conventions
# --------------------------------------------------------------------------
def factor_keys(N: int):
    """Packed factor order: k ascending, then i ascending with i != k."""
    return [(k, i) for k in range(N) for i in range(N) if i != k]


def uniform_ranks(N: int, R: int) -> np.ndarray:
    r = np.full((N, N), R, dtype=np.int64)
    np.fill_diagonal(r, 0)
    return r


def factor_shapes(dims, ranks):
    return [((k, i), (int(ranks[k][i]), int(dims[k]))) for (k, i) in factor_keys(len(dims))]


def num_factor_entries(dims, ranks) -> int:
    return sum(r * n for _, (r, n) in factor_shapes(dims, ranks))


def pack(G: FactorDict, dims, ranks) -> np.ndarray:
    parts = []
    for key, shape in factor_shapes(dims, ranks):
        a = np.asarray(G[key], dtype=np.float64)
        assert a.shape == shape, (key, a.shape, shape)
        parts.append(a.reshape(-1))
    return np.ascontiguousarray(np.concatenate(parts))


def unpack(flat, dims, ranks) -> FactorDict:
    flat = np.asarray(flat, dtype=np.float64)
    out, off = {}, 0
    for key, (r, n) in factor_shapes(dims, ranks):
        out[key] = flat[off:off + r * n].reshape(r, n).copy()
        off += r * n
    assert off == flat.size
    return out


# --------------------------------------------------------------------------
# problem container
# --------------------------------------------------------------------------
@dataclass
class Problem:
    name: str
    dims: Tuple[int, ...]
    ranks: np.ndarray
    O: np.ndarray            # observed tensor, float32, zero off the mask
    mask: np.ndarray         # uint8, 1 = observed
    X_true: np.ndarray       # ground truth, float32
    G0: FactorDict           # initial factors (float64)
    rho: float = 0.1
    sweeps: int = 20
    meta: dict = field(default_factory=dict)

    @property
    def nX(self) -> int:
        return int(np.prod(self.dims))


@dataclass
class Draws:
    """Everything random about one workload instance, before assembly."""
    name: str
    dims: Tuple[int, ...]
    ranks: np.ndarray
    planted: FactorDict      # factors of the planted iFCTN part
    rng_state: dict          # generator state after the factor draws
    sweeps: int
    rho: float = 0.1
    extra: dict = field(default_factory=dict)


CONFIGS = {
    # name: (dims, rank, sweeps)
    "planted30": ((30, 30, 30), 2, 20),
    "msi256": ((256, 256, 31), 6, 100),
    "traffic214": ((214, 61, 144), 4, 200),
    "video144": ((144, 176, 3, 50), 5, 150),
}

DESCRIPTIONS = {
    "planted30": "order-3 30x30x30, planted iFCTN R=2 with N(0,1) factors, unit max, "
                 "50% uniform sampling, noiseless, rho=0.1, 20 sweeps",
    "msi256": "order-3 256x256x31 multispectral-image-shaped: planted iFCTN R=6 + 20 Gaussian "
              "bumps with smooth spectral profiles + N(0,0.01^2) noise, min-max [0,1], "
              "10% uniform sampling, 100 sweeps",
    "traffic214": "order-3 214x61x144 traffic-shaped: nonnegative planted iFCTN R=4 with a daily "
                  "sinusoidal profile, 5% outliers set to 0, 20% uniform sampling minus 10% "
                  "whole missing (sensor, day) fibres, 200 sweeps",
    "video144": "order-4 144x176x3x50 colour-video-shaped: planted iFCTN R=5 + a smooth texture "
                "translated per frame (bilinear, wrap), min-max [0,1], 5% uniform sampling, "
                "150 sweeps",
}


def _draw_factors(rng, dims, ranks, kind: str) -> FactorDict:
    G = {}
    for key, shape in factor_shapes(dims, ranks):
        if kind == "normal":
            G[key] = rng.standard_normal(shape)
        else:
            G[key] = rng.uniform(0.0, 1.0, size=shape)
    return G


def draw(name: str, seed: int = 0, dims=None, rank=None) -> Draws:
    """Random draws for a named workload (optionally at other dims / rank)."""
    d0, r0, sweeps = CONFIGS[name]
    dims = tuple(int(x) for x in (dims or d0))
    R = int(rank or r0)
    N = len(dims)
    ranks = uniform_ranks(N, R)
    rng = np.random.default_rng(seed)
    kind = "normal" if name == "planted30" else "uniform"
    planted = _draw_factors(rng, dims, ranks, kind)
    extra = {}
    if name == "traffic214":
        # daily profile on the time-slot mode: scaling columns of one factor of
        # that mode keeps the planted part exactly of iFCTN rank R.
        T = dims[2]
        phi = rng.uniform(0.0, 2.0 * math.pi)
        prof = 1.0 + 0.5 * np.sin(2.0 * math.pi * np.arange(T) / T + phi)
        planted[(2, 0)] = planted[(2, 0)] * prof[None, :]
        extra["phase"] = phi
    return Draws(name, dims, ranks, planted, rng.bit_generator.state, sweeps, 0.1, extra)


def _gaussian_bumps(rng, H, W, B, count=20):
    y = np.arange(H, dtype=np.float64)[:, None, None]
    x = np.arange(W, dtype=np.float64)[None, :, None]
    b = np.arange(B, dtype=np.float64)[None, None, :]
    out = np.zeros((H, W, B))
    for _ in range(count):
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        sig = rng.uniform(8, 32)
        mu, s, a = rng.uniform(0, B), rng.uniform(4, 12), rng.uniform(0.2, 1.0)
        spatial = np.exp(-((y - cy) ** 2 + (x - cx) ** 2) / (2 * sig * sig))
        spectral = a * np.exp(-((b - mu) ** 2) / (2 * s * s))
        out += spatial * spectral
    return out


def _translated_texture(rng, H, W, C, T):
    # smooth periodic texture from a few low-frequency Fourier modes
    yy, xx = np.meshgrid(np.arange(H) / H, np.arange(W) / W, indexing="ij")
    tex = np.zeros((H, W, C))
    for c in range(C):
        for _ in range(12):
            u, v = rng.integers(-4, 5), rng.integers(-4, 5)
            a, ph = rng.uniform(0.2, 1.0), rng.uniform(0, 2 * math.pi)
            tex[:, :, c] += a * np.cos(2 * math.pi * (u * yy + v * xx) + ph)
    # smooth translation path, bilinear sampling with wrap-around
    vy, vx = rng.uniform(-1.5, 1.5), rng.uniform(-1.5, 1.5)
    ay, ax = rng.uniform(2, 8), rng.uniform(2, 8)
    out = np.empty((H, W, C, T))
    gy, gx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    for t in range(T):
        dy = vy * t + ay * math.sin(2 * math.pi * t / T)
        dx = vx * t + ax * math.cos(2 * math.pi * t / T)
        sy, sx = gy + dy, gx + dx
        y0, x0 = np.floor(sy).astype(np.int64), np.floor(sx).astype(np.int64)
        fy, fx = sy - y0, sx - x0
        y0m, y1m = y0 % H, (y0 + 1) % H
        x0m, x1m = x0 % W, (x0 + 1) % W
        for c in range(C):
            t00 = tex[y0m, x0m, c]
            t01 = tex[y0m, x1m, c]
            t10 = tex[y1m, x0m, c]
            t11 = tex[y1m, x1m, c]
            out[:, :, c, t] = ((1 - fy) * ((1 - fx) * t00 + fx * t01)
                               + fy * ((1 - fx) * t10 + fx * t11))
    return out


def _minmax(a):
    lo, hi = a.min(), a.max()
    return (a - lo) / (hi - lo) if hi > lo else np.zeros_like(a)


def initial_factors(rng, dims, ranks, observed_rms: float) -> FactorDict:
    """G0 ~ U(0,1) * s, with s chosen so that a product of e edge matrices of
    i.i.d. U(0, s) factors has mean close to the observed RMS value."""
    N = len(dims)
    e = N * (N - 1) // 2
    Rbar = float(np.mean([ranks[a][b] for a in range(N) for b in range(N) if a != b]))
    m = max(observed_rms, 1e-12)
    s = math.sqrt(4.0 * m ** (1.0 / e) / Rbar)
    return {key: rng.uniform(0.0, 1.0, size=shape) * s
            for key, shape in factor_shapes(dims, ranks)}


def finish(d: Draws, core: np.ndarray) -> Problem:
    """Turn an assembled planted tensor ``core`` (= iFCTN of ``d.planted``)
    into a completion problem: add the non-low-rank structure, normalise,
    sample the mask and draw the initial factors."""
    rng = np.random.default_rng()
    rng.bit_generator.state = d.rng_state
    dims = d.dims
    core = np.asarray(core, dtype=np.float64).reshape(dims)
    meta = dict(d.extra)
    if d.name == "planted30":
        X = core / np.max(np.abs(core))
        mask = rng.random(dims) < 0.5
    elif d.name == "msi256":
        X = core / np.max(np.abs(core))
        X = X + _gaussian_bumps(rng, *dims)
        X = X + rng.normal(0.0, 0.01, size=dims)
        X = _minmax(X)
        mask = rng.random(dims) < 0.10
    elif d.name == "traffic214":
        X = core / np.max(np.abs(core))
        meta["X_clean"] = X.astype(np.float32)
        out = rng.random(dims) < 0.05
        X = np.where(out, 0.0, X)
        keep = rng.random(dims) < 0.20
        fibre_missing = rng.random(dims[:2]) < 0.10
        mask = keep & ~fibre_missing[:, :, None]
    elif d.name == "video144":
        X = core / np.max(np.abs(core))
        X = X + _minmax(_translated_texture(rng, *dims))
        X = _minmax(X)
        mask = rng.random(dims) < 0.05
    else:
        raise KeyError(d.name)
    X32 = X.astype(np.float32)
    mask_u8 = mask.astype(np.uint8)
    O = np.where(mask, X32, np.float32(0.0)).astype(np.float32)
    obs = X32[mask].astype(np.float64)
    rms = float(np.sqrt(np.mean(obs * obs))) if obs.size else 1.0
    G0 = initial_factors(rng, dims, d.ranks, rms)
    return Problem(d.name, dims, d.ranks, O, mask_u8, X32, G0, d.rho, d.sweeps, meta)


def problem(name: str, seed: int, assemble: Callable[[tuple, np.ndarray, FactorDict], np.ndarray],
            dims=None, rank=None) -> Problem:
    """Draw, assemble the planted part with ``assemble(dims, ranks, G)``, finish."""
    d = draw(name, seed, dims=dims, rank=rank)
    core = assemble(d.dims, d.ranks, d.planted)
    return finish(d, core)


def random_problem(dims, ranks, seed: int, keep: float = 0.5, rho: float = 0.1,
                   sweeps: int = 3) -> Problem:
    """A small unstructured problem (uniform data, Bernoulli mask) for parity
    tests of arbitrary shapes and ranks; no planted structure is needed."""
    rng = np.random.default_rng(seed)
    dims = tuple(int(x) for x in dims)
    ranks = np.asarray(ranks, dtype=np.int64)
    X = rng.uniform(0.0, 1.0, size=dims).astype(np.float32)
    mask = rng.random(dims) < keep
    O = np.where(mask, X, np.float32(0.0)).astype(np.float32)
    obs = X[mask].astype(np.float64)
    rms = float(np.sqrt(np.mean(obs * obs))) if obs.size else 1.0
    G0 = initial_factors(rng, dims, ranks, rms)
    return Problem("random", dims, ranks, O, mask.astype(np.uint8), X, G0, rho, sweeps)


# --------------------------------------------------------------------------
# served mix: many completion requests with Poisson arrivals
# --------------------------------------------------------------------------
SERVED = dict(n=512, rate=200.0, orders=(3, 4, 5), size_lo=16, size_hi=256, cap=4194304,
              ranks=(2, 3, 4, 5, 6), keeps=(0.05, 0.10, 0.30), t_max=100, eps=1e-5, noise=0.01)


@dataclass
class ServedSpec:
    index: int
    arrival: float            # seconds after the first arrival window opens
    dims: tuple
    ranks: np.ndarray
    keep: float
    seed: int                 # seed of this request's own tensors
    planted: FactorDict       # N(0, 1) planted factors


def served_dims(rng, N, lo, hi, cap):
    """Mode sizes ~ U{lo..hi}; when the product exceeds the cap every mode is
    scaled by (cap / product)^(1/N), floored, and kept >= lo."""
    dims = [int(x) for x in rng.integers(lo, hi + 1, size=N)]
    prod = math.prod(dims)
    if prod > cap:
        f = (cap / prod) ** (1.0 / N)
        dims = [max(lo, int(math.floor(d * f))) for d in dims]
        while math.prod(dims) > cap:          # floating-point edge: shave the largest mode
            m = int(np.argmax(dims))
            dims[m] -= 1
    return tuple(dims)


def served_requests(n=None, seed=0, **over):
    """Shapes, ranks, sampling ratios, arrival times and planted factors of
    the served mix (random draws only)."""
    cfg = dict(SERVED)
    cfg.update(over)
    n = cfg["n"] if n is None else n
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for q in range(n):
        t += float(rng.exponential(1.0 / cfg["rate"]))
        N = int(rng.choice(cfg["orders"]))
        dims = served_dims(rng, N, cfg["size_lo"], cfg["size_hi"], cfg["cap"])
        R = int(rng.choice(cfg["ranks"]))
        keep = float(rng.choice(cfg["keeps"]))
        ranks = uniform_ranks(N, R)
        rs = int(rng.integers(0, 2 ** 31 - 1))
        planted = _draw_factors(np.random.default_rng(rs), dims, ranks, "normal")
        out.append(ServedSpec(q, t, dims, ranks, keep, rs, planted))
    return out


def served_problem(spec: ServedSpec, core: np.ndarray) -> Problem:
    """Finish one served request from its assembled planted tensor: unit max,
    N(0, 0.01^2) noise, Bernoulli(keep) mask, initial factors."""
    rng = np.random.default_rng(spec.seed + 1)
    X = np.asarray(core, dtype=np.float64).reshape(spec.dims)
    X = X / np.max(np.abs(X))
    X = X + rng.normal(0.0, SERVED["noise"], size=spec.dims)
    mask = rng.random(spec.dims) < spec.keep
    X32 = X.astype(np.float32)
    O = np.where(mask, X32, np.float32(0.0)).astype(np.float32)
    obs = X32[mask].astype(np.float64)
    rms = float(np.sqrt(np.mean(obs * obs))) if obs.size else 1.0
    G0 = initial_factors(rng, spec.dims, spec.ranks, rms)
    return Problem(f"served{spec.index}", spec.dims, spec.ranks, O, mask.astype(np.uint8), X32, G0, 0.1,
                   SERVED["t_max"])


# --------------------------------------------------------------------------
# the paper's synthetic workload and rank grids (Sec. 5)
# --------------------------------------------------------------------------
def tucker_problem(seed: int = 0, missing: float = 0.8, dims=(20, 20, 20, 20), tucker=(5, 5, 5, 5),
                   rank: int = 3) -> Problem:
    """Order-4 20^4 tensor of Tucker rank (5,5,5,5) with core and factor
    matrices drawn from U(0,1) (the synthetic experiment of Sec. 5), divided
    by its largest entry, with a uniform random missing rate.  `rank` is the
    iFCTN rank of every edge the solver uses; the rank grid below varies it."""
    rng = np.random.default_rng(seed)
    core = rng.uniform(0.0, 1.0, size=tucker)
    X = core
    for m, (I, r) in enumerate(zip(dims, tucker)):
        U = rng.uniform(0.0, 1.0, size=(I, r))
        X = np.moveaxis(np.tensordot(U, X, axes=([1], [m])), 0, m)   # mode-m product
    X = X / np.max(np.abs(X))
    mask = rng.random(dims) >= missing
    X32 = X.astype(np.float32)
    O = np.where(mask, X32, np.float32(0.0)).astype(np.float32)
    obs = X32[mask].astype(np.float64)
    rms = float(np.sqrt(np.mean(obs * obs))) if obs.size else 1.0
    ranks = uniform_ranks(len(dims), rank)
    G0 = initial_factors(rng, dims, ranks, rms)
    return Problem("tucker20", tuple(dims), ranks, O, mask.astype(np.uint8), X32, G0, 0.1, 1000,
                   {"missing": missing, "tucker": tucker})


def rank_grid_uniform(N: int, values=(2, 3, 4, 5, 6, 7, 8)):
    """One rank matrix per value, every edge equal."""
    return [uniform_ranks(N, v) for v in values]


def rank_grid_msi(r12=(3, 6, 9, 15, 30, 36), r13=(3, 6, 9)):
    """The image rank grid of Sec. 5 for order-3 tensors: R_{1,2} over one set
    and R_{1,3} = R_{2,3} over another (0-based modes: R[0][1], R[0][2] = R[1][2]),
    18 rank matrices by default."""
    out = []
    for a in r12:
        for b in r13:
            r = np.zeros((3, 3), dtype=np.int64)
            r[0][1] = r[1][0] = a
            r[0][2] = r[2][0] = r[1][2] = r[2][1] = b
            out.append(r)
    return out


def initial_factors_for(p: Problem, ranks, seed: int):
    """Initial factors for another rank matrix on the same problem (same
    scaling rule as the workloads)."""
    obs = p.O[p.mask.astype(bool)].astype(np.float64)
    rms = float(np.sqrt(np.mean(obs * obs))) if obs.size else 1.0
    return initial_factors(np.random.default_rng(seed), p.dims, ranks, rms)


def fibre_missing_mask(dims, ratio: float, fibre_mode: int, seed: int = 0):
    """Fibre-missing sampling: whole mode-`fibre_mode` fibres are missing
    (for an image-shaped H x W x B tensor and fibre_mode = 2, every band of a
    missing pixel), chosen uniformly at a given ratio of the fibres."""
    rng = np.random.default_rng(seed)
    other = [d for m, d in enumerate(dims) if m != fibre_mode]
    keep = rng.random(other) >= ratio
    return np.repeat(np.expand_dims(keep, fibre_mode), dims[fibre_mode], axis=fibre_mode).astype(np.uint8)

