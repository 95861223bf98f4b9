"""Seeded synthetic workloads shaped like the paper's evaluation data (Section 6, Table 1).

The paper evaluates on public embedding / descriptor sets that are not shipped here, so every input
is drawn from a Gaussian mixture whose principal-component spectrum decays like the "long-tailed"
variance profile the paper observes after PCA (Section 3.2).  This module holds only the generator:
none of the search method's arithmetic lives here, and both the CPU oracle tests and the GPU path
draw their inputs from it.

Construction (all in float64, stored as float32):
  * a Haar-random orthonormal basis U (D x D) from the QR of a Gaussian matrix, with the usual
    sign fix on diag(R);
  * a spectrum lambda_1 >= ... >= lambda_D with trace D;
  * the cluster structure lives in the leading ``cluster_dims`` axes: there a share ``between`` of
    each axis' variance lambda_i comes from the component centres and the rest from the spread inside
    a component; the remaining axes carry within-component spread only;
  * component centres mu_c = U_h diag(sqrt(between * lambda_h)) z_c, z_c ~ N(0, I);
  * points x = mu_c + U diag(sqrt(w)) z, with w_i = (1 - between) lambda_i on the leading axes and
    w_i = lambda_i elsewhere, and the component c drawn from the mixture weights.
The expected covariance of the mixture is U diag(lambda) U^T, so the PCA spectrum of the data follows
lambda up to sampling noise, and the trailing axes are centred and decorrelated, which is the data
model the paper's residual bound assumes (Section 4.2, Eq 6).

Seeds: the mixture itself (basis, spectrum scale, centres, weights) comes from ``model_seed``; every
sample of points draws from its own ``draw_seed`` so base vectors and queries are independent draws of
the same distribution.
"""
from __future__ import annotations

import dataclasses
import hashlib
import os
from typing import Optional

import numpy as np

__all__ = [
    "MixtureSpec",
    "spectrum",
    "variance_fraction",
    "build_model",
    "sample",
    "workload",
    "WORKLOADS",
]


@dataclasses.dataclass(frozen=True)
class MixtureSpec:
    D: int
    n_comp: int
    decay: float                # lambda_i proportional to i^-decay (power-law spectrum)
    between: float = 0.75       # share of a leading axis' variance that separates the components
    cluster_dims: int = 16      # number of leading axes that carry the cluster structure
    weights: str = "uniform"    # "uniform" or "zipf"
    zipf_s: float = 1.1
    spectrum: str = "power"     # "power" or "head_tail" (power-law head holding head_frac of the variance)
    head_dims: int = 200
    head_frac: float = 0.9
    normalize: bool = False     # L2-normalise every sample (embedding-like data)
    model_seed: int = 0


def spectrum(spec: MixtureSpec) -> np.ndarray:
    """Per-axis variances lambda_i (descending, trace D) of the within-component Gaussian."""
    D = spec.D
    i = np.arange(1, D + 1, dtype=np.float64)
    if spec.spectrum == "power":
        lam = i ** (-spec.decay)
    elif spec.spectrum == "head_tail":
        h = min(spec.head_dims, D)
        head = i[:h] ** (-spec.decay)
        head = head / head.sum() * spec.head_frac
        tail = np.full(D - h, (1.0 - spec.head_frac) / max(D - h, 1))
        lam = np.concatenate([head, tail])
    else:
        raise ValueError(f"unknown spectrum {spec.spectrum!r}")
    return lam * (D / lam.sum())


def variance_fraction(spec: MixtureSpec, d: int) -> float:
    """Closed-form share of the total variance held by the leading d axes of the construction."""
    lam = spectrum(spec)
    return float(lam[:d].sum() / lam.sum())


def _haar(D: int, rng: np.random.Generator) -> np.ndarray:
    g = rng.standard_normal((D, D))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


@dataclasses.dataclass
class MixtureModel:
    spec: MixtureSpec
    basis: np.ndarray      # U, D x D float64 (columns = axes)
    lam: np.ndarray        # lambda, D float64
    centres: np.ndarray    # n_comp x D float64
    weights: np.ndarray    # n_comp float64, sums to 1
    mix: np.ndarray        # U diag(sqrt(w)), D x D float32 (row-vector form: x = z @ mix.T)


def build_model(spec: MixtureSpec) -> MixtureModel:
    rng = np.random.default_rng([spec.model_seed, 0x5EED])
    U = _haar(spec.D, rng)
    lam = spectrum(spec)
    h = min(spec.cluster_dims, spec.D) if spec.n_comp > 1 else 0
    w = lam.copy()
    w[:h] *= 1.0 - spec.between
    A = U * np.sqrt(w)[None, :]
    zc = rng.standard_normal((spec.n_comp, h))
    centres = (zc * np.sqrt(spec.between * lam[:h])[None, :]) @ U[:, :h].T
    if spec.weights == "uniform":
        wts = np.full(spec.n_comp, 1.0 / spec.n_comp)
    elif spec.weights == "zipf":
        ranks = np.arange(1, spec.n_comp + 1, dtype=np.float64)
        wt = ranks ** (-spec.zipf_s)
        wt = wt[rng.permutation(spec.n_comp)]
        wts = wt / wt.sum()
    else:
        raise ValueError(f"unknown weights {spec.weights!r}")
    return MixtureModel(spec, U, lam, centres, wts, A.astype(np.float32))


def sample(model: MixtureModel, n: int, draw_seed: int, chunk: int = 65536) -> np.ndarray:
    """n points of the mixture as a C-contiguous float32 array (n x D).

    Rows are drawn in fixed chunks of 65,536, each from its own seeded stream, so the result does
    not depend on how many threads produce it."""
    spec = model.spec
    chunk = 65536
    out = np.empty((n, spec.D), dtype=np.float32)
    centres32 = model.centres.astype(np.float32)
    mixT = np.ascontiguousarray(model.mix.T)

    def one(ci: int):
        s = ci * chunk
        e = min(n, s + chunk)
        rng = np.random.default_rng([spec.model_seed, 0xD7A1, draw_seed, ci])
        comp = rng.choice(spec.n_comp, size=e - s, p=model.weights)
        z = rng.standard_normal((e - s, spec.D), dtype=np.float32)
        blk = z @ mixT
        blk += centres32[comp]
        if spec.normalize:
            b64 = blk.astype(np.float64)
            nrm = np.sqrt(np.einsum("ij,ij->i", b64, b64))
            nrm[nrm == 0] = 1.0
            blk = (b64 / nrm[:, None]).astype(np.float32)
        out[s:e] = blk

    nchunks = (n + chunk - 1) // chunk
    if nchunks <= 1:
        for ci in range(nchunks):
            one(ci)
    else:
        import concurrent.futures as cf
        workers = max(1, min(16, os.cpu_count() or 1))
        with cf.ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one, range(nchunks)))
    return out


# Workloads: sizes, spectra and mixture structure of the shapes the search path is exercised on.
#   small    : 20k x 128, 64 uniform components, lambda_i ~ i^-1, clusters in the top 16 axes
#   gist1m   : 1M x 960 (GIST-shaped), 1,024 Zipf(1.1)-weighted components, lambda_i ~ i^-1.2,
#              clusters in the top 64 axes
#   deep10m  : 10M x 128, 256 components, lambda_i ~ i^-0.8, clusters in the top 32 axes
#   openai2m : 2M x 1536 unit vectors, one Gaussian with 90% of the variance in the top 200 axes
WORKLOADS = {
    "small": dict(spec=MixtureSpec(D=128, n_comp=64, decay=1.0, model_seed=1001), N=20_000, nq=100),
    "gist1m": dict(spec=MixtureSpec(D=960, n_comp=1024, decay=1.2, weights="zipf", zipf_s=1.1,
                                    cluster_dims=64, model_seed=1002), N=1_000_000, nq=10_000),
    "deep10m": dict(spec=MixtureSpec(D=128, n_comp=256, decay=0.8, cluster_dims=32,
                                     model_seed=1003), N=10_000_000,
                    nq=10_000),
    "openai2m": dict(spec=MixtureSpec(D=1536, n_comp=1, decay=1.0, spectrum="head_tail",
                                      normalize=True, model_seed=1004), N=2_000_000, nq=20_000),
}


def _cache_dir() -> Optional[str]:
    d = os.environ.get("MRQ_DATA_CACHE")
    if d is None:
        d = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), ".cache")
    try:
        os.makedirs(d, exist_ok=True)
    except OSError:
        return None
    return d


def workload(name: str, N: Optional[int] = None, nq: Optional[int] = None, cache: bool = True):
    """(base, queries, spec) for a named workload; N / nq override the default sizes.

    Base vectors use draw seed 1, queries draw seed 2 of the same mixture.  Arrays of more than a few
    MB are cached on disk (with a SHA-256 of their bytes checked on reload) so repeated runs do not
    pay for generation again.
    """
    w = WORKLOADS[name]
    spec = w["spec"]
    N = w["N"] if N is None else N
    nq = w["nq"] if nq is None else nq
    model = build_model(spec)
    cdir = _cache_dir() if cache else None

    def get(tag, n, seed):
        path = None
        if cdir is not None and n * spec.D * 4 > (8 << 20):
            path = os.path.join(cdir, f"{name}_{tag}_{n}_{spec.model_seed}.npy")
            if os.path.exists(path) and os.path.exists(path + ".sha256"):
                arr = np.load(path, mmap_mode=None)
                want = open(path + ".sha256").read().strip()
                if hashlib.sha256(arr.tobytes()).hexdigest() == want and arr.shape == (n, spec.D):
                    return arr
        arr = sample(model, n, seed)
        if path is not None:
            np.save(path, arr)
            with open(path + ".sha256", "w") as f:
                f.write(hashlib.sha256(arr.tobytes()).hexdigest())
        return arr

    return get("base", N, 1), get("query", nq, 2), spec
