"""Seeded synthetic elastic-net problems (inputs only).

This module produces the inputs that both the FP64 CPU oracle and the GPU
solver consume.  It holds none of the solver's arithmetic: it draws designs,
true coefficient vectors and noise, standardises the design, and applies the
lambda recipe of the simulation study (Sec. 4.1: lambda1 = alpha*c*lambda_max,
lambda2 = (1-alpha)*c*lambda_max, lambda_max = ||A^T b||_inf / alpha), which is
part of the problem statement, not of the method.

Random numbers come from numpy's Philox-4x64 counter-based generator.  Every
block of columns has its own key (seed, tag, block index), so a design is the
same whatever the thread count, and any column block can be regenerated alone.

Layout.  A (m x n) is returned column-major as an (n, m) C-contiguous array
`AT` (row j of AT is column j of A, leading dimension m).  Storage variants:
'f64', 'f32', 'bf16' (bf16 as uint16 bit patterns, round-to-nearest-even from
the f32 value).  The dequantised float64 copy of a stored design is what an
FP64 reference solve on "the stored A" uses.

Designs (Sec. 4.1 for the Gaussian one; the block-Toeplitz and SNP-like ones
stand in for the paper's collinear polynomial-expansion data and its genotype
data, which are not available):
  gauss     A_ij iid N(0,1)
  toeplitz  independent blocks of `block` columns; inside a block
            a_1 = e_1, a_j = rho*a_{j-1} + sqrt(1-rho^2)*e_j, so that
            corr(a_i, a_j) = rho^|i-j|
  snp       G_ij ~ Binomial(2, p_j), p_j ~ U[0.05, 0.5]; constant columns are
            redrawn
Every design is then standardised: each column centred to mean 0 and scaled to
unit l2 norm.
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Optional

import numpy as np

__all__ = [
    "CONFIGS", "Problem", "make_problem", "make_design", "f32_to_bf16_bits",
    "bf16_bits_to_f64", "serving_requests", "path_grid",
]

# Workload recipes.  Sizes and the lambda recipe are the benchmark workloads;
# the c_lambda / alpha / snr values follow Sec. 4.1 (snr = var(A x_t) / s^2).
CONFIGS = {
    # plain FP64 single solve, small (the one an oracle solve finishes in seconds)
    "c1": dict(m=100, n=2000, design="gauss", k=10, snr=5.0, alpha=0.5, c_lam=0.5, tol=1e-10),
    # FP64 vs FP32-stored design, block-Toeplitz correlation rho=0.6, blocks of 50
    "c2": dict(m=500, n=100_000, design="toeplitz", rho=0.6, block=50, k=20, snr=5.0,
               alpha=0.5, c_lam=0.3, tol=1e-6),
    # precision form, single large solve (4 GB in FP32)
    "c3": dict(m=1000, n=1_000_000, design="gauss", k=50, snr=3.0, alpha=0.5, c_lam=0.1, tol=1e-6),
    # warm-started path, SNP-like design, 100 log-spaced c_lambda in [0.01, 1]
    "c4": dict(m=500, n=200_000, design="snp", k=30, snr=5.0, alpha=0.7, c_lam=1.0, tol=1e-6),
}

_CHUNK = 2000  # columns per RNG block (a multiple of the Toeplitz block size 50)


def _rng(seed: int, tag: int, block: int) -> np.random.Generator:
    key = np.array([seed & 0xFFFFFFFFFFFFFFFF, ((tag & 0xFFFFFFFF) << 32) | (block & 0xFFFFFFFF)],
                   dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


_TAG_DESIGN, _TAG_SIGNAL, _TAG_NOISE, _TAG_REQ = 1, 2, 3, 4


def _design_block(design: str, m: int, c0: int, c1: int, seed: int, rho: float, block: int) -> np.ndarray:
    """Raw (unstandardised) columns c0..c1-1 as a (c1-c0, m) float64 array."""
    g = _rng(seed, _TAG_DESIGN, c0 // _CHUNK)
    nc = c1 - c0
    if design == "gauss":
        return g.standard_normal((nc, m))
    if design == "toeplitz":
        e = g.standard_normal((nc, m))
        out = np.empty_like(e)
        s = math.sqrt(1.0 - rho * rho)
        for j in range(nc):
            if (c0 + j) % block == 0:
                out[j] = e[j]
            else:
                out[j] = rho * out[j - 1] + s * e[j]
        return out
    if design == "snp":
        p = g.uniform(0.05, 0.5, size=nc)
        u = g.random((2, nc, m))
        out = (u[0] < p[:, None]).astype(np.float64) + (u[1] < p[:, None])
        # a constant column cannot be standardised: redraw it from the same stream
        for j in np.nonzero(out.max(axis=1) == out.min(axis=1))[0]:
            while True:
                u = g.random((2, m))
                col = (u[0] < p[j]).astype(np.float64) + (u[1] < p[j])
                if col.max() != col.min():
                    break
            out[j] = col
        return out
    raise ValueError(f"unknown design {design!r}")


def f32_to_bf16_bits(a32: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); returns uint16 bits."""
    u = np.ascontiguousarray(a32, dtype=np.float32).view(np.uint32)
    bias = np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))
    return ((u + bias) >> np.uint32(16)).astype(np.uint16)


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def make_design(design: str, m: int, n: int, seed: int, store: str = "f64", rho: float = 0.6,
                block: int = 50, want_f64: bool = True, threads: Optional[int] = None):
    """Standardised design.  Returns (AT_stored, AT64) where AT64 is the float64
    value of the stored design (the exact upcast), or None if not wanted.

    For store='f64' both are the same array.
    """
    if store not in ("f64", "f32", "bf16"):
        raise ValueError(store)
    sdt = {"f64": np.float64, "f32": np.float32, "bf16": np.uint16}[store]
    AT = np.empty((n, m), dtype=sdt)
    AT64 = AT if store == "f64" else (np.empty((n, m), dtype=np.float64) if want_f64 else None)

    def work(c0):
        c1 = min(n, c0 + _CHUNK)
        X = _design_block(design, m, c0, c1, seed, rho, block)
        X -= X.mean(axis=1, keepdims=True)
        X /= np.sqrt(np.einsum("ij,ij->i", X, X))[:, None]
        if store == "f64":
            AT[c0:c1] = X
        elif store == "f32":
            x32 = X.astype(np.float32)
            AT[c0:c1] = x32
            if AT64 is not None:
                AT64[c0:c1] = x32
        else:
            bits = f32_to_bf16_bits(X.astype(np.float32))
            AT[c0:c1] = bits
            if AT64 is not None:
                AT64[c0:c1] = bf16_bits_to_f64(bits)

    starts = list(range(0, n, _CHUNK))
    nt = threads or min(16, os.cpu_count() or 1)
    if nt > 1 and len(starts) > 1:
        with ThreadPoolExecutor(nt) as ex:
            list(ex.map(work, starts))
    else:
        for c0 in starts:
            work(c0)
    return AT, AT64


@dataclasses.dataclass
class Problem:
    name: str
    m: int
    n: int
    store: str
    AT: np.ndarray             # (n, m) stored design, column-major A
    AT64: Optional[np.ndarray] # (n, m) float64 value of the stored design
    b: np.ndarray
    x_true: np.ndarray
    lam1: float
    lam2: float
    alpha: float
    c_lam: float
    lam_max: float
    tol: float
    seed: int


def _signal(design: str, n: int, k: int, seed: int, block: int) -> np.ndarray:
    g = _rng(seed, _TAG_SIGNAL, 0)
    x = np.zeros(n)
    if design == "toeplitz":
        nb = n // block
        blocks = g.choice(nb, size=k, replace=False)
        idx = blocks * block + g.integers(0, block, size=k)
    else:
        idx = g.choice(n, size=k, replace=False)
    vals = g.uniform(1.0, 3.0, size=k) * np.where(g.random(k) < 0.5, -1.0, 1.0)
    x[idx] = vals
    return x


def _matvec(AT64: np.ndarray, x: np.ndarray) -> np.ndarray:
    nz = np.nonzero(x)[0]
    return AT64[nz].T @ x[nz]


def store_design(ATo: np.ndarray, store: str, want_f64: bool = True):
    """Round a float64 design to its storage type.  Returns (AT_stored, AT64)
    with AT64 the exact float64 value of the stored entries (None if not
    wanted; the original itself for 'f64')."""
    if store == "f64":
        return ATo, ATo
    a32 = ATo.astype(np.float32)
    if store == "f32":
        return a32, (a32.astype(np.float64) if want_f64 else None)
    if store == "bf16":
        bits = f32_to_bf16_bits(a32)
        del a32
        return bits, (bf16_bits_to_f64(bits) if want_f64 else None)
    raise ValueError(store)


def make_problem(cfg, seed: int = 0, store: str = "f64", want_f64: bool = True, **over) -> Problem:
    """Build one seeded problem.  `cfg` is a key of CONFIGS or a dict with the
    same fields (m, n, design, k, snr, alpha, c_lam, tol, [rho, block])."""
    if isinstance(cfg, str):
        name = cfg
        c = dict(CONFIGS[cfg])
    else:
        name = cfg.get("name", "custom")
        c = dict(cfg)
    c.update(over)
    m, n = int(c["m"]), int(c["n"])
    design = c["design"]
    rho = float(c.get("rho", 0.6))
    block = int(c.get("block", 50))
    # lambda_max and the response are defined on the float64 standardised
    # design; a reduced-precision copy is a stored variant of that design.
    ATo, _ = make_design(design, m, n, seed, "f64", rho, block)
    x_true = _signal(design, n, int(c["k"]), seed, block)
    Ax = _matvec(ATo, x_true)
    s2 = float(np.var(Ax)) / float(c["snr"])
    eps = _rng(seed, _TAG_NOISE, 0).standard_normal(m) * math.sqrt(s2)
    b = Ax + eps
    alpha, c_lam = float(c["alpha"]), float(c["c_lam"])
    lam_max = float(np.max(np.abs(ATo @ b))) / alpha
    lam1 = alpha * c_lam * lam_max
    lam2 = (1.0 - alpha) * c_lam * lam_max
    AT, AT64 = store_design(ATo, store, want_f64)
    return Problem(name, m, n, store, AT, AT64, b, x_true, lam1, lam2, alpha, c_lam, lam_max,
                   float(c.get("tol", 1e-6)), seed)


def path_grid(nlam: int = 100, lo: float = 0.01, hi: float = 1.0) -> np.ndarray:
    """Decreasing log-spaced c_lambda grid (the path workload uses 100 points, 1 -> 0.01)."""
    return np.exp(np.linspace(math.log(hi), math.log(lo), nlam))


def serving_requests(count: int, seed: int = 0, m_range=(100, 2000), n_range=(10_000, 500_000)):
    """Per-request parameters of the serving stream (no arrays): m and n
    log-uniform, Gaussian-Toeplitz (rho ~ U[0,0.8], block 50) or SNP-like with
    equal probability, alpha ~ U[0.2,0.9], c_lambda ~ U[0.05,0.8], FP32 or
    BF16 storage with equal probability, k=20, snr=5."""
    g = _rng(seed, _TAG_REQ, 0)
    out = []
    for i in range(count):
        m = int(round(math.exp(g.uniform(math.log(m_range[0]), math.log(m_range[1])))))
        n = int(round(math.exp(g.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        n = max(50, (n // 50) * 50)
        snp = g.random() < 0.5
        out.append(dict(
            name=f"req{i}", m=m, n=n, design="snp" if snp else "toeplitz",
            rho=float(g.uniform(0.0, 0.8)), block=50, k=20, snr=5.0,
            alpha=float(g.uniform(0.2, 0.9)), c_lam=float(g.uniform(0.05, 0.8)), tol=1e-6,
            store="f32" if g.random() < 0.5 else "bf16", seed=int(seed * 100003 + i + 1)))
    return out


def make_problem_device(cfg: dict, seed: int, store: str, device) -> dict:
    """The recipe of make_problem drawn on the GPU with torch's seeded
    generator (same distributions, different random stream): for workloads
    where only throughput is measured and no oracle compares the result, such
    as the serving stream, whose designs (up to 1e9 entries) would take
    minutes to draw on the host.  Returns a dict with the torch tensors AT
    (n, m; float64, float32 or bfloat16 by `store`) and b (m, float64), and
    m, n, store, lam1, lam2."""
    import torch
    m, n = int(cfg["m"]), int(cfg["n"])
    design = cfg["design"]
    rho, block = float(cfg.get("rho", 0.6)), int(cfg.get("block", 50))
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 1_000_003 + 17)
    f32 = torch.float32
    if design == "gauss":
        X = torch.randn((n, m), generator=g, device=device, dtype=f32)
    elif design == "toeplitz":
        X = torch.randn((n, m), generator=g, device=device, dtype=f32)
        nb = (n + block - 1) // block
        pad = nb * block - n
        if pad:
            X = torch.cat([X, torch.zeros((pad, m), device=device, dtype=f32)])
        Xb = X.view(nb, block, m)
        s = math.sqrt(1.0 - rho * rho)
        for j in range(1, block):  # a_j = rho a_{j-1} + sqrt(1 - rho^2) e_j inside each block
            Xb[:, j].mul_(s).add_(Xb[:, j - 1], alpha=rho)
        X = X[:n]
    elif design == "snp":
        p = 0.05 + 0.45 * torch.rand((n, 1), generator=g, device=device, dtype=f32)
        X = (torch.rand((n, m), generator=g, device=device, dtype=f32) < p).to(f32)
        X += (torch.rand((n, m), generator=g, device=device, dtype=f32) < p).to(f32)
        for _ in range(100):  # redraw constant columns
            const = (X.amax(dim=1) == X.amin(dim=1)).nonzero().flatten()
            if const.numel() == 0:
                break
            pc = p[const]
            X[const] = ((torch.rand((const.numel(), m), generator=g, device=device) < pc).to(f32)
                        + (torch.rand((const.numel(), m), generator=g, device=device) < pc).to(f32))
    else:
        raise ValueError(design)
    X -= X.mean(dim=1, keepdim=True)
    X /= torch.linalg.vector_norm(X, dim=1, keepdim=True)
    k = int(cfg["k"])
    idx = torch.randperm(n, generator=g, device=device)[:k]
    vals = (1.0 + 2.0 * torch.rand(k, generator=g, device=device, dtype=torch.float64)) * \
        torch.where(torch.rand(k, generator=g, device=device) < 0.5, -1.0, 1.0).to(torch.float64)
    Ax = (X[idx].to(torch.float64).T @ vals)
    s2 = float(Ax.var(unbiased=False)) / float(cfg["snr"])
    b = Ax + torch.randn(m, generator=g, device=device, dtype=torch.float64) * math.sqrt(s2)
    alpha, c_lam = float(cfg["alpha"]), float(cfg["c_lam"])
    lam_max = float((X @ b.to(f32)).abs().max()) / alpha
    if store == "f32":
        AT = X.contiguous()
    elif store == "bf16":
        AT = X.to(torch.bfloat16).contiguous()
    else:
        AT = X.to(torch.float64).contiguous()
    return dict(AT=AT, b=b.contiguous(), m=m, n=n, store=store, lam1=alpha * c_lam * lam_max,
                lam2=(1.0 - alpha) * c_lam * lam_max)
