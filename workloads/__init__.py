"""Seeded synthetic SPD workloads (CSR, int32 indices, fp64 values).

This module builds inputs only.  It holds none of the solver's arithmetic and is
shared, as plain data, by the CPU oracle tests and by the GPU path.

Families:
  * 2D / 3D Dirichlet Laplacians with unscaled integer stencils (4/-1 and 6/-1),
    lexicographic ordering, boundary eliminated.  The integer stencil keeps every
    entry exact in fp16 and bf16.  (The paper's Poisson experiment, section 5.2,
    uses the h-scaled 5-point stencil; the unscaled one has the same spectrum up
    to a constant factor.)
  * random-pattern SPD: a symmetric random pattern from the configuration model
    (random stub matching, self loops and duplicate pairs dropped), N(0,1)
    off-diagonal values, strict diagonal dominance (a_ii = sum_j |a_ij| + 1) and
    then a symmetric log-uniform diagonal scaling D A D, D_ii = 10**u_i,
    u_i ~ U[0, spread].  Dominance makes the unscaled matrix SPD; the congruence
    keeps it SPD and raises its condition number.
  * banded SPD: a full band of half-width w with the same value, dominance and
    scaling recipe.
  * right-hand sides b ~ U[-1, 1].

All generators take an explicit seed for numpy.random.default_rng.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    """A square CSR matrix: row_ptr int32[n+1], col int32[nnz], val float64[nnz]."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        a[rows, self.col] = self.val
        return a

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def _from_coo(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray, name: str) -> CSR:
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order].astype(np.int32)
    vals = np.ascontiguousarray(vals[order], dtype=np.float64)
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32 indices")
    return CSR(n, row_ptr.astype(np.int32), np.ascontiguousarray(cols), vals, name)


def laplacian_2d(N: int) -> CSR:
    """5-point Laplacian on an N x N interior grid: 4 on the diagonal, -1 off it."""
    n = N * N
    idx = np.arange(n, dtype=np.int64)
    x = idx % N
    y = idx // N
    rows = [idx]
    cols = [idx]
    vals = [np.full(n, 4.0)]
    for cond, off in ((y > 0, -N), (x > 0, -1), (x < N - 1, 1), (y < N - 1, N)):
        r = idx[cond]
        rows.append(r)
        cols.append(r + off)
        vals.append(np.full(r.size, -1.0))
    return _from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals),
                     f"lap2d_{N}")


def laplacian_3d(N: int) -> CSR:
    """7-point Laplacian on an N^3 interior grid: 6 on the diagonal, -1 off it."""
    n = N * N * N
    idx = np.arange(n, dtype=np.int64)
    x = idx % N
    y = (idx // N) % N
    z = idx // (N * N)
    rows = [idx]
    cols = [idx]
    vals = [np.full(n, 6.0)]
    for cond, off in ((z > 0, -N * N), (y > 0, -N), (x > 0, -1),
                      (x < N - 1, 1), (y < N - 1, N), (z < N - 1, N * N)):
        r = idx[cond]
        rows.append(r)
        cols.append(r + off)
        vals.append(np.full(r.size, -1.0))
    return _from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals),
                     f"lap3d_{N}")


def laplacian_nnz(N: int, d: int) -> int:
    """Closed form nnz of the d-dimensional Laplacian on N^d points."""
    n = N ** d
    return (2 * d + 1) * n - 2 * d * N ** (d - 1)


def laplacian_eigs(N: int, d: int) -> np.ndarray:
    """Closed-form spectrum of the unscaled d-dimensional Dirichlet Laplacian."""
    j = np.arange(1, N + 1)
    lam1 = 4.0 * np.sin(j * np.pi / (2.0 * (N + 1))) ** 2
    grids = np.meshgrid(*([lam1] * d), indexing="ij")
    return np.sort(sum(grids).ravel())


def _dominant_scaled(n: int, lo: np.ndarray, hi: np.ndarray, offv: np.ndarray,
                     spread: float, rng: np.random.Generator, name: str) -> CSR:
    rows = np.concatenate([lo, hi])
    cols = np.concatenate([hi, lo])
    v = np.concatenate([offv, offv])
    absum = np.bincount(rows, weights=np.abs(v), minlength=n)
    diag_idx = np.arange(n, dtype=np.int64)
    rows = np.concatenate([rows, diag_idx])
    cols = np.concatenate([cols, diag_idx])
    v = np.concatenate([v, absum + 1.0])
    if spread > 0:
        d = 10.0 ** rng.uniform(0.0, spread, n)
        v = v * (d[rows] * d[cols])      # d_i d_j == d_j d_i bitwise: exact symmetry
    return _from_coo(n, rows, cols, v, name)


def random_spd(n: int, seed: int, spread: float, tmin: int = 8, tmax: int = 26) -> CSR:
    """Random-pattern SPD matrix, configuration model with t_i ~ U{tmin..tmax} stubs.

    Rows hold 1 + (at most t_i) entries, so tmin=8, tmax=26 gives 9..27 nnz/row.
    """
    rng = np.random.default_rng(seed)
    t = rng.integers(tmin, tmax + 1, size=n)
    stubs = np.repeat(np.arange(n, dtype=np.int64), t)
    rng.shuffle(stubs)
    if stubs.size % 2:
        stubs = stubs[:-1]
    i = stubs[0::2]
    j = stubs[1::2]
    keep = i != j
    i, j = i[keep], j[keep]
    key = np.unique(np.minimum(i, j) * n + np.maximum(i, j))
    lo = key // n
    hi = key % n
    offv = rng.standard_normal(key.size)
    return _dominant_scaled(n, lo, hi, offv, spread, rng, f"rspd_{n}_{seed}")


def banded_spd(n: int, w: int, seed: int, spread: float) -> CSR:
    """Full band of half-width w (bandwidth 2w+1), same recipe as random_spd."""
    rng = np.random.default_rng(seed)
    los, his = [], []
    for d in range(1, w + 1):
        r = np.arange(n - d, dtype=np.int64)
        los.append(r)
        his.append(r + d)
    lo = np.concatenate(los) if los else np.zeros(0, np.int64)
    hi = np.concatenate(his) if his else np.zeros(0, np.int64)
    offv = rng.standard_normal(lo.size)
    return _dominant_scaled(n, lo, hi, offv, spread, rng, f"band_{n}_{w}_{seed}")


def rhs(n: int, seed: int) -> np.ndarray:
    """b ~ U[-1, 1]."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


# Diagonal-scaling spread that puts the condition number of random_spd near a
# target.  D A0 D with D_ii = 10**u, u ~ U[0, s], stretches the spectrum of the
# dominant matrix A0 (kappa0 ~ 1e1) by about 10**(2 s) at the extremes; the
# factor 0.5 below is that relation, and the measured condition number is always
# reported beside any result.
def spread_for_kappa(kappa: float, kappa0: float = 10.0) -> float:
    return max(0.0, 0.5 * (math.log10(kappa) - math.log10(kappa0)))


def family_system(seed: int, n_lo: float = 1e4, n_hi: float = 5e5,
                  kappa_lo: float = 1e2, kappa_hi: float = 1e8) -> CSR:
    """Training / held-out family: seed mod 3 picks 2D Laplacian, 3D Laplacian or random SPD."""
    rng = np.random.default_rng(seed)
    fam = seed % 3
    if fam == 0:
        N = int(round(math.sqrt(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))))))
        return laplacian_2d(max(N, 2))
    if fam == 1:
        N = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))) ** (1.0 / 3.0)))
        return laplacian_3d(max(N, 2))
    n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
    kappa = math.exp(rng.uniform(math.log(kappa_lo), math.log(kappa_hi)))
    return random_spd(n, seed, spread_for_kappa(kappa))


def batch_system(seed: int, n_lo: float = 1e3, n_hi: float = 2e5,
                 kappa_lo: float = 1e2, kappa_hi: float = 1e4) -> CSR:
    """Batched-solve family: even seed banded (w ~ U{1..15}), odd seed random pattern (5..27 nnz/row)."""
    rng = np.random.default_rng(seed)
    n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
    kappa = math.exp(rng.uniform(math.log(kappa_lo), math.log(kappa_hi)))
    if seed % 2 == 0:
        w = int(rng.integers(1, 16))
        return banded_spd(n, w, seed, spread_for_kappa(kappa))
    return random_spd(n, seed, spread_for_kappa(kappa), tmin=4, tmax=26)


# ---------------------------------------------------------------------------
# The paper's own synthetic families (section 5): inputs for the replication
# mode, not for the benchmark.
# ---------------------------------------------------------------------------
def bbt_system(seed: int, n: int = 5000, density_reading: str = "pairs", ood: bool = False) -> CSR:
    """A = B B^T + beta I (section 5.1): B sparse n x n with N(0, 1) values at
    index pairs drawn uniformly with replacement, beta ~ U(1e-4, 1e-2).

    The paper gives two sizes for B's pattern: about 1 % of its elements
    nonzero, and 5,000 index pairs.  density_reading "pairs" takes n pairs (5,000
    at n = 5,000), "percent" takes 1 % of n^2; ood scales the count by
    U(0.8, 1.2) (the out-of-distribution sets).  Pairs that repeat add up."""
    rng = np.random.default_rng(seed)
    m = n if density_reading == "pairs" else int(round(0.01 * n * n))
    if ood:
        m = int(round(m * rng.uniform(0.8, 1.2)))
    bi = rng.integers(0, n, m)
    bj = rng.integers(0, n, m)
    bv = rng.standard_normal(m)
    beta = rng.uniform(1e-4, 1e-2)
    # (B B^T)_{ik} = sum_j B_ij B_kj: pair every entry with every entry of the same column j
    order = np.argsort(bj, kind="stable")
    bi, bj, bv = bi[order], bj[order], bv[order]
    starts = np.flatnonzero(np.r_[True, bj[1:] != bj[:-1]])
    ends = np.r_[starts[1:], m]
    rows, cols, vals = [], [], []
    for s, e in zip(starts, ends):
        ii = bi[s:e]
        vv = bv[s:e]
        rows.append(np.repeat(ii, e - s))
        cols.append(np.tile(ii, e - s))
        vals.append(np.outer(vv, vv).ravel())
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(np.full(n, beta))
    r = np.concatenate(rows).astype(np.int64)
    c = np.concatenate(cols).astype(np.int64)
    v = np.concatenate(vals)
    # sum duplicate (i, k) entries in a fixed order (sorted keys), so the
    # matrix is exactly symmetric
    key = r * n + c
    uk, inv = np.unique(key, return_inverse=True)
    acc = np.zeros(uk.size)
    np.add.at(acc, inv, v)
    return _from_coo(n, (uk // n).astype(np.int64), (uk % n).astype(np.int64), acc,
                     f"bbt_{n}_{density_reading}_{seed}")


def poisson_subdomain(seed: int, N: int = 80):
    """The 2D Poisson family of section 5.2: -lap u = f on a random subdomain
    [ax, bx] x [ay, by] of [0, 2]^2 (ax ~ U(0, 1.9), bx = ax + U(0.1, 2 - ax),
    likewise in y), N x N interior points, h = (b - a) / (N + 1) per direction,
    the 5-point stencil (2/hx^2 + 2/hy^2 on the diagonal), Dirichlet data g
    constant, linear or sinusoidal per edge and a source f zero, sinusoidal or
    polynomial, each with equal probability.  Returns (A, b): b holds f and the
    boundary values moved to the right-hand side."""
    rng = np.random.default_rng(seed)
    ax = rng.uniform(0.0, 1.9)
    bx = ax + rng.uniform(0.1, 2.0 - ax)
    ay = rng.uniform(0.0, 1.9)
    by = ay + rng.uniform(0.1, 2.0 - ay)
    hx, hy = (bx - ax) / (N + 1), (by - ay) / (N + 1)
    cx, cy = 1.0 / (hx * hx), 1.0 / (hy * hy)
    n = N * N
    idx = np.arange(n, dtype=np.int64)
    ix, iy = idx % N, idx // N
    rows, cols, vals = [idx], [idx], [np.full(n, 2.0 * cx + 2.0 * cy)]
    for cond, off, w in ((iy > 0, -N, cy), (ix > 0, -1, cx), (ix < N - 1, 1, cx), (iy < N - 1, N, cy)):
        r = idx[cond]
        rows.append(r)
        cols.append(r + off)
        vals.append(np.full(r.size, -w))
    A = _from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals),
                  f"poisson_{N}_{seed}")

    def edge_fn():
        kind = rng.integers(0, 3)
        p, q = rng.uniform(-1.0, 1.0, 2)
        if kind == 0:
            return lambda t: np.full_like(t, p)
        if kind == 1:
            return lambda t: p + q * t
        w = rng.uniform(0.5, 3.0)
        return lambda t: p * np.sin(w * np.pi * t)

    g_left, g_right, g_bottom, g_top = edge_fn(), edge_fn(), edge_fn(), edge_fn()
    kind = rng.integers(0, 3)
    c1, c2, c3 = rng.uniform(-1.0, 1.0, 3)
    xs = ax + (ix + 1) * hx
    ys = ay + (iy + 1) * hy
    if kind == 0:
        f = np.zeros(n)
    elif kind == 1:
        f = c1 * np.sin(np.pi * xs) * np.sin(np.pi * ys)
    else:
        f = c1 + c2 * xs * ys + c3 * xs * xs
    b = f.copy()
    b[ix == 0] += cx * g_left(ys[ix == 0])
    b[ix == N - 1] += cx * g_right(ys[ix == N - 1])
    b[iy == 0] += cy * g_bottom(xs[iy == 0])
    b[iy == N - 1] += cy * g_top(xs[iy == N - 1])
    return A, b
