"""Seeded synthetic inputs for HWPM (shared by the tests, the oracle and the
benchmark; holds none of the matching arithmetic).

Every matrix is square, stored as CSC (col_ptr int64[n+1], row_idx int32[nnz]
strictly increasing inside each column, w float64[nnz]) with w = log|a_ij|
(the paper's "Option B" objective: the sum of logs maximises the product of
the matched magnitudes).  Each generator also returns a *planted* perfect
matching: the generators guarantee a nonzero diagonal before applying a
seeded random row permutation pi (row r -> pi[r]), so mate[j] = pi[j] is a
perfect matching contained in the pattern.  The planted matching is a
structural property of the input, not a result of the method.

Workload recipes (PCG64; structure seed 1000+k, values 2000+k, permutation
3000+k for workload k):
  random    per column d rows drawn uniformly with replacement, union the
            diagonal, duplicates removed; |a| = 10**U(-3, 3).
  stencil   27-point stencil on an nx*ny*nz grid (symmetric pattern);
            off-diagonal |a| = 10**U(-4, 0), diagonal |a| = U(1e-6, 10).
  rmat      R-MAT (a,b,c,d) = (0.57,0.19,0.19,0.05), 2**scale vertices,
            edge factor 16 samples (row = source, column = destination),
            duplicates removed, union the identity; |a| = 10**U(-3, 3).
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np

LN10 = np.log(10.0)


@dataclass
class Workload:
    name: str
    n: int
    col_ptr: np.ndarray  # int64[n+1]
    row_idx: np.ndarray  # int32[nnz]
    w: np.ndarray        # float64[nnz]
    planted: np.ndarray  # int32[n]: planted perfect matching, planted[j] = row of column j

    @property
    def nnz(self) -> int:
        return int(self.row_idx.size)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _assemble(name, n, cols, rows, w, perm_seed, is_sorted_unique=False) -> Workload:
    """Build a CSC from (cols, rows, w) triples, then permute rows by a seeded pi.

    cols/rows are int64 arrays without duplicates; the planted matching is the
    permuted diagonal."""
    pi = _rng(perm_seed).permutation(n).astype(np.int64)
    prow = pi[rows]
    key = cols * np.int64(n) + prow
    order = np.argsort(key, kind="stable")
    key = key[order]
    w = np.ascontiguousarray(w[order], dtype=np.float64)
    row_idx = (key % n).astype(np.int32)
    col = key // n
    counts = np.bincount(col, minlength=n).astype(np.int64)
    col_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=col_ptr[1:])
    planted = pi.astype(np.int32)  # column j holds the old diagonal a_jj at row pi[j]
    return Workload(name, n, col_ptr, row_idx, w, planted)


def random_matrix(n: int, d: int, seed_struct: int, seed_val: int, seed_perm: int,
                  name: str = "random") -> Workload:
    """Per column d uniform rows (with replacement) union the diagonal; log-uniform
    magnitudes in [1e-3, 1e3]."""
    rs = _rng(seed_struct)
    cols = np.repeat(np.arange(n, dtype=np.int64), d)
    rows = rs.integers(0, n, size=n * d, dtype=np.int64)
    key = np.concatenate([cols * n + rows, np.arange(n, dtype=np.int64) * (n + 1)])
    key = np.unique(key)
    cols, rows = key // n, key % n
    u = _rng(seed_val).uniform(-3.0, 3.0, size=key.size)
    w = np.log(np.power(10.0, u))
    return _assemble(name, n, cols, rows, w, seed_perm)


def stencil27(nx: int, ny: int, nz: int, seed_val: int, seed_perm: int,
              name: str = "stencil27", n_keep: int | None = None) -> Workload:
    """27-point stencil on an nx*ny*nz grid (vertex v = x + nx*(y + ny*z)).

    With n_keep < nx*ny*nz the matrix is the leading n_keep x n_keep block
    (used to size a stencil to an arbitrary n)."""
    N = nx * ny * nz
    n = N if n_keep is None else int(n_keep)
    v = np.arange(n, dtype=np.int64)
    x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
    cols_l, rows_l = [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                xx, yy, zz = x + dx, y + dy, z + dz
                ok = (xx >= 0) & (xx < nx) & (yy >= 0) & (yy < ny) & (zz >= 0) & (zz < nz)
                nb = xx + nx * (yy + ny * zz)
                ok &= nb < n
                cols_l.append(v[ok])
                rows_l.append(nb[ok])
    cols = np.concatenate(cols_l)
    rows = np.concatenate(rows_l)
    key = np.sort(cols * n + rows)
    cols, rows = key // n, key % n
    rv = _rng(seed_val)
    diag = rows == cols
    u_off = rv.uniform(-4.0, 0.0, size=key.size)
    u_diag = rv.uniform(1e-6, 10.0, size=key.size)
    w = np.where(diag, np.log(u_diag), np.log(np.power(10.0, u_off)))
    return _assemble(name, n, cols, rows, w, seed_perm)


def rmat(scale: int, edge_factor: int, seed_struct: int, seed_val: int, seed_perm: int,
         abcd=(0.57, 0.19, 0.19, 0.05), name: str = "rmat") -> Workload:
    """R-MAT graph: each sample descends `scale` quadrant levels; row = source,
    column = destination; duplicates removed; union the identity."""
    n = 1 << scale
    m = n * edge_factor
    a, b, c, _ = abcd
    rs = _rng(seed_struct)
    src = np.zeros(m, dtype=np.int64)
    dst = np.zeros(m, dtype=np.int64)
    t_ab, t_abc = np.float32(a + b), np.float32(a + b + c)
    t_a = np.float32(a)
    for _lvl in range(scale):
        u = rs.random(m, dtype=np.float32)
        src <<= 1
        dst <<= 1
        src += (u >= t_ab)
        dst += ((u >= t_a) & (u < t_ab)) | (u >= t_abc)
        del u
    key = np.concatenate([dst * n + src, np.arange(n, dtype=np.int64) * (n + 1)])
    del src, dst
    key = np.unique(key)
    cols, rows = key // n, key % n
    del key
    u = _rng(seed_val).uniform(-3.0, 3.0, size=cols.size)
    w = np.log(np.power(10.0, u))
    return _assemble(name, n, cols, rows, w, seed_perm)


# --------------------------------------------------------------------------
# The named workloads.

def workload(k: int, cache_dir: str | None = None) -> Workload:
    """Workload k:
      0  random, n = 2,000, 8 rows per column (+ diagonal)
      1  random, n = 2**20, 16 rows per column (+ diagonal), about 17.8M nonzeros
      2  27-point stencil on 100^3 (n = 10**6, 26,463,592 nonzeros)
      3  R-MAT scale 22, edge factor 16, union identity (about 69M nonzeros)
    """
    if cache_dir is None:
        cache_dir = os.environ.get("HWPM_CACHE_DIR", "/tmp/hwpm_workloads")
    path = os.path.join(cache_dir, f"workload{k}.npz") if k > 0 else None
    if path and os.path.exists(path):
        z = np.load(path)
        return Workload(str(z["name"]), int(z["n"]), z["col_ptr"], z["row_idx"], z["w"], z["planted"])
    s, v, p = 1000 + k, 2000 + k, 3000 + k
    if k == 0:
        wl = random_matrix(2000, 8, s, v, p, name="random_n2000_d8")
    elif k == 1:
        wl = random_matrix(1 << 20, 16, s, v, p, name="random_n1048576_d16")
    elif k == 2:
        wl = stencil27(100, 100, 100, v, p, name="stencil27_100cubed")
    elif k == 3:
        wl = rmat(22, 16, s, v, p, name="rmat_scale22_ef16")
    else:
        raise ValueError(f"unknown workload {k}")
    if path:
        try:
            os.makedirs(cache_dir, exist_ok=True)
            tmp = path + f".tmp{os.getpid()}.npz"
            np.savez(tmp, name=wl.name, n=wl.n, col_ptr=wl.col_ptr, row_idx=wl.row_idx,
                     w=wl.w, planted=wl.planted)
            os.replace(tmp, path)
        except OSError:
            pass
    return wl


def small_random(n: int, d: int, seed: int, integer_weights: bool = False,
                 weight_range: int = 10) -> Workload:
    """Small random case for tests: workload-0 structure at any n, optionally with
    small integer weights (exact sums, many ties)."""
    rs = _rng(seed)
    cols = np.repeat(np.arange(n, dtype=np.int64), d)
    rows = rs.integers(0, max(n, 1), size=n * d, dtype=np.int64)
    key = np.concatenate([cols * n + rows, np.arange(n, dtype=np.int64) * (n + 1)])
    key = np.unique(key)
    cols, rows = key // max(n, 1), key % max(n, 1)
    if integer_weights:
        w = rs.integers(-weight_range, weight_range + 1, size=key.size).astype(np.float64)
    else:
        w = np.log(np.power(10.0, rs.uniform(-3.0, 3.0, size=key.size)))
    return _assemble(f"small_random_n{n}_d{d}_s{seed}", n, cols, rows, w, seed + 7)


def from_dense(a: np.ndarray, planted=None, name: str = "dense") -> Workload:
    """CSC of a dense array whose NaN entries are structural zeros; w = a (used
    verbatim: hand-built cases give weights directly)."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    assert a.shape == (n, n)
    mask = ~np.isnan(a)
    col_ptr = np.zeros(n + 1, dtype=np.int64)
    col_ptr[1:] = np.cumsum(mask.sum(axis=0))
    rows, cols = [], []
    for j in range(n):
        r = np.nonzero(mask[:, j])[0]
        rows.append(r)
    row_idx = np.concatenate(rows).astype(np.int32) if n else np.zeros(0, np.int32)
    w = np.concatenate([a[mask[:, j], j] for j in range(n)]) if n else np.zeros(0)
    if planted is None:
        planted = np.arange(n, dtype=np.int32)
    return Workload(name, n, col_ptr, row_idx, np.ascontiguousarray(w, dtype=np.float64),
                    np.asarray(planted, dtype=np.int32))


def magnitudes(wl: Workload) -> np.ndarray:
    """|a_ij| of a workload whose weights are log|a_ij| (the inverse map)."""
    return np.exp(wl.w)


def with_weights(wl: Workload, w: np.ndarray, suffix: str) -> Workload:
    return Workload(wl.name + suffix, wl.n, wl.col_ptr, wl.row_idx,
                    np.ascontiguousarray(w, dtype=np.float64), wl.planted)


def option_a(wl: Workload) -> Workload:
    """The sum objective ("Option A"): weights |a_ij| instead of log|a_ij|."""
    return with_weights(wl, magnitudes(wl), "_sum")


def equilibrated(wl: Workload) -> Workload:
    """Diagonal scaling so that the largest magnitude of every row, then of
    every column, is 1 (the preprocessing the paper applies before matching);
    weights log of the scaled magnitudes, so many are exactly 0."""
    a = magnitudes(wl)
    cols = np.repeat(np.arange(wl.n), np.diff(wl.col_ptr))
    rmax = np.zeros(wl.n)
    np.maximum.at(rmax, wl.row_idx, a)
    a = a / rmax[wl.row_idx]
    cmax = np.zeros(wl.n)
    np.maximum.at(cmax, cols, a)
    a = a / cmax[cols]
    return with_weights(wl, np.log(a), "_equil")


# --------------------------------------------------------------------------
# The serving stream: many matrices of uneven size.

SERVING_SEED = 4000


def serving_matrix(index: int, seed: int = SERVING_SEED) -> Workload:
    """Matrix `index` of the serving stream: n = round(10**U(2, 5)); with
    probability 1/2 the random generator of workload 0 (8 rows per column plus
    the diagonal), else a 27-point stencil on a g x g x h box with
    g = floor(cbrt(n)), h = ceil(n / g**2), cut to its leading n x n block,
    with workload 2's value distribution.  Every draw of matrix `index` comes
    from generators seeded by (seed, index) alone, so any subset of the stream
    can be generated independently."""
    rs = np.random.Generator(np.random.PCG64([seed, index]))
    n = int(round(10.0 ** rs.uniform(2.0, 5.0)))
    s1, s2, s3 = (int(x) for x in rs.integers(0, 2 ** 62, size=3))
    if rs.random() < 0.5:
        return random_matrix(n, 8, s1, s2, s3, name=f"serve{index}_random_n{n}")
    g = max(1, int(np.floor(np.cbrt(n) + 1e-9)))
    h = -(-n // (g * g))
    return stencil27(g, g, h, s2, s3, name=f"serve{index}_stencil_n{n}", n_keep=n)


def poisson_arrivals(count: int, rate: float, seed: int = SERVING_SEED) -> np.ndarray:
    """Arrival times (seconds from the start) of a Poisson process of the given
    rate: cumulative sums of seeded exponential gaps."""
    gaps = np.random.Generator(np.random.PCG64([seed, 1 << 40])).exponential(1.0 / rate, size=count)
    return np.cumsum(gaps)
