"""Seeded synthetic MIP instances in the shapes of the paper's workloads.

This module only draws instances: it builds the constraint matrix (CSR and CSC
of the same matrix), row senses, right-hand sides from a hidden feasible point,
variable bounds, integrality flags and objective. It holds none of the tabu
search arithmetic, so both the CPU oracle and the HIP library consume its
output without sharing any computation.

Problem form (paper section 3.1, problem statement):
    min c^T x  s.t.  rows with sense 'L' (<=), 'G' (>=), 'E' (=),
                     l <= x <= u,  x_j integer for is_int[j] = 1.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) and is fully
deterministic for a given seed and size.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SENSE_L = ord("L")
SENSE_G = ord("G")
SENSE_E = ord("E")


@dataclass
class MIP:
    """A MIP in original (un-normalised) form, host arrays only."""

    n: int
    m: int
    csr_row_ptr: np.ndarray  # int64, m+1
    csr_col: np.ndarray  # int32, nnz
    csr_val: np.ndarray  # float64, nnz
    csc_col_ptr: np.ndarray  # int64, n+1
    csc_row: np.ndarray  # int32, nnz
    csc_val: np.ndarray  # float64, nnz
    sense: np.ndarray  # uint8, m  ('L','G','E')
    rhs: np.ndarray  # float64, m
    lb: np.ndarray  # float64, n  (may be -inf)
    ub: np.ndarray  # float64, n  (may be +inf)
    is_int: np.ndarray  # uint8, n
    obj: np.ndarray  # float64, n
    name: str = ""
    hidden_x: np.ndarray | None = field(default=None, repr=False)

    @property
    def nnz(self) -> int:
        return int(self.csr_col.shape[0])

    @property
    def nnz_obj(self) -> int:
        return int(np.count_nonzero(self.obj))

    def counts(self) -> dict:
        s = self.sense
        return {
            "n": self.n,
            "m": self.m,
            "nnz": self.nnz,
            "nnz_obj": self.nnz_obj,
            "rows_L": int(np.count_nonzero(s == SENSE_L)),
            "rows_G": int(np.count_nonzero(s == SENSE_G)),
            "rows_E": int(np.count_nonzero(s == SENSE_E)),
        }


# ---------------------------------------------------------------------------
# layout helpers (pure index bookkeeping)
# ---------------------------------------------------------------------------

def _ptr_from_counts(counts: np.ndarray) -> np.ndarray:
    ptr = np.zeros(counts.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    return ptr


def coo_to_csr_csc(n: int, m: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray):
    """Build CSR (rows sorted, columns ascending within a row) and CSC
    (columns sorted, rows ascending within a column) from COO triplets with no
    duplicate (row, col) pairs."""
    rows = rows.astype(np.int64, copy=False)
    cols = cols.astype(np.int64, copy=False)
    key = rows * max(n, 1) + cols
    o = np.argsort(key, kind="stable")
    csr_col = cols[o].astype(np.int32)
    csr_val = vals[o].astype(np.float64)
    csr_ptr = _ptr_from_counts(np.bincount(rows, minlength=m)[:m])
    key = cols * max(m, 1) + rows
    o = np.argsort(key, kind="stable")
    csc_row = rows[o].astype(np.int32)
    csc_val = vals[o].astype(np.float64)
    csc_ptr = _ptr_from_counts(np.bincount(cols, minlength=n)[:n])
    return csr_ptr, csr_col, csr_val, csc_ptr, csc_row, csc_val


def _distinct_per_group(rng: np.random.Generator, group_sizes: np.ndarray, universe: int) -> tuple:
    """For group g draw group_sizes[g] distinct values in [0, universe),
    uniformly without replacement. Returns (group_id, value) arrays sorted by
    (group, value). Duplicates from a with-replacement draw are redrawn until
    none remain, which keeps the draw uniform over distinct subsets."""
    group_sizes = np.minimum(group_sizes.astype(np.int64), universe)
    gid = np.repeat(np.arange(group_sizes.shape[0], dtype=np.int64), group_sizes)
    val = rng.integers(0, universe, size=gid.shape[0], dtype=np.int64)
    while True:
        key = gid * universe + val
        o = np.argsort(key, kind="stable")
        key = key[o]
        gid = gid[o]
        val = val[o]
        dup = np.zeros(key.shape[0], dtype=bool)
        dup[1:] = key[1:] == key[:-1]
        nd = int(np.count_nonzero(dup))
        if nd == 0:
            return gid, val
        val[dup] = rng.integers(0, universe, size=nd, dtype=np.int64)


def _signed_nonzero_ints(rng: np.random.Generator, size: int, amax: int) -> np.ndarray:
    """Uniform over {-amax..amax} minus {0}."""
    mag = rng.integers(1, amax + 1, size=size)
    sgn = rng.integers(0, 2, size=size) * 2 - 1
    return (mag * sgn).astype(np.float64)


def _row_activity(csr_ptr, csr_col, csr_val, x) -> np.ndarray:
    prod = csr_val * x[csr_col]
    m = csr_ptr.shape[0] - 1
    rows = np.repeat(np.arange(m, dtype=np.int64), np.diff(csr_ptr))
    return np.bincount(rows, weights=prod, minlength=m)[:m]


def _finish(n, m, rows, cols, vals, sense, rhs_fn, lb, ub, is_int, obj, hidden, name):
    csr_ptr, csr_col, csr_val, csc_ptr, csc_row, csc_val = coo_to_csr_csc(n, m, rows, cols, vals)
    act = _row_activity(csr_ptr, csr_col, csr_val, hidden)
    rhs = rhs_fn(act)
    return MIP(n=n, m=m, csr_row_ptr=csr_ptr, csr_col=csr_col, csr_val=csr_val,
               csc_col_ptr=csc_ptr, csc_row=csc_row, csc_val=csc_val,
               sense=sense.astype(np.uint8), rhs=rhs.astype(np.float64),
               lb=lb.astype(np.float64), ub=ub.astype(np.float64),
               is_int=is_int.astype(np.uint8), obj=obj.astype(np.float64),
               name=name, hidden_x=hidden)


# ---------------------------------------------------------------------------
# workload 1: tiny all-binary knapsack-style MIP
# ---------------------------------------------------------------------------

def tiny_binary(seed: int = 0, n: int = 200, m: int = 100, row_nnz: int = 10) -> MIP:
    """n binary variables, m '<=' rows of row_nnz distinct random columns,
    coefficients U{1..9}, rhs = floor(row sum / 2), objective U{-10..10}."""
    rng = np.random.default_rng(seed)
    cols = np.argsort(rng.random((m, n)), axis=1)[:, :row_nnz]
    cols = np.sort(cols, axis=1).reshape(-1)
    rows = np.repeat(np.arange(m), row_nnz)
    vals = rng.integers(1, 10, size=m * row_nnz).astype(np.float64)
    obj = rng.integers(-10, 11, size=n).astype(np.float64)
    rowsum = np.bincount(rows, weights=vals, minlength=m)
    sense = np.full(m, SENSE_L, dtype=np.uint8)
    lb = np.zeros(n)
    ub = np.ones(n)
    is_int = np.ones(n, dtype=np.uint8)
    hidden = np.zeros(n)
    return _finish(n, m, rows, cols, vals, sense, lambda act: np.floor(0.5 * rowsum),
                   lb, ub, is_int, obj, hidden, f"tiny_binary(seed={seed})")


# ---------------------------------------------------------------------------
# workload 2: general MIP (binary / bounded integer / continuous)
# ---------------------------------------------------------------------------

def general(seed: int = 0, n: int = 100_000, m: int = 50_000, mean_row_nnz: float = 8.0,
            sigma: float = 1.0, max_row_nnz: int = 2000, amax: int = 20) -> MIP:
    """60 % binary, 30 % integer in [0,100], 10 % continuous in [0,1000]
    (types by random permutation); 40 % '<=', 40 % '>=', 20 % '=' rows in
    random order; row lengths clamp(round(LogNormal(ln(mean)-sigma^2/2, sigma)),
    1, max_row_nnz); columns per row uniform without replacement; coefficients
    U{-amax..amax}\\{0}; rhs from a hidden feasible point, slack U[0,5]
    (real) on inequalities, exact on equalities; objective U{-10..10}."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    nb = int(round(0.6 * n))
    ni = int(round(0.3 * n))
    vtype = np.empty(n, dtype=np.int8)
    vtype[perm[:nb]] = 0
    vtype[perm[nb:nb + ni]] = 1
    vtype[perm[nb + ni:]] = 2
    lb = np.zeros(n)
    ub = np.where(vtype == 0, 1.0, np.where(vtype == 1, 100.0, 1000.0))
    is_int = (vtype != 2).astype(np.uint8)

    rperm = rng.permutation(m)
    nl = int(round(0.4 * m))
    ng = int(round(0.4 * m))
    sense = np.empty(m, dtype=np.uint8)
    sense[rperm[:nl]] = SENSE_L
    sense[rperm[nl:nl + ng]] = SENSE_G
    sense[rperm[nl + ng:]] = SENSE_E

    mu = math.log(mean_row_nnz) - 0.5 * sigma * sigma
    lens = np.clip(np.rint(rng.lognormal(mu, sigma, size=m)), 1, min(max_row_nnz, n)).astype(np.int64)
    rows, cols = _distinct_per_group(rng, lens, n)
    vals = _signed_nonzero_ints(rng, rows.shape[0], amax)

    hidden = np.where(vtype == 0, rng.integers(0, 2, size=n).astype(np.float64),
                      np.where(vtype == 1, rng.integers(0, 101, size=n).astype(np.float64),
                               rng.uniform(0.0, 1000.0, size=n)))
    slack = rng.uniform(0.0, 5.0, size=m)
    obj = rng.integers(-10, 11, size=n).astype(np.float64)

    def rhs_fn(act):
        return np.where(sense == SENSE_L, act + slack, np.where(sense == SENSE_G, act - slack, act))

    return _finish(n, m, rows, cols, vals, sense, rhs_fn, lb, ub, is_int, obj, hidden,
                   f"general(seed={seed},n={n},m={m})")


# ---------------------------------------------------------------------------
# workload 3: large power-law MIP (all integer)
# ---------------------------------------------------------------------------

def zipf_degrees(n: int, nnz: int, exponent: float = 1.1, cap: int = 100_000) -> np.ndarray:
    """Rank degrees d_k = clamp(round(C k^-exponent), 1, cap), k = 1..n, with
    C chosen by bisection so that sum(d) is as close to nnz as possible."""
    k = np.arange(1, n + 1, dtype=np.float64)
    base = k ** (-exponent)

    def total(c):
        return int(np.clip(np.rint(c * base), 1, cap).sum())

    lo, hi = 0.0, float(nnz) * 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if total(mid) < nnz:
            lo = mid
        else:
            hi = mid
    c = hi if abs(total(hi) - nnz) <= abs(total(lo) - nnz) else lo
    return np.clip(np.rint(c * base), 1, cap).astype(np.int64)


def powerlaw(seed: int = 0, n: int = 2_000_000, m: int = 1_000_000, nnz: int = 20_000_000,
             cap: int = 100_000, exponent: float = 1.1, umax: int = 50, amax: int = 9,
             frac_eq: float = 0.2) -> MIP:
    """All variables integer in [0, umax]; (1-frac_eq) '<=' and frac_eq '='
    rows in random order; column degrees rank-Zipf(exponent) capped at cap and
    assigned to variables by a random permutation; each column's rows uniform
    without replacement; coefficients U{-amax..amax}\\{0}; hidden point
    U{0..umax}; rhs = activity + U{0..5} on '<=' rows, exact on '=' rows;
    objective U{-10..10}."""
    rng = np.random.default_rng(seed)
    cap = min(cap, m)
    deg_rank = zipf_degrees(n, nnz, exponent, cap)
    var_of_rank = rng.permutation(n)
    deg = np.empty(n, dtype=np.int64)
    deg[var_of_rank] = deg_rank
    cols, rows = _distinct_per_group(rng, deg, m)
    vals = _signed_nonzero_ints(rng, rows.shape[0], amax)

    rperm = rng.permutation(m)
    ne = int(round(frac_eq * m))
    sense = np.full(m, SENSE_L, dtype=np.uint8)
    sense[rperm[:ne]] = SENSE_E

    lb = np.zeros(n)
    ub = np.full(n, float(umax))
    is_int = np.ones(n, dtype=np.uint8)
    hidden = rng.integers(0, umax + 1, size=n).astype(np.float64)
    slack = rng.integers(0, 6, size=m).astype(np.float64)
    obj = rng.integers(-10, 11, size=n).astype(np.float64)

    def rhs_fn(act):
        return np.where(sense == SENSE_L, act + slack, act)

    return _finish(n, m, rows, cols, vals, sense, rhs_fn, lb, ub, is_int, obj, hidden,
                   f"powerlaw(seed={seed},n={n},m={m},nnz={nnz})")


# ---------------------------------------------------------------------------
# workload 4: pool of general instances of uneven size for batched walks
# ---------------------------------------------------------------------------

def batch_pool_sizes(total_nnz: int = 20_000_000, nmin: int = 10_000, nmax: int = 500_000,
                     base_seed: int = 1000) -> list:
    """(seed, n) for pool instances: n log-uniform in [nmin, nmax] drawn from
    default_rng(seed), seed = base_seed + p, until the expected constraint
    nonzeros (8 per row, n/2 rows) reach total_nnz."""
    out = []
    acc = 0
    p = 0
    while acc < total_nnz:
        s = base_seed + p
        r = np.random.default_rng(s)
        npv = int(round(math.exp(r.uniform(math.log(nmin), math.log(nmax)))))
        out.append((s, npv))
        acc += 4 * npv
        p += 1
    return out


def batch_pool(total_nnz: int = 20_000_000, nmin: int = 10_000, nmax: int = 500_000,
               base_seed: int = 1000) -> list:
    return [general(seed=s, n=npv, m=npv // 2)
            for s, npv in batch_pool_sizes(total_nnz, nmin, nmax, base_seed)]


# ---------------------------------------------------------------------------
# small mixed instances for parity and edge-case tests
# ---------------------------------------------------------------------------

def random_mixed(seed: int, n: int = 40, m: int = 30, max_row_nnz: int = 6, amax: int = 5,
                 frac_bin: float = 0.3, frac_int: float = 0.4, int_width: int = 12,
                 cont_ub: float = 20.0, inf_bounds: float = 0.0, integer_data: bool = True,
                 long_cols: int = 0, long_deg: int = 0) -> MIP:
    """Small instance mixing binary, bounded integer and continuous variables,
    all three row senses, optional infinite bounds and optional long columns.
    With integer_data the hidden point, rhs and slacks are integers."""
    rng = np.random.default_rng(seed)
    u = rng.random(n)
    vtype = np.where(u < frac_bin, 0, np.where(u < frac_bin + frac_int, 1, 2))
    lo_int = rng.integers(-3, 4, size=n).astype(np.float64)
    lb = np.where(vtype == 0, 0.0, np.where(vtype == 1, lo_int, 0.0))
    ub = np.where(vtype == 0, 1.0, np.where(vtype == 1, lo_int + rng.integers(1, int_width, size=n), cont_ub))
    if inf_bounds > 0:
        kill_lo = (rng.random(n) < inf_bounds) & (vtype != 0)
        kill_hi = (rng.random(n) < inf_bounds) & (vtype != 0)
        lb = np.where(kill_lo, -np.inf, lb)
        ub = np.where(kill_hi, np.inf, ub)
    is_int = (vtype != 2).astype(np.uint8)
    lens = rng.integers(1, max_row_nnz + 1, size=m)
    rows, cols = _distinct_per_group(rng, lens, n)
    if long_cols > 0 and long_deg > 0:
        extra_c = rng.choice(n, size=min(long_cols, n), replace=False)
        er, ec = [], []
        for c in extra_c:
            rr = rng.choice(m, size=min(long_deg, m), replace=False)
            er.append(rr)
            ec.append(np.full(rr.shape[0], c))
        rows = np.concatenate([rows] + er)
        cols = np.concatenate([cols] + ec)
        key = rows * n + cols
        _, keep = np.unique(key, return_index=True)
        rows = rows[keep]
        cols = cols[keep]
    vals = _signed_nonzero_ints(rng, rows.shape[0], amax)
    if not integer_data:
        vals = vals * rng.uniform(0.5, 1.5, size=vals.shape[0])
    sense = np.array([SENSE_L, SENSE_G, SENSE_E], dtype=np.uint8)[rng.integers(0, 3, size=m)]
    lo_f = np.where(np.isfinite(lb), lb, -5.0)
    hi_f = np.where(np.isfinite(ub), ub, lo_f + 10.0)
    hidden = np.where(is_int == 1, np.floor(lo_f + rng.random(n) * (hi_f - lo_f + 1)), lo_f + rng.random(n) * (hi_f - lo_f))
    hidden = np.minimum(hidden, hi_f)
    if integer_data:
        hidden = np.where(is_int == 1, hidden, np.round(hidden))
        slack = rng.integers(0, 4, size=m).astype(np.float64)
    else:
        slack = rng.uniform(0.0, 3.0, size=m)
    obj = rng.integers(-5, 6, size=n).astype(np.float64)
    if not integer_data:
        obj = obj * 0.75

    def rhs_fn(act):
        return np.where(sense == SENSE_L, act + slack, np.where(sense == SENSE_G, act - slack, act))

    return _finish(n, m, rows, cols, vals, sense, rhs_fn, lb, ub, is_int, obj, hidden,
                   f"random_mixed(seed={seed})")


def random_point(mip: MIP, seed: int, frac_outside: float = 0.0) -> np.ndarray:
    """A seeded point inside the bounds, integral on integer variables."""
    rng = np.random.default_rng(seed)
    lo = np.where(np.isfinite(mip.lb), mip.lb, -10.0)
    hi = np.where(np.isfinite(mip.ub), mip.ub, lo + 20.0)
    lo = np.where(np.isfinite(mip.lb), lo, hi - 20.0)
    x = lo + rng.random(mip.n) * (hi - lo)
    xi = np.floor(lo + rng.random(mip.n) * (hi - lo + 1))
    x = np.where(mip.is_int == 1, np.minimum(xi, hi), x)
    return x.astype(np.float64)


def random_weights(size: int, seed: int, wmax: int = 8) -> np.ndarray:
    """Seeded integer-valued constraint weights in [1, wmax] (float32)."""
    rng = np.random.default_rng(seed)
    return rng.integers(1, wmax + 1, size=size).astype(np.float32)


# the workloads named by the benchmark configurations
CONFIGS = {
    "tiny_binary": dict(fn=tiny_binary, kwargs=dict(seed=0), iters=1000, tenure=10),
    "general": dict(fn=general, kwargs=dict(seed=0), iters=10_000, tenure=10),
    "powerlaw": dict(fn=powerlaw, kwargs=dict(seed=0), iters=10_000, tenure=10),
}
