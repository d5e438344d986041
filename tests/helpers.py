"""Small shared test helpers: hand-built MIPs and the pure-Python SplitMix64."""
from __future__ import annotations

import numpy as np

import mipgen

MASK64 = (1 << 64) - 1


def splitmix64_py(seed: int, index: int) -> int:
    """(index+1)-th output of SplitMix64 from state `seed` (Steele, Lea &
    Flood 2014), in Python integers."""
    z = (seed + (index + 1) * 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def make_mip(n, rows, lb, ub, is_int, obj=None):
    """rows: list of (dict col -> coef, sense char, rhs)."""
    r_idx, c_idx, vals = [], [], []
    for i, (coef, _, _) in enumerate(rows):
        for c, v in sorted(coef.items()):
            r_idx.append(i)
            c_idx.append(c)
            vals.append(float(v))
    m = len(rows)
    csr = mipgen.coo_to_csr_csc(n, m, np.array(r_idx, dtype=np.int64), np.array(c_idx, dtype=np.int64),
                                np.array(vals, dtype=np.float64))
    sense = np.array([ord(s) for _, s, _ in rows], dtype=np.uint8)
    rhs = np.array([float(b) for _, _, b in rows], dtype=np.float64)
    obj = np.zeros(n) if obj is None else np.asarray(obj, dtype=np.float64)
    return mipgen.MIP(n=n, m=m, csr_row_ptr=csr[0], csr_col=csr[1], csr_val=csr[2], csc_col_ptr=csr[3],
                      csc_row=csr[4], csc_val=csr[5], sense=sense, rhs=rhs,
                      lb=np.asarray(lb, dtype=np.float64), ub=np.asarray(ub, dtype=np.float64),
                      is_int=np.asarray(is_int, dtype=np.uint8), obj=obj, name="hand")


def normalised_weights(orig_row, sign, per_original_row_weights, cutoff_w=1.0):
    """Expand weights listed per normalised row (in normalised order) plus the cutoff."""
    return np.concatenate([np.asarray(per_original_row_weights, dtype=np.float32),
                           np.array([cutoff_w], dtype=np.float32)])


def tabu_until_from_trace(trace, n, tenure):
    """Last iteration through which each variable is tabu, from a walk's trace
    (a variable moved at iteration k is tabu through k + tenure)."""
    t = np.full(n, -1, dtype=np.int64)
    moved = trace["var"] >= 0
    t[trace["var"][moved]] = trace["iter"][moved] + tenure  # later moves overwrite earlier ones
    return t
