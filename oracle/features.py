"""CPU reference of the proposal network's inputs.

TEST INFRASTRUCTURE ONLY: used by the tests; the product library never
imports it and shares no code with it.

The inputs are a design of this project, not of the paper (the paper scores
every column exactly each iteration, section 3.1 "Scoring Functions"); they
are written here from their definitions, in plain FP64 loops over each
column's normalised rows (an equality row counts as its two normalised rows;
the objective cutoff row is excluded), each value rounded once to bfloat16:

  0  sum of w over violated rows / sum of w over all rows (0 without rows)
  1  log2(1 + stored nonzeros of the column)
  2  c_j / max |c| (0 when c = 0)
  3  s_last / (sum of w), clamped to [-4, 4] (0 without rows)
  4  binary, 5 integer but not binary, 6 continuous (1 or 0)
  7  (x - l) / (u - l); 0.5 with an infinite bound; 0 when l = u
  8  log2(1 + min(u - l, 2^20)); 20 with an infinite bound
  9  violated rows / rows (0 without rows)
  10 sum over violated rows of |a| min(r, 1000) / (1000 sum |a|)
  11 sign(xhat_last - x)
  12 min(k - last_move, 1024) / 1024
  13 min(k - k_last_full, 64) / 64
  14 V / m' (violated normalised rows, cutoff row included when active)
  15 log2(1 + moves)

A row is violated when its residual exceeds eps. A column is proposable when
it is binary, or integer with finite bounds and at most 64 values (any
length), or when its normalised entries, plus one for a nonzero objective
coefficient, plus two bounds, number at most 4096; other columns get
all-zero rows.
"""
from __future__ import annotations

import math

import numpy as np

from . import mlp

SUBSET_CAP = 4096


def column_rows(mip, orig_row, sign):
    """For every column, its normalised rows as (row index, coefficient)."""
    norm_of = [[] for _ in range(mip.m)]
    for k, (i, sg) in enumerate(zip(orig_row, sign)):
        norm_of[int(i)].append((k, int(sg)))
    cols = []
    for j in range(mip.n):
        lst = []
        for p in range(int(mip.csc_col_ptr[j]), int(mip.csc_col_ptr[j + 1])):
            a = float(mip.csc_val[p])
            if a == 0.0:
                continue
            for k, sg in norm_of[int(mip.csc_row[p])]:
                lst.append((k, sg * a))
        cols.append(lst)
    return cols


def proposable(mip, cols, lb, ub):
    out = np.zeros(mip.n, dtype=bool)
    for j in range(mip.n):
        l, u = float(lb[j]), float(ub[j])
        narrow = bool(mip.is_int[j]) and math.isfinite(l) and math.isfinite(u) and u - l + 1 <= 64
        entries = len(cols[j]) + (1 if mip.obj[j] != 0.0 else 0) + 2
        out[j] = narrow or entries <= SUBSET_CAP
    return out


def inputs(mip, oracle_problem, x, w, cutoff_rhs, s_last, xhat_last, last_move, moves, k, k_last_full,
           refresh=None):
    """Network inputs (n x 16, FP64 values of bfloat16 numbers) and the
    proposable mask. `refresh` = (x, w, cutoff_rhs) of the point where the
    row aggregates (inputs 0, 3, 9, 10) were last refreshed; defaults to the
    current point."""
    P = oracle_problem
    eps = P.eps
    orig_row, sign = P.norm_rows()
    lb, ub, is_bin = P.bounds()
    cols = column_rows(mip, orig_row, sign)
    ok = proposable(mip, cols, lb, ub)
    r_now, V = P.residual(x, cutoff_rhs)
    if refresh is None:
        r_ref, w_ref = r_now, w
    else:
        r_ref, _ = P.residual(refresh[0], refresh[2])
        w_ref = refresh[1]
    cmax = float(np.max(np.abs(mip.obj))) if mip.n else 0.0
    out = np.zeros((mip.n, 16))
    for j in range(mip.n):
        if not ok[j]:
            continue
        sw = swv = nv = ne = sa = sav = 0.0
        for (row, a) in cols[j]:
            wr = float(w_ref[row])
            r = float(r_ref[row])
            sw += wr
            ne += 1.0
            sa += abs(a)
            if r > eps:
                swv += wr
                nv += 1.0
                sav += abs(a) * min(r, 1000.0)
        l, u = float(lb[j]), float(ub[j])
        deg = sum(1 for p in range(int(mip.csc_col_ptr[j]), int(mip.csc_col_ptr[j + 1])) if mip.csc_val[p] != 0.0)
        f = out[j]
        f[0] = swv / sw if sw > 0 else 0.0
        f[1] = math.log2(1.0 + deg)
        f[2] = float(mip.obj[j]) / cmax if cmax > 0 else 0.0
        f[3] = min(max(float(s_last[j]) / sw, -4.0), 4.0) if sw > 0 else 0.0
        binary = bool(is_bin[j])
        f[4] = 1.0 if binary else 0.0
        f[5] = 1.0 if (mip.is_int[j] and not binary) else 0.0
        f[6] = 0.0 if mip.is_int[j] else 1.0
        xj = float(x[j])
        if not (math.isfinite(l) and math.isfinite(u)):
            f[7] = 0.5
            f[8] = 20.0
        else:
            f[7] = (xj - l) / (u - l) if u > l else 0.0
            f[8] = math.log2(1.0 + min(u - l, 2.0 ** 20))
        f[9] = nv / ne if ne > 0 else 0.0
        f[10] = sav / (1000.0 * sa) if sa > 0 else 0.0
        d = float(xhat_last[j]) - xj
        f[11] = 1.0 if d > 0 else (-1.0 if d < 0 else 0.0)
        f[12] = min(k - int(last_move[j]), 1024) / 1024.0
        f[13] = min(k - k_last_full, 64) / 64.0
        f[14] = V / max(P.mp, 1)
        f[15] = math.log2(1.0 + int(moves[j]))
    return mlp.bf16(out), ok
