"""Exact-arithmetic reference used to pin the CPU oracle.

Pure Python with fractions.Fraction: no floating point, no code shared with
the oracle or with the HIP library. Only for tiny instances.

Definitions (CHAP section 3.1):
  * a normalised row is  sum_k a_ik x_k <= b_i ; 'G' rows are negated and 'E'
    rows become a (row, negated row) pair ("Memory Considerations");
  * the penalty p_ij and the score s_j of a move ("Scoring Functions"), with
    the comparison "y > b" read as residual > eps;
  * the best shift (Eq. 1) maximises s_j over the variable's domain D_j; the
    step function changes only at breakpoints, bounds and the incumbent
    ("Best Shift Moves"), so Algorithm 1 scans the candidate set
    C_j = ({l_j, u_j} U {t_ij}) within [l_j, u_j], minus the incumbent.
"""
from __future__ import annotations

import math
from fractions import Fraction

INF = float("inf")


def F(v) -> Fraction:
    return Fraction(v)


class ExactProblem:
    def __init__(self, mip, eps: float = 1e-6):
        self.n = mip.n
        self.eps = F(eps)
        self.rows = []  # list of (dict col -> Fraction, rhs Fraction)
        self.orig = []
        self.sign = []
        for i in range(mip.m):
            lo, hi = int(mip.csr_row_ptr[i]), int(mip.csr_row_ptr[i + 1])
            coef = {int(mip.csr_col[k]): F(float(mip.csr_val[k])) for k in range(lo, hi)
                    if mip.csr_val[k] != 0}
            b = F(float(mip.rhs[i]))
            s = chr(int(mip.sense[i]))
            if s in ("L", "E"):
                self.rows.append((coef, b))
                self.orig.append(i)
                self.sign.append(1)
            if s in ("G", "E"):
                self.rows.append(({c: -v for c, v in coef.items()}, -b))
                self.orig.append(i)
                self.sign.append(-1)
        self.mp = len(self.rows)
        self.is_int = [bool(v) for v in mip.is_int]
        self.lb, self.ub = [], []
        for j in range(mip.n):
            l, u = float(mip.lb[j]), float(mip.ub[j])
            if self.is_int[j]:
                l = math.ceil(l) if math.isfinite(l) else l
                u = math.floor(u) if math.isfinite(u) else u
            self.lb.append(l)
            self.ub.append(u)
        self.obj = [F(float(c)) for c in mip.obj]
        self.obj_integral = all(c == 0 or (self.is_int[j] and c.denominator == 1)
                                for j, c in enumerate(self.obj))
        self.cols = [[] for _ in range(mip.n)]
        for i, (coef, _) in enumerate(self.rows):
            for c, v in coef.items():
                self.cols[c].append((i, v))

    def is_binary(self, j):
        return self.is_int[j] and self.lb[j] == 0 and self.ub[j] == 1

    # ---- residuals -------------------------------------------------------
    def residual(self, x, cutoff=None):
        x = [F(float(v)) for v in x]
        r = [sum((v * x[c] for c, v in coef.items()), Fraction(0)) - b for coef, b in self.rows]
        rc = None
        if cutoff is not None:
            rc = sum((c * x[j] for j, c in enumerate(self.obj) if c != 0), Fraction(0)) - F(cutoff)
        return r, rc

    def column(self, j, cutoff_active):
        out = list(self.cols[j])
        if cutoff_active and self.obj[j] != 0:
            out.append((self.mp, self.obj[j]))
        return out

    # ---- scores ----------------------------------------------------------
    def penalty(self, r, r2, w):
        eps = self.eps
        if r <= eps < r2:
            return -w
        if r2 <= eps < r:
            return w
        if eps < r2 < r:
            return w / 2
        if eps < r < r2:
            return -w / 2
        return Fraction(0)

    def score(self, j, xbar, xnew, r_all, w, cutoff_active):
        """s_j(xnew, xbar) = sum_i p_ij (direct definition)."""
        d = F(xnew) - F(xbar)
        s = Fraction(0)
        for i, a in self.column(j, cutoff_active):
            s += self.penalty(r_all[i], r_all[i] + a * d, F(float(w[i])))
        return s

    def breakpoint(self, j, xbar, r, a):
        t = F(xbar) + (self.eps - r) / a
        if self.is_int[j]:
            t = Fraction(math.floor(t)) if a > 0 else Fraction(math.ceil(t))
        return t

    def candidates(self, j, xbar, r_all, cutoff_active):
        c = set()
        l, u = self.lb[j], self.ub[j]
        if math.isfinite(l):
            c.add(F(l))
        if math.isfinite(u):
            c.add(F(u))
        for i, a in self.column(j, cutoff_active):
            c.add(self.breakpoint(j, xbar, r_all[i], a))
        lo = F(l) if math.isfinite(l) else None
        hi = F(u) if math.isfinite(u) else None
        return sorted(p for p in c if (lo is None or p >= lo) and (hi is None or p <= hi) and p != F(xbar))

    def best_shift(self, j, x, r_all, w, cutoff_active):
        """(xhat, s): smallest maximiser over C_j (or the flip for a binary),
        (xbar, 0) if no candidate scores above zero."""
        xbar = F(float(x[j]))
        if self.is_binary(j):
            cand = [1 - xbar]
        else:
            cand = self.candidates(j, xbar, r_all, cutoff_active)
        best, arg = None, None
        for p in cand:
            s = self.score(j, xbar, p, r_all, w, cutoff_active)
            if best is None or s > best:
                best, arg = s, p
        if best is None or best <= 0:
            return xbar, Fraction(0)
        return arg, best

    def brute_force_max(self, j, x, r_all, w, cutoff_active):
        """max over every integer of D_j except the incumbent (finite bounds)."""
        xbar = F(float(x[j]))
        vals = []
        for p in range(int(self.lb[j]), int(self.ub[j]) + 1):
            if F(p) == xbar:
                continue
            vals.append((self.score(j, xbar, p, r_all, w, cutoff_active), p))
        return vals

    # ---- tabu walk (same readings as the oracle, exact arithmetic) -------
    def start_point(self, seed, splitmix):
        x = []
        for j in range(self.n):
            l, u = self.lb[j], self.ub[j]
            if seed != 0 and self.is_int[j] and math.isfinite(l) and math.isfinite(u):
                h = splitmix(seed, j)
                x.append(F(l) + (h % (int(u - l) + 1)))
            else:
                x.append(F(min(max(0.0, l), u)))
        return x

    def tabu_run(self, iters, tenure, x0):
        """Residuals, the objective and the cutoff residual are exact
        rationals; the oracle holds them rounded once to FP64 (compare with
        float(), which rounds a Fraction to nearest)."""
        x = [F(v) for v in x0]
        n, mp = self.n, self.mp
        w = [Fraction(1)] * (mp + 1)
        tabu = [-1] * n
        fbest = None
        bc = None
        trace = []

        def resid():
            r, rc = self.residual(x, None)
            r = list(r)
            if bc is not None:
                r.append(sum((c * x[j] for j, c in enumerate(self.obj) if c != 0), Fraction(0)) - bc)
            else:
                r.append(Fraction(0))
            return r

        def nviol(r):
            v = sum(1 for i in range(mp) if r[i] > self.eps)
            if bc is not None and r[mp] > self.eps:
                v += 1
            return v

        def objective():
            return sum((c * x[j] for j, c in enumerate(self.obj) if c != 0), Fraction(0))

        r = resid()
        V = nviol(r)

        def check():
            nonlocal fbest, bc, r, V
            if V != 0:
                return
            f = objective()
            if fbest is None or f < fbest:
                fbest = f
            # delta and the cutoff right-hand side are FP64 numbers computed as
            # the reading writes them: delta = 1 for an integral objective, else
            # 1e-4 max(1, |f_best|), and b_c = f_best - delta, each rounded
            fb = float(fbest)
            delta = 1.0 if self.obj_integral else 1e-4 * max(1.0, abs(fb))
            bc = Fraction(fb - delta)
            r = resid()
            V = nviol(r)

        check()
        for k in range(iters):
            r = resid()
            V = nviol(r)
            active = bc is not None
            wf = [float(v) for v in w]
            res = [self.best_shift(j, x, r, wf, active) for j in range(n)]
            j_all = j_nt = -1
            for j in range(n):
                s = res[j][1]
                if not s > 0:
                    continue
                if j_all < 0 or s > res[j_all][1]:
                    j_all = j
                if k > tabu[j] and (j_nt < 0 or s > res[j_nt][1]):
                    j_nt = j
            jstar, kind = -1, 2
            if j_all >= 0 and k > tabu[j_all]:
                jstar, kind = j_all, 0
            elif j_all >= 0:
                d = res[j_all][0] - x[j_all]
                V2 = V
                for i, a in self.column(j_all, active):
                    v0 = r[i] > self.eps
                    v1 = r[i] + a * d > self.eps
                    V2 += (-1 if (v0 and not v1) else 0) + (1 if (v1 and not v0) else 0)
                if V2 == 0:
                    jstar, kind = j_all, 1
                elif j_nt >= 0:
                    jstar, kind = j_nt, 0
            if jstar < 0:
                for i in range(mp):
                    if r[i] > self.eps:
                        w[i] += 1
                if active and r[mp] > self.eps:
                    w[mp] += 1
                trace.append((k, -1, kind, 0, 0, 0, V, objective()))
            else:
                old = x[jstar]
                x[jstar] = res[jstar][0]
                tabu[jstar] = k + tenure
                r = resid()
                V = nviol(r)
                trace.append((k, jstar, kind, old, x[jstar], res[jstar][1], V, objective()))
            check()
        return trace, x, w, fbest, bc, resid()
