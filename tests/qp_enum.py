"""Exact small convex QPs by active-set enumeration (a test checker).

Solves  min 1/2 x'Hx + f'x  s.t.  E x = e,  lo <= C x <= hi
by trying active sets in order of size: each row of C is free, held at its
lower bound or held at its upper bound.  For a candidate the KKT system

    [H  E'  Ca'] [x ]   [-f]
    [E  0   0  ] [nu] = [ e]
    [Ca 0   0  ] [mu]   [ b]

is solved; the candidate is accepted when x satisfies every bound and every
multiplier has the sign of its bound (mu <= 0 at a lower bound, >= 0 at an
upper bound).  For a convex problem any accepted point is optimal.  This is
the textbook KKT characterisation and shares nothing with the ADMM path.
"""
from __future__ import annotations

import itertools

import numpy as np


def solve_qp_enum(H, f, E, e, C, lo, hi, max_active=None, tol=1e-9):
    H = np.asarray(H, float)
    f = np.asarray(f, float)
    n = H.shape[0]
    E = np.zeros((0, n)) if E is None else np.asarray(E, float).reshape(-1, n)
    e = np.zeros(0) if e is None else np.asarray(e, float).reshape(-1)
    C = np.zeros((0, n)) if C is None else np.asarray(C, float).reshape(-1, n)
    lo = np.asarray(lo, float).reshape(-1)
    hi = np.asarray(hi, float).reshape(-1)
    m = C.shape[0]
    me = E.shape[0]
    scale = max(1.0, np.abs(H).max(), np.abs(f).max() if f.size else 1.0)
    if max_active is None:
        max_active = min(m, n)
    for na in range(0, max_active + 1):
        for rows in itertools.combinations(range(m), na):
            sides_opts = []
            for r in rows:
                opts = []
                if np.isfinite(lo[r]):
                    opts.append(-1)
                if np.isfinite(hi[r]):
                    opts.append(+1)
                sides_opts.append(opts)
            for sides in itertools.product(*sides_opts):
                Ca = C[list(rows)] if na else np.zeros((0, n))
                b = np.array([lo[r] if s < 0 else hi[r] for r, s in zip(rows, sides)])
                k = n + me + na
                K = np.zeros((k, k))
                K[:n, :n] = H
                K[:n, n:n + me] = E.T
                K[n:n + me, :n] = E
                K[:n, n + me:] = Ca.T
                K[n + me:, :n] = Ca
                rhs = np.concatenate([-f, e, b])
                try:
                    if np.linalg.cond(K) > 1e12:
                        continue
                    sol = np.linalg.solve(K, rhs)
                except np.linalg.LinAlgError:
                    continue
                x = sol[:n]
                mu = sol[n + me:]
                cx = C @ x
                ptol = tol * max(1.0, np.abs(x).max())
                if np.any(cx < lo - ptol) or np.any(cx > hi + ptol):
                    continue
                sgn = np.array(sides, float)
                if np.any(sgn * mu < -tol * scale):
                    continue
                return x
    raise RuntimeError("no KKT point found")
