"""Flexible GMRES, right preconditioned (test infrastructure).

The paper uses GMRES without restart and one V-cycle per iteration
(Sec. 4.4, Sec. 5).  Because the mixed-precision and learned preconditioners
vary between applications, the flexible variant is used (Z holds the
preconditioned directions).  Orthogonalisation: classical Gram-Schmidt applied
twice (CGS2).  Least squares by Givens rotations.  Stop when the implicit
residual estimate is <= rtol * ||b||; the explicit residual is then recomputed
and the iteration restarts from x if it is still too large (reading G14).
Iteration count = number of preconditioner applications.
"""
import numpy as np


def fgmres(apply, precond, b, rtol=1e-8, max_it=100, restart=100):
    n = len(b)
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    history = []          # implicit estimates ||r_j||/||b||, explicit at (re)starts
    total = 0
    if bnorm == 0.0:
        return x, 0, [0.0]
    while True:
        r = b - apply(x)
        beta = np.linalg.norm(r)
        history.append(beta / bnorm)
        if beta <= rtol * bnorm or total >= max_it:
            return x, total, history
        m = restart
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        j = 0
        while j < m and total < max_it:
            z = precond(V[j])
            Z.append(z)
            w = apply(z)
            h = np.zeros(j + 2)
            for _ in range(2):                           # CGS2
                c = np.array([v @ w for v in V])
                for ci, v in zip(c, V):
                    w = w - ci * v
                h[: j + 1] += c
            hn = np.linalg.norm(w)
            h[j + 1] = hn
            for i in range(j):                            # earlier rotations
                t = cs[i] * h[i] + sn[i] * h[i + 1]
                h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1]
                h[i] = t
            den = np.hypot(h[j], h[j + 1])
            cs[j], sn[j] = h[j] / den, h[j + 1] / den
            h[j], h[j + 1] = den, 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            H[: j + 2, j] = h
            total += 1
            j += 1
            history.append(abs(g[j]) / bnorm)
            if abs(g[j]) <= rtol * bnorm or hn == 0.0:
                break
            V.append(w / hn)
        y = np.zeros(j)
        for i in range(j - 1, -1, -1):                    # back substitution
            y[i] = (g[i] - H[i, i + 1:j] @ y[i + 1:]) / H[i, i]
        for yi, zi in zip(y, Z):
            x = x + yi * zi
