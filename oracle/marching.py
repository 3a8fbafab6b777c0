"""Time marching over slabs with inhomogeneous Dirichlet data (test
infrastructure).

Eq. (AlgSysTMS) of Sec. 3.2: slab after slab, the system of one slab is
solved with the coupling of its first subinterval to the end value V_0 of
the previous slab moved to the right-hand side, B_1 - C^1 V_0, C^1 =
-C^tau (x) [M_h; 0].  Here a slab holds N subintervals (N = 1 is the paper's
time-marching case; the global system of Eq. (GloSys) is one slab of all
subintervals).  Dirichlet data g (values at the Dirichlet velocity nodes at
every temporal dof) are lifted: with gD = g on Dirichlet entries and 0
elsewhere, the homogeneous system S x0 = b,
    b = f - S_full gD - C^1 V_0   on free velocity rows and pressure rows,
    b = 0                         on Dirichlet rows,
is solved and x = x0 + gD.  S_full is Eq. (GloSys) with every column kept
(the homogeneous operator of `SpaceTimeLevel` zeroes the Dirichlet columns).
The temporal dofs sit at the right Radau points, so the end value of a slab
is the velocity of the last temporal dof of its last subinterval.
"""
import numpy as np

from .spacetime import SpaceTimeLevel


def full_apply(L: SpaceTimeLevel, x, v0=None):
    """S_full x, plus for the first subinterval -C^tau (x) M_h v0 (the term
    C^1 V_0), Eq. (InAlg)/(DefDtauh) with no Dirichlet row or column removed."""
    s = L.sp
    y = np.zeros_like(x)
    for n in range(L.N):
        Mx = [s.Mh @ x[L.v_index(n, b)] for b in range(L.nt)]
        Ax = [s.Ah @ x[L.v_index(n, b)] for b in range(L.nt)]
        if n > 0:
            prev = [s.Mh @ x[L.v_index(n - 1, b)] for b in range(L.nt)]
        elif v0 is not None:
            prev = [np.zeros(L.Mv)] * (L.nt - 1) + [s.Mh @ v0]   # only the last dof of V_0 couples
        else:
            prev = None
        for a in range(L.nt):
            yv = np.zeros(L.Mv)
            yp = np.zeros(L.Mp)
            for b in range(L.nt):
                yv += L.K[a, b] * Mx[b] + L.Mtau[a, b] * Ax[b]
                yv -= L.Mtau[a, b] * (s.B.T @ x[L.p_index(n, b)])
                yp -= L.Mtau[a, b] * (s.B @ x[L.v_index(n, b)])
                if prev is not None:
                    yv -= L.Ctau[a, b] * prev[b]
            y[L.v_index(n, a)] = yv
            y[L.p_index(n, a)] = yp
    return y


def dirichlet_part(L: SpaceTimeLevel, g):
    """gD: g on the Dirichlet velocity entries, 0 elsewhere."""
    return np.where(L.dirichlet_mask(), g, 0.0)


def slab_rhs(L: SpaceTimeLevel, f=None, v0=None, g=None):
    """b = f - S_full gD - C^1 V_0 on free rows, 0 on Dirichlet rows."""
    f = np.zeros(L.ndofs) if f is None else np.asarray(f, dtype=float)
    gD = np.zeros(L.ndofs) if g is None else dirichlet_part(L, g)
    b = f - full_apply(L, gD, v0)
    b[L.dirichlet_mask()] = 0.0
    return b


def end_value(L: SpaceTimeLevel, x):
    """Velocity of the last temporal dof of the last subinterval."""
    return x[L.v_index(L.N - 1, L.nt - 1)].copy()


def solve_slab(L: SpaceTimeLevel, solve, f=None, v0=None, g=None):
    """x = solve(b) + gD, solve a solver of the homogeneous slab system."""
    x = solve(slab_rhs(L, f, v0, g))
    if g is not None:
        x = x + dirichlet_part(L, g)
    return x


def march(L: SpaceTimeLevel, solve, n_slabs, f=None, g=None, v0=None):
    """Slab after slab; f and g are (n_slabs, ndofs) arrays or None.
    Returns the (n_slabs, ndofs) solutions."""
    xs = []
    for s in range(n_slabs):
        x = solve_slab(L, solve, None if f is None else f[s], v0, None if g is None else g[s])
        xs.append(x)
        v0 = end_value(L, x)
    return np.array(xs)
