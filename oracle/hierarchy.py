"""Multigrid level lists (test infrastructure).

A level is a dict(n=cells per direction, r=pressure degree, k=DG degree,
N=subintervals).  Lists are returned finest first (index 0 = finest).

* ``build_levels``: the build's default placement (reading G12): first halve r
  and k together on the fine mesh (p before h, principle P2 of Sec. 4.4;
  k -> floor(k/2) and r -> floor(r/2), Eq. (Assmp:MG2)), each floored at its
  minimum; then halve the mesh size down to the coarsest mesh.  Optional
  temporal h-coarsening N -> N/2 is aligned with the coarsest spatial h-steps
  (space before time, P1; space-time coarsening at the coarse end, P3).  It
  is off by default: on the slab workloads it costs iterations (a slab then
  keeps all N subintervals down to the coarsest level, solved exactly).
* ``construct_hierarchy`` / ``combine_hierarchies``: Alg. 2 and Alg. 3 as
  described in Sec. 4.4, used to check the worked example of App. C and the
  smoother sizes of Table 2(b).
"""
from .elements import vanka_block_size


def build_levels(n, r, k, N, n_coarse=1, r_min=1, k_min=1, time_h=False, placement="paper"):
    """Level list, finest first, as dicts (n, r, k, N).

    placement "paper" (default): Alg. 2 builds a spatial list (halve r on the
    fine mesh down to r_min, then halve the mesh size down to n_coarse) and a
    temporal list (halve k down to k_min, then, if time_h, halve N down to
    1); Alg. 3 pads the shorter list at its fine end and pairs the lists
    level by level, so temporal coarsening happens on the coarsest levels
    (principles P3/P4 of Sec. 4.4, App. C).
    placement "top": r and k are halved together on the fine mesh first
    (kept for comparison; it converges poorly for k >= 1, see DESIGN)."""
    if placement == "paper":
        space = [(n, r)]
        while r > r_min:
            r = max(r // 2, r_min)
            space.append((n, r))
        while n > n_coarse:
            n //= 2
            space.append((n, r))
        time = [(N, k)]
        while k > k_min:
            k = max(k // 2, k_min)
            time.append((N, k))
        if time_h:
            while N > 1:
                N //= 2
                time.append((N, k))
        L = max(len(space), len(time))
        space = [space[0]] * (L - len(space)) + space
        time = [time[0]] * (L - len(time)) + time
        return [dict(n=a[0], r=a[1], k=b[1], N=b[0]) for a, b in zip(space, time)]
    levels = [dict(n=n, r=r, k=k, N=N)]
    while r > r_min or k > k_min:
        r = max(r // 2, r_min) if r > r_min else r
        k = max(k // 2, k_min) if k > k_min else k
        levels.append(dict(n=n, r=r, k=k, N=N))
    h_steps = 0
    m = n
    while m > n_coarse:
        m //= 2
        h_steps += 1
    t_steps = 0
    if time_h:
        M = N
        while M > 1:
            M //= 2
            t_steps += 1
    for s in range(h_steps):
        n //= 2
        if time_h and s >= h_steps - t_steps:
            N = max(N // 2, 1)
        levels.append(dict(n=n, r=r, k=k, N=N))
    return levels


def construct_hierarchy(h_fine, h_coarse, p_fine, p_min, literal_h_loop=False):
    """Alg. 2: returns a list of (h, p), coarsest first.

    The printed h-loop pushes the already-halved degree; here it restarts from
    p_min.  With literal_h_loop=False the h-loop starts at 2h (each pushed mesh
    is new); with literal_h_loop=True it starts at h, so one extra (h, p_min)
    entry is emitted (reading G12)."""
    H = []
    h, p = h_fine, p_fine
    while p >= p_min:
        H.insert(0, (h, p))
        p //= 2
    p = p_min
    if not literal_h_loop:
        h *= 2
    while h <= h_coarse:
        H.insert(0, (h, p))
        h *= 2
    return H


def combine_hierarchies(Hh, Ht):
    """Alg. 3: pad the shorter list with its last (finest) entry at the fine
    end, then pair level by level.  Returns [(h, r, tau, k)] coarsest first."""
    Hh, Ht = list(Hh), list(Ht)
    L = max(len(Hh), len(Ht))
    while len(Ht) < L:
        Ht.append(Ht[-1])
    while len(Hh) < L:
        Hh.append(Hh[-1])
    return [(Hh[i][0], Hh[i][1], Ht[i][0], Ht[i][1]) for i in range(L)]


def paper_levels(n_fine, r, k, mode):
    """Level lists of the paper's examples, coarsest first, as (n, r, k).

    mode 'appendix': Alg. 2 with the fixed h-loop for space and time (App. C).
    mode 'table2'  : the same, but the temporal list uses the literal h-loop
                     (one extra (tau, k_min) entry); reproduces Table 2(b).
    Time is not coarsened geometrically (tau_fine = tau_coarse)."""
    Hh = construct_hierarchy(1.0 / n_fine, 1.0, r, 1)
    Ht = construct_hierarchy(1.0, 1.0, k, 1, literal_h_loop=(mode == "table2"))
    out = []
    for h, rr, tau, kk in combine_hierarchies(Hh, Ht):
        out.append((int(round(1.0 / h)), rr, kk))
    return out


def smoother_entries(levels, d):
    """N_sm^el: total entries of all cell-patch matrices of one subinterval,
    sum over levels of n_cells * b^2 (Table 2(b))."""
    return sum((lv[0] ** d) * vanka_block_size(d, lv[1], lv[2]) ** 2 for lv in levels)


def space_time_dofs(d, n, r, k, N):
    """All space-time dofs of a slab, Dirichlet dofs included (the paper's
    convention for N_dof, Eq. (throughput))."""
    from math import comb
    q = r + 1
    return N * (k + 1) * (d * (n * q + 1) ** d + n ** d * comb(r + d, d))
