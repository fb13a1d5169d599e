"""Seeded synthetic workloads (input recipes only).

The lattices, column counts, seeds and time-step counts of the workloads the
tests and the benchmark run.  Nothing here computes any part of the method:
states and disorder are drawn by the library (on the GPU) and by the oracle
(on the CPU) from the seeds given here, each with its own implementation of
the counter-based generator.

The paper's test system (twisted bilayer graphene, Sec. III) cannot be
rebuilt from its text; these lattices stand in for its size range
(5e7 to 1e9 orbitals in Fig. 1).
"""
import numpy as np

# Plain method, CPU-sized: 64 x 64 square lattice, |H| = 4.1.
SQUARE64 = dict(kind="square", Lx=64, Ly=64, t=1.0, W=0.0, disorder_seed=0, R=1,
                seed_states=1, Nt=1024)

# Graphene, 1024 x 1024 cells (2 097 152 orbitals), 4 random-phase columns
# and 64 LDOS sites.
GRAPHENE1024 = dict(kind="honeycomb", Lx=1024, Ly=1024, t=-2.7, W=0.0, disorder_seed=0, R=4,
                    n_sites=64, seed_states=2, seed_sites=3, Nt=2048)

# Disordered graphene, 4096 x 4096 cells (33 554 432 orbitals), Anderson
# disorder W = 1 eV, 16 random-phase columns, block size from the cost model.
DISORDERED_GRAPHENE4096 = dict(kind="honeycomb", Lx=4096, Ly=4096, t=-2.7, W=1.0,
                               disorder_seed=4, R=16, seed_states=5, Nt=2048)

# Large square lattice, 31623 x 31623 (1 000 014 129 orbitals), W = 0.5,
# 4 random-phase columns.
SQUARE31623 = dict(kind="square", Lx=31623, Ly=31623, t=1.0, W=0.5, disorder_seed=6, R=4,
                   seed_states=7, Nt=4096)

# Stand-in for the paper's magic-angle twisted bilayer graphene supercell
# (4 763 200 atoms, matrix densities D_H = 60, 120, 230; Sec. III): the
# long-range square lattice below, 2182 x 2182 sites (4 761 124 orbitals),
# hopping -1 * exp(-(d - 1)/2) to every site within r_cut, on-site energies
# W = 0.5; r_cut 4.3, 6.1, 8.6 give D_H = 61, 121, 233.  Random-phase
# states per density as in the paper's protocol (10, 5, 2), Nt = 4096.
LONG_RANGE2182 = dict(L=2182, t0=-1.0, decay=2.0, W=0.5, seed=1, seed_states=9, Nt=4096,
                      cases=[dict(r_cut=4.3, D=61, R=10), dict(r_cut=6.1, D=121, R=5),
                             dict(r_cut=8.6, D=233, R=2)])


def batch32(seed=8, n=32):
    """Uneven batch: n lattices alternating square (t = 1 eV) and honeycomb
    (t = -2.7 eV), sides drawn from 128..2048 cells, W uniform in [0, 2] eV,
    1..8 random-phase columns each; 1024 time steps."""
    rng = np.random.default_rng(seed)
    sides = [128, 256, 512, 1024, 2048]
    out = []
    for i in range(n):
        kind = "square" if i % 2 == 0 else "honeycomb"
        L = int(sides[rng.integers(len(sides))])
        out.append(dict(kind=kind, Lx=L, Ly=L, t=1.0 if kind == "square" else -2.7,
                        W=float(rng.uniform(0.0, 2.0)), disorder_seed=100 + i,
                        R=int(rng.integers(1, 9)), seed_states=200 + i))
    return out, 1024


def scaled(cfg, **over):
    """A copy of a workload with some fields replaced (scaled-down parity
    cases keep the kind, hopping, disorder and seeds)."""
    d = dict(cfg)
    d.update(over)
    return d


def long_range_square(L, r_cut, t0=1.0, decay=1.0, W=0.0, seed=0):
    """Stand-in for the paper's dense twisted-bilayer Hamiltonians (matrix
    density D_H = 60..230): an L x L periodic square lattice (orbital
    s = y*L + x) with hopping t0 * exp(-(d - 1)/decay) to every site at
    distance 0 < d <= r_cut, and on-site energies W*(u - 1/2) from numpy's
    generator seeded with `seed`.  Returns (col, val) in ELL form, [N][D]
    each, with the on-site entry first; D_H = D = 1 + #{lattice vectors
    0 < |v| <= r_cut}.  L must exceed 2 r_cut (no duplicate neighbours)."""
    if L <= 2 * r_cut:
        raise ValueError("L must exceed 2 r_cut")
    R = int(np.floor(r_cut))
    offs = [(dx, dy) for dy in range(-R, R + 1) for dx in range(-R, R + 1)
            if 0 < dx * dx + dy * dy <= r_cut * r_cut]
    N = L * L
    D = 1 + len(offs)
    col = np.empty((N, D), dtype=np.int32)
    val = np.empty((N, D), dtype=np.float64)
    s = np.arange(N, dtype=np.int64)
    y, x = s // L, s % L
    col[:, 0] = s
    val[:, 0] = W * (np.random.default_rng(seed).random(N) - 0.5) if W else 0.0
    for k, (dx, dy) in enumerate(offs, start=1):
        col[:, k] = ((y + dy) % L) * L + (x + dx) % L
        val[:, k] = t0 * np.exp(-(np.sqrt(dx * dx + dy * dy) - 1.0) / decay)
    return col, val


def long_range_square_positions(L):
    """Coordinates of the orbitals of long_range_square (orbital s at
    (s mod L, s div L)) and the periodic box (L, L)."""
    s = np.arange(L * L)
    return np.stack([(s % L).astype(np.float64), (s // L).astype(np.float64)], 1), (float(L),
                                                                                      float(L))


def random_symmetric_ell(N, n_pairs, seed=0, diag=True):
    """A random real symmetric matrix of irregular row lengths in ELL form:
    n_pairs off-diagonal pairs (i, j), i != j, drawn uniformly (duplicates
    dropped), each with one normal value placed at (i, j) and (j, i), plus a
    normal diagonal when diag.  Rows are padded to the longest with col = -1
    (val = 0).  Returns (col int32 [N][D], val float64 [N][D])."""
    rng = np.random.default_rng(seed)
    i = rng.integers(0, N, size=n_pairs)
    j = rng.integers(0, N, size=n_pairs)
    keep = i != j
    a, b = np.minimum(i[keep], j[keep]), np.maximum(i[keep], j[keep])
    pairs = np.unique(np.stack([a, b], 1), axis=0)
    v = rng.normal(size=len(pairs))
    rows = [[] for _ in range(N)]
    if diag:
        d = rng.normal(size=N)
        for s in range(N):
            rows[s].append((s, d[s]))
    for (p, q), x in zip(pairs, v):
        rows[p].append((q, x))
        rows[q].append((p, x))
    D = max(1, max(len(r) for r in rows))
    col = np.full((N, D), -1, dtype=np.int32)
    val = np.zeros((N, D), dtype=np.float64)
    for s, r in enumerate(rows):
        for k, (c, x) in enumerate(r):
            col[s, k] = c
            val[s, k] = x
    return col, val


def long_range_with_far_pairs(L=48, r_cut=3.0, n_rows=160, extra=70, seed=6):
    """The long-range square lattice of long_range_square (t0 = -1,
    decay 1.5, W = 0.7) with `extra` additional symmetric entries of normal
    values (scale 0.3) between each of the first n_rows rows and uniformly
    drawn far rows: most slices of 128 neighbouring rows still name a few
    hundred columns, the slices that hold those rows name thousands.
    Rows are padded to the longest with col = -1.  Returns (col int32
    [N][D], val float64 [N][D])."""
    col, val = long_range_square(L, r_cut, t0=-1.0, decay=1.5, W=0.7, seed=seed)
    N = col.shape[0]
    rng = np.random.default_rng(seed)
    rows = [list(zip(col[s].tolist(), val[s].tolist())) for s in range(N)]
    for s in range(n_rows):
        for j in rng.choice(N, size=extra, replace=False):
            j = int(j)
            if j == s or any(c == j for c, _ in rows[s]):
                continue
            v = float(rng.normal()) * 0.3
            rows[s].append((j, v))
            rows[j].append((s, v))
    D = max(len(r) for r in rows)
    c2 = np.full((N, D), -1, dtype=np.int32)
    v2 = np.zeros((N, D), dtype=np.float64)
    for s, r in enumerate(rows):
        for k, (c, v) in enumerate(r):
            c2[s, k] = c
            v2[s, k] = v
    return c2, v2
