"""FP64 CPU oracle for concurrent stochastic propagation (arXiv:2510.17432).

TEST INFRASTRUCTURE ONLY.  This package is the independent checker for the
GPU library: only tests/, __graft_entry__.smoke() and the cpu_baseline leg of
bench.py may import it.  It shares no code with the GPU library and never
imports it.

Contents, each following the passage cited beside it:
  * SplitMix64 counter generator (Steele, Lea & Flood 2014) -- inputs;
  * chain / square / honeycomb lattices with Anderson disorder -- Sec. II.B
    (matrix density) and the lattice conventions stated in ``Lattice``;
  * spectral half-width |H| by a Gershgorin bound times a margin -- Sec. II.A
    names the rescaling H~ = (H - H0)/|H|, not how |H| is found;
  * Bessel / Chebyshev coefficients and truncation order -- App. B, Sec. II.A;
  * sequential and state-based concurrent propagation -- Sec. II.A Eq. (TE),
    Sec. II.B time blocks (C code in csp_oracle.c);
  * moment-based propagation, in time blocks or in one block with the
    halving of Eq. (cheby_prod) -- Sec. II.A, Sec. III DOS-Concurrent-M;
  * Hamiltonians given explicitly in ELL form (any matrix density D_H);
  * quasi-eigenstates by forward and backward sequential propagation and
    the sum of Eq. QE_coeff (QE section, QE-Sequential);
  * site positions, the current operator J = i[H, X], and the electronic
    conductivity correlation of Eq. dc_corr by sequential propagation
    (EC-Sequential) and by Chebyshev moments (EC-Concurrent-M), with the
    conductivity integral of Eq. DC (EC section);
  * band-structure closed forms of clean periodic lattices (any size);
  * DOS from the correlation function -- Sec. III.

Pins: see tests/test_oracle_*.py.  Every routine here is pinned by at least
one test against a closed form, a library routine, a printed value of the
paper or brute force; none is "parity unpinned".
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

_LIB = None

KIND_CHAIN, KIND_SQUARE, KIND_HONEYCOMB = 0, 1, 2
KINDS = {"chain": KIND_CHAIN, "square": KIND_SQUARE, "honeycomb": KIND_HONEYCOMB}

_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load (building first if absent) the C part of the oracle."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(_build.LIB):
        _build.build()
    L = ctypes.CDLL(_build.LIB)
    L.orc_splitmix64.restype = ctypes.c_uint64
    L.orc_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    L.orc_splitmix64_stream.restype = None
    L.orc_splitmix64_stream.argtypes = [ctypes.c_uint64, ctypes.c_int64, _u64p]
    L.orc_draw.restype = ctypes.c_uint64
    L.orc_draw.argtypes = [ctypes.c_uint64] * 3
    L.orc_u01.restype = ctypes.c_double
    L.orc_u01.argtypes = [ctypes.c_uint64]
    L.orc_below.restype = ctypes.c_int64
    L.orc_below.argtypes = [ctypes.c_uint64, ctypes.c_int64]
    L.orc_lattice_sites.restype = ctypes.c_int64
    L.orc_lattice_sites.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64]
    L.orc_lattice_bonds.restype = ctypes.c_int64
    L.orc_lattice_bonds.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_int, ctypes.c_int, _i64p, _i64p]
    L.orc_onsite.restype = None
    L.orc_onsite.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, _dp]
    L.orc_build_csr.restype = None
    L.orc_build_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i64p,
                                ctypes.c_double, _dp, _i64p, _i64p, _dp]
    L.orc_bessel_j.restype = ctypes.c_int
    L.orc_bessel_j.argtypes = [ctypes.c_double, ctypes.c_int64, _dp]
    L.orc_cheb_coeffs.restype = ctypes.c_int
    L.orc_cheb_coeffs.argtypes = [ctypes.c_double, ctypes.c_int64, _dp]
    L.orc_truncation.restype = ctypes.c_int64
    L.orc_truncation.argtypes = [ctypes.c_double, ctypes.c_double]
    L.orc_propagate.restype = ctypes.c_int
    L.orc_propagate.argtypes = [ctypes.c_int64, _i64p, _i64p, _dp,
                                ctypes.c_double, ctypes.c_double, ctypes.c_int64, _dp,
                                ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int64, _dp, _dp, _i64p]
    L.orc_propagate_moments.restype = ctypes.c_int
    L.orc_propagate_moments.argtypes = [ctypes.c_int64, _i64p, _i64p, _dp,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int64, _dp,
                                        ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int64, ctypes.c_int, _dp, _dp, _i64p]
    L.orc_quasi_eigenstates.restype = ctypes.c_int
    L.orc_quasi_eigenstates.argtypes = [ctypes.c_int64, _i64p, _i64p, _dp,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int64, _dp,
                                        ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int64, _dp, _dp, _i64p]
    L.orc_chebyshev_vectors.restype = ctypes.c_int
    L.orc_chebyshev_vectors.argtypes = [ctypes.c_int64, _i64p, _i64p, _dp,
                                        ctypes.c_double, ctypes.c_double, _dp,
                                        ctypes.c_int64, _dp]
    L.orc_site_positions.restype = None
    L.orc_site_positions.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, _dp, _dp]
    L.orc_lattice_bond_vectors.restype = ctypes.c_int64
    L.orc_lattice_bond_vectors.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_int, ctypes.c_int, _dp, _dp]
    L.orc_current_bonds.restype = None
    L.orc_current_bonds.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i64p, _dp,
                                    ctypes.c_double, _dp, _dp]
    L.orc_current_csr.restype = None
    L.orc_current_csr.argtypes = [ctypes.c_int64, _i64p, _i64p, _dp, _dp, ctypes.c_double,
                                  _dp, _dp]
    L.orc_ec_sequential.restype = ctypes.c_int
    L.orc_ec_sequential.argtypes = [ctypes.c_int64, _i64p, _i64p, _dp, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int64, _dp, ctypes.c_int64, _dp,
                                    _dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double, _dp,
                                    _i64p]
    _LIB = L
    return L


def _p(a, t):
    return a.ctypes.data_as(t)


# ---------------------------------------------------------------- generator
def splitmix64(seed: int, k: int) -> int:
    """Output number k (0-based) of SplitMix64 seeded with `seed`."""
    return int(lib().orc_splitmix64(seed & (2**64 - 1), k))


def splitmix64_stream(seed: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.uint64)
    lib().orc_splitmix64_stream(seed & (2**64 - 1), n, _p(out, _u64p))
    return out


def draw(seed: int, stream: int, index: int) -> int:
    return int(lib().orc_draw(seed & (2**64 - 1), stream, index))


def u01(bits: int) -> float:
    return float(lib().orc_u01(bits))


def below(bits: int, n: int) -> int:
    return int(lib().orc_below(bits, n))


# ---------------------------------------------------------------- lattices
class Lattice:
    """Tight-binding lattice with uniform hopping t and Anderson disorder.

    Orbital order: chain s = ix; square s = iy*Lx + ix; honeycomb
    s = 2*(iy*Lx + ix) + sigma (sigma 0 = A, 1 = B) with bonds A(ix,iy)-B(ix,iy),
    A(ix,iy)-B(ix-1,iy), A(ix,iy)-B(ix,iy-1).  H_ab = t on every bond (repeated
    bonds add), H_ss = eps_s = W*(u_s - 1/2) with u_s drawn from stream 0 of
    `disorder_seed`.
    """

    def __init__(self, kind, Lx, Ly=1, t=1.0, W=0.0, disorder_seed=0,
                 periodic_x=True, periodic_y=True):
        self.kind = KINDS[kind] if isinstance(kind, str) else int(kind)
        self.Lx, self.Ly = int(Lx), int(Ly) if self.kind != KIND_CHAIN else 1
        self.t, self.W = float(t), float(W)
        self.seed = int(disorder_seed)
        self.px, self.py = int(bool(periodic_x)), int(bool(periodic_y))
        L = lib()
        self.N = int(L.orc_lattice_sites(self.kind, self.Lx, self.Ly))
        nb = L.orc_lattice_bonds(self.kind, self.Lx, self.Ly, self.px, self.py, None, None)
        self.bond_a = np.zeros(nb, dtype=np.int64)
        self.bond_b = np.zeros(nb, dtype=np.int64)
        L.orc_lattice_bonds(self.kind, self.Lx, self.Ly, self.px, self.py,
                            _p(self.bond_a, _i64p), _p(self.bond_b, _i64p))
        self.eps = np.zeros(self.N, dtype=np.float64)
        L.orc_onsite(self.N, self.W, self.seed & (2**64 - 1), _p(self.eps, _dp))
        nnz = 2 * nb + self.N
        self.rowptr = np.zeros(self.N + 1, dtype=np.int64)
        self.col = np.zeros(nnz, dtype=np.int64)
        self.val = np.zeros(nnz, dtype=np.float64)
        L.orc_build_csr(self.N, nb, _p(self.bond_a, _i64p), _p(self.bond_b, _i64p),
                        self.t, _p(self.eps, _dp), _p(self.rowptr, _i64p),
                        _p(self.col, _i64p), _p(self.val, _dp))

    @property
    def nbonds(self):
        return len(self.bond_a)

    def degree(self):
        """Number of bond ends at each orbital (repeated bonds counted)."""
        d = np.zeros(self.N, dtype=np.int64)
        np.add.at(d, self.bond_a, 1)
        np.add.at(d, self.bond_b, 1)
        return d

    def halfwidth(self, margin=1.025):
        """|H| = margin * max_s (|eps_s| + deg(s)|t|): Gershgorin's row bound,
        which encloses every eigenvalue, so H~ has its spectrum in [-1, 1]."""
        return margin * float(np.max(np.abs(self.eps) + self.degree() * abs(self.t)))

    def scipy_csr(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.N, self.N))

    def dense(self):
        return self.scipy_csr().toarray()


# ---------------------------------------------------------------- states
def random_phase_states(N: int, R: int, seed: int) -> np.ndarray:
    """psi_r(s) = exp(2 pi i u_{r,s}) / sqrt(N), u from stream r of `seed`.
    Returned as [N][R] (state r is column r)."""
    L = lib()
    u = np.empty((N, R), dtype=np.float64)
    sd = seed & (2**64 - 1)
    for r in range(R):
        for s in range(N):
            u[s, r] = L.orc_u01(L.orc_draw(sd, r, s))
    return np.exp(2j * np.pi * u) / math.sqrt(N)


def random_phase_states_fast(N: int, R: int, seed: int) -> np.ndarray:
    """Vectorised copy of random_phase_states (same draws, numpy uint64
    arithmetic); pinned to the loop version in the tests."""
    G = np.uint64(0x9E3779B97F4A7C15)
    s_idx = np.arange(N, dtype=np.uint64)
    out = np.empty((N, R), dtype=np.complex128)
    with np.errstate(over="ignore"):
        for r in range(R):
            k = (np.uint64(r) << np.uint64(40)) + s_idx
            z = np.uint64(seed & (2**64 - 1)) + (k + np.uint64(1)) * G
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            z = z ^ (z >> np.uint64(31))
            u = (z >> np.uint64(11)).astype(np.float64) * 2.0**-53
            out[:, r] = np.exp(2j * np.pi * u) / math.sqrt(N)
    return out


def ldos_sites(N: int, n_sites: int, seed: int) -> np.ndarray:
    """The first n_sites distinct values floor(bits_i * N / 2^64), i = 0, 1, ...
    of stream 0 of `seed` (the localized states |r> of Sec. III)."""
    if n_sites > N:
        raise ValueError("more sites than orbitals")
    L = lib()
    out, seen, i = [], set(), 0
    sd = seed & (2**64 - 1)
    while len(out) < n_sites:
        s = int(L.orc_below(L.orc_draw(sd, 0, i), N))
        i += 1
        if s not in seen:
            seen.add(s)
            out.append(s)
    return np.array(out, dtype=np.int64)


def site_states(N: int, sites) -> np.ndarray:
    """Unit vectors e_r as columns of an [N][len(sites)] array."""
    out = np.zeros((N, len(sites)), dtype=np.complex128)
    for k, s in enumerate(sites):
        out[s, k] = 1.0
    return out


# ---------------------------------------------------------------- coefficients
def bessel_j(x: float, nmax: int) -> np.ndarray:
    J = np.zeros(nmax + 1, dtype=np.float64)
    rc = lib().orc_bessel_j(float(x), int(nmax), _p(J, _dp))
    if rc:
        raise ValueError("bessel_j failed (%d)" % rc)
    return J


def cheb_coeffs(x: float, nmax: int) -> np.ndarray:
    """c_0 = J_0(x), c_n = 2(-i)^n J_n(x): exp(-i x y) = sum_n c_n T_n(y)."""
    c = np.zeros(nmax + 1, dtype=np.complex128)
    rc = lib().orc_cheb_coeffs(float(x), int(nmax), _p(c.view(np.float64), _dp))
    if rc:
        raise ValueError("cheb_coeffs failed (%d)" % rc)
    return c


def truncation(x: float, eta: float = 1e-14) -> int:
    """N(x): first order above x whose coefficient magnitude is <= eta."""
    n = int(lib().orc_truncation(float(x), float(eta)))
    if n < 0:
        raise ValueError("bad truncation arguments")
    return n


# ---------------------------------------------------------------- propagation
def propagate(lat, psi0, Nt, b=0, Hn=None, H0=0.0, tau=math.pi, eta=1e-14,
              margin=1.025, return_final=False):
    """Correlations <psi0_r|psi_r(t_j)>, j = 0..Nt, as an array [(Nt+1)][R].

    b = 0: sequential form psi(t_j) = exp(-iH tau) psi(t_{j-1}) (Sec. II.A);
    b >= 1: state-based concurrent form in time blocks of b steps (Eq. TE,
    Sec. II.B).  psi0 is [N][R].  Returns (corr, counters) with counters a
    dict of amxsy / axpy / dot counts (Sec. II.B definitions; the t = 0
    correlation is counted under 'dot0').  With return_final=True a third
    item, the final states psi(t_Nt) as [N][R], is returned."""
    psi0 = np.asarray(psi0, dtype=np.complex128)
    if psi0.ndim == 1:
        psi0 = psi0[:, None]
    N, R = psi0.shape
    if N != lat.N:
        raise ValueError("state length does not match the lattice")
    if Hn is None:
        Hn = lat.halfwidth(margin)
    cols = np.ascontiguousarray(psi0.T)
    corr = np.zeros((R, Nt + 1), dtype=np.complex128)
    cnt = np.zeros(4, dtype=np.int64)
    fin = np.zeros((R, N), dtype=np.complex128)
    rc = lib().orc_propagate(N, _p(lat.rowptr, _i64p), _p(lat.col, _i64p), _p(lat.val, _dp),
                             float(H0), float(Hn), R, _p(cols.view(np.float64), _dp),
                             int(Nt), float(tau), float(eta), int(b),
                             _p(corr.view(np.float64), _dp), _p(fin.view(np.float64), _dp),
                             _p(cnt, _i64p))
    if rc:
        raise RuntimeError("orc_propagate failed (%d)" % rc)
    counters = {"amxsy": int(cnt[0]), "axpy": int(cnt[1]),
                "dot": int(cnt[2]), "dot0": int(cnt[3])}
    if return_final:
        return corr.T.copy(), counters, fin.T.copy()
    return corr.T.copy(), counters


def propagate_moments(lat, psi0, Nt, b=None, halving=True, Hn=None, H0=0.0, tau=math.pi,
                      eta=1e-14, margin=1.025, return_final=False):
    """Correlations [(Nt+1)][R] by the moment-based form (Sec. II.A) in
    blocks of b steps (b = None: one block, the DOS-Concurrent-M form of
    Sec. III), optionally with the halving of Eq. (cheby_prod) (one block
    only).  Returns (corr, counters) with counters amxsy (recursion steps),
    axpy (carry updates), dot (moments from inner products) and dot0."""
    psi0 = np.asarray(psi0, dtype=np.complex128)
    if psi0.ndim == 1:
        psi0 = psi0[:, None]
    N, R = psi0.shape
    if N != lat.N:
        raise ValueError("state length does not match the lattice")
    if Hn is None:
        Hn = lat.halfwidth(margin)
    if b is None:
        b = Nt
    cols = np.ascontiguousarray(psi0.T)
    corr = np.zeros((R, Nt + 1), dtype=np.complex128)
    cnt = np.zeros(4, dtype=np.int64)
    fin = np.zeros((R, N), dtype=np.complex128)
    rc = lib().orc_propagate_moments(N, _p(lat.rowptr, _i64p), _p(lat.col, _i64p),
                                     _p(lat.val, _dp), float(H0), float(Hn), R,
                                     _p(cols.view(np.float64), _dp), int(Nt), float(tau),
                                     float(eta), int(b), int(bool(halving)),
                                     _p(corr.view(np.float64), _dp),
                                     _p(fin.view(np.float64), _dp) if return_final else None,
                                     _p(cnt, _i64p))
    if rc:
        raise RuntimeError("orc_propagate_moments failed (%d)" % rc)
    counters = {"amxsy": int(cnt[0]), "axpy": int(cnt[1]),
                "dot": int(cnt[2]), "dot0": int(cnt[3])}
    if return_final:
        return corr.T.copy(), counters, fin.T.copy()
    return corr.T.copy(), counters


class SparseLattice:
    """A Hamiltonian given explicitly in ELL form: row s holds the entries
    (col[s][k], val[s][k]), k < D; col < 0 marks padding.  It is used by
    every propagation routine here exactly as a lattice (CSR rowptr / col /
    val, N), so that general matrices of any density D_H (Sec. II.B) run
    through the same oracle.  pos ([N][2]) and box ((Bx, By), 0 = open) give
    the orbital coordinates for the current operator; displacements are
    taken to the nearest periodic image."""

    def __init__(self, col, val, pos=None, box=(0.0, 0.0)):
        col = np.asarray(col, dtype=np.int64)
        val = np.asarray(val, dtype=np.float64)
        if col.shape != val.shape or col.ndim != 2:
            raise ValueError("col and val must both be [N][D]")
        self.N, self.D = col.shape
        self.ell_col, self.ell_val = col, val
        keep = col >= 0
        counts = keep.sum(1)
        self.rowptr = np.zeros(self.N + 1, dtype=np.int64)
        self.rowptr[1:] = np.cumsum(counts)
        self.col = np.ascontiguousarray(col[keep])
        self.val = np.ascontiguousarray(val[keep])
        self.pos = None if pos is None else np.ascontiguousarray(pos, dtype=np.float64)
        self.box = (float(box[0]), float(box[1]))

    def halfwidth(self, margin=1.025):
        """margin * max_s sum_k |H_sk| (Gershgorin, H0 = 0), the row sum taken
        in k order with plain additions."""
        acc = np.zeros(self.N)
        for k in range(self.D):
            acc = acc + np.where(self.ell_col[:, k] >= 0, np.abs(self.ell_val[:, k]), 0.0)
        return margin * float(acc.max())

    def dense(self):
        H = np.zeros((self.N, self.N))
        for s in range(self.N):
            for p in range(self.rowptr[s], self.rowptr[s + 1]):
                H[s, self.col[p]] += self.val[p]
        return H


def quasi_eigenstates(lat, psi0, Nt, energies, Hn=None, H0=0.0, tau=math.pi, eta=1e-14,
                      margin=1.025):
    """Quasi-eigenstates Psi_r(E) (QE section, Eq. QE) by the sequential form:
    forward and backward propagation by exp(-+iH tau_p) step by step and the
    sum of Eq. QE_coeff over the propagated states,
      Psi(E) = tau_p sum_{j=0}^{Nt} (2 - delta_j0)/2 [e^{iE't_j} psi(t_j) + e^{-iE't_j} psi(-t_j)],
    tau_p = tau / Hn, t_j = j tau_p, E' = E - H0.  The weights are those of
    Eq. QE_coeff as printed (quadrature weight tau_p, no 1/(2 pi)), so Psi(E)
    is 2 pi times the integral of Eq. QE.  psi0 is [N][R]; returns
    ([n_E][N][R] complex, counters)."""
    psi0 = np.asarray(psi0, dtype=np.complex128)
    if psi0.ndim == 1:
        psi0 = psi0[:, None]
    N, R = psi0.shape
    if N != lat.N:
        raise ValueError("state length does not match the lattice")
    if Hn is None:
        Hn = lat.halfwidth(margin)
    E = np.ascontiguousarray(np.asarray(energies, dtype=np.float64).ravel())
    nE = len(E)
    cols = np.ascontiguousarray(psi0.T)
    out = np.zeros((R, nE, N), dtype=np.complex128)
    cnt = np.zeros(4, dtype=np.int64)
    rc = lib().orc_quasi_eigenstates(N, _p(lat.rowptr, _i64p), _p(lat.col, _i64p),
                                     _p(lat.val, _dp), float(H0), float(Hn), R,
                                     _p(cols.view(np.float64), _dp), int(Nt), float(tau),
                                     float(eta), nE, _p(E, _dp), _p(out.view(np.float64), _dp),
                                     _p(cnt, _i64p))
    if rc:
        raise RuntimeError("orc_quasi_eigenstates failed (%d)" % rc)
    counters = {"amxsy": int(cnt[0]), "axpy": int(cnt[1])}
    return np.ascontiguousarray(out.transpose(1, 2, 0)), counters


# ---------------------------------------------------------------- conductivity
def positions(lat):
    """Orbital coordinates [N][2] (conventions in orc_site_positions; for an
    explicit matrix the ones it was given)."""
    if isinstance(lat, SparseLattice):
        if lat.pos is None:
            raise ValueError("explicit matrix without positions")
        return lat.pos.copy()
    x = np.zeros(lat.N)
    y = np.zeros(lat.N)
    lib().orc_site_positions(lat.kind, lat.Lx, lat.Ly, _p(x, _dp), _p(y, _dp))
    return np.stack([x, y], axis=1)


def bond_vectors(lat):
    """r_b - r_a for every bond (a, b) of the lattice, [nbonds][2]."""
    vx = np.zeros(lat.nbonds)
    vy = np.zeros(lat.nbonds)
    n = lib().orc_lattice_bond_vectors(lat.kind, lat.Lx, lat.Ly, lat.px, lat.py,
                                       _p(vx, _dp), _p(vy, _dp))
    assert n == lat.nbonds
    return np.stack([vx, vy], axis=1)


def current(lat, alpha, psi):
    """J_alpha psi with J = i [H, X_alpha] (EC section, hbar = e = 1): from
    the bond list and bond vectors for a lattice, from the CSR matrix and the
    coordinates (nearest image) for an explicit matrix.  psi is [N] or [N][R]."""
    psi = np.asarray(psi, dtype=np.complex128)
    one = psi.ndim == 1
    cols = psi[:, None] if one else psi
    out = np.zeros_like(cols)
    if isinstance(lat, SparseLattice):
        x = np.ascontiguousarray(positions(lat)[:, alpha])
        for r in range(cols.shape[1]):
            v = np.ascontiguousarray(cols[:, r])
            o = np.zeros_like(v)
            lib().orc_current_csr(lat.N, _p(lat.rowptr, _i64p), _p(lat.col, _i64p),
                                  _p(lat.val, _dp), _p(x, _dp), lat.box[alpha],
                                  _p(v.view(np.float64), _dp), _p(o.view(np.float64), _dp))
            out[:, r] = o
    else:
        v_a = np.ascontiguousarray(bond_vectors(lat)[:, alpha])
        for r in range(cols.shape[1]):
            v = np.ascontiguousarray(cols[:, r])
            o = np.zeros_like(v)
            lib().orc_current_bonds(lat.N, lat.nbonds, _p(lat.bond_a, _i64p),
                                    _p(lat.bond_b, _i64p), _p(v_a, _dp), lat.t,
                                    _p(v.view(np.float64), _dp), _p(o.view(np.float64), _dp))
            out[:, r] = o
    return out[:, 0] if one else out


def _ec_inputs(lat, psi0, qe, alpha):
    psi0 = np.asarray(psi0, dtype=np.complex128)
    if psi0.ndim == 1:
        psi0 = psi0[:, None]
    qe = np.asarray(qe, dtype=np.complex128)
    if qe.ndim == 2:
        qe = qe[:, :, None]
    nE, N, R = qe.shape
    if psi0.shape != (N, R) or N != lat.N:
        raise ValueError("shapes: psi0 [N][R], qe [n_E][N][R]")
    Jpsi = current(lat, alpha, psi0)                           # [N][R]
    X = np.stack([current(lat, alpha, qe[e]) for e in range(nE)])   # [nE][N][R]
    nrm = np.abs(np.einsum("sr,esr->er", psi0.conj(), qe))        # [nE][R]
    return psi0, qe, Jpsi, X, nrm


def ec_correlation(lat, psi0, qe, Nt, alpha, Hn=None, H0=0.0, tau=math.pi, eta=1e-14,
                   margin=1.025):
    """EC correlation of Eq. dc_corr by EC-Sequential: C(t_j, E) =
    <psi|J e^{iHt_j} J|Psi(E)> / |<psi|Psi(E)>| = <e^{-iHt_j} J psi|J Psi(E)> /
    |<psi|Psi(E)>|, t_j = j tau / Hn, j = 0..Nt, propagating J psi step by
    step.  psi0 is [N][R], qe the quasi-eigenstates [n_E][N][R].  Returns
    ([n_E][Nt+1][R] complex, counters)."""
    if Hn is None:
        Hn = lat.halfwidth(margin)
    psi0, qe, Jpsi, X, nrm = _ec_inputs(lat, psi0, qe, alpha)
    nE, N, R = qe.shape
    Jc = np.ascontiguousarray(Jpsi.T)                              # [R][N]
    Xc = np.ascontiguousarray(X.transpose(2, 0, 1))                # [R][nE][N]
    nr = np.ascontiguousarray(nrm.T)                               # [R][nE]
    out = np.zeros((R, nE, Nt + 1), dtype=np.complex128)
    cnt = np.zeros(4, dtype=np.int64)
    rc = lib().orc_ec_sequential(N, _p(lat.rowptr, _i64p), _p(lat.col, _i64p),
                                 _p(lat.val, _dp), float(H0), float(Hn), R,
                                 _p(Jc.view(np.float64), _dp), nE, _p(Xc.view(np.float64), _dp),
                                 _p(nr, _dp), int(Nt), float(tau), float(eta),
                                 _p(out.view(np.float64), _dp), _p(cnt, _i64p))
    if rc:
        raise RuntimeError("orc_ec_sequential failed (%d)" % rc)
    return (np.ascontiguousarray(out.transpose(1, 2, 0)),
            {"amxsy": int(cnt[0]), "axpy": int(cnt[1]), "dot": int(cnt[2])})


def ec_moments(lat, psi0, qe, Nt, alpha, Hn=None, H0=0.0, tau=math.pi, eta=1e-14, margin=1.025):
    """EC-Concurrent-M (Eq. dc_mom and the reconstruction after it): moments
    m_n(E) = <J psi|T_n(H~)|J Psi(E)>, n = 0..N(Nt tau), from the Chebyshev
    vectors of J psi (no halving: bra and ket differ), then C(t_j, E) =
    e^{iH0 t_j} sum_{n <= N(j tau)} c_n(j tau)^* m_n(E) / |<psi|Psi(E)>|.
    Returns ([n_E][Nt+1][R] correlations, [N+1][n_E][R] moments)."""
    if Hn is None:
        Hn = lat.halfwidth(margin)
    psi0, qe, Jpsi, X, nrm = _ec_inputs(lat, psi0, qe, alpha)
    nE, N, R = qe.shape
    nmax = truncation(Nt * tau, eta)
    m = np.zeros((nmax + 1, nE, R), dtype=np.complex128)
    for r in range(R):
        phi = chebyshev_vectors(lat, Jpsi[:, r], nmax, Hn, H0)     # [nmax+1][N]
        m[:, :, r] = phi.conj() @ X[:, :, r].T
    corr = np.zeros((nE, Nt + 1, R), dtype=np.complex128)
    tp = tau / Hn
    for j in range(Nt + 1):
        nj = 0 if j == 0 else truncation(j * tau, eta)
        c = cheb_coeffs(j * tau, nj) if j > 0 else np.array([1.0 + 0j])
        corr[:, j, :] = np.exp(1j * H0 * j * tp) * np.einsum("n,ner->er", c.conj(), m[:nj + 1])
    return corr / nrm[:, None, :], m


def ec_sigma(corr, energies, Hn, tau=math.pi, dos_over_area=None):
    """Conductivity integral of Eq. DC on the computed times: sigma(E) =
    D(E)/A * tau_p sum_j w_j Re[e^{-iE t_j} C(t_j, E)], trapezoid weights
    (1/2 at j = 0 and j = Nt), tau_p = tau / Hn.  corr is [n_E][Nt+1][R];
    dos_over_area [n_E] (default 1).  Returns [n_E][R]."""
    corr = np.asarray(corr)
    nE, T, R = corr.shape
    E = np.asarray(energies, dtype=np.float64)
    tp = tau / Hn
    w = np.ones(T)
    w[0] = w[-1] = 0.5
    if T == 1:
        w[0] = 0.0
    ph = np.exp(-1j * np.outer(E, np.arange(T) * tp))                # [nE][T]
    s = tp * np.einsum("t,et,etr->er", w, ph, corr).real
    dA = np.ones(nE) if dos_over_area is None else np.asarray(dos_over_area, dtype=np.float64)
    return dA[:, None] * s


def chebyshev_vectors(lat, x, nmax, Hn, H0=0.0):
    """[T_0(H~)x, ..., T_nmax(H~)x] as an array [nmax+1][N]."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    out = np.zeros((nmax + 1, lat.N), dtype=np.complex128)
    rc = lib().orc_chebyshev_vectors(lat.N, _p(lat.rowptr, _i64p), _p(lat.col, _i64p),
                                     _p(lat.val, _dp), float(H0), float(Hn),
                                     _p(x.view(np.float64), _dp), int(nmax),
                                     _p(out.view(np.float64), _dp))
    if rc:
        raise RuntimeError("orc_chebyshev_vectors failed")
    return out


# ---------------------------------------------------------------- DOS
def hann(Nt):
    j = np.arange(-Nt, Nt)
    return 0.5 * (1.0 + np.cos(np.pi * j / Nt))


def dos(corr, Hn, window="hann", H0=0.0):
    """Density of states from correlations (Sec. III).

    D(E) = (1/2pi) int exp(iEt) C(t) dt with C(-t) = conj C(t), sampled at
    t_j = j tau, tau = pi/|H|, j = -Nt..Nt-1, windowed by w_j, at energies
    E_k = |H| k / Nt, k = -Nt..Nt-1:
        D(E_k) = (tau/2pi) sum_j w_j C_j exp(i pi k j / Nt),
    evaluated as a 2Nt-point inverse FFT.  The correlations of propagate()
    carry the centred propagator exp(-i (H - H0) t) of the rescaled
    expansion (Sec. II.A), so their transform at E_k is the density at the
    true energy H0 + E_k; the returned energies are H0 + E_k.  corr is
    [(Nt+1)][R]; returns (E [2Nt], D [2Nt][R] real, max |Im D| as a
    check)."""
    corr = np.asarray(corr, dtype=np.complex128)
    if corr.ndim == 1:
        corr = corr[:, None]
    Nt = corr.shape[0] - 1
    R = corr.shape[1]
    j = np.arange(-Nt, Nt)
    C = np.where(j[:, None] >= 0, corr[np.abs(j)], np.conj(corr[np.abs(j)]))
    if window == "hann":
        w = hann(Nt)
    elif window == "none":
        w = np.ones(2 * Nt)
    else:
        raise ValueError(window)
    x = w[:, None] * C
    # position m = j mod 2Nt
    xm = np.zeros((2 * Nt, R), dtype=np.complex128)
    xm[j % (2 * Nt)] = x
    S = np.fft.ifft(xm, axis=0) * (2 * Nt)        # S[k] = sum_m xm[m] e^{+2pi i k m / 2Nt}
    k = np.arange(-Nt, Nt)
    tau = math.pi / Hn
    D = (tau / (2 * math.pi)) * S[k % (2 * Nt)]
    E = H0 + Hn * k / Nt
    return E, D.real.copy(), float(np.max(np.abs(D.imag)))


def dos_direct(corr, Hn, window="hann", H0=0.0):
    """The same sum as dos(), written out term by term (small Nt only)."""
    corr = np.asarray(corr, dtype=np.complex128)
    if corr.ndim == 1:
        corr = corr[:, None]
    Nt = corr.shape[0] - 1
    tau = math.pi / Hn
    w = hann(Nt) if window == "hann" else np.ones(2 * Nt)
    E = np.zeros(2 * Nt)
    D = np.zeros((2 * Nt, corr.shape[1]), dtype=np.complex128)
    for ik, k in enumerate(range(-Nt, Nt)):
        E[ik] = H0 + Hn * k / Nt
        for ij, jj in enumerate(range(-Nt, Nt)):
            Cj = corr[jj] if jj >= 0 else np.conj(corr[-jj])
            D[ik] += w[ij] * Cj * np.exp(1j * math.pi * k * jj / Nt)
    return E, (tau / (2 * math.pi)) * D


# ---------------------------------------------------------------- closed forms
def _bloch_modes(kind, Lx, Ly, t, psi):
    """Band energies w_q and weights of a clean periodic lattice such that
    <psi_r|exp(-iHt)|psi_r> = sum_q [P_qr cos(w_q t) - i Q_qr sin(w_q t)].

    square: E(k) = 2t (cos kx + cos ky), P = |psi_k|^2, Q = P E/|E| (so that
    the sum is sum_k |psi_k|^2 exp(-i E_k t)); chain likewise with
    E = 2t cos k.  honeycomb (orbital 2(y Lx + x) + sigma, bonds
    A(x,y)-B(x,y), A(x,y)-B(x-1,y), A(x,y)-B(x,y-1)): the 2x2 Bloch matrix
    [[0, g], [g*, 0]] with g(k) = t (1 + e^{-i k1} + e^{-i k2}) has the
    propagator cos(|g|t) I - i sin(|g|t)/|g| H(k), so w = |g|,
    P = |a_k|^2 + |b_k|^2 and Q = 2 Re(conj(a_k) g b_k)/|g| (0 where g = 0,
    where that term vanishes for every t)."""
    psi = np.asarray(psi, dtype=np.complex128)
    if psi.ndim == 1:
        psi = psi[:, None]
    R = psi.shape[1]
    if kind == "chain":
        E = 2 * t * np.cos(2 * np.pi * np.arange(Lx) / Lx)
        P = np.abs(np.fft.fft(psi, axis=0)) ** 2 / Lx
        w = np.abs(E)
        Q = P * np.sign(E)[:, None]
        return w, P, Q
    if kind == "square":
        kx = 2 * np.pi * np.arange(Lx) / Lx
        ky = 2 * np.pi * np.arange(Ly) / Ly
        E = (2 * t * (np.cos(kx)[None, :] + np.cos(ky)[:, None])).ravel()
        P = np.empty((Lx * Ly, R))
        for r in range(R):
            P[:, r] = (np.abs(np.fft.fft2(psi[:, r].reshape(Ly, Lx))) ** 2).ravel() / (Lx * Ly)
        return np.abs(E), P, P * np.sign(E)[:, None]
    if kind == "honeycomb":
        k1 = 2 * np.pi * np.arange(Lx) / Lx
        k2 = 2 * np.pi * np.arange(Ly) / Ly
        g = (t * (1 + np.exp(-1j * k1)[None, :] + np.exp(-1j * k2)[:, None])).ravel()
        mag = np.abs(g)
        nz = mag > 0
        inv = np.where(nz, 1.0 / np.where(nz, mag, 1.0), 0.0)
        P = np.empty((Lx * Ly, R))
        Q = np.empty((Lx * Ly, R))
        for r in range(R):
            a = psi[:, r].reshape(Ly, Lx, 2)
            ha = (np.fft.fft2(a[:, :, 0]) / math.sqrt(Lx * Ly)).ravel()
            hb = (np.fft.fft2(a[:, :, 1]) / math.sqrt(Lx * Ly)).ravel()
            P[:, r] = np.abs(ha) ** 2 + np.abs(hb) ** 2
            # conj(a) g b + conj(b) conj(g) a = 2 Re(conj(a) g b)
            Q[:, r] = 2.0 * np.real(np.conj(ha) * g * hb) * inv
        return mag, P, Q
    raise ValueError(kind)


def bloch_corr(kind, Lx, Ly, t, psi, times):
    """<psi_r|exp(-iHt)|psi_r> of a clean periodic lattice (chain, square,
    honeycomb) from its band structure, at arbitrary times: H is diagonal in
    crystal momentum (see _bloch_modes).  psi is [N][R]; returns
    [len(times)][R] complex128.  Cost O(N len(times) + N R log N)."""
    w, P, Q = _bloch_modes(kind, Lx, Ly, t, psi)
    times = np.asarray(times, dtype=np.float64)
    out = np.zeros((len(times), P.shape[1]), dtype=np.complex128)
    for i0 in range(0, len(times), 16):
        ph = np.outer(times[i0:i0 + 16], w)
        out[i0:i0 + ph.shape[0]] = np.cos(ph) @ P - 1j * (np.sin(ph) @ Q)
    return out


def bloch_corr_uniform(kind, Lx, Ly, t, psi, tau, n, threads=None):
    """bloch_corr at the n uniform times t_j = j tau, j = 0..n-1.  Blocks of
    16 consecutive times share one table exp(-i w m tau), m < 16, so a block
    costs one exp per mode plus a complex product:
    exp(-i w (j0 + m) tau) = exp(-i w j0 tau) exp(-i w m tau).  With
    C = sum_q [(P+Q)/2 e^{-iwt} + (P-Q)/2 e^{+iwt}] each block is one complex
    matrix product.  Blocks are independent and run on a thread pool."""
    import concurrent.futures as cf
    w, P, Q = _bloch_modes(kind, Lx, Ly, t, psi)
    R = P.shape[1]
    B = 16
    Wm = np.concatenate([(P + Q) / 2, (P - Q) / 2], axis=1).astype(np.complex128)
    step_m = np.exp(-1j * np.outer(np.arange(B) * tau, w))     # [B][q]
    out = np.zeros((n, R), dtype=np.complex128)

    def block(j0):
        m = min(B, n - j0)
        z = step_m[:m] * np.exp(-1j * (j0 * tau) * w)[None, :]
        y = z @ Wm                     # [m][2R]: sum W+ e^{-iwt}, sum W- e^{-iwt}
        out[j0:j0 + m] = y[:, :R] + np.conj(y[:, R:])

    nthr = threads or min(16, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(nthr) as ex:
        list(ex.map(block, range(0, n, B)))
    return out


def bloch_return_amplitude(kind, Lx, Ly, t, tau, n):
    """<r|exp(-iHt_j)|r>, t_j = j tau, j = 0..n-1, of a clean periodic
    lattice.  It is the same for every orbital r (translation symmetry, and
    on the honeycomb the A-B symmetry of the propagator's diagonal
    cos(|g| t)), so the local density of states is site independent."""
    N = orc_sites(kind, Lx, Ly)
    unit = np.zeros((N, 1), dtype=np.complex128)
    unit[0, 0] = 1.0
    return bloch_corr_uniform(kind, Lx, Ly, t, unit, tau, n)[:, 0]


def orc_sites(kind, Lx, Ly):
    return int(lib().orc_lattice_sites(KINDS[kind], Lx, Ly))
