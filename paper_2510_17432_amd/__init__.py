"""Python binding of libcsp: concurrent stochastic propagation on MI355X.

Argument marshalling only: every step runs in the HIP kernels of
``libcsp.so`` (built by ``paper_2510_17432_amd.build``).  PyTorch supplies
device memory and the stream; nothing here computes on the host.  Importing
this package fails loudly if the library has not been built.

The function names follow ``include/csp.h``; see that header for the meaning
of every argument.
"""
import atexit
import ctypes
import math
import os
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libcsp.so is not built; run `python paper_2510_17432_amd/build.py` "
                      "(or __graft_entry__.build()) first")

_lib = ctypes.CDLL(LIB_PATH)

# ------------------------------------------------------------------ constants
CSP_OK, CSP_EINVAL, CSP_ENOMEM, CSP_EHIP, CSP_EUNSUPPORTED, CSP_ENUMERIC = 0, -1, -2, -3, -4, -5
CSP_CHAIN, CSP_SQUARE, CSP_HONEYCOMB, CSP_SPARSE = 0, 1, 2, 3
KINDS = {"chain": CSP_CHAIN, "square": CSP_SQUARE, "honeycomb": CSP_HONEYCOMB}
CSP_C64, CSP_C128 = 0, 1
CSP_FP64_SEQ, CSP_FP64_CONC, CSP_FP32_CONC = 0, 1, 2
MODES = {"fp64_seq": CSP_FP64_SEQ, "fp64_conc": CSP_FP64_CONC, "fp32_conc": CSP_FP32_CONC}
CSP_ASSEMBLE_STATES, CSP_ASSEMBLE_MOMENTS = 0, 1
CSP_WINDOW_HANN, CSP_WINDOW_NONE = 0, 1

_STATUS = {0: "CSP_OK", -1: "CSP_EINVAL", -2: "CSP_ENOMEM", -3: "CSP_EHIP",
           -4: "CSP_EUNSUPPORTED", -5: "CSP_ENUMERIC"}


class CspError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, str(status)), msg))
        self.status = status


# ------------------------------------------------------------------ structs
class LatticeDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("periodic_x", ctypes.c_int32),
                ("periodic_y", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("Lx", ctypes.c_int64), ("Ly", ctypes.c_int64),
                ("t", ctypes.c_double), ("W", ctypes.c_double),
                ("disorder_seed", ctypes.c_uint64), ("bound_margin", ctypes.c_double),
                ("halfwidth_override", ctypes.c_double), ("center", ctypes.c_double)]


class LatticeInfo(ctypes.Structure):
    _fields_ = [("n_orb", ctypes.c_int64), ("rows", ctypes.c_int64),
                ("orb_per_row", ctypes.c_int64), ("H0", ctypes.c_double),
                ("halfwidth", ctypes.c_double), ("gershgorin", ctypes.c_double),
                ("max_degree", ctypes.c_int32), ("has_onsite", ctypes.c_int32),
                ("ell_windowed", ctypes.c_int32), ("ell_max_window", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("Nt", ctypes.c_int64), ("tau_tilde", ctypes.c_double), ("eta", ctypes.c_double),
                ("mode", ctypes.c_int32), ("assembly", ctypes.c_int32),
                ("block_b", ctypes.c_int32), ("chunk_K", ctypes.c_int32),
                ("mem_cap_bytes", ctypes.c_uint64), ("profile", ctypes.c_int32),
                ("check_norm", ctypes.c_int32), ("norm_tol", ctypes.c_double),
                ("graph", ctypes.c_int32), ("reserved1", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("block_b", ctypes.c_int32), ("chunk_K", ctypes.c_int32),
                ("n_blocks", ctypes.c_int32), ("n_groups", ctypes.c_int32),
                ("amxsy", ctypes.c_int64), ("axpy", ctypes.c_int64), ("dot", ctypes.c_int64),
                ("spmm_launches", ctypes.c_int64), ("contract_launches", ctypes.c_int64),
                ("ms_total", ctypes.c_double), ("ms_spmm", ctypes.c_double),
                ("ms_contract", ctypes.c_double), ("spmm_bytes", ctypes.c_double),
                ("contract_bytes", ctypes.c_double), ("contract_flops", ctypes.c_double),
                ("workspace_bytes", ctypes.c_uint64), ("model_cost", ctypes.c_double * 8),
                ("graph_blocks", ctypes.c_int32), ("n_passes", ctypes.c_int32),
                ("spmm_steps", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "model_cost"}
        d["model_cost"] = list(self.model_cost)
        return d


class Tuning(ctypes.Structure):
    _fields_ = [("spmm_vec", ctypes.c_int32), ("spmm_seg_rows", ctypes.c_int32),
                ("contract_wg_per_cu", ctypes.c_int32), ("block_b", ctypes.c_int32),
                ("t_amxsy_us", ctypes.c_double), ("t_order_us", ctypes.c_double * 2),
                ("model_cost_ms", ctypes.c_double * 8), ("n_candidates", ctypes.c_int32),
                ("spmm_steps", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_
             if k not in ("t_order_us", "model_cost_ms")}
        d["t_order_us"] = list(self.t_order_us)
        d["model_cost_ms"] = list(self.model_cost_ms)
        return d


_vp = ctypes.c_void_p
_P = ctypes.POINTER


def _sig(name, args, res=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_sig("csp_abi_version", [])
_sig("csp_last_error", [], ctypes.c_char_p)
_sig("csp_context_create", [ctypes.c_int, _vp, _P(_vp)])
_sig("csp_context_destroy", [_vp])
_sig("csp_context_trim", [_vp])
_sig("csp_lattice_create", [_vp, _P(LatticeDesc), _P(_vp)])
_sig("csp_lattice_create_sparse", [_vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp, ctypes.c_double,
                                   _P(_vp)])
_sig("csp_lattice_set_positions", [_vp, _vp, ctypes.c_double, ctypes.c_double])
_sig("csp_lattice_destroy", [_vp])
_sig("csp_lattice_get_info", [_vp, _P(LatticeInfo)])
_sig("csp_lattice_onsite", [_vp, _vp])
_sig("csp_lattice_neighbors", [_vp, _vp])
_sig("csp_states_random_phase", [_vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                 ctypes.c_int32, _vp, ctypes.c_int32, ctypes.c_int32])
_sig("csp_ldos_sites", [_vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, _vp])
_sig("csp_states_sites", [_vp, ctypes.c_int64, ctypes.c_int32, _vp, ctypes.c_int32, _vp,
                          ctypes.c_int32, ctypes.c_int32])
_sig("csp_chebyshev_coefficients", [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_int32, _vp,
                                    _P(ctypes.c_int32)])
_sig("csp_chebyshev_step", [_vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, ctypes.c_int32])
_sig("csp_propagate", [_vp, _vp, _vp, ctypes.c_int32, _P(Params), _vp, _vp, _P(Report)])
_sig("csp_ec_correlation", [_vp, _vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _P(Params),
                           ctypes.c_int32, _vp, _P(Report)])
_sig("csp_ec_sigma", [_vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                     _P(ctypes.c_double), ctypes.c_double, ctypes.c_double, _P(ctypes.c_double),
                     _vp])
_sig("csp_propagate_batch", [_vp, ctypes.c_int32, _P(_vp), _P(_vp), _P(ctypes.c_int32),
                             _P(Params), _P(_vp), _P(Report)])
_sig("csp_dos", [_vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                 ctypes.c_double, ctypes.c_int32, _vp, _vp, _vp])
_sig("csp_dos_noalloc", [_vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                         ctypes.c_double, ctypes.c_double, ctypes.c_int32, _vp, _vp, _vp])
_sig("csp_select_block", [_vp, _vp, ctypes.c_int32, _P(Params), _P(ctypes.c_int32), _P(Report)])
_sig("csp_quasi_eigenstates", [_vp, _vp, _vp, ctypes.c_int32, _P(Params), ctypes.c_int32,
                               _P(ctypes.c_double), _vp, _P(Report)])
_sig("csp_autotune", [_vp, ctypes.c_int32, _P(_vp), _P(ctypes.c_int32), _P(Params), _P(Tuning)])
_sig("csp_set_tuning", [_vp, ctypes.c_int32, _P(_vp), _P(ctypes.c_int32), _P(Params), _P(Tuning)])
_sig("csp_bandwidth_probe", [_vp, ctypes.c_uint64, _P(ctypes.c_double)])


def _check(rc):
    if rc != CSP_OK:
        raise CspError(rc, _lib.csp_last_error().decode(errors="replace"))


def abi_version():
    return _lib.csp_abi_version()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dtype_code(t):
    import torch
    if t.dtype == torch.complex64:
        return CSP_C64
    if t.dtype == torch.complex128:
        return CSP_C128
    raise TypeError("state blocks must be complex64 or complex128, got %s" % t.dtype)


# ------------------------------------------------------------------ objects
_LIVE_CONTEXTS = weakref.WeakSet()


@atexit.register
def _close_all():
    # Lattices before their context, everything before the HIP runtime and
    # torch's allocator are torn down at interpreter exit.
    for c in list(_LIVE_CONTEXTS):
        try:
            c.close()
        except Exception:
            pass


class Context:
    """csp_context on a device, ordered on a torch stream (default: current).

    A lattice must not outlive the context it was built on: closing the
    context closes its lattices first."""

    def __init__(self, device=0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        self._lattices = weakref.WeakSet()
        h = ctypes.c_void_p()
        _check(_lib.csp_context_create(device, ctypes.c_void_p(stream.cuda_stream),
                                       ctypes.byref(h)))
        self.handle = h
        _LIVE_CONTEXTS.add(self)

    def close(self):
        if self.handle:
            for lat in list(self._lattices):
                lat.close()
            _check(_lib.csp_context_destroy(self.handle))
            self.handle = None

    def trim(self):
        _check(_lib.csp_context_trim(self.handle))

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Lattice:
    """csp_lattice; see csp_lattice_desc for the conventions."""

    def __init__(self, ctx, kind, Lx, Ly=1, t=1.0, W=0.0, disorder_seed=0, periodic_x=True,
                 periodic_y=True, bound_margin=0.0, halfwidth_override=0.0, center=0.0):
        self.ctx = ctx
        d = LatticeDesc()
        d.kind = KINDS[kind] if isinstance(kind, str) else int(kind)
        d.periodic_x, d.periodic_y = int(bool(periodic_x)), int(bool(periodic_y))
        d.Lx, d.Ly = int(Lx), int(Ly)
        d.t, d.W = float(t), float(W)
        d.disorder_seed = int(disorder_seed) & (2**64 - 1)
        d.bound_margin, d.halfwidth_override, d.center = (float(bound_margin),
                                                           float(halfwidth_override), float(center))
        self.desc = d
        h = ctypes.c_void_p()
        _check(_lib.csp_lattice_create(ctx.handle, ctypes.byref(d), ctypes.byref(h)))
        self._finish(ctx, h)

    def _finish(self, ctx, h):
        self.handle = h
        ctx._lattices.add(self)
        info = LatticeInfo()
        _check(_lib.csp_lattice_get_info(h, ctypes.byref(info)))
        self.info = info
        self.N = info.n_orb
        self.halfwidth = info.halfwidth

    @classmethod
    def sparse(cls, ctx, col, val, margin=0.0):
        """Explicit Hamiltonian in ELL form: host arrays col (int32, [N][D],
        negative = padding) and val (float64, [N][D]); see
        csp_lattice_create_sparse."""
        import numpy as np
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        if col.ndim != 2 or col.shape != val.shape:
            raise ValueError("col and val must both be [N][D]")
        self = cls.__new__(cls)
        self.ctx = ctx
        self.desc = None
        h = ctypes.c_void_p()
        _check(_lib.csp_lattice_create_sparse(
            ctx.handle, col.shape[0], col.shape[1], col.ctypes.data_as(_vp),
            val.ctypes.data_as(_vp), float(margin), ctypes.byref(h)))
        self._finish(ctx, h)
        return self

    def set_positions(self, pos, box=(0.0, 0.0)):
        """Orbital coordinates [N][2] of an explicit matrix and its periodic
        box (0 = open); see csp_lattice_set_positions."""
        import numpy as np
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        if pos.shape != (self.N, 2):
            raise ValueError("pos must be [N][2]")
        _check(_lib.csp_lattice_set_positions(self.handle, pos.ctypes.data_as(_vp),
                                              float(box[0]), float(box[1])))

    def onsite(self):
        import torch
        out = torch.empty(self.N, dtype=torch.float64, device="cuda:%d" % self.ctx.device)
        _check(_lib.csp_lattice_onsite(self.handle, _ptr(out)))
        self.ctx.stream.synchronize()
        return out

    def neighbors(self):
        import torch
        out = torch.empty((self.N, self.info.max_degree), dtype=torch.int64,
                          device="cuda:%d" % self.ctx.device)
        _check(_lib.csp_lattice_neighbors(self.handle, _ptr(out)))
        self.ctx.stream.synchronize()
        return out

    def close(self):
        if getattr(self, "handle", None):
            if not self.ctx.handle:
                raise CspError(CSP_EINVAL, "lattice outlived its context")
            _check(_lib.csp_lattice_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ states
def csp_states_random_phase(ctx, psi, R, seed, col0=0):
    """Fill columns col0..col0+R-1 of the [N][ld] complex tensor psi."""
    N, ld = psi.shape
    _check(_lib.csp_states_random_phase(ctx.handle, N, R, int(seed) & (2**64 - 1),
                                        _dtype_code(psi), _ptr(psi), ld, col0))


def csp_ldos_sites(ctx, N, n, seed):
    import torch
    out = torch.empty(n, dtype=torch.int64, device="cuda:%d" % ctx.device)
    _check(_lib.csp_ldos_sites(ctx.handle, N, n, int(seed) & (2**64 - 1), _ptr(out)))
    return out


def csp_states_sites(ctx, psi, sites, col0=0):
    N, ld = psi.shape
    _check(_lib.csp_states_sites(ctx.handle, N, int(sites.numel()), _ptr(sites),
                                 _dtype_code(psi), _ptr(psi), ld, col0))


def csp_chebyshev_coefficients(ctx, x, nmax, eta=1e-14):
    """Returns (complex128 tensor c[0..nmax], truncation order N(x))."""
    import torch
    out = torch.empty(nmax + 1, dtype=torch.complex128, device="cuda:%d" % ctx.device)
    n = ctypes.c_int32()
    _check(_lib.csp_chebyshev_coefficients(ctx.handle, float(x), float(eta), int(nmax),
                                           _ptr(out), ctypes.byref(n)))
    return out, n.value


def csp_chebyshev_step(ctx, lat, x, y, first=False):
    """first: y = H~ x; else y = 2 H~ x - y.  x, y: [N][R] complex tensors."""
    N, R = x.shape
    _check(_lib.csp_chebyshev_step(ctx.handle, lat.handle, R, _dtype_code(x), _ptr(x), _ptr(y),
                                   int(bool(first))))


def make_params(Nt, mode="fp32_conc", block_b=0, chunk_K=0, tau_tilde=math.pi, eta=1e-14,
                assembly=CSP_ASSEMBLE_STATES, mem_cap_bytes=0, profile=False, check_norm=False,
                norm_tol=0.0, graph=0):
    p = Params()
    p.Nt = int(Nt)
    p.tau_tilde = float(tau_tilde)
    p.eta = float(eta)
    p.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    p.assembly = int(assembly)
    p.block_b = int(block_b)
    p.chunk_K = int(chunk_K)
    p.mem_cap_bytes = int(mem_cap_bytes)
    p.profile = int(bool(profile))
    p.check_norm = int(bool(check_norm))
    p.norm_tol = float(norm_tol)
    p.graph = int(graph)
    return p


def csp_propagate(ctx, lat, psi0, params, corr=None, final=None):
    """Correlations [(Nt+1)][R] complex128 (device tensor) and the report."""
    import torch
    N, R = psi0.shape
    if corr is None:
        corr = torch.empty((params.Nt + 1, R), dtype=torch.complex128, device=psi0.device)
    rep = Report()
    _check(_lib.csp_propagate(ctx.handle, lat.handle, _ptr(psi0), R, ctypes.byref(params),
                              _ptr(corr), _ptr(final), ctypes.byref(rep)))
    return corr, rep


def csp_quasi_eigenstates(ctx, lat, psi0, params, energies, out=None):
    """Quasi-eigenstates [n_E][N][R] (device tensor, dtype of psi0) and the
    report, by the energy-based concurrent form."""
    import torch
    N, R = psi0.shape
    E = [float(e) for e in energies]
    if out is None:
        out = torch.empty((len(E), N, R), dtype=psi0.dtype, device=psi0.device)
    Ev = (ctypes.c_double * len(E))(*E)
    rep = Report()
    _check(_lib.csp_quasi_eigenstates(ctx.handle, lat.handle, _ptr(psi0), R,
                                      ctypes.byref(params), len(E), Ev, _ptr(out),
                                      ctypes.byref(rep)))
    return out, rep


def csp_ec_correlation(ctx, lat, alpha, psi0, qe, params, corr=None):
    """EC correlation (Eq. dc_corr) by EC-Concurrent-M: [n_E][Nt+1][R]
    complex128 (device tensor) and the report.  psi0 [N][R], qe [n_E][N][R]
    (from csp_quasi_eigenstates), dtype per mode."""
    import torch
    N, R = psi0.shape
    nE = qe.shape[0]
    if tuple(qe.shape) != (nE, N, R) or qe.dtype != psi0.dtype:
        raise ValueError("qe must be [n_E][N][R] of the dtype of psi0")
    if corr is None:
        corr = torch.empty((nE, params.Nt + 1, R), dtype=torch.complex128, device=psi0.device)
    rep = Report()
    _check(_lib.csp_ec_correlation(ctx.handle, lat.handle, int(alpha), _ptr(psi0), R, _ptr(qe),
                                   ctypes.byref(params), nE, _ptr(corr), ctypes.byref(rep)))
    return corr, rep


def csp_ec_sigma(ctx, corr, halfwidth, energies, tau_tilde=math.pi, dos_over_area=None):
    """Conductivity of Eq. DC from csp_ec_correlation's output: [n_E][R] FP64."""
    import torch
    nE, T, R = corr.shape
    E = [float(e) for e in energies]
    if len(E) != nE:
        raise ValueError("one energy per row of corr")
    Ev = (ctypes.c_double * nE)(*E)
    dA = None if dos_over_area is None else (ctypes.c_double * nE)(*[float(x) for x in dos_over_area])
    out = torch.empty((nE, R), dtype=torch.float64, device=corr.device)
    _check(_lib.csp_ec_sigma(ctx.handle, _ptr(corr), T - 1, R, nE, Ev, float(halfwidth),
                             float(tau_tilde), dA, _ptr(out)))
    return out


def csp_propagate_batch(ctx, lats, psi0s, params, corrs=None):
    import torch
    n = len(lats)
    if corrs is None:
        corrs = [torch.empty((params.Nt + 1, p.shape[1]), dtype=torch.complex128,
                             device=p.device) for p in psi0s]
    L = (ctypes.c_void_p * n)(*[l.handle.value for l in lats])
    P = (ctypes.c_void_p * n)(*[p.data_ptr() for p in psi0s])
    Rs = (ctypes.c_int32 * n)(*[p.shape[1] for p in psi0s])
    C = (ctypes.c_void_p * n)(*[c.data_ptr() for c in corrs])
    rep = Report()
    _check(_lib.csp_propagate_batch(ctx.handle, n, L, P, Rs, ctypes.byref(params), C,
                                    ctypes.byref(rep)))
    return corrs, rep


def csp_dos(ctx, corr, halfwidth, tau_tilde=math.pi, window=CSP_WINDOW_HANN, center=0.0):
    """(E [2Nt], D [2Nt][R], Dmean [2Nt]) as float64 device tensors; center is
    the lattice's spectral centre H0 (the energies are center + E_k)."""
    import torch
    Nt = corr.shape[0] - 1
    R = corr.shape[1]
    dev = corr.device
    E = torch.empty(2 * Nt, dtype=torch.float64, device=dev)
    D = torch.empty((2 * Nt, R), dtype=torch.float64, device=dev)
    Dm = torch.empty(2 * Nt, dtype=torch.float64, device=dev)
    _check(_lib.csp_dos(ctx.handle, _ptr(corr), Nt, R, float(halfwidth), float(center),
                        float(tau_tilde), int(window), _ptr(E), _ptr(D), _ptr(Dm)))
    return E, D, Dm


def csp_dos_noalloc(ctx, corr, halfwidth, E, D, Dmean=None, tau_tilde=math.pi,
                    window=CSP_WINDOW_HANN, center=0.0):
    """csp_dos into caller-owned float64 device tensors E [2Nt], D [2Nt][R]
    and Dmean [2Nt] (or None); the library allocates nothing and does not
    synchronise the stream."""
    Nt = corr.shape[0] - 1
    R = corr.shape[1]
    _check(_lib.csp_dos_noalloc(ctx.handle, _ptr(corr), Nt, R, float(halfwidth), float(center),
                                float(tau_tilde), int(window), _ptr(E), _ptr(D), _ptr(Dmean)))


def csp_select_block(ctx, lat, R, params):
    b = ctypes.c_int32()
    rep = Report()
    _check(_lib.csp_select_block(ctx.handle, lat.handle, R, ctypes.byref(params),
                                 ctypes.byref(b), ctypes.byref(rep)))
    return b.value, rep


def csp_autotune(ctx, lats, Rs, params):
    """Measure launch shapes and the block size for these instances (cached in
    the context for later propagations of the same shape)."""
    n = len(lats)
    L = (ctypes.c_void_p * n)(*[l.handle.value for l in lats])
    Rv = (ctypes.c_int32 * n)(*[int(r) for r in Rs])
    t = Tuning()
    _check(_lib.csp_autotune(ctx.handle, n, L, Rv, ctypes.byref(params), ctypes.byref(t)))
    return t


def csp_set_tuning(ctx, lats, Rs, params, tuning):
    """Install a tuning record for the shape of these instances."""
    n = len(lats)
    L = (ctypes.c_void_p * n)(*[l.handle.value for l in lats])
    Rv = (ctypes.c_int32 * n)(*[int(r) for r in Rs])
    _check(_lib.csp_set_tuning(ctx.handle, n, L, Rv, ctypes.byref(params), ctypes.byref(tuning)))


def csp_bandwidth_probe(ctx, nbytes=1 << 30):
    """Streaming GB/s of this device: (read only, write only, 2 reads + 1 write)."""
    out = (ctypes.c_double * 3)()
    _check(_lib.csp_bandwidth_probe(ctx.handle, int(nbytes), out))
    return tuple(out)
