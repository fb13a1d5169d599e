/*
 * csp.h -- concurrent stochastic propagation on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libcsp.  The library evaluates exp(-i H t) applied to blocks of
 * random-phase (or localized) states of a sparse tight-binding Hamiltonian by
 * a Chebyshev expansion (arXiv:2510.17432, Sec. II.A and App. B), assembles
 * the states at many time points from blocks of Chebyshev vectors
 * (state-based concurrent form, Eq. (TE), with the time blocks of Sec. II.B),
 * reduces them to the correlation functions C(t_j) = <psi0|psi(t_j)> and
 * turns those into the density of states (Sec. III).
 *
 * Conventions shared by every entry point:
 *   - Every function returns a csp_status; 0 is success.  Nothing throws
 *     across the ABI.  On failure csp_last_error() returns a message that is
 *     local to the calling thread and valid until its next csp_* call.
 *   - "dev_" pointers are device pointers on the context's device; "host"
 *     pointers are ordinary host memory.  The caller owns every buffer it
 *     passes in; the library owns contexts, lattices and its workspace.
 *   - State blocks are laid out [N][ld]: orbital-major, the ld columns of one
 *     orbital contiguous, each value an interleaved complex number
 *     (re, im) of the stated dtype.  Columns col0 .. col0+R-1 are used.
 *   - Correlations are complex128 laid out [(Nt+1)][R] (time-major).
 *   - All work is ordered on the context's HIP stream.  Calls that return
 *     values to the host synchronise that stream before returning.
 *   - Sizes are int64 wherever an orbital count can exceed 2^31.
 */
#ifndef CSP_H
#define CSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CSP_ABI_VERSION 3

typedef enum {
    CSP_OK = 0,
    CSP_EINVAL = -1,        /* bad argument, shape or combination */
    CSP_ENOMEM = -2,        /* device memory (or the given cap) too small */
    CSP_EHIP = -3,          /* a HIP runtime call failed */
    CSP_EUNSUPPORTED = -4,  /* valid request this build does not implement */
    CSP_ENUMERIC = -5       /* non-finite value or norm guard tripped */
} csp_status;

typedef enum {
    CSP_CHAIN = 0, CSP_SQUARE = 1, CSP_HONEYCOMB = 2,
    CSP_SPARSE = 3       /* matrix given explicitly (csp_lattice_create_sparse) */
} csp_lattice_kind;

/* Value type of a state block. */
typedef enum { CSP_C64 = 0 /* complex float */, CSP_C128 = 1 /* complex double */ } csp_dtype;

/* How the propagation is carried out (Sec. II.A, Sec. II.B, Sec. III). */
typedef enum {
    /* Sequential form: psi(t_j) = exp(-i H tau) psi(t_{j-1}), each step a
     * Chebyshev expansion of order N(tau); complex128 throughout.  This is
     * the plain form the concurrent method is compared against. */
    CSP_FP64_SEQ = 0,
    /* State-based concurrent form in time blocks, complex128 throughout;
     * the block contraction uses FP64 fused multiply-adds. */
    CSP_FP64_CONC = 1,
    /* State-based concurrent form: complex64 Chebyshev recursion, block
     * contraction on MFMA in split-bfloat16 (three products, FP32
     * accumulation), carried block-final state in FP32, correlations
     * finished in FP64.  psi0 must be complex64. */
    CSP_FP32_CONC = 2
} csp_mode;

/* How correlations are taken from a block of Chebyshev vectors. */
typedef enum {
    /* Assemble psi(t_j) = sum_n c_n(j tau) T_n(H~) s_k for every j of the
     * block (Eq. TE) and reduce <psi0|psi(t_j)> in the same kernel. */
    CSP_ASSEMBLE_STATES = 0,
    /* Moment-based form (Sec. II.A): reduce the block moments
     * mu_n = <psi0|T_n(H~) s_k> in the recursion kernel's epilogue and form
     * C(t_j) = sum_n c_n(j tau) mu_n in FP64; four Chebyshev vectors per
     * column are kept (phi_n, phi_{n-1} and the two newest orders of a
     * recursion launch) besides psi0.  With one block (block_b = 0 or >= Nt) and no final
     * state requested this is DOS-Concurrent-M of Sec. III with the halving
     * identity of Eq. (cheby_prod): mu_0 and mu_1 are reduced against psi0,
     * every other moment from mu_2k = 2<phi_k|phi_k> - mu_0 and
     * mu_2k+1 = 2<phi_k+1|phi_k> - mu_1 (the paper takes mu_n up to N/2
     * directly; the identity is the same), so only N/2 recursion steps run
     * and psi0 is read once.  With several blocks the recursion
     * epilogue also accumulates the carried state.  Same correlations as
     * CSP_ASSEMBLE_STATES up to rounding. */
    CSP_ASSEMBLE_MOMENTS = 1
} csp_assembly;

typedef enum { CSP_WINDOW_HANN = 0, CSP_WINDOW_NONE = 1 } csp_window;

/* Lattice description.  Orbital order: chain s = ix; square s = iy*Lx+ix;
 * honeycomb s = 2*(iy*Lx+ix)+sigma (sigma 0 = A, 1 = B) with bonds
 * A(ix,iy)-B(ix,iy), A(ix,iy)-B(ix-1,iy), A(ix,iy)-B(ix,iy-1).  H_ab = t on
 * every bond (bonds that repeat on small periodic lattices add),
 * H_ss = W*(u_s - 1/2) with u_s the SplitMix64 draw s of stream 0 of
 * disorder_seed mapped to [0,1) by its top 53 bits. */
typedef struct {
    int32_t kind;              /* csp_lattice_kind */
    int32_t periodic_x;        /* nonzero: wrap in x */
    int32_t periodic_y;        /* nonzero: wrap in y (ignored for chains) */
    int32_t reserved0;
    int64_t Lx, Ly;            /* cells; Ly ignored for chains */
    double t;                  /* hopping */
    double W;                  /* Anderson disorder width (0: clean) */
    uint64_t disorder_seed;
    double bound_margin;       /* |H| = margin * Gershgorin bound; 0 -> 1.025 */
    double halfwidth_override; /* > 0: use this |H| instead */
    double center;             /* spectral centre H0 (Sec. II.A) */
} csp_lattice_desc;

typedef struct {
    int64_t n_orb;             /* N */
    int64_t rows;              /* Ly (1 for chains) */
    int64_t orb_per_row;       /* Lx (chain, square) or 2*Lx (honeycomb) */
    double H0, halfwidth;      /* rescaling H~ = (H - H0)/halfwidth */
    double gershgorin;         /* max_s |eps_s - H0| + deg(s)|t| */
    int32_t max_degree;        /* 2, 4 or 3 bond ends per orbital */
    int32_t has_onsite;        /* W != 0 */
    int32_t ell_windowed;      /* explicit matrix: its recursion stages each
                                  slice's window of phi_n in LDS (see
                                  csp_lattice_create_sparse) */
    int32_t ell_max_window;    /* explicit matrix, windowed: largest window */
} csp_lattice_info;

typedef struct {
    int64_t Nt;                /* time steps; correlations for j = 0..Nt */
    double tau_tilde;          /* rescaled step |H|*tau; 0 -> pi (Sec. II.A) */
    double eta;                /* truncation threshold; 0 -> 1e-14 */
    int32_t mode;              /* csp_mode */
    int32_t assembly;          /* csp_assembly */
    int32_t block_b;           /* time-block size; 0 -> the selection rule
                                  (state assembly) or one block (moment
                                  assembly); the sequential mode uses 1 */
    int32_t chunk_K;           /* Chebyshev vectors kept per contraction;
                                  0 -> as many as fit (multiple of 16) */
    uint64_t mem_cap_bytes;    /* workspace cap; 0 -> free device memory */
    int32_t profile;           /* nonzero: time kernel classes with events */
    int32_t check_norm;        /* nonzero: after every time block check on the
                                  GPU that the carried state kept the norm of
                                  psi0 (the propagator is unitary) and that
                                  every new correlation is finite with
                                  |C_j| <= (1 + norm_tol) <psi0|psi0>;
                                  a violation makes the call return
                                  CSP_ENUMERIC naming the first failing block */
    double norm_tol;           /* relative tolerance of the guard; 0 -> 1e-3 */
    int32_t graph;             /* state assembly: capture one time block's
                                  launches in a HIP graph and replay it for
                                  every full block; 0 = on for
                                  csp_propagate_batch, off for csp_propagate;
                                  1 = on; -1 = off.  Ignored when profile is
                                  set.  If capture fails the launches are
                                  issued directly (same results). */
    int32_t reserved1;
} csp_params;

/* What a propagation did.  Operation counts are per state column and follow
 * the definitions of Sec. II.B and Tab. (cost): amxsy = Chebyshev recursion
 * steps; axpy = (n, j) coefficient pairs of the block sums (state assembly)
 * or carry updates (moment assembly); dot = correlations after t = 0 (state
 * assembly) or moments taken from inner products (moment assembly). */
typedef struct {
    int32_t block_b, chunk_K, n_blocks, n_groups;
    int64_t amxsy, axpy, dot;
    int64_t spmm_launches, contract_launches;
    double ms_total;           /* host wall time of the call */
    double ms_spmm;            /* event time of recursion kernels (profile) */
    double ms_contract;        /* event time of contraction kernels (profile) */
    double spmm_bytes;         /* algorithmic bytes of all recursion steps */
    double contract_bytes;     /* algorithmic bytes of all contractions */
    double contract_flops;     /* MFMA (or FMA) flops of all contractions */
    uint64_t workspace_bytes;
    double model_cost[8];      /* selection-rule cost of b = 1,2,4,...,128 */
    int32_t graph_blocks;      /* time blocks replayed from a HIP graph */
    int32_t n_passes;          /* column windows run one after another
                                  because all columns at once exceed the
                                  memory cap (1 = all columns together) */
    int32_t spmm_steps;        /* Chebyshev steps per recursion launch (the
                                  last launch of a block may do fewer) */
    int32_t reserved;
} csp_report;

/* Launch shapes and time-block size measured by csp_autotune. */
typedef struct {
    int32_t spmm_vec;          /* complex values per lane in a recursion
                                  strip (one wavefront covers 64 * vec
                                  consecutive values of a lattice row) */
    int32_t spmm_seg_rows;     /* lattice rows per recursion work item */
    int32_t contract_wg_per_cu;/* contraction workgroups per compute unit */
    int32_t block_b;           /* time-block size from the cost model (state
                                  assembly; 0 for the moment assembly, which
                                  always runs one block) */
    double t_amxsy_us;         /* one recursion step over all columns, best
                                  shape (launch time / spmm_steps) */
    double t_order_us[2];      /* contraction time per Chebyshev order for
                                  b <= 32 and b <= 64 (state assembly) */
    double model_cost_ms[8];   /* modelled propagation time at
                                  b = 1, 2, 4, ..., 128; -1 where b is not
                                  allowed or does not fit */
    int32_t n_candidates;      /* recursion shapes timed */
    int32_t spmm_steps;        /* Chebyshev steps per recursion launch
                                  (orders kept in registers between steps) */
} csp_tuning;

typedef struct csp_context csp_context;
typedef struct csp_lattice csp_lattice;

/* Library ABI version (CSP_ABI_VERSION). */
int csp_abi_version(void);

/* Thread-local message describing the last failure of this thread. */
const char *csp_last_error(void);

/* Create a context on HIP device `device` whose work is ordered on
 * `hip_stream` (a hipStream_t; NULL = the null stream).  The stream stays
 * owned by the caller and must outlive the context. */
csp_status csp_context_create(int device, void *hip_stream, csp_context **out);
csp_status csp_context_destroy(csp_context *ctx);

/* Build a lattice on the context's device: on-site energies (FP64 and an
 * FP32 copy) by the generator above and the half-width |H| by Gershgorin's
 * row bound times the margin, reduced on the GPU in FP64 (Sec. II.A asks
 * for H0 and |H|; it obtains them by Lanczos).  A lattice has at most
 * 2^31 - 1 orbitals (CSP_EUNSUPPORTED beyond). */
csp_status csp_lattice_create(csp_context *ctx, const csp_lattice_desc *desc,
                              csp_lattice **out);
/* A Hamiltonian given explicitly, for matrices of any density D_H (Sec. II.B;
 * the paper's speedups are measured at D_H = 60..230): N orbitals, D entries
 * per row in ELL form, row s holding (col[s*D+k], val[s*D+k]) for k < D;
 * col < 0 marks padding (its val is ignored).  The matrix must be real
 * symmetric (not checked).  Host arrays, copied (the caller keeps them) to
 * the device in slices of 128 rows, [N/128][D][128], with the values in
 * FP64 and FP32.  H0 = 0 and |H| = margin * max_s sum_k |val_sk|
 * (Gershgorin, reduced on the GPU in FP64; margin <= 0 selects 1.025).
 * Such a lattice runs through every propagation entry point; its recursion
 * applies one Chebyshev step per launch (a gathered sparse product).  When
 * at least half of the slices of 128 rows, regrouped to be compact in the
 * matrix graph, name at most 2048 distinct columns that each serve four or
 * more entries, a second, windowed copy of the matrix is kept (rows per
 * slice, 16-bit window-local and 32-bit global columns, FP64 and FP32
 * values: 18 B per entry, rows padded to a multiple of 4 entries, besides
 * the 16 of the slice layout) and the recursion stages each slice's window
 * of phi_n in LDS; csp_lattice_get_info reports it.  Otherwise, in complex64 a
 * call on it keeps, per group of Rg columns, two orbital-major copies of
 * floor(Rg/2) column pairs (32 floor(Rg/2) N bytes) in context memory
 * outside mem_cap_bytes, released by csp_context_trim.
 * csp_lattice_onsite and csp_lattice_neighbors return CSP_EUNSUPPORTED for
 * it.  Errors: CSP_EINVAL for N outside [1, 2^31), D outside [1, 4096], a
 * column index >= N, a non-finite value or an all-zero matrix; CSP_ENOMEM
 * when the device cannot hold the 16 D N bytes of the matrix (about 34 D N
 * with the windowed copy). */
csp_status csp_lattice_create_sparse(csp_context *ctx, int64_t N, int32_t D, const int32_t *col,
                                     const double *val, double margin, csp_lattice **out);
/* Orbital coordinates of an explicit matrix, for the current operator
 * (EC section): pos [N][2] (x, y) host array, copied; box_x, box_y the
 * periodic box lengths (0 = open direction); displacements between two
 * orbitals are taken to the nearest image.  CSP_EUNSUPPORTED for stencil
 * lattices, whose coordinates are fixed (chain: site ix at (ix, 0); square:
 * (ix, iy); honeycomb with unit C-C distance: cell (ix, iy) at
 * ix a1 + iy a2, a1 = (sqrt3, 0), a2 = (sqrt3/2, 3/2), orbital A at the cell
 * origin and B at + (sqrt3/2, 1/2)); CSP_EINVAL for non-finite values or a
 * negative box. */
csp_status csp_lattice_set_positions(csp_lattice *lat, const double *pos, double box_x,
                                     double box_y);
csp_status csp_lattice_destroy(csp_lattice *lat);
csp_status csp_lattice_get_info(const csp_lattice *lat, csp_lattice_info *out);

/* Copy the FP64 on-site energies into dev_eps[N]. */
csp_status csp_lattice_onsite(const csp_lattice *lat, double *dev_eps);

/* Write the neighbour table dev_nbr[N][max_deg] (int64 orbital indices, -1
 * where a bond is absent at an open edge; repeated bonds appear twice), in
 * the order left, right, down, up (square), left, right (chain) or
 * B(ix), B(ix-1), B(iy-1) for A and A(ix), A(ix+1), A(iy+1) for B. */
csp_status csp_lattice_neighbors(const csp_lattice *lat, int64_t *dev_nbr);

/* Random-phase states (Sec. II.A; phases uniform, norm 1):
 * psi_r(s) = exp(2 pi i u_{r,s}) / sqrt(N), u_{r,s} from stream r of `seed`,
 * written into columns col0+r of the [N][ld] block dev_psi (dtype C64 or
 * C128; C64 values are the FP64 values rounded). */
csp_status csp_states_random_phase(csp_context *ctx, int64_t N, int32_t R, uint64_t seed,
                                   int32_t dtype, void *dev_psi, int32_t ld, int32_t col0);

/* Localized sites for the LDOS (Sec. III): the first n distinct values
 * floor(bits_i * N / 2^64) of stream 0 of `seed`, into dev_sites[n]. */
csp_status csp_ldos_sites(csp_context *ctx, int64_t N, int32_t n, uint64_t seed,
                          int64_t *dev_sites);

/* Unit vectors e_{sites[k]} into columns col0+k of dev_psi (other entries of
 * those columns are zeroed). */
csp_status csp_states_sites(csp_context *ctx, int64_t N, int32_t n, const int64_t *dev_sites,
                            int32_t dtype, void *dev_psi, int32_t ld, int32_t col0);

/* Chebyshev coefficients of exp(-i x y) on [-1, 1] (App. B):
 * c_0 = J_0(x), c_n = 2(-i)^n J_n(x), computed on the GPU in FP64 with
 * Miller's backward recurrence; writes complex128 dev_c[0..nmax].  If
 * n_trunc is not NULL it receives the truncation order N(x) for threshold
 * eta (Sec. II.A: the first order above x whose coefficient is <= eta). */
csp_status csp_chebyshev_coefficients(csp_context *ctx, double x, double eta, int32_t nmax,
                                      double *dev_c, int32_t *n_trunc);

/* One Chebyshev recursion step on an [N][R] block (amxsy, Sec. II.B):
 * first != 0: y = H~ x; otherwise y = 2 H~ x - y.  dtype C64 or C128,
 * 1 <= R <= 64, x and y distinct. */
csp_status csp_chebyshev_step(csp_context *ctx, const csp_lattice *lat, int32_t R,
                              int32_t dtype, const void *dev_x, void *dev_y, int32_t first);

/* Propagate the R states dev_psi0 ([N][R], dtype per mode) for Nt steps of
 * the rescaled size params->tau_tilde and write the correlations
 * dev_corr[(Nt+1)][R] (complex128, device) with
 * C_r(t_j) = <psi0_r|psi_r(t_j)>, psi_r(t_j) = exp(-i H~ j tau~) psi0_r: the
 * propagator is the Chebyshev expansion of exp(-i H~ tau~) of Sec. II.A, so
 * with a spectral centre H0 != 0 the states and correlations carry
 * exp(-i (H - H0) t_j), i.e. C_r(t_j) = exp(i H0 t_j) <psi0_r|exp(-i H t_j)|psi0_r>
 * (csp_dos takes H0 as its centre to place the DOS on the true energies).
 * dev_final (may be NULL) receives psi(t_Nt) in the layout and dtype of
 * psi0.  rep may be NULL. */
csp_status csp_propagate(csp_context *ctx, const csp_lattice *lat, const void *dev_psi0,
                         int32_t R, const csp_params *params, double *dev_corr,
                         void *dev_final, csp_report *rep);

/* Quasi-eigenstates (QE section), the energy-based concurrent form
 * QE-Concurrent-E: for each of the R states psi0_r (dev_psi0, [N][R], dtype
 * per mode) and each of the n_E energies (host array, units of t), with
 * tau = params->tau_tilde / |H|, t_j = j tau, E' = E - H0,
 *   Psi_r(E) = sum_{n=0}^{N(Nt tau~)} C_n(E) T_n(H~) psi0_r,
 *   C_n(E) = tau [ delta_n0 + sum_{j=1..Nt, n <= N(j tau~)}
 *                  2 a_n(j tau~) Re((-i)^n e^{i E' t_j}) ]
 * (a_0 = J_0, a_n = 2 J_n): the forward and backward time sums of Eq. QE
 * merged as in Eq. QE_coeff, no window.  This equals
 * tau sum_{j=0}^{Nt} (2 - delta_j0)/2 [e^{iE't_j} psi(t_j) + e^{-iE't_j} psi(-t_j)]
 * of the sequentially propagated states up to rounding.  This is Eq. QE_coeff
 * as printed: its quadrature weight is tau with no factor 1/(2 pi), so
 * Psi(E) is 2 pi times the integral of Eq. QE (the factor cancels in the
 * normalised conductivity correlation).  Writes dev_qe
 * [n_E][N][R] in the dtype of psi0.  params->mode CSP_FP32_CONC (complex64
 * recursion, split-bf16 MFMA accumulation) or CSP_FP64_CONC (complex128);
 * 1 <= n_E <= 128 (one recursion serves all energies, contracted in tiles of
 * 32 or 16 energies); 1 <= Nt <= 2^20.  Coefficients are FP64 on
 * the GPU.  CSP_ENOMEM when a 16-order ring of all columns with the n_E
 * accumulated states does not fit (call per column then).  rep may be NULL.
 * params->block_b >= 1 selects the state-based form QE-Concurrent-S
 * instead: time blocks of b steps carry psi(+-t_kb) forward and backward
 * (Eq. TE per block, as in the propagation), and each block adds
 * sum_n C_n^k(E) T_n s_k^+ + conj(C_n^k(E)) T_n s_k^- with the complex block
 * coefficients C_n^k(E) = tau sum_{j=1..b_k} c_n(j tau~) e^{iE' t_{kb+j}} (the
 * j = 0 term tau psi0 on the first block, half on each side), the next
 * carried states being one more row of the same contraction; the same
 * result up to rounding, with 1 <= n_E <= 31 (FP32) or 15 (FP64). */
csp_status csp_quasi_eigenstates(csp_context *ctx, const csp_lattice *lat,
                                 const void *dev_psi0, int32_t R, const csp_params *params,
                                 int32_t n_E, const double *energies, void *dev_qe,
                                 csp_report *rep);

/* Electronic-conductivity correlation (EC section, Eq. dc_corr) by the
 * moment-based concurrent form EC-Concurrent-M (Eq. dc_mom and the
 * reconstruction after it): for the R states psi_r (dev_psi0, [N][R]) and
 * their quasi-eigenstates Psi_r(E_e) (dev_qe, [n_E][N][R], as written by
 * csp_quasi_eigenstates with the same lattice), direction alpha (0 = x,
 * 1 = y), t_j = j params->tau_tilde / |H|, j = 0..Nt,
 *   C_r(t_j, E_e) = <psi_r|J e^{iHt_j} J|Psi_r(E_e)> / |<psi_r|Psi_r(E_e)>|,
 * J = i [H, X_alpha] (hbar = 1; the charge factor of the current drops out
 * of C, which is quadratic in J).  Computed as the moments
 * m_n = <J psi|T_n(H~)|J Psi(E)>, n = 0..N(Nt tau~), of one Chebyshev
 * recursion of J psi per state (no halving: bra and ket differ) contracted
 * against all n_E bras at once, then C = e^{iH0 t} sum_n c_n(t~)^* m_n /
 * |<psi|Psi(E)>| in FP64.  Writes dev_corr [n_E][Nt+1][R] complex128.
 * dtype of psi0 and qe per params->mode: CSP_FP32_CONC (complex64, moments
 * on split-bf16 MFMA with FP32 accumulation over slices of orbitals, FP64
 * across slices) or CSP_FP64_CONC (complex128); 1 <= n_E <= 128 (one
 * recursion serves all energies); 1 <= Nt <= 2^20.  Explicit matrices need
 * csp_lattice_set_positions first (CSP_EINVAL otherwise); CSP_EUNSUPPORTED
 * when Nt R n_E exceeds 2^31 - 1 (call per group of columns).  rep may be NULL. */
csp_status csp_ec_correlation(csp_context *ctx, const csp_lattice *lat, int32_t alpha,
                              const void *dev_psi0, int32_t R, const void *dev_qe,
                              const csp_params *params, int32_t n_E, double *dev_corr,
                              csp_report *rep);

/* Conductivity of Eq. DC on the computed times: dev_sigma[n_E][R] (FP64,
 * device) = D(E_e)/A * tau sum_{j=0}^{Nt} w_j Re[e^{-i E_e t_j} C_r(t_j, E_e)],
 * tau = tau_tilde / halfwidth, t_j = j tau, trapezoid weights (w_0 = w_Nt =
 * 1/2), from dev_corr [n_E][Nt+1][R] of csp_ec_correlation.  energies and
 * dos_over_area (D(E)/A per energy; NULL = 1) are host arrays of n_E. */
csp_status csp_ec_sigma(csp_context *ctx, const double *dev_corr, int64_t Nt, int32_t R,
                        int32_t n_E, const double *energies, double halfwidth,
                        double tau_tilde, const double *dos_over_area, double *dev_sigma);

/* Many lattices in one set of launches: instance i has lattice lats[i],
 * states dev_psi0[i] ([N_i][R[i]]) and correlations dev_corr[i]
 * ([(Nt+1)][R[i]]).  Every instance uses the same params (Nt, mode, b); the
 * recursion of all instances is one launch per Chebyshev step and the
 * contraction one launch per chunk; with the state assembly one time
 * block's launches are captured in a HIP graph and replayed per block
 * (params->graph). */
csp_status csp_propagate_batch(csp_context *ctx, int32_t n_inst, const csp_lattice *const *lats,
                               const void *const *dev_psi0, const int32_t *R,
                               const csp_params *params, double *const *dev_corr,
                               csp_report *rep);

/* Density of states from correlations (Sec. III): with t_j = j*tau,
 * tau = tau_tilde/halfwidth, C_{-j} = conj(C_j) and window w_j,
 * D_r(H0 + E_k) = (tau/2pi) Re sum_{j=-Nt}^{Nt-1} w_j C_j exp(i E_k t_j) at
 * E_k = k*pi/(Nt*tau), k = -Nt..Nt-1.  The correlations are those of
 * csp_propagate, which carry the centred propagator exp(-i (H - H0) t), so
 * this is the transform of Sec. III placed on the energies H0 + E_k of the
 * true spectrum [H0 - halfwidth, H0 + halfwidth]: pass the lattice's H0 as
 * `center` (0 for the default lattices).  dev_corr is [(Nt+1)][R]
 * complex128; writes dev_E[2Nt] (= center + E_k), dev_D[2Nt][R] and, if not
 * NULL, the column mean dev_Dmean[2Nt], all FP64 on the device.  Uses a
 * table of 2Nt complex128 twiddles that it allocates and frees; returns
 * after the stream has finished.  Errors: CSP_EINVAL for Nt < 1, R < 1,
 * halfwidth <= 0, a non-finite center or an unknown window. */
csp_status csp_dos(csp_context *ctx, const double *dev_corr, int64_t Nt, int32_t R,
                   double halfwidth, double center, double tau_tilde, int32_t window,
                   double *dev_E, double *dev_D, double *dev_Dmean);

/* The same DOS transform as csp_dos, for callers that cannot allocate
 * device memory: code being captured into a HIP graph, tight serving loops,
 * harnesses that forbid hipMalloc.  Arguments, layout and results are those
 * of csp_dos.  The 2 Nt complex128 twiddles live in a static device array
 * of the library instead of a per-call allocation, so Nt is limited to
 * CSP_DOS_NOALLOC_MAX_NT (8 MiB of device memory, held on every device the
 * library runs on until the process ends); a larger Nt is rejected with
 * CSP_EINVAL before any work is enqueued.  The call allocates nothing,
 * enqueues its kernels on the context's stream and returns without
 * synchronising (launch errors are reported; results are ready when the
 * stream reaches them).  Every call on one device shares that device's
 * array: calls that overlap on one device (other streams, other host
 * threads) race on it; calls ordered on one stream do not. */
#define CSP_DOS_NOALLOC_MAX_NT 262144
csp_status csp_dos_noalloc(csp_context *ctx, const double *dev_corr, int64_t Nt, int32_t R,
                           double halfwidth, double center, double tau_tilde, int32_t window,
                           double *dev_E, double *dev_D, double *dev_Dmean);

/* Autotuner.  For the instances (lats[i], R[i]) with params->mode and
 * params->assembly, times on this device every recursion launch shape
 * (values per lane in {2, 4}, Chebyshev steps per launch in {1, 2, 4, 8} as
 * compiled for the precision and assembly, rows per work item in
 * {8, ..., 128}) and, for the state assembly, the contraction at 2, 4 and 8
 * workgroups per compute unit for time tiles of 32 and 64, then picks the
 * time-block size b by the cost
 * model of Sec. II.B with measured operation costs:
 *   C(b) = sum over blocks k [ N_k t_amxsy + (N_k + 1) t_order(b) ],
 * N_k = N(b_k tau) (the last block is shorter when b does not divide Nt).
 * This is the paper's C = N_amxsy t_amxsy + N_axpy t_axpy with the axpy term
 * replaced by what it costs here: one MFMA pass over a Chebyshev vector
 * performs the axpys of that order for every time point of the block.
 * Only b whose workspace fits params->mem_cap_bytes are allowed.  The
 * result is cached in the context under the instances' shape (lattice
 * kinds and sizes, column groups, precision, assembly); csp_propagate and
 * csp_propagate_batch use a cached entry for their shape: its launch shapes
 * always, its b when params->block_b is 0.  The states and correlation
 * buffers of the caller are not touched (the timing uses workspace). */
csp_status csp_autotune(csp_context *ctx, int32_t n_inst, const csp_lattice *const *lats,
                        const int32_t *R, const csp_params *params, csp_tuning *out);

/* Installs a tuning record (for instance one saved from csp_autotune on an
 * earlier run) for the shape of these instances, as csp_autotune would
 * cache it; later propagations of that shape use it.  Fails with
 * CSP_EINVAL when a launch shape in *tuning is not compiled for
 * params->mode and params->assembly. */
csp_status csp_set_tuning(csp_context *ctx, int32_t n_inst, const csp_lattice *const *lats,
                          const int32_t *R, const csp_params *params,
                          const csp_tuning *tuning);

/* Time-block size of csp_autotune for one lattice with R columns: runs the
 * autotuner (or takes its cached entry) and returns its block_b; rep (may be
 * NULL) receives the model costs in model_cost. */
csp_status csp_select_block(csp_context *ctx, const csp_lattice *lat, int32_t R,
                            const csp_params *params, int32_t *b_out, csp_report *rep);

/* Streaming bandwidth of this device: plain grid-stride streams of 16-byte
 * accesses over `bytes` per array (workspace), best of several launch
 * widths, in GB/s: gbs_out[0] read only, [1] write only, [2] two reads and
 * one write (the access mix of a recursion step, counted as 3 x bytes).
 * These are the practical ceilings beside the published HBM peak. */
csp_status csp_bandwidth_probe(csp_context *ctx, uint64_t bytes, double *gbs_out);

/* Free cached workspace of the context (and the explicit-matrix copies). */
csp_status csp_context_trim(csp_context *ctx);

#ifdef __cplusplus
}
#endif

#endif /* CSP_H */
