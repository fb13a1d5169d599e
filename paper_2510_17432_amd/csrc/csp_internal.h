// Internal definitions of libcsp: device-side data structures, the
// generator, lattice geometry and the host-side launch wrappers that the API
// layer (api.cpp) calls.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>
#include <stdint.h>

#include "csp.h"

namespace csp {

// ------------------------------------------------------------------ limits
constexpr int kMaxGroupCols = 32;     // columns per propagation group (power of 2)
constexpr int kMaxStepCols = 64;      // columns accepted by the single-step API
constexpr int kContractThreads = 256; // contraction workgroup (4 waves)
constexpr int kMaxJTiles = 2;         // 32-wide time tiles: b <= 64 on MFMA
constexpr int kMaxFp64B = 16;         // b limit of the FP64 contraction

// ------------------------------------------------------------------ generator
// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014).  The generator's state
// advances by the golden-ratio increment and every output is the state passed
// through a xor-shift-multiply finaliser, so output k of the generator seeded
// with s depends only on s + (k+1)*increment.  Draw `index` of `stream` is
// output (stream << 40) + index.
__host__ __device__ inline uint64_t sm64_finalise(uint64_t z) {
  z ^= z >> 30;
  z *= 0xbf58476d1ce4e5b9ULL;
  z ^= z >> 27;
  z *= 0x94d049bb133111ebULL;
  z ^= z >> 31;
  return z;
}
__host__ __device__ inline uint64_t rng_draw(uint64_t seed, uint64_t stream, uint64_t index) {
  const uint64_t counter = (stream << 40) + index;
  return sm64_finalise(seed + (counter + 1ULL) * 0x9e3779b97f4a7c15ULL);
}
// Top 53 bits as a double in [0, 1).
__host__ __device__ inline double rng_unit(uint64_t bits) {
  return static_cast<double>(bits >> 11) * (1.0 / 9007199254740992.0);
}

// ------------------------------------------------------------------ geometry
struct Geom {
  int32_t kind;        // csp_lattice_kind
  int32_t px, py;      // periodic flags
  int32_t pad;
  int64_t Lx, Ly;      // cells (Ly = 1 for chains)
  int64_t N;           // orbitals
  int64_t opr;         // orbitals per row: Lx, or 2*Lx for honeycomb
};

__host__ __device__ inline int max_degree(int kind) {
  return kind == CSP_CHAIN ? 2 : (kind == CSP_SQUARE ? 4 : 3);
}

// Neighbour k of orbital s (-1 if the bond is cut by an open edge).
__host__ __device__ inline int64_t neighbour(const Geom& g, int64_t s, int k) {
  if (g.kind == CSP_CHAIN) {
    int64_t x = s;
    if (k == 0) return x > 0 ? x - 1 : (g.px ? g.Lx - 1 : -1);
    return x + 1 < g.Lx ? x + 1 : (g.px ? 0 : -1);
  }
  if (g.kind == CSP_SQUARE) {
    int64_t y = s / g.Lx, x = s - y * g.Lx;
    switch (k) {
      case 0: return x > 0 ? s - 1 : (g.px ? s + g.Lx - 1 : -1);
      case 1: return x + 1 < g.Lx ? s + 1 : (g.px ? s - x : -1);
      case 2: return y > 0 ? s - g.Lx : (g.py ? s + (g.Ly - 1) * g.Lx : -1);
      default: return y + 1 < g.Ly ? s + g.Lx : (g.py ? x : -1);
    }
  }
  // honeycomb
  int64_t cell = s >> 1;
  int sig = static_cast<int>(s & 1);
  int64_t y = cell / g.Lx, x = cell - y * g.Lx;
  if (sig == 0) {  // A(x, y): B(x, y), B(x-1, y), B(x, y-1)
    switch (k) {
      case 0: return s + 1;
      case 1: return x > 0 ? s - 1 : (g.px ? 2 * (y * g.Lx + g.Lx - 1) + 1 : -1);
      default: return y > 0 ? 2 * ((y - 1) * g.Lx + x) + 1 : (g.py ? 2 * ((g.Ly - 1) * g.Lx + x) + 1 : -1);
    }
  }
  // B(x, y): A(x, y), A(x+1, y), A(x, y+1)
  switch (k) {
    case 0: return s - 1;
    case 1: return x + 1 < g.Lx ? s + 1 : (g.px ? 2 * (y * g.Lx) : -1);
    default: return y + 1 < g.Ly ? 2 * ((y + 1) * g.Lx + x) : (g.py ? 2 * x : -1);
  }
}

// ------------------------------------------------------------------ recursion
// Vectors of a column group are column-major, [Rg][N]: column c is values
// c*N .. c*N + N - 1, a lattice vector in the lattice's orbital order.
//
// One instance of a recursion launch: a lattice and a column group, its
// Chebyshev slots base + slot * slot_stride.
struct ChebInst {
  int32_t kind, px, py, Rg;
  int64_t Ly, opr, N;          // rows, values per row (Lx or 2 Lx), orbitals
  // layout of the group's vectors: row r of a column starts at r * pitch
  // (pitch >= opr; the positions opr..pitch-1 are padding, zero and never
  // written by the recursion), column c at c * cstride
  int64_t pitch, cstride;
  int64_t n_strips, n_segs;    // work items of one column: strips x row segments
  int64_t item0;               // first work item (wave) of this instance
  double alpha;                // 2 t / |H|
  double beta0;                // -2 H0 / |H|
  double onsite_scale;         // 2 / |H|
  const void* eps;             // per-orbital on-site energy (float or double), may be null
  void* base;                  // slot array
  int64_t slot_stride;         // complex values between slots
  const void* src;             // phi_n of a block's first launch (slot_cur < 0)
  const void* psi0;            // psi0 of the group (moment epilogue)
  void* carry;                 // carried state (moment epilogue, nlev = 1)
  const int32_t* ell_col;      // explicit matrix (kind CSP_SPARSE): [N/128][D][128] indices
  const void* ell_val;         // same layout, float or double; padding entries are 0
  int64_t wave0;               // first wave of this instance (explicit-matrix runs)
  int32_t ell_D;               // entries per row
  int32_t ell_ct;              // columns per wave (windowed: per workgroup tile)
  // explicit matrix, complex64: orbital-major copies of phi_n for the gathers,
  // two buffers of sh_pairs column pairs, [2][sh_pairs][N][2] complex values
  // (null: gathers read the column-major vectors)
  void* ell_shadow;
  int64_t sh_pairs;
  // explicit matrix, windowed layout (null: the slice layout above): slices
  // of 128 rows compact in the matrix graph, [n_segs][128] rows, entries in
  // quads [n_segs][ceil(D/4)][128][4] with window-local and global columns,
  // per-slice windows (the distinct columns a slice names, ascending)
  const int32_t* ellw_rows;    // row of each lane (-1: none)
  const uint16_t* ellw_loc;    // window-local column of each entry
  const int32_t* ellw_col;     // column of each entry (slices not staged)
  const void* ellw_val;        // value of each entry, float or double
  const int64_t* ellw_off;     // [n_segs + 1] window offsets into ellw_idx
  const int32_t* ellw_idx;     // window columns
  int64_t ellw_lds_cap;        // largest window a workgroup stages (x its columns)
};

// Per-launch arguments: levels l = 1..nlev produce phi_{n+l} from
// phi_n (slot_cur, or src when slot_cur < 0) and phi_{n-1} (slot_prev).
struct ChebStep {
  int32_t nlev;
  int32_t first;               // block start: phi_1 = H~ phi_0, no phi_{n-1}
  int32_t slot_cur, slot_prev;
  int32_t slot_out[8];         // slot receiving level l+1 (-1: not stored)
  int32_t copy_slot;           // slot receiving phi_n itself (-1: none)
  int32_t seg_rows;            // rows per work item
  int32_t ow;                  // owned values per strip (64 V - 2 margin)
  int32_t dot_psi0, dot_self;  // moment epilogue sums (see k_cheb)
  int32_t carry_mode;          // 0 none; 1 carry = cc0 phi_n + sum_l ccl[l-1] phi_{n+l};
                               // 2 carry += sum_l ccl[l-1] phi_{n+l}
  int32_t mom_slot;            // launch index inside the partial-sum buffer
  // explicit matrices: shadow buffer holding phi_n (-1: none, gather from the
  // column-major vector) and the one receiving phi_{n+1} (-1: not written)
  int32_t sh_in, sh_out;
  int32_t pad;
  double cc0[2];               // complex coefficient of phi_n (carry_mode 1)
  double ccl[8][2];            // complex coefficient of level l (phi_{n+l})
  double* partial;             // [slot][KT][items][4] complex records
  int64_t total_items;
};

// Consecutive instances of one lattice class (honeycomb or not, with or
// without on-site energies) and their work items; one launch per run.
struct ChebRun {
  int inst0, n_inst;
  int64_t item0, n_items;      // work items (stencil); moment records (explicit matrix)
  bool honey, eps, sparse;
  int ct;                      // explicit matrix: columns per wave (workgroup if windowed)
  int64_t wave0, n_waves;      // explicit matrix: waves (workgroups if windowed) of the run
  bool win;                    // explicit matrix in the windowed layout
  int64_t win_cap;             // windowed: LDS complex values of the run's largest tile
};
// mom: moment epilogue; carry: also the carried state (moment epilogue only)
hipError_t launch_cheb(bool fp64, int vec, int kt, bool mom, bool carry, const ChebInst* d_inst,
                       const std::vector<ChebRun>& runs, const ChebStep& st, hipStream_t s);
// Explicit (ELL) matrices: one Chebyshev step per launch, 64 rows of one
// column per wave (item = column * row chunks + chunk).
hipError_t launch_cheb_ell(bool fp64, bool mom, bool carry, int ct, const ChebInst* d_inst,
                           int n_inst, int64_t wave_lo, int64_t wave_hi, const ChebStep& st,
                           hipStream_t s);
// columns per wave of the explicit-matrix kernel for a group of Rg columns
int ell_columns_per_wave(bool fp64, int Rg);
// Windowed layout: one workgroup of 128 threads per (slice, tile of ct
// columns) stages the slice's window of phi_n in LDS (wg_lo .. wg_hi - 1
// over the run's instances, I.wave0 = first workgroup of an instance).
hipError_t launch_cheb_ellw(bool fp64, bool mom, bool carry, int ct, int64_t lds_values,
                            const ChebInst* d_inst, int n_inst, int64_t wg_lo, int64_t wg_hi,
                            const ChebStep& st, hipStream_t s);
// columns per workgroup of the windowed kernel for a group of Rg columns
// whose slices stage windows of up to `window` positions
int ellw_columns_per_group(bool fp64, int Rg, int64_t window);
// LDS bytes a windowed workgroup may stage
constexpr int64_t kEllwLdsBytes = 64 * 1024;

// Host side of the windowed layout (built at lattice creation).
struct EllWindows {
  int64_t n_slices = 0;
  int64_t max_window = 0;
  int D4 = 0;                    // quads of entries per row
  std::vector<int32_t> rows;     // [n_slices][128]
  std::vector<int64_t> off;      // [n_slices + 1]
  std::vector<int32_t> idx;      // windows, ascending per slice
  std::vector<uint16_t> loc;     // [n_slices][D4][128][4]
  std::vector<int32_t> col;      // [n_slices][D4][128][4]
  std::vector<double> v64;       // [n_slices][D4][128][4]
  std::vector<float> v32;        // same, FP32
};
bool build_ell_windows(int64_t N, int D, const int32_t* col, const double* val, EllWindows* w);
// max_s sum_k |val_sk| (k in order, FP64): one maximum per block into partial
hipError_t launch_ell_gershgorin(int64_t N, int D, const double* d_val, double* d_partial,
                                 int n_partial, hipStream_t s);
// (values per lane, steps per launch) pairs with a compiled kernel
bool cheb_shape_supported(bool fp64, int vec, int kt, bool mom);
bool cheb_carry_supported(bool fp64, int vec, int kt);
// margin positions per strip side: kt rounded up to a multiple of vec
int cheb_margin(int vec, int kt);

// Moment records -> per-step sums dots[row][4][Rg] (complex FP64), rows
// n0 + slot*kt + level for every record slot and level up to max_row.
struct MomInst {
  int64_t tile0, n_tiles;      // first work item and work items of the instance
  int32_t Rg, pad;
  double* dots;                // [n_rows][4][Rg] complex
};
hipError_t launch_cheb_mom_finish(const MomInst* d_mi, int n_inst, const double* partial,
                                  int64_t total_items, int kt, int n_slots, int n0, int max_row,
                                  hipStream_t s);
// Moments of a block from the step sums (halving: every moment above mu_1 from the self products)
// and correlations corr[(t0 + j) * ldc + col0 + r] = sum_n c_n(j tau) mu_n[r]
// for j = 1..bk (table a as produced by launch_bessel, row j-1 for x = j tau).
struct MomCorrInst {
  const double* dots;      // [steps + 1][4][Rg] complex, row n = step producing order n
  double* mu;              // [Nk + 1][Rg] complex (output of the assemble pass)
  double* corr;
  int64_t ldc;
  int32_t Rg, col0;
};
hipError_t launch_mom_corr(const MomCorrInst* d_mc, int n_inst, int Nk, int halving,
                           const double* d_a, int lda, const int32_t* d_ntrunc, int bk,
                           int64_t t0, int rg_max, hipStream_t s);

hipError_t launch_mom_corr_only(const MomCorrInst* d_mc, int n_inst, const double* d_a, int lda,
                                const int32_t* d_ntrunc, int bk, int64_t t0, int rg_max,
                                hipStream_t s);

// ------------------------------------------------------------------ conductivity
// out[v][s] = (J_alpha in[v])[s], J = i [H, X_alpha], for nvec vectors of N
// complex values (T = float or double): stencil lattices from their bond
// vectors, explicit matrices from the coordinates pos [N][2] (nearest image
// in a box of box[alpha] > 0).
hipError_t launch_current_stencil(bool fp64, const Geom& g, double t, int alpha, const void* in,
                                  void* out, int64_t nvec, hipStream_t s);
hipError_t launch_current_ell(bool fp64, int64_t N, int D, const int32_t* ell_col,
                              const double* ell_v64, const double* pos, double box, int alpha,
                              const void* in, void* out, int64_t nvec, hipStream_t s);
// nrm[q0 + c nE + e] = |<psi[c]|qe[e][c]>| for a group (psi [Rg][N], qe [nE][Rg][N])
hipError_t launch_ec_norm(bool fp64, int64_t N, int Rg, int nE, const void* psi, const void* qe,
                          double* nrm, int q0, hipStream_t s);
// Ring of S Chebyshev slots split into G parts of S / G slots: ring
// position k (order n sits at k = n mod S) is stored in slot
// (k mod G) S / G + k / G, so the consecutive orders that one recursion
// launch writes and one contraction chunk reads lie in all G parts of the
// ring's address range instead of one (measured faster on MI355X for rings
// of tens of GB).  The next position's slot is S / G further, less S - 1
// when that passes the end.
__host__ __device__ inline int ring_slot(int k, int S, int G) {
  return (k % G) * (S / G) + k / G;
}
// G for a ring of S slots: 3, 4 or 2 when it divides S, else 1 (in order).
int ring_parts(int S);

// Moments of one chunk of orders against the bras of a group (EC-Concurrent-M).
struct EcInst {
  const void* slots;        // ring [S][Rg][N]
  int64_t slot_stride;      // complex values between slots
  const void* bra;          // J Psi(E): [nE][Rg][N]
  void* partial;            // [Rg][n_slices][K][ldp] complex (float or double)
  int64_t N;
  int64_t slice_len;        // orbitals per slice (multiple of 8)
  int32_t Rg, n_slices;
  int32_t wg0, n_wg;        // workgroups: Rg * n_slices
  int32_t q0, pad;          // first moment column of the group (col0 * nE)
};
// Energies per tile of the complex128 conductivity moments: 16, or 24 for more
// than 16 energies (fewer tiles re-reading each chunk of orders).
__host__ __device__ constexpr int ec64_tile(int nE) { return nE > 16 ? 24 : 16; }
struct EcArgs {
  int32_t n_inst, n_lo, n_cnt, S;
  int32_t G;                // ring parts: position k in slot ring_slot(k, S, G)
  int32_t nE, K, total_wg;
  int32_t ldp;              // energies per partial row: n_etiles x tile (32 FP32, ec64_tile FP64)
  double* mu;               // [Nmax + 1][ldmu] complex, column q = (col0 + c) nE + e
  int64_t ldmu;
};
hipError_t launch_ec_moments(bool fp64, const EcInst* d_inst, int n_inst, const EcArgs& a,
                             hipStream_t s);
hipError_t launch_ec_mu_finish(bool fp64, const EcInst* d_inst, int n_inst, int rg_max,
                               const EcArgs& a, hipStream_t s);
// out[e][j][r] = conj(G_j) e^{i H0 j tau} / nrm, G_0 = mu row 0, G_j (j >= 1) from g
hipError_t launch_ec_finish(int Nt, int R, int nE, const double* mu, const double* g,
                            const double* nrm, double H0, double tau, double* out, hipStream_t s);
hipError_t launch_ec_sigma(int64_t Nt, int R, int nE, const double* corr, const double* E,
                           const double* dA, double tau, double* sigma, hipStream_t s);

// ------------------------------------------------------------------ contraction
// Every workgroup of an instance works on one column of the group: column
// c = (workgroup / wpc) with wpc workgroups per column, so its correlation
// sums belong to that column alone.
struct ContractInst {
  const void* slots;        // slot array of the group
  int64_t slot_stride;      // complex values
  int64_t N;                // values per column
  int32_t Rg;               // columns of the group (power of 2, <= 32)
  int32_t wpc;              // workgroups per column
  const void* psi0;         // psi0 of the group [Rg][N]
  void* carry;              // carried state [Rg][N]
  double* partial;          // [n_wg][b] complex (2 doubles), n_wg = Rg * wpc
  int32_t wg0, n_wg;        // workgroups of this instance in the launch
};

struct ContractArgs {
  int32_t n_inst;
  int32_t n_lo, n_cnt;      // orders n_lo .. n_lo + n_cnt - 1 of this chunk
  int32_t S;                // ring size: order n at ring position n % S
  int32_t G;                // ring parts: position k in slot ring_slot(k, S, G)
  int32_t first_chunk;      // write (1) or accumulate (0) carry and partials
  int32_t jtiles;           // 32-wide time tiles (FP32 MFMA path)
  int32_t bcols;            // time points of the block (b_k)
  int32_t total_wg;
  const void* bop;          // FP32 path: B operands in MFMA lane layout
  const void* coef;         // FP64 path: complex c[n][j], [n_cnt][bcols]
  const void* ccarry;       // carry coefficients: float a_n (FP32 path) or complex double (FP64)
};

hipError_t launch_contract_f32(const ContractInst* d_inst, const ContractArgs& a, hipStream_t s);
hipError_t launch_contract_f64(const ContractInst* d_inst, const ContractArgs& a, hipStream_t s);

// Finish: corr[(t0 + j) * ldc + col0 + c] = sum_{sub < wpc} partial[c * wpc + sub][j-1],
// j = 1..b, for every column c of the group.
struct FinishInst {
  const double* partial;
  int32_t wpc, Rg;
  double* corr;             // device correlation array of the instance
  int64_t ldc;              // columns of the caller's correlation array
  int32_t col0;
  int32_t pad;
};
// t0_dev (may be null): device copy of t0, read at run time (graph replays).
hipError_t launch_finish(const FinishInst* d_inst, int n_inst, int bcols, int64_t t0,
                         const int64_t* t0_dev, hipStream_t s);
// d_blk[0] += b, d_blk[1] += 1 (the block counter of graph replays).
hipError_t launch_advance(int64_t* d_blk, int64_t b, hipStream_t s);

// ------------------------------------------------------------------ quasi-eigenstates
// One column group of a quasi-eigenstate contraction: Chebyshev ring as in
// the state assembly, accumulators out [Rg][nE][N] (complex, working precision).
struct QeInst {
  const void* slots;
  int64_t slot_stride;      // complex values between slots
  int64_t N;
  int32_t Rg, wpc;          // columns, workgroups per column
  void* out;
  int32_t wg0, n_wg;
  void* carry;              // carried state (row nE of complex coefficients), [Rg][N]
  int32_t conj;             // use the conjugate coefficients (backward propagation)
  int32_t pad;
};
struct QeArgs {
  int32_t n_inst;
  int32_t n_lo, n_cnt;      // orders n_lo .. n_lo + n_cnt - 1 of this chunk
  int32_t S;                // ring size: order n at ring position n % S
  int32_t G;                // ring parts: position k in slot ring_slot(k, S, G)
  int32_t first_chunk;      // write (1) or accumulate (0) the states
  int32_t nE;               // energies
  int32_t total_wg;
  int32_t cplx;             // complex coefficients (state-based form) with a carry row nE
  int32_t carry_first;      // write (1) or accumulate (0) the carried state
  int32_t e_tile_stride;    // operand entries between energy tiles (grid y): 32 energies
                            // per tile in FP32, B in FP64
  const void* bop;          // FP32: A operands C_n(E) in the MFMA lane layout, per tile
  const void* coef;         // FP64: [n_cnt][B] complex, per tile
};
// QE-Concurrent-S, one time block of bk steps starting at time index J0:
// C[e][n] = tau sum_{j=1..bk, n <= N(j tau~)} c_n(j tau~) e^{i (E_e - H0)(J0 + j) tau}
// (+ tau/2 at n = 0 when first: the j = 0 term, shared by both directions),
// e < nE, and the carry row C[nE][n] = c_n(bk tau~);
// n = 0..Nk, complex, ldc = Nk + 1.
hipError_t launch_qes_coeffs(const double* d_a, int lda, const int32_t* d_ntr, int bk,
                             int64_t J0, int nE, const double* d_E, double H0, double tau,
                             int first, int Nk, double* d_C, hipStream_t s);
// FP32: complex A operands (rows x 16 orders per step, MFMA lane layout); FP64: [n_cnt][B]
hipError_t launch_pack_qes(const double* d_C, int ldc, int rows, int n_lo, int n_cnt,
                           void* d_bop, hipStream_t s);
hipError_t launch_pack_qes64(const double* d_C, int ldc, int rows, int B, int n_lo, int n_cnt,
                             double* d_coef, hipStream_t s);
// a += b over n complex values (float or double)
hipError_t launch_add_complex(bool fp64, int64_t n, void* d_a, const void* d_b, hipStream_t s);
// C[e][n] = tau (delta_n0 + sum_j 2 a_n(j tau~) Re((-i)^n e^{i (E_e - H0) j tau})), n <= nmax;
// d_cs: scratch [nE][Nt] double2.
hipError_t launch_qe_coeffs(const double* d_a, int lda, const int32_t* d_ntr, int Nt, int nE,
                            const double* d_E, double H0, double tau, int nmax, double* d_cs,
                            double* d_C, hipStream_t s);
hipError_t launch_pack_qe64(const double* d_C, int ldc, int nE, int B, int n_lo, int n_cnt,
                            double* d_coef, hipStream_t s);
hipError_t launch_contract_qe(bool fp64, const QeInst* d_inst, const QeArgs& a, hipStream_t s);
hipError_t launch_qe_scatter(int64_t N, int Rg, int nE, int ld, int col0, bool fp64_in,
                             const void* d_in, int out_dtype, void* d_out, hipStream_t s);

// ------------------------------------------------------------------ coefficients
// For x_j = (j + 1) * tau, j = 0..nx-1: a[j][n] = J_n(x_j) (n = 0) or
// 2 J_n(x_j) (n >= 1) for n <= nmax, and ntrunc[j] = N(x_j).  clip: orders
// beyond x_j + 40 + 25 x_j^(1/3) (past the truncation) are stored as 0.
hipError_t launch_bessel(double tau, int nx, int nmax, double eta, bool clip, double* d_a,
                         int32_t* d_ntrunc, hipStream_t s);
// Complex c_n(x) = (-i)^n a_n written as complex128 [nmax+1].
hipError_t launch_complex_coeffs(const double* d_a, int nmax, double* d_c, hipStream_t s);
// B-operand table of the MFMA contraction for orders n_lo..n_lo+n_cnt-1 and
// time columns j = 1..bcols (a is [bcols][lda] as produced by launch_bessel),
// plus the FP32 carry coefficients a[bcols-1][n].
hipError_t launch_pack_bop(const double* d_a, int lda, const int32_t* d_ntrunc, int bcols,
                           int jtiles, int n_lo, int n_cnt, void* d_bop, float* d_ccarry,
                           hipStream_t s);
// FP64 complex coefficient table c[n - n_lo][j] and carry coefficients.
hipError_t launch_pack_c64(const double* d_a, int lda, const int32_t* d_ntrunc, int bcols,
                           int n_lo, int n_cnt, double* d_coef, double* d_ccarry,
                           hipStream_t s);
size_t bop_bytes(int jtiles, int n_cnt);

// ------------------------------------------------------------------ setup kernels
hipError_t launch_onsite(const Geom& g, double W, uint64_t seed, double* d_eps64,
                         float* d_eps32, hipStream_t s);
hipError_t launch_gershgorin(const Geom& g, const double* d_eps, double t, double H0,
                             double* d_rowmax_partial, int n_partial, hipStream_t s);
hipError_t launch_neighbours(const Geom& g, int64_t* d_nbr, hipStream_t s);
hipError_t launch_random_phase(int64_t N, int R, uint64_t seed, int dtype, void* d_psi,
                               int ld, int col0, hipStream_t s);
hipError_t launch_ldos_sites(int64_t N, int n, uint64_t seed, int64_t* d_sites, hipStream_t s);
hipError_t launch_site_states(int64_t N, int n, const int64_t* d_sites, int dtype, void* d_psi,
                              int ld, int col0, hipStream_t s);
// Copy columns col0..col0+Rg-1 of an [N][ld] block (dtype) into a dense
// column-major group of the path's precision (fp64 selects double2 output).
// With pitch > 0 the group's rows of opr values are pitch values apart and
// its columns N / opr * pitch apart, the padding written as zero; pitch 0:
// columns of N values.  launch_scatter_cols is the inverse.
hipError_t launch_gather_cols(int64_t N, int ld, int col0, int Rg, int in_dtype,
                              const void* d_in, bool fp64, void* d_out, hipStream_t s,
                              int64_t opr = 0, int64_t pitch = 0);
hipError_t launch_scatter_cols(int64_t N, int ld, int col0, int Rg, int out_dtype,
                               const void* d_in, bool fp64, void* d_out, hipStream_t s,
                               int64_t opr = 0, int64_t pitch = 0);
// Zero the row padding (positions opr..pitch-1 of every row) of n_slots x Rg
// vectors: vector c of slot k at base + k * slot_stride + c * cstride.
hipError_t launch_zero_pad(void* d_base, int n_slots, int64_t slot_stride, int Rg,
                           int64_t cstride, int64_t Ly, int64_t opr, int64_t pitch, bool fp64,
                           hipStream_t s);
// C_0: corr[col0 + r] = <psi0_r|psi0_r> for an [N][Rg] group, FP64 result.
hipError_t launch_self_dot(int64_t N, int Rg, const void* d_psi, bool fp64, double* d_corr,
                           int col0, double* d_scratch, int n_scratch_wg, hipStream_t s);
// Moments -> correlations: corr[t0 + j][col0 + r] = sum_n c_n(j tau) mu_n[r].
hipError_t launch_moment_corr(const double* d_mu_partial, int n_tiles, int Rg, int n_cnt,
                              const double* d_a, int lda, const int32_t* d_ntrunc, int bcols,
                              int64_t t0, double* d_corr, int64_t ldc, int col0,
                              hipStream_t s);
// Norm guard after a block (see k_guard); d_carry may be null.
// blk_dev (may be null): device (t0, block) read at run time (graph replays).
hipError_t launch_guard(int64_t N, int Rg, const void* d_carry, bool fp64, const double* d_corr,
                        int64_t ldc, int col0, int64_t t0, int bk, double tol, int block,
                        const int64_t* blk_dev, int* d_flag, double* d_scratch,
                        int n_scratch_wg, hipStream_t s);
// Device address of this device's static twiddle scratch of
// csp_dos_noalloc (2 CSP_DOS_NOALLOC_MAX_NT complex128), looked up once per
// device with that device current and kept for the process.
hipError_t dos_noalloc_scratch(int device, double** out);
// DOS of the centred correlations on the energies center + E_k; d_twiddle
// holds 2 Nt complex128 values (written here before they are read).
hipError_t launch_dos(const double* d_corr, int64_t Nt, int R, double halfwidth, double center,
                      double tau_tilde, int window, double* d_E, double* d_D, double* d_Dmean,
                      double* d_twiddle, hipStream_t s);

// ------------------------------------------------------------------ probe
// kind 0: read a, 1: write c, 2: c = 2a - b; n16 = 16-byte elements.
hipError_t launch_probe(int kind, const void* a, const void* b, void* c, float* sink, int64_t n16,
                        int grid, hipStream_t s);

// ------------------------------------------------------------------ helpers
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Workgroup b of g runs on XCD b % 8; return the logical index that gives each
// XCD one contiguous range of logical indices (so that neighbouring tiles of a
// lattice share the L2 of one XCD).
__device__ inline int64_t xcd_remap(int64_t b, int64_t g) {
  const int64_t q = g / 8, rem = g % 8;
  const int64_t x = b % 8, k = b / 8;
  return x * q + (x < rem ? x : rem) + k;
}

}  // namespace csp
