/*
 * csp_oracle.c -- plain FP64 CPU oracle for concurrent stochastic propagation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code,
 * header or generated table with the GPU library; it is written directly
 * from the paper (arXiv:2510.17432) and from the published definitions of
 * the generator and of Miller's recurrence named below.
 *
 * What it computes, all in double precision complex:
 *   - a counter-based SplitMix64 generator (Steele, Lea & Flood, OOPSLA 2014);
 *   - chain / square / honeycomb tight-binding lattices with Anderson
 *     on-site disorder, as an explicit bond list and a CSR matrix;
 *   - Bessel functions J_n(x) by Miller's backward recurrence normalised with
 *     the Neumann sum J_0 + 2 sum_k J_2k = 1, the Chebyshev coefficients
 *     c_n(x) of exp(-i H x) (App. B) and the truncation order N(x) (Sec. II.A);
 *   - sequential propagation psi(t_j) = exp(-i H tau) psi(t_{j-1}) with the
 *     correlation <psi0|psi(t_j)> (Sec. II.A, Sec. III);
 *   - state-based concurrent propagation in time blocks, Eq. (TE) with the
 *     blocks of Sec. II.B, with the same correlations;
 *   - moment-based propagation (Sec. II.A) in blocks, and in one block with
 *     the halving of Eq. (cheby_prod) (DOS-Concurrent-M of Sec. III);
 *   - quasi-eigenstates by sequential forward and backward propagation
 *     (QE section, Eq. QE summed as in Eq. QE_coeff);
 *   - site positions and bond vectors of the lattices, the current operator
 *     J_a = i [H, X_a] applied from the bond list or from a CSR matrix with
 *     positions, and the electronic-conductivity correlation of Eq. dc_corr
 *     by sequential propagation of J psi (EC-Sequential).
 * Operation counters (amxsy / axpy / dot) follow the definitions of Sec. II.B
 * so that tests can compare them with Tab. (cost).
 *
 * Layout of every state array handed in or out: column-major per state,
 * i.e. a state is N contiguous complex values and R states follow each other.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* SplitMix64.  The generator keeps a 64-bit state that advances by the  */
/* odd constant GAMMA; output k (k = 0, 1, ...) of the generator seeded  */
/* with s is therefore mix(s + (k + 1) * GAMMA), which makes it a        */
/* counter-based generator.                                              */
/* ------------------------------------------------------------------ */
static const uint64_t GAMMA = 0x9e3779b97f4a7c15ULL;

static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Output number k of SplitMix64 seeded with `seed`. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k)
{
    return mix64(seed + (k + 1) * GAMMA);
}

/* The same generator run statefully, for the equivalence test. */
void orc_splitmix64_stream(uint64_t seed, int64_t n, uint64_t *out)
{
    uint64_t x = seed;
    for (int64_t i = 0; i < n; ++i) {
        x += GAMMA;
        out[i] = mix64(x);
    }
}

/* Draw `index` of stream `stream`: counter = stream * 2^40 + index. */
uint64_t orc_draw(uint64_t seed, uint64_t stream, uint64_t index)
{
    return orc_splitmix64(seed, (stream << 40) + index);
}

/* Uniform double in [0, 1) from the top 53 bits. */
double orc_u01(uint64_t bits)
{
    return (double)(bits >> 11) * 0x1.0p-53;
}

/* Uniform integer in [0, n) by the multiply-high map floor(bits * n / 2^64). */
int64_t orc_below(uint64_t bits, int64_t n)
{
    return (int64_t)(((unsigned __int128)bits * (unsigned __int128)(uint64_t)n) >> 64);
}

/* ------------------------------------------------------------------ */
/* Lattices.  kind 0 = chain (s = ix), 1 = square (s = iy*Lx + ix),     */
/* 2 = honeycomb (s = 2*(iy*Lx + ix) + sigma, sigma 0 = A, 1 = B).      */
/* Honeycomb bonds: A(ix,iy)-B(ix,iy), A(ix,iy)-B(ix-1,iy),             */
/* A(ix,iy)-B(ix,iy-1).  Periodic directions wrap modulo L.             */
/* ------------------------------------------------------------------ */
int64_t orc_lattice_sites(int kind, int64_t Lx, int64_t Ly)
{
    switch (kind) {
    case 0: return Lx;
    case 1: return Lx * Ly;
    case 2: return 2 * Lx * Ly;
    default: return -1;
    }
}

/* Writes the bond list (a[i], b[i]); returns the number of bonds.  With
 * a == NULL only counts. */
int64_t orc_lattice_bonds(int kind, int64_t Lx, int64_t Ly, int px, int py,
                          int64_t *a, int64_t *b)
{
    int64_t nb = 0;
#define BOND(u, v) do { if (a) { a[nb] = (u); b[nb] = (v); } ++nb; } while (0)
    if (kind == 0) {
        for (int64_t ix = 0; ix < Lx; ++ix) {
            if (ix + 1 < Lx) BOND(ix, ix + 1);
            else if (px) BOND(ix, 0);
        }
    } else if (kind == 1) {
        for (int64_t iy = 0; iy < Ly; ++iy)
            for (int64_t ix = 0; ix < Lx; ++ix) {
                int64_t s = iy * Lx + ix;
                if (ix + 1 < Lx) BOND(s, s + 1);
                else if (px) BOND(s, iy * Lx);
                if (iy + 1 < Ly) BOND(s, s + Lx);
                else if (py) BOND(s, ix);
            }
    } else if (kind == 2) {
        for (int64_t iy = 0; iy < Ly; ++iy)
            for (int64_t ix = 0; ix < Lx; ++ix) {
                int64_t A = 2 * (iy * Lx + ix);
                BOND(A, A + 1);
                if (ix >= 1) BOND(A, 2 * (iy * Lx + ix - 1) + 1);
                else if (px) BOND(A, 2 * (iy * Lx + Lx - 1) + 1);
                if (iy >= 1) BOND(A, 2 * ((iy - 1) * Lx + ix) + 1);
                else if (py) BOND(A, 2 * ((Ly - 1) * Lx + ix) + 1);
            }
    } else {
        return -1;
    }
#undef BOND
    return nb;
}

/* Anderson disorder: eps_s = W * (u_s - 1/2), u_s from stream 0 of `seed`. */
void orc_onsite(int64_t N, double W, uint64_t seed, double *eps)
{
    for (int64_t s = 0; s < N; ++s)
        eps[s] = W * (orc_u01(orc_draw(seed, 0, (uint64_t)s)) - 0.5);
}

/* CSR of H: H_ab = H_ba = t for every bond (repeated bonds add up),
 * H_ss = eps_s.  rowptr has N+1 entries, col/val 2*nbonds + N entries.
 * Within a row the diagonal comes first, then bond entries in bond order. */
void orc_build_csr(int64_t N, int64_t nbonds, const int64_t *a, const int64_t *b,
                   double t, const double *eps,
                   int64_t *rowptr, int64_t *col, double *val)
{
    int64_t *fill = (int64_t *)calloc((size_t)N, sizeof(int64_t));
    for (int64_t s = 0; s <= N; ++s) rowptr[s] = 0;
    for (int64_t s = 0; s < N; ++s) rowptr[s + 1] += 1;
    for (int64_t i = 0; i < nbonds; ++i) {
        rowptr[a[i] + 1] += 1;
        rowptr[b[i] + 1] += 1;
    }
    for (int64_t s = 0; s < N; ++s) rowptr[s + 1] += rowptr[s];
    for (int64_t s = 0; s < N; ++s) {
        col[rowptr[s]] = s;
        val[rowptr[s]] = eps ? eps[s] : 0.0;
        fill[s] = 1;
    }
    for (int64_t i = 0; i < nbonds; ++i) {
        int64_t u = a[i], v = b[i];
        col[rowptr[u] + fill[u]] = v; val[rowptr[u] + fill[u]] = t; fill[u]++;
        col[rowptr[v] + fill[v]] = u; val[rowptr[v] + fill[v]] = t; fill[v]++;
    }
    free(fill);
}

/* ------------------------------------------------------------------ */
/* Bessel functions by Miller's backward recurrence.                    */
/* J_{k-1}(x) = (2k/x) J_k(x) - J_{k+1}(x), started at an order M far   */
/* beyond both n_max and x with (J_{M+1}, J_M) = (0, 1), then scaled so */
/* that J_0 + 2 (J_2 + J_4 + ...) = 1.  Values above 1e250 trigger a    */
/* rescale of everything computed so far (the smallest ones underflow   */
/* harmlessly to zero).  Valid for x >= 0.                              */
/* ------------------------------------------------------------------ */
static int64_t miller_start(double x, int64_t nmax)
{
    double hi = (double)nmax > x ? (double)nmax : x;
    int64_t M = (int64_t)ceil(hi + 30.0 + 20.0 * cbrt(x > 1.0 ? x : 1.0));
    if (M & 1) M += 1;
    return M;
}

int orc_bessel_j(double x, int64_t nmax, double *J)
{
    if (nmax < 0 || !(x >= 0.0)) return -1;
    if (x == 0.0) {
        J[0] = 1.0;
        for (int64_t n = 1; n <= nmax; ++n) J[n] = 0.0;
        return 0;
    }
    int64_t M = miller_start(x, nmax);
    double *w = (double *)malloc((size_t)(M + 2) * sizeof(double));
    if (!w) return -2;
    w[M + 1] = 0.0;
    w[M] = 1.0;
    for (int64_t k = M; k >= 1; --k) {
        w[k - 1] = (2.0 * (double)k / x) * w[k] - w[k + 1];
        if (fabs(w[k - 1]) > 1e250) {
            for (int64_t i = k - 1; i <= M + 1; ++i) w[i] *= 1e-250;
        }
    }
    double norm = w[0];
    for (int64_t k = 2; k <= M; k += 2) norm += 2.0 * w[k];
    for (int64_t n = 0; n <= nmax; ++n) J[n] = w[n] / norm;
    free(w);
    return 0;
}

/* Chebyshev coefficients of exp(-i x y) on y in [-1, 1] (App. B):
 * c_0 = J_0(x), c_n = 2 (-i)^n J_n(x). */
int orc_cheb_coeffs(double x, int64_t nmax, cplx *c)
{
    double *J = (double *)malloc((size_t)(nmax + 1) * sizeof(double));
    if (!J) return -2;
    int rc = orc_bessel_j(x, nmax, J);
    if (rc) { free(J); return rc; }
    const cplx mi_pow[4] = {1.0, -I, -1.0, I};   /* (-i)^n for n mod 4 */
    c[0] = J[0];
    for (int64_t n = 1; n <= nmax; ++n) c[n] = 2.0 * mi_pow[n & 3] * J[n];
    free(J);
    return 0;
}

/* Truncation order (Sec. II.A): the coefficients must exceed eta for every
 * order below N.  Orders below x can pass through a zero of J_n by accident,
 * so N is the first order above x whose coefficient is at most eta.  The
 * expansion then runs over n = 0..N inclusive. */
int64_t orc_truncation(double x, double eta)
{
    if (!(x >= 0.0) || !(eta > 0.0)) return -1;
    int64_t nmax = (int64_t)ceil(x + 40.0 + 25.0 * cbrt(x > 1.0 ? x : 1.0));
    double *J = (double *)malloc((size_t)(nmax + 1) * sizeof(double));
    if (!J) return -2;
    orc_bessel_j(x, nmax, J);
    int64_t N = -1;
    for (int64_t n = (int64_t)floor(x) + 1; n <= nmax; ++n) {
        double cn = (n == 0) ? fabs(J[0]) : 2.0 * fabs(J[n]);
        if (cn <= eta) { N = n; break; }
    }
    free(J);
    return N;
}

/* ------------------------------------------------------------------ */
/* Propagation.                                                         */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    const int64_t *rowptr, *col;
    const double *val;
    double H0, Hn;          /* rescaled H = (H - H0) / Hn */
} orc_ham;

/* y <- a * Ht x - y   (amxsy of Sec. II.B with M = Ht) */
static void amxsy(const orc_ham *H, double a, const cplx *x, cplx *y)
{
    const double inv = 1.0 / H->Hn;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < H->n; ++s) {
        cplx acc = -H->H0 * x[s];
        for (int64_t p = H->rowptr[s]; p < H->rowptr[s + 1]; ++p)
            acc += H->val[p] * x[H->col[p]];
        y[s] = a * (acc * inv) - y[s];
    }
}

/* y <- a x + y */
static void axpy(int64_t n, cplx a, const cplx *x, cplx *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) y[s] += a * x[s];
}

/* <x|y> = sum conj(x) y, summed in index order per thread then in thread
 * order (OpenMP reduction on real and imaginary parts). */
static cplx dot(int64_t n, const cplx *x, const cplx *y)
{
    double re = 0.0, im = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : re, im)
    for (int64_t s = 0; s < n; ++s) {
        cplx v = conj(x[s]) * y[s];
        re += creal(v);
        im += cimag(v);
    }
    return re + I * im;
}

static void copy_scaled(int64_t n, cplx a, const cplx *x, cplx *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) y[s] = a * x[s];
}

/* counters: [0] amxsy, [1] axpy, [2] dot (the correlation at t = 0 is
 * counted separately in [3]). */

/* Sequential form: psi(t_j) = sum_{n=0}^{N(tau)} c_n(tau) T_n(Ht) psi(t_{j-1}),
 * corr[j] = <psi0|psi(t_j)>, j = 0..Nt, for one state. */
static int propagate_one_sequential(const orc_ham *H, const cplx *psi0, int64_t Nt,
                                    double tau, double eta, cplx *corr, cplx *final_out,
                                    int64_t *cnt)
{
    const int64_t n = H->n;
    int64_t Ntr = orc_truncation(tau, eta);
    if (Ntr < 1) return -1;
    cplx *c = (cplx *)malloc((size_t)(Ntr + 1) * sizeof(cplx));
    cplx *psi = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *p0 = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *p1 = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *acc = (cplx *)malloc((size_t)n * sizeof(cplx));
    if (!c || !psi || !p0 || !p1 || !acc) return -2;
    orc_cheb_coeffs(tau, Ntr, c);

    memcpy(psi, psi0, (size_t)n * sizeof(cplx));
    corr[0] = dot(n, psi0, psi);
    cnt[3] += 1;
    for (int64_t j = 1; j <= Nt; ++j) {
        /* phi_0 = psi, phi_1 = Ht psi */
        memcpy(p0, psi, (size_t)n * sizeof(cplx));
        memset(p1, 0, (size_t)n * sizeof(cplx));
        amxsy(H, 1.0, p0, p1); cnt[0]++;
        copy_scaled(n, c[0], p0, acc);
        axpy(n, c[1], p1, acc); cnt[1]++;
        for (int64_t k = 2; k <= Ntr; ++k) {
            /* phi_k = 2 Ht phi_{k-1} - phi_{k-2}, written over phi_{k-2} */
            amxsy(H, 2.0, p1, p0); cnt[0]++;
            cplx *tmp = p0; p0 = p1; p1 = tmp;
            axpy(n, c[k], p1, acc); cnt[1]++;
        }
        cplx *tmp = psi; psi = acc; acc = tmp;
        corr[j] = dot(n, psi0, psi); cnt[2]++;
    }
    if (final_out) memcpy(final_out, psi, (size_t)n * sizeof(cplx));
    free(c); free(psi); free(p0); free(p1); free(acc);
    return 0;
}

/* State-based concurrent form in time blocks of b steps (Eq. TE and the
 * blocks of Sec. II.B): within block k starting from s_k = psi(t_{kb}),
 * psi(t_{kb+j}) = sum_{n=0}^{N(j tau)} c_n(j tau) T_n(Ht) s_k, j = 1..b_k,
 * with b_k = min(b, Nt - kb); the next block starts from psi(t_{kb+b_k}).
 * The Chebyshev vectors are generated once per block and each is added to
 * every state whose expansion still includes its order. */
static int propagate_one_concurrent(const orc_ham *H, const cplx *psi0, int64_t Nt,
                                    double tau, double eta, int64_t b,
                                    cplx *corr, cplx *final_out, int64_t *cnt)
{
    const int64_t n = H->n;
    if (b < 1) return -1;
    int64_t *Nj = (int64_t *)malloc((size_t)(b + 1) * sizeof(int64_t));
    for (int64_t j = 1; j <= b; ++j) {
        Nj[j] = orc_truncation((double)j * tau, eta);
        if (Nj[j] < 1) return -1;
    }
    int64_t Nmax = Nj[b];
    cplx *c = (cplx *)malloc((size_t)(b + 1) * (size_t)(Nmax + 1) * sizeof(cplx));
    for (int64_t j = 1; j <= b; ++j)
        orc_cheb_coeffs((double)j * tau, Nj[j], c + (size_t)j * (size_t)(Nmax + 1));
#define COEF(jj, nn) c[(size_t)(jj) * (size_t)(Nmax + 1) + (size_t)(nn)]
    cplx *s = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *p0 = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *p1 = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *acc = (cplx *)malloc((size_t)b * (size_t)n * sizeof(cplx));
    if (!s || !p0 || !p1 || !acc) return -2;

    memcpy(s, psi0, (size_t)n * sizeof(cplx));
    corr[0] = dot(n, psi0, s);
    cnt[3] += 1;
    for (int64_t t0 = 0; t0 < Nt; t0 += b) {
        int64_t bk = (Nt - t0 < b) ? (Nt - t0) : b;
        int64_t Nk = Nj[bk];
        memcpy(p0, s, (size_t)n * sizeof(cplx));
        memset(p1, 0, (size_t)n * sizeof(cplx));
        amxsy(H, 1.0, p0, p1); cnt[0]++;
        for (int64_t j = 1; j <= bk; ++j) {
            cplx *aj = acc + (size_t)(j - 1) * (size_t)n;
            copy_scaled(n, COEF(j, 0), p0, aj);
            axpy(n, COEF(j, 1), p1, aj); cnt[1]++;
        }
        for (int64_t k = 2; k <= Nk; ++k) {
            amxsy(H, 2.0, p1, p0); cnt[0]++;
            cplx *tmp = p0; p0 = p1; p1 = tmp;
            for (int64_t j = 1; j <= bk; ++j) {
                if (k > Nj[j]) continue;
                axpy(n, COEF(j, k), p1, acc + (size_t)(j - 1) * (size_t)n); cnt[1]++;
            }
        }
        for (int64_t j = 1; j <= bk; ++j) {
            corr[t0 + j] = dot(n, psi0, acc + (size_t)(j - 1) * (size_t)n);
            cnt[2]++;
        }
        memcpy(s, acc + (size_t)(bk - 1) * (size_t)n, (size_t)n * sizeof(cplx));
    }
    if (final_out) memcpy(final_out, s, (size_t)n * sizeof(cplx));
#undef COEF
    free(Nj); free(c); free(s); free(p0); free(p1); free(acc);
    return 0;
}

/* Propagate R states (each N contiguous complex values, states back to
 * back) and write corr[r * (Nt + 1) + j] = <psi0_r|psi_r(t_j)>.
 * b = 0 selects the sequential form; b >= 1 the concurrent form with blocks
 * of b steps.  tau is the rescaled time step (pi for DOS).  final_states
 * (may be NULL) receives psi_r(t_Nt) laid out like psi0.  counters[0..3]
 * are accumulated. */
int orc_propagate(int64_t n, const int64_t *rowptr, const int64_t *col, const double *val,
                  double H0, double Hn, int64_t R, const cplx *psi0, int64_t Nt,
                  double tau, double eta, int64_t b, cplx *corr, cplx *final_states,
                  int64_t *counters)
{
    orc_ham H = {n, rowptr, col, val, H0, Hn};
    if (n < 1 || R < 1 || Nt < 0 || !(Hn > 0.0)) return -1;
    for (int64_t r = 0; r < R; ++r) {
        const cplx *p = psi0 + (size_t)r * (size_t)n;
        cplx *cr = corr + (size_t)r * (size_t)(Nt + 1);
        cplx *fr = final_states ? final_states + (size_t)r * (size_t)n : NULL;
        int rc = (b == 0) ? propagate_one_sequential(&H, p, Nt, tau, eta, cr, fr, counters)
                          : propagate_one_concurrent(&H, p, Nt, tau, eta, b, cr, fr, counters);
        if (rc) return rc;
    }
    return 0;
}

/* Apply T_n(Ht) to one state for n = 0..nmax (for eigenvector tests):
 * out[k * n_sites + s] = (T_k(Ht) x)_s. */
int orc_chebyshev_vectors(int64_t n, const int64_t *rowptr, const int64_t *col,
                          const double *val, double H0, double Hn,
                          const cplx *x, int64_t nmax, cplx *out)
{
    orc_ham H = {n, rowptr, col, val, H0, Hn};
    if (nmax < 0) return -1;
    memcpy(out, x, (size_t)n * sizeof(cplx));
    if (nmax == 0) return 0;
    cplx *o1 = out + (size_t)n;
    memset(o1, 0, (size_t)n * sizeof(cplx));
    amxsy(&H, 1.0, out, o1);
    for (int64_t k = 2; k <= nmax; ++k) {
        cplx *dst = out + (size_t)k * (size_t)n;
        memcpy(dst, out + (size_t)(k - 2) * (size_t)n, (size_t)n * sizeof(cplx));
        amxsy(&H, 2.0, out + (size_t)(k - 1) * (size_t)n, dst);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Moment-based form (Sec. II.A, moment-based implementation; Sec. III  */
/* DOS-Concurrent-M).  Within a block starting from s_k the Chebyshev   */
/* moments mu_n = <psi0|T_n(Ht) s_k> give                               */
/*   C(t_{kb+j}) = sum_{n=0}^{N(j tau)} c_n(j tau) mu_n,  j = 1..b_k,   */
/* the order of the time and polynomial sums of the sequential form     */
/* interchanged.  With more than one block the next block starts from   */
/* s_{k+1} = sum_n c_n(b_k tau) T_n(Ht) s_k.                            */
/*                                                                      */
/* halving (only for one block, where s_0 = psi0, and no final state):  */
/* with 2 T_m T_n = T_{m+n} + T_{|m-n|} (Eq. cheby_prod) and T_n        */
/* Hermitian, the moments above h = floor(N/2) follow from inner        */
/* products of vectors already generated:                               */
/*   mu_{2k}   = 2 <phi_k|phi_k>     - mu_0,                            */
/*   mu_{2k+1} = 2 <phi_{k+1}|phi_k> - mu_1,                            */
/* so the recursion stops at order ceil(N/2).  (Eq. cheby-moment as     */
/* printed omits the factor 2 on the inner products; with T_0 = 1 the   */
/* identity at m = n gives 2 T_n^2 = T_{2n} + 1, which fixes it.)       */
/* Counters: [0] recursion steps, [1] carry axpys, [2] moments taken    */
/* from inner products (n >= 1), [3] t = 0 correlations.               */
/* ------------------------------------------------------------------ */
static int propagate_one_moments(const orc_ham *H, const cplx *psi0, int64_t Nt, double tau,
                                 double eta, int64_t b, int halving, cplx *corr,
                                 cplx *final_out, int64_t *cnt)
{
    const int64_t n = H->n;
    if (b < 1) return -1;
    if (b > Nt && Nt > 0) b = Nt;
    const int single = (b >= Nt);
    if (halving && (!single || final_out)) return -1;
    int64_t *Nj = (int64_t *)malloc((size_t)(b + 1) * sizeof(int64_t));
    for (int64_t j = 1; j <= b; ++j) {
        Nj[j] = orc_truncation((double)j * tau, eta);
        if (Nj[j] < 1) return -1;
    }
    const int64_t Nmax = Nj[b];
    cplx *c = (cplx *)malloc((size_t)(b + 1) * (size_t)(Nmax + 1) * sizeof(cplx));
    for (int64_t j = 1; j <= b; ++j)
        orc_cheb_coeffs((double)j * tau, Nj[j], c + (size_t)j * (size_t)(Nmax + 1));
#define COEF(jj, nn) c[(size_t)(jj) * (size_t)(Nmax + 1) + (size_t)(nn)]
    cplx *mu = (cplx *)malloc((size_t)(Nmax + 1) * sizeof(cplx));
    cplx *s = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *s_next = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *p0 = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *p1 = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *self = (cplx *)malloc((size_t)(Nmax + 2) * sizeof(cplx));   /* <phi_k|phi_k> */
    cplx *cross = (cplx *)malloc((size_t)(Nmax + 2) * sizeof(cplx));  /* <phi_k|phi_{k-1}> */
    if (!mu || !s || !s_next || !p0 || !p1 || !self || !cross) return -2;

    memcpy(s, psi0, (size_t)n * sizeof(cplx));
    corr[0] = dot(n, psi0, s);
    cnt[3] += 1;
    for (int64_t t0 = 0; t0 < Nt; t0 += b) {
        const int64_t bk = (Nt - t0 < b) ? (Nt - t0) : b;
        const int64_t Nk = Nj[bk];
        const int carry = !single || final_out != NULL;
        const int64_t top = halving ? (Nk + 1) / 2 : Nk;      /* highest order generated */
        const int64_t h = Nk / 2;
        /* phi_0 = s, phi_1 = Ht s */
        memcpy(p0, s, (size_t)n * sizeof(cplx));
        memset(p1, 0, (size_t)n * sizeof(cplx));
        amxsy(H, 1.0, p0, p1); cnt[0]++;
        mu[0] = dot(n, psi0, p0);
        mu[1] = dot(n, psi0, p1); cnt[2]++;
        if (halving) {
            self[1] = dot(n, p1, p1);
            cross[1] = dot(n, p1, p0);
        }
        if (carry) {
            copy_scaled(n, COEF(bk, 0), p0, s_next);
            axpy(n, COEF(bk, 1), p1, s_next); cnt[1]++;
        }
        for (int64_t k = 2; k <= top; ++k) {
            amxsy(H, 2.0, p1, p0); cnt[0]++;       /* p0 <- phi_k */
            cplx *tmp = p0; p0 = p1; p1 = tmp;     /* p1 = phi_k, p0 = phi_{k-1} */
            if (!halving || k <= h) { mu[k] = dot(n, psi0, p1); cnt[2]++; }
            if (halving) {
                self[k] = dot(n, p1, p1);
                cross[k] = dot(n, p1, p0);
            }
            if (carry) { axpy(n, COEF(bk, k), p1, s_next); cnt[1]++; }
        }
        if (halving) {
            for (int64_t m = h + 1; m <= Nk; ++m) {
                if (m % 2 == 0) mu[m] = 2.0 * self[m / 2] - mu[0];
                else mu[m] = 2.0 * cross[(m + 1) / 2] - mu[1];
                cnt[2]++;
            }
        }
        for (int64_t j = 1; j <= bk; ++j) {
            cplx acc = 0.0;
            for (int64_t m = 0; m <= Nj[j]; ++m) acc += COEF(j, m) * mu[m];
            corr[t0 + j] = acc;
        }
        if (carry) { cplx *tmp = s; s = s_next; s_next = tmp; }
    }
    if (final_out) memcpy(final_out, s, (size_t)n * sizeof(cplx));
#undef COEF
    free(Nj); free(c); free(mu); free(s); free(s_next); free(p0); free(p1); free(self); free(cross);
    return 0;
}

/* Moment-based propagation of R states (layout as orc_propagate).  b >= 1
 * is the block size (b >= Nt: one block), halving selects the doubling
 * identity for the upper half of the moments (one block only). */
int orc_propagate_moments(int64_t n, const int64_t *rowptr, const int64_t *col,
                          const double *val, double H0, double Hn, int64_t R, const cplx *psi0,
                          int64_t Nt, double tau, double eta, int64_t b, int halving,
                          cplx *corr, cplx *final_states, int64_t *counters)
{
    orc_ham H = {n, rowptr, col, val, H0, Hn};
    if (n < 1 || R < 1 || Nt < 1 || !(Hn > 0.0)) return -1;
    for (int64_t r = 0; r < R; ++r) {
        const cplx *p = psi0 + (size_t)r * (size_t)n;
        cplx *cr = corr + (size_t)r * (size_t)(Nt + 1);
        cplx *fr = final_states ? final_states + (size_t)r * (size_t)n : NULL;
        int rc = propagate_one_moments(&H, p, Nt, tau, eta, b, halving, cr, fr, counters);
        if (rc) return rc;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Quasi-eigenstates (QE section, Eq. QE), sequential form (QE-Sequential): */
/* the state is propagated forward and backward in time step by step,      */
/*   psi(+-t_j) = sum_{n=0}^{N(tau)} c_n(+-tau) T_n(Ht) psi(+-t_{j-1}),     */
/* with c_n(-x) = conj(c_n(x)) (J_n real), and the time integral of Eq. QE   */
/* is the sum of Eq. QE_coeff taken over the propagated states:              */
/*   Psi(E) = tau_p sum_{j=0}^{Nt} (2 - delta_{j0})/2                        */
/*            [ e^{i E' t_j} psi(t_j) + e^{-i E' t_j} psi(-t_j) ],            */
/* t_j = j tau_p, tau_p = tau / Hn (physical time step), E' = E - H0.        */
/* Eq. QE_coeff as printed weighs by tau_p with no 1/(2 pi), so this is     */
/* 2 pi times the integral of Eq. QE.                                       */
/* ------------------------------------------------------------------ */

/* out <- sum_{k=0}^{Ntr} c[k] T_k(Ht) in, with p0, p1 scratch (amxsy and
 * axpy counted as in the sequential propagation). */
static void cheb_apply(const orc_ham *H, const cplx *c, int64_t Ntr, const cplx *in,
                       cplx *out, cplx *p0, cplx *p1, int64_t *cnt)
{
    const int64_t n = H->n;
    memcpy(p0, in, (size_t)n * sizeof(cplx));
    memset(p1, 0, (size_t)n * sizeof(cplx));
    amxsy(H, 1.0, p0, p1); cnt[0]++;
    copy_scaled(n, c[0], p0, out);
    axpy(n, c[1], p1, out); cnt[1]++;
    for (int64_t k = 2; k <= Ntr; ++k) {
        amxsy(H, 2.0, p1, p0); cnt[0]++;
        cplx *tmp = p0; p0 = p1; p1 = tmp;
        axpy(n, c[k], p1, out); cnt[1]++;
    }
}

/* R states psi0 (column-major, N values each), nE energies E[e]; writes
 * out[(r * nE + e) * n + s] = Psi_r(E_e)_s. */
int orc_quasi_eigenstates(int64_t n, const int64_t *rowptr, const int64_t *col,
                          const double *val, double H0, double Hn, int64_t R,
                          const cplx *psi0, int64_t Nt, double tau, double eta, int64_t nE,
                          const double *E, cplx *out, int64_t *counters)
{
    orc_ham H = {n, rowptr, col, val, H0, Hn};
    if (n < 1 || R < 1 || Nt < 0 || nE < 1 || !(Hn > 0.0)) return -1;
    const int64_t Ntr = orc_truncation(tau, eta);
    if (Ntr < 1) return -1;
    cplx *cf = (cplx *)malloc((size_t)(Ntr + 1) * sizeof(cplx));
    cplx *cb = (cplx *)malloc((size_t)(Ntr + 1) * sizeof(cplx));
    cplx *fw = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *bw = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *nx = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *p0 = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *p1 = (cplx *)malloc((size_t)n * sizeof(cplx));
    if (!cf || !cb || !fw || !bw || !nx || !p0 || !p1) return -2;
    orc_cheb_coeffs(tau, Ntr, cf);
    for (int64_t k = 0; k <= Ntr; ++k) cb[k] = conj(cf[k]);
    const double tp = tau / Hn;
    for (int64_t r = 0; r < R; ++r) {
        const cplx *ps = psi0 + (size_t)r * (size_t)n;
        cplx *o = out + (size_t)r * (size_t)nE * (size_t)n;
        /* j = 0: (1/2)(psi0 + psi0) */
        for (int64_t e = 0; e < nE; ++e) copy_scaled(n, tp, ps, o + (size_t)e * (size_t)n);
        memcpy(fw, ps, (size_t)n * sizeof(cplx));
        memcpy(bw, ps, (size_t)n * sizeof(cplx));
        for (int64_t j = 1; j <= Nt; ++j) {
            cheb_apply(&H, cf, Ntr, fw, nx, p0, p1, counters);
            cplx *t = fw; fw = nx; nx = t;
            cheb_apply(&H, cb, Ntr, bw, nx, p0, p1, counters);
            t = bw; bw = nx; nx = t;
            for (int64_t e = 0; e < nE; ++e) {
                const double th = (E[e] - H0) * (double)j * tp;
                cplx *oe = o + (size_t)e * (size_t)n;
                axpy(n, tp * cexp(I * th), fw, oe);
                axpy(n, tp * cexp(-I * th), bw, oe);
            }
        }
    }
    free(cf); free(cb); free(fw); free(bw); free(nx); free(p0); free(p1);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Geometry and the current operator (EC section).                     */
/* Chain: site ix at (ix, 0).  Square: (ix, iy).  Honeycomb with unit   */
/* C-C distance: cell (ix, iy) at ix a1 + iy a2, a1 = (sqrt3, 0),       */
/* a2 = (sqrt3/2, 3/2); A at the cell origin, B at + d, d = (a1+a2)/3 = */
/* (sqrt3/2, 1/2), so the three bonds of A(ix,iy) -- to B(ix,iy),       */
/* B(ix-1,iy), B(ix,iy-1) -- point along d, d - a1, d - a2 (unit        */
/* length).                                                             */
/* ------------------------------------------------------------------ */
void orc_site_positions(int kind, int64_t Lx, int64_t Ly, double *x, double *y)
{
    const double r3 = sqrt(3.0);
    if (kind == 0) {
        for (int64_t ix = 0; ix < Lx; ++ix) { x[ix] = (double)ix; y[ix] = 0.0; }
    } else if (kind == 1) {
        for (int64_t iy = 0; iy < Ly; ++iy)
            for (int64_t ix = 0; ix < Lx; ++ix) {
                x[iy * Lx + ix] = (double)ix;
                y[iy * Lx + ix] = (double)iy;
            }
    } else if (kind == 2) {
        for (int64_t iy = 0; iy < Ly; ++iy)
            for (int64_t ix = 0; ix < Lx; ++ix) {
                const int64_t A = 2 * (iy * Lx + ix);
                x[A] = r3 * (double)ix + 0.5 * r3 * (double)iy;
                y[A] = 1.5 * (double)iy;
                x[A + 1] = x[A] + 0.5 * r3;
                y[A + 1] = y[A] + 0.5;
            }
    }
}

/* Bond vectors r_b - r_a of the bonds (a, b) of orc_lattice_bonds, in the
 * same order; a bond closing a periodic boundary has the vector of its
 * kind (the displacement between the two sites as neighbours).  Returns
 * the number of bonds. */
int64_t orc_lattice_bond_vectors(int kind, int64_t Lx, int64_t Ly, int px, int py,
                                 double *vx, double *vy)
{
    int64_t nb = 0;
    const double r3 = sqrt(3.0);
#define VEC(u, v) do { vx[nb] = (u); vy[nb] = (v); ++nb; } while (0)
    if (kind == 0) {
        for (int64_t ix = 0; ix < Lx; ++ix)
            if (ix + 1 < Lx || px) VEC(1.0, 0.0);
    } else if (kind == 1) {
        for (int64_t iy = 0; iy < Ly; ++iy)
            for (int64_t ix = 0; ix < Lx; ++ix) {
                if (ix + 1 < Lx || px) VEC(1.0, 0.0);
                if (iy + 1 < Ly || py) VEC(0.0, 1.0);
            }
    } else if (kind == 2) {
        for (int64_t iy = 0; iy < Ly; ++iy)
            for (int64_t ix = 0; ix < Lx; ++ix) {
                VEC(0.5 * r3, 0.5);
                if (ix >= 1 || px) VEC(-0.5 * r3, 0.5);
                if (iy >= 1 || py) VEC(0.0, -1.0);
            }
    } else {
        return -1;
    }
#undef VEC
    return nb;
}

/* out <- J psi for H_ab = t on the bonds (a, b) with bond vectors v (one
 * Cartesian component): [H, X]_ab = H_ab (x_b - x_a), so J = i [H, X] has
 * J_ab = i t v and J_ba = -i t v; on-site terms commute with X and drop
 * out. */
void orc_current_bonds(int64_t N, int64_t nbonds, const int64_t *a, const int64_t *b,
                       const double *v, double t, const cplx *psi, cplx *out)
{
    for (int64_t s = 0; s < N; ++s) out[s] = 0.0;
    for (int64_t i = 0; i < nbonds; ++i) {
        out[a[i]] += I * t * v[i] * psi[b[i]];
        out[b[i]] += -I * t * v[i] * psi[a[i]];
    }
}

/* out <- J psi for a CSR matrix and site coordinates x (one Cartesian
 * component): (J psi)_s = i sum_p H_{s,col_p} d_p psi_{col_p}, d_p =
 * x_{col_p} - x_s reduced to the nearest image when box > 0. */
void orc_current_csr(int64_t N, const int64_t *rowptr, const int64_t *col, const double *val,
                     const double *x, double box, const cplx *psi, cplx *out)
{
    for (int64_t s = 0; s < N; ++s) {
        cplx acc = 0.0;
        for (int64_t p = rowptr[s]; p < rowptr[s + 1]; ++p) {
            double d = x[col[p]] - x[s];
            if (box > 0.0) d -= box * nearbyint(d / box);
            acc += I * val[p] * d * psi[col[p]];
        }
        out[s] = acc;
    }
}

/* EC-Sequential (EC section): for each state r and energy e,
 *   corr[(r nE + e)(Nt + 1) + j] = <exp(-i H t_j) Jpsi_r | X_{r,e}> / nrm[r nE + e]
 *                                  (times exp(i H0 t_j)),
 * t_j = j tau / Hn, with exp(-i (H - H0) tau / Hn) applied step by step by
 * the Chebyshev expansion c_n(tau); X_{r,e} = J Psi_r(E_e) and nrm the
 * magnitudes |<psi_r|Psi_r(E_e)>|, all given.  Jpsi is [R][n], X [R][nE][n]. */
int orc_ec_sequential(int64_t n, const int64_t *rowptr, const int64_t *col, const double *val,
                      double H0, double Hn, int64_t R, const cplx *Jpsi, int64_t nE,
                      const cplx *X, const double *nrm, int64_t Nt, double tau, double eta,
                      cplx *corr, int64_t *counters)
{
    orc_ham H = {n, rowptr, col, val, H0, Hn};
    if (n < 1 || R < 1 || Nt < 0 || nE < 1 || !(Hn > 0.0)) return -1;
    const int64_t Ntr = orc_truncation(tau, eta);
    if (Ntr < 1) return -1;
    cplx *cf = (cplx *)malloc((size_t)(Ntr + 1) * sizeof(cplx));
    cplx *v = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *nx = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *p0 = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *p1 = (cplx *)malloc((size_t)n * sizeof(cplx));
    if (!cf || !v || !nx || !p0 || !p1) return -2;
    orc_cheb_coeffs(tau, Ntr, cf);
    const double tp = tau / Hn;
    for (int64_t r = 0; r < R; ++r) {
        memcpy(v, Jpsi + (size_t)r * (size_t)n, (size_t)n * sizeof(cplx));
        for (int64_t j = 0; j <= Nt; ++j) {
            if (j > 0) {
                cheb_apply(&H, cf, Ntr, v, nx, p0, p1, counters);
                cplx *t = v; v = nx; nx = t;
            }
            const cplx ph = cexp(I * H0 * (double)j * tp);
            for (int64_t e = 0; e < nE; ++e) {
                const cplx *xe = X + ((size_t)r * (size_t)nE + (size_t)e) * (size_t)n;
                corr[((size_t)r * (size_t)nE + (size_t)e) * (size_t)(Nt + 1) + (size_t)j] =
                    ph * dot(n, v, xe) / nrm[r * nE + e];
                counters[2] += 1;
            }
        }
    }
    free(cf); free(v); free(nx); free(p0); free(p1);
    return 0;
}
