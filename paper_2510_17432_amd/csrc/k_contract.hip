// Block contraction of Chebyshev vectors with expansion coefficients
// (state-based concurrent form, Eq. TE):
//   psi(t_{kb+j}) = sum_n c_n(j tau) phi_n,   j = 1..b_k,
// fused with the correlation reduction <psi0|psi(t_{kb+j})> and with the
// carried state s_{k+1} = psi(t_{kb+b_k}) (Sec. II.B time blocks).
//
// FP32 path (MFMA).  With c_n(x) = (-i)^n a_n(x), a_n real (App. B:
// a_0 = J_0, a_n = 2 J_n), write X_n = (-i)^n phi_n = p_n + i q_n.  Then
//   Re psi_j = sum_n p_n a_{n,j},   Im psi_j = sum_n q_n a_{n,j},
// two real products of a [32 values x K orders] tile with one real
// [K x 32 times] coefficient tile, which run on v_mfma_f32_32x32x16_bf16.
// Each FP32 operand is split x = hi + lo with hi = bf16(x),
// lo = bf16(x - hi), and the product is hi*hi + hi*lo + lo*hi, accumulated
// in FP32.  This is not FP32-exact: hi + lo keeps 16 significant bits
// (|x - hi - lo| <= 2^-18 |x|), and the dropped lo*lo term is up to
// 2^-18 |ab|, so each product carries a relative error of at most about
// 3 * 2^-18 = 1.1e-5; the observed DOS error against complex128 (about 1e-5
// relative on the graphene and 1e9-orbital workloads) is of that size, ten
// times inside the 1e-4 target.  The carried state uses plain FP32 FMAs on
// the same loaded values, since its error would feed every later block.
//
// Every workgroup works on one column of the group (groups are stored
// column-major, [Rg][N]), so all of its correlation sums belong to that
// column.  One wave owns one 32-value tile of the column at a time: lane
// (i = lane%32, h = lane/32) loads value i of orders 8h..8h+7 of each
// 16-order step (coalesced: for a fixed order the 32 lanes read 256
// contiguous bytes), with the next step's values already in flight.  The B
// operand (lane (j, h) holds time j, orders 8h..8h+7) is staged in LDS once
// per launch.  The accumulator holds psi for rows 8(v/4) + 4h + v%4 and time
// lane%32; the epilogue multiplies by conj(psi0) (loaded with the tile's
// first orders, one value per lane, and passed between lanes) and adds the
// tile's rows into one FP32 sum per lane and time, then the workgroup reduces
// in FP64 in a fixed order and writes its partial sums, one per time point.
#include <algorithm>

#include "csp_internal.h"

namespace csp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

struct BopEntry {
  bf16x8 hi;
  bf16x8 lo;
};

// complex64 values through global-address-space pointers
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) f32x2 gf2;
__device__ __forceinline__ float2 ldg2(const gf2* p) {
  const f32x2 t = *p;
  return make_float2(t.x, t.y);
}
// Chebyshev vectors are read once per contraction: non-temporal loads
// (measured on MI355X, graphene workload: 29.65 -> 29.23 ms per launch)
__device__ __forceinline__ float2 ldg2_stream(const gf2* p) {
  const f32x2 t = __builtin_nontemporal_load(p);
  return make_float2(t.x, t.y);
}
__device__ __forceinline__ void stg2(gf2* p, float2 v) {
  f32x2 t;
  t.x = v.x;
  t.y = v.y;
  *p = t;
}

size_t bop_bytes(int jtiles, int n_cnt) {
  return sizeof(BopEntry) * 64 * (size_t)jtiles * (size_t)ceil_div(n_cnt, 16);
}

template <int JT>
__global__ __launch_bounds__(kContractThreads) __attribute__((amdgpu_waves_per_eu(JT == 1 ? 4 : 2))) void k_contract_f32(
    const ContractInst* __restrict__ insts, ContractArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n_kb = (a.n_cnt + 15) >> 4;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int il = lane & 31, h = lane >> 5;

  const int nb_entries = n_kb * JT * 64;
  BopEntry* sb = reinterpret_cast<BopEntry*>(smem);
  const size_t bop_sz = sizeof(BopEntry) * (size_t)nb_entries;
  const size_t red_sz = sizeof(double2) * JT * 32;
  float* sc = reinterpret_cast<float*>(smem + (bop_sz > red_sz ? bop_sz : red_sz));
  double2* sred = reinterpret_cast<double2*>(smem);

  {
    const BopEntry* gb = static_cast<const BopEntry*>(a.bop);
    for (int e = tid; e < nb_entries; e += kContractThreads) sb[e] = gb[e];
    const float* gc = static_cast<const float*>(a.ccarry);
    for (int e = tid; e < n_kb * 16; e += kContractThreads) sc[e] = e < a.n_cnt ? gc[e] : 0.f;
  }
  __syncthreads();

  const int64_t wg = xcd_remap(blockIdx.x, gridDim.x);
  int ii = 0;
  while (ii + 1 < a.n_inst && wg >= insts[ii + 1].wg0) ++ii;
  const ContractInst& I = insts[ii];
  const int64_t wgl = wg - I.wg0;
  const int64_t col = wgl / I.wpc, sub = wgl - col * I.wpc;
  const int64_t N = I.N;
  const int64_t coff = col * N;
  const gf2* slots = (const gf2*)(I.slots) + coff;
  const gf2* psi0 = (const gf2*)(I.psi0) + coff;
  gf2* carry = (gf2*)(I.carry) + coff;
  const int64_t n_tiles = ceil_div(N, 32);
  const int64_t sstr = I.slot_stride;

  // per-lane correlation sums of time lane%32 (+ 32 jt) over the rows seen
  float pr[JT], pi[JT];
#pragma unroll
  for (int jt = 0; jt < JT; ++jt) { pr[jt] = 0.f; pi[jt] = 0.f; }

  const int64_t stride_tiles = (int64_t)I.wpc * 4;
  for (int64_t tile = sub * 4 + wave; tile < n_tiles; tile += stride_tiles) {
    const int64_t m = tile * 32 + il;
    const bool mv = m < N;
    f32x16 accR[JT], accI[JT];
#pragma unroll
    for (int jt = 0; jt < JT; ++jt)
#pragma unroll
      for (int v = 0; v < 16; ++v) { accR[jt][v] = 0.f; accI[jt][v] = 0.f; }
    float cr = 0.f, ci = 0.f;
    // psi0 of the tile, value il in both half-waves (used after the orders),
    // and the carried state of row il (half-wave 0, after the first chunk):
    // both loaded with the orders, so the tile waits for memory once
    const float2 p0l = mv ? ldg2(psi0 + m) : make_float2(0.f, 0.f);
    const float2 cold =
        (h == 0 && mv && !a.first_chunk) ? ldg2(carry + m) : make_float2(0.f, 0.f);

    // Orders of the next 16-order step are in flight while the current one
    // is multiplied (its values are converted to bf16 first, so the loads
    // can reuse their registers).
    float2 xn[8];
    // order n sits at ring position n % S, in slot ring_slot(n % S)
    const int part = a.S / a.G;
    auto load_step = [&](int kb) {
      const int rel0 = kb * 16 + h * 8;
      int k = (a.n_lo + rel0) % a.S;
      int ps = ring_slot(k, a.S, a.G);
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        xn[v] = (mv && rel0 + v < a.n_cnt) ? ldg2_stream(slots + (int64_t)ps * sstr + m)
                                            : make_float2(0.f, 0.f);
        // next position (S wraps to 0) and its slot, without branches
        const int kn = k + 1, pn = ps + part;
        ps = kn == a.S ? 0 : (pn >= a.S ? pn - (a.S - 1) : pn);
        k = kn == a.S ? 0 : kn;
      }
    };
    load_step(0);
    for (int kb = 0; kb < n_kb; ++kb) {
      const int r0 = kb * 16 + h * 8;
      float2 x[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) x[v] = xn[v];
      bf16x8 phi, plo, qhi, qlo;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int n = a.n_lo + r0 + v;
        float p, q;
        switch (n & 3) {            // (-i)^n (u + i w)
          case 0: p = x[v].x;  q = x[v].y;  break;
          case 1: p = x[v].y;  q = -x[v].x; break;
          case 2: p = -x[v].x; q = -x[v].y; break;
          default: p = -x[v].y; q = x[v].x; break;
        }
        const float cc = sc[r0 + v];
        cr = fmaf(cc, p, cr);
        ci = fmaf(cc, q, ci);
        const __bf16 ph = static_cast<__bf16>(p);
        const __bf16 qh = static_cast<__bf16>(q);
        phi[v] = ph;
        qhi[v] = qh;
        plo[v] = static_cast<__bf16>(p - static_cast<float>(ph));
        qlo[v] = static_cast<__bf16>(q - static_cast<float>(qh));
      }
      if (kb + 1 < n_kb) load_step(kb + 1);
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) {
        const BopEntry be = sb[(kb * JT + jt) * 64 + lane];
        accR[jt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(phi, be.hi, accR[jt], 0, 0, 0);
        accR[jt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(phi, be.lo, accR[jt], 0, 0, 0);
        accR[jt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(plo, be.hi, accR[jt], 0, 0, 0);
        accI[jt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qhi, be.hi, accI[jt], 0, 0, 0);
        accI[jt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qhi, be.lo, accI[jt], 0, 0, 0);
        accI[jt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qlo, be.hi, accI[jt], 0, 0, 0);
      }
    }

    // Carried state: the two half-waves hold complementary orders of row il.
    cr += __shfl_xor(cr, 32);
    ci += __shfl_xor(ci, 32);
    if (h == 0 && mv)
      stg2(carry + m, a.first_chunk ? make_float2(cr, ci) : make_float2(cr + cold.x, ci + cold.y));

    // Correlation epilogue: conj(psi0[row]) * psi[row, time] summed over
    // the 16 rows 8(v/4) + 4h + v%4 of this lane; psi0 of row rho comes from
    // lane rho (rows past N hold 0).
    float tr[JT], ti[JT];
#pragma unroll
    for (int jt = 0; jt < JT; ++jt) { tr[jt] = 0.f; ti[jt] = 0.f; }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int rho = 8 * (v >> 2) + 4 * h + (v & 3);
      const float p0x = __shfl(p0l.x, rho), p0y = __shfl(p0l.y, rho);
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) {
        const float re = accR[jt][v], im = accI[jt][v];
        tr[jt] = fmaf(p0x, re, fmaf(p0y, im, tr[jt]));
        ti[jt] = fmaf(p0x, im, fmaf(-p0y, re, ti[jt]));
      }
    }
#pragma unroll
    for (int jt = 0; jt < JT; ++jt) {
      pr[jt] += tr[jt];
      pi[jt] += ti[jt];
    }
  }

  // Workgroup reduction in FP64, fixed order: per lane over its 16 rows,
  // then waves 0..3 and half-waves 0, 1 into sred[time].
  __syncthreads();  // LDS B operands are no longer needed
  for (int e = tid; e < JT * 32; e += kContractThreads) sred[e] = make_double2(0.0, 0.0);
  __syncthreads();
  double sx[JT], sy[JT];
#pragma unroll
  for (int jt = 0; jt < JT; ++jt) {
    sx[jt] = static_cast<double>(pr[jt]);
    sy[jt] = static_cast<double>(pi[jt]);
  }
  for (int w = 0; w < 4; ++w) {
    for (int half = 0; half < 2; ++half) {
      if (wave == w && h == half) {
#pragma unroll
        for (int jt = 0; jt < JT; ++jt) {
          double2& d = sred[jt * 32 + il];
          d.x += sx[jt];
          d.y += sy[jt];
        }
      }
      __syncthreads();
    }
  }
  double2* part = reinterpret_cast<double2*>(I.partial) + wgl * (int64_t)a.bcols;
  for (int e = tid; e < a.bcols; e += kContractThreads) {
    const double2 v = sred[e];
    if (a.first_chunk) {
      part[e] = v;
    } else {
      double2 o = part[e];
      o.x += v.x;
      o.y += v.y;
      part[e] = o;
    }
  }
}

// FP64 contraction: one value per thread, B (<= 16) time columns in
// registers, complex coefficients c[n][j] in LDS; each workgroup works on
// one column.
template <int B>
__global__ __launch_bounds__(kContractThreads) void k_contract_f64(
    const ContractInst* __restrict__ insts, ContractArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  double2* scoef = reinterpret_cast<double2*>(smem);           // [n_cnt][B]
  double2* scc = scoef + (size_t)a.n_cnt * B;                  // [n_cnt]
  double2* sred = scc + a.n_cnt;                               // [256]
  const int tid = threadIdx.x;
  {
    const double2* gc = static_cast<const double2*>(a.coef);
    for (int e = tid; e < a.n_cnt * B; e += kContractThreads) {
      const int n = e / B, j = e - n * B;
      scoef[e] = j < a.bcols ? gc[(size_t)n * a.bcols + j] : make_double2(0.0, 0.0);
    }
    const double2* gcc = static_cast<const double2*>(a.ccarry);
    for (int e = tid; e < a.n_cnt; e += kContractThreads) scc[e] = gcc[e];
  }
  __syncthreads();

  const int64_t wg = xcd_remap(blockIdx.x, gridDim.x);
  int ii = 0;
  while (ii + 1 < a.n_inst && wg >= insts[ii + 1].wg0) ++ii;
  const ContractInst& I = insts[ii];
  const int64_t wgl = wg - I.wg0;
  const int64_t col = wgl / I.wpc, sub = wgl - col * I.wpc;
  const int64_t N = I.N;
  const int64_t coff = col * N;
  const double2* slots = static_cast<const double2*>(I.slots) + coff;
  const double2* psi0 = static_cast<const double2*>(I.psi0) + coff;
  double2* carry = static_cast<double2*>(I.carry) + coff;

  double2 part[B];
#pragma unroll
  for (int j = 0; j < B; ++j) part[j] = make_double2(0.0, 0.0);

  const int64_t step = (int64_t)I.wpc * kContractThreads;
  for (int64_t m = sub * kContractThreads + tid; m < N; m += step) {
    double2 acc[B];
#pragma unroll
    for (int j = 0; j < B; ++j) acc[j] = make_double2(0.0, 0.0);
    double2 cy = make_double2(0.0, 0.0);
    for (int rel = 0; rel < a.n_cnt; ++rel) {
      const double2 x =
          slots[(int64_t)ring_slot((a.n_lo + rel) % a.S, a.S, a.G) * I.slot_stride + m];
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const double2 c = scoef[rel * B + j];
        acc[j].x = fma(c.x, x.x, fma(-c.y, x.y, acc[j].x));
        acc[j].y = fma(c.x, x.y, fma(c.y, x.x, acc[j].y));
      }
      const double2 c = scc[rel];
      cy.x = fma(c.x, x.x, fma(-c.y, x.y, cy.x));
      cy.y = fma(c.x, x.y, fma(c.y, x.x, cy.y));
    }
    if (!a.first_chunk) {
      const double2 o = carry[m];
      cy.x += o.x;
      cy.y += o.y;
    }
    carry[m] = cy;
    const double2 p0 = psi0[m];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      part[j].x = fma(p0.x, acc[j].x, fma(p0.y, acc[j].y, part[j].x));
      part[j].y = fma(p0.x, acc[j].y, fma(-p0.y, acc[j].x, part[j].y));
    }
  }

  // Sum over the 256 threads in a fixed tree (FP64).
  double2* outp = reinterpret_cast<double2*>(I.partial) + wgl * (int64_t)a.bcols;
  for (int j = 0; j < a.bcols && j < B; ++j) {
    double2 pj = part[0];
#pragma unroll
    for (int k = 1; k < B; ++k)
      if (k == j) pj = part[k];   // static register indices
    sred[tid] = pj;
    __syncthreads();
    for (int w = kContractThreads / 2; w > 0; w >>= 1) {   // fixed tree
      if (tid < w) {
        sred[tid].x += sred[tid + w].x;
        sred[tid].y += sred[tid + w].y;
      }
      __syncthreads();
    }
    if (tid == 0) {
      const double2 s = sred[0];
      double2* d = outp + j;
      if (a.first_chunk) {
        *d = s;
      } else {
        double2 o = *d;
        o.x += s.x;
        o.y += s.y;
        *d = o;
      }
    }
    __syncthreads();
  }
}

hipError_t launch_contract_f32(const ContractInst* d_inst, const ContractArgs& a, hipStream_t s) {
  if (a.total_wg <= 0 || a.n_cnt <= 0) return hipSuccess;
  const size_t bsz = bop_bytes(a.jtiles, a.n_cnt);
  const size_t rsz = sizeof(double2) * a.jtiles * 32;
  const size_t lds = (bsz > rsz ? bsz : rsz) + sizeof(float) * 16 * ceil_div(a.n_cnt, 16);
  const dim3 grid(a.total_wg), block(kContractThreads);
  if (a.jtiles == 1)
    hipLaunchKernelGGL(k_contract_f32<1>, grid, block, lds, s, d_inst, a);
  else if (a.jtiles == 2)
    hipLaunchKernelGGL(k_contract_f32<2>, grid, block, lds, s, d_inst, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_contract_f64(const ContractInst* d_inst, const ContractArgs& a, hipStream_t s) {
  if (a.total_wg <= 0 || a.n_cnt <= 0) return hipSuccess;
  int B = 1;
  while (B < a.bcols) B *= 2;
  if (B > kMaxFp64B) return hipErrorInvalidValue;
  const size_t lds = sizeof(double2) * ((size_t)a.n_cnt * B + a.n_cnt + kContractThreads);
  const dim3 grid(a.total_wg), block(kContractThreads);
  switch (B) {
    case 1: hipLaunchKernelGGL(k_contract_f64<1>, grid, block, lds, s, d_inst, a); break;
    case 2: hipLaunchKernelGGL(k_contract_f64<2>, grid, block, lds, s, d_inst, a); break;
    case 4: hipLaunchKernelGGL(k_contract_f64<4>, grid, block, lds, s, d_inst, a); break;
    case 8: hipLaunchKernelGGL(k_contract_f64<8>, grid, block, lds, s, d_inst, a); break;
    case 16: hipLaunchKernelGGL(k_contract_f64<16>, grid, block, lds, s, d_inst, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Sum the workgroup partials of every column in workgroup order (FP64).
// The block's first time index comes from t0_dev[0] when it is given (a
// block replayed from a HIP graph), else from t0.
__global__ void k_finish(const FinishInst* __restrict__ insts, int n_inst, int bcols,
                         int64_t t0, const int64_t* __restrict__ t0_dev) {
  const int ii = blockIdx.y;
  if (ii >= n_inst) return;
  const FinishInst& I = insts[ii];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= bcols * I.Rg) return;
  if (t0_dev) t0 = t0_dev[0];
  const int j = e / I.Rg, c = e - j * I.Rg;
  const double2* p = reinterpret_cast<const double2*>(I.partial);
  double sx = 0.0, sy = 0.0;
  for (int w = 0; w < I.wpc; ++w) {
    const double2 v = p[((int64_t)c * I.wpc + w) * bcols + j];
    sx += v.x;
    sy += v.y;
  }
  double2* cr = reinterpret_cast<double2*>(I.corr);
  cr[(t0 + 1 + j) * I.ldc + I.col0 + c] = make_double2(sx, sy);
}

hipError_t launch_finish(const FinishInst* d_inst, int n_inst, int bcols, int64_t t0,
                         const int64_t* t0_dev, hipStream_t s) {
  const int need = bcols * kMaxGroupCols;
  const dim3 grid(static_cast<unsigned>(ceil_div(need, 256)), n_inst), block(256);
  hipLaunchKernelGGL(k_finish, grid, block, 0, s, d_inst, n_inst, bcols, t0, t0_dev);
  return hipGetLastError();
}

// Block counter of graph replays: [0] first time index of the next block,
// [1] its block number.
__global__ void k_advance(int64_t* __restrict__ blk, int64_t b) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    blk[0] += b;
    blk[1] += 1;
  }
}

hipError_t launch_advance(int64_t* d_blk, int64_t b, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, d_blk, b);
  return hipGetLastError();
}

}  // namespace csp
