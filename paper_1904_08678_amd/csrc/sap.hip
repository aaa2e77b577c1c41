// Schwarz alternating procedure (SAP) on the fine lattice.  The paper names
// SAP as the smoother DDalphaAMG normally uses and as a feature its Grid
// implementation lacks (Sec. 2.1, Sec. 4), without a definition; the reading
// here is the multiplicative Schwarz method on red-black coloured domains:
// the domains are the level-0 aggregates, coloured by the parity of their
// coarse coordinates.  For each colour, every domain B of that colour forms
// r_B = b_B - (D x)_B with the current x, runs `iters` MR steps on
// D_B e = r_B from e = 0 (D_B: D with the couplings leaving B dropped) and sets
// x_B += e.  Domains of one colour do not couple, so one launch per colour
// handles all of them; the launch reads x on the other colour (fixed) and
// writes x only on its own domains.
//
// One workgroup per domain (A <= 256 sites, contiguous in the aggregate-major
// site order).  Waves are split by direction group g (NG groups: group g
// applies the hops of directions g*4/NG .. (g+1)*4/NG - 1 and, for g < 2 when
// NG = 4 or always when NG = 2, the clover block of chirality g) and by site
// quarter; the group partials meet in LDS, where the domain residual also
// lives between MR steps.  Each thread owns 12/NG spin-colour components of
// one site for the updates and the inner products (FP64 accumulation).
#include "wilson_ops.h"

namespace wcmg {

namespace {
constexpr int kSapMaxA = 256;

template <typename R, int NG>
struct SapShared {
  cplx<R> rho[12][kSapMaxA];
  cplx<R> part[NG][12][kSapMaxA];
  double red[16][3];
};

// acc += the hops of direction mu (both signs) at device site s; the
// neighbour spinor comes from global memory (FROM_LDS = false: the full
// operator on x) or from the domain residual in LDS (FROM_LDS = true: D_B,
// hops whose neighbour lies outside the domain are skipped).
template <typename R, int MU, bool FROM_LDS>
__device__ inline void sap_hops(cplx<R> (&acc)[12], const cplx<R>* __restrict__ x, const cplx<R>* __restrict__ U,
                                const int* __restrict__ nbr, long V, long s, long base, int A,
                                const cplx<R> (*rho)[kSapMaxA]) {
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    const bool fwd = f == 0;
    const long y = nbr[(long)(2 * MU + f) * V + s];
    const long ls = fwd ? s : y;
    cplx<R> p[12];
    if (FROM_LDS) {
      const long oy = y - base;
      if (oy < 0 || oy >= A) continue;
#pragma unroll
      for (int k = 0; k < 12; ++k) p[k] = rho[k][oy];
    } else {
#pragma unroll
      for (int k = 0; k < 12; ++k) p[k] = x[(long)k * V + y];
    }
    cplx<R> u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = U[(long)(MU * 9 + e) * V + ls];
    if (fwd) hop_core<R, MU, true>(acc, p, u);
    else hop_core<R, MU, false>(acc, p, u);
    // FP64: one hop's operands at a time (all four in flight exceed the registers)
    if constexpr (sizeof(R) == 8) __builtin_amdgcn_sched_barrier(0);
  }
}

template <typename R, int CHI>
__device__ inline void sap_clover_lds(cplx<R> (&acc)[12], const R* __restrict__ clov, long V, long s, int o,
                                      const cplx<R> (*rho)[kSapMaxA]) {
  constexpr int RC = 16 / sizeof(R);
  typedef typename std::conditional<sizeof(R) == 4, float4, double2>::type V16;
  R e[36];
  const V16* cb = (const V16*)(clov + (long)CHI * 36 * V);
#pragma unroll
  for (int q = 0; q < 36 / RC; ++q) {
    const V16 c = cb[(long)q * V + s];
    if constexpr (RC == 4) {
      e[q * 4 + 0] = c.x;
      e[q * 4 + 1] = c.y;
      e[q * 4 + 2] = c.z;
      e[q * 4 + 3] = c.w;
    } else {
      e[q * 2 + 0] = c.x;
      e[q * 2 + 1] = c.y;
    }
  }
  cplx<R> p[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) p[k] = rho[CHI * 6 + k][o];
  clover_block_apply<R, CHI>(acc, e, p);
}

// The partial of group g (directions and clover chirality) at device site s.
template <typename R, int NG, bool FROM_LDS>
__device__ inline void sap_group(int g, cplx<R> (&acc)[12], const cplx<R>* __restrict__ x,
                                 const cplx<R>* __restrict__ U, const R* __restrict__ clov,
                                 const int* __restrict__ nbr, long V, long s, long base, int A, int o,
                                 const cplx<R> (*rho)[kSapMaxA]) {
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = mkc((R)0, (R)0);
  if (g == 0) {
    if (FROM_LDS) sap_clover_lds<R, 0>(acc, clov, V, s, o, rho);
    else clover_chirality<R, 0>(acc, x, clov, V, s);
  } else if (g == 1) {
    if (FROM_LDS) sap_clover_lds<R, 1>(acc, clov, V, s, o, rho);
    else clover_chirality<R, 1>(acc, x, clov, V, s);
  }
  if (NG == 4) {
    if (g == 0) sap_hops<R, 0, FROM_LDS>(acc, x, U, nbr, V, s, base, A, rho);
    else if (g == 1) sap_hops<R, 1, FROM_LDS>(acc, x, U, nbr, V, s, base, A, rho);
    else if (g == 2) sap_hops<R, 2, FROM_LDS>(acc, x, U, nbr, V, s, base, A, rho);
    else sap_hops<R, 3, FROM_LDS>(acc, x, U, nbr, V, s, base, A, rho);
  } else {
    if (g == 0) {
      sap_hops<R, 0, FROM_LDS>(acc, x, U, nbr, V, s, base, A, rho);
      sap_hops<R, 1, FROM_LDS>(acc, x, U, nbr, V, s, base, A, rho);
    } else {
      sap_hops<R, 2, FROM_LDS>(acc, x, U, nbr, V, s, base, A, rho);
      sap_hops<R, 3, FROM_LDS>(acc, x, U, nbr, V, s, base, A, rho);
    }
  }
}

// One thread's operator data for direction group G of NG = 2 (directions 2G
// and 2G+1, clover chirality G): its four links (forward U_mu(s), backward
// U_mu(s - mu)), the four neighbour sites and the 36 reals of its clover
// block, loaded once and kept in registers for the residual and every MR step.
template <typename R>
struct SapOps {
  cplx<R> u[4][9];
  long y[4];
  R cl[36];
};

template <typename R, int G>
__device__ inline void sap_load_ops(SapOps<R>& op, const cplx<R>* __restrict__ U, const R* __restrict__ clov,
                                    const int* __restrict__ nbr, long V, long s) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int mu = 2 * G + j / 2, f = j % 2;
    op.y[j] = nbr[(long)(2 * mu + f) * V + s];
    const long ls = f == 0 ? s : op.y[j];
#pragma unroll
    for (int e = 0; e < 9; ++e) op.u[j][e] = U[(long)(mu * 9 + e) * V + ls];
  }
  constexpr int RC = 16 / sizeof(R);
  typedef typename std::conditional<sizeof(R) == 4, float4, double2>::type V16;
  const V16* cb = (const V16*)(clov + (long)G * 36 * V);
#pragma unroll
  for (int q = 0; q < 36 / RC; ++q) {
    const V16 c = cb[(long)q * V + s];
    if constexpr (RC == 4) {
      op.cl[q * 4 + 0] = c.x;
      op.cl[q * 4 + 1] = c.y;
      op.cl[q * 4 + 2] = c.z;
      op.cl[q * 4 + 3] = c.w;
    } else {
      op.cl[q * 2 + 0] = c.x;
      op.cl[q * 2 + 1] = c.y;
    }
  }
}

template <typename R, int G, int J, bool FROM_LDS>
__device__ inline void sap_hop_j(cplx<R> (&acc)[12], const SapOps<R>& op, const cplx<R>* __restrict__ x, long V,
                                 long base, int A, const cplx<R> (*rho)[kSapMaxA]) {
  constexpr int MU = 2 * G + J / 2;
  constexpr bool FWD = J % 2 == 0;
  cplx<R> p[12];
  if (FROM_LDS) {
    const long oy = op.y[J] - base;
    if (oy < 0 || oy >= A) return;
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k] = rho[k][oy];
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k] = x[(long)k * V + op.y[J]];
  }
  hop_core<R, MU, FWD>(acc, p, op.u[J]);
}

template <typename R, int G, bool FROM_LDS>
__device__ inline void sap_apply_ops(cplx<R> (&acc)[12], const SapOps<R>& op, const cplx<R>* __restrict__ x,
                                     long V, long s, long base, int A, int o, const cplx<R> (*rho)[kSapMaxA]) {
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = mkc((R)0, (R)0);
  cplx<R> p[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) p[k] = FROM_LDS ? rho[G * 6 + k][o] : x[(long)(G * 6 + k) * V + s];
  clover_block_apply<R, G>(acc, op.cl, p);
  sap_hop_j<R, G, 0, FROM_LDS>(acc, op, x, V, base, A, rho);
  sap_hop_j<R, G, 1, FROM_LDS>(acc, op, x, V, base, A, rho);
  sap_hop_j<R, G, 2, FROM_LDS>(acc, op, x, V, base, A, rho);
  sap_hop_j<R, G, 3, FROM_LDS>(acc, op, x, V, base, A, rho);
}
}  // namespace

// x and b: [nrhs][12][V] (right-hand side r at offset r * 12 * V); doms: the
// aggregate indices of this colour (one workgroup each, blockIdx.y = rhs).
template <typename R, int NG, bool CACHE>
__global__ void __launch_bounds__(NG * 256) k_sap(cplx<R>* __restrict__ x, const cplx<R>* __restrict__ b,
                                              const cplx<R>* __restrict__ U, const R* __restrict__ clov,
                                              const int* __restrict__ nbr, long V, int A,
                                              const int* __restrict__ doms, int iters,
                                              const int* __restrict__ run, int rs) {
  constexpr int NC = 12 / NG;  // components owned per thread
  __shared__ SapShared<R, NG> sh;
  const long r = blockIdx.y;
  if (run && !run[r * rs]) return;
  const int NQ = (A + 63) / 64;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = wave / NQ, quarter = wave - g * NQ;
  const int o = quarter * 64 + lane;
  const bool valid = o < A;
  const long base = (long)doms[blockIdx.x] * A;
  const long s = base + o;
  x += r * 12 * V;
  b += r * 12 * V;
  const cplx<R>(*rho)[kSapMaxA] = sh.rho;
  cplx<R> acc[12];
  static_assert(!CACHE || NG == 2, "register-resident operators need two direction groups");
  SapOps<R> op;
  if (CACHE && valid) {
    if (g == 0) sap_load_ops<R, 0>(op, U, clov, nbr, V, s);
    else sap_load_ops<R, 1>(op, U, clov, nbr, V, s);
  }
  // residual r_B = b - D x at the domain's sites (full operator, global x)
  if (valid) {
    if (!CACHE) sap_group<R, NG, false>(g, acc, x, U, clov, nbr, V, s, base, A, o, rho);
    else if (g == 0) sap_apply_ops<R, 0, false>(acc, op, x, V, s, base, A, o, rho);
    else sap_apply_ops<R, 1, false>(acc, op, x, V, s, base, A, o, rho);
#pragma unroll
    for (int k = 0; k < 12; ++k) sh.part[g][k][o] = acc[k];
  }
  __syncthreads();
  // between MR steps the owner's residual entries live in LDS only (rho) and
  // q = D_B rho is re-summed from the partials when needed: registers hold e
  cplx<R> e[NC];
  if (valid) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int k = g * NC + c;
      cplx<R> dx = sh.part[0][k][o];
#pragma unroll
      for (int h = 1; h < NG; ++h) dx = cadd(dx, sh.part[h][k][o]);
      sh.rho[k][o] = csub(b[(long)k * V + s], dx);
      e[c] = mkc((R)0, (R)0);
    }
  }
  const int nwaves = (int)(blockDim.x >> 6);
  for (int it = 0; it < iters; ++it) {
    __syncthreads();  // rho complete
    if (valid) {
      if (!CACHE) sap_group<R, NG, true>(g, acc, x, U, clov, nbr, V, s, base, A, o, rho);
      else if (g == 0) sap_apply_ops<R, 0, true>(acc, op, x, V, s, base, A, o, rho);
      else sap_apply_ops<R, 1, true>(acc, op, x, V, s, base, A, o, rho);
#pragma unroll
      for (int k = 0; k < 12; ++k) sh.part[g][k][o] = acc[k];
    }
    __syncthreads();
    double pr = 0.0, pi = 0.0, pp = 0.0;
    if (valid) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int k = g * NC + c;
        cplx<R> v = sh.part[0][k][o];
#pragma unroll
        for (int h = 1; h < NG; ++h) v = cadd(v, sh.part[h][k][o]);
        const cplx<R> w = sh.rho[k][o];
        // <q, rho> = sum conj(q) rho
        pr += (double)v.re * w.re + (double)v.im * w.im;
        pi += (double)v.re * w.im - (double)v.im * w.re;
        pp += (double)v.re * v.re + (double)v.im * v.im;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      pr += __shfl_xor(pr, off, 64);
      pi += __shfl_xor(pi, off, 64);
      pp += __shfl_xor(pp, off, 64);
    }
    if (lane == 0) {
      sh.red[wave][0] = pr;
      sh.red[wave][1] = pi;
      sh.red[wave][2] = pp;
    }
    __syncthreads();
    double tr = 0.0, ti = 0.0, tp = 0.0;
    for (int w = 0; w < nwaves; ++w) {
      tr += sh.red[w][0];
      ti += sh.red[w][1];
      tp += sh.red[w][2];
    }
    if (tp == 0.0) break;  // D_B rho = 0: rho = 0, nothing left to do (uniform)
    const cplx<R> alpha = mkc((R)(tr / tp), (R)(ti / tp));
    if (valid) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int k = g * NC + c;
        cplx<R> v = sh.part[0][k][o];
#pragma unroll
        for (int h = 1; h < NG; ++h) v = cadd(v, sh.part[h][k][o]);
        cplx<R> w = sh.rho[k][o];
        cfma(e[c], alpha, w);
        cfma(w, cneg(alpha), v);
        sh.rho[k][o] = w;
      }
    }
  }
  if (valid) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const long at = (long)(g * NC + c) * V + s;
      x[at] = cadd(x[at], e[c]);
    }
  }
}

template <typename R>
void launch_sap(cplx<R>* x, const cplx<R>* b, const cplx<R>* U, const R* clov, const int* nbr, long V, int A,
                const int* doms, int ndoms, int iters, int nrhs, const int* run, int rs, hipStream_t st) {
  require(A >= 1 && A <= kSapMaxA, WCMG_ERR_ARG, "SAP domains hold at most 256 sites");
  // FP32 keeps each thread's links and clover block in registers across the
  // MR steps; FP64 (twice the registers) reloads them from the caches
  constexpr int NG = 2;
  constexpr bool CACHE = sizeof(R) == 4;
  const int NQ = (A + 63) / 64;
  WCMG_LAUNCH((k_sap<R, NG, CACHE>), dim3(ndoms, nrhs), dim3(NG * NQ * 64), 0, st, x, b, U, clov, nbr, V, A, doms,
              iters, run, rs);
  WCMG_CHECK_LAUNCH();
}
template void launch_sap<float>(cf32*, const cf32*, const cf32*, const float*, const int*, long, int, const int*, int,
                                int, int, const int*, int, hipStream_t);
template void launch_sap<double>(cd64*, const cd64*, const cd64*, const double*, const int*, long, int, const int*,
                                 int, int, int, const int*, int, hipStream_t);

}  // namespace wcmg
