// Even-odd (red-black) preconditioning of the fine operator (Sec. 2.1 and
// Sec. 4 name red-black preconditioning as a feature DDalphaAMG uses and the
// Grid implementation lacks, without writing it down).  Reading: sites are
// even or odd by the parity of x+y+z+t; with A = (4 + m0) + C and the hopping
// terms H_eo, H_oe between the parities,
//   Dhat = A_oo - H_oe A_ee^{-1} H_eo
// on the odd sites.  Fields keep their full length with the even part zero;
// the hops are the hopping-only Dslash, and the site-local pieces (A, its
// inverse, parity masks, the final reconstruction of x_e) are the kernels
// here.  A^{-1} is stored in the packed layout of A: per chirality a
// Hermitian 6 x 6 block as 6 diagonal reals and the 15 entries below the
// diagonal, in 16-byte chunks of a [2][36 / RC][V][RC] array.
#include "wilson_ops.h"

namespace wcmg {

namespace {
template <typename R>
__device__ inline void load_block(const R* __restrict__ blk, int chi, long V, long s, R (&e)[36]) {
  constexpr int RC = 16 / sizeof(R);
  typedef typename std::conditional<sizeof(R) == 4, float4, double2>::type V16;
  const V16* cb = (const V16*)(blk + (long)chi * 36 * V);
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
}

template <typename R>
__device__ inline void store_block(R* __restrict__ blk, int chi, long V, long s, const double (&e)[36]) {
  constexpr int RC = 16 / sizeof(R);
  typedef typename std::conditional<sizeof(R) == 4, float4, double2>::type V16;
  V16* cb = (V16*)(blk + (long)chi * 36 * V);
#pragma unroll
  for (int q = 0; q < 36 / RC; ++q) {
    V16 c;
    if constexpr (RC == 4) {
      c.x = (R)e[q * 4 + 0];
      c.y = (R)e[q * 4 + 1];
      c.z = (R)e[q * 4 + 2];
      c.w = (R)e[q * 4 + 3];
    } else {
      c.x = (R)e[q * 2 + 0];
      c.y = (R)e[q * 2 + 1];
    }
    cb[(long)q * V + s] = c;
  }
}
}  // namespace

// Per site and chirality: invert the Hermitian 6 x 6 block of A (FP64
// Gauss-Jordan elimination with partial pivoting; every row index is a
// compile-time constant, pivot rows are swapped by selects) and store the
// inverse, also Hermitian, packed in FP64 and FP32.  bad: set when a pivot
// vanishes.
__global__ void __launch_bounds__(128) k_clover_invert(const double* __restrict__ A, long V,
                                                        double* __restrict__ inv64, float* __restrict__ inv32,
                                                        int* __restrict__ bad) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= 2 * V) return;
  const int chi = (int)(t / V);
  const long s = t - chi * V;
  double e[36];
  load_block<double>(A, chi, V, s, e);
  cd64 m[6][6], w[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) w[i][j] = mkc(i == j ? 1.0 : 0.0, 0.0);
#pragma unroll
  for (int i = 0; i < 6; ++i) m[i][i] = mkc(e[i], 0.0);
  int idx = 0;
#pragma unroll
  for (int i = 1; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < i; ++j, ++idx) {
      m[i][j] = mkc(e[6 + 2 * idx], e[7 + 2 * idx]);
      m[j][i] = mkc(e[6 + 2 * idx], -e[7 + 2 * idx]);
    }
  bool singular = false;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    // pivot: the largest |m[r][k]|, r >= k
    int p = k;
    double best = m[k][k].re * m[k][k].re + m[k][k].im * m[k][k].im;
#pragma unroll
    for (int r = k + 1; r < 6; ++r) {
      const double a = m[r][k].re * m[r][k].re + m[r][k].im * m[r][k].im;
      if (a > best) {
        best = a;
        p = r;
      }
    }
    if (best == 0.0) singular = true;
#pragma unroll
    for (int r = k + 1; r < 6; ++r) {
      if (r == p) {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          const cd64 a = m[k][j], b = w[k][j];
          m[k][j] = m[r][j];
          w[k][j] = w[r][j];
          m[r][j] = a;
          w[r][j] = b;
        }
      }
    }
    const cd64 d = m[k][k];
    const double dn = d.re * d.re + d.im * d.im;
    const cd64 di = dn > 0.0 ? mkc(d.re / dn, -d.im / dn) : mkc(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      m[k][j] = cmul(m[k][j], di);
      w[k][j] = cmul(w[k][j], di);
    }
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      if (r == k) continue;
      const cd64 f = m[r][k];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        cfma(m[r][j], cneg(f), m[k][j]);
        cfma(w[r][j], cneg(f), w[k][j]);
      }
    }
  }
  if (singular) atomicOr(bad, 1);
  double o[36];
#pragma unroll
  for (int i = 0; i < 6; ++i) o[i] = w[i][i].re;
  idx = 0;
#pragma unroll
  for (int i = 1; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < i; ++j, ++idx) {
      o[6 + 2 * idx] = w[i][j].re;
      o[7 + 2 * idx] = w[i][j].im;
    }
  store_block<double>(inv64, chi, V, s, o);
  store_block<float>(inv32, chi, V, s, o);
}

// Parity-masked site-local operations (B: packed per-site blocks, A or A^{-1};
// sites with par != keep get 0, except in mode 3; in may alias out):
//   mode 0: out = B in        mode 1: out = B in - aux
//   mode 2: out = in          mode 3: out = B (in - aux) on parity keep, out kept elsewhere
//   mode 4: out = in - aux
template <typename R>
__global__ void __launch_bounds__(256) k_eo_local(const cplx<R>* in, const cplx<R>* __restrict__ aux,
                                                   cplx<R>* out, const R* __restrict__ B,
                                                   const unsigned char* __restrict__ par, int keep, int mode,
                                                   long V) {
  const long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= V) return;
  const bool on = par[s] == keep;
  if (!on) {
    if (mode != 3)
#pragma unroll
      for (int k = 0; k < 12; ++k) out[(long)k * V + s] = mkc((R)0, (R)0);
    return;
  }
  cplx<R> v[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    v[k] = in[(long)k * V + s];
    if (mode == 3 || mode == 4) v[k] = csub(v[k], aux[(long)k * V + s]);
  }
  if (mode == 2 || mode == 4) {
#pragma unroll
    for (int k = 0; k < 12; ++k) out[(long)k * V + s] = v[k];
    return;
  }
  cplx<R> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = mkc((R)0, (R)0);
  R e[36];
  cplx<R> p[6];
  load_block<R>(B, 0, V, s, e);
#pragma unroll
  for (int k = 0; k < 6; ++k) p[k] = v[k];
  clover_block_apply<R, 0>(acc, e, p);
  load_block<R>(B, 1, V, s, e);
#pragma unroll
  for (int k = 0; k < 6; ++k) p[k] = v[6 + k];
  clover_block_apply<R, 1>(acc, e, p);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    cplx<R> r = acc[k];
    if (mode == 1) r = csub(r, aux[(long)k * V + s]);
    out[(long)k * V + s] = r;
  }
}

namespace {
// One hop of the compact operator: the neighbour's spinor from the compact
// field of the other parity (pos: full site index -> compact index), the link
// from the full-lattice field.
template <typename R, int MU, bool FWD>
__device__ inline void hop_compact(cplx<R> (&acc)[12], const cplx<R>* __restrict__ in, const cplx<R>* __restrict__ U,
                                   const int* __restrict__ nbr, const int* __restrict__ pos, long V, long Vh, long s) {
  const long y = nbr[(long)(2 * MU + (FWD ? 0 : 1)) * V + s];
  const long yc = pos[y];
  cplx<R> p[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) p[k] = in[(long)k * Vh + yc];
  const long ls = FWD ? s : y;
  cplx<R> u[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = U[(long)(MU * 9 + e) * V + ls];
  hop_core<R, MU, FWD>(acc, p, u);
}

// o = B p for one chirality's Hermitian 6 x 6 block, packed as 6 diagonal
// reals and the 15 entries below the diagonal (B_ji = conj(B_ij)).
template <typename R>
__device__ inline void block6(const R (&e)[36], const cplx<R> (&p)[6], cplx<R> (&o)[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) o[i] = cscale(e[i], p[i]);
  int idx = 0;
#pragma unroll
  for (int i = 1; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < i; ++j, ++idx) {
      const cplx<R> a = mkc(e[6 + 2 * idx], e[7 + 2 * idx]);
      cfma(o[i], a, p[j]);
      cfmac(o[j], a, p[i]);
    }
}
}  // namespace

// The two halves of the Schur complement on parity-compact fields (each
// compact field holds one parity: component k of compact site j at k Vh + j).
// For the target sites tgt[j] (full index, compact index j): h = the eight
// hops from the other parity's values in `in`, then
//   mode 0: out_j = B h               (B = A^{-1}: u_e = A_ee^{-1} H_eo x_o)
//   mode 1: out_j = B aux_j - h       (B = A: y_o = A_oo x_o - H_oe u_e)
// B: the packed per-site blocks [2][36 / RC][V][RC] at the full index.
// A workgroup of 4 waves owns 64 target sites; wave mu takes the two hops
// along mu, the partial spinors meet in LDS in a fixed order, and waves 0 and
// 1 apply chirality 0 and 1 of the site-local block.
template <typename R>
__global__ void __launch_bounds__(256) k_schur_hop(const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out,
                                                    const cplx<R>* __restrict__ aux, const cplx<R>* __restrict__ U,
                                                    const R* __restrict__ B, const int* __restrict__ nbr,
                                                    const int* __restrict__ tgt, const int* __restrict__ pos, long V,
                                                    long Vh, int mode, const int* __restrict__ run) {
  if (run && !*run) return;
  long blk, r;
  if (!item_rhs((Vh + 63) / 64, 1, &blk, &r)) return;
  __shared__ cplx<R> part[4][12][64];
  const int lane = threadIdx.x & 63;
  const int mu = threadIdx.x >> 6;  // wave-uniform
  const long j = blk * 64 + lane;
  const bool valid = j < Vh;
  const long s = valid ? tgt[j] : 0;
  cplx<R> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = mkc((R)0, (R)0);
  if (valid) {
    if (mu == 0) {
      hop_compact<R, 0, true>(acc, in, U, nbr, pos, V, Vh, s);
      hop_compact<R, 0, false>(acc, in, U, nbr, pos, V, Vh, s);
    } else if (mu == 1) {
      hop_compact<R, 1, true>(acc, in, U, nbr, pos, V, Vh, s);
      hop_compact<R, 1, false>(acc, in, U, nbr, pos, V, Vh, s);
    } else if (mu == 2) {
      hop_compact<R, 2, true>(acc, in, U, nbr, pos, V, Vh, s);
      hop_compact<R, 2, false>(acc, in, U, nbr, pos, V, Vh, s);
    } else {
      hop_compact<R, 3, true>(acc, in, U, nbr, pos, V, Vh, s);
      hop_compact<R, 3, false>(acc, in, U, nbr, pos, V, Vh, s);
    }
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) part[mu][k][lane] = acc[k];
  __syncthreads();
  if (mu >= 2 || !valid) return;
  const int chi = mu;
  cplx<R> h[6], pin[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const int k = chi * 6 + i;
    h[i] = cadd(cadd(cadd(part[0][k][lane], part[1][k][lane]), part[2][k][lane]), part[3][k][lane]);
    pin[i] = mode == 0 ? h[i] : aux[(long)k * Vh + j];
  }
  R e[36];
  load_block<R>(B, chi, V, s, e);
  cplx<R> o[6];
  block6<R>(e, pin, o);
#pragma unroll
  for (int i = 0; i < 6; ++i) out[(long)(chi * 6 + i) * Vh + j] = mode == 1 ? csub(o[i], h[i]) : o[i];
}

template <typename R>
void launch_schur_hop(const cplx<R>* in, cplx<R>* out, const cplx<R>* aux, const cplx<R>* U, const R* B,
                      const int* nbr, const int* tgt, const int* pos, long V, long Vh, int mode, const int* run,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_schur_hop<R>, dim3(item_rhs_grid(nblocks(Vh, 64), 1)), dim3(kBlock), 0, st, in, out, aux, U,
                     B, nbr, tgt, pos, V, Vh, mode, run);
  WCMG_CHECK_LAUNCH();
}
template void launch_schur_hop<double>(const cd64*, cd64*, const cd64*, const cd64*, const double*, const int*,
                                       const int*, const int*, long, long, int, const int*, hipStream_t);

// Odd-site compaction: compact[k][j] = full[k][odd[j]] (gather), and
// full[k][s] = compact[k][pos[s]] on odd sites, 0 on even ones (scatter).
template <typename R>
__global__ void __launch_bounds__(256) k_eo_gather(const cplx<R>* __restrict__ full, cplx<R>* __restrict__ compact,
                                                    const int* __restrict__ odd, long V, long Vh) {
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (j >= Vh) return;
  const long s = odd[j];
#pragma unroll
  for (int k = 0; k < 12; ++k) compact[(long)k * Vh + j] = full[(long)k * V + s];
}

template <typename R>
__global__ void __launch_bounds__(256) k_eo_scatter(const cplx<R>* __restrict__ compact, cplx<R>* __restrict__ full,
                                                     const int* __restrict__ pos, const unsigned char* __restrict__ par,
                                                     long V, long Vh) {
  const long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= V) return;
  const bool odd = par[s] == 1;
  const long j = odd ? pos[s] : 0;
#pragma unroll
  for (int k = 0; k < 12; ++k) full[(long)k * V + s] = odd ? compact[(long)k * Vh + j] : mkc((R)0, (R)0);
}

template <typename R>
void launch_eo_gather(const cplx<R>* full, cplx<R>* compact, const int* odd, long V, long Vh, hipStream_t st) {
  hipLaunchKernelGGL(k_eo_gather<R>, dim3(nblocks(Vh)), dim3(kBlock), 0, st, full, compact, odd, V, Vh);
  WCMG_CHECK_LAUNCH();
}
template <typename R>
void launch_eo_scatter(const cplx<R>* compact, cplx<R>* full, const int* pos, const unsigned char* par, long V,
                       long Vh, hipStream_t st) {
  hipLaunchKernelGGL(k_eo_scatter<R>, dim3(nblocks(V)), dim3(kBlock), 0, st, compact, full, pos, par, V, Vh);
  WCMG_CHECK_LAUNCH();
}
template void launch_eo_gather<double>(const cd64*, cd64*, const int*, long, long, hipStream_t);
template void launch_eo_scatter<double>(const cd64*, cd64*, const int*, const unsigned char*, long, long,
                                        hipStream_t);

void launch_clover_invert(const double* A, long V, double* inv64, float* inv32, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_clover_invert, dim3(nblocks(2 * V, 128)), dim3(128), 0, st, A, V, inv64, inv32, bad);
  WCMG_CHECK_LAUNCH();
}

template <typename R>
void launch_eo_local(const cplx<R>* in, const cplx<R>* aux, cplx<R>* out, const R* B, const unsigned char* par,
                     int keep, int mode, long V, hipStream_t st) {
  hipLaunchKernelGGL(k_eo_local<R>, dim3(nblocks(V)), dim3(kBlock), 0, st, in, aux, out, B, par, keep, mode, V);
  WCMG_CHECK_LAUNCH();
}
template void launch_eo_local<double>(const cd64*, const cd64*, cd64*, const double*, const unsigned char*, int, int,
                                      long, hipStream_t);
template void launch_eo_local<float>(const cf32*, const cf32*, cf32*, const float*, const unsigned char*, int, int,
                                     long, hipStream_t);

}  // namespace wcmg
