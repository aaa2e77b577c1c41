// Intergrid operators and coarsening (Sec. 2.1 Aggregation / CoarsenedMatrix,
// Sec. 2.2 chirality-preserving prolongator, Sec. 3 blockProject).
//
// Restriction is owned per coarse site (one workgroup per aggregate, the
// race-free scheme of Sec. 3): the workgroup walks its aggregate through the
// coarse-to-fine lookup table, every lane accumulates partial inner products
// of one chirality, and a fixed-order wave + LDS reduction produces the
// coarse components.
// No atomics, so results are bitwise reproducible.
//
// Prolongator storage: P holds nv vectors [nv][level layout]; the chirality
// half chi of vector i, orthonormalised aggregate by aggregate, is column
// b = chi * nv + i of P (Sec. 2.2).  Chirality is implicit: nothing is stored
// twice and no explicit zeros are kept.
#include <type_traits>

#include "wilson_ops.h"

namespace wcmg {

// coarse(c, b) = sum_{x in c} sum_{k in chi(b)} conj(P_{b mod nv}(x)_k) fine(x)_k
// grid item_rhs_grid(Vc, nrhs), block 512: waves 0-3 take chirality 0 and
// waves 4-7 chirality 1 of the aggregate's sites (a lane per site), so each
// lane keeps nv accumulators and each wave reduces nv entries; the four
// waves of a chirality are then added in order in LDS.
template <typename R, int NB>
__global__ void __launch_bounds__(512) k_restrict(const cplx<R>* __restrict__ fine, cplx<R>* __restrict__ coarse,
                                                   const cplx<R>* __restrict__ P, FieldLayout lay,
                                                   const int* __restrict__ agg_sites, int A, long Vc,
                                                   int nrhs, const int* __restrict__ run, int rs) {
  long c, r;
  if (!item_rhs(Vc, nrhs, &c, &r)) return;
  if (run && !run[r * rs]) return;
  constexpr int nv = NB / 2;
  __shared__ cd64 lds[8][nv];
  fine += r * lay.size();
  coarse += r * Vc * NB;
  const int h = lay.ns / 2;
  const long pstride = lay.size();
  const int chi = threadIdx.x >> 8;  // wave-uniform
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  cd64 acc[nv];
#pragma unroll
  for (int i = 0; i < nv; ++i) acc[i] = mkc(0.0, 0.0);
  for (int o = threadIdx.x & 255; o < A; o += 256) {
    const long s = agg_sites[c * A + o];
    cplx<R> pa[nv];
#pragma unroll
    for (int i = 0; i < nv; ++i) pa[i] = mkc((R)0, (R)0);
    for (int k = 0; k < h; ++k) {
      const long e = lay.at(s, chi * h + k);
      const cplx<R> v = fine[e];
#pragma unroll
      for (int i = 0; i < nv; ++i) cfmac(pa[i], P[i * pstride + e], v);
    }
#pragma unroll
    for (int i = 0; i < nv; ++i) acc[i] = cadd(acc[i], ccast<double>(pa[i]));
  }
#pragma unroll
  for (int i = 0; i < nv; ++i) {
    double re = acc[i].re, im = acc[i].im;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      re += __shfl_xor(re, off, 64);
      im += __shfl_xor(im, off, 64);
    }
    if (lane == 0) lds[wave][i] = mkc(re, im);
  }
  __syncthreads();
  if (threadIdx.x < NB) {
    const int q = threadIdx.x / nv, i = threadIdx.x - q * nv;
    cd64 t = mkc(0.0, 0.0);
#pragma unroll
    for (int w = 0; w < 4; ++w) t = cadd(t, lds[4 * q + w][i]);
    coarse[c * NB + threadIdx.x] = ccast<R>(t);
  }
}

// k_restrict for FP32 fields whose aggregates have at most 256 sites and a
// number of components per chirality divisible by KP: each thread takes one
// site, so no FP64 accumulators are live while its loads are in flight, and it
// loads KP components' operands per pass (the same products in the same order,
// so the result equals k_restrict's bit for bit).
template <int NB, int KP>
__global__ void __launch_bounds__(512) k_restrict_one(const cf32* __restrict__ fine, cf32* __restrict__ coarse,
                                                       const cf32* __restrict__ P, FieldLayout lay,
                                                       const int* __restrict__ agg_sites, int A, long Vc, int nrhs,
                                                       const int* __restrict__ run, int rs) {
  long c, r;
  if (!item_rhs(Vc, nrhs, &c, &r)) return;
  if (run && !run[r * rs]) return;
  constexpr int nv = NB / 2;
  __shared__ cd64 lds[8][nv];
  fine += r * lay.size();
  coarse += r * Vc * NB;
  const int h = lay.ns / 2;
  const long pstride = lay.size();
  const int chi = threadIdx.x >> 8;  // wave-uniform
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int o = threadIdx.x & 255;
  cf32 pa[nv];
#pragma unroll
  for (int i = 0; i < nv; ++i) pa[i] = mkc(0.f, 0.f);
  if (o < A) {
    const long s = agg_sites[c * A + o];
    for (int k = 0; k < h; k += KP) {
      long e[KP];
      cf32 v[KP], pk[KP][nv];
#pragma unroll
      for (int q = 0; q < KP; ++q) {
        e[q] = lay.at(s, chi * h + k + q);
        v[q] = fine[e[q]];
      }
#pragma unroll
      for (int q = 0; q < KP; ++q)
#pragma unroll
        for (int i = 0; i < nv; ++i) pk[q][i] = P[i * pstride + e[q]];
#pragma unroll
      for (int i = 0; i < nv; ++i)
#pragma unroll
        for (int q = 0; q < KP; ++q) cfmac(pa[i], pk[q][i], v[q]);
    }
  }
#pragma unroll
  for (int i = 0; i < nv; ++i) {
    double re = (double)pa[i].re, im = (double)pa[i].im;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      re += __shfl_xor(re, off, 64);
      im += __shfl_xor(im, off, 64);
    }
    if (lane == 0) lds[wave][i] = mkc(re, im);
  }
  __syncthreads();
  if (threadIdx.x < NB) {
    const int q = threadIdx.x / nv, i = threadIdx.x - q * nv;
    cd64 t = mkc(0.0, 0.0);
#pragma unroll
    for (int w = 0; w < 4; ++w) t = cadd(t, lds[4 * q + w][i]);
    coarse[c * NB + threadIdx.x] = ccast<float>(t);
  }
}

// fine(x)_k (+)= sum_{i} P_i(x)_k coarse(c(x), chi(k) * nv + i); thread per site,
// grid item_rhs_grid(site blocks, nrhs).
template <typename R, int NB>
__global__ void __launch_bounds__(256) k_prolong(const cplx<R>* __restrict__ coarse, cplx<R>* __restrict__ fine,
                                                  const cplx<R>* __restrict__ P, FieldLayout lay,
                                                  const int* __restrict__ coarse_of, long Vc, int accumulate,
                                                  int nrhs, const int* __restrict__ run, int rs) {
  long sb, r;
  if (!item_rhs((lay.V + blockDim.x - 1) / blockDim.x, nrhs, &sb, &r)) return;
  if (run && !run[r * rs]) return;
  constexpr int nv = NB / 2;
  const long s = sb * blockDim.x + threadIdx.x;
  if (s >= lay.V) return;
  fine += r * lay.size();
  coarse += r * Vc * NB;
  const long c = coarse_of[s];
  const int h = lay.ns / 2;
  const long pstride = lay.size();
  cplx<R> phi[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) phi[b] = coarse[c * NB + b];
#pragma unroll
  for (int chi = 0; chi < 2; ++chi)
    for (int k = 0; k < h; ++k) {
      const long e = lay.at(s, chi * h + k);
      cplx<R> t = mkc((R)0, (R)0);
#pragma unroll
      for (int i = 0; i < nv; ++i) cfma(t, P[i * pstride + e], phi[chi * nv + i]);
      if (accumulate) t = cadd(t, fine[e]);
      fine[e] = t;
    }
}

// Several right-hand sides of a level-0 FP32 field (layout [B][12][V]) per
// launch, each aggregate's slice of P read once.  Padding workgroups (the grid
// is a multiple of the 8 XCDs) return at once.
__device__ inline long agg_of_block(long Vc) {
  const long G = gridDim.x, h = blockIdx.x;
  const long c = (h % 8) * (G / 8) + h / 8;  // each XCD a contiguous range of aggregates
  return c < Vc ? c : -1;
}

// coarse_r(c, chi * nv + i) = sum_{x in c} sum_{k < 6} conj(P_i(x)_{6 chi + k}) fine_r(x)_{6 chi + k}
// One workgroup of four waves per aggregate and chirality (blockIdx.y).  A lane
// is one of 16 consecutive sites of its wave's current group and one of four
// (vector half, right-hand-side half) variants, so a load instruction covers
// 16 sites of two arrays and every line of P and of the fields is requested
// once; a lane keeps NH x RH accumulators, summed over its sites at the end
// (shuffles within the 16 lanes of a variant, then the four waves in LDS).
template <int NB, int RH>
__global__ void __launch_bounds__(256) k_restrict_mrhs(const cf32* __restrict__ fine, cf32* __restrict__ coarse,
                                                    const cf32* __restrict__ P, long V,
                                                    const int* __restrict__ agg_sites, int A, long Vc, int nrhs,
                                                    const int* __restrict__ run, int rs) {
  constexpr int NV = NB / 2, NH = NV / 2;
  __shared__ cf32 red[4][4][NH * RH];  // [wave][variant][accumulator]
  const long c = agg_of_block(Vc);
  if (c < 0) return;  // the whole workgroup
  const int chi = blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int var = lane >> 4, sl = lane & 15;
  const int ih = var >> 1, rh = var & 1;
  bool act[RH];
#pragma unroll
  for (int j = 0; j < RH; ++j) {
    const int r = rh * RH + j;
    act[j] = r < nrhs && (!run || run[(long)r * rs]);
  }
  const long fs = 12 * V;
  cf32 acc[NH][RH];
#pragma unroll
  for (int i = 0; i < NH; ++i)
#pragma unroll
    for (int j = 0; j < RH; ++j) acc[i][j] = mkc(0.f, 0.f);
  for (int o0 = 16 * wave; o0 < A; o0 += 64) {
    const int o = o0 + sl;
    if (o < A) {
      const long s = agg_sites[c * A + o];
      constexpr int KU = 2;  // components whose loads are in flight together
#pragma unroll KU
      for (int k = 0; k < 6; ++k) {
        const long e = (long)(chi * 6 + k) * V + s;
        cf32 v[RH];
#pragma unroll
        for (int j = 0; j < RH; ++j) v[j] = act[j] ? fine[(long)(rh * RH + j) * fs + e] : mkc(0.f, 0.f);
#pragma unroll
        for (int i = 0; i < NH; ++i) {
          const cf32 p = P[(long)(ih * NH + i) * fs + e];
#pragma unroll
          for (int j = 0; j < RH; ++j) cfmac(acc[i][j], p, v[j]);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NH; ++i)
#pragma unroll
    for (int j = 0; j < RH; ++j) {
      float re = acc[i][j].re, im = acc[i][j].im;
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) {  // the 16 site lanes of this variant
        re += __shfl_xor(re, off, 64);
        im += __shfl_xor(im, off, 64);
      }
      if (sl == 0) red[wave][var][i * RH + j] = mkc(re, im);
    }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 4 * NH * RH) {
    const int v = t / (NH * RH), q = t - v * (NH * RH);
    const int i = q / RH, j = q - i * RH;
    const int r = (v & 1) * RH + j;
    cf32 sum = red[0][v][q];
#pragma unroll
    for (int w = 1; w < 4; ++w) sum = cadd(sum, red[w][v][q]);
    if (r < nrhs && (!run || run[(long)r * rs]))
      coarse[((long)r * Vc + c) * NB + chi * NV + (v >> 1) * NH + i] = sum;
  }
}

// fine_r(x)_{6 chi + k} (+)= sum_i P_i(x)_{6 chi + k} coarse_r(c(x), chi * nv + i).
// Four workgroups per aggregate, one per quarter of the spin-colour components
// (blockIdx.y: components 3y .. 3y + 2, chirality y / 2): the aggregate's
// coarse vectors of every right-hand side go to LDS (read back as
// broadcasts); a thread takes a site and all right-hand sides, so P is read
// once, in whole lines, with few registers per thread.
template <int NB>
__global__ void __launch_bounds__(256) k_prolong_mrhs(const cf32* __restrict__ coarse, cf32* __restrict__ fine,
                                                   const cf32* __restrict__ P, long V,
                                                   const int* __restrict__ agg_sites, int A, long Vc, int accumulate,
                                                   int nrhs, const int* __restrict__ run, int rs) {
  constexpr int NV = NB / 2;
  __shared__ cf32 cv[16][NB];
  __shared__ int live[16];
  const long c = agg_of_block(Vc);
  if (c < 0) return;  // the whole workgroup
  for (int t = threadIdx.x; t < nrhs * NB; t += blockDim.x) {
    const int r = t / NB, q = t - r * NB;
    cv[r][q] = coarse[((long)r * Vc + c) * NB + q];
  }
  if (threadIdx.x < 16) live[threadIdx.x] = threadIdx.x < nrhs && (!run || run[(long)threadIdx.x * rs]);
  __syncthreads();
  const long fs = 12 * V;
  const int chi = blockIdx.y >> 1;
  for (int o = threadIdx.x; o < A; o += blockDim.x) {
    const long s = agg_sites[c * A + o];
#pragma unroll 1
    for (int k = 3 * blockIdx.y; k < 3 * blockIdx.y + 3; ++k) {
      const long e = (long)k * V + s;
      cf32 p[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) p[i] = P[(long)i * fs + e];
      for (int r = 0; r < nrhs; ++r) {
        if (!live[r]) continue;
        cf32 t = mkc(0.f, 0.f);
#pragma unroll
        for (int i = 0; i < NV; ++i) cfma(t, p[i], cv[r][chi * NV + i]);
        cf32* out = fine + (long)r * fs + e;
        if (accumulate) t = cadd(t, *out);
        *out = t;
      }
    }
  }
}

// Per aggregate and chirality: modified Gram-Schmidt of the nv vectors in
// index order, each vector projected twice against the earlier ones, then
// normalised (FP64).  Breakdown when the projected norm falls below 1e-10 of
// the norm before projection.  grid (Vc, 2), block 256.
__device__ inline double block_sum1(double v, double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += lds[w];
  return s;
}

__global__ void __launch_bounds__(256) k_block_orthonormalise(cd64* __restrict__ vecs, FieldLayout lay,
                                                               const int* __restrict__ agg_sites, int A, int nv,
                                                               int* __restrict__ breakdown) {
  __shared__ double lds[16];
  const long c = blockIdx.x;
  const int chi = blockIdx.y;
  const int h = lay.ns / 2;
  const int nel = A * h;
  const long vstride = lay.size();
  auto elem = [&](int e) -> long {
    const int o = e % A, k = e / A;
    return lay.at(agg_sites[c * A + o], chi * h + k);
  };
  for (int i = 0; i < nv; ++i) {
    cd64* vi = vecs + i * vstride;
    double pre = 0.0;
    for (int e = threadIdx.x; e < nel; e += blockDim.x) {
      cd64 v = vi[elem(e)];
      pre += v.re * v.re + v.im * v.im;
    }
    pre = sqrt(block_sum1(pre, lds));
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < i; ++j) {
        const cd64* vj = vecs + j * vstride;
        double pr = 0.0, pi = 0.0;
        for (int e = threadIdx.x; e < nel; e += blockDim.x) {
          const long q = elem(e);
          cd64 a = vj[q], b = vi[q];
          pr += a.re * b.re + a.im * b.im;
          pi += a.re * b.im - a.im * b.re;
        }
        pr = block_sum1(pr, lds);
        pi = block_sum1(pi, lds);
        for (int e = threadIdx.x; e < nel; e += blockDim.x) {
          const long q = elem(e);
          cd64 a = vj[q], b = vi[q];
          b.re -= pr * a.re - pi * a.im;
          b.im -= pr * a.im + pi * a.re;
          vi[q] = b;
        }
        __syncthreads();
      }
    double post = 0.0;
    for (int e = threadIdx.x; e < nel; e += blockDim.x) {
      cd64 v = vi[elem(e)];
      post += v.re * v.re + v.im * v.im;
    }
    post = sqrt(block_sum1(post, lds));
    if (!(post > 1e-10 * pre) || pre == 0.0) {
      if (threadIdx.x == 0) atomicOr(breakdown, 1);
      post = post > 0.0 ? post : 1.0;
    }
    const double inv = 1.0 / post;
    for (int e = threadIdx.x; e < nel; e += blockDim.x) {
      const long q = elem(e);
      cd64 v = vi[q];
      vi[q] = mkc(v.re * inv, v.im * inv);
    }
    __syncthreads();
  }
}

// Register-resident variant for blocks of up to 4 * 512 elements: a workgroup
// of 512 threads holds the whole (aggregate, chirality) block of all NV vectors
// in registers (EPT elements per thread), reads and writes it once, and
// orthonormalises with classical Gram-Schmidt applied twice: the projections
// of vector i on all earlier vectors come out of one block reduction per pass
// (fixed order: waves in index order).  Same result as the modified form up to
// rounding; same breakdown rule.
template <int NV, int EPT>
__global__ void __launch_bounds__(512) k_block_orth_reg(cd64* __restrict__ vecs, FieldLayout lay,
                                                         const int* __restrict__ agg_sites, int A,
                                                         int* __restrict__ breakdown) {
  __shared__ cd64 red[8][NV];
  __shared__ cd64 tot[NV];
  const long c = blockIdx.x;
  const int chi = blockIdx.y;
  const int h = lay.ns / 2;
  const int nel = A * h;
  const long vs = lay.size();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  long q[EPT];
  bool ok[EPT];
#pragma unroll
  for (int t = 0; t < EPT; ++t) {
    const int e = threadIdx.x + t * (int)blockDim.x;
    ok[t] = e < nel;
    const int o = ok[t] ? e % A : 0, k = ok[t] ? e / A : 0;
    q[t] = lay.at(agg_sites[c * A + o], chi * h + k);
  }
  cd64 v[NV][EPT];
#pragma unroll
  for (int j = 0; j < NV; ++j)
#pragma unroll
    for (int t = 0; t < EPT; ++t) v[j][t] = ok[t] ? vecs[j * vs + q[t]] : mkc(0.0, 0.0);
  // wave-reduce one complex value into red[wave][slot]
  auto wave_put = [&](double re, double im, int slot) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      re += __shfl_xor(re, off, 64);
      im += __shfl_xor(im, off, 64);
    }
    if (lane == 0) red[wave][slot] = mkc(re, im);
  };
  // sum the n slots over the waves in index order into tot
  auto finish = [&](int n) {
    __syncthreads();
    if ((int)threadIdx.x < n) {
      cd64 s = mkc(0.0, 0.0);
      for (int w = 0; w < nw; ++w) s = cadd(s, red[w][threadIdx.x]);
      tot[threadIdx.x] = s;
    }
    __syncthreads();
  };
  for (int i = 0; i < NV; ++i) {
    cd64 vi[EPT];
#pragma unroll
    for (int j = 0; j < NV; ++j)
      if (j == i)
#pragma unroll
        for (int t = 0; t < EPT; ++t) vi[t] = v[j][t];
    double n2 = 0.0;
#pragma unroll
    for (int t = 0; t < EPT; ++t) n2 += vi[t].re * vi[t].re + vi[t].im * vi[t].im;
    wave_put(n2, 0.0, 0);
    finish(1);
    const double pre = sqrt(tot[0].re);
    for (int pass = 0; pass < 2 && i > 0; ++pass) {
#pragma unroll
      for (int j = 0; j < NV; ++j)
        if (j < i) {
          double pr = 0.0, pim = 0.0;
#pragma unroll
          for (int t = 0; t < EPT; ++t) {
            pr += v[j][t].re * vi[t].re + v[j][t].im * vi[t].im;
            pim += v[j][t].re * vi[t].im - v[j][t].im * vi[t].re;
          }
          wave_put(pr, pim, j);
        }
      finish(i);
#pragma unroll
      for (int j = 0; j < NV; ++j)
        if (j < i) {
          const cd64 pj = tot[j];
#pragma unroll
          for (int t = 0; t < EPT; ++t) {
            vi[t].re -= pj.re * v[j][t].re - pj.im * v[j][t].im;
            vi[t].im -= pj.re * v[j][t].im + pj.im * v[j][t].re;
          }
        }
    }
    n2 = 0.0;
#pragma unroll
    for (int t = 0; t < EPT; ++t) n2 += vi[t].re * vi[t].re + vi[t].im * vi[t].im;
    wave_put(n2, 0.0, 0);
    finish(1);
    double post = sqrt(tot[0].re);
    if (!(post > 1e-10 * pre) || pre == 0.0) {
      if (threadIdx.x == 0) atomicOr(breakdown, 1);
      post = post > 0.0 ? post : 1.0;
    }
    const double inv = 1.0 / post;
#pragma unroll
    for (int j = 0; j < NV; ++j)
      if (j == i)
#pragma unroll
        for (int t = 0; t < EPT; ++t) v[j][t] = mkc(vi[t].re * inv, vi[t].im * inv);
  }
#pragma unroll
  for (int j = 0; j < NV; ++j)
#pragma unroll
    for (int t = 0; t < EPT; ++t)
      if (ok[t]) vecs[j * vs + q[t]] = v[j][t];
}

// Column fields of P: col_b(x)_k = P_{b mod nv}(x)_k on chirality half b / nv,
// zero on the other half.  out [NB][layout].  grid (sites, NB).
__global__ void k_prolongator_columns(const cd64* __restrict__ P, FieldLayout lay, int nv, cd64* __restrict__ out) {
  const long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= lay.V) return;
  const int b = blockIdx.y;
  const int i = b % nv, chi = b / nv;
  const int h = lay.ns / 2;
  for (int k = 0; k < lay.ns; ++k) {
    const long e = lay.at(s, k);
    out[b * lay.size() + e] = (k / h == chi) ? P[i * lay.size() + e] : mkc(0.0, 0.0);
  }
}

// Galerkin projection of one term of the level operator (Sec. 2.1 CoarsenOperator):
// W_b = Mdir_d(column b of P) (or Mdiag for d = 0) is projected on the rows of
// P aggregate by aggregate; contributions of sites whose d-neighbour lies in
// the same aggregate go to block 0, the rest to block d.
//
// One workgroup per aggregate computes, chirality by chirality, the small
// product P_chi^dag W_chi (nv x NB, K = A * ns/2 rows) for both targets at once:
// row tiles of P and W are staged in LDS (one coalesced read of each from
// HBM), each thread accumulates an AB x BB block of outputs for both targets
// over the rows of its row group, and the row groups are added in a fixed
// order.  FP64.
template <int NB, int AB, int BB>
__global__ void __launch_bounds__(256) k_galerkin_project(const cd64* __restrict__ W, const cd64* __restrict__ P,
                                                           FieldLayout lay, const int* __restrict__ agg_sites,
                                                           const int* __restrict__ coarse_of,
                                                           const int* __restrict__ nbr_d, int A, long Vc, int d,
                                                           int dint, cd64* __restrict__ M) {
  constexpr int nv = NB / 2;
  constexpr int T = 32;  // rows per tile
  constexpr int TPG = (nv / AB) * (NB / BB);  // threads per row group
  __shared__ cd64 Pt[T][nv], Wt[T][NB];
  __shared__ cd64 res[2][nv][NB];
  __shared__ unsigned char ext[T];
  const long c = blockIdx.x;
  const int tid = threadIdx.x;
  const int ngroups = (int)blockDim.x / TPG;
  const int grp = tid / TPG, q = tid - grp * TPG;
  const bool active = grp < ngroups;
  const int a0 = (q / (NB / BB)) * AB, b0 = (q % (NB / BB)) * BB;
  const int h = lay.ns / 2;
  const int R = A * h;
  const long vs = lay.size();
  for (int chi = 0; chi < 2; ++chi) {
    cd64 acc[2][AB][BB];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int x = 0; x < AB; ++x)
#pragma unroll
        for (int y = 0; y < BB; ++y) acc[t][x][y] = mkc(0.0, 0.0);
    for (int r0 = 0; r0 < R; r0 += T) {
      const int nr = min(T, R - r0);
      __syncthreads();
      // rows ordered so that consecutive rows are consecutive in memory
      for (int idx = tid; idx < nr * (nv + NB); idx += blockDim.x) {
        const int rr = idx % nr, col = idx / nr;
        const int r = r0 + rr;
        const int o = lay.soa ? r % A : r / h, k = lay.soa ? r / A : r % h;
        const long sidx = agg_sites[c * A + o];
        const long e = lay.at(sidx, chi * h + k);
        if (col < nv) Pt[rr][col] = P[col * vs + e];
        else Wt[rr][col - nv] = W[(col - nv) * vs + e];
        if (col == 0) ext[rr] = (d != 0 && coarse_of[nbr_d[sidx]] != c) ? 1 : 0;
      }
      __syncthreads();
      if (active) {
        for (int rr = grp; rr < nr; rr += ngroups) {
          cd64 p[AB], w[BB];
#pragma unroll
          for (int x = 0; x < AB; ++x) p[x] = Pt[rr][a0 + x];
#pragma unroll
          for (int y = 0; y < BB; ++y) w[y] = Wt[rr][b0 + y];
          if (ext[rr]) {
#pragma unroll
            for (int x = 0; x < AB; ++x)
#pragma unroll
              for (int y = 0; y < BB; ++y) cfmac(acc[1][x][y], p[x], w[y]);
          } else {
#pragma unroll
            for (int x = 0; x < AB; ++x)
#pragma unroll
              for (int y = 0; y < BB; ++y) cfmac(acc[0][x][y], p[x], w[y]);
          }
        }
      }
    }
    // row groups added in index order
    for (int g = 0; g < ngroups; ++g) {
      __syncthreads();
      if (active && grp == g)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int x = 0; x < AB; ++x)
#pragma unroll
            for (int y = 0; y < BB; ++y)
              res[t][a0 + x][b0 + y] = g == 0 ? acc[t][x][y] : cadd(res[t][a0 + x][b0 + y], acc[t][x][y]);
    }
    __syncthreads();
    for (int e = tid; e < 2 * nv * NB; e += blockDim.x) {
      const int t = e / (nv * NB), ab = e - t * nv * NB, a = ab / NB, b = ab - a * NB;
      if (t == 1 && d == 0) continue;
      const int dd = t == 0 ? dint : d;
      cd64* m = M + ((c * 9 + dd) * NB + chi * nv + a) * NB + b;
      *m = cadd(*m, res[t][a][b]);
    }
  }
}

// Level 0 without the intermediate images: column (i, chi) of P is the
// chirality-chi half of vector i, and its image under Mdir_d at site x is the
// hop of that half-spinor from the d-neighbour (under Mdiag: the chirality-chi
// block of (4 + m0) + C at x).  Per tile of TS sites the images of all NB
// columns are formed in LDS for the components of the chirality being
// projected, then projected as in k_galerkin_project.  FP64.
namespace {
__device__ inline void image_hop(int d, cd64 (&acc)[12], const cd64 (&p)[12], const cd64 (&u)[9]) {
  switch (d) {
    case 1: hop_core<double, 0, true>(acc, p, u); break;
    case 2: hop_core<double, 0, false>(acc, p, u); break;
    case 3: hop_core<double, 1, true>(acc, p, u); break;
    case 4: hop_core<double, 1, false>(acc, p, u); break;
    case 5: hop_core<double, 2, true>(acc, p, u); break;
    case 6: hop_core<double, 2, false>(acc, p, u); break;
    case 7: hop_core<double, 3, true>(acc, p, u); break;
    default: hop_core<double, 3, false>(acc, p, u); break;
  }
}
}  // namespace

template <int NB, int AB, int BB>
__global__ void __launch_bounds__(256) k_galerkin_fused(const cd64* __restrict__ P, const cd64* __restrict__ U,
                                                         const double* __restrict__ clov, const int* __restrict__ nbr,
                                                         long V, const int* __restrict__ agg_sites,
                                                         const int* __restrict__ coarse_of, int A, int d, int dint,
                                                         cd64* __restrict__ M) {
  constexpr int nv = NB / 2;
  constexpr int TS = 8, T = TS * 6;  // sites and rows per tile
  constexpr int TPG = (nv / AB) * (NB / BB);
  __shared__ cd64 Pt[T][nv], Wt[T][NB];
  __shared__ cd64 res[2][nv][NB];
  __shared__ unsigned char ext[TS];
  const long c = blockIdx.x;
  const int tid = threadIdx.x;
  const int ngroups = (int)blockDim.x / TPG;
  const int grp = tid / TPG, q = tid - grp * TPG;
  const bool active = grp < ngroups;
  const int a0 = (q / (NB / BB)) * AB, b0 = (q % (NB / BB)) * BB;
  const long vs = 12 * V;
  for (int chi = 0; chi < 2; ++chi) {
    cd64 acc[2][AB][BB];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int x = 0; x < AB; ++x)
#pragma unroll
        for (int y = 0; y < BB; ++y) acc[t][x][y] = mkc(0.0, 0.0);
    for (int o0 = 0; o0 < A; o0 += TS) {
      const int ns = min(TS, A - o0);
      __syncthreads();
      // rows of P for the components of chirality chi
      for (int idx = tid; idx < ns * 6 * nv; idx += blockDim.x) {
        const int ts = idx % ns, r2 = idx / ns, kk = r2 % 6, a = r2 / 6;
        const long x = agg_sites[c * A + o0 + ts];
        Pt[ts * 6 + kk][a] = P[a * vs + (long)(chi * 6 + kk) * V + x];
      }
      // images of the columns at the tile's sites
      for (int item = tid; item < ns * NB; item += blockDim.x) {
        const int ts = item % ns, b = item / ns;
        const int cb = b / nv, i = b - cb * nv;
        const long x = agg_sites[c * A + o0 + ts];
        const cd64* Pi = P + i * vs;
        cd64 img[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) img[k] = mkc(0.0, 0.0);
        if (d == 0) {
          if (cb == 0) clover_chirality<double, 0>(img, Pi, clov, V, x);
          else clover_chirality<double, 1>(img, Pi, clov, V, x);
        } else {
          const long y = nbr[(long)(d - 1) * V + x];
          const int mu = (d - 1) >> 1;
          const long ls = (d & 1) ? x : y;
          cd64 p[12], u[9];
#pragma unroll
          for (int k = 0; k < 12; ++k) p[k] = (k / 6 == cb) ? Pi[(long)k * V + y] : mkc(0.0, 0.0);
#pragma unroll
          for (int e = 0; e < 9; ++e) u[e] = U[(long)(mu * 9 + e) * V + ls];
          image_hop(d, img, p, u);
        }
#pragma unroll
        for (int kk = 0; kk < 6; ++kk) {
          // select component chi * 6 + kk without dynamic register indexing
          cd64 v = img[kk];
          if (chi == 1) v = img[6 + kk];
          Wt[ts * 6 + kk][b] = v;
        }
        if (b == 0) ext[ts] = (d != 0 && coarse_of[nbr[(long)(d - 1) * V + x]] != c) ? 1 : 0;
      }
      __syncthreads();
      if (active) {
        for (int rr = grp; rr < ns * 6; rr += ngroups) {
          cd64 p[AB], w[BB];
#pragma unroll
          for (int x = 0; x < AB; ++x) p[x] = Pt[rr][a0 + x];
#pragma unroll
          for (int y = 0; y < BB; ++y) w[y] = Wt[rr][b0 + y];
          if (ext[rr / 6]) {
#pragma unroll
            for (int x = 0; x < AB; ++x)
#pragma unroll
              for (int y = 0; y < BB; ++y) cfmac(acc[1][x][y], p[x], w[y]);
          } else {
#pragma unroll
            for (int x = 0; x < AB; ++x)
#pragma unroll
              for (int y = 0; y < BB; ++y) cfmac(acc[0][x][y], p[x], w[y]);
          }
        }
      }
    }
    for (int g = 0; g < ngroups; ++g) {
      __syncthreads();
      if (active && grp == g)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int x = 0; x < AB; ++x)
#pragma unroll
            for (int y = 0; y < BB; ++y)
              res[t][a0 + x][b0 + y] = g == 0 ? acc[t][x][y] : cadd(res[t][a0 + x][b0 + y], acc[t][x][y]);
    }
    __syncthreads();
    for (int e = tid; e < 2 * nv * NB; e += blockDim.x) {
      const int t = e / (nv * NB), ab = e - t * nv * NB, a = ab / NB, b = ab - a * NB;
      if (t == 1 && d == 0) continue;
      const int dd = t == 0 ? dint : d;
      cd64* m = M + ((c * 9 + dd) * NB + chi * nv + a) * NB + b;
      *m = cadd(*m, res[t][a][b]);
    }
  }
}

// ---------------------------------------------------------------- launchers
#define NB_SWITCH(nb, ...)                                     \
  switch (nb) {                                                 \
    case 8: { constexpr int NBc = 8; __VA_ARGS__; } break;            \
    case 12: { constexpr int NBc = 12; __VA_ARGS__; } break;          \
    case 16: { constexpr int NBc = 16; __VA_ARGS__; } break;          \
    case 24: { constexpr int NBc = 24; __VA_ARGS__; } break;          \
    case 32: { constexpr int NBc = 32; __VA_ARGS__; } break;          \
    case 40: { constexpr int NBc = 40; __VA_ARGS__; } break;          \
    case 4: { constexpr int NBc = 4; __VA_ARGS__; } break;            \
    case 6: { constexpr int NBc = 6; __VA_ARGS__; } break;            \
    case 20: { constexpr int NBc = 20; __VA_ARGS__; } break;          \
    default: throw Error(WCMG_ERR_ARG, "unsupported coarse block size Nb = " + std::to_string(nb)); \
  }

bool supported_nb(int nb) {
  return nb == 4 || nb == 6 || nb == 8 || nb == 12 || nb == 16 || nb == 20 || nb == 24 || nb == 32 || nb == 40;
}

// The multi-RHS forms serve FP32 level-0 fields with 2..16 right-hand sides
// and Nb in {8, 12, 16, 24}.
static bool transfer_mrhs(int nb, int nrhs, const FieldLayout& lay) {
  return lay.soa && lay.ns == 12 && nrhs >= 2 && nrhs <= 16 && (nb == 8 || nb == 12 || nb == 16 || nb == 24);
}
// right-hand sides per half in the restriction: ceil(nrhs / 2) rounded up to 1, 2, 4, 6 or 8
#define RH_SWITCH(nrhs, ...)                                                    \
  switch ((nrhs + 1) / 2) {                                                     \
    case 1: { constexpr int RHc = 1; __VA_ARGS__; } break;                      \
    case 2: { constexpr int RHc = 2; __VA_ARGS__; } break;                      \
    case 3:                                                                     \
    case 4: { constexpr int RHc = 4; __VA_ARGS__; } break;                      \
    case 5:                                                                     \
    case 6: { constexpr int RHc = 6; __VA_ARGS__; } break;                      \
    default: { constexpr int RHc = 8; __VA_ARGS__; } break;                     \
  }
#define NB_SWITCH_MRHS(nb, ...)                                                 \
  switch (nb) {                                                                 \
    case 8: { constexpr int NBc = 8; __VA_ARGS__; } break;                      \
    case 12: { constexpr int NBc = 12; __VA_ARGS__; } break;                    \
    case 16: { constexpr int NBc = 16; __VA_ARGS__; } break;                    \
    default: { constexpr int NBc = 24; __VA_ARGS__; } break;                    \
  }

template <typename R>
void launch_restrict(const cplx<R>* fine, cplx<R>* coarse, const cplx<R>* P, FieldLayout lay, const int* agg_sites,
                     int A, long Vc, int nb, int nrhs, const int* run, hipStream_t st, int rs) {
  if (std::is_same<R, float>::value && transfer_mrhs(nb, nrhs, lay)) {
    const dim3 g((unsigned)((Vc + 7) / 8 * 8), 2);
    NB_SWITCH_MRHS(nb, RH_SWITCH(nrhs, WCMG_LAUNCH((k_restrict_mrhs<NBc, RHc>), g, dim3(256), 0, st, (const cf32*)fine,
                                                   (cf32*)coarse, (const cf32*)P, lay.V, agg_sites, A, Vc, nrhs, run,
                                                   rs)));
  } else if (std::is_same<R, float>::value && A <= 256 && (lay.ns / 2) % 3 == 0) {
    NB_SWITCH(nb, WCMG_LAUNCH((k_restrict_one<NBc, 3>), dim3(item_rhs_grid(Vc, nrhs)), dim3(512), 0, st,
                               (const cf32*)fine, (cf32*)coarse, (const cf32*)P, lay, agg_sites, A, Vc, nrhs, run,
                               rs));
  } else if (std::is_same<R, float>::value && A <= 256 && (lay.ns / 2) % 2 == 0) {
    NB_SWITCH(nb, WCMG_LAUNCH((k_restrict_one<NBc, 2>), dim3(item_rhs_grid(Vc, nrhs)), dim3(512), 0, st,
                               (const cf32*)fine, (cf32*)coarse, (const cf32*)P, lay, agg_sites, A, Vc, nrhs, run,
                               rs));
  } else {
    NB_SWITCH(nb, WCMG_LAUNCH((k_restrict<R, NBc>), dim3(item_rhs_grid(Vc, nrhs)), dim3(512), 0, st, fine, coarse, P,
                               lay, agg_sites, A, Vc, nrhs, run, rs));
  }
  WCMG_CHECK_LAUNCH();
}
template <typename R>
void launch_prolong(const cplx<R>* coarse, cplx<R>* fine, const cplx<R>* P, FieldLayout lay, const int* coarse_of,
                    long Vc, int nb, int accumulate, int nrhs, const int* run, hipStream_t st, int rs,
                    const int* agg_sites, int A) {
  if (std::is_same<R, float>::value && agg_sites && transfer_mrhs(nb, nrhs, lay)) {
    const dim3 g((unsigned)((Vc + 7) / 8 * 8), 4);
    NB_SWITCH_MRHS(nb, WCMG_LAUNCH((k_prolong_mrhs<NBc>), g, dim3(256), 0, st, (const cf32*)coarse, (cf32*)fine,
                                   (const cf32*)P, lay.V, agg_sites, A, Vc, accumulate, nrhs, run, rs));
  } else {
    NB_SWITCH(nb, WCMG_LAUNCH((k_prolong<R, NBc>), dim3(item_rhs_grid(nblocks(lay.V), nrhs)), dim3(kBlock), 0, st,
                               coarse, fine, P, lay, coarse_of, Vc, accumulate, nrhs, run, rs));
  }
  WCMG_CHECK_LAUNCH();
}
#define INST_TR(R)                                                                                                 \
  template void launch_restrict<R>(const cplx<R>*, cplx<R>*, const cplx<R>*, FieldLayout, const int*, int, long, int, \
                                   int, const int*, hipStream_t, int);                                             \
  template void launch_prolong<R>(const cplx<R>*, cplx<R>*, const cplx<R>*, FieldLayout, const int*, long, int, int, \
                                  int, const int*, hipStream_t, int, const int*, int);
INST_TR(double)
INST_TR(float)

template <int NV>
static bool orth_reg(int ept, cd64* vecs, FieldLayout lay, const int* agg_sites, int A, long Vc, int* breakdown,
                     hipStream_t st) {
  const dim3 g((unsigned)Vc, 2), b(512);
  switch (ept) {
    case 1: hipLaunchKernelGGL((k_block_orth_reg<NV, 1>), g, b, 0, st, vecs, lay, agg_sites, A, breakdown); return true;
    case 2: hipLaunchKernelGGL((k_block_orth_reg<NV, 2>), g, b, 0, st, vecs, lay, agg_sites, A, breakdown); return true;
    case 3: hipLaunchKernelGGL((k_block_orth_reg<NV, 3>), g, b, 0, st, vecs, lay, agg_sites, A, breakdown); return true;
    default: return false;
  }
}

void launch_block_orthonormalise(cd64* vecs, FieldLayout lay, const int* agg_sites, int A, long Vc, int nv,
                                 int* breakdown, hipStream_t st) {
  const int ept = (A * (lay.ns / 2) + 511) / 512;
  bool done = false;
  switch (nv) {  // register-resident form for the common block sizes
    case 4: done = orth_reg<4>(ept, vecs, lay, agg_sites, A, Vc, breakdown, st); break;
    case 6: done = orth_reg<6>(ept, vecs, lay, agg_sites, A, Vc, breakdown, st); break;
    case 8: done = orth_reg<8>(ept, vecs, lay, agg_sites, A, Vc, breakdown, st); break;
    case 12: done = orth_reg<12>(ept, vecs, lay, agg_sites, A, Vc, breakdown, st); break;
    case 16: done = ept <= 2 && orth_reg<16>(ept, vecs, lay, agg_sites, A, Vc, breakdown, st); break;
    default: break;
  }
  if (!done)
    hipLaunchKernelGGL(k_block_orthonormalise, dim3(Vc, 2), dim3(kBlock), 0, st, vecs, lay, agg_sites, A, nv,
                       breakdown);
  WCMG_CHECK_LAUNCH();
}

void launch_prolongator_columns(const cd64* P, FieldLayout lay, int nv, cd64* out, hipStream_t st) {
  hipLaunchKernelGGL(k_prolongator_columns, dim3(nblocks(lay.V), 2 * nv), dim3(kBlock), 0, st, P, lay, nv, out);
  WCMG_CHECK_LAUNCH();
}

void launch_galerkin_fused(const cd64* P, const cd64* U, const double* clov, const int* nbr, long V,
                           const int* agg_sites, const int* coarse_of, int A, long Vc, int nb, int d, int dint,
                           cd64* M, hipStream_t st) {
  NB_SWITCH(nb, hipLaunchKernelGGL((k_galerkin_fused<NBc, (NBc / 2) % 2 == 0 ? 2 : 1, NBc % 4 == 0 ? 4 : 2>),
                                    dim3(Vc), dim3(kBlock), 0, st, P, U, clov, nbr, V, agg_sites, coarse_of, A, d,
                                    dint, M));
  WCMG_CHECK_LAUNCH();
}

void launch_galerkin_project(const cd64* W, const cd64* P, FieldLayout lay, const int* agg_sites,
                             const int* coarse_of, const int* nbr_d, int A, long Vc, int nb, int d, int dint,
                             cd64* M, hipStream_t st) {
  NB_SWITCH(nb, hipLaunchKernelGGL((k_galerkin_project<NBc, (NBc / 2) % 2 == 0 ? 2 : 1, NBc % 4 == 0 ? 4 : 2>),
                                    dim3(Vc), dim3(kBlock), 0, st, W, P, lay, agg_sites, coarse_of, nbr_d, A, Vc, d,
                                    dint, M));
  WCMG_CHECK_LAUNCH();
}

// The backward terms from the forward ones.  The level operator is
// gamma5-hermitian term by term (the -mu hop is the gamma5-conjugated adjoint
// of the +mu hop) and P preserves chirality, so with s = sigma3 = +1 on the
// first Nb/2 coarse components and -1 on the rest (Sec. 2.2),
//   Mdir_{-mu}(c) = s Mdir_{+mu}(c - mu)^dag s,
// and the part of Mdiag that -mu hops inside an aggregate contribute is
// s X_mu^dag s, X_mu being the part from the +mu hops inside it.  On entry the
// -mu slot of site c holds X_mu; the first kernel adds X_mu + s X_mu^dag s to
// Mdiag (mu in order), the second overwrites the -mu slots.  FP64.
__global__ void k_mirror_diag(cd64* __restrict__ M, long Vc, int nb) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long per = (long)nb * nb;
  if (e >= Vc * per) return;
  const long c = e / per;
  const int i = (int)((e % per) / nb), j = (int)(e % nb);
  const double sij = ((i < nb / 2) == (j < nb / 2)) ? 1.0 : -1.0;
  cd64* Mc = M + c * 9 * per;
  cd64 acc = Mc[(long)i * nb + j];
  for (int mu = 0; mu < 4; ++mu) {
    const cd64* X = Mc + (2 * mu + 2) * per;
    const cd64 a = X[(long)i * nb + j], b = X[(long)j * nb + i];
    acc = cadd(acc, a);
    acc = cadd(acc, mkc(sij * b.re, -sij * b.im));
  }
  Mc[(long)i * nb + j] = acc;
}

__global__ void k_mirror_hops(cd64* __restrict__ M, const int* __restrict__ nbr, long Vc, int nb) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long per = (long)nb * nb;
  if (e >= 4 * Vc * per) return;
  const int mu = (int)(e / (Vc * per));
  const long r = e % (Vc * per);
  const long c = r / per;
  const int i = (int)((r % per) / nb), j = (int)(r % nb);
  const double sij = ((i < nb / 2) == (j < nb / 2)) ? 1.0 : -1.0;
  const long cm = nbr[(long)(2 * mu + 1) * Vc + c];  // c - mu
  const cd64 b = M[(cm * 9 + 2 * mu + 1) * per + (long)j * nb + i];
  M[(c * 9 + 2 * mu + 2) * per + (long)i * nb + j] = mkc(sij * b.re, -sij * b.im);
}

void launch_galerkin_mirror(cd64* M, const int* nbr_c, long Vc, int nb, hipStream_t st) {
  const long per = (long)nb * nb;
  hipLaunchKernelGGL(k_mirror_diag, dim3(nblocks(Vc * per)), dim3(kBlock), 0, st, M, Vc, nb);
  hipLaunchKernelGGL(k_mirror_hops, dim3(nblocks(4 * Vc * per)), dim3(kBlock), 0, st, M, nbr_c, Vc, nb);
  WCMG_CHECK_LAUNCH();
}

}  // namespace wcmg
