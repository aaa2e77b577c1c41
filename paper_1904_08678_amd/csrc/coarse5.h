// Five-point coarse storage and its per-row block-stencil product, shared by
// the coarse apply and the fused coarse GMRES.
#pragma once

#include "coarse_common.h"

namespace wcmg {

// Only Mdiag and the forward blocks Mdir_{+mu} are stored (q = d5 * (Nb/K) + j/K,
// d5 = 0: Mdiag, d5 = 1 + mu: Mdir_{+mu}); the backward blocks follow from
// sigma3-hermiticity of the coarse operator (Sec. 2.2: P preserves chirality;
// Sec. 4: five independent stencil points),
//   Mdir_{-mu}(c) = s Mdir_{+mu}(c - mu)^dag s,   s = +1 on the first Nb/2
// components, -1 on the rest,
// so row i of the backward term is column i of the neighbour's forward block.
// The workgroup stages rows j of the forward blocks of the (-mu)-neighbours of
// its sites in LDS (coalesced: consecutive j are consecutive chunks) and every
// lane reads its column from there.
template <int P, int NB, int S>
struct Five {
  static constexpr int K = BlkTraits<P>::K;
  static constexpr int NCH = NB / K;           // chunks per block row
  static constexpr int RW = 256 / S;           // rows per workgroup
  static constexpr int SM = (RW - 1) / NB + 2; // sites a workgroup's rows can touch
  // rows j staged per round: the largest divisor of NB whose tile fits 20 KB
  // (several workgroups per CU stay resident)
  static constexpr int jt() {
    int best = 1;
    for (int d = 1; d <= NB; ++d)
      if (NB % d == 0 && SM * NCH * (d + 1) * 16 <= 20480) best = d;
    return best;
  }
  static constexpr int JT = jt();
};

template <int P>
__device__ inline cplx<typename BlkTraits<P>::R> chunk_elem(const Chunk16* c, int k) {
  typedef typename BlkTraits<P>::R R;
  if constexpr (P == WCMG_F64) {
    cplx<R> m[1];
    decode<P>(*c, m);
    return m[0];
  } else if constexpr (P == WCMG_F32) {
    return ((const cf32*)c)[k];
  } else {
    const uint32_t w = ((const uint32_t*)c)[k];
    return mkc(__builtin_bit_cast(float, w << 16), __builtin_bit_cast(float, w & 0xffff0000u));
  }
}

// Row t of D_c in from five-point storage.  Every thread of the (256-thread)
// workgroup must call it (it stages through LDS and synchronises); row0 is the
// workgroup's first row, and lanes with valid == false only help staging.
template <int P, int NB, int S>
__device__ inline cplx<typename BlkTraits<P>::R> coarse_row5(const Chunk16* __restrict__ blk,
                                                              const cplx<typename BlkTraits<P>::R>* __restrict__ in,
                                                              const int* __restrict__ nbr, long Vc, long row0,
                                                              long t, int sub, bool valid) {
  typedef typename BlkTraits<P>::R R;
  typedef Five<P, NB, S> F;
  constexpr int K = F::K, NCH = F::NCH, SM = F::SM, JT = F::JT;
  __shared__ Chunk16 tile[SM][NCH][JT + 1];
  const long rows = Vc * NB;
  const long site = valid ? t / NB : 0;
  const int i = (int)(t % NB);
  cplx<R> acc = mkc((R)0, (R)0), acc2 = mkc((R)0, (R)0);
  if (valid) {
    constexpr int nq = 5 * NCH;
#pragma unroll
    for (int q0 = 0; q0 < nq; q0 += S) {
      const int q = q0 + sub;
      if (q < nq) {
        const int d5 = q / NCH, jc = q - d5 * NCH;
        const long src = d5 == 0 ? site : (long)nbr[(long)(2 * d5 - 2) * Vc + site];
        const Chunk16 c = blk[(long)q * rows + t];
        cplx<R> m[K];
        decode<P>(c, m);
        const cplx<R>* phi = in + src * NB + jc * K;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          if (k & 1) cfma(acc2, m[k], phi[k]);
          else cfma(acc, m[k], phi[k]);
        }
      }
    }
  }
  // backward terms: s_i sum_j conj(Mdir_{+mu}(c')[j][i]) s_j in_j(c'), c' = c - mu
  const long s_lo = row0 / NB;
  const long s_hi = min(Vc - 1, (row0 + F::RW - 1) / NB);
  const int ns = (int)(s_hi - s_lo + 1);
  const int g = (int)(site - s_lo), qi = i / K, ki = i - qi * K;
  cplx<R> bwd = mkc((R)0, (R)0);
  for (int mu = 0; mu < 4; ++mu) {
    const long cm = valid ? (long)nbr[(long)(2 * mu + 1) * Vc + site] : 0;
    const cplx<R>* phi = in + cm * NB;
    for (int j0 = 0; j0 < NB; j0 += JT) {
      __syncthreads();
      for (int idx = threadIdx.x; idx < ns * NCH * JT; idx += blockDim.x) {
        const int jj = idx % JT, r2 = idx / JT, q = r2 % NCH, gg = r2 / NCH;
        const long cs = nbr[(long)(2 * mu + 1) * Vc + s_lo + gg];
        tile[gg][q][jj] = blk[(long)((1 + mu) * NCH + q) * rows + cs * NB + j0 + jj];
      }
      __syncthreads();
      if (valid) {
#pragma unroll
        for (int jj = sub; jj < JT; jj += S) {
          const int j = j0 + jj;
          const cplx<R> m = chunk_elem<P>(&tile[g][qi][jj], ki);
          cplx<R> x = phi[j];
          if (j >= NB / 2) x = mkc(-x.re, -x.im);
          cfmac(bwd, m, x);
        }
      }
    }
  }
  if (i >= NB / 2) bwd = mkc(-bwd.re, -bwd.im);
  acc = cadd(cadd(acc, acc2), bwd);
#pragma unroll
  for (int off = 1; off < S; off <<= 1) {
    acc.re += __shfl_xor(acc.re, off, 64);
    acc.im += __shfl_xor(acc.im, off, 64);
  }
  return acc;
}

}  // namespace wcmg
