// Coarse-operator block format and the per-row block-stencil product shared by
// the coarse apply and the fused coarse GMRES.
//
// A 16-byte chunk holds K consecutive columns j of one block row, K = 1 (FP64),
// 2 (FP32), 4 (BF16 pairs).  Chunks are ordered [q = d * (Nb/K) + j/K][site * Nb + i]
// (d = 0: Mdiag, d = 1..8: Mdir in the order +x,-x,+y,-y,+z,-z,+t,-t), so lanes
// owning consecutive output rows read consecutive chunks.
#pragma once

#include "kernels.h"

namespace wcmg {

template <>
struct BlkTraits<WCMG_F64> {
  typedef double R;
  static constexpr int K = 1;
};
template <>
struct BlkTraits<WCMG_F32> {
  typedef float R;
  static constexpr int K = 2;
};
template <>
struct BlkTraits<WCMG_BF16> {
  typedef float R;
  static constexpr int K = 4;
};

struct alignas(16) Chunk16 {
  uint32_t w[4];
};
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// A chunk of the block stream, read once per apply: non-temporal, so the
// stream does not evict from L2 the neighbour vectors that nine sites share.
__device__ inline Chunk16 load_stream(const Chunk16* p) {
  const u32x4 raw = __builtin_nontemporal_load((const u32x4*)p);
  Chunk16 c;
  c.w[0] = raw.x;
  c.w[1] = raw.y;
  c.w[2] = raw.z;
  c.w[3] = raw.w;
  return c;
}

template <int P>
__device__ inline void decode(const Chunk16& c, cplx<typename BlkTraits<P>::R> (&m)[BlkTraits<P>::K]) {
  if constexpr (P == WCMG_F64) {
    m[0].re = __builtin_bit_cast(double, ((uint64_t)c.w[1] << 32) | c.w[0]);
    m[0].im = __builtin_bit_cast(double, ((uint64_t)c.w[3] << 32) | c.w[2]);
  } else if constexpr (P == WCMG_F32) {
    m[0].re = __builtin_bit_cast(float, c.w[0]);
    m[0].im = __builtin_bit_cast(float, c.w[1]);
    m[1].re = __builtin_bit_cast(float, c.w[2]);
    m[1].im = __builtin_bit_cast(float, c.w[3]);
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      m[k].re = __builtin_bit_cast(float, c.w[k] << 16);
      m[k].im = __builtin_bit_cast(float, c.w[k] & 0xffff0000u);
    }
  }
}

// Map the hardware workgroup index to a logical one so that each of the 8 XCDs
// (which receive workgroups round-robin) owns a contiguous range of rows.
__device__ inline long xcd_block(long b, long nb) {
  if (nb % 8 != 0) return b;
  return (b % 8) * (nb / 8) + b / 8;
}

// Row t of (D_c in) restricted to the directions in dmask, computed by S
// adjacent lanes (sub = 0..S-1) that split the nine blocks' chunks; every lane
// of the group returns the full sum.  `scale` multiplies the input vector.
template <int P, int NB, int S>
__device__ inline cplx<typename BlkTraits<P>::R> coarse_row(const Chunk16* __restrict__ blk,
                                                             const cplx<typename BlkTraits<P>::R>* __restrict__ in,
                                                             const int* __restrict__ nbr, long Vc, int nb_rt,
                                                             long t, int sub, int dmask, bool valid) {
  typedef typename BlkTraits<P>::R R;
  constexpr int K = BlkTraits<P>::K;
  const int nb = NB > 0 ? NB : nb_rt;
  const long rows = Vc * nb;
  const int nchunk = nb / K;
  cplx<R> acc = mkc((R)0, (R)0), acc2 = mkc((R)0, (R)0);
  if (valid) {
    const long site = t / nb;
    long src[9];
    src[0] = site;
#pragma unroll
    for (int d = 1; d < 9; ++d) src[d] = ((dmask >> d) & 1) ? (long)nbr[(long)(d - 1) * Vc + site] : 0;
    if (NB > 0) {
      constexpr int nq = 9 * (NB > 0 ? NB : K) / K;
#pragma unroll
      for (int q0 = 0; q0 < nq; q0 += S) {
        const int q = q0 + sub;
        if (q < nq) {
          const int d = q / (nq / 9), jc = q - d * (nq / 9);
          if ((dmask >> d) & 1) {
            const Chunk16 c = load_stream(blk + (long)q * rows + t);
            cplx<R> m[K];
            decode<P>(c, m);
            const cplx<R>* phi = in + src[d] * nb + jc * K;
#pragma unroll
            for (int k = 0; k < K; ++k) {
              if (k & 1) cfma(acc2, m[k], phi[k]);
              else cfma(acc, m[k], phi[k]);
            }
          }
        }
      }
    } else {
      const int nq = 9 * nchunk;
      for (int q = sub; q < nq; q += S) {
        const int d = q / nchunk, jc = q - d * nchunk;
        if (!((dmask >> d) & 1)) continue;
        const Chunk16 c = load_stream(blk + (long)q * rows + t);
        cplx<R> m[K];
        decode<P>(c, m);
        const cplx<R>* phi = in + src[d] * nb + jc * K;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          if (k & 1) cfma(acc2, m[k], phi[k]);
          else cfma(acc, m[k], phi[k]);
        }
      }
    }
  }
  acc = cadd(acc, acc2);
#pragma unroll
  for (int off = 1; off < S; off <<= 1) {
    acc.re += __shfl_xor(acc.re, off, 64);
    acc.im += __shfl_xor(acc.im, off, 64);
  }
  return acc;
}

// Sub-lanes per row for a launch of `rows` output rows: enough lanes to give
// every CU several waves on small (cache-resident) coarse lattices, one lane
// per row on large ones.
inline int coarse_split(long rows) {
  int S = 1;
  while (S < 8 && rows * S < 256L * 256 * 4) S <<= 1;
  return S;
}

}  // namespace wcmg
