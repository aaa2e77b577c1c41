// Coarse operator: application of Mdiag plus the eight Mdir blocks
// (Sec. 2.1: the coarse matrix is applied through its diagonal part and its
// hops in single directions; nine dense Nb x Nb complex blocks per site).
//
// One thread owns one output row (site, i): it streams row i of the nine
// blocks and the neighbour vectors, accumulates in FP32 (or FP64), and writes
// out(site, i).  No cross-lane reduction, no atomics.
//
// Device block layout (all precisions): a 16-byte chunk holds K consecutive
// columns j of one row, K = 1 (FP64), 2 (FP32), 4 (BF16).  Chunks are ordered
//   [d = 0..8][j / K][site * Nb + i]
// so at a fixed (d, j/K) the lanes of a wave, which own consecutive rows,
// read consecutive 16-byte chunks: every block load is a fully coalesced
// dwordx4 stream.  Vectors are [Vc][Nb] complex; the neighbour vector chunk is
// the same address for all rows of a site (a broadcast served by the cache).
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

// decode chunk -> K complex values in R
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

// Map the hardware workgroup index to a logical one so that the 8 XCDs (which
// receive workgroups round-robin) each own a contiguous range of sites: their
// private L2 then holds the neighbour vectors of their own range.
__device__ inline long xcd_block(long b, long nb) {
  if (nb % 8 != 0) return b;
  return (b % 8) * (nb / 8) + b / 8;
}

template <int P, int NB>
__global__ void __launch_bounds__(256) k_coarse_apply(const Chunk16* __restrict__ blk,
                                                       const cplx<typename BlkTraits<P>::R>* __restrict__ in,
                                                       cplx<typename BlkTraits<P>::R>* __restrict__ out,
                                                       const int* __restrict__ nbr, long Vc, int nb_rt, int dmask,
                                                       int accumulate, const int* __restrict__ run) {
  typedef typename BlkTraits<P>::R R;
  constexpr int K = BlkTraits<P>::K;
  if (run && !*run) return;
  const int nb = NB > 0 ? NB : nb_rt;
  const long rows = Vc * nb;
  const long t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= rows) return;
  const long r = blockIdx.y;
  in += r * rows;
  out += r * rows;
  const long site = t / nb;
  const int nchunk = nb / K;
  cplx<R> acc = mkc((R)0, (R)0);
  cplx<R> acc2 = mkc((R)0, (R)0);
#pragma unroll
  for (int d = 0; d < 9; ++d) {
    if (!((dmask >> d) & 1)) continue;
    const long src = d == 0 ? site : (long)nbr[(long)(d - 1) * Vc + site];
    const cplx<R>* phi = in + src * nb;
    const Chunk16* bp = blk + (long)d * nchunk * rows + t;
#pragma unroll
    for (int jc = 0; jc < nchunk; ++jc) {
      Chunk16 c = bp[(long)jc * rows];
      cplx<R> m[K];
      decode<P>(c, m);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (k & 1) cfma(acc2, m[k], phi[jc * K + k]);
        else cfma(acc, m[k], phi[jc * K + k]);
      }
    }
  }
  acc = cadd(acc, acc2);
  if (accumulate) acc = cadd(acc, out[t]);
  out[t] = acc;
}

// canonical FP64 [Vc][9][Nb][Nb] -> device chunk layout of precision P
template <int P>
__global__ void k_blocks_to_device(const cd64* __restrict__ src, long Vc, int nb, Chunk16* __restrict__ dst) {
  typedef typename BlkTraits<P>::R R;
  constexpr int K = BlkTraits<P>::K;
  const long rows = Vc * nb;
  const int nchunk = nb / K;
  const long total = 9L * nchunk * rows;
  long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (q >= total) return;
  const long t = q % rows;
  const long dj = q / rows;
  const int jc = (int)(dj % nchunk), d = (int)(dj / nchunk);
  const long site = t / nb;
  const int i = (int)(t % nb);
  Chunk16 c;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    cd64 v = src[((site * 9 + d) * nb + i) * nb + jc * K + k];
    if constexpr (P == WCMG_F64) {
      uint64_t a = __builtin_bit_cast(uint64_t, v.re), b = __builtin_bit_cast(uint64_t, v.im);
      c.w[0] = (uint32_t)a;
      c.w[1] = (uint32_t)(a >> 32);
      c.w[2] = (uint32_t)b;
      c.w[3] = (uint32_t)(b >> 32);
    } else if constexpr (P == WCMG_F32) {
      c.w[2 * k] = __builtin_bit_cast(uint32_t, (float)v.re);
      c.w[2 * k + 1] = __builtin_bit_cast(uint32_t, (float)v.im);
    } else {
      uint32_t re = f32_to_bf16((float)v.re), im = f32_to_bf16((float)v.im);
      c.w[k] = re | (im << 16);
    }
  }
  dst[((long)d * nchunk + jc) * rows + t] = c;
}

// complex64 canonical -> complex128 canonical (for loading FP32 blocks)
__global__ void k_c64_to_c128(const cf32* __restrict__ in, cd64* __restrict__ out, long n) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) out[i] = mkc((double)in[i].re, (double)in[i].im);
}

size_t device_block_bytes(long Vc, int nb, int prec) {
  int K = prec == WCMG_F64 ? 1 : prec == WCMG_F32 ? 2 : 4;
  return 9UL * (nb / K) * Vc * nb * 16UL;
}

void launch_blocks_to_device(const cd64* src, long Vc, int nb, int prec, void* dst, hipStream_t st) {
  int K = prec == WCMG_F64 ? 1 : prec == WCMG_F32 ? 2 : 4;
  require(nb % K == 0, WCMG_ERR_ARG, "block size not a multiple of the storage chunk");
  long total = 9L * (nb / K) * Vc * nb;
  if (prec == WCMG_F64)
    hipLaunchKernelGGL(k_blocks_to_device<WCMG_F64>, dim3(nblocks(total)), dim3(kBlock), 0, st, src, Vc, nb,
                       (Chunk16*)dst);
  else if (prec == WCMG_F32)
    hipLaunchKernelGGL(k_blocks_to_device<WCMG_F32>, dim3(nblocks(total)), dim3(kBlock), 0, st, src, Vc, nb,
                       (Chunk16*)dst);
  else
    hipLaunchKernelGGL(k_blocks_to_device<WCMG_BF16>, dim3(nblocks(total)), dim3(kBlock), 0, st, src, Vc, nb,
                       (Chunk16*)dst);
  WCMG_CHECK_LAUNCH();
}

void launch_c64_to_c128(const cf32* in, cd64* out, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_c64_to_c128, dim3(nblocks(n)), dim3(kBlock), 0, st, in, out, n);
  WCMG_CHECK_LAUNCH();
}

template <int P, int NB>
static void launch_ca(const void* blk, const void* in, void* out, const int* nbr, long Vc, int nb, int dmask,
                      int accumulate, int nrhs, const int* run, hipStream_t st) {
  typedef typename BlkTraits<P>::R R;
  long rows = Vc * nb;
  hipLaunchKernelGGL((k_coarse_apply<P, NB>), dim3(nblocks(rows), nrhs), dim3(kBlock), 0, st, (const Chunk16*)blk,
                     (const cplx<R>*)in, (cplx<R>*)out, nbr, Vc, nb, dmask, accumulate, run);
}

template <int P>
static void dispatch_nb(const void* blk, const void* in, void* out, const int* nbr, long Vc, int nb, int dmask,
                        int accumulate, int nrhs, const int* run, hipStream_t st) {
  switch (nb) {
    case 8: launch_ca<P, 8>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st); break;
    case 12: launch_ca<P, 12>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st); break;
    case 16: launch_ca<P, 16>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st); break;
    case 24: launch_ca<P, 24>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st); break;
    case 32: launch_ca<P, 32>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st); break;
    case 40: launch_ca<P, 40>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st); break;
    default: launch_ca<P, 0>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st); break;
  }
}

void launch_coarse_apply(int prec, const void* blk, const void* in, void* out, const int* nbr, long Vc, int nb,
                         int dmask, int accumulate, int nrhs, const int* run, hipStream_t st) {
  if (prec == WCMG_F64) dispatch_nb<WCMG_F64>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st);
  else if (prec == WCMG_F32) dispatch_nb<WCMG_F32>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st);
  else dispatch_nb<WCMG_BF16>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st);
  WCMG_CHECK_LAUNCH();
}

}  // namespace wcmg
