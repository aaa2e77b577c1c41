// Coarse operator: application of Mdiag plus the eight Mdir blocks
// (Sec. 2.1: the coarse matrix is applied through its diagonal part and its
// hops in single directions; nine dense Nb x Nb complex blocks per site).
//
// S adjacent lanes own one output row (site, i): they split the row's chunks
// of the nine blocks, accumulate in FP32 (or FP64) and combine with S-1
// shuffles.  S = 1 on large lattices (one dwordx4 stream per lane); S > 1 on
// small, cache-resident coarse lattices so that enough waves are in flight.
// No atomics.  Block layout and chunk decoding: coarse_common.h.
#include "coarse_common.h"

namespace wcmg {

template <int P, int NB, int S>
__global__ void __launch_bounds__(256) k_coarse_apply(const Chunk16* __restrict__ blk,
                                                       const cplx<typename BlkTraits<P>::R>* __restrict__ in,
                                                       cplx<typename BlkTraits<P>::R>* __restrict__ out,
                                                       const int* __restrict__ nbr, long Vc, int nb_rt, int dmask,
                                                       int accumulate, const int* __restrict__ run, int rs) {
  typedef typename BlkTraits<P>::R R;
  if (run && !run[(long)blockIdx.y * rs]) return;
  const int nb = NB > 0 ? NB : nb_rt;
  const long rows = Vc * nb;
  const long g = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const long t = g / S;
  const int sub = (int)(g % S);
  const bool valid = t < rows;
  const long r = blockIdx.y;
  cplx<R> acc = coarse_row<P, NB, S>(blk, in + r * rows, nbr, Vc, nb, t, sub, dmask, valid);
  if (!valid || sub != 0) return;
  out += r * rows;
  if (accumulate) acc = cadd(acc, out[t]);
  out[t] = acc;
}

// canonical FP64 [Vc][9][Nb][Nb] -> device chunk layout of precision P
template <int P>
__global__ void k_blocks_to_device(const cd64* __restrict__ src, long Vc, int nb, Chunk16* __restrict__ dst) {
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

// complex128 -> complex64, optionally rounded on to BF16 (nearest even) and
// widened back: the values that BF16 block storage holds
__global__ void k_c128_to_c64(const cd64* __restrict__ in, cf32* __restrict__ out, long n, int bf16) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= n) return;
  float re = (float)in[e].re, im = (float)in[e].im;
  if (bf16) {
    re = bf16_to_f32(f32_to_bf16(re));
    im = bf16_to_f32(f32_to_bf16(im));
  }
  out[e] = mkc(re, im);
}

void launch_c128_to_c64(const cd64* in, cf32* out, long n, int bf16, hipStream_t st) {
  hipLaunchKernelGGL(k_c128_to_c64, dim3(nblocks(n)), dim3(kBlock), 0, st, in, out, n, bf16);
  WCMG_CHECK_LAUNCH();
}

void launch_c64_to_c128(const cf32* in, cd64* out, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_c64_to_c128, dim3(nblocks(n)), dim3(kBlock), 0, st, in, out, n);
  WCMG_CHECK_LAUNCH();
}

template <int P, int NB, int S>
static void launch_ca(const void* blk, const void* in, void* out, const int* nbr, long Vc, int nb, int dmask,
                      int accumulate, int nrhs, const int* run, hipStream_t st, int rs) {
  typedef typename BlkTraits<P>::R R;
  long rows = Vc * nb;
  WCMG_LAUNCH((k_coarse_apply<P, NB, S>), dim3(nblocks(rows * S), nrhs), dim3(kBlock), 0, st, (const Chunk16*)blk,
              (const cplx<R>*)in, (cplx<R>*)out, nbr, Vc, nb, dmask, accumulate, run, rs);
}

template <int P, int NB>
static void dispatch_s(const void* blk, const void* in, void* out, const int* nbr, long Vc, int nb, int dmask,
                       int accumulate, int nrhs, const int* run, hipStream_t st, int rs) {
  switch (coarse_split(Vc * nb * nrhs)) {
    case 1: launch_ca<P, NB, 1>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st, rs); break;
    case 2: launch_ca<P, NB, 2>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st, rs); break;
    case 4: launch_ca<P, NB, 4>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st, rs); break;
    default: launch_ca<P, NB, 8>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st, rs); break;
  }
}

template <int P>
static void dispatch_nb(const void* blk, const void* in, void* out, const int* nbr, long Vc, int nb, int dmask,
                        int accumulate, int nrhs, const int* run, hipStream_t st, int rs) {
  switch (nb) {
    case 8: dispatch_s<P, 8>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st, rs); break;
    case 12: dispatch_s<P, 12>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st, rs); break;
    case 16: dispatch_s<P, 16>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st, rs); break;
    case 24: dispatch_s<P, 24>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st, rs); break;
    case 32: dispatch_s<P, 32>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st, rs); break;
    case 40: dispatch_s<P, 40>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st, rs); break;
    default: dispatch_s<P, 0>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st, rs); break;
  }
}

void launch_coarse_apply(int prec, const void* blk, const void* in, void* out, const int* nbr, long Vc, int nb,
                         int dmask, int accumulate, int nrhs, const int* run, hipStream_t st, int rs) {
  if (prec == WCMG_F64) dispatch_nb<WCMG_F64>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st, rs);
  else if (prec == WCMG_F32) dispatch_nb<WCMG_F32>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st, rs);
  else dispatch_nb<WCMG_BF16>(blk, in, out, nbr, Vc, nb, dmask, accumulate, nrhs, run, st, rs);
  WCMG_CHECK_LAUNCH();
}

}  // namespace wcmg
