// Coarse operator from five-point storage: Mdiag and the four forward blocks
// per coarse site, the backward hops taken as sigma3-conjugated adjoints of
// the neighbours' forward blocks (layout: coarse5.h).  Two forms:
// * large lattices (one lane per row): the owner of each forward block also
//   forms its backward contribution and scatters it to a buffer of four
//   fields, added by a second launch, so that five blocks per site are read
//   from memory instead of nine;
// * small, cache-resident lattices (several lanes per row): the consumer
//   reads the neighbour's forward block columns through LDS (coarse_row5),
//   in one launch.
#include "coarse5.h"

namespace wcmg {

template <int P, int NB, int S>
__global__ void __launch_bounds__(256) k_coarse_apply5(const Chunk16* __restrict__ blk,
                                                        const cplx<typename BlkTraits<P>::R>* __restrict__ in,
                                                        cplx<typename BlkTraits<P>::R>* __restrict__ out,
                                                        const int* __restrict__ nbr, long Vc, int accumulate,
                                                        const int* __restrict__ run, int rs) {
  typedef typename BlkTraits<P>::R R;
  if (run && !run[(long)blockIdx.y * rs]) return;
  const long rows = Vc * NB;
  const long xb = xcd_block(blockIdx.x, gridDim.x);
  const long g = xb * blockDim.x + threadIdx.x;
  const long t = g / S;
  const int sub = (int)(g % S);
  const bool valid = t < rows;
  const long r = blockIdx.y;
  cplx<R> acc = coarse_row5<P, NB, S>(blk, in + r * rows, nbr, Vc, xb * (blockDim.x / S), t, sub, valid);
  if (!valid || sub != 0) return;
  out += r * rows;
  if (accumulate) acc = cadd(acc, out[t]);
  out[t] = acc;
}

// One lane per output row, the owner computing the backward hops: the
// workgroup's G sites stream Mdiag and their four forward blocks once (lane i
// reads row i), and each forward block Mdir_{+mu}(c), kept in LDS, also gives
// the backward contribution of c to its +mu neighbour,
//   tmp[mu][c + mu] = s Mdir_{+mu}(c)^dag s in(c)
// (lane i acting as column i).  k_coarse5_combine then adds the four tmp
// fields to out in the order mu = 0..3.  Every block is read from memory once.
template <int P, int NB>
struct Owner5 {
  static constexpr int K = BlkTraits<P>::K;
  static constexpr int NCH = NB / K;
  static constexpr int bytes_per_site = NB * (NCH + 1) * 16 + NB * (int)sizeof(cplx<typename BlkTraits<P>::R>);
  static constexpr int G0 = 256 / NB;
  static constexpr int G1 = 49152 / bytes_per_site;
  static constexpr int G = G0 < G1 ? G0 : (G1 > 0 ? G1 : 1);  // sites per workgroup
};

template <int P, int NB>
__global__ void __launch_bounds__(256) k_coarse_apply5_owner(const Chunk16* __restrict__ blk,
                                                              const cplx<typename BlkTraits<P>::R>* __restrict__ in,
                                                              cplx<typename BlkTraits<P>::R>* __restrict__ out,
                                                              cplx<typename BlkTraits<P>::R>* __restrict__ tmp,
                                                              const int* __restrict__ nbr, long Vc, int nrhs,
                                                              int accumulate, const int* __restrict__ run, int rs) {
  typedef typename BlkTraits<P>::R R;
  typedef Owner5<P, NB> O;
  constexpr int K = O::K, NCH = O::NCH, G = O::G;
  __shared__ Chunk16 tile[G][NB][NCH + 1];
  __shared__ cplx<R> phs[G][NB];
  const long r = blockIdx.y;
  if (run && !run[r * rs]) return;
  const long rows = Vc * NB;
  const long xb = xcd_block(blockIdx.x, gridDim.x);
  const int g = threadIdx.x / NB, i = threadIdx.x - g * NB;
  const long c = xb * G + g;
  const bool valid = g < G && c < Vc;
  const long t = c * NB + i;
  in += r * rows;
  out += r * rows;
  const R si = i < NB / 2 ? (R)1 : (R)-1;
  if (valid) {
    const cplx<R> v = in[t];
    phs[g][i] = mkc(si * v.re, si * v.im);
  }
  cplx<R> acc = mkc((R)0, (R)0), acc2 = mkc((R)0, (R)0);
  if (valid) {
#pragma unroll
    for (int jc = 0; jc < NCH; ++jc) {
      cplx<R> m[K];
      decode<P>(blk[(long)jc * rows + t], m);
      const cplx<R>* phi = in + c * NB + jc * K;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (k & 1) cfma(acc2, m[k], phi[k]);
        else cfma(acc, m[k], phi[k]);
      }
    }
  }
  for (int mu = 0; mu < 4; ++mu) {
    const long cp = valid ? (long)nbr[(long)(2 * mu) * Vc + c] : 0;  // c + mu
    if (valid) {
#pragma unroll
      for (int jc = 0; jc < NCH; ++jc) {
        const Chunk16 ch = blk[(long)((1 + mu) * NCH + jc) * rows + t];
        tile[g][i][jc] = ch;
        cplx<R> m[K];
        decode<P>(ch, m);
        const cplx<R>* phi = in + cp * NB + jc * K;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          if (k & 1) cfma(acc2, m[k], phi[k]);
          else cfma(acc, m[k], phi[k]);
        }
      }
    }
    __syncthreads();
    if (valid) {
      // column i of the block: y_i = s_i sum_a conj(M[a][i]) s_a in_a(c)
      const int qi = i / K, ki = i - qi * K;
      cplx<R> y = mkc((R)0, (R)0), y2 = mkc((R)0, (R)0);
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        if (a & 1) cfmac(y2, chunk_elem<P>(&tile[g][a][qi], ki), phs[g][a]);
        else cfmac(y, chunk_elem<P>(&tile[g][a][qi], ki), phs[g][a]);
      }
      y = cadd(y, y2);
      tmp[((long)mu * nrhs + r) * rows + cp * NB + i] = mkc(si * y.re, si * y.im);
    }
    __syncthreads();
  }
  if (!valid) return;
  acc = cadd(acc, acc2);
  if (accumulate) acc = cadd(acc, out[t]);
  out[t] = acc;
}

template <typename R>
__global__ void k_coarse5_combine(cplx<R>* __restrict__ out, const cplx<R>* __restrict__ tmp, long n,
                                  const int* __restrict__ run, int rs, long rows) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= n) return;
  if (run && !run[(e / rows) * rs]) return;
  cplx<R> v = out[e];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) v = cadd(v, tmp[mu * n + e]);
  out[e] = v;
}

// canonical FP64 [Vc][9][Nb][Nb] -> five-point chunk layout of precision P
template <int P>
__global__ void k_blocks_to_device5(const cd64* __restrict__ src, long Vc, int nb, Chunk16* __restrict__ dst) {
  constexpr int K = BlkTraits<P>::K;
  const long rows = Vc * nb;
  const int nchunk = nb / K;
  const long total = 5L * nchunk * rows;
  const long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (q >= total) return;
  const long t = q % rows;
  const long dj = q / rows;
  const int jc = (int)(dj % nchunk), d5 = (int)(dj / nchunk);
  const int d = d5 == 0 ? 0 : 2 * d5 - 1;
  const long site = t / nb;
  const int i = (int)(t % nb);
  Chunk16 c;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const cd64 v = src[((site * 9 + d) * nb + i) * nb + jc * K + k];
    if constexpr (P == WCMG_F64) {
      const uint64_t a = __builtin_bit_cast(uint64_t, v.re), b = __builtin_bit_cast(uint64_t, v.im);
      c.w[0] = (uint32_t)a;
      c.w[1] = (uint32_t)(a >> 32);
      c.w[2] = (uint32_t)b;
      c.w[3] = (uint32_t)(b >> 32);
    } else if constexpr (P == WCMG_F32) {
      c.w[2 * k] = __builtin_bit_cast(uint32_t, (float)v.re);
      c.w[2 * k + 1] = __builtin_bit_cast(uint32_t, (float)v.im);
    } else {
      const uint32_t re = f32_to_bf16((float)v.re), im = f32_to_bf16((float)v.im);
      c.w[k] = re | (im << 16);
    }
  }
  dst[((long)d5 * nchunk + jc) * rows + t] = c;
}

size_t device_block5_bytes(long Vc, int nb, int prec) {
  const int K = prec == WCMG_F64 ? 1 : prec == WCMG_F32 ? 2 : 4;
  return 5UL * (nb / K) * Vc * nb * 16UL;
}

void launch_blocks_to_device5(const cd64* src, long Vc, int nb, int prec, void* dst, hipStream_t st) {
  const int K = prec == WCMG_F64 ? 1 : prec == WCMG_F32 ? 2 : 4;
  require(nb % K == 0, WCMG_ERR_ARG, "block size not a multiple of the storage chunk");
  const long total = 5L * (nb / K) * Vc * nb;
  if (prec == WCMG_F64)
    hipLaunchKernelGGL(k_blocks_to_device5<WCMG_F64>, dim3(nblocks(total)), dim3(kBlock), 0, st, src, Vc, nb,
                       (Chunk16*)dst);
  else if (prec == WCMG_F32)
    hipLaunchKernelGGL(k_blocks_to_device5<WCMG_F32>, dim3(nblocks(total)), dim3(kBlock), 0, st, src, Vc, nb,
                       (Chunk16*)dst);
  else
    hipLaunchKernelGGL(k_blocks_to_device5<WCMG_BF16>, dim3(nblocks(total)), dim3(kBlock), 0, st, src, Vc, nb,
                       (Chunk16*)dst);
  WCMG_CHECK_LAUNCH();
}

template <int P, int NB, int S>
static void launch_ca5(const void* blk, const void* in, void* out, const int* nbr, long Vc, int accumulate, int nrhs,
                       const int* run, hipStream_t st, int rs) {
  typedef typename BlkTraits<P>::R R;
  const long rows = Vc * NB;
  WCMG_LAUNCH((k_coarse_apply5<P, NB, S>), dim3(nblocks(rows * S), nrhs), dim3(kBlock), 0, st, (const Chunk16*)blk,
              (const cplx<R>*)in, (cplx<R>*)out, nbr, Vc, accumulate, run, rs);
}

template <int P, int NB>
static void dispatch5_s(const void* blk, const void* in, void* out, void* tmp, const int* nbr, long Vc,
                        int accumulate, int nrhs, const int* run, hipStream_t st, int rs) {
  typedef typename BlkTraits<P>::R R;
  switch (coarse_split(Vc * NB * nrhs)) {
    case 1:
      if (tmp) {
        constexpr int G = Owner5<P, NB>::G;
        const long n = Vc * NB * nrhs;
        WCMG_LAUNCH((k_coarse_apply5_owner<P, NB>), dim3((unsigned)((Vc + G - 1) / G), nrhs), dim3(G * NB), 0, st,
                    (const Chunk16*)blk, (const cplx<R>*)in, (cplx<R>*)out, (cplx<R>*)tmp, nbr, Vc, nrhs, accumulate,
                    run, rs);
        hipLaunchKernelGGL(k_coarse5_combine<R>, dim3(nblocks(n)), dim3(kBlock), 0, st, (cplx<R>*)out,
                           (const cplx<R>*)tmp, n, run, rs, Vc * NB);
      } else {
        launch_ca5<P, NB, 1>(blk, in, out, nbr, Vc, accumulate, nrhs, run, st, rs);
      }
      break;
    case 2: launch_ca5<P, NB, 2>(blk, in, out, nbr, Vc, accumulate, nrhs, run, st, rs); break;
    case 4: launch_ca5<P, NB, 4>(blk, in, out, nbr, Vc, accumulate, nrhs, run, st, rs); break;
    default: launch_ca5<P, NB, 8>(blk, in, out, nbr, Vc, accumulate, nrhs, run, st, rs); break;
  }
}

template <int P>
static void dispatch5_nb(const void* blk, const void* in, void* out, void* tmp, const int* nbr, long Vc, int nb,
                         int accumulate, int nrhs, const int* run, hipStream_t st, int rs) {
  switch (nb) {
    case 8: dispatch5_s<P, 8>(blk, in, out, tmp, nbr, Vc, accumulate, nrhs, run, st, rs); break;
    case 12: dispatch5_s<P, 12>(blk, in, out, tmp, nbr, Vc, accumulate, nrhs, run, st, rs); break;
    case 16: dispatch5_s<P, 16>(blk, in, out, tmp, nbr, Vc, accumulate, nrhs, run, st, rs); break;
    case 24: dispatch5_s<P, 24>(blk, in, out, tmp, nbr, Vc, accumulate, nrhs, run, st, rs); break;
    case 32: dispatch5_s<P, 32>(blk, in, out, tmp, nbr, Vc, accumulate, nrhs, run, st, rs); break;
    default: throw Error(WCMG_ERR_ARG, "five-point coarse storage: unsupported Nb = " + std::to_string(nb));
  }
}

bool five_point_supported(int nb) { return nb == 8 || nb == 12 || nb == 16 || nb == 24 || nb == 32; }

bool coarse5_uses_owner(long Vc, int nb, int nrhs) { return coarse_split(Vc * nb * nrhs) == 1; }

void launch_coarse_apply5(int prec, const void* blk, const void* in, void* out, void* tmp, const int* nbr, long Vc,
                          int nb, int accumulate, int nrhs, const int* run, hipStream_t st, int rs) {
  if (prec == WCMG_F64) dispatch5_nb<WCMG_F64>(blk, in, out, tmp, nbr, Vc, nb, accumulate, nrhs, run, st, rs);
  else if (prec == WCMG_F32) dispatch5_nb<WCMG_F32>(blk, in, out, tmp, nbr, Vc, nb, accumulate, nrhs, run, st, rs);
  else dispatch5_nb<WCMG_BF16>(blk, in, out, tmp, nbr, Vc, nb, accumulate, nrhs, run, st, rs);
  WCMG_CHECK_LAUNCH();
}

}  // namespace wcmg
