// Batched coarse apply (up to 16 right-hand sides) on the matrix cores.
//
// For one coarse site and one direction d the product out += M_d phi is a
// complex [Nb x Nb] x [Nb x nrhs] GEMM.  Written in real arithmetic,
//   [out_re]   [ M_re  -M_im ] [phi_re]
//   [out_im] = [ M_im   M_re ] [phi_im],
// a [2Nb x 2Nb] x [2Nb x nrhs] real GEMM; the nine directions concatenate
// along K.  It runs on v_mfma_f32_16x16x4_f32 (A 16x4, B 4x16, D 16x16 per
// wave): output rows are grouped in 16-row tiles — for every full block of 16
// rows i a "real" tile and an "imaginary" tile, and for a remainder of 8 rows
// one mixed tile (8 real rows, then the same 8 imaginary rows).  The real and
// imaginary tiles of the same rows need the same block elements (the real tile
// uses (M_re, -M_im), the imaginary one (M_im, M_re)), so each element is
// loaded once and used twice from registers.  N = 16 columns hold the RHS.
//
// MFMA lane layouts (16x16x4 f32, wave64): A[i][k] in lane i + 16k, B[k][j] in
// lane j + 16k, D[i][j] in lane j + 16 (i / 4), register i % 4.  Lane l thus
// needs, for every k-step, block row (l % 16) of its tile and column
// 4 * step + l / 16: the Nb / 4 complex values M[row][l/16 + 4m], m < Nb / 4.
//
// Device block layout ("fragment order"): for each site and direction, first
// the full 16-row blocks (lane-major: [chunk][64 lanes]), then the 8-row
// remainder ([chunk][32 lane ids]); a chunk is 2 complex FP32 (16 B) or 2
// complex BF16 (8 B).  Every block element is stored exactly once and each
// load instruction of a wave reads contiguous memory.
//
// Vectors are right-hand-side major: field r at in + r * Vc * Nb, [Vc][Nb].
#include "coarse_common.h"

namespace wcmg {

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int P>
struct MfmaChunk;
template <>
struct MfmaChunk<WCMG_F32> {
  typedef float4 T;  // 2 complex FP32
  __device__ static void decode(const T& c, cf32& a, cf32& b) {
    a = mkc(c.x, c.y);
    b = mkc(c.z, c.w);
  }
};
template <>
struct MfmaChunk<WCMG_BF16> {
  typedef uint2 T;  // 2 complex BF16
  __device__ static void decode(const T& c, cf32& a, cf32& b) {
    a = mkc(__builtin_bit_cast(float, c.x << 16), __builtin_bit_cast(float, c.x & 0xffff0000u));
    b = mkc(__builtin_bit_cast(float, c.y << 16), __builtin_bit_cast(float, c.y & 0xffff0000u));
  }
};

// chunks per site and direction
__host__ __device__ constexpr long mfma_chunks_per_dir(int nb) {
  return (long)(nb / 8) * (64 * (nb / 16) + ((nb % 16) ? 32 : 0));
}

// Chunks of one direction's blocks held in registers: full 16-row blocks and
// the 8-row remainder (compile-time recursion keeps indices constant).
template <int P, int NCK>
struct BlockRegs {
  typename MfmaChunk<P>::T c[NCK];
};

template <int P, int NCK, int K>
__device__ __forceinline__ void mfma_load_chunks(BlockRegs<P, NCK>& r, const typename MfmaChunk<P>::T* __restrict__ base,
                                                 int stride, int idx) {
  if constexpr (K < NCK) {
    // the block stream is read once: non-temporal, so it does not evict the
    // neighbour vectors that nine sites share from L2
    if constexpr (sizeof(typename MfmaChunk<P>::T) == 16) {
      const u32x4 raw = __builtin_nontemporal_load((const u32x4*)(base + (long)K * stride + idx));
      r.c[K] = __builtin_bit_cast(typename MfmaChunk<P>::T, raw);
    } else {
      typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
      const u32x2 raw = __builtin_nontemporal_load((const u32x2*)(base + (long)K * stride + idx));
      r.c[K] = __builtin_bit_cast(typename MfmaChunk<P>::T, raw);
    }
    mfma_load_chunks<P, NCK, K + 1>(r, base, stride, idx);
  }
}

// One coarse site of one operator, all of its (up to 16) right-hand sides, by
// one wave.  Shared by the single-operator and the ragged launches.
template <int P, int NB>
__device__ __forceinline__ void mfma_site(const typename MfmaChunk<P>::T* __restrict__ blk,
                                          const cf32* __restrict__ in, cf32* __restrict__ out,
                                          const int* __restrict__ nbr, long Vc, int nrhs,
                                          const int* __restrict__ run, int run_stride, long site) {
  constexpr int Q = NB / 16;                 // full 16-row blocks
  constexpr bool REM = (NB % 16) != 0;       // one 8-row remainder
  constexpr int NCK = NB / 8;                // chunks per lane
  constexpr int NM = NB / 4;                 // complex values per lane (k-steps per half)
  constexpr long CPD = mfma_chunks_per_dir(NB);
  typedef typename MfmaChunk<P>::T CT;
  const int lane = threadIdx.x & 63;
  const int col = lane & 15;   // RHS column
  const int kq = lane >> 4;    // k offset within a step
  const bool rhs_ok = col < nrhs && (!run || run[(long)col * run_stride]);
  const long fs = Vc * NB;     // field stride between right-hand sides
  const cf32* inr = in + (long)(rhs_ok ? col : 0) * fs + kq;
  f32x4 acc[2 * Q + (REM ? 1 : 0)];
#pragma unroll
  for (int t = 0; t < 2 * Q + (REM ? 1 : 0); ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const CT* bsite = blk + site * 9 * CPD;
  const int rid = (lane & 7) + 8 * kq;  // remainder rows 16Q + (lane & 7), duplicated for lanes 8..15
  // operands of the current direction; the next direction's are loaded while
  // this one's matrix-core work runs
  BlockRegs<P, NCK> ca0, ca1, cr;
  static_assert(Q <= 2, "at most two full 16-row blocks");
  cf32 b[NM];
  long srcs[8];
#pragma unroll
  for (int d = 0; d < 8; ++d) srcs[d] = nbr[(long)d * Vc + site];
  if (Q > 0) mfma_load_chunks<P, NCK, 0>(ca0, bsite, 64, lane);
  if (Q > 1) mfma_load_chunks<P, NCK, 0>(ca1, bsite + NCK * 64, 64, lane);
  if (REM) mfma_load_chunks<P, NCK, 0>(cr, bsite + Q * NCK * 64, 32, rid);
#pragma unroll
  for (int m = 0; m < NM; ++m) b[m] = inr[site * NB + 4 * m];
#pragma unroll 1
  for (int d = 0; d < 9; ++d) {
    cf32 a[Q > 0 ? Q : 1][NM], ar[NM], bc[NM];
#pragma unroll
    for (int c = 0; c < NCK; ++c) {
      if (Q > 0) MfmaChunk<P>::decode(ca0.c[c], a[0][2 * c], a[0][2 * c + 1]);
      if (Q > 1) MfmaChunk<P>::decode(ca1.c[c], a[Q > 1 ? 1 : 0][2 * c], a[Q > 1 ? 1 : 0][2 * c + 1]);
      if (REM) MfmaChunk<P>::decode(cr.c[c], ar[2 * c], ar[2 * c + 1]);
    }
#pragma unroll
    for (int m = 0; m < NM; ++m) bc[m] = rhs_ok ? b[m] : mkc(0.f, 0.f);
    if (d < 8) {
      const CT* bn = bsite + (d + 1) * CPD;
      if (Q > 0) mfma_load_chunks<P, NCK, 0>(ca0, bn, 64, lane);
      if (Q > 1) mfma_load_chunks<P, NCK, 0>(ca1, bn + NCK * 64, 64, lane);
      if (REM) mfma_load_chunks<P, NCK, 0>(cr, bn + Q * NCK * 64, 32, rid);
      long src = srcs[0];
#pragma unroll
      for (int k = 1; k < 8; ++k) src = d == k ? srcs[k] : src;
#pragma unroll
      for (int m = 0; m < NM; ++m) b[m] = inr[src * NB + 4 * m];
    }
    const bool rem_im = (lane & 15) >= 8;
#pragma unroll
    for (int s = 0; s < 2 * NM; ++s) {
      const bool lo = s < NM;  // first half of K: phi_re rows; second half: phi_im rows
      const int m = lo ? s : s - NM;
      const float bf = lo ? bc[m].re : bc[m].im;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const float are = lo ? a[q][m].re : -a[q][m].im;  // real rows: (M_re, -M_im)
        const float aim = lo ? a[q][m].im : a[q][m].re;   // imaginary rows: (M_im, M_re)
        acc[2 * q] = __builtin_amdgcn_mfma_f32_16x16x4f32(are, bf, acc[2 * q], 0, 0, 0);
        acc[2 * q + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(aim, bf, acc[2 * q + 1], 0, 0, 0);
      }
      if (REM) {
        const float av = rem_im ? (lo ? ar[m].im : ar[m].re) : (lo ? ar[m].re : -ar[m].im);
        acc[2 * Q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bf, acc[2 * Q], 0, 0, 0);
      }
    }
  }
  // D[i][col] in lane col + 16 (i / 4), register i % 4
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * q + 4 * kq + v;
      if (rhs_ok) out[(long)col * fs + site * NB + i] = mkc(acc[2 * q][v], acc[2 * q + 1][v]);
    }
  if (REM) {
    // mixed tile: rows 0..7 real parts (lanes with kq < 2), rows 8..15 imaginary parts (kq >= 2)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float other = __shfl_xor(acc[2 * Q][v], 32, 64);
      const int i = 16 * Q + 4 * kq + v;
      if (kq < 2 && rhs_ok) out[(long)col * fs + site * NB + i] = mkc(acc[2 * Q][v], other);
    }
  }
}

template <int P, int NB>
__global__ void __launch_bounds__(256) k_coarse_apply_mfma(const typename MfmaChunk<P>::T* __restrict__ blk,
                                                            const cf32* __restrict__ in, cf32* __restrict__ out,
                                                            const int* __restrict__ nbr, long Vc, int nrhs,
                                                            const int* __restrict__ run, int run_stride) {
  const int wv = threadIdx.x >> 6;
  const long blk_id = (gridDim.x % 8 == 0) ? (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8 : blockIdx.x;
  const long site = blk_id * (blockDim.x >> 6) + wv;
  if (site >= Vc) return;  // wave-uniform
  mfma_site<P, NB>(blk, in, out, nbr, Vc, nrhs, run, run_stride, site);
}

// Ragged batch: several coarse operators (same Nb and storage), each with its
// own lattice, blocks, neighbour table and fields, in one launch over the sum
// of their sites; wave w of the grid takes global site w, and the table's
// prefix offsets name its operator.  The table travels as a kernel argument.
template <int P, int NB>
__global__ void __launch_bounds__(256) k_coarse_apply_mfma_ragged(RaggedTable t) {
  const int wv = threadIdx.x >> 6;
  const long blk_id = (gridDim.x % 8 == 0) ? (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8 : blockIdx.x;
  const long g = blk_id * (blockDim.x >> 6) + wv;
  if (g >= t.site0[t.n]) return;  // wave-uniform
  int p = 0;
  while (p + 1 < t.n && g >= t.site0[p + 1]) ++p;
  const RaggedProblem& q = t.p[p];
  mfma_site<P, NB>((const typename MfmaChunk<P>::T*)q.blk, q.in, q.out, q.nbr, q.Vc, q.nrhs, q.run, q.rs,
                   g - t.site0[p]);
}

// canonical FP64 [Vc][9][Nb][Nb] -> fragment order of precision P
template <int P>
__global__ void k_blocks_to_mfma(const cd64* __restrict__ src, long Vc, int nb, typename MfmaChunk<P>::T* dst) {
  const int Q = nb / 16, NCK = nb / 8;
  const long cpd = mfma_chunks_per_dir(nb);
  const long total = Vc * 9 * cpd;
  const long g = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (g >= total) return;
  const long site = g / (9 * cpd);
  const int d = (int)((g / cpd) % 9);
  long r = g % cpd;
  int row, kq, c;
  if (r < (long)Q * NCK * 64) {
    const int q = (int)(r / (NCK * 64));
    r %= NCK * 64;
    c = (int)(r / 64);
    const int lane = (int)(r % 64);
    row = 16 * q + (lane & 15);
    kq = lane >> 4;
  } else {
    r -= (long)Q * NCK * 64;
    c = (int)(r / 32);
    const int id = (int)(r % 32);
    row = 16 * Q + (id & 7);
    kq = id >> 3;
  }
  const cd64* m = src + ((site * 9 + d) * nb + row) * nb;
  const cd64 e0 = m[kq + 4 * (2 * c)], e1 = m[kq + 4 * (2 * c + 1)];
  typename MfmaChunk<P>::T out;
  if constexpr (P == WCMG_F32) {
    out = make_float4((float)e0.re, (float)e0.im, (float)e1.re, (float)e1.im);
  } else {
    const uint32_t a = (uint32_t)f32_to_bf16((float)e0.re) | ((uint32_t)f32_to_bf16((float)e0.im) << 16);
    const uint32_t b = (uint32_t)f32_to_bf16((float)e1.re) | ((uint32_t)f32_to_bf16((float)e1.im) << 16);
    out = make_uint2(a, b);
  }
  dst[g] = out;
}

bool mfma_supported_nb(int nb) { return nb == 8 || nb == 16 || nb == 24 || nb == 32 || nb == 40; }

size_t mfma_block_bytes(long Vc, int nb, int prec) {
  return (size_t)Vc * 9 * mfma_chunks_per_dir(nb) * (prec == WCMG_F32 ? 16 : 8);
}

void launch_blocks_to_mfma(const cd64* src, long Vc, int nb, int prec, void* dst, hipStream_t st) {
  require(mfma_supported_nb(nb) && (prec == WCMG_F32 || prec == WCMG_BF16), WCMG_ERR_ARG,
          "matrix-core layout needs Nb in {8,16,24,32,40} and FP32 or BF16 storage");
  const long total = Vc * 9 * mfma_chunks_per_dir(nb);
  if (prec == WCMG_F32)
    hipLaunchKernelGGL(k_blocks_to_mfma<WCMG_F32>, dim3(nblocks(total)), dim3(kBlock), 0, st, src, Vc, nb,
                       (float4*)dst);
  else
    hipLaunchKernelGGL(k_blocks_to_mfma<WCMG_BF16>, dim3(nblocks(total)), dim3(kBlock), 0, st, src, Vc, nb,
                       (uint2*)dst);
  WCMG_CHECK_LAUNCH();
}

template <int P, int NB>
static void mfma_t(const void* blk, const cf32* in, cf32* out, const int* nbr, long Vc, int nrhs, const int* run,
                   int run_stride, hipStream_t st) {
  WCMG_LAUNCH((k_coarse_apply_mfma<P, NB>), dim3((unsigned)((Vc + 3) / 4)), dim3(kBlock), 0, st,
              (const typename MfmaChunk<P>::T*)blk, in, out, nbr, Vc, nrhs, run, run_stride);
}
template <int P>
static void mfma_nb(int nb, const void* blk, const cf32* in, cf32* out, const int* nbr, long Vc, int nrhs,
                    const int* run, int run_stride, hipStream_t st) {
  switch (nb) {
    case 8: mfma_t<P, 8>(blk, in, out, nbr, Vc, nrhs, run, run_stride, st); break;
    case 16: mfma_t<P, 16>(blk, in, out, nbr, Vc, nrhs, run, run_stride, st); break;
    case 24: mfma_t<P, 24>(blk, in, out, nbr, Vc, nrhs, run, run_stride, st); break;
    case 32: mfma_t<P, 32>(blk, in, out, nbr, Vc, nrhs, run, run_stride, st); break;
    case 40: mfma_t<P, 40>(blk, in, out, nbr, Vc, nrhs, run, run_stride, st); break;
    default: throw Error(WCMG_ERR_ARG, "matrix-core coarse apply: unsupported Nb");
  }
}

// out = D_c in for nrhs <= 16 right-hand sides (RHS-major fields, FP32).
template <int P>
static void mfma_ragged_nb(const RaggedTable& t, long total, hipStream_t st) {
  const dim3 g((unsigned)((total + 3) / 4)), b(kBlock);
  switch (t.nb) {
    case 8: WCMG_LAUNCH((k_coarse_apply_mfma_ragged<P, 8>), g, b, 0, st, t); break;
    case 16: WCMG_LAUNCH((k_coarse_apply_mfma_ragged<P, 16>), g, b, 0, st, t); break;
    case 24: WCMG_LAUNCH((k_coarse_apply_mfma_ragged<P, 24>), g, b, 0, st, t); break;
    case 32: WCMG_LAUNCH((k_coarse_apply_mfma_ragged<P, 32>), g, b, 0, st, t); break;
    default: WCMG_LAUNCH((k_coarse_apply_mfma_ragged<P, 40>), g, b, 0, st, t); break;
  }
}

void launch_coarse_apply_mfma_ragged(int prec, RaggedTable t, hipStream_t st) {
  require(t.n >= 1 && t.n <= kRaggedMax, WCMG_ERR_ARG, "ragged batch takes 1..8 operators");
  require(mfma_supported_nb(t.nb) && (prec == WCMG_F32 || prec == WCMG_BF16), WCMG_ERR_ARG,
          "ragged batch: matrix-core layout (Nb in {8,16,24,32,40}, FP32 or BF16 storage)");
  t.site0[0] = 0;
  for (int p = 0; p < t.n; ++p) {
    require(t.p[p].nrhs >= 1 && t.p[p].nrhs <= 16, WCMG_ERR_ARG, "ragged batch: 1..16 right-hand sides per operator");
    t.site0[p + 1] = t.site0[p] + t.p[p].Vc;
  }
  if (prec == WCMG_F32) mfma_ragged_nb<WCMG_F32>(t, t.site0[t.n], st);
  else mfma_ragged_nb<WCMG_BF16>(t, t.site0[t.n], st);
  WCMG_CHECK_LAUNCH();
}

void launch_coarse_apply_mfma(int prec, int nb, const void* blk, const cf32* in, cf32* out, const int* nbr, long Vc,
                              int nrhs, const int* run, int run_stride, hipStream_t st) {
  require(nrhs >= 1 && nrhs <= 16, WCMG_ERR_ARG, "matrix-core coarse apply takes 1..16 right-hand sides");
  if (prec == WCMG_F32) mfma_nb<WCMG_F32>(nb, blk, in, out, nbr, Vc, nrhs, run, run_stride, st);
  else mfma_nb<WCMG_BF16>(nb, blk, in, out, nbr, Vc, nrhs, run, run_stride, st);
  WCMG_CHECK_LAUNCH();
}

}  // namespace wcmg
