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
#include <atomic>

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

// Tile counts of one site: Q full 16-row blocks, an 8-row remainder, NM
// complex values per lane and direction (k-steps per half of K).
template <int NB>
struct MfmaShape {
  static constexpr int Q = NB / 16;
  static constexpr bool REM = (NB % 16) != 0;
  static constexpr int NCK = NB / 8;
  static constexpr int NM = NB / 4;
  static constexpr int NT = 2 * Q + (REM ? 1 : 0);  // accumulator tiles
  static_assert(Q <= 2, "at most two full 16-row blocks");
};

// The matrix-core work of one direction: acc += [M_re -M_im; M_im M_re] phi
// with the block fragments a (full tiles) and ar (remainder) and the right-hand
// side values bc of this lane (column lane % 16, rows lane / 16 + 4 m).
template <int NB>
__device__ __forceinline__ void mfma_direction(f32x4 (&acc)[MfmaShape<NB>::NT],
                                               const cf32 (&a)[MfmaShape<NB>::Q > 0 ? MfmaShape<NB>::Q : 1]
                                                              [MfmaShape<NB>::NM],
                                               const cf32 (&ar)[MfmaShape<NB>::NM], const cf32 (&bc)[MfmaShape<NB>::NM],
                                               int lane) {
  constexpr int Q = MfmaShape<NB>::Q, NM = MfmaShape<NB>::NM;
  constexpr bool REM = MfmaShape<NB>::REM;
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

// Decode one direction's chunks into complex fragments.
template <int P, int NB>
__device__ __forceinline__ void mfma_decode(const BlockRegs<P, MfmaShape<NB>::NCK>& ca0,
                                            const BlockRegs<P, MfmaShape<NB>::NCK>& ca1,
                                            const BlockRegs<P, MfmaShape<NB>::NCK>& cr,
                                            cf32 (&a)[MfmaShape<NB>::Q > 0 ? MfmaShape<NB>::Q : 1][MfmaShape<NB>::NM],
                                            cf32 (&ar)[MfmaShape<NB>::NM]) {
  constexpr int Q = MfmaShape<NB>::Q, NCK = MfmaShape<NB>::NCK;
  constexpr bool REM = MfmaShape<NB>::REM;
#pragma unroll
  for (int c = 0; c < NCK; ++c) {
    if (Q > 0) MfmaChunk<P>::decode(ca0.c[c], a[0][2 * c], a[0][2 * c + 1]);
    if (Q > 1) MfmaChunk<P>::decode(ca1.c[c], a[Q > 1 ? 1 : 0][2 * c], a[Q > 1 ? 1 : 0][2 * c + 1]);
    if (REM) MfmaChunk<P>::decode(cr.c[c], ar[2 * c], ar[2 * c + 1]);
  }
}

// Issue the loads of one direction's chunks (base: that direction's stream).
template <int P, int NB>
__device__ __forceinline__ void mfma_issue(BlockRegs<P, MfmaShape<NB>::NCK>& ca0, BlockRegs<P, MfmaShape<NB>::NCK>& ca1,
                                           BlockRegs<P, MfmaShape<NB>::NCK>& cr,
                                           const typename MfmaChunk<P>::T* __restrict__ base, int lane, int rid) {
  constexpr int Q = MfmaShape<NB>::Q, NCK = MfmaShape<NB>::NCK;
  constexpr bool REM = MfmaShape<NB>::REM;
  if (Q > 0) mfma_load_chunks<P, NCK, 0>(ca0, base, 64, lane);
  if (Q > 1) mfma_load_chunks<P, NCK, 0>(ca1, base + NCK * 64, 64, lane);
  if (REM) mfma_load_chunks<P, NCK, 0>(cr, base + Q * NCK * 64, 32, rid);
}

// D[i][col] in lane col + 16 (i / 4), register i % 4
template <int NB>
__device__ __forceinline__ void mfma_store(const f32x4 (&acc)[MfmaShape<NB>::NT], cf32* __restrict__ out, long fs,
                                           long site, int lane, bool rhs_ok) {
  constexpr int Q = MfmaShape<NB>::Q;
  constexpr bool REM = MfmaShape<NB>::REM;
  const int col = lane & 15, kq = lane >> 4;
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

// One coarse site of one operator, all of its (up to 16) right-hand sides, by
// one wave, neighbour vectors read straight from memory.  Shared by the
// single-operator and the ragged launches.
template <int P, int NB>
__device__ __forceinline__ void mfma_site(const typename MfmaChunk<P>::T* __restrict__ blk,
                                          const cf32* __restrict__ in, cf32* __restrict__ out,
                                          const int* __restrict__ nbr, long Vc, int nrhs,
                                          const int* __restrict__ run, int run_stride, long site) {
  typedef MfmaShape<NB> S;
  constexpr int NM = S::NM;
  constexpr long CPD = mfma_chunks_per_dir(NB);
  typedef typename MfmaChunk<P>::T CT;
  const int lane = threadIdx.x & 63;
  const int col = lane & 15;   // RHS column
  const int kq = lane >> 4;    // k offset within a step
  const bool rhs_ok = col < nrhs && (!run || run[(long)col * run_stride]);
  const long fs = Vc * NB;     // field stride between right-hand sides
  // columns without a live right-hand side compute on column 0's values and
  // are never stored (the columns of the product are independent)
  const cf32* inr = in + (long)(rhs_ok ? col : 0) * fs + kq;
  f32x4 acc[S::NT];
#pragma unroll
  for (int t = 0; t < S::NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const CT* bsite = blk + site * 9 * CPD;
  const int rid = (lane & 7) + 8 * kq;  // remainder rows 16Q + (lane & 7), duplicated for lanes 8..15
  // operands of the current direction; the next direction's are loaded while
  // this one's matrix-core work runs
  BlockRegs<P, S::NCK> ca0, ca1, cr;
  cf32 b[NM];
  long srcs[8];
#pragma unroll
  for (int d = 0; d < 8; ++d) srcs[d] = nbr[(long)d * Vc + site];
  mfma_issue<P, NB>(ca0, ca1, cr, bsite, lane, rid);
#pragma unroll
  for (int m = 0; m < NM; ++m) b[m] = inr[site * NB + 4 * m];
#pragma unroll 1
  for (int d = 0; d < 9; ++d) {
    cf32 a[S::Q > 0 ? S::Q : 1][NM], ar[NM], bc[NM];
    mfma_decode<P, NB>(ca0, ca1, cr, a, ar);
#pragma unroll
    for (int m = 0; m < NM; ++m) bc[m] = b[m];
    if (d < 8) {
      mfma_issue<P, NB>(ca0, ca1, cr, bsite + (d + 1) * CPD, lane, rid);
      long src = srcs[0];
#pragma unroll
      for (int k = 1; k < 8; ++k) src = d == k ? srcs[k] : src;
#pragma unroll
      for (int m = 0; m < NM; ++m) b[m] = inr[src * NB + 4 * m];
    }
    mfma_direction<NB>(acc, a, ar, bc, lane);
  }
  mfma_store<NB>(acc, out, fs, site, lane, rhs_ok);
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

// ---- neighbour vectors staged in LDS
//
// A workgroup of S waves takes S consecutive sites of one x-row of a
// lexicographic coarse lattice (x fastest, S divides Lx).  The vectors its nine
// directions read are then whole row segments: the segment itself, extended by
// one site on each side, serves Mdiag, +x and -x, and each of the six other
// directions reads the same x-range of a neighbouring row.  The workgroup
// copies each segment once into LDS for all right-hand sides (direct-to-LDS
// loads, which hold no registers) while the previous segment is in use.  A
// site's neighbour vector then arrives from L2 as part of a contiguous row
// instead of as one 192-byte piece per right-hand side for each of its nine
// readers; the block stream is read per wave as in the direct kernel.

template <int NB, int S>
struct StageShape {
  static constexpr int U = NB / 2;     // 16-byte units per site vector
  static constexpr int SLOTS = S + 2;  // sites of the largest segment
  // 16-byte units per right-hand side row, padded to 32 bytes past a multiple
  // of 256 so that the 16 columns of a B-fragment read spread over the banks
  static constexpr int RSU = ((SLOTS * U * 16 - 32 + 255) / 256) * 16 + 2;
};

template <int NB, int S>
__host__ __device__ constexpr size_t mfma_stage_bytes(int nrhs) {
  return 2 * (size_t)nrhs * StageShape<NB, S>::RSU * 16;
}

typedef __attribute__((address_space(3))) void lds_void;

// Copy segment g (0: the workgroup's own sites with one site of x-halo on each
// side; 1..6: the neighbouring row in direction +y,-y,+z,-z,+t,-t) of every live
// right-hand side into LDS row block `dst`.  Each load instruction of a wave
// fills 64 consecutive 16-byte LDS units; lanes whose unit is padding, beyond
// the segment or of a masked right-hand side are switched off.
template <int NB, int S>
__device__ __forceinline__ void stage_segment(float4* dst, const cf32* __restrict__ in, long fs, int nrhs,
                                              uint32_t live, int g, long site0, long left, long right, long base,
                                              int wv, int lane) {
  typedef StageShape<NB, S> ST;
  const int nslots = g == 0 ? S + 2 : S;
  const int npos = nrhs * ST::RSU;
  // a fixed, unrolled count (enough for 16 right-hand sides) keeps the number
  // of loads issued here known to the compiler's wait counting
  constexpr int NI = (16 * ST::RSU + 64 * S - 1) / (64 * S);
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int pos0 = 64 * (wv + S * i);
    if (pos0 >= npos) break;  // wave-uniform
    const int pos = pos0 + lane;
    const int r = pos / ST::RSU, w = pos - r * ST::RSU;
    const int slot = w / ST::U, c = w - slot * ST::U;
    long src;
    if (g == 0) src = slot == 0 ? left : slot == S + 1 ? right : site0 + slot - 1;
    else src = base + slot;
    if (pos < npos && slot < nslots && ((live >> r) & 1u)) {
      const float4* gp = (const float4*)(in + (long)r * fs + src * NB) + c;
      __builtin_amdgcn_global_load_lds((const void*)gp, (lds_void*)(dst + pos0), 16, 0, 0);
    }
  }
}

// wait for every vector-memory operation of this wave (the direct-to-LDS
// copies are not tracked by the compiler's own waits): vmcnt(0), expcnt and
// lgkmcnt left open
__device__ __forceinline__ void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// The workgroup's outputs (S sites x nrhs x Nb) leave through LDS: each wave
// puts its accumulators there, then the workgroup writes every right-hand
// side's S consecutive site vectors as whole 16-byte units, so a store
// instruction covers contiguous lines instead of 8-byte pieces of sixteen.
template <int NB, int S>
__device__ __forceinline__ void stage_store(const f32x4 (&acc)[MfmaShape<NB>::NT], float4* buf, cf32* __restrict__ out,
                                            long fs, long site0, int nrhs, uint32_t live, int wv, int lane) {
  typedef MfmaShape<NB> SH;
  typedef StageShape<NB, S> ST;
  constexpr int Q = SH::Q;
  constexpr bool REM = SH::REM;
  const int col = lane & 15, kq = lane >> 4;
  cf32* row = (cf32*)(buf + col * ST::RSU) + wv * NB;  // [rhs][site in workgroup][Nb], rhs stride RSU units
  const bool in_buf = col < nrhs;                       // the buffer holds nrhs rows
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (in_buf) row[16 * q + 4 * kq + v] = mkc(acc[2 * q][v], acc[2 * q + 1][v]);
  if (REM) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float other = __shfl_xor(acc[2 * Q][v], 32, 64);
      if (kq < 2 && in_buf) row[16 * Q + 4 * kq + v] = mkc(acc[2 * Q][v], other);
    }
  }
  __syncthreads();
  constexpr int UR = S * ST::U;  // 16-byte units of one right-hand side's S site vectors
  const int nunits = nrhs * UR;
  for (int t = threadIdx.x; t < nunits; t += 64 * S) {
    const int r = t / UR, u = t - r * UR;
    if ((live >> r) & 1u) ((float4*)(out + (long)r * fs + site0 * NB))[u] = buf[r * ST::RSU + u];
  }
}

template <int P, int NB, int S, bool OS>
__global__ void __launch_bounds__(64 * S) k_coarse_apply_mfma_lds(const typename MfmaChunk<P>::T* __restrict__ blk,
                                                                   const cf32* __restrict__ in,
                                                                   cf32* __restrict__ out,
                                                                   const int* __restrict__ nbr, long Vc, int nrhs,
                                                                   const int* __restrict__ run, int run_stride) {
  typedef MfmaShape<NB> SH;
  typedef StageShape<NB, S> ST;
  constexpr int NM = SH::NM;
  constexpr long CPD = mfma_chunks_per_dir(NB);
  extern __shared__ float4 stage[];  // [2][nrhs][RSU] 16-byte units
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int col = lane & 15, kq = lane >> 4;
  const long site0 = xcd_block(blockIdx.x, gridDim.x) * S;
  const long site = site0 + wv;
  const long fs = Vc * NB;
  // live right-hand sides (bit r), the same in every wave
  const bool live_lane = lane < nrhs && (!run || run[(long)lane * run_stride]);
  const uint32_t live = (uint32_t)(__ballot(live_lane) & 0xffffu);
  const bool rhs_ok = (live >> col) & 1u;
  const int rc = rhs_ok ? col : 0;  // dead columns compute on column 0 and are not stored
  // segment sources: x-halo and the first site of each neighbouring row
  const long left = nbr[1 * Vc + site0], right = nbr[0 * Vc + site0 + S - 1];
  long base[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) base[k] = nbr[(long)(k + 2) * Vc + site0];
  const int rows = nrhs * ST::RSU;  // units per buffer
  f32x4 acc[SH::NT];
#pragma unroll
  for (int t = 0; t < SH::NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const typename MfmaChunk<P>::T* bsite = blk + site * 9 * CPD;
  const int rid = (lane & 7) + 8 * kq;
  BlockRegs<P, SH::NCK> ca0, ca1, cr;
  mfma_issue<P, NB>(ca0, ca1, cr, bsite, lane, rid);
  stage_segment<NB, S>(stage, in, fs, nrhs, live, 0, site0, left, right, 0, wv, lane);
  wait_vm_all();
  __syncthreads();
#pragma unroll 1
  for (int d = 0; d < 9; ++d) {
    const int g = d < 3 ? 0 : d - 2;  // segment of direction d
    cf32 a[SH::Q > 0 ? SH::Q : 1][NM], ar[NM], bc[NM];
    mfma_decode<P, NB>(ca0, ca1, cr, a, ar);
    if (d < 8) mfma_issue<P, NB>(ca0, ca1, cr, bsite + (d + 1) * CPD, lane, rid);
    const int slot = d == 0 ? wv + 1 : d == 1 ? wv + 2 : wv;
    const cf32* sv = (const cf32*)(stage + (g & 1) * rows + rc * ST::RSU) + slot * NB + kq;
#pragma unroll
    for (int m = 0; m < NM; ++m) bc[m] = sv[4 * m];
    // the next segment is copied once this group's last LDS reads are issued
    // (no LDS read follows a copy before the wait at the group's end), and
    // lands while this direction's matrix-core work runs
    if (d >= 2 && d < 8) {
      long nb_base = base[0];
#pragma unroll
      for (int k = 1; k < 6; ++k) nb_base = g == k ? base[k] : nb_base;
      stage_segment<NB, S>(stage + ((g + 1) & 1) * rows, in, fs, nrhs, live, g + 1, site0, left, right, nb_base, wv,
                           lane);
    }
    mfma_direction<NB>(acc, a, ar, bc, lane);
    if (d >= 2 && d < 8) {
      wait_vm_all();
      __syncthreads();
    }
  }
  // buffer 1 held segment 5, last read before the barrier that ended its group
  if (OS) stage_store<NB, S>(acc, stage + rows, out, fs, site0, nrhs, live, wv, lane);
  else mfma_store<NB>(acc, out, fs, site, lane, rhs_ok);
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

// Largest dynamic LDS of a staged launch (the CU's 160 KB).
constexpr size_t kMaxStageBytes = 160 * 1024;

template <int P, int NB, int S, bool OS>
static void mfma_lds_t(const void* blk, const cf32* in, cf32* out, const int* nbr, long Vc, int nrhs, const int* run,
                       int run_stride, hipStream_t st) {
  const size_t lds = mfma_stage_bytes<NB, S>(nrhs);
  require(lds <= kMaxStageBytes, WCMG_ERR_ARG, "staged matrix-core apply: LDS stage exceeds 160 KB");
  // dynamic LDS above 64 KB is opted into once per kernel and device
  static std::atomic<uint64_t> opted{0};
  int dev = 0;
  WCMG_HIP(hipGetDevice(&dev));
  const uint64_t bit = 1ull << (dev & 63);
  if (!(opted.load() & bit)) {
    WCMG_HIP(hipFuncSetAttribute((const void*)k_coarse_apply_mfma_lds<P, NB, S, OS>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxStageBytes));
    opted.fetch_or(bit);
  }
  WCMG_LAUNCH((k_coarse_apply_mfma_lds<P, NB, S, OS>), dim3((unsigned)(Vc / S)), dim3(64 * S), lds, st,
              (const typename MfmaChunk<P>::T*)blk, in, out, nbr, Vc, nrhs, run, run_stride);
}

template <int P, int NB>
static void mfma_tile(int tile, const void* blk, const cf32* in, cf32* out, const int* nbr, long Vc, int nrhs,
                      const int* run, int run_stride, hipStream_t st) {
  switch (tile) {
    case 0: mfma_t<P, NB>(blk, in, out, nbr, Vc, nrhs, run, run_stride, st); break;
    case 4: mfma_lds_t<P, NB, 4, true>(blk, in, out, nbr, Vc, nrhs, run, run_stride, st); break;
    case 8: mfma_lds_t<P, NB, 8, true>(blk, in, out, nbr, Vc, nrhs, run, run_stride, st); break;
    case 16: mfma_lds_t<P, NB, 16, true>(blk, in, out, nbr, Vc, nrhs, run, run_stride, st); break;
    case 5: mfma_lds_t<P, NB, 4, false>(blk, in, out, nbr, Vc, nrhs, run, run_stride, st); break;
    case 9: mfma_lds_t<P, NB, 8, false>(blk, in, out, nbr, Vc, nrhs, run, run_stride, st); break;
    default: throw Error(WCMG_ERR_ARG, "matrix-core coarse apply: tile must be 0, 4, 5, 8, 9 or 16");
  }
}

template <int P>
static void mfma_nb(int nb, int tile, const void* blk, const cf32* in, cf32* out, const int* nbr, long Vc, int nrhs,
                    const int* run, int run_stride, hipStream_t st) {
  switch (nb) {
    case 8: mfma_tile<P, 8>(tile, blk, in, out, nbr, Vc, nrhs, run, run_stride, st); break;
    case 16: mfma_tile<P, 16>(tile, blk, in, out, nbr, Vc, nrhs, run, run_stride, st); break;
    case 24: mfma_tile<P, 24>(tile, blk, in, out, nbr, Vc, nrhs, run, run_stride, st); break;
    case 32: mfma_tile<P, 32>(tile, blk, in, out, nbr, Vc, nrhs, run, run_stride, st); break;
    case 40: mfma_tile<P, 40>(tile, blk, in, out, nbr, Vc, nrhs, run, run_stride, st); break;
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

bool mfma_tile_ok(int tile, int nb, long Vc, int Lx, int nrhs) {
  if (tile == 0) return true;
  if (tile == 5 || tile == 9) tile -= 1;  // the same tiles with per-wave output stores
  if ((tile != 4 && tile != 8 && tile != 16) || Lx % tile != 0 || Vc % tile != 0) return false;
  const int rsu = (((tile + 2) * (nb / 2) * 16 - 32 + 255) / 256) * 16 + 2;  // StageShape<nb, tile>::RSU
  return 2 * (size_t)nrhs * rsu * 16 <= kMaxStageBytes;
}

void launch_coarse_apply_mfma(int prec, int nb, const void* blk, const cf32* in, cf32* out, const int* nbr, long Vc,
                              int nrhs, const int* run, int run_stride, hipStream_t st, int tile, int Lx) {
  require(nrhs >= 1 && nrhs <= 16, WCMG_ERR_ARG, "matrix-core coarse apply takes 1..16 right-hand sides");
  require(tile == 0 || (Lx > 0 && mfma_tile_ok(tile, nb, Vc, Lx, nrhs)), WCMG_ERR_ARG,
          "staged matrix-core apply: the tile must divide the lattice's x extent");
  if (prec == WCMG_F32) mfma_nb<WCMG_F32>(nb, tile, blk, in, out, nbr, Vc, nrhs, run, run_stride, st);
  else mfma_nb<WCMG_BF16>(nb, tile, blk, in, out, nbr, Vc, nrhs, run, run_stride, st);
  WCMG_CHECK_LAUNCH();
}

}  // namespace wcmg
