// The coarsest-level GMRES (Sec. 2.1: GMRES is the coarse-grid solver) as one
// persistent launch for a whole solve (every workgroup resident at once, with
// grid-wide barriers), when the coarse operator fits the chip's LDS: each workgroup owns at most two coarse sites, loads their nine
// blocks into LDS once and keeps them there for every matrix-vector product
// of every Arnoldi step and restart.  The Krylov basis V and its image
// Z = A V stay in LDS too, for the workgroup's own rows.
//
// Each Arnoldi step takes one grid-wide reduction, of h1 = V^H p_j and
// |p_j|^2 together, where p_j = A v_j - s v_j with the shift s = Re h_00 of
// the restart cycle (s = 0 for the first step): the coarse operator is
// dominated by its diagonal, so A v_j lies mostly along v_j, and projecting
// p_j instead spans the same Krylov space with far less cancellation.  Then
// w1 = p_j - V h1 with |w1|^2 = |p_j|^2 - |h1|^2 (V orthonormal), and
// A w1 = A p_j - Z h1 (Z = A V at the own rows), where A p_j needs p_j at the
// neighbouring sites, which that reduction's barrier has made visible.
// Gram-Schmidt is repeated (a second reduction, of h2 = V^H w1 and |w1|^2)
// only when |w1|^2 < |p_j|^2 / 4, i.e. when the first pass removed more than
// three quarters of |p_j|^2 (the criterion of Daniel, Gragg, Kaufman and
// Stewart, with 1/4 in place of their 1/2: on these operators the first pass
// removes about 65%, the previous basis vector's share, which is mild
// cancellation); A w2 = A w1 - Z h2.  The Hessenberg column of A is
// h1 + s e_j (+ h2), and v_{j+1} = w / |w|, z_{j+1} = A w / |w|.
// Every workgroup sums the per-workgroup partials itself in a fixed order,
// so every workgroup holds bit-identical reductions, Givens rotations,
// control decisions (convergence, iteration limit, breakdown,
// reorthogonalisation) and, at the end of a restart cycle, the same
// least-squares solution y.
//
// Grid barrier: every workgroup waits for every other's flag (a phase number
// in its own 128-byte line), with one agent-scope release fence before the
// flag is raised and one acquire fence after the wait, both taken by one
// thread for the whole workgroup after every wave's stores have completed
// (on this chip each fence is a whole-L2 write-back or invalidate).  After
// the barrier, data that other workgroups wrote (partials, the vectors the
// stencil reads) is read with plain loads: the invalidate has dropped stale
// lines from this XCD's L2, and the first workgroup of an XCD to read a line
// brings it in for the others (agent-scope loads would bypass L2 and send
// every workgroup's reads of the same partials to memory).  The phase
// numbers continue from launch to launch (a device word holds the phase
// reached, read by every workgroup at the start and written by workgroup 0
// at the end), so the flags need no clearing, and workgroup 0 reports a normal
// end in a host-mapped mailbox: the launch's sequence number and its
// iteration count in a ring of report slots, so the host can check a launch
// later without stopping the stream.  A waiting thread gives up after a
// wall-clock timeout: the error word is set and every workgroup leaves
// without reporting; a launch that starts with the error word set returns
// x = 0 at once; the host clears the flags when it next checks.  A fault in
// the launch configuration cannot hang the device.
#include <map>

#include "coarse_common.h"

namespace wcmg {
namespace {
constexpr int kPMaxM1 = 41;     // restart + 1 (restart <= 40)
constexpr int kPSpw = 2;        // coarse sites per workgroup, at most
constexpr int kPStride = 48;    // partial slots (cd64) per workgroup and phase buffer
constexpr int kBarWords = 64;   // bar[2]: error word, bar[3..6]: report, bar[8]: phase; flags follow
constexpr int kBarPhase = 8;    // the phase the flags have reached, carried from launch to launch
constexpr int kFlagWords = 32;  // one 128-byte line per workgroup flag
constexpr int kPRtri = kPMaxM1 * (kPMaxM1 - 1) / 2;  // packed upper triangle, 40 columns

template <int P, int NB>
struct PShape {
  typedef typename BlkTraits<P>::R R;
  static constexpr int K = BlkTraits<P>::K, NCH = NB / K, NQ = 9 * NCH;
  static constexpr int rows = kPSpw * NB;  // LDS rows per workgroup
  static constexpr int s0 = 256 / rows;
  // lanes per row: the largest power of two that fits, at most 16
  static constexpr int S = s0 >= 16 ? 16 : s0 >= 8 ? 8 : s0 >= 4 ? 4 : s0 >= 2 ? 2 : 1;
  static constexpr size_t lds = (size_t)NQ * rows * 16 + 2 * (size_t)kPMaxM1 * rows * sizeof(cplx<R>) +
                                (size_t)kPSpw * 9 * NB * sizeof(cplx<R>) + (size_t)kPRtri * 16 +
                                (size_t)(4 * (kPMaxM1 + 1) + 4 * (kPMaxM1 + 1) + 2 * kPMaxM1) * 16 + 128;
  static constexpr bool fits = lds <= 160 * 1024;
};

// Returns false when a wait timed out, here or in another workgroup.
__device__ inline bool pbarrier(unsigned* bar, unsigned G, unsigned phase, int* fail, long long tick_limit) {
  unsigned* err = bar + 2;
  unsigned* flags = bar + kBarWords;
  // the workgroup barrier does not wait for stores: every wave first waits
  // until its own stores have reached this XCD's L2, so that the one
  // write-back below covers the whole workgroup's writes of this phase
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(flags + (size_t)kFlagWords * blockIdx.x, phase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  int bad = 0;
  const long long t0 = wall_clock64();
  for (unsigned g = threadIdx.x; g < G && !bad; g += blockDim.x) {
    unsigned seen;
    unsigned spins = 0;
    while ((seen = __hip_atomic_load(flags + (size_t)kFlagWords * g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) <
           phase) {
      // the error word and the clock are looked at every 16th poll only, so a
      // poll is one memory round trip (every poll with a zero time limit)
      if ((++spins & 15) != 0 && tick_limit > 0) {
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        bad = 1;
        break;
      }
      if (wall_clock64() - t0 > tick_limit) {
        if (__hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
          bar[3] = blockIdx.x;
          bar[4] = phase;
          bar[5] = g;
          bar[6] = seen;
        }
        bad = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  if (bad) *fail = 1;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();
  return *fail == 0;
}

__device__ inline cd64 shfl_xor_c(cd64 v, int off) {
  return mkc(__shfl_xor(v.re, off, 64), __shfl_xor(v.im, off, 64));
}

// Wave sums of eight entries at once: at offsets 32, 16 and 8 each lane
// keeps half of its remaining entries and receives its partner's share of
// them, then a butterfly over the last three lane bits; lane l ends with the
// sum of entry 4 b5 + 2 b4 + b3 (the bits of l), in a fixed order.
__device__ inline cd64 wred8(cd64 (&a)[8], int lane) {
  const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const cd64 send = h5 ? a[k] : a[k + 4], keep = h5 ? a[k + 4] : a[k];
    a[k] = cadd(keep, shfl_xor_c(send, 32));
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const cd64 send = h4 ? a[k] : a[k + 2], keep = h4 ? a[k + 2] : a[k];
    a[k] = cadd(keep, shfl_xor_c(send, 16));
  }
  cd64 v;
  {
    const cd64 send = h3 ? a[0] : a[1], keep = h3 ? a[1] : a[0];
    v = cadd(keep, shfl_xor_c(send, 8));
  }
  v = cadd(v, shfl_xor_c(v, 4));
  v = cadd(v, shfl_xor_c(v, 2));
  v = cadd(v, shfl_xor_c(v, 1));
  return v;
}
__device__ inline int wred8_entry(int lane) { return ((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1); }

// conj(a) b in FP64 (products of FP32 values are exact in FP64)
__device__ inline cd64 cdotd(cf32 a, cf32 b) {
  return mkc((double)a.re * b.re + (double)a.im * b.im, (double)a.re * b.im - (double)a.im * b.re);
}
}  // namespace

template <int P, int NB>
__global__ void __launch_bounds__(256) k_cg_persistent(
    const Chunk16* __restrict__ blk, const int* __restrict__ nbr, long Vc, const cplx<typename BlkTraits<P>::R>* b,
    cplx<typename BlkTraits<P>::R>* x, cplx<typename BlkTraits<P>::R>* zg, cplx<typename BlkTraits<P>::R>* r,
    cd64* part, cd64* misc, int* st, const int* parent, int m, double tol, int limit, int fixed, unsigned* bar,
    int seq, int* mailbox, long long tick_limit) {
  typedef PShape<P, NB> Sh;
  typedef typename Sh::R R;
  constexpr int K = Sh::K, NCH = Sh::NCH, NQ = Sh::NQ, ROWS = Sh::rows, SL = Sh::S;
  __shared__ Chunk16 tile[NQ][ROWS];
  __shared__ cplx<R> vl[kPMaxM1][ROWS];  // v_i at the own rows
  __shared__ cplx<R> zl[kPMaxM1][ROWS];  // A v_i at the own rows
  __shared__ cplx<R> ust[kPSpw][9][NB];  // the applied vector at the sites' stencil points
  __shared__ cd64 rtri[kPRtri];          // rotated Hessenberg R, column j at j (j + 1) / 2
  __shared__ cd64 red[4][kPMaxM1 + 1];
  __shared__ cd64 hs[kPMaxM1 + 1];       // reduced entries of the current phase
  __shared__ cd64 hcol[kPMaxM1 + 1], gv[kPMaxM1 + 1], csv[kPMaxM1], snv[kPMaxM1];
  __shared__ cd64 yv[kPMaxM1];
  __shared__ double scal[3];             // 0: |u|^2 of the next basis vector, 1: |b|^2 of the first cycle, 2: shift
  __shared__ int ctl[5];                 // 0: continue the cycle, 1: live, 2: jdone, 3: total, 4: reorthogonalise
  __shared__ int fail;
  const unsigned G = gridDim.x;
  const long n = Vc * NB;
  const long row0 = (long)blockIdx.x * ROWS;
  const int nrow = (int)min((long)ROWS, n - row0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = tid / SL, sub = tid - lr * SL;
  const bool own = lr < nrow && sub == 0;  // this thread holds row row0 + lr of every vector
  const long t = row0 + lr;
  const int lrc = min(lr, ROWS - 1);       // LDS row for unconditional reads (used only when own)

  // a wait of an earlier launch timed out and the flags have not been cleared
  // since: no barrier can be trusted, so this solve returns x = 0 (a weaker
  // preconditioner for the outer solve) and reports nothing
  if (__hip_atomic_load(bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
    if (own) x[t] = mkc((R)0, (R)0);
    return;
  }
  const unsigned phase0 = __hip_atomic_load(bar + kBarPhase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

  if (tid == 0) {
    fail = 0;
    ctl[1] = parent ? *parent : 1;
    ctl[2] = 0;
    ctl[3] = 0;
  }
  __syncthreads();
  if (blockIdx.x == 0 && tid == 0) {
    st[1] = ctl[1];
    st[0] = ctl[1];
    st[2] = 0;
    st[3] = 0;
    st[4] = 0;
  }
  // the normal end of the launch, reported by workgroup 0 (after every
  // barrier has been passed, unless a wait timed out somewhere)
  auto report = [&](unsigned final_phase) {
    if (blockIdx.x == 0 && tid == 0 && __hip_atomic_load(bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      __hip_atomic_store(bar + kBarPhase, final_phase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int* slot = mailbox + kCgpSlot0 + 2 * (seq & (kCgpSlots - 1));
      __hip_atomic_store(slot + 1, ctl[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(slot, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(mailbox + 1, ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(mailbox + 3, ctl[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(mailbox, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  };
  if (!ctl[1]) {  // uniform: every workgroup reads the same flag
    report(phase0);
    return;
  }

  // this workgroup's rows of the nine blocks, resident for the whole solve
  {
    // eight loads in flight per thread (indices past the end re-read the
    // last chunk and are not stored)
    const int total = NQ * nrow;
    for (int base = tid; base < total; base += 8 * 256) {
      Chunk16 c[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int idx = min(base + 256 * k, total - 1);
        const int q = idx / nrow, rr = idx - q * nrow;
        c[k] = blk[(long)q * n + row0 + rr];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int idx = base + 256 * k;
        if (idx < total) {
          const int q = idx / nrow, rr = idx - q * nrow;
          tile[q][rr] = c[k];
        }
      }
    }
  }
  __syncthreads();

  // (A u) at this thread's row (every lane of the row gets the sum): the
  // vector at the nine stencil points of the workgroup's sites is staged in
  // LDS (ust, flat index e = k + NB (d + 9 site); the source rows are fixed
  // for the whole solve and kept in registers), then SL lanes split the
  // row's chunks
  const int nsites = nrow / NB;
  constexpr int kStage = (kPSpw * 9 * NB + 255) / 256;
  long srcrow[kStage];
#pragma unroll
  for (int kk = 0; kk < kStage; ++kk) {
    const int e = tid + 256 * kk;
    srcrow[kk] = -1;
    if (e < nsites * 9 * NB) {
      const int k = e % NB, dd = (e / NB) % 9, ls = e / (9 * NB);
      const long site = row0 / NB + ls;
      srcrow[kk] = (dd == 0 ? site : (long)nbr[(long)(dd - 1) * Vc + site]) * NB + k;
    }
  }
  cplx<R>* ustf = &ust[0][0][0];
  // the stencil's source values are loaded into registers first, so their
  // loads can be in flight together with others (the reduction's partials)
  auto stage_load = [&](const cplx<R>* u, cplx<R>(&sv)[kStage]) __attribute__((always_inline)) {
#pragma unroll
    for (int kk = 0; kk < kStage; ++kk) sv[kk] = srcrow[kk] >= 0 ? u[srcrow[kk]] : mkc((R)0, (R)0);
  };
  auto apply_staged = [&](const cplx<R>(&sv)[kStage]) __attribute__((always_inline)) -> cplx<R> {
    __syncthreads();  // the previous apply's readers are done with ust
#pragma unroll
    for (int kk = 0; kk < kStage; ++kk)
      if (srcrow[kk] >= 0) ustf[tid + 256 * kk] = sv[kk];
    __syncthreads();
    cplx<R> acc = mkc((R)0, (R)0), acc2 = mkc((R)0, (R)0);
    if (lr < nrow) {
      const int ls = lr / NB;
#pragma unroll
      for (int q0 = 0; q0 < NQ; q0 += SL) {
        const int q = q0 + sub;
        if (q < NQ) {
          const int d = q / NCH, jc = q - d * NCH;
          cplx<R> mm[K];
          decode<P>(tile[q][lr], mm);
          const cplx<R>* phi = &ust[ls][d][jc * K];
#pragma unroll
          for (int k = 0; k < K; ++k) {
            if (k & 1) cfma(acc2, mm[k], phi[k]);
            else cfma(acc, mm[k], phi[k]);
          }
        }
      }
    }
    acc = cadd(acc, acc2);
#pragma unroll
    for (int off = 1; off < SL; off <<= 1) {
      acc.re += __shfl_xor(acc.re, off, 64);
      acc.im += __shfl_xor(acc.im, off, 64);
    }
    return acc;
  };
  auto apply_row = [&](const cplx<R>* u) __attribute__((always_inline)) -> cplx<R> {
    cplx<R> sv[kStage];
    stage_load(u, sv);
    return apply_staged(sv);
  };

  // Grid-wide sums of cnt entries: this workgroup's partials go to
  // part[pb][block][i]; after the barrier every workgroup adds the G
  // partials of each entry in the same order into hs.  Two partial buffers,
  // alternating by phase: a workgroup that has finished reading one phase may
  // write the next phase's partials while a slower one still reads the
  // previous phase's, and it can only come back to a buffer after the next
  // barrier, which every reader of that buffer has reached.
  unsigned phase = phase0;
  int pb = 0;
  const int ent = wred8_entry(lane);
  // reduce_begin: this workgroup's partials, then the grid barrier;
  // reduce_end: the sums into hs.  Loads issued between the two overlap the
  // partials' loads.
  auto reduce_begin = [&](int cnt, auto contrib) -> bool {
    for (int i0 = 0; i0 < cnt; i0 += 8) {
      cd64 a[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const cd64 v = contrib(min(i0 + k, cnt - 1));
        a[k] = own && i0 + k < cnt ? v : mkc(0.0, 0.0);
      }
      const cd64 s = wred8(a, lane);
      if ((lane & 7) == 0 && i0 + ent < cnt) red[wave][i0 + ent] = s;
    }
    __syncthreads();
    if (tid < cnt)
      part[((size_t)pb * G + blockIdx.x) * kPStride + tid] =
          cadd(cadd(red[0][tid], red[1][tid]), cadd(red[2][tid], red[3][tid]));
    return pbarrier(bar, G, ++phase, &fail, tick_limit);
  };
  auto reduce_end = [&](int cnt) {
    for (int i0 = 0; i0 < cnt; i0 += 8) {
      cd64 a[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) a[k] = mkc(0.0, 0.0);
      for (unsigned g = tid; g < G; g += blockDim.x) {
        const cd64* pg = part + ((size_t)pb * G + g) * kPStride + i0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          // every slot is in bounds (i0 + k < kPStride); only the first cnt count
          const cd64 v = pg[k];
          if (i0 + k < cnt) a[k] = cadd(a[k], v);
        }
      }
      const cd64 s = wred8(a, lane);
      if ((lane & 7) == 0 && i0 + ent < cnt) red[wave][i0 + ent] = s;
    }
    __syncthreads();
    if (tid < cnt) hs[tid] = cadd(cadd(red[0][tid], red[1][tid]), cadd(red[2][tid], red[3][tid]));
    __syncthreads();
    pb ^= 1;
  };
  auto reduce = [&](int cnt, auto contrib) -> bool {
    if (!reduce_begin(cnt, contrib)) return false;
    reduce_end(cnt);
    return true;
  };

  const int max_cycles = (limit + m - 1) / m;
  cplx<R> xv = mkc((R)0, (R)0);
  cplx<R> pj = mkc((R)0, (R)0);  // p_j at the own row, as stored in zg
  if (own) x[t] = xv;
  for (int cyc = 0; cyc < max_cycles; ++cyc) {
    // residual of the current x (zero on the first cycle: u0 = b)
    const cplx<R>* u0 = b;
    if (cyc > 0) {
      if (!pbarrier(bar, G, ++phase, &fail, tick_limit)) return;  // x complete
      const cplx<R> ax = apply_row(x);
      if (own) r[t] = csub(b[t], ax);
      u0 = r;
    }
    const cplx<R> uo = own ? u0[t] : mkc((R)0, (R)0);
    // |u0|^2 (the barrier also completes u0 everywhere)
    if (!reduce(1, [&](int) { return mkc((double)uo.re * uo.re + (double)uo.im * uo.im, 0.0); })) return;
    if (tid == 0) {
      const double b2 = hs[0].re;
      if (cyc == 0) scal[1] = b2;
      scal[0] = b2;
      const double bn = sqrt(scal[1]), beta = sqrt(b2);
      ctl[2] = 0;
      ctl[0] = 1;
      if (ctl[3] >= limit || bn == 0.0 || beta == 0.0 || (!fixed && beta <= tol * bn) || !(beta == beta)) {
        ctl[0] = 0;
        ctl[1] = 0;
        if (blockIdx.x == 0) st[4] = !(beta == beta) ? 3 : 1;
      } else {
        for (int i = 0; i <= kPMaxM1; ++i) gv[i] = mkc(0.0, 0.0);
        gv[0] = mkc(beta, 0.0);
      }
      if (blockIdx.x == 0) {
        misc[1] = mkc(b2, 0.0);
        if (cyc == 0) misc[0] = mkc(b2, 0.0);
        misc[2].re = bn > 0 ? beta / bn : 0.0;
      }
    }
    __syncthreads();
    if (!ctl[0]) break;
    {
      // v_0 = u0 / beta, z_0 = A u0 / beta
      const cplx<R> au = apply_row(u0);
      const R inv = (R)(1.0 / sqrt(scal[0]));
      if (own) {
        vl[0][lr] = cscale(inv, uo);
        zl[0][lr] = cscale(inv, au);
        pj = zl[0][lr];
        zg[t] = pj;
      }
    }

    for (int j = 0; j < m; ++j) {
      // h1 = V^H z_j and |z_j|^2 (the barrier also completes z_j, which the
      // apply below reads at the neighbouring sites; z_j alternates between
      // two global buffers, so a workgroup writing z_{j+1} cannot overwrite
      // rows a slower one still reads)
      const cplx<R> zj = pj;
      if (!reduce_begin(j + 2, [&](int i) {
            return i <= j ? cdotd(vl[i][lrc], zj) : mkc((double)zj.re * zj.re + (double)zj.im * zj.im, 0.0);
          }))
        return;
      cplx<R> sv[kStage];
      stage_load(zg + (long)(j & 1) * n, sv);
      reduce_end(j + 2);
      cplx<R> aw = apply_staged(sv);
      cplx<R> wv = zj;
      if (own)
#pragma unroll 4
        for (int i = 0; i <= j; ++i) {
          const cplx<R> h = cneg(mkc((R)hs[i].re, (R)hs[i].im));
          cfma(wv, h, vl[i][lr]);
          cfma(aw, h, zl[i][lr]);
        }
      if (tid == 0) {
        double n1 = hs[j + 1].re;
        for (int i = 0; i <= j; ++i) {
          hcol[i] = hs[i];
          n1 -= hs[i].re * hs[i].re + hs[i].im * hs[i].im;
        }
        if (j == 0) scal[2] = hs[0].re;  // the shift of the later steps
        else hcol[j].re += scal[2];
        scal[0] = n1;
        ctl[4] = n1 < 0.25 * hs[j + 1].re;
      }
      __syncthreads();
      if (ctl[4]) {
        // h2 = V^H w1 and |w1|^2 (computed from w1 itself)
        if (!reduce(j + 2, [&](int i) {
              return i <= j ? cdotd(vl[i][lrc], wv) : mkc((double)wv.re * wv.re + (double)wv.im * wv.im, 0.0);
            }))
          return;
        if (own)
          for (int i = 0; i <= j; ++i) {
            const cplx<R> h = cneg(mkc((R)hs[i].re, (R)hs[i].im));
            cfma(wv, h, vl[i][lr]);
            cfma(aw, h, zl[i][lr]);
          }
        if (tid == 0) {
          double n2 = hs[j + 1].re;
          for (int i = 0; i <= j; ++i) {
            hcol[i] = cadd(hcol[i], hs[i]);
            n2 -= hs[i].re * hs[i].re + hs[i].im * hs[i].im;
          }
          scal[0] = n2;
        }
      }
      // |w|^2 and the Givens rotation of the Hessenberg column
      if (tid == 0) {
        const double hn2 = scal[0] > 0.0 ? scal[0] : 0.0;
        const double hn = sqrt(hn2);
        scal[0] = hn2;
        // the entry being rotated down the column stays in registers, so the
        // loads of the next rotation do not wait for this one's stores
        cd64 a = hcol[0];
#pragma unroll 4
        for (int i = 0; i < j; ++i) {
          const cd64 bb = hcol[i + 1], ci = csv[i], si = snv[i];
          cd64 tt = cmul(ci, a);
          cfma(tt, si, bb);
          cd64 uu = cmul(cneg(cconj(si)), a);
          cfma(uu, cconj(ci), bb);
          hcol[i] = tt;
          a = uu;
        }
        const double den = sqrt(a.re * a.re + a.im * a.im + hn2);
        const cd64 cc = den == 0.0 ? mkc(1.0, 0.0) : mkc(a.re / den, -a.im / den);
        const cd64 ss = den == 0.0 ? mkc(0.0, 0.0) : mkc(hn / den, 0.0);
        csv[j] = cc;
        snv[j] = ss;
        hcol[j] = mkc(den, 0.0);
        for (int i = 0; i <= j; ++i) rtri[j * (j + 1) / 2 + i] = hcol[i];
        const cd64 gj = gv[j];
        gv[j + 1] = den == 0.0 ? gj : cmul(cneg(cconj(ss)), gj);  // den == 0: singular column, dropped
        gv[j] = cmul(cc, gj);
        ctl[2] = den == 0.0 ? j : j + 1;
        ctl[3] += 1;
        const double bn = sqrt(scal[1]);
        const double est = bn > 0 ? sqrt(gv[j + 1].re * gv[j + 1].re + gv[j + 1].im * gv[j + 1].im) / bn : 0.0;
        bool stop = false;
        int reason = 0;
        if (ctl[3] >= limit) {
          stop = true;
          reason = 2;
        }
        if (!fixed && est <= tol) {
          stop = true;
          reason = 1;
        }
        if (hn == 0.0 || !(est == est)) {
          stop = true;
          reason = (est == est) ? (den == 0.0 ? 4 : 1) : 3;
        }
        if (stop) ctl[1] = 0;
        ctl[0] = (stop || j + 1 == m) ? 0 : 1;
        if (blockIdx.x == 0) {
          misc[3] = mkc(hn2, 0.0);
          misc[2].re = est;
          if (stop) st[4] = reason;
        }
      }
      __syncthreads();
      if (!ctl[0]) break;
      const R inv = (R)(1.0 / sqrt(scal[0]));
      if (own) {
        const cplx<R> v1 = cscale(inv, wv), z1 = cscale(inv, aw);
        vl[j + 1][lr] = v1;
        zl[j + 1][lr] = z1;
        pj = csub(z1, cscale((R)scal[2], v1));
        zg[(long)((j + 1) & 1) * n + t] = pj;
      }
    }
    // y from the leading jdone x jdone triangle (every workgroup its own,
    // bit-identical copy), then x += V y at the own rows
    const int jd = ctl[2];
    if (tid == 0)
      for (int i = jd - 1; i >= 0; --i) {
        cd64 s = gv[i];
        for (int k = i + 1; k < jd; ++k) s = csub(s, cmul(rtri[k * (k + 1) / 2 + i], yv[k]));
        const cd64 d = rtri[i * (i + 1) / 2 + i];
        const double dd = d.re * d.re + d.im * d.im;
        yv[i] = dd > 0.0 ? mkc((s.re * d.re + s.im * d.im) / dd, (s.im * d.re - s.re * d.im) / dd) : mkc(0.0, 0.0);
      }
    __syncthreads();
    if (own) {
      for (int k = 0; k < jd; ++k) cfma(xv, mkc((R)yv[k].re, (R)yv[k].im), vl[k][lr]);
      x[t] = xv;
    }
    if (!ctl[1]) break;
  }
  if (blockIdx.x == 0 && tid == 0) {
    st[0] = 0;
    st[1] = ctl[1];
    st[2] = 0;
    st[3] = ctl[3];
  }
  report(phase);
}

namespace {
template <int P, int NB>
bool cgp_shape_fits() {
  if constexpr (PShape<P, NB>::fits) return true;
  else return false;
}

// Returns false (and launches nothing) when the workgroups cannot all be
// co-resident.  The grid is launched as an ordinary kernel (one workgroup per
// CU at most, nothing else on the stream while it runs, so all workgroups are
// resident together); coop: through the cooperative-launch API instead, which
// guarantees co-residency at a few microseconds more per launch.  Every barrier
// wait has a time limit either way.  The device properties and the occupancy
// are queried once per device: per launch they cost host time the device
// waited for.
template <int P, int NB>
bool cgp_launch(const void* blk, const int* nbr, long Vc, const void* b, void* x, void* z, void* r, cd64* part,
                cd64* misc, int* st, const int* parent, int m, double tol, int limit, int fixed, unsigned* bar,
                int seq, int* mailbox, long long tick_limit, bool coop_api, hipStream_t stream) {
  if constexpr (!PShape<P, NB>::fits) {
    return false;
  } else {
    typedef typename BlkTraits<P>::R R;
    auto kern = k_cg_persistent<P, NB>;
    // device properties and the occupancy, per device (queried once)
    struct Props {
      int cus = 0, coop = 0, per_cu = -1;
    };
    static thread_local std::map<int, Props> props;
    int dev = 0;
    WCMG_HIP(hipGetDevice(&dev));
    Props& pr = props[dev];
    if (pr.per_cu < 0) {
      WCMG_HIP(hipDeviceGetAttribute(&pr.cus, hipDeviceAttributeMultiprocessorCount, dev));
      WCMG_HIP(hipDeviceGetAttribute(&pr.coop, hipDeviceAttributeCooperativeLaunch, dev));
      WCMG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&pr.per_cu, kern, 256, 0));
    }
    const long G = (Vc + kPSpw - 1) / kPSpw;
    if ((coop_api && !pr.coop) || pr.per_cu < 1 || G > (long)pr.cus * pr.per_cu || m + 1 > kPMaxM1 || m < 1)
      return false;
    const Chunk16* bk = (const Chunk16*)blk;
    const cplx<R>* bc = (const cplx<R>*)b;
    cplx<R>* xx = (cplx<R>*)x;
    cplx<R>* zz = (cplx<R>*)z;
    cplx<R>* rr = (cplx<R>*)r;
    void* args[] = {(void*)&bk,   (void*)&nbr, (void*)&Vc,    (void*)&bc,    (void*)&xx,    (void*)&zz,
                    (void*)&rr,   (void*)&part, (void*)&misc, (void*)&st,    (void*)&parent, (void*)&m,
                    (void*)&tol,  (void*)&limit, (void*)&fixed, (void*)&bar, (void*)&seq,
                    (void*)&mailbox, (void*)&tick_limit};
    if (coop_api)
      WCMG_HIP(hipLaunchCooperativeKernel((const void*)kern, dim3((unsigned)G), dim3(256), args, 0, stream));
    else
      WCMG_HIP(hipLaunchKernel((const void*)kern, dim3((unsigned)G), dim3(256), args, 0, stream));
    return true;
  }
}
}  // namespace

bool cg_persistent_fits(int prec, int nb, long Vc) {
  if (Vc < 1 || Vc > 2L * 256 * 4) return false;  // refined by the occupancy check at launch
  if (prec == WCMG_F32) {
    switch (nb) {
      case 8: return cgp_shape_fits<WCMG_F32, 8>();
      case 12: return cgp_shape_fits<WCMG_F32, 12>();
      case 16: return cgp_shape_fits<WCMG_F32, 16>();
      case 24: return cgp_shape_fits<WCMG_F32, 24>();
      case 32: return cgp_shape_fits<WCMG_F32, 32>();
      default: return false;
    }
  }
  if (prec == WCMG_BF16) {
    switch (nb) {
      case 8: return cgp_shape_fits<WCMG_BF16, 8>();
      case 12: return cgp_shape_fits<WCMG_BF16, 12>();
      case 16: return cgp_shape_fits<WCMG_BF16, 16>();
      case 24: return cgp_shape_fits<WCMG_BF16, 24>();
      case 32: return cgp_shape_fits<WCMG_BF16, 32>();
      default: return false;
    }
  }
  return false;
}

size_t cg_persistent_part_elems(long Vc) { return (size_t)2 * kPStride * (size_t)((Vc + kPSpw - 1) / kPSpw); }
size_t cg_persistent_bar_words(long Vc) { return (size_t)kBarWords + (size_t)kFlagWords * ((Vc + kPSpw - 1) / kPSpw); }

bool launch_cg_persistent(int prec, int nb, const void* blk, const int* nbr, long Vc, const void* b, void* x,
                          void* z, void* r, cd64* part, cd64* misc, int* st, const int* parent, int m, double tol,
                          int limit, int fixed, unsigned* bar, int seq, int* mailbox, double timeout_s,
                          bool coop_api, hipStream_t stream) {
  if (!cg_persistent_fits(prec, nb, Vc)) return false;
  static thread_local std::map<int, int> rate;
  int dev = 0;
  WCMG_HIP(hipGetDevice(&dev));
  if (!rate.count(dev)) WCMG_HIP(hipDeviceGetAttribute(&rate[dev], hipDeviceAttributeWallClockRate, dev));
  const int khz = rate[dev];
  const long long tick_limit = (long long)(timeout_s * 1000.0 * (khz > 0 ? khz : 100000));
#define CGP(PP, NBc) \
  return cgp_launch<PP, NBc>(blk, nbr, Vc, b, x, z, r, part, misc, st, parent, m, tol, limit, fixed, bar, \
                             seq, mailbox, tick_limit, coop_api, stream)
  if (prec == WCMG_F32) {
    switch (nb) {
      case 8: CGP(WCMG_F32, 8);
      case 12: CGP(WCMG_F32, 12);
      case 16: CGP(WCMG_F32, 16);
      case 24: CGP(WCMG_F32, 24);
      default: CGP(WCMG_F32, 32);
    }
  }
  switch (nb) {
    case 8: CGP(WCMG_BF16, 8);
    case 12: CGP(WCMG_BF16, 12);
    case 16: CGP(WCMG_BF16, 16);
    case 24: CGP(WCMG_BF16, 24);
    default: CGP(WCMG_BF16, 32);
  }
#undef CGP
}

}  // namespace wcmg
