// The coarsest-level GMRES (Sec. 2.1: GMRES is the coarse-grid solver) as one
// cooperative launch for a whole solve, when the coarse operator fits the
// chip's LDS: each workgroup owns at most two coarse sites, loads their nine
// blocks into LDS once, and keeps them there for every matrix-vector product
// of every Arnoldi step and restart.  The steps are those of the fused
// four-kernel form (coarse_gmres.hip): w = A u / |u| with v_j = u / |u|,
// classical Gram-Schmidt applied twice, |w|^2, Givens rotation; the kernel
// boundaries between them become grid barriers, and every workgroup reduces
// the per-workgroup partials (double-buffered by phase) itself in a fixed
// order, so every control decision (convergence, iteration limit, breakdown)
// is taken identically by all workgroups.  Workgroup 0 keeps the Hessenberg matrix, solves for y at
// the end of a restart cycle and writes the state words.
//
// Grid barrier: a counter and a generation word in device memory, with
// agent-scope release/acquire fences around them; a waiting workgroup gives
// up after a wall-clock timeout (the error word is set, every later barrier
// passes at once and the host redoes the solve with the multi-kernel form),
// so a fault in the launch configuration cannot hang the device.
#include "coarse_common.h"

namespace wcmg {

namespace {
constexpr int kPMaxM1 = 41;  // restart + 1 (restart <= 40)
constexpr int kPSpw = 2;     // coarse sites per workgroup, at most

// bar: [0] arrival counter, [1] generation, [2] error word, [3..6] the first
// timed-out workgroup's report (workgroup, barriers it had passed, counter
// and generation it saw).  nb_passed: this workgroup's barrier count (LDS).
__device__ inline bool pbarrier(unsigned* bar, unsigned nblocks, int* nb_passed, long long tick_limit) {
  __shared__ int failed;
  unsigned* err = bar + 2;
  // every wave releases its own global writes (L2 write-back) before arriving
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    int bad = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    if (!bad) {
      const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (arrived == nblocks - 1) {
        __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        const long long t0 = wall_clock64();
        while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
          const bool other = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
          if (other || wall_clock64() - t0 > tick_limit) {
            if (!other && __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
              bar[3] = blockIdx.x;
              bar[4] = (unsigned)*nb_passed;
              bar[5] = __hip_atomic_load(&bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              bar[6] = gen;
            }
            bad = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
    }
    failed = bad;
    ++*nb_passed;
  }
  __syncthreads();
  // every wave acquires for itself: one wave's cache invalidation is not
  // ordered before the other waves' later loads, which could then read the
  // previous phase's partials from this XCD's L2
  __threadfence();
  return failed == 0;
}

// Loads of data that other workgroups (possibly on other XCDs) wrote during
// this launch: agent-scope atomic loads, which read the coherent copy instead
// of a line this XCD's L2 may still hold from an earlier phase.
__device__ inline cd64 ld_shared(const cd64* p) {
  const unsigned long long* q = (const unsigned long long*)p;
  const unsigned long long a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return mkc(__builtin_bit_cast(double, a), __builtin_bit_cast(double, b));
}
__device__ inline cf32 ld_shared(const cf32* p) {
  const unsigned long long a =
      __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return mkc(__builtin_bit_cast(float, (unsigned)a), __builtin_bit_cast(float, (unsigned)(a >> 32)));
}

__device__ inline cd64 pwsum(cd64 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.re += __shfl_xor(v.re, off, 64);
    v.im += __shfl_xor(v.im, off, 64);
  }
  return v;
}

// Device scalars of one solve, in the layout of the fused path's (H, cs, sn,
// g, y, misc): H [(m+1) x m] row-major, then m, m, m+1, m entries, then misc.
struct PScalars {
  cd64 *H, *y, *misc;
  __device__ PScalars(cd64* S, int m) {
    H = S;
    y = S + (m + 1) * m + 2 * m + (m + 1);
    misc = y + m;
  }
};

template <int NB>
struct PShape {
  static constexpr int rows = kPSpw * NB;  // LDS rows per workgroup
  static constexpr int s0 = 256 / rows;
  // lanes per row: the largest power of two that fits, at most 16
  static constexpr int S = s0 >= 16 ? 16 : s0 >= 8 ? 8 : s0 >= 4 ? 4 : s0 >= 2 ? 2 : 1;
};
}  // namespace

template <int P, int NB>
__global__ void __launch_bounds__(256) k_cg_persistent(
    const Chunk16* __restrict__ blk, const int* __restrict__ nbr, long Vc, const cplx<typename BlkTraits<P>::R>* b,
    cplx<typename BlkTraits<P>::R>* x, cplx<typename BlkTraits<P>::R>* V, cplx<typename BlkTraits<P>::R>* w,
    cplx<typename BlkTraits<P>::R>* r, cd64* part, cd64* S, int* st, const int* parent, int m, double tol,
    int limit, int fixed, unsigned* bar, long long tick_limit) {
  typedef typename BlkTraits<P>::R R;
  constexpr int K = BlkTraits<P>::K, NCH = NB / K, NQ = 9 * NCH;
  constexpr int ROWS = PShape<NB>::rows, SL = PShape<NB>::S;
  __shared__ Chunk16 tile[NQ][ROWS];
  __shared__ cd64 red[4][kPMaxM1];
  __shared__ cd64 hs[kPMaxM1];  // reduced entries of the current phase
  __shared__ cd64 hcol[kPMaxM1], csv[kPMaxM1], snv[kPMaxM1], gv[kPMaxM1];
  __shared__ double scal[4];    // 0: |u|^2 of the vector being applied, 1: |b|^2 of the first cycle
  __shared__ int ctl[4];        // 0: continue the cycle, 1: live, 2: jdone, 3: total
  __shared__ int nbar;          // barriers passed (diagnostics)
  __shared__ cplx<R> ust[kPSpw][9][NB];  // the applied vector at the sites' stencil points
  const unsigned G = gridDim.x;
  const long n = Vc * NB;
  const long row0 = (long)blockIdx.x * ROWS;
  const int nrow = (int)min((long)ROWS, n - row0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = tid / SL, sub = tid - lr * SL;
  const bool own = lr < nrow && sub == 0;  // this thread holds row row0 + lr of every vector
  const long t = row0 + lr;
  PScalars c(S, m);

  // live flag of this solve (the caller's run flag)
  if (tid == 0) {
    nbar = 0;
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
  if (!ctl[1]) return;  // uniform: every workgroup reads the same flag

  // this workgroup's rows of the nine blocks, resident for the whole solve
  for (int idx = tid; idx < NQ * nrow; idx += blockDim.x) {
    const int q = idx / nrow, rr = idx - q * nrow;
    tile[q][rr] = blk[(long)q * n + row0 + rr];
  }
  __syncthreads();

  // (A u)_t for this thread's row: the vector at the nine stencil points of
  // the workgroup's sites is staged in LDS (coherent loads), then SL lanes
  // split the row's chunks
  const int nsites = nrow / NB;
  auto apply_row = [&](const cplx<R>* u) -> cplx<R> {
    __syncthreads();  // the previous apply's readers are done with ust
    for (int e = tid; e < nsites * 9 * NB; e += blockDim.x) {
      const int k = e % NB, dd = (e / NB) % 9, ls = e / (9 * NB);
      const long site = row0 / NB + ls;
      const long src = dd == 0 ? site : (long)nbr[(long)(dd - 1) * Vc + site];
      ust[ls][dd][k] = ld_shared(u + src * NB + k);
    }
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
  // per-workgroup partials of cnt entries (entry-major: part[i * G + block]).
  // Two buffers, alternating by phase: a workgroup that has finished reducing
  // one phase may write the next phase's partials while a slower one still
  // reads the previous phase's; it can only come back to a buffer after the
  // next barrier, which every reader of that buffer has reached.
  int pb = 0;
  auto block_partials = [&](int cnt, auto contrib) {
    for (int i = 0; i < cnt; ++i) {
      const cd64 s = pwsum(own ? contrib(i) : mkc(0.0, 0.0));
      if (lane == 0) red[wave][i] = s;
    }
    __syncthreads();
    if (tid < cnt) {
      cd64 s = mkc(0.0, 0.0);
      for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s = cadd(s, red[q][tid]);
      part[(long)(pb * kPMaxM1 + tid) * G + blockIdx.x] = s;
    }
  };
  // every workgroup: hs[i] = sum over the G partials of entry i (fixed order)
  auto grid_reduce = [&](int cnt) {
    for (int i = wave; i < cnt; i += (int)(blockDim.x >> 6)) {
      cd64 s = mkc(0.0, 0.0);
      for (unsigned g = lane; g < G; g += 64) s = cadd(s, ld_shared(part + (long)(pb * kPMaxM1 + i) * G + g));
      s = pwsum(s);
      if (lane == 0) hs[i] = s;
    }
    __syncthreads();
    pb ^= 1;
  };

  const int max_cycles = (limit + m - 1) / m;
  cplx<R> xv = mkc((R)0, (R)0);
  if (own) x[t] = xv;
  for (int cyc = 0; cyc < max_cycles; ++cyc) {
    // residual of the current x (zero on the first cycle: u0 = b)
    const cplx<R>* u0 = b;
    if (cyc > 0) {
      if (!pbarrier(bar, G, &nbar, tick_limit)) return;  // x complete
      const cplx<R> ax = apply_row(x);
      if (own) r[t] = csub(b[t], ax);
      u0 = r;
    }
    {
      const cplx<R> uv = own ? u0[t] : mkc((R)0, (R)0);
      const double q = (double)uv.re * uv.re + (double)uv.im * uv.im;
      block_partials(1, [&](int) { return mkc(q, 0.0); });
    }
    if (!pbarrier(bar, G, &nbar, tick_limit)) return;
    grid_reduce(1);
    if (tid == 0) {
      const double b2 = hs[0].re;
      scal[0] = b2;
      if (cyc == 0) scal[1] = b2;
      const double bn = sqrt(scal[1]), beta = sqrt(b2);
      ctl[2] = 0;
      ctl[0] = 1;
      if (ctl[3] >= limit || bn == 0.0 || beta == 0.0 || (!fixed && beta <= tol * bn) || !(beta == beta)) {
        ctl[0] = 0;
        ctl[1] = 0;
        if (blockIdx.x == 0) st[4] = !(beta == beta) ? 3 : 1;
      } else {
        for (int i = 0; i < kPMaxM1; ++i) gv[i] = mkc(0.0, 0.0);
        gv[0] = mkc(beta, 0.0);
      }
      if (blockIdx.x == 0) {
        c.misc[1] = mkc(b2, 0.0);
        if (cyc == 0) c.misc[0] = mkc(b2, 0.0);
        c.misc[2].re = bn > 0 ? beta / bn : 0.0;
      }
    }
    __syncthreads();
    if (!ctl[0]) break;

    const cplx<R>* u = u0;
    for (int j = 0; j < m; ++j) {
      // 1. w = A u / |u|, v_j = u / |u|, partials of <v_i, w>
      const double inv = 1.0 / sqrt(scal[0]);
      const cplx<R> au = apply_row(u);
      cplx<R> vj = mkc((R)0, (R)0), wv = mkc((R)0, (R)0);
      if (own) {
        const cplx<R> ut = u[t];
        vj = mkc((R)(ut.re * inv), (R)(ut.im * inv));
        wv = mkc((R)(au.re * inv), (R)(au.im * inv));
        V[(long)j * n + t] = vj;
      }
      auto dots = [&](int i) {
        const cplx<R> vi = i == j ? vj : V[(long)i * n + t];
        return mkc((double)vi.re * wv.re + (double)vi.im * wv.im, (double)vi.re * wv.im - (double)vi.im * wv.re);
      };
      block_partials(j + 1, dots);
      if (!pbarrier(bar, G, &nbar, tick_limit)) return;
      grid_reduce(j + 1);
      // 2. and 3. two classical Gram-Schmidt passes
      for (int pass = 0; pass < 2; ++pass) {
        if (tid <= j) hcol[tid] = pass == 0 ? hs[tid] : cadd(hcol[tid], hs[tid]);
        if (own)
          for (int i = 0; i <= j; ++i) {
            const cplx<R> hi = mkc((R)hs[i].re, (R)hs[i].im);
            cfma(wv, cneg(hi), i == j ? vj : V[(long)i * n + t]);
          }
        __syncthreads();
        if (pass == 0) {
          block_partials(j + 1, dots);
        } else {
          if (own) w[t] = wv;
          const double q = (double)wv.re * wv.re + (double)wv.im * wv.im;
          block_partials(1, [&](int) { return mkc(q, 0.0); });
        }
        if (!pbarrier(bar, G, &nbar, tick_limit)) return;
        grid_reduce(pass == 0 ? j + 1 : 1);
      }
      // 4. |w|^2 and the Givens rotation of column j (every workgroup)
      if (tid == 0) {
        const double hn2 = hs[0].re, hn = sqrt(hn2);
        scal[0] = hn2;
        for (int i = 0; i < j; ++i) {
          const cd64 a = hcol[i], bb = hcol[i + 1];
          cd64 tt = cmul(csv[i], a);
          cfma(tt, snv[i], bb);
          cd64 uu = cmul(cneg(cconj(snv[i])), a);
          cfma(uu, cconj(csv[i]), bb);
          hcol[i] = tt;
          hcol[i + 1] = uu;
        }
        const cd64 a = hcol[j];
        const double den = sqrt(a.re * a.re + a.im * a.im + hn2);
        const cd64 cc = den == 0.0 ? mkc(1.0, 0.0) : mkc(a.re / den, -a.im / den);
        const cd64 ss = den == 0.0 ? mkc(0.0, 0.0) : mkc(hn / den, 0.0);
        csv[j] = cc;
        snv[j] = ss;
        hcol[j] = mkc(den, 0.0);
        hcol[j + 1] = mkc(0.0, 0.0);
        const cd64 gj = gv[j];
        gv[j + 1] = cmul(cneg(cconj(ss)), gj);
        gv[j] = cmul(cc, gj);
        ctl[2] = j + 1;
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
          reason = (est == est) ? 1 : 3;
        }
        if (stop) ctl[1] = 0;
        ctl[0] = (stop || j + 1 == m) ? 0 : 1;
        if (blockIdx.x == 0) {
          for (int i = 0; i <= j + 1 && i < m + 1; ++i)
            if (i * m + j < (m + 1) * m) c.H[i * m + j] = hcol[i];
          c.misc[3] = mkc(hn2, 0.0);
          c.misc[2].re = est;
          if (stop) st[4] = reason;
        }
      }
      __syncthreads();
      u = w;
      if (!ctl[0]) break;
      // the next step reads w at neighbouring rows: written before the last barrier
    }
    // y from the leading jdone x jdone triangle (every workgroup, its own copy)
    const int jd = ctl[2];
    if (tid == 0 && blockIdx.x == 0) {
      for (int i = jd - 1; i >= 0; --i) {
        cd64 s = gv[i];
        for (int k = i + 1; k < jd; ++k) s = csub(s, cmul(c.H[i * m + k], c.y[k]));
        const cd64 d = c.H[i * m + i];
        const double dd = d.re * d.re + d.im * d.im;
        c.y[i] = mkc((s.re * d.re + s.im * d.im) / dd, (s.im * d.re - s.re * d.im) / dd);
      }
    }
    if (!pbarrier(bar, G, &nbar, tick_limit)) return;  // y written by workgroup 0
    if (own) {
      for (int k = 0; k < jd; ++k) {
        const cd64 yk = ld_shared(c.y + k);
        cfma(xv, mkc((R)yk.re, (R)yk.im), V[(long)k * n + t]);
      }
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
}

// Returns false (and launches nothing) when the operator does not fit: more
// than 2 * (co-resident workgroups) coarse sites, an unsupported Nb, FP64
// storage, or no cooperative launch.
template <int P, int NB>
static bool cgp_launch(const void* blk, const int* nbr, long Vc, const void* b, void* x, void* V, void* w, void* r,
                       cd64* part, cd64* S, int* st, const int* parent, int m, double tol, int limit, int fixed,
                       unsigned* bar, long long tick_limit, hipStream_t stream) {
  typedef typename BlkTraits<P>::R R;
  auto kern = k_cg_persistent<P, NB>;
  int dev = 0, cus = 0, coop = 0, per_cu = 0;
  WCMG_HIP(hipGetDevice(&dev));
  WCMG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  WCMG_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  WCMG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0));
  const long G = (Vc + kPSpw - 1) / kPSpw;
  if (!coop || per_cu < 1 || G > (long)cus * per_cu || m + 1 > kPMaxM1) return false;
  const Chunk16* bk = (const Chunk16*)blk;
  const cplx<R>* bc = (const cplx<R>*)b;
  cplx<R>* xx = (cplx<R>*)x;
  cplx<R>* vv = (cplx<R>*)V;
  cplx<R>* ww = (cplx<R>*)w;
  cplx<R>* rr = (cplx<R>*)r;
  void* args[] = {(void*)&bk, (void*)&nbr, (void*)&Vc, (void*)&bc, (void*)&xx, (void*)&vv, (void*)&ww, (void*)&rr,
                  (void*)&part, (void*)&S, (void*)&st, (void*)&parent, (void*)&m, (void*)&tol, (void*)&limit,
                  (void*)&fixed, (void*)&bar, (void*)&tick_limit};
  WCMG_HIP(hipLaunchCooperativeKernel((const void*)kern, dim3((unsigned)G), dim3(256), args, 0, stream));
  return true;
}

bool cg_persistent_fits(int prec, int nb, long Vc) {
  if (prec == WCMG_F64 || !(nb == 8 || nb == 12 || nb == 16 || nb == 24 || nb == 32)) return false;
  return Vc >= 1 && Vc <= 2 * 256 * 4;  // refined by the occupancy check at launch
}

bool launch_cg_persistent(int prec, int nb, const void* blk, const int* nbr, long Vc, const void* b, void* x,
                          void* V, void* w, void* r, cd64* part, cd64* S, int* st, const int* parent, int m,
                          double tol, int limit, int fixed, unsigned* bar, double timeout_s, hipStream_t stream) {
  if (!cg_persistent_fits(prec, nb, Vc)) return false;
  int dev = 0, khz = 0;
  WCMG_HIP(hipGetDevice(&dev));
  WCMG_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  const long long tick_limit = (long long)(timeout_s * 1000.0 * (khz > 0 ? khz : 100000));
#define CGP(PP, NBc) \
  return cgp_launch<PP, NBc>(blk, nbr, Vc, b, x, V, w, r, part, S, st, parent, m, tol, limit, fixed, bar, \
                             tick_limit, stream)
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
