// Vector kernels for the Krylov solvers (Sec. 2.1: MR, GMRES, FGMRES).
//
// Reductions are deterministic: a fixed grid of workgroups writes one FP64
// partial per workgroup, and a single workgroup adds the partials in index
// order.  Scalars (inner products, Givens rotations, step lengths) stay in
// device memory; the update kernels read them there, so a solver iteration
// needs no host round trip.  Every kernel takes a `run` flag: when it is 0 the
// kernel returns at once (this is how converged solves skip their remaining,
// already enqueued work).
#include "kernels.h"

namespace wcmg {

constexpr int kRedBlocks = 2048;  // partials per reduction (fixed: results do not depend on timing)

inline int red_blocks(long n) { return (int)std::min<long>(kRedBlocks, std::max<long>(1, (n + 1023) / 1024)); }

__device__ inline cd64 wave_sum(cd64 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.re += __shfl_xor(v.re, off, 64);
    v.im += __shfl_xor(v.im, off, 64);
  }
  return v;
}

// partial[blk][k] = sum over this block's range of conj(a_k[i]) b[i], k < m.
// The a_k are taken KT at a time, so b is read once per tile and KT
// independent loads are in flight per element.
template <typename R>
__global__ void __launch_bounds__(256) k_dot_partial(const cplx<R>* __restrict__ a, long astride, int m,
                                                      const int* __restrict__ m_dev, const cplx<R>* __restrict__ b,
                                                      long n, cd64* __restrict__ partial, int mstride,
                                                      const int* __restrict__ run) {
  if (run && !*run) return;
  if (m_dev) m = *m_dev;
  constexpr int KT = 8;
  __shared__ cd64 lds[4][KT];
  const long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k0 = 0; k0 < m; k0 += KT) {
    cd64 s[KT];
#pragma unroll
    for (int q = 0; q < KT; ++q) s[q] = mkc(0.0, 0.0);
    for (long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const cplx<R> y = b[i];
#pragma unroll
      for (int q = 0; q < KT; ++q)
        if (k0 + q < m) {
          const cplx<R> x = a[(k0 + q) * astride + i];
          s[q].re += (double)x.re * y.re + (double)x.im * y.im;
          s[q].im += (double)x.re * y.im - (double)x.im * y.re;
        }
    }
#pragma unroll
    for (int q = 0; q < KT; ++q) {
      s[q] = wave_sum(s[q]);
      if (lane == 0) lds[wave][q] = s[q];
    }
    __syncthreads();
    if (threadIdx.x < KT && k0 + (int)threadIdx.x < m) {
      cd64 t = mkc(0.0, 0.0);
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = cadd(t, lds[w][threadIdx.x]);
      partial[(long)blockIdx.x * mstride + k0 + threadIdx.x] = t;
    }
    __syncthreads();
  }
}

// out[k * ostride] (op)= sum_g partial[g][k]; mode 0: store, 1: add, 2: subtract.
// One workgroup per k; each lane sums a strided subset of the partials, then a
// fixed-order wave and LDS reduction (deterministic).
__global__ void __launch_bounds__(256) k_dot_finish(const cd64* __restrict__ partial, int G, int m,
                                                     const int* __restrict__ m_dev, int mstride,
                                                     cd64* __restrict__ out, int ostride, int mode,
                                                     const int* __restrict__ run) {
  if (run && !*run) return;
  if (m_dev) m = *m_dev;
  const int k = blockIdx.x;
  if (k >= m) return;
  __shared__ cd64 lds[4];
  cd64 s = mkc(0.0, 0.0);
  s = strided_sum<8>(threadIdx.x, blockDim.x, G, [&](int g) { return partial[(long)g * mstride + k]; });
  s = wave_sum(s);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    cd64 t = mkc(0.0, 0.0);
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = cadd(t, lds[w]);
    cd64* o = out + (long)k * ostride;
    if (mode == 0) *o = t;
    else if (mode == 1) *o = cadd(*o, t);
    else *o = csub(*o, t);
  }
}

// y[i] += sign * sum_{k<m} coef[k * cstride] * V_k[i]
template <typename R>
__global__ void __launch_bounds__(256) k_multi_axpy(cplx<R>* __restrict__ y, const cplx<R>* __restrict__ V,
                                                     long vstride, int m, const int* __restrict__ m_dev,
                                                     const cd64* __restrict__ coef, int cstride, double sign, long n,
                                                     const int* __restrict__ run) {
  if (run && !*run) return;
  if (m_dev) m = *m_dev;
  // grid-stride (the grid may be capped below one thread per element)
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    cplx<R> acc = y[i];
    for (int k = 0; k < m; ++k) {
      cd64 c = coef[(long)k * cstride];
      cplx<R> cc = mkc((R)(sign * c.re), (R)(sign * c.im));
      cfma(acc, cc, V[k * vstride + i]);
    }
    y[i] = acc;
  }
}

// y[i] += sign * sum_{k<m} coef[k] V_k[i], then per-workgroup partials of |y|^2
// (grid-stride over a fixed number of workgroups, so partials are deterministic).
template <typename R>
__global__ void __launch_bounds__(256) k_multi_axpy_norm(cplx<R>* __restrict__ y, const cplx<R>* __restrict__ V,
                                                          long vstride, int m, const cd64* __restrict__ coef,
                                                          int cstride, double sign, long n,
                                                          cd64* __restrict__ partial, const int* __restrict__ run) {
  if (run && !*run) return;
  __shared__ cd64 lds[4];
  const long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  double q = 0.0;
  for (long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    cplx<R> acc = y[i];
    for (int k = 0; k < m; ++k) {
      const cd64 c = coef[(long)k * cstride];
      cfma(acc, mkc((R)(sign * c.re), (R)(sign * c.im)), V[k * vstride + i]);
    }
    y[i] = acc;
    q += (double)acc.re * acc.re + (double)acc.im * acc.im;
  }
  cd64 s = wave_sum(mkc(q, 0.0));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    cd64 t = mkc(0.0, 0.0);
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = cadd(t, lds[w]);
    partial[blockIdx.x] = t;
  }
}

// Single-reduction Arnoldi step, first sweep: y = V_{j+1} - s V_j written
// back (s = *shift; no shift when shift is null), then per-workgroup partials
// of <V_q, y> for q <= j and of |y|^2 (entry j + 1), mstride entries per
// workgroup.  Columns are taken KT at a time; only the first tile forms y.
// Elements are dealt out grid-stride (workgroup b takes blocks b, b + G, ...
// of 256 elements), so the resident workgroups read one contiguous window of
// each vector at a time.
template <typename R>
__global__ void __launch_bounds__(256) k_arnoldi_dots(cplx<R>* __restrict__ V, long n, int j,
                                                       const cd64* __restrict__ shift, cd64* __restrict__ partial,
                                                       int mstride, const int* __restrict__ run) {
  if (run && !*run) return;
  constexpr int KT = 8;
  __shared__ cd64 lds[4][KT];
  const int m = j + 2;
  const long gs = (long)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const R sh = shift ? (R)shift->re : (R)0;
  cplx<R>* yv = V + (long)(j + 1) * n;
  for (int k0 = 0; k0 < m; k0 += KT) {
    cd64 s[KT];
#pragma unroll
    for (int q = 0; q < KT; ++q) s[q] = mkc(0.0, 0.0);
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += gs) {
      // every load of the tile first (vector index clamped to j, so each
      // address is valid and y is taken by value below), then the stores
      cplx<R> y = yv[i];
      cplx<R> xs[KT];
#pragma unroll
      for (int q = 0; q < KT; ++q) {
        const int k = k0 + q;
        xs[q] = V[(long)(k <= j ? k : j) * n + i];
      }
      if (k0 == 0 && shift) {
        const cplx<R> vj = V[(long)j * n + i];
        y = csub(y, cscale(sh, vj));
        yv[i] = y;
      }
#pragma unroll
      for (int q = 0; q < KT; ++q) {
        const int k = k0 + q;
        if (k < m) {
          const cplx<R> x = k == j + 1 ? y : xs[q];
          s[q].re += (double)x.re * y.re + (double)x.im * y.im;
          s[q].im += (double)x.re * y.im - (double)x.im * y.re;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < KT; ++q) {
      s[q] = wave_sum(s[q]);
      if (lane == 0) lds[wave][q] = s[q];
    }
    __syncthreads();
    if (threadIdx.x < KT && k0 + (int)threadIdx.x < m) {
      cd64 t = mkc(0.0, 0.0);
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = cadd(t, lds[w][threadIdx.x]);
      partial[(long)blockIdx.x * mstride + k0 + threadIdx.x] = t;
    }
    __syncthreads();
  }
}

// Single-reduction Arnoldi step, last sweep: y = (y - sum_{k<m} coef[k] V_k)
// / sqrt(*nrm2) (y = 0 when *nrm2 is 0).
template <typename R>
__global__ void __launch_bounds__(256) k_update_scale(cplx<R>* __restrict__ y, const cplx<R>* __restrict__ V,
                                                       long vstride, int m, const cd64* __restrict__ coef,
                                                       const cd64* __restrict__ nrm2, long n,
                                                       const int* __restrict__ run) {
  if (run && !*run) return;
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double q = nrm2->re;
  const R inv = q > 0.0 ? (R)(1.0 / sqrt(q)) : (R)0;
  cplx<R> acc = y[i];
  for (int k = 0; k < m; ++k) {
    const cd64 c = coef[k];
    cfma(acc, mkc((R)-c.re, (R)-c.im), V[k * vstride + i]);
  }
  y[i] = cscale(inv, acc);
}

// y = a * x + b * y with real constants
template <typename R>
__global__ void k_axpby(cplx<R>* __restrict__ y, const cplx<R>* __restrict__ x, R a, R b, long n,
                        const int* __restrict__ run) {
  if (run && !*run) return;
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  cplx<R> v = x[i];
  if (b == (R)0) {
    y[i] = mkc(a * v.re, a * v.im);
  } else {
    cplx<R> w = y[i];
    y[i] = mkc(a * v.re + b * w.re, a * v.im + b * w.im);
  }
}

// y = x * (1 / sqrt(nrm2->re))  (nrm2 holds a squared norm)
template <typename R>
__global__ void k_scale_inv_norm(cplx<R>* __restrict__ y, const cplx<R>* __restrict__ x, const cd64* __restrict__ nrm2,
                                 long n, const int* __restrict__ run) {
  if (run && !*run) return;
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = 1.0 / sqrt(nrm2->re);
  cplx<R> v = x[i];
  y[i] = mkc((R)(s * v.re), (R)(s * v.im));
}

template <typename R>
__global__ void k_zero(cplx<R>* __restrict__ y, long n, const int* __restrict__ run) {
  if (run && !*run) return;
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) y[i] = mkc((R)0, (R)0);
}

// y = a - b
template <typename R>
__global__ void k_sub(cplx<R>* __restrict__ y, const cplx<R>* __restrict__ a, const cplx<R>* __restrict__ b, long n,
                      const int* __restrict__ run) {
  if (run && !*run) return;
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) y[i] = csub(a[i], b[i]);
}

template <typename Ti, typename To>
__global__ void k_convert(const cplx<Ti>* __restrict__ x, cplx<To>* __restrict__ y, long n, const int* __restrict__ run) {
  if (run && !*run) return;
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] = ccast<To>(x[i]);
}

// MR update: dots[0] = <p, r>, dots[1] = <p, p>; alpha = dots0 / dots1;
// x += alpha r; r -= alpha p.
template <typename R>
__global__ void k_mr_update(cplx<R>* __restrict__ x, cplx<R>* __restrict__ r, const cplx<R>* __restrict__ p,
                            const cd64* __restrict__ dots, long n, const int* __restrict__ run) {
  if (run && !*run) return;
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double pp = dots[1].re;
  const cd64 al = pp > 0.0 ? mkc(dots[0].re / pp, dots[0].im / pp) : mkc(0.0, 0.0);
  const cplx<R> a = mkc((R)al.re, (R)al.im);
  cplx<R> xi = x[i], ri = r[i], pi = p[i];
  cfma(xi, a, ri);
  cfma(ri, cneg(a), pi);
  x[i] = xi;
  r[i] = ri;
}

// The MR update with the step length formed from the operator's
// per-workgroup partials (part[2g] = <p, r>_g, part[2g+1] = <p, p>_g, g < G)
// by every workgroup itself, in the order of k_dot_finish (the first 256
// threads: per-thread strided sums, wave sums, waves in order), so all
// workgroups hold the same alpha and it equals the one a separate
// k_dot_finish launch would give.  xout != nullptr: the updated x is written
// there in FP64 (x itself is left as is).  A fixed grid of kMrGrid workgroups
// of kMrBlock threads (one per CU) keeps the partials' reads down; each thread
// updates four elements per pass, and the first pass's operands are loaded
// before the partials are summed, so the two latencies overlap.
constexpr int kMrGrid = 256;
constexpr int kMrBlock = 1024;
template <typename R>
__global__ void __launch_bounds__(kMrBlock) k_mr_update_part(cplx<R>* __restrict__ x, cplx<R>* __restrict__ r,
                                                              const cplx<R>* __restrict__ p,
                                                              const cd64* __restrict__ part, int G, long n,
                                                              const int* __restrict__ run, cd64* __restrict__ xout) {
  if (run && !*run) return;
  __shared__ cd64 lds[2][4];
  const long stride = (long)gridDim.x * blockDim.x;
  long i0 = blockIdx.x * (long)blockDim.x + threadIdx.x;
  cplx<R> xi[4], ri[4], pi[4];
  auto load = [&](long b) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long i = b + u * stride;
      if (i < n) {
        xi[u] = x[i];
        ri[u] = r[i];
        pi[u] = p[i];
      }
    }
  };
  load(i0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x < 256) {
    cd64 s0 = mkc(0.0, 0.0), s1 = mkc(0.0, 0.0);
    // rows threadIdx.x, + 256, ... in order, eight rows' loads in flight at once
    for (int g0 = threadIdx.x; g0 < G; g0 += 8 * 256) {
      cd64 a[8], b[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int g = min(g0 + 256 * u, G - 1);
        a[u] = part[2L * g];
        b[u] = part[2L * g + 1];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (g0 + 256 * u < G) {
          s0 = cadd(s0, a[u]);
          s1 = cadd(s1, b[u]);
        }
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    if (lane == 0) {
      lds[0][wave] = s0;
      lds[1][wave] = s1;
    }
  }
  __syncthreads();
  cd64 t0 = mkc(0.0, 0.0), t1 = mkc(0.0, 0.0);
  for (int w = 0; w < 4; ++w) {
    t0 = cadd(t0, lds[0][w]);
    t1 = cadd(t1, lds[1][w]);
  }
  const double pp = t1.re;
  const cd64 al = pp > 0.0 ? mkc(t0.re / pp, t0.im / pp) : mkc(0.0, 0.0);
  const cplx<R> a = mkc((R)al.re, (R)al.im), na = cneg(a);
  for (; i0 < n; i0 += 4 * stride) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long i = i0 + u * stride;
      if (i < n) {
        cfma(xi[u], a, ri[u]);
        cfma(ri[u], na, pi[u]);
        if (xout) xout[i] = ccast<double>(xi[u]);
        else x[i] = xi[u];
        r[i] = ri[u];
      }
    }
    if (i0 + 4 * stride < n) load(i0 + 4 * stride);
  }
}

// partial[blk][0] = <p, r>, partial[blk][1] = <p, p>
template <typename R>
__global__ void __launch_bounds__(256) k_dot2_partial(const cplx<R>* __restrict__ p, const cplx<R>* __restrict__ r,
                                                       long n, cd64* __restrict__ partial,
                                                       const int* __restrict__ run) {
  if (run && !*run) return;
  __shared__ cd64 lds[8];
  const long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  cd64 s = mkc(0.0, 0.0), q = mkc(0.0, 0.0);
  for (long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    cplx<R> x = p[i], y = r[i];
    s.re += (double)x.re * y.re + (double)x.im * y.im;
    s.im += (double)x.re * y.im - (double)x.im * y.re;
    q.re += (double)x.re * x.re + (double)x.im * x.im;
  }
  s = wave_sum(s);
  q = wave_sum(q);
  if (lane == 0) {
    lds[wave] = s;
    lds[4 + wave] = q;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    cd64 a = mkc(0.0, 0.0), b = mkc(0.0, 0.0);
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      a = cadd(a, lds[w]);
      b = cadd(b, lds[4 + w]);
    }
    partial[blockIdx.x * 2] = a;
    partial[blockIdx.x * 2 + 1] = b;
  }
}

// ---------------------------------------------------------------- GMRES control (single lane)
// State block (int): [0] run, [1] live, [2] jdone, [3] total, [4] reason.
// Scalar block (cd64): H [(m+1) x m], cs [m], sn [m], g [m+1], y [m],
//   then misc: [0] bnorm^2 (re), [1] beta^2 (re), [2] est (re), [3] hn^2 (re).
__global__ void k_gmres_init(int* st, const int* parent) {
  st[1] = parent ? *parent : 1;
  st[0] = st[1];
  st[2] = 0;
  st[3] = 0;
  st[4] = 0;
  st[6] = 0;  // arrival count of k_dot_finish_sr
}

// Start of a restart cycle: beta = ||r||; decide whether to iterate.
__global__ void k_gmres_cycle_start(int* st, cd64* S, int m, double tol, int limit, int fixed) {
  st[0] = 0;
  st[2] = 0;
  if (!st[1]) return;
  cd64* g = S + (m + 1) * m + 2 * m;
  cd64* misc = S + (m + 1) * m + 2 * m + (m + 1) + m;
  const double bn = sqrt(misc[0].re), beta = sqrt(misc[1].re);
  misc[2].re = bn > 0 ? beta / bn : 0.0;
  if (st[3] >= limit || bn == 0.0 || beta == 0.0 || (!fixed && beta <= tol * bn) || !(beta == beta)) {
    st[1] = 0;
    st[4] = !(beta == beta) ? 3 : 1;
    return;
  }
  for (int i = 0; i <= m; ++i) g[i] = mkc(0.0, 0.0);
  g[0] = mkc(beta, 0.0);
  st[0] = 1;
}

// Single-reduction Arnoldi step, bookkeeping (one thread).  stage 0, with d
// the first sweep's j + 2 sums (<v_i, w'> and |w'|^2 for w' = A z_j - s v_j):
// column j of H = d (+ s on the diagonal; at j = 0 there is no shift and s is
// set to Re d_0 for the later steps of the cycle), hn^2 = |w'|^2 - |d|^2, and
// st[5] = 1 (repeat the projection) when that is below |w'|^2 / 4.
// stage 1 (only when st[5]), with d2 the second sweep's sums: column j += d2,
// hn^2 = |w1|^2 - |d2|^2, and d = d2 for the final update.
// Stage 0 of the single-reduction step's bookkeeping (one thread): the
// Hessenberg column from the first projection's sums d, the shift, |w1|^2,
// and whether the projection is repeated (st[5]).
__device__ inline void gmres_sr_stage0(int* st, cd64* S, int m, int j, const cd64* d) {
  cd64* H = S;
  cd64* misc = S + (m + 1) * m + 2 * m + (m + 1) + m;
  st[5] = 0;
  if (!st[0]) return;
  const double n0 = d[j + 1].re;
  double n1 = n0;
  for (int i = 0; i <= j; ++i) {
    H[i * m + j] = d[i];
    n1 -= d[i].re * d[i].re + d[i].im * d[i].im;
  }
  if (j == 0) misc[4] = mkc(d[0].re, 0.0);
  else H[j * m + j].re += misc[4].re;
  misc[3] = mkc(n1 > 0.0 ? n1 : 0.0, 0.0);
  st[5] = n1 < 0.25 * n0 ? 1 : 0;
}

__global__ void k_gmres_sr(int* st, cd64* S, int m, int j, cd64* d, const cd64* d2, int stage) {
  cd64* H = S;
  cd64* misc = S + (m + 1) * m + 2 * m + (m + 1) + m;
  if (stage == 0) {
    gmres_sr_stage0(st, S, m, j, d);
  } else {
    if (!st[0] || !st[5]) return;
    double n2 = d2[j + 1].re;
    for (int i = 0; i <= j; ++i) {
      H[i * m + j] = cadd(H[i * m + j], d2[i]);
      n2 -= d2[i].re * d2[i].re + d2[i].im * d2[i].im;
      d[i] = d2[i];
    }
    misc[3] = mkc(n2 > 0.0 ? n2 : 0.0, 0.0);
  }
}

// k_dot_finish of the first projection's j + 2 sums (one workgroup per sum,
// into d) followed by stage 0 of the step's bookkeeping, run by the last
// workgroup to finish (arrival count in st[6], zeroed by k_gmres_init and by
// that workgroup), so the two need one launch.
__global__ void __launch_bounds__(256) k_dot_finish_sr(const cd64* __restrict__ partial, int G, int j, cd64* d,
                                                        int* st, cd64* S, int m) {
  const int k = blockIdx.x, nk = j + 2;
  if (!st[0]) {
    if (k == 0 && threadIdx.x == 0) st[5] = 0;
    return;
  }
  __shared__ cd64 lds[4];
  __shared__ int last;
  cd64 s = mkc(0.0, 0.0);
  s = strided_sum<8>(threadIdx.x, blockDim.x, G, [&](int g) { return partial[(long)g * nk + k]; });
  s = wave_sum(s);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    cd64 t = mkc(0.0, 0.0);
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = cadd(t, lds[w]);
    d[k] = t;
    __threadfence();  // the sum is visible before the arrival is counted
    last = atomicAdd(st + 6, 1) == nk - 1;
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    __threadfence();  // and the other workgroups' sums are seen after it
    st[6] = 0;
    gmres_sr_stage0(st, S, m, j, d);
  }
}

// Givens update for column j (after H[0..j][j] and hn^2 = misc[3]).
__device__ void gmres_givens_body(int* st, cd64* S, int m, int j, double tol, int limit, int fixed,
                                  int stop_on_estimate) {
  if (!st[0]) return;
  cd64* H = S;
  cd64* cs = S + (m + 1) * m;
  cd64* sn = cs + m;
  cd64* g = sn + m;
  cd64* misc = g + (m + 1) + m;
  const double hn = sqrt(misc[3].re);
  H[(j + 1) * m + j] = mkc(hn, 0.0);
  // the entry rotated down the column stays in a register, so a rotation's
  // loads do not wait for the previous one's stores (the same arithmetic)
  cd64 a = H[j];
  for (int i = 0; i < j; ++i) {
    const cd64 b = H[(i + 1) * m + j], ci = cs[i], si = sn[i];
    cd64 t = cmul(ci, a);
    cfma(t, si, b);
    cd64 u = cmul(cneg(cconj(si)), a);
    cfma(u, cconj(ci), b);
    H[i * m + j] = t;
    a = u;
  }
  const double den = sqrt(a.re * a.re + a.im * a.im + hn * hn);
  cd64 c = den == 0.0 ? mkc(1.0, 0.0) : mkc(a.re / den, -a.im / den);  // conj(a)/den
  cd64 s = den == 0.0 ? mkc(0.0, 0.0) : mkc(hn / den, 0.0);
  cs[j] = c;
  sn[j] = s;
  H[j * m + j] = mkc(den, 0.0);
  H[(j + 1) * m + j] = mkc(0.0, 0.0);
  // den == 0: A z_j adds nothing (a singular Hessenberg column); the column is
  // dropped from the least-squares solve and the residual stays |g_j|
  const cd64 gj = g[j];
  g[j + 1] = den == 0.0 ? gj : cmul(cneg(cconj(s)), gj);
  g[j] = cmul(c, gj);
  st[2] = den == 0.0 ? j : j + 1;
  st[3] += 1;
  const double bn = sqrt(misc[0].re);
  const double est = bn > 0 ? sqrt(g[j + 1].re * g[j + 1].re + g[j + 1].im * g[j + 1].im) / bn : 0.0;
  misc[2].re = est;
  bool stop = false;
  if (st[3] >= limit) {
    stop = true;
    st[1] = 0;
    st[4] = 2;
  }
  if (!fixed && est <= tol) {
    stop = true;
    if (stop_on_estimate) {
      st[1] = 0;
      st[4] = 1;
    }
  }
  if (hn == 0.0 || !(est == est)) {
    stop = true;
    st[1] = 0;
    st[4] = (est == est) ? (den == 0.0 ? 4 : 1) : 3;
  }
  if (stop || j + 1 == m) st[0] = 0;
}
__global__ void k_gmres_givens(int* st, cd64* S, int m, int j, double tol, int limit, int fixed,
                               int stop_on_estimate) {
  gmres_givens_body(st, S, m, j, tol, limit, fixed, stop_on_estimate);
}

// The end of a single-reduction Arnoldi step in one workgroup: when the
// second projection ran (st[5]), its G2 per-workgroup partials (mstride =
// j + 2 entries each) are summed in k_dot_finish's order, then the stage-1
// bookkeeping of k_gmres_sr, then the Givens update of column j.  d2: j + 2
// entries of scratch for the sums (written and read by thread 0 only).
__device__ inline void gmres_sr_finish_body(int* st, cd64* S, int m, int j, cd64* d, cd64* d2,
                                            const cd64* __restrict__ part2, int G2, double tol, int limit,
                                            int fixed, int stop_on_estimate) {
  __shared__ cd64 lds[4];
  if (!st[0]) return;
  const bool reorth = st[5] != 0;  // the same value in every thread
  if (reorth) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < j + 2; ++k) {
      cd64 v = mkc(0.0, 0.0);
      for (int g = threadIdx.x; g < G2; g += blockDim.x) v = cadd(v, part2[(long)g * (j + 2) + k]);
      v = wave_sum(v);
      if (lane == 0) lds[wave] = v;
      __syncthreads();
      if (threadIdx.x == 0) {
        cd64 t = mkc(0.0, 0.0);
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = cadd(t, lds[w]);
        d2[k] = t;
      }
      __syncthreads();
    }
  }
  if (threadIdx.x != 0) return;
  if (reorth) {
    cd64* H = S;
    cd64* misc = S + (m + 1) * m + 2 * m + (m + 1) + m;
    double n2 = d2[j + 1].re;
    for (int i = 0; i <= j; ++i) {
      H[i * m + j] = cadd(H[i * m + j], d2[i]);
      n2 -= d2[i].re * d2[i].re + d2[i].im * d2[i].im;
      d[i] = d2[i];
    }
    misc[3] = mkc(n2 > 0.0 ? n2 : 0.0, 0.0);
  }
  gmres_givens_body(st, S, m, j, tol, limit, fixed, stop_on_estimate);
}

// Copies n state words to out[1..n] (host-mapped memory), then writes the
// publication number to out[0] (one thread).
__device__ inline void publish_words(const int* st, int n, int* out, int seq) {
  for (int i = 0; i < n; ++i) __hip_atomic_store(out + 1 + i, st[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __threadfence_system();
  __hip_atomic_store(out, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// pub != nullptr: afterwards st[0..pub_n) is published as k_publish_state
// would (publication pub_seq), in the same launch.
__global__ void __launch_bounds__(256) k_gmres_sr_finish(int* st, cd64* S, int m, int j, cd64* d, cd64* d2,
                                                          const cd64* __restrict__ part2, int G2, double tol,
                                                          int limit, int fixed, int stop_on_estimate, int* pub,
                                                          int pub_seq, int pub_n) {
  gmres_sr_finish_body(st, S, m, j, d, d2, part2, G2, tol, limit, fixed, stop_on_estimate);
  if (pub && threadIdx.x == 0) publish_words(st, pub_n, pub, pub_seq);
}
void launch_gmres_sr_finish(int* st_, cd64* S, int m, int j, cd64* d, cd64* d2, const cd64* part2, int G2,
                            double tol, int limit, int fixed, int stop_on_est, hipStream_t st, int* pub, int pub_seq,
                            int pub_n) {
  hipLaunchKernelGGL(k_gmres_sr_finish, dim3(1), dim3(kBlock), 0, st, st_, S, m, j, d, d2, part2, G2, tol, limit,
                     fixed, stop_on_est, pub, pub_seq, pub_n);
  WCMG_CHECK_LAUNCH();
}

// Back substitution H y = g on the leading jdone x jdone triangle.
__global__ void k_gmres_solve_y(const int* st, cd64* S, int m) {
  const int jd = st[2];
  if (jd == 0) return;
  cd64* H = S;
  cd64* g = S + (m + 1) * m + 2 * m;
  cd64* y = g + (m + 1);
  for (int i = jd - 1; i >= 0; --i) {
    cd64 s = g[i];
    for (int k = i + 1; k < jd; ++k) {
      cd64 t = cmul(H[i * m + k], y[k]);
      s = csub(s, t);
    }
    const cd64 d = H[i * m + i];
    const double dd = d.re * d.re + d.im * d.im;
    y[i] = dd > 0.0 ? mkc((s.re * d.re + s.im * d.im) / dd, (s.im * d.re - s.re * d.im) / dd) : mkc(0.0, 0.0);
  }
}

__global__ void k_gmres_cycle_end(int* st) {
  st[2] = 0;
  st[0] = 0;
}

// ---------------------------------------------------------------- launchers
template <typename R>
void launch_dot(const cplx<R>* a, long astride, int m, const int* m_dev, const cplx<R>* b, long n, cd64* partial,
                int mstride, cd64* out, int ostride, int mode, const int* run, hipStream_t st) {
  int G = red_blocks(n);
  hipLaunchKernelGGL(k_dot_partial<R>, dim3(G), dim3(kBlock), 0, st, a, astride, m, m_dev, b, n, partial, mstride, run);
  WCMG_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_dot_finish, dim3(m), dim3(kBlock), 0, st, partial, G, m, m_dev, mstride, out, ostride, mode, run);
  WCMG_CHECK_LAUNCH();
}

int reduction_blocks(long n) { return red_blocks(n); }

template <typename R>
void launch_multi_axpy_norm(cplx<R>* y, const cplx<R>* V, long vstride, int m, const cd64* coef, int cstride,
                            double sign, long n, cd64* partial, const int* run, hipStream_t st) {
  hipLaunchKernelGGL(k_multi_axpy_norm<R>, dim3(red_blocks(n)), dim3(kBlock), 0, st, y, V, vstride, m, coef, cstride,
                     sign, n, partial, run);
  WCMG_CHECK_LAUNCH();
}
template void launch_multi_axpy_norm<double>(cd64*, const cd64*, long, int, const cd64*, int, double, long, cd64*,
                                             const int*, hipStream_t);
template void launch_multi_axpy_norm<float>(cf32*, const cf32*, long, int, const cd64*, int, double, long, cd64*,
                                            const int*, hipStream_t);



void launch_dot_finish(const cd64* partial, int G, int m, int mstride, cd64* out, int ostride, int mode,
                       const int* run, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_finish, dim3(m), dim3(kBlock), 0, st, partial, G, m, (const int*)nullptr, mstride, out,
                     ostride, mode, run);
  WCMG_CHECK_LAUNCH();
}

template <typename R>
void launch_multi_axpy(cplx<R>* y, const cplx<R>* V, long vstride, int m, const int* m_dev, const cd64* coef,
                       int cstride, double sign, long n, const int* run, hipStream_t st, int grid) {
  const long g = nblocks(n);
  hipLaunchKernelGGL(k_multi_axpy<R>, dim3((unsigned)(grid > 0 && grid < g ? grid : g)), dim3(kBlock), 0, st, y, V,
                     vstride, m, m_dev, coef, cstride, sign, n, run);
  WCMG_CHECK_LAUNCH();
}

template <typename R>
void launch_axpby(cplx<R>* y, const cplx<R>* x, double a, double b, long n, const int* run, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby<R>, dim3(nblocks(n)), dim3(kBlock), 0, st, y, x, (R)a, (R)b, n, run);
  WCMG_CHECK_LAUNCH();
}

template <typename R>
void launch_scale_inv_norm(cplx<R>* y, const cplx<R>* x, const cd64* nrm2, long n, const int* run, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_inv_norm<R>, dim3(nblocks(n)), dim3(kBlock), 0, st, y, x, nrm2, n, run);
  WCMG_CHECK_LAUNCH();
}

template <typename R>
void launch_zero(cplx<R>* y, long n, const int* run, hipStream_t st) {
  hipLaunchKernelGGL(k_zero<R>, dim3(nblocks(n)), dim3(kBlock), 0, st, y, n, run);
  WCMG_CHECK_LAUNCH();
}
template <typename R>
void launch_sub(cplx<R>* y, const cplx<R>* a, const cplx<R>* b, long n, const int* run, hipStream_t st) {
  hipLaunchKernelGGL(k_sub<R>, dim3(nblocks(n)), dim3(kBlock), 0, st, y, a, b, n, run);
  WCMG_CHECK_LAUNCH();
}

template <typename Ti, typename To>
void launch_convert(const cplx<Ti>* x, cplx<To>* y, long n, const int* run, hipStream_t st) {
  hipLaunchKernelGGL((k_convert<Ti, To>), dim3(nblocks(n)), dim3(kBlock), 0, st, x, y, n, run);
  WCMG_CHECK_LAUNCH();
}

template <typename R>
void launch_mr_update(cplx<R>* x, cplx<R>* r, const cplx<R>* p, const cd64* dots, long n, const int* run,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_mr_update<R>, dim3(nblocks(n)), dim3(kBlock), 0, st, x, r, p, dots, n, run);
  WCMG_CHECK_LAUNCH();
}

template <typename R>
void launch_mr_update_part(cplx<R>* x, cplx<R>* r, const cplx<R>* p, const cd64* part, int G, long n, const int* run,
                           hipStream_t st, cd64* xout) {
  hipLaunchKernelGGL(k_mr_update_part<R>, dim3((unsigned)std::min<long>(kMrGrid, nblocks(n, kMrBlock))), dim3(kMrBlock), 0, st, x,
                     r, p, part, G, n, run, xout);
  WCMG_CHECK_LAUNCH();
}

template <typename R>
void launch_mr_dots_update(cplx<R>* x, cplx<R>* r, const cplx<R>* p, long n, cd64* partial, cd64* dots,
                           const int* run, hipStream_t st) {
  int G = red_blocks(n);
  hipLaunchKernelGGL(k_dot2_partial<R>, dim3(G), dim3(kBlock), 0, st, p, r, n, partial, run);
  WCMG_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_dot_finish, dim3(2), dim3(kBlock), 0, st, partial, G, 2, (const int*)nullptr, 2, dots, 1, 0, run);
  WCMG_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_mr_update<R>, dim3(nblocks(n)), dim3(kBlock), 0, st, x, r, p, dots, n, run);
  WCMG_CHECK_LAUNCH();
}

#define INST_BLAS(R)                                                                                                \
  template void launch_dot<R>(const cplx<R>*, long, int, const int*, const cplx<R>*, long, cd64*, int, cd64*, int,   \
                              int, const int*, hipStream_t);                                                        \
  template void launch_multi_axpy<R>(cplx<R>*, const cplx<R>*, long, int, const int*, const cd64*, int, double, long, \
                                     const int*, hipStream_t, int);                                                 \
  template void launch_axpby<R>(cplx<R>*, const cplx<R>*, double, double, long, const int*, hipStream_t);            \
  template void launch_zero<R>(cplx<R>*, long, const int*, hipStream_t);                                             \
  template void launch_sub<R>(cplx<R>*, const cplx<R>*, const cplx<R>*, long, const int*, hipStream_t);              \
  template void launch_scale_inv_norm<R>(cplx<R>*, const cplx<R>*, const cd64*, long, const int*, hipStream_t);      \
  template void launch_mr_update<R>(cplx<R>*, cplx<R>*, const cplx<R>*, const cd64*, long, const int*, hipStream_t); \
  template void launch_mr_update_part<R>(cplx<R>*, cplx<R>*, const cplx<R>*, const cd64*, int, long, const int*,      \
                                         hipStream_t, cd64*);                                                       \
  template void launch_mr_dots_update<R>(cplx<R>*, cplx<R>*, const cplx<R>*, long, cd64*, cd64*, const int*,         \
                                         hipStream_t);
INST_BLAS(double)
INST_BLAS(float)
template void launch_convert<double, float>(const cd64*, cf32*, long, const int*, hipStream_t);
template void launch_convert<float, double>(const cf32*, cd64*, long, const int*, hipStream_t);
template void launch_convert<double, double>(const cd64*, cd64*, long, const int*, hipStream_t);
template void launch_convert<float, float>(const cf32*, cf32*, long, const int*, hipStream_t);

void launch_gmres_init(int* st_, const int* parent, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_init, dim3(1), dim3(1), 0, st, st_, parent);
  WCMG_CHECK_LAUNCH();
}
void launch_gmres_cycle_start(int* st_, cd64* S, int m, double tol, int limit, int fixed, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_cycle_start, dim3(1), dim3(1), 0, st, st_, S, m, tol, limit, fixed);
  WCMG_CHECK_LAUNCH();
}
void launch_gmres_givens(int* st_, cd64* S, int m, int j, double tol, int limit, int fixed, int stop_on_est,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_givens, dim3(1), dim3(1), 0, st, st_, S, m, j, tol, limit, fixed, stop_on_est);
  WCMG_CHECK_LAUNCH();
}
void launch_dot_finish_sr(const cd64* partial, int G, int j, cd64* d, int* st_, cd64* S, int m, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_finish_sr, dim3(j + 2), dim3(kBlock), 0, st, partial, G, j, d, st_, S, m);
  WCMG_CHECK_LAUNCH();
}
void launch_gmres_sr(int* st_, cd64* S, int m, int j, cd64* d, const cd64* d2, int stage, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_sr, dim3(1), dim3(1), 0, st, st_, S, m, j, d, d2, stage);
  WCMG_CHECK_LAUNCH();
}
template <typename R>
void launch_arnoldi_dots(cplx<R>* V, long n, int j, const cd64* shift, cd64* partial, int mstride, const int* run,
                         hipStream_t st, int grid) {
  hipLaunchKernelGGL(k_arnoldi_dots<R>, dim3(grid > 0 ? grid : red_blocks(n)), dim3(kBlock), 0, st, V, n, j, shift,
                     partial, mstride, run);
  WCMG_CHECK_LAUNCH();
}
template <typename R>
void launch_update_scale(cplx<R>* y, const cplx<R>* V, long vstride, int m, const cd64* coef, const cd64* nrm2,
                         long n, const int* run, hipStream_t st) {
  hipLaunchKernelGGL(k_update_scale<R>, dim3(nblocks(n)), dim3(kBlock), 0, st, y, V, vstride, m, coef, nrm2, n, run);
  WCMG_CHECK_LAUNCH();
}
template void launch_arnoldi_dots<double>(cd64*, long, int, const cd64*, cd64*, int, const int*, hipStream_t, int);
template void launch_arnoldi_dots<float>(cf32*, long, int, const cd64*, cd64*, int, const int*, hipStream_t, int);
template void launch_update_scale<double>(cd64*, const cd64*, long, int, const cd64*, const cd64*, long, const int*,
                                          hipStream_t);
template void launch_update_scale<float>(cf32*, const cf32*, long, int, const cd64*, const cd64*, long, const int*,
                                         hipStream_t);
void launch_gmres_solve_y(const int* st_, cd64* S, int m, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_solve_y, dim3(1), dim3(1), 0, st, st_, S, m);
  WCMG_CHECK_LAUNCH();
}
void launch_gmres_cycle_end(int* st_, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_cycle_end, dim3(1), dim3(1), 0, st, st_);
  WCMG_CHECK_LAUNCH();
}

// Copies n state words to host-mapped memory (out[1..n]) and then writes the
// publication number to out[0]: a host that reads the number reads the words
// of that publication.
__global__ void __launch_bounds__(64) k_publish_state(const int* __restrict__ st, int n, int* out, int seq) {
  for (int i = threadIdx.x; i < n; i += 64) __hip_atomic_store(out + 1 + i, st[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(out, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
void launch_publish_state(const int* st_, int n, int* out, int seq, hipStream_t st) {
  hipLaunchKernelGGL(k_publish_state, dim3(1), dim3(64), 0, st, st_, n, out, seq);
  WCMG_CHECK_LAUNCH();
}

}  // namespace wcmg
