// Batched vector kernels: B independent Krylov solves (one per right-hand
// side) advancing through shared launches.  Fields are right-hand-side major
// (field r at base + r * rstride); every solve has its own state words, scalars
// and `run` flag (run[r * rs]), so a converged right-hand side drops out while
// the others continue.  blockIdx.y is the right-hand side.  Reductions are
// deterministic (fixed partition, fixed-order sums), as in blas.hip.
#include "kernels.h"

namespace wcmg {

namespace {
constexpr int kRed = 512;
inline int red_b(long n) { return (int)std::min<long>(kRed, std::max<long>(1, (n + 1023) / 1024)); }

__device__ inline cd64 wsum2(cd64 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.re += __shfl_xor(v.re, off, 64);
    v.im += __shfl_xor(v.im, off, 64);
  }
  return v;
}
__device__ inline bool live_r(const int* run, int rs, int r) { return !run || run[(long)r * rs]; }
}  // namespace

// partial[r][blk][k] = sum conj(a_{r,k}[i]) b_r[i] over this block's range, k < m;
// the a_k are taken KT at a time (b read once per tile, KT loads in flight).
template <typename R>
__global__ void __launch_bounds__(256) k_bdot_partial(const cplx<R>* __restrict__ a, long avs, long ars, int m,
                                                       const cplx<R>* __restrict__ b, long brs, long n,
                                                       cd64* __restrict__ partial, int mstride,
                                                       const int* __restrict__ run, int rs) {
  const int r = blockIdx.y;
  if (!live_r(run, rs, r)) return;
  constexpr int KT = 8;
  __shared__ cd64 lds[4][KT];
  a += r * ars;
  b += r * brs;
  partial += (long)r * gridDim.x * mstride;
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
          const cplx<R> x = a[(k0 + q) * avs + i];
          s[q].re += (double)x.re * y.re + (double)x.im * y.im;
          s[q].im += (double)x.re * y.im - (double)x.im * y.re;
        }
    }
#pragma unroll
    for (int q = 0; q < KT; ++q) {
      s[q] = wsum2(s[q]);
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

// Single-reduction Arnoldi step, first sweep, per right-hand side:
// y_r = V_{r,j+1} - s_r V_{r,j} written back (s_r = shift[r * shs]; no shift
// when shift is null), then partial[r][blk][k] = <V_{r,k}, y_r> for k <= j
// and |y_r|^2 at k = j + 1.  Only the first tile of columns forms y.
template <typename R>
__global__ void __launch_bounds__(256) k_barnoldi_dots(cplx<R>* __restrict__ V, long vvs, long vrs, int j, long n,
                                                        const cd64* __restrict__ shift, long shs,
                                                        cd64* __restrict__ partial, int mstride,
                                                        const int* __restrict__ run, int rs) {
  const int r = blockIdx.y;
  if (!live_r(run, rs, r)) return;
  constexpr int KT = 8;
  __shared__ cd64 lds[4][KT];
  const int m = j + 2;
  V += r * vrs;
  partial += (long)r * gridDim.x * mstride;
  const R sh = shift ? (R)shift[r * shs].re : (R)0;
  cplx<R>* yv = V + (long)(j + 1) * vvs;
  const long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k0 = 0; k0 < m; k0 += KT) {
    cd64 s[KT];
#pragma unroll
    for (int q = 0; q < KT; ++q) s[q] = mkc(0.0, 0.0);
    for (long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      // every load of the tile first (vector index clamped to j, so each
      // address is valid and y is taken by value below), then the stores
      cplx<R> y = yv[i];
      cplx<R> xs[KT];
#pragma unroll
      for (int q = 0; q < KT; ++q) {
        const int k = k0 + q;
        xs[q] = V[(long)(k <= j ? k : j) * vvs + i];
      }
      if (k0 == 0 && shift) {
        const cplx<R> vj = V[(long)j * vvs + i];
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
      s[q] = wsum2(s[q]);
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

// Single-reduction Arnoldi step, last sweep, per right-hand side:
// y_r = (y_r - sum_{k<m} coef_r[k] V_{r,k}) / sqrt(nrm2_r) (0 when nrm2_r is 0).
template <typename R>
__global__ void __launch_bounds__(256) k_bupdate_scale(cplx<R>* __restrict__ y, long yrs,
                                                        const cplx<R>* __restrict__ V, long vvs, long vrs, int m,
                                                        const cd64* __restrict__ coef, long crs,
                                                        const cd64* __restrict__ nrm2, long nrs, long n,
                                                        const int* __restrict__ run, int rs) {
  const int r = blockIdx.y;
  if (!live_r(run, rs, r)) return;
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  y += r * yrs;
  V += r * vrs;
  coef += r * crs;
  const double q = nrm2[r * nrs].re;
  const R inv = q > 0.0 ? (R)(1.0 / sqrt(q)) : (R)0;
  cplx<R> acc = y[i];
  for (int k = 0; k < m; ++k) {
    const cd64 c = coef[k];
    cfma(acc, mkc((R)-c.re, (R)-c.im), V[(long)k * vvs + i]);
  }
  y[i] = cscale(inv, acc);
}

// Second half of a Gram-Schmidt pass in one sweep over the basis:
//   y_r -= sum_{k<m} coef_r[k] V_{r,k}, then partial[r][blk][k] = <V_{r,k}, y_r> of
// the updated y.  Each element's m basis entries stay in registers between the
// update and the inner products (m <= kFusedMaxM).
template <typename R>
__global__ void __launch_bounds__(256) k_bmulti_axpy_dot(cplx<R>* __restrict__ y, long yrs,
                                                          const cplx<R>* __restrict__ V, long vvs, long vrs, int m,
                                                          const cd64* __restrict__ coef, int cks, long crs, long n,
                                                          cd64* __restrict__ partial, int mstride,
                                                          const int* __restrict__ run, int rs) {
  constexpr int MM = kFusedMaxM;
  const int r = blockIdx.y;
  if (!live_r(run, rs, r)) return;
  __shared__ cd64 lds[4][MM];
  y += r * yrs;
  V += r * vrs;
  coef += r * crs;
  partial += (long)r * gridDim.x * mstride;
  cplx<R> c[MM];
#pragma unroll
  for (int k = 0; k < MM; ++k) {
    const cd64 v = k < m ? coef[(long)k * cks] : mkc(0.0, 0.0);
    c[k] = mkc((R)-v.re, (R)-v.im);
  }
  cd64 s[MM];
#pragma unroll
  for (int k = 0; k < MM; ++k) s[k] = mkc(0.0, 0.0);
  const long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  for (long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    cplx<R> v[MM];
#pragma unroll
    for (int k = 0; k < MM; ++k)
      if (k < m) v[k] = V[k * vvs + i];
    cplx<R> acc = y[i];
#pragma unroll
    for (int k = 0; k < MM; ++k)
      if (k < m) cfma(acc, c[k], v[k]);
    y[i] = acc;
#pragma unroll
    for (int k = 0; k < MM; ++k)
      if (k < m) {
        s[k].re += (double)v[k].re * acc.re + (double)v[k].im * acc.im;
        s[k].im += (double)v[k].re * acc.im - (double)v[k].im * acc.re;
      }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < MM; ++k)
    if (k < m) {
      s[k] = wsum2(s[k]);
      if (lane == 0) lds[wave][k] = s[k];
    }
  __syncthreads();
  if ((int)threadIdx.x < m) {
    cd64 t = mkc(0.0, 0.0);
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = cadd(t, lds[w][threadIdx.x]);
    partial[(long)blockIdx.x * mstride + threadIdx.x] = t;
  }
}

// out[r][k] (op)= sum_g partial[r][g][k]; grid (m, B); mode 0 store, 1 add
__global__ void __launch_bounds__(256) k_bdot_finish(const cd64* __restrict__ partial, int G, int m, int mstride,
                                                      cd64* __restrict__ out, int ostride, long ors, int mode,
                                                      const int* __restrict__ run, int rs) {
  const int r = blockIdx.y, k = blockIdx.x;
  if (!live_r(run, rs, r) || k >= m) return;
  __shared__ cd64 lds[4];
  partial += (long)r * G * mstride;
  cd64 s = mkc(0.0, 0.0);
  s = strided_sum<8>(threadIdx.x, blockDim.x, G, [&](int g) { return partial[(long)g * mstride + k]; });
  s = wsum2(s);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    cd64 t = mkc(0.0, 0.0);
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = cadd(t, lds[w]);
    cd64* o = out + r * ors + (long)k * ostride;
    *o = mode == 0 ? t : cadd(*o, t);
  }
}

// y_r += sign * sum_{k < m_r} coef_r[k] V_{r,k}; m_r = m_dev ? m_dev[r * ms] : m.
// With norm_part: per-block partials of |y_r|^2 (grid-stride, fixed partition).
template <typename R>
__global__ void __launch_bounds__(256) k_bmulti_axpy(cplx<R>* __restrict__ y, long yrs, const cplx<R>* __restrict__ V,
                                                      long vvs, long vrs, int m, const int* __restrict__ m_dev, int ms,
                                                      const cd64* __restrict__ coef, int cks, long crs, double sign,
                                                      long n, cd64* __restrict__ norm_part,
                                                      const int* __restrict__ run, int rs) {
  const int r = blockIdx.y;
  if (!live_r(run, rs, r)) return;
  if (m_dev) m = m_dev[(long)r * ms];
  y += r * yrs;
  V += r * vrs;
  coef += r * crs;
  __shared__ cd64 lds[4];
  double q = 0.0;
  if (norm_part) {
    const long chunk = (n + gridDim.x - 1) / gridDim.x;
    const long lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    for (long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      cplx<R> acc = y[i];
      for (int k = 0; k < m; ++k) {
        const cd64 c = coef[(long)k * cks];
        cfma(acc, mkc((R)(sign * c.re), (R)(sign * c.im)), V[k * vvs + i]);
      }
      y[i] = acc;
      q += (double)acc.re * acc.re + (double)acc.im * acc.im;
    }
    cd64 s = wsum2(mkc(q, 0.0));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) lds[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      cd64 t = mkc(0.0, 0.0);
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = cadd(t, lds[w]);
      norm_part[(long)r * gridDim.x + blockIdx.x] = t;
    }
    return;
  }
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    cplx<R> acc = y[i];
    for (int k = 0; k < m; ++k) {
      const cd64 c = coef[(long)k * cks];
      cfma(acc, mkc((R)(sign * c.re), (R)(sign * c.im)), V[k * vvs + i]);
    }
    y[i] = acc;
  }
}

// elementwise on B fields: op 0 y = 0, 1 y = x, 2 y = x - z, 3 y = x / sqrt(nrm2_r), 4 y = -x
template <typename Ti, typename To>
__global__ void __launch_bounds__(256) k_belem(To* __restrict__ y, long yrs, const Ti* __restrict__ x, long xrs,
                                                const Ti* __restrict__ z, long zrs, const cd64* __restrict__ nrm2,
                                                long nrs, long n, int op, const int* __restrict__ run, int rs) {
  const int r = blockIdx.y;
  if (!live_r(run, rs, r)) return;
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  y += r * yrs;
  typedef decltype(To::re) RO;
  if (op == 0) {
    y[i] = mkc((RO)0, (RO)0);
    return;
  }
  const Ti v = x[r * xrs + i];
  if (op == 1) y[i] = mkc((RO)v.re, (RO)v.im);
  else if (op == 2) {
    const Ti w = z[r * zrs + i];
    y[i] = mkc((RO)(v.re - w.re), (RO)(v.im - w.im));
  } else if (op == 3) {
    const double s = 1.0 / sqrt(nrm2[r * nrs].re);
    y[i] = mkc((RO)(s * v.re), (RO)(s * v.im));
  } else {
    y[i] = mkc((RO)-v.re, (RO)-v.im);
  }
}

// MR update per right-hand side: alpha_r = dots_r[0] / dots_r[1]
template <typename R>
__global__ void __launch_bounds__(256) k_bmr_update(cplx<R>* __restrict__ x, cplx<R>* __restrict__ r_,
                                                     const cplx<R>* __restrict__ p, long rsf,
                                                     const cd64* __restrict__ dots, long n,
                                                     const int* __restrict__ run, int rs) {
  const int r = blockIdx.y;
  if (!live_r(run, rs, r)) return;
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const cd64* d = dots + 2 * r;
  const double pp = d[1].re;
  const cd64 al = pp > 0.0 ? mkc(d[0].re / pp, d[0].im / pp) : mkc(0.0, 0.0);
  const cplx<R> a = mkc((R)al.re, (R)al.im);
  x += r * rsf;
  r_ += r * rsf;
  p += r * rsf;
  cplx<R> xi = x[i], ri = r_[i], pi = p[i];
  cfma(xi, a, ri);
  cfma(ri, cneg(a), pi);
  x[i] = xi;
  r_[i] = ri;
}

// ---- batched GMRES control: thread r of one workgroup owns solve r.
// State (int, stride 8): [0] run, [1] live, [2] jdone, [3] total, [4] reason.
// Scalars (cd64, stride ss): H, cs, sn, g, y, misc as in blas.hip.
__global__ void k_bgmres_init(int* st, int B, const int* parent, int prs) {
  const int r = threadIdx.x;
  if (r >= B) return;
  int* s = st + 8 * r;
  s[1] = parent ? parent[(long)r * prs] : 1;
  s[0] = s[1];
  s[2] = s[3] = s[4] = 0;
}

__global__ void k_bgmres_cycle_start(int* st, cd64* S, long ss, int B, int m, double tol, int limit, int fixed) {
  const int r = threadIdx.x;
  if (r >= B) return;
  int* s = st + 8 * r;
  cd64* Sr = S + r * ss;
  s[0] = 0;
  s[2] = 0;
  if (!s[1]) return;
  cd64* g = Sr + (m + 1) * m + 2 * m;
  cd64* misc = g + (m + 1) + m;
  const double bn = sqrt(misc[0].re), beta = sqrt(misc[1].re);
  misc[2].re = bn > 0 ? beta / bn : 0.0;
  if (s[3] >= limit || bn == 0.0 || beta == 0.0 || (!fixed && beta <= tol * bn) || !(beta == beta)) {
    s[1] = 0;
    s[4] = !(beta == beta) ? 3 : 1;
    return;
  }
  for (int i = 0; i <= m; ++i) g[i] = mkc(0.0, 0.0);
  g[0] = mkc(beta, 0.0);
  s[0] = 1;
}

// Single-reduction Arnoldi step, bookkeeping, one thread per right-hand side
// (the batched form of k_gmres_sr): stage 0 takes the first sweep's sums d_r
// (column j of H, the shift, hn^2 = |w'|^2 - |d|^2, st[5] = repeat the
// projection); stage 1, where st[5], adds the second sweep's sums d2_r.
__global__ void k_bgmres_sr(int* st, cd64* S, long ss, int B, int m, int j, cd64* d, cd64* d2, int stage) {
  const int r = threadIdx.x;
  if (r >= B) return;
  int* s = st + 8 * r;
  cd64* H = S + r * ss;
  cd64* misc = H + (m + 1) * m + 2 * m + (m + 1) + m;
  cd64* dr = d + r * ss;
  const cd64* d2r = d2 + r * ss;
  if (stage == 0) {
    s[5] = 0;
    if (!s[0]) return;
    const double n0 = dr[j + 1].re;
    double n1 = n0;
    for (int i = 0; i <= j; ++i) {
      H[i * m + j] = dr[i];
      n1 -= dr[i].re * dr[i].re + dr[i].im * dr[i].im;
    }
    if (j == 0) misc[4] = mkc(dr[0].re, 0.0);
    else H[j * m + j].re += misc[4].re;
    misc[3] = mkc(n1 > 0.0 ? n1 : 0.0, 0.0);
    s[5] = n1 < 0.25 * n0 ? 1 : 0;
  } else {
    if (!s[0] || !s[5]) return;
    double n2 = d2r[j + 1].re;
    for (int i = 0; i <= j; ++i) {
      H[i * m + j] = cadd(H[i * m + j], d2r[i]);
      n2 -= d2r[i].re * d2r[i].re + d2r[i].im * d2r[i].im;
      dr[i] = d2r[i];
    }
    misc[3] = mkc(n2 > 0.0 ? n2 : 0.0, 0.0);
  }
}

__global__ void k_bgmres_givens(int* st, cd64* S, long ss, int B, int m, int j, double tol, int limit, int fixed,
                                int stop_on_est) {
  const int r = threadIdx.x;
  if (r >= B) return;
  int* s = st + 8 * r;
  if (!s[0]) return;
  cd64* H = S + r * ss;
  cd64* cs = H + (m + 1) * m;
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
  const cd64 c = den == 0.0 ? mkc(1.0, 0.0) : mkc(a.re / den, -a.im / den);
  const cd64 sv = den == 0.0 ? mkc(0.0, 0.0) : mkc(hn / den, 0.0);
  cs[j] = c;
  sn[j] = sv;
  H[j * m + j] = mkc(den, 0.0);
  H[(j + 1) * m + j] = mkc(0.0, 0.0);
  const cd64 gj = g[j];
  g[j + 1] = den == 0.0 ? gj : cmul(cneg(cconj(sv)), gj);  // den == 0: singular column, dropped
  g[j] = cmul(c, gj);
  s[2] = den == 0.0 ? j : j + 1;
  s[3] += 1;
  const double bn = sqrt(misc[0].re);
  const double est = bn > 0 ? sqrt(g[j + 1].re * g[j + 1].re + g[j + 1].im * g[j + 1].im) / bn : 0.0;
  misc[2].re = est;
  bool stop = false;
  if (s[3] >= limit) {
    stop = true;
    s[1] = 0;
    s[4] = 2;
  }
  if (!fixed && est <= tol) {
    stop = true;
    if (stop_on_est) {
      s[1] = 0;
      s[4] = 1;
    }
  }
  if (hn == 0.0 || !(est == est)) {
    stop = true;
    s[1] = 0;
    s[4] = (est == est) ? (den == 0.0 ? 4 : 1) : 3;
  }
  if (stop || j + 1 == m) s[0] = 0;
}

__global__ void k_bgmres_solve_y(const int* st, cd64* S, long ss, int B, int m) {
  const int r = threadIdx.x;
  if (r >= B) return;
  const int jd = st[8 * r + 2];
  if (jd == 0) return;
  cd64* H = S + r * ss;
  cd64* g = H + (m + 1) * m + 2 * m;
  cd64* y = g + (m + 1);
  for (int i = jd - 1; i >= 0; --i) {
    cd64 s = g[i];
    for (int k = i + 1; k < jd; ++k) s = csub(s, cmul(H[i * m + k], y[k]));
    const cd64 d = H[i * m + i];
    const double dd = d.re * d.re + d.im * d.im;
    y[i] = dd > 0.0 ? mkc((s.re * d.re + s.im * d.im) / dd, (s.im * d.re - s.re * d.im) / dd) : mkc(0.0, 0.0);
  }
}

__global__ void k_bgmres_cycle_end(int* st, int B) {
  const int r = threadIdx.x;
  if (r >= B) return;
  st[8 * r + 2] = 0;
  st[8 * r] = 0;
}

// ---------------------------------------------------------------- launchers
int bred_blocks(long n) { return red_b(n); }

template <typename R>
void launch_bdot(const cplx<R>* a, long avs, long ars, int m, const cplx<R>* b, long brs, long n, int B,
                 cd64* partial, cd64* out, int ostride, long ors, int mode, const int* run, int rs, hipStream_t st) {
  const int G = red_b(n);
  hipLaunchKernelGGL(k_bdot_partial<R>, dim3(G, B), dim3(kBlock), 0, st, a, avs, ars, m, b, brs, n, partial, m, run,
                     rs);
  WCMG_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_bdot_finish, dim3(m, B), dim3(kBlock), 0, st, partial, G, m, m, out, ostride, ors, mode, run,
                     rs);
  WCMG_CHECK_LAUNCH();
}

template <typename R>
void launch_bmulti_axpy_dot(cplx<R>* y, long yrs, const cplx<R>* V, long vvs, long vrs, int m, const cd64* coef,
                            int cks, long crs, long n, int B, cd64* partial, const int* run, int rs, hipStream_t st) {
  require(m >= 1 && m <= kFusedMaxM, WCMG_ERR_ARG, "fused Gram-Schmidt sweep takes at most 20 vectors");
  const int G = red_b(n);
  hipLaunchKernelGGL(k_bmulti_axpy_dot<R>, dim3(G, B), dim3(kBlock), 0, st, y, yrs, V, vvs, vrs, m, coef, cks, crs, n,
                     partial, m, run, rs);
  WCMG_CHECK_LAUNCH();
}

template <typename R>
void launch_barnoldi_dots(cplx<R>* V, long vvs, long vrs, int j, long n, const cd64* shift, long shs,
                          cd64* partial, int B, const int* run, int rs, hipStream_t st) {
  hipLaunchKernelGGL(k_barnoldi_dots<R>, dim3(red_b(n), B), dim3(kBlock), 0, st, V, vvs, vrs, j, n, shift, shs,
                     partial, j + 2, run, rs);
  WCMG_CHECK_LAUNCH();
}
template <typename R>
void launch_bupdate_scale(cplx<R>* y, long yrs, const cplx<R>* V, long vvs, long vrs, int m, const cd64* coef,
                          long crs, const cd64* nrm2, long nrs, long n, int B, const int* run, int rs,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_bupdate_scale<R>, dim3(nblocks(n), B), dim3(kBlock), 0, st, y, yrs, V, vvs, vrs, m, coef, crs,
                     nrm2, nrs, n, run, rs);
  WCMG_CHECK_LAUNCH();
}
void launch_bgmres_sr(int* st_, cd64* S, long ss, int B, int m, int j, cd64* d, cd64* d2, int stage, hipStream_t st) {
  hipLaunchKernelGGL(k_bgmres_sr, dim3(1), dim3(64), 0, st, st_, S, ss, B, m, j, d, d2, stage);
  WCMG_CHECK_LAUNCH();
}

void launch_bdot_finish(const cd64* partial, int G, int m, int mstride, int B, cd64* out, int ostride, long ors,
                        int mode, const int* run, int rs, hipStream_t st) {
  hipLaunchKernelGGL(k_bdot_finish, dim3(m, B), dim3(kBlock), 0, st, partial, G, m, mstride, out, ostride, ors, mode,
                     run, rs);
  WCMG_CHECK_LAUNCH();
}

template <typename R>
void launch_bmulti_axpy(cplx<R>* y, long yrs, const cplx<R>* V, long vvs, long vrs, int m, const int* m_dev, int ms,
                        const cd64* coef, int cks, long crs, double sign, long n, int B, cd64* norm_part,
                        const int* run, int rs, hipStream_t st) {
  const unsigned G = norm_part ? (unsigned)red_b(n) : std::min<unsigned>(nblocks(n), 4096u);
  hipLaunchKernelGGL(k_bmulti_axpy<R>, dim3(G, B), dim3(kBlock), 0, st, y, yrs, V, vvs, vrs, m, m_dev, ms, coef, cks,
                     crs, sign, n, norm_part, run, rs);
  WCMG_CHECK_LAUNCH();
}

template <typename Ti, typename To>
void launch_belem(To* y, long yrs, const Ti* x, long xrs, const Ti* z, long zrs, const cd64* nrm2, long nrs, long n,
                  int B, int op, const int* run, int rs, hipStream_t st) {
  hipLaunchKernelGGL((k_belem<Ti, To>), dim3(nblocks(n), B), dim3(kBlock), 0, st, y, yrs, x, xrs, z, zrs, nrm2, nrs,
                     n, op, run, rs);
  WCMG_CHECK_LAUNCH();
}

template <typename R>
void launch_bmr_update(cplx<R>* x, cplx<R>* r, const cplx<R>* p, long rsf, const cd64* dots, long n, int B,
                       const int* run, int rs, hipStream_t st) {
  hipLaunchKernelGGL(k_bmr_update<R>, dim3(nblocks(n), B), dim3(kBlock), 0, st, x, r, p, rsf, dots, n, run, rs);
  WCMG_CHECK_LAUNCH();
}

void launch_bgmres_init(int* st_, int B, const int* parent, int prs, hipStream_t st) {
  hipLaunchKernelGGL(k_bgmres_init, dim3(1), dim3(64), 0, st, st_, B, parent, prs);
  WCMG_CHECK_LAUNCH();
}
void launch_bgmres_cycle_start(int* st_, cd64* S, long ss, int B, int m, double tol, int limit, int fixed,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_bgmres_cycle_start, dim3(1), dim3(64), 0, st, st_, S, ss, B, m, tol, limit, fixed);
  WCMG_CHECK_LAUNCH();
}
void launch_bgmres_givens(int* st_, cd64* S, long ss, int B, int m, int j, double tol, int limit, int fixed,
                          int stop_on_est, hipStream_t st) {
  hipLaunchKernelGGL(k_bgmres_givens, dim3(1), dim3(64), 0, st, st_, S, ss, B, m, j, tol, limit, fixed, stop_on_est);
  WCMG_CHECK_LAUNCH();
}
void launch_bgmres_solve_y(const int* st_, cd64* S, long ss, int B, int m, hipStream_t st) {
  hipLaunchKernelGGL(k_bgmres_solve_y, dim3(1), dim3(64), 0, st, st_, S, ss, B, m);
  WCMG_CHECK_LAUNCH();
}
void launch_bgmres_cycle_end(int* st_, int B, hipStream_t st) {
  hipLaunchKernelGGL(k_bgmres_cycle_end, dim3(1), dim3(64), 0, st, st_, B);
  WCMG_CHECK_LAUNCH();
}

#define INST_B(R)                                                                                                    \
  template void launch_bdot<R>(const cplx<R>*, long, long, int, const cplx<R>*, long, long, int, cd64*, cd64*, int,   \
                               long, int, const int*, int, hipStream_t);                                             \
  template void launch_bmulti_axpy<R>(cplx<R>*, long, const cplx<R>*, long, long, int, const int*, int, const cd64*, \
                                      int, long, double, long, int, cd64*, const int*, int, hipStream_t);           \
  template void launch_bmr_update<R>(cplx<R>*, cplx<R>*, const cplx<R>*, long, const cd64*, long, int, const int*,    \
                                     int, hipStream_t);                                                             \
  template void launch_bmulti_axpy_dot<R>(cplx<R>*, long, const cplx<R>*, long, long, int, const cd64*, int, long,      \
                                          long, int, cd64*, const int*, int, hipStream_t);                          \
  template void launch_barnoldi_dots<R>(cplx<R>*, long, long, int, long, const cd64*, long, cd64*, int, const int*,    \
                                        int, hipStream_t);                                                          \
  template void launch_bupdate_scale<R>(cplx<R>*, long, const cplx<R>*, long, long, int, const cd64*, long,            \
                                        const cd64*, long, long, int, const int*, int, hipStream_t);
INST_B(double)
INST_B(float)
template void launch_belem<cd64, cd64>(cd64*, long, const cd64*, long, const cd64*, long, const cd64*, long, long, int,
                                       int, const int*, int, hipStream_t);
template void launch_belem<cf32, cf32>(cf32*, long, const cf32*, long, const cf32*, long, const cd64*, long, long, int,
                                       int, const int*, int, hipStream_t);
template void launch_belem<cd64, cf32>(cf32*, long, const cd64*, long, const cd64*, long, const cd64*, long, long, int,
                                       int, const int*, int, hipStream_t);
template void launch_belem<cf32, cd64>(cd64*, long, const cf32*, long, const cf32*, long, const cd64*, long, long, int,
                                       int, const int*, int, hipStream_t);

}  // namespace wcmg
