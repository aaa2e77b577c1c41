// GMRES on the coarsest level (Sec. 2.1: the coarse-grid solver is GMRES),
// with each Arnoldi step fused into four kernels:
//   1. w = A u / |u| and v_j = u / |u| (the previous step's normalisation is
//      folded in by linearity), plus per-workgroup partials of <v_i, w>, i <= j;
//   2. every workgroup reduces those partials itself (fixed order, identical in
//      all workgroups), w -= V h on its rows, partials of the second pass;
//   3. the same for the second Gram-Schmidt pass (CGS2), partials of |w|^2;
//   4. one workgroup reduces |w|^2 and applies the Givens rotations.
// Scalars and control words stay on the device; state words as in blas.hip.
#include "coarse5.h"

namespace wcmg {

constexpr int kMaxM1 = 41;  // restart length + 1 (restart <= 40)

struct CgScalars {
  cd64 *H, *cs, *sn, *g, *y, *misc;
};
__device__ inline CgScalars cg_scalars(cd64* S, int m) {
  CgScalars c;
  c.H = S;
  c.cs = S + (m + 1) * m;
  c.sn = c.cs + m;
  c.g = c.sn + m;
  c.y = c.g + (m + 1);
  c.misc = c.y + m;
  return c;
}

__device__ inline cd64 wsum(cd64 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.re += __shfl_xor(v.re, off, 64);
    v.im += __shfl_xor(v.im, off, 64);
  }
  return v;
}

// part[blk][i] = sum over the workgroup of c_i(lane), for i < cnt (fixed order).
// c(i) is a device lambda giving the lane's contribution to entry i.
template <typename F>
__device__ inline void multi_block_sum(int cnt, F c, cd64* lds /*[4][kMaxM1]*/, cd64* out /*cnt entries*/) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i = 0; i < cnt; ++i) {
    cd64 s = wsum(c(i));
    if (lane == 0) lds[wave * kMaxM1 + i] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < cnt) {
    cd64 s = mkc(0.0, 0.0);
    for (int w = 0; w < nw; ++w) s = cadd(s, lds[w * kMaxM1 + threadIdx.x]);
    out[threadIdx.x] = s;
  }
}

// partials of |r|^2 (one entry per workgroup, stride m1)
template <typename R>
__global__ void __launch_bounds__(256) k_cg_norm_partial(const cplx<R>* __restrict__ r, long n,
                                                          cd64* __restrict__ part, int m1,
                                                          const int* __restrict__ run) {
  if (run && !*run) return;
  __shared__ cd64 lds[4 * kMaxM1];
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  cplx<R> v = t < n ? r[t] : mkc((R)0, (R)0);
  const double q = (double)v.re * v.re + (double)v.im * v.im;
  multi_block_sum(1, [=](int) { return mkc(q, 0.0); }, lds, part + (long)blockIdx.x * m1);
}

// Start of a restart cycle: beta^2 from the partials; decide whether to iterate.
__global__ void __launch_bounds__(256) k_cg_cycle_start(int* st, cd64* S, int m, const cd64* __restrict__ part,
                                                         int G, int m1, int first, double tol, int limit,
                                                         int fixed) {
  __shared__ cd64 lds[4];
  const int live = st[1];
  if (!live) {
    if (threadIdx.x == 0) {
      st[0] = 0;
      st[2] = 0;
    }
    return;
  }
  cd64 s = mkc(0.0, 0.0);
  s = strided_sum<8>(threadIdx.x, blockDim.x, G, [&](int g) { return part[(long)g * m1]; });
  s = wsum(s);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds[wave] = s;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double b2 = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) b2 += lds[w].re;
  CgScalars c = cg_scalars(S, m);
  c.misc[1] = mkc(b2, 0.0);
  if (first) c.misc[0] = mkc(b2, 0.0);
  st[0] = 0;
  st[2] = 0;
  const double bn = sqrt(c.misc[0].re), beta = sqrt(b2);
  c.misc[2].re = bn > 0 ? beta / bn : 0.0;
  if (st[3] >= limit || bn == 0.0 || beta == 0.0 || (!fixed && beta <= tol * bn) || !(beta == beta)) {
    st[1] = 0;
    st[4] = !(beta == beta) ? 3 : 1;
    return;
  }
  for (int i = 0; i <= m; ++i) c.g[i] = mkc(0.0, 0.0);
  c.g[0] = mkc(beta, 0.0);
  st[0] = 1;
}

// Step 1: w = A u / |u|, v_j = u / |u|, partials of <v_i, w> for i <= j.
template <int P, int NB, int S, bool FIVE>
__global__ void __launch_bounds__(256) k_cg_apply(const Chunk16* __restrict__ blk, const int* __restrict__ nbr,
                                                   long Vc, const cplx<typename BlkTraits<P>::R>* __restrict__ u,
                                                   const cd64* __restrict__ unrm2,
                                                   cplx<typename BlkTraits<P>::R>* __restrict__ V, int j,
                                                   cplx<typename BlkTraits<P>::R>* __restrict__ wout,
                                                   cd64* __restrict__ part, int m1, const int* __restrict__ run) {
  typedef typename BlkTraits<P>::R R;
  if (!*run) return;
  __shared__ cd64 lds[4 * kMaxM1];
  const long n = Vc * NB;
  const long xb = xcd_block(blockIdx.x, gridDim.x);
  const long g = xb * blockDim.x + threadIdx.x;
  const long t = g / S;
  const int sub = (int)(g % S);
  const bool valid = t < n;
  const double inv = 1.0 / sqrt(unrm2->re);
  cplx<R> acc;
  if constexpr (FIVE) acc = coarse_row5<P, NB, S>(blk, u, nbr, Vc, xb * (blockDim.x / S), t, sub, valid);
  else acc = coarse_row<P, NB, S>(blk, u, nbr, Vc, NB, t, sub, 0x1ff, valid);
  const bool own = valid && sub == 0;
  cplx<R> vj = mkc((R)0, (R)0), wv = mkc((R)0, (R)0);
  if (own) {
    const cplx<R> ut = u[t];
    vj = mkc((R)(ut.re * inv), (R)(ut.im * inv));
    wv = mkc((R)(acc.re * inv), (R)(acc.im * inv));
    V[(long)j * n + t] = vj;
    wout[t] = wv;
  }
  multi_block_sum(
      j + 1,
      [=](int i) {
        const cplx<R> vi = i == j ? vj : (own ? V[(long)i * n + t] : mkc((R)0, (R)0));
        return mkc((double)vi.re * wv.re + (double)vi.im * wv.im, (double)vi.re * wv.im - (double)vi.im * wv.re);
      },
      lds, part + (long)blockIdx.x * m1);
}

// Steps 2 and 3: reduce the partials of <v_i, w> (identically in every
// workgroup), record them in column j of H, w -= V h on this workgroup's
// rows, then partials of the next pass (pass 0) or of |w|^2 (pass 1).
template <typename R>
__global__ void __launch_bounds__(256) k_cg_orth(cplx<R>* __restrict__ V, int j, cplx<R>* __restrict__ w, long n,
                                                  const cd64* __restrict__ part_in, int G_in, cd64* __restrict__ S,
                                                  int m, int pass, cd64* __restrict__ part_out,
                                                  const int* __restrict__ run) {
  if (!*run) return;
  __shared__ cd64 h[kMaxM1];
  __shared__ cd64 lds[4 * kMaxM1];
  const int m1 = m + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i = wave; i <= j; i += nw) {
    cd64 s = mkc(0.0, 0.0);
    for (int gg = lane; gg < G_in; gg += 64) s = cadd(s, part_in[(long)gg * m1 + i]);
    s = wsum(s);
    if (lane == 0) h[i] = s;
  }
  __syncthreads();
  if (blockIdx.x == 0 && (int)threadIdx.x <= j) {
    cd64* Hij = S + threadIdx.x * m + j;
    *Hij = pass == 0 ? h[threadIdx.x] : cadd(*Hij, h[threadIdx.x]);
  }
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const bool valid = t < n;
  cplx<R> wv = mkc((R)0, (R)0);
  if (valid) {
    wv = w[t];
    for (int i = 0; i <= j; ++i) {
      const cplx<R> hi = mkc((R)h[i].re, (R)h[i].im);
      cfma(wv, cneg(hi), V[(long)i * n + t]);
    }
    w[t] = wv;
  }
  if (pass == 0) {
    multi_block_sum(
        j + 1,
        [=](int i) {
          const cplx<R> vi = valid ? V[(long)i * n + t] : mkc((R)0, (R)0);
          return mkc((double)vi.re * wv.re + (double)vi.im * wv.im, (double)vi.re * wv.im - (double)vi.im * wv.re);
        },
        lds, part_out + (long)blockIdx.x * m1);
  } else {
    const double q = (double)wv.re * wv.re + (double)wv.im * wv.im;
    multi_block_sum(1, [=](int) { return mkc(q, 0.0); }, lds, part_out + (long)blockIdx.x * m1);
  }
}

// Step 4: hn^2 = |w|^2 from the partials, Givens update of column j.
__global__ void __launch_bounds__(256) k_cg_givens(int* st, cd64* S, int m, int j, const cd64* __restrict__ part,
                                                    int G, double tol, int limit, int fixed) {
  __shared__ cd64 lds[4];
  if (!st[0]) return;
  const int m1 = m + 1;
  cd64 s = mkc(0.0, 0.0);
  s = strided_sum<8>(threadIdx.x, blockDim.x, G, [&](int g) { return part[(long)g * m1]; });
  s = wsum(s);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds[wave] = s;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double hn2 = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) hn2 += lds[w].re;
  CgScalars c = cg_scalars(S, m);
  c.misc[3] = mkc(hn2, 0.0);
  const double hn = sqrt(hn2);
  cd64* H = c.H;
  // the entry rotated down the column stays in a register, so a rotation's
  // loads do not wait for the previous one's stores (the same arithmetic)
  cd64 a = H[j];
  for (int i = 0; i < j; ++i) {
    const cd64 b = H[(i + 1) * m + j], ci = c.cs[i], si = c.sn[i];
    cd64 t = cmul(ci, a);
    cfma(t, si, b);
    cd64 u = cmul(cneg(cconj(si)), a);
    cfma(u, cconj(ci), b);
    H[i * m + j] = t;
    a = u;
  }
  const double den = sqrt(a.re * a.re + a.im * a.im + hn2);
  const cd64 cc = den == 0.0 ? mkc(1.0, 0.0) : mkc(a.re / den, -a.im / den);
  const cd64 ss = den == 0.0 ? mkc(0.0, 0.0) : mkc(hn / den, 0.0);
  c.cs[j] = cc;
  c.sn[j] = ss;
  H[j * m + j] = mkc(den, 0.0);
  H[(j + 1) * m + j] = mkc(0.0, 0.0);
  const cd64 gj = c.g[j];
  c.g[j + 1] = den == 0.0 ? gj : cmul(cneg(cconj(ss)), gj);  // den == 0: singular column, dropped
  c.g[j] = cmul(cc, gj);
  st[2] = den == 0.0 ? j : j + 1;
  st[3] += 1;
  const double bn = sqrt(c.misc[0].re);
  const double est = bn > 0 ? sqrt(c.g[j + 1].re * c.g[j + 1].re + c.g[j + 1].im * c.g[j + 1].im) / bn : 0.0;
  c.misc[2].re = est;
  bool stop = false;
  if (st[3] >= limit) {
    stop = true;
    st[1] = 0;
    st[4] = 2;
  }
  if (!fixed && est <= tol) {
    stop = true;
    st[1] = 0;
    st[4] = 1;
  }
  if (hn == 0.0 || !(est == est)) {
    stop = true;
    st[1] = 0;
    st[4] = (est == est) ? (den == 0.0 ? 4 : 1) : 3;
  }
  if (stop || j + 1 == m) st[0] = 0;
}

// ---------------------------------------------------------------- launchers
template <typename R>
void launch_cg_norm_partial(const cplx<R>* r, long n, cd64* part, int m1, const int* run, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_norm_partial<R>, dim3(nblocks(n)), dim3(kBlock), 0, st, r, n, part, m1, run);
  WCMG_CHECK_LAUNCH();
}
template void launch_cg_norm_partial<double>(const cd64*, long, cd64*, int, const int*, hipStream_t);
template void launch_cg_norm_partial<float>(const cf32*, long, cd64*, int, const int*, hipStream_t);

void launch_cg_cycle_start(int* stw, cd64* S, int m, const cd64* part, int G, int first, double tol, int limit,
                           int fixed, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_cycle_start, dim3(1), dim3(kBlock), 0, st, stw, S, m, part, G, m + 1, first, tol, limit,
                     fixed);
  WCMG_CHECK_LAUNCH();
}

template <int P, int NB, int S>
static void cg_apply_t(bool five, const void* blk, const int* nbr, long Vc, const void* u, const cd64* unrm2,
                       void* V, int j, void* wout, cd64* part, int m1, const int* run, hipStream_t st) {
  typedef typename BlkTraits<P>::R R;
  if (five)
    WCMG_LAUNCH((k_cg_apply<P, NB, S, true>), dim3(nblocks(Vc * NB * S)), dim3(kBlock), 0, st, (const Chunk16*)blk,
                nbr, Vc, (const cplx<R>*)u, unrm2, (cplx<R>*)V, j, (cplx<R>*)wout, part, m1, run);
  else
    WCMG_LAUNCH((k_cg_apply<P, NB, S, false>), dim3(nblocks(Vc * NB * S)), dim3(kBlock), 0, st, (const Chunk16*)blk,
                nbr, Vc, (const cplx<R>*)u, unrm2, (cplx<R>*)V, j, (cplx<R>*)wout, part, m1, run);
}
template <int P, int NB>
static void cg_apply_s(int S, bool five, const void* blk, const int* nbr, long Vc, const void* u, const cd64* unrm2,
                       void* V, int j, void* wout, cd64* part, int m1, const int* run, hipStream_t st) {
  if (S == 1) cg_apply_t<P, NB, 1>(five, blk, nbr, Vc, u, unrm2, V, j, wout, part, m1, run, st);
  else if (S == 2) cg_apply_t<P, NB, 2>(five, blk, nbr, Vc, u, unrm2, V, j, wout, part, m1, run, st);
  else if (S == 4) cg_apply_t<P, NB, 4>(five, blk, nbr, Vc, u, unrm2, V, j, wout, part, m1, run, st);
  else cg_apply_t<P, NB, 8>(five, blk, nbr, Vc, u, unrm2, V, j, wout, part, m1, run, st);
}
template <int P>
static void cg_apply_nb(int nb, int S, bool five, const void* blk, const int* nbr, long Vc, const void* u,
                        const cd64* unrm2, void* V, int j, void* wout, cd64* part, int m1, const int* run,
                        hipStream_t st) {
  switch (nb) {
    case 8: cg_apply_s<P, 8>(S, five, blk, nbr, Vc, u, unrm2, V, j, wout, part, m1, run, st); break;
    case 12: cg_apply_s<P, 12>(S, five, blk, nbr, Vc, u, unrm2, V, j, wout, part, m1, run, st); break;
    case 16: cg_apply_s<P, 16>(S, five, blk, nbr, Vc, u, unrm2, V, j, wout, part, m1, run, st); break;
    case 24: cg_apply_s<P, 24>(S, five, blk, nbr, Vc, u, unrm2, V, j, wout, part, m1, run, st); break;
    case 32: cg_apply_s<P, 32>(S, five, blk, nbr, Vc, u, unrm2, V, j, wout, part, m1, run, st); break;
    default: throw Error(WCMG_ERR_ARG, "fused coarse GMRES: unsupported Nb");
  }
}

bool cg_fused_supported(int nb) { return nb == 8 || nb == 12 || nb == 16 || nb == 24 || nb == 32; }

// Returns the number of workgroups of the apply step (the partial count).
int launch_cg_apply(int prec, int nb, const void* blk, const int* nbr, long Vc, const void* u, const cd64* unrm2,
                    void* V, int j, void* wout, cd64* part, int m1, const int* run, hipStream_t st, bool five) {
  const int S = coarse_split(Vc * nb);
  if (prec == WCMG_F64) cg_apply_nb<WCMG_F64>(nb, S, five, blk, nbr, Vc, u, unrm2, V, j, wout, part, m1, run, st);
  else if (prec == WCMG_F32) cg_apply_nb<WCMG_F32>(nb, S, five, blk, nbr, Vc, u, unrm2, V, j, wout, part, m1, run, st);
  else cg_apply_nb<WCMG_BF16>(nb, S, five, blk, nbr, Vc, u, unrm2, V, j, wout, part, m1, run, st);
  WCMG_CHECK_LAUNCH();
  return (int)nblocks(Vc * nb * S);
}

template <typename R>
void launch_cg_orth(cplx<R>* V, int j, cplx<R>* w, long n, const cd64* part_in, int G_in, cd64* S, int m, int pass,
                    cd64* part_out, const int* run, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_orth<R>, dim3(nblocks(n)), dim3(kBlock), 0, st, V, j, w, n, part_in, G_in, S, m, pass,
                     part_out, run);
  WCMG_CHECK_LAUNCH();
}
template void launch_cg_orth<double>(cd64*, int, cd64*, long, const cd64*, int, cd64*, int, int, cd64*, const int*,
                                     hipStream_t);
template void launch_cg_orth<float>(cf32*, int, cf32*, long, const cd64*, int, cd64*, int, int, cd64*, const int*,
                                    hipStream_t);

void launch_cg_givens(int* stw, cd64* S, int m, int j, const cd64* part, int G, double tol, int limit, int fixed,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_cg_givens, dim3(1), dim3(kBlock), 0, st, stw, S, m, j, part, G, tol, limit, fixed);
  WCMG_CHECK_LAUNCH();
}

}  // namespace wcmg
