// Fine level: clover term, field packing and the Wilson-clover operator.
//
// Device layout of level 0 (aggregate-major, Sec. 3 of the paper: the fine
// lattice is linearised aggregate by aggregate so restriction reads contiguous
// memory):  device site s = c * A + o, with c the aggregate and o the offset
// inside it.  Fields are structure-of-arrays over sites:
//   spinor   [12][V]      complex (component k = 3*spin + colour)
//   links    [4][9][V]    complex, U_mu(s) row-major; the antiperiodic sign of
//                         the t boundary is folded into U_t on the last slice
//   clover   [2][36/RC][V][RC] real: per chirality a packed Hermitian 6x6 block
//                         of (4 + m0) + C: 6 diagonal reals, then the 15
//                         entries below the diagonal (row i > col j, row-major)
//                         as re, im, in 16-byte chunks of RC reals
//   nbr      [8][V]       int32 neighbour site in direction d = 1..8
#include <type_traits>

#include "wilson_ops.h"

namespace wcmg {

// ---------------------------------------------------------------- clover build
// Q_{mu nu}(x): sum of the four plaquette leaves in the mu-nu plane through x.
// Computed on the lexicographic lattice directly from the caller's links.
struct Su3 {
  cd64 m[9];
};
__device__ inline Su3 su3_load(const cd64* U, long site, int mu) {
  Su3 r;
  const cd64* p = U + (site * 4 + mu) * 9;
#pragma unroll
  for (int i = 0; i < 9; ++i) r.m[i] = p[i];
  return r;
}
__device__ inline Su3 su3_mm(const Su3& a, const Su3& b) {
  Su3 c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cd64 s = mkc(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) cfma(s, a.m[i * 3 + k], b.m[k * 3 + j]);
      c.m[i * 3 + j] = s;
    }
  return c;
}
// a * b^dag
__device__ inline Su3 su3_mmd(const Su3& a, const Su3& b) {
  Su3 c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cd64 s = mkc(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) cfma(s, a.m[i * 3 + k], cconj(b.m[j * 3 + k]));
      c.m[i * 3 + j] = s;
    }
  return c;
}
// a^dag * b
__device__ inline Su3 su3_mdm(const Su3& a, const Su3& b) {
  Su3 c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cd64 s = mkc(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) cfmac(s, a.m[k * 3 + i], b.m[k * 3 + j]);
      c.m[i * 3 + j] = s;
    }
  return c;
}

struct Lex {
  int L[4];
  __device__ long shift(long i, int mu, int step) const {
    int x[4];
    long r = i;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      x[m] = (int)(r % L[m]);
      r /= L[m];
    }
    x[mu] = (x[mu] + step + L[mu]) % L[mu];
    return x[0] + (long)L[0] * (x[1] + (long)L[1] * (x[2] + (long)L[2] * x[3]));
  }
};

// F_{mu nu}(x) = (Q - Q^dag) / 8
__device__ Su3 field_strength(const cd64* U, const Lex& lx, long x, int mu, int nu) {
  long xpm = lx.shift(x, mu, 1), xpn = lx.shift(x, nu, 1);
  long xmm = lx.shift(x, mu, -1), xmn = lx.shift(x, nu, -1);
  long xmm_pn = lx.shift(xmm, nu, 1), xmm_mn = lx.shift(xmm, nu, -1), xmn_pm = lx.shift(xmn, mu, 1);
  Su3 Q, t;
  // x -> x+mu -> x+mu+nu -> x+nu -> x
  t = su3_mm(su3_load(U, x, mu), su3_load(U, xpm, nu));
  t = su3_mmd(t, su3_load(U, xpn, mu));
  Q = su3_mmd(t, su3_load(U, x, nu));
  // x -> x+nu -> x+nu-mu -> x-mu -> x
  t = su3_mmd(su3_load(U, x, nu), su3_load(U, xmm_pn, mu));
  t = su3_mmd(t, su3_load(U, xmm, nu));
  t = su3_mm(t, su3_load(U, xmm, mu));
#pragma unroll
  for (int i = 0; i < 9; ++i) Q.m[i] = cadd(Q.m[i], t.m[i]);
  // x -> x-mu -> x-mu-nu -> x-nu -> x
  {
    Su3 a = su3_load(U, xmm, mu), b = su3_load(U, xmm_mn, nu);
    // a^dag b^dag = (b a)^dag
    Su3 ba = su3_mm(b, a);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) t.m[i * 3 + j] = cconj(ba.m[j * 3 + i]);
  }
  t = su3_mm(t, su3_load(U, xmm_mn, mu));
  t = su3_mm(t, su3_load(U, xmn, nu));
#pragma unroll
  for (int i = 0; i < 9; ++i) Q.m[i] = cadd(Q.m[i], t.m[i]);
  // x -> x-nu -> x-nu+mu -> x+mu -> x
  t = su3_mdm(su3_load(U, xmn, nu), su3_load(U, xmn, mu));
  t = su3_mm(t, su3_load(U, xmn_pm, nu));
  t = su3_mmd(t, su3_load(U, x, mu));
#pragma unroll
  for (int i = 0; i < 9; ++i) Q.m[i] = cadd(Q.m[i], t.m[i]);
  Su3 F;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) F.m[i * 3 + j] = cscale(0.125, csub(Q.m[i * 3 + j], cconj(Q.m[j * 3 + i])));
  return F;
}

// Clover term per chirality in the chiral basis.  With X_l the colour matrices
//   chirality +: X1 = F_xt - F_yz, X2 = F_yt + F_xz, X3 = F_zt - F_xy
//   chirality -: X1 = -F_xt - F_yz, X2 = F_xz - F_yt, X3 = -F_zt - F_xy
// the 6x6 block is c_sw (i/2) sum_l sigma_l (x) X_l, i.e. spin blocks
//   (0,0) = X3, (0,1) = X1 - i X2, (1,0) = X1 + i X2, (1,1) = -X3, times c_sw i/2.
// Output: [V][2][6][6] complex128, lexicographic.
__global__ void k_clover_build(const cd64* __restrict__ U, Lex lx, long V, double csw, cd64* __restrict__ out) {
  long x = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (x >= V) return;
  Su3 Fxy = field_strength(U, lx, x, 0, 1), Fxz = field_strength(U, lx, x, 0, 2), Fxt = field_strength(U, lx, x, 0, 3);
  Su3 Fyz = field_strength(U, lx, x, 1, 2), Fyt = field_strength(U, lx, x, 1, 3), Fzt = field_strength(U, lx, x, 2, 3);
  for (int chi = 0; chi < 2; ++chi) {
    double s = chi == 0 ? 1.0 : -1.0;
    cd64* blk = out + (x * 2 + chi) * 36;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        int e = a * 3 + b;
        cd64 X1 = csub(cscale(s, Fxt.m[e]), Fyz.m[e]);
        cd64 X2 = cadd(Fxz.m[e], cscale(s, Fyt.m[e]));
        cd64 X3 = csub(cscale(s, Fzt.m[e]), Fxy.m[e]);
        cd64 b00 = X3, b11 = cneg(X3);
        cd64 b01 = csub(X1, ci(X2)), b10 = cadd(X1, ci(X2));
        // times c_sw * i / 2
        blk[(0 * 3 + a) * 6 + 0 * 3 + b] = cscale(0.5 * csw, ci(b00));
        blk[(0 * 3 + a) * 6 + 1 * 3 + b] = cscale(0.5 * csw, ci(b01));
        blk[(1 * 3 + a) * 6 + 0 * 3 + b] = cscale(0.5 * csw, ci(b10));
        blk[(1 * 3 + a) * 6 + 1 * 3 + b] = cscale(0.5 * csw, ci(b11));
      }
  }
}

// Pack (4 + m0) + C into the device clover layout, in device site order:
// per chirality the 36 reals (6 diagonal, then the 15 lower-triangle entries
// as re, im) in 16-byte chunks of RC = 16 / sizeof(R) reals: [chi][36/RC][V][RC].
template <typename R>
__global__ void k_pack_clover(const cd64* __restrict__ blocks, const int* __restrict__ perm, long V, double m0,
                              R* __restrict__ out) {
  constexpr int RC = 16 / sizeof(R);
  long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= V) return;
  long x = perm[s];
  for (int chi = 0; chi < 2; ++chi) {
    const cd64* b = blocks + (x * 2 + chi) * 36;
    R e[36];
    for (int i = 0; i < 6; ++i) e[i] = (R)(4.0 + m0 + b[i * 6 + i].re);
    int idx = 0;
    for (int i = 1; i < 6; ++i)
      for (int j = 0; j < i; ++j, ++idx) {
        e[6 + 2 * idx] = (R)b[i * 6 + j].re;
        e[7 + 2 * idx] = (R)b[i * 6 + j].im;
      }
    R* o = out + (long)chi * 36 * V;
    for (int q = 0; q < 36 / RC; ++q)
      for (int r = 0; r < RC; ++r) o[((long)q * V + s) * RC + r] = e[q * RC + r];
  }
}

template <typename R>
__global__ void k_pack_links(const cd64* __restrict__ U, const int* __restrict__ perm, long V, int Lt, long Vs,
                             int antiperiodic, cplx<R>* __restrict__ out) {
  long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= V) return;
  long x = perm[s];
  bool last_t = (x / Vs) == Lt - 1;
  for (int mu = 0; mu < 4; ++mu) {
    double sg = (mu == 3 && antiperiodic && last_t) ? -1.0 : 1.0;
    for (int e = 0; e < 9; ++e) {
      cd64 u = U[(x * 4 + mu) * 9 + e];
      out[(long)(mu * 9 + e) * V + s] = mkc((R)(sg * u.re), (R)(sg * u.im));
    }
  }
}

// canonical [V][12] (lexicographic) <-> device [12][V] (aggregate-major)
template <typename Ti, typename To>
__global__ void k_pack_fermion(const cplx<Ti>* __restrict__ in, const int* __restrict__ perm, long V,
                               cplx<To>* __restrict__ out) {
  long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= V) return;
  long x = perm[s];
  long r = blockIdx.y;
  in += r * V * 12;
  out += r * V * 12;
#pragma unroll
  for (int k = 0; k < 12; ++k) out[(long)k * V + s] = ccast<To>(in[x * 12 + k]);
}
template <typename Ti, typename To>
__global__ void k_unpack_fermion(const cplx<Ti>* __restrict__ in, const int* __restrict__ perm, long V,
                                 cplx<To>* __restrict__ out) {
  long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= V) return;
  long x = perm[s];
  long r = blockIdx.y;
  in += r * V * 12;
  out += r * V * 12;
#pragma unroll
  for (int k = 0; k < 12; ++k) out[x * 12 + k] = ccast<To>(in[(long)k * V + s]);
}

// ---------------------------------------------------------------- Wilson-clover operator
// out = sum of the selected terms of D applied to in.
// terms: bit 0 = Mdiag ((4+m0) + C), bit d (1..8) = Mdir_d.
//
// A workgroup of 4 waves owns 64 consecutive sites; wave mu computes the two
// hops along direction mu for all 64 sites (waves 0 and 1 also the clover
// block of chirality 0 and 1), so every branch is wave-uniform and four times
// as many loads are in flight as with one lane per site.  The four partial
// spinors are combined in LDS in a fixed order.  ALL: every term (the whole
// operator, the common case) with no per-term branches, so the compiler can
// issue both hops' loads together.
// dots != nullptr: per-workgroup partials of <out, in> and <out, out> (the
// inner products of an MR step, where in = r and out = D r) go to
// dots[2*blk], dots[2*blk+1].  Waves 0 and 1 then write the output of their
// chirality and form the products with the input components they loaded for
// the clover block.  bsub != nullptr (without dots): out = bsub - D in, the
// residual of in for the right-hand side bsub.
// The two hops along MU (selected by the terms mask unless ALL), neighbours
// from the site arithmetic (GEO) or from the table.
// L2 (with GEO): two-row links U2 (hop_at2), the t-boundary sign of the
// rebuilt third row from the site coordinates.
template <typename R, int MU, bool GEO, bool ALL, bool L2>
__device__ inline void hops_mu(cplx<R> (&acc)[12], const cplx<R>* __restrict__ in, const cplx<R>* __restrict__ U,
                               const int* __restrict__ nbr, const SiteGeom& geo, long V, long s, int terms) {
  long yf, yb;
  R sf = (R)1, sb = (R)1;
  if constexpr (GEO) {
    uint32_t f, b;
    if constexpr (L2 && MU == 3) {
      bool last, first;
      geo.hop_sites_edge<MU>((uint32_t)s, f, b, last, first);
      // U_t(s) carries the sign when s is on the last t slice, U_t(s - t) when s is on the first
      if (geo.anti) {
        sf = last ? (R)-1 : (R)1;
        sb = first ? (R)-1 : (R)1;
      }
    } else {
      geo.hop_sites<MU>((uint32_t)s, f, b);
    }
    yf = f;
    yb = b;
  } else {
    yf = nbr[(long)(2 * MU) * V + s];
    yb = nbr[(long)(2 * MU + 1) * V + s];
  }
  if constexpr (L2) {
    if (ALL || (terms & (1 << (2 * MU + 1)))) hop_at2<R, MU, true>(acc, in, U, V, s, yf, sf);
    if (ALL || (terms & (1 << (2 * MU + 2)))) hop_at2<R, MU, false>(acc, in, U, V, s, yb, sb);
  } else {
    if (ALL || (terms & (1 << (2 * MU + 1)))) hop_at<R, MU, true>(acc, in, U, V, s, yf);
    if (ALL || (terms & (1 << (2 * MU + 2)))) hop_at<R, MU, false>(acc, in, U, V, s, yb);
  }
}

template <typename R, bool ALL, bool GEO, bool L2>
__global__ void __launch_bounds__(256) k_wilson(const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out,
                                                 const cplx<R>* __restrict__ U, const R* __restrict__ clov,
                                                 const int* __restrict__ nbr, SiteGeom geo, long V, int terms,
                                                 int nrhs, cd64* __restrict__ dots, const int* __restrict__ run,
                                                 int rs, const cplx<R>* __restrict__ bsub) {
  const long nblk = (V + 63) / 64;
  long blk, r;
  if (!item_rhs(nblk, nrhs, &blk, &r)) return;
  if (run && !run[r * rs]) return;
  __shared__ cplx<R> part[4][12][64];
  __shared__ cd64 red[8];
  // FP32 with dots: the own-site input of both chiralities, shared by the four waves
  __shared__ cplx<R> pinl[sizeof(R) == 4 ? 12 : 1][64];
  const int lane = threadIdx.x & 63;
  const int mu = threadIdx.x >> 6;  // wave-uniform
  const long s = blk * 64 + lane;
  const bool valid = s < V;
  in += r * 12 * V;
  out += r * 12 * V;
  cplx<R> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = mkc((R)0, (R)0);
  // waves 0 and 1: the input at the own site, chirality mu
  cplx<R> pin[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) pin[k] = mkc((R)0, (R)0);
  if (valid) {
    if (mu < 2 && (ALL || (terms & 1) || dots)) {
#pragma unroll
      for (int k = 0; k < 6; ++k) pin[k] = in[(long)(mu * 6 + k) * V + s];
    }
    if (ALL || (terms & 1)) {
      if (mu == 0) clover_chirality_p<R, 0>(acc, pin, clov, V, s);
      if (mu == 1) clover_chirality_p<R, 1>(acc, pin, clov, V, s);
    }
    if (mu == 0) hops_mu<R, 0, GEO, ALL, L2>(acc, in, U, nbr, geo, V, s, terms);
    else if (mu == 1) hops_mu<R, 1, GEO, ALL, L2>(acc, in, U, nbr, geo, V, s, terms);
    else if (mu == 2) hops_mu<R, 2, GEO, ALL, L2>(acc, in, U, nbr, geo, V, s, terms);
    else hops_mu<R, 3, GEO, ALL, L2>(acc, in, U, nbr, geo, V, s, terms);
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) part[mu][k][lane] = acc[k];
  if constexpr (sizeof(R) == 4) {
    if (dots && mu < 2)
#pragma unroll
      for (int c = 0; c < 6; ++c) pinl[6 * mu + c][lane] = pin[c];
  }
  __syncthreads();
  if (!dots) {
    // wave mu writes components 3 mu .. 3 mu + 2 (spin mu), summed over the 4 waves in order
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int k = 3 * mu + c;
      cplx<R> v = part[0][k][lane];
      v = cadd(v, part[1][k][lane]);
      v = cadd(v, part[2][k][lane]);
      v = cadd(v, part[3][k][lane]);
      if (valid) {
        if (bsub) v = csub(bsub[r * 12 * V + (long)k * V + s], v);
        out[(long)k * V + s] = v;
      }
    }
    return;
  }
  if constexpr (sizeof(R) == 4) {
    // every wave writes the three components of spin mu and forms their
    // products with the input (from LDS); the four waves' sums are added in order
    double pr = 0.0, pi = 0.0, pp = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int k = 3 * mu + c;
      cplx<R> v = part[0][k][lane];
      v = cadd(v, part[1][k][lane]);
      v = cadd(v, part[2][k][lane]);
      v = cadd(v, part[3][k][lane]);
      if (valid) {
        out[(long)k * V + s] = v;
        const cplx<R> x = pinl[k][lane];
        pr += (double)v.re * x.re + (double)v.im * x.im;
        pi += (double)v.re * x.im - (double)v.im * x.re;
        pp += (double)v.re * v.re + (double)v.im * v.im;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      pr += __shfl_xor(pr, off, 64);
      pi += __shfl_xor(pi, off, 64);
      pp += __shfl_xor(pp, off, 64);
    }
    if (lane == 0) {
      red[2 * mu] = mkc(pr, pi);
      red[2 * mu + 1] = mkc(pp, 0.0);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const long bi = r * nblk + blk;
      dots[2 * bi] = cadd(cadd(red[0], red[2]), cadd(red[4], red[6]));
      dots[2 * bi + 1] = cadd(cadd(red[1], red[3]), cadd(red[5], red[7]));
    }
    return;
  }
  // waves 0 and 1 write the six components of chirality mu and form the
  // products with the input they hold
  if (mu < 2) {
    double pr = 0.0, pi = 0.0, pp = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const int k = 6 * mu + c;
      cplx<R> v = part[0][k][lane];
      v = cadd(v, part[1][k][lane]);
      v = cadd(v, part[2][k][lane]);
      v = cadd(v, part[3][k][lane]);
      if (valid) {
        out[(long)k * V + s] = v;
        const cplx<R> x = pin[c];
        pr += (double)v.re * x.re + (double)v.im * x.im;
        pi += (double)v.re * x.im - (double)v.im * x.re;
        pp += (double)v.re * v.re + (double)v.im * v.im;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      pr += __shfl_xor(pr, off, 64);
      pi += __shfl_xor(pi, off, 64);
      pp += __shfl_xor(pp, off, 64);
    }
    if (lane == 0) {
      red[2 * mu] = mkc(pr, pi);
      red[2 * mu + 1] = mkc(pp, 0.0);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const long bi = r * nblk + blk;
    dots[2 * bi] = cadd(red[0], red[2]);
    dots[2 * bi + 1] = cadd(red[1], red[3]);
  }
}

// Raw buffer access to one FP32 spinor field [12][V]: a 32-bit per-lane byte
// offset (the site) plus a wave-uniform one (the component), so a neighbour
// costs one address VGPR instead of a 64-bit pointer per component.  Accesses
// past the field's size read 0 and are not written.
struct SpinorBuf {
  __amdgpu_buffer_rsrc_t rs;
  __device__ SpinorBuf(const cf32* base, long V)
      : rs(__builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(12 * V * 8), 0x00020000)) {}
  __device__ cf32 ld(unsigned site_off, unsigned comp_off) const {
    return __builtin_bit_cast(cf32, __builtin_amdgcn_raw_buffer_load_b64(rs, site_off, comp_off, 0));
  }
  __device__ void st(cf32 v, unsigned site_off, unsigned comp_off) const {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(rs, 0, 0, 0)), v),
                                          rs, site_off, comp_off, 0);
  }
};

// Several right-hand sides at once (FP32).  A workgroup owns 64 consecutive
// sites and first stages their links (U_mu(x) and U_mu(x - mu), 8 x 9 complex)
// and clover blocks (2 x 36 reals) in LDS; wave w then applies the whole
// operator to right-hand sides w, w + 4, ... with lane = site, reading the
// gauge data from LDS.  Links and clover thus cross HBM once per launch
// instead of once per right-hand side.  dots: per-(RHS, workgroup) partials
// of <out, in> and <out, out> at dots[2 * (r * gridDim.x + blk)].
__global__ void __launch_bounds__(512) k_wilson_mrhs(const cf32* __restrict__ in, cf32* __restrict__ out,
                                                      const cf32* __restrict__ U, const float* __restrict__ clov,
                                                      const int* __restrict__ nbr, long V, int B,
                                                      cd64* __restrict__ dots, const int* __restrict__ run, int rs) {
  __shared__ cf32 lnk[8][9][64];
  __shared__ float4 clv[2][9][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform (scalar)
  const int nw = blockDim.x >> 6;
  const long blk = (gridDim.x % 8 == 0) ? (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8 : blockIdx.x;
  const long s = blk * 64 + lane;
  const bool valid = s < V;
  const long sv = valid ? s : 0;  // in-bounds stand-in for the tail lanes
  // stage: thread (wave, lane) loads rows wave, wave + nw, ... of its site
  {
    int yb[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) yb[mu] = nbr[(long)(2 * mu + 1) * V + sv];
    for (int q = wave; q < 72; q += nw) {
      const int d = q / 9, e = q - 9 * (q / 9), mu = d >> 1;
      const long site = (d & 1) ? (long)yb[mu] : sv;
      lnk[d][e][lane] = U[(long)(mu * 9 + e) * V + site];
    }
    const float4* cb = (const float4*)clov;
    for (int q = wave; q < 18; q += nw) {
      const int chi = q / 9, c = q - 9 * (q / 9);
      clv[chi][c][lane] = cb[((long)chi * 9 + c) * V + sv];
    }
  }
  // right-hand sides still running, as a wave-uniform bit mask (B <= 64)
  const bool on_lane = lane < B && (!run || run[(long)lane * rs]);
  const uint64_t act = __ballot(on_lane);
  const int nact = __popcll(act);
  __syncthreads();
  int yn[8];
#pragma unroll
  for (int d = 0; d < 8; ++d) yn[d] = nbr[(long)d * V + sv];
  const unsigned so = (unsigned)sv * 8u;
  const unsigned cs = (unsigned)V * 8u;  // component stride in bytes
  // wave w takes the active right-hand sides w, w + nw, ...
  for (int j = wave; j < nact; j += nw) {
    // re-read the gauge data from LDS per right-hand side: kept in registers
    // across the loop it would not fit the register file
    asm volatile("" ::: "memory");
    uint64_t m = act;
    for (int t = 0; t < j; ++t) m &= m - 1;  // drop the j lowest set bits
    const long r = __builtin_ctzll(m);
    const SpinorBuf inb(in + r * 12 * V, V);
    cf32 acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = mkc(0.f, 0.f);
    cf32 self[12];  // the site's own spinor: clover term, then the dots
#pragma unroll
    for (int chi = 0; chi < 2; ++chi) {
      float e[36];
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const float4 v = clv[chi][c][lane];
        e[4 * c] = v.x;
        e[4 * c + 1] = v.y;
        e[4 * c + 2] = v.z;
        e[4 * c + 3] = v.w;
      }
      cf32 p[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) p[k] = self[chi * 6 + k] = inb.ld(so, (chi * 6 + k) * cs);
      if (chi == 0) clover_block_apply<float, 0>(acc, e, p);
      else clover_block_apply<float, 1>(acc, e, p);
    }
#define WCMG_MRHS_HOP(MU, FWD)                                                  \
    {                                                                           \
      constexpr int d = 2 * MU + (FWD ? 0 : 1);                                 \
      cf32 p[12], u[9];                                                         \
      const unsigned yo = (unsigned)yn[d] * 8u;                                 \
      _Pragma("unroll") for (int k = 0; k < 12; ++k) p[k] = inb.ld(yo, k * cs); \
      _Pragma("unroll") for (int e = 0; e < 9; ++e) u[e] = lnk[d][e][lane];     \
      hop_core<float, MU, FWD>(acc, p, u);                                      \
    }
    WCMG_MRHS_HOP(0, true)
    WCMG_MRHS_HOP(0, false)
    WCMG_MRHS_HOP(1, true)
    WCMG_MRHS_HOP(1, false)
    WCMG_MRHS_HOP(2, true)
    WCMG_MRHS_HOP(2, false)
    WCMG_MRHS_HOP(3, true)
    WCMG_MRHS_HOP(3, false)
#undef WCMG_MRHS_HOP
    double pr = 0.0, pi = 0.0, pp = 0.0;
    if (valid) {
      const SpinorBuf outb(out + r * 12 * V, V);
#pragma unroll
      for (int k = 0; k < 12; ++k) outb.st(acc[k], so, k * cs);
      if (dots) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          const cf32 x = self[k];
          pr += (double)acc[k].re * x.re + (double)acc[k].im * x.im;
          pi += (double)acc[k].re * x.im - (double)acc[k].im * x.re;
          pp += (double)acc[k].re * acc[k].re + (double)acc[k].im * acc[k].im;
        }
      }
    }
    if (dots) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        pr += __shfl_xor(pr, off, 64);
        pi += __shfl_xor(pi, off, 64);
        pp += __shfl_xor(pp, off, 64);
      }
      if (lane == 0) {
        const long bi = r * gridDim.x + blockIdx.x;
        dots[2 * bi] = mkc(pr, pi);
        dots[2 * bi + 1] = mkc(pp, 0.0);
      }
    }
  }
}

// ---------------------------------------------------------------- launchers
void launch_clover_build(const cd64* U, const int L[4], double csw, cd64* out, hipStream_t st) {
  Lex lx;
  long V = 1;
  for (int m = 0; m < 4; ++m) {
    lx.L[m] = L[m];
    V *= L[m];
  }
  hipLaunchKernelGGL(k_clover_build, dim3(nblocks(V, 128)), dim3(128), 0, st, U, lx, V, csw, out);
  WCMG_CHECK_LAUNCH();
}

template <typename R>
void launch_pack_clover(const cd64* blocks, const int* perm, long V, double m0, R* out, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_clover<R>, dim3(nblocks(V)), dim3(kBlock), 0, st, blocks, perm, V, m0, out);
  WCMG_CHECK_LAUNCH();
}
template void launch_pack_clover<double>(const cd64*, const int*, long, double, double*, hipStream_t);
template void launch_pack_clover<float>(const cd64*, const int*, long, double, float*, hipStream_t);

template <typename R>
void launch_pack_links(const cd64* U, const int* perm, const int L[4], int antiperiodic, cplx<R>* out,
                       hipStream_t st) {
  long V = (long)L[0] * L[1] * L[2] * L[3];
  long Vs = (long)L[0] * L[1] * L[2];
  hipLaunchKernelGGL(k_pack_links<R>, dim3(nblocks(V)), dim3(kBlock), 0, st, U, perm, V, L[3], Vs, antiperiodic,
                     out);
  WCMG_CHECK_LAUNCH();
}
template void launch_pack_links<double>(const cd64*, const int*, const int*, int, cd64*, hipStream_t);
template void launch_pack_links<float>(const cd64*, const int*, const int*, int, cf32*, hipStream_t);

template <typename Ti, typename To>
void launch_pack_fermion(const cplx<Ti>* in, const int* perm, long V, int nrhs, cplx<To>* out, hipStream_t st) {
  hipLaunchKernelGGL((k_pack_fermion<Ti, To>), dim3(nblocks(V), nrhs), dim3(kBlock), 0, st, in, perm, V, out);
  WCMG_CHECK_LAUNCH();
}
template <typename Ti, typename To>
void launch_unpack_fermion(const cplx<Ti>* in, const int* perm, long V, int nrhs, cplx<To>* out, hipStream_t st) {
  hipLaunchKernelGGL((k_unpack_fermion<Ti, To>), dim3(nblocks(V), nrhs), dim3(kBlock), 0, st, in, perm, V, out);
  WCMG_CHECK_LAUNCH();
}
#define INST_PACK(Ti, To)                                                                                  \
  template void launch_pack_fermion<Ti, To>(const cplx<Ti>*, const int*, long, int, cplx<To>*, hipStream_t); \
  template void launch_unpack_fermion<Ti, To>(const cplx<Ti>*, const int*, long, int, cplx<To>*, hipStream_t);
INST_PACK(double, double)
INST_PACK(double, float)
INST_PACK(float, float)
INST_PACK(float, double)

template <typename R, bool ALL>
static void launch_wilson_t(const cplx<R>* in, cplx<R>* out, const cplx<R>* U, const R* clov, const int* nbr,
                            const SiteGeom* geo, long V, int terms, int nrhs, const int* run, hipStream_t st,
                            cd64* dots, int rs, const cplx<R>* bsub, const cplx<R>* U2) {
  const dim3 grid(item_rhs_grid(nblocks(V, 64), nrhs));
  if (geo && U2)
    WCMG_LAUNCH((k_wilson<R, ALL, true, true>), grid, dim3(kBlock), 0, st, in, out, U2, clov, nbr, *geo, V, terms,
                nrhs, dots, run, rs, bsub);
  else if (geo)
    WCMG_LAUNCH((k_wilson<R, ALL, true, false>), grid, dim3(kBlock), 0, st, in, out, U, clov, nbr, *geo, V, terms,
                nrhs, dots, run, rs, bsub);
  else
    WCMG_LAUNCH((k_wilson<R, ALL, false, false>), grid, dim3(kBlock), 0, st, in, out, U, clov, nbr, SiteGeom(), V,
                terms, nrhs, dots, run, rs, bsub);
}

template <typename R>
void launch_wilson(const cplx<R>* in, cplx<R>* out, const cplx<R>* U, const R* clov, const int* nbr, long V,
                   int terms, int nrhs, const int* run, hipStream_t st, cd64* dots, int rs, const cplx<R>* bsub,
                   const SiteGeom* geo, const cplx<R>* U2) {
  require(!bsub || (!dots && terms == 0x1ff), WCMG_ERR_ARG, "Dslash: the residual form takes the whole operator");
  require(!geo || V < (1L << 31), WCMG_ERR_DIMS, "Dslash: lattice too large for 32-bit site arithmetic");
  if (terms == 0x1ff)
    launch_wilson_t<R, true>(in, out, U, clov, nbr, geo, V, terms, nrhs, run, st, dots, rs, bsub, U2);
  else
    launch_wilson_t<R, false>(in, out, U, clov, nbr, geo, V, terms, nrhs, run, st, dots, rs, bsub, U2);
  WCMG_CHECK_LAUNCH();
}
template void launch_wilson<double>(const cd64*, cd64*, const cd64*, const double*, const int*, long, int, int,
                                    const int*, hipStream_t, cd64*, int, const cd64*, const SiteGeom*, const cd64*);
template void launch_wilson<float>(const cf32*, cf32*, const cf32*, const float*, const int*, long, int, int,
                                   const int*, hipStream_t, cd64*, int, const cf32*, const SiteGeom*, const cf32*);

// Two-row link storage (the Dslash's): rows 0 and 1 of every U_mu(s), device
// site order, the antiperiodic sign folded in as in k_pack_links, in 16-byte
// chunks [mu][6/K][V][K] of K = 16 / sizeof(cplx<R>) complex values.
template <typename R>
__global__ void k_pack_links2(const cd64* __restrict__ U, const int* __restrict__ perm, long V, int Lt, long Vs,
                              int antiperiodic, cplx<R>* __restrict__ out) {
  constexpr int K = 16 / sizeof(cplx<R>);
  const long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= V) return;
  const long x = perm[s];
  const bool last_t = (x / Vs) == Lt - 1;
  for (int mu = 0; mu < 4; ++mu) {
    const double sg = (mu == 3 && antiperiodic && last_t) ? -1.0 : 1.0;
    for (int e = 0; e < 6; ++e) {
      const cd64 u = U[(x * 4 + mu) * 9 + e];
      out[((long)(mu * (6 / K) + e / K) * V + s) * K + e % K] = mkc((R)(sg * u.re), (R)(sg * u.im));
    }
  }
}

// Largest deviation of row 2 from conj(row0 x row1) over the links in each
// block of 256 (0 for SU(3) links up to rounding); part[blockIdx.x].
__global__ void k_su3_defect(const cd64* __restrict__ U, long n_links, double* __restrict__ part) {
  __shared__ double red[kBlock / 64];
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  double d = 0.0;
  if (e < n_links) {
    const cd64* u = U + e * 9;
    const cd64 r2[3] = {cconj(csub(cmul(u[1], u[5]), cmul(u[2], u[4]))),
                        cconj(csub(cmul(u[2], u[3]), cmul(u[0], u[5]))),
                        cconj(csub(cmul(u[0], u[4]), cmul(u[1], u[3])))};
    for (int c = 0; c < 3; ++c) {
      const cd64 t = csub(u[6 + c], r2[c]);
      d = fmax(d, fmax(fabs(t.re), fabs(t.im)));
    }
  }
  for (int off = 32; off > 0; off >>= 1) d = fmax(d, __shfl_xor(d, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = d;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) m = fmax(m, red[w]);
    part[blockIdx.x] = m;
  }
}

template <typename R>
void launch_pack_links2(const cd64* U, const int* perm, const int L[4], int antiperiodic, cplx<R>* out,
                        hipStream_t st) {
  const long V = (long)L[0] * L[1] * L[2] * L[3];
  const long Vs = (long)L[0] * L[1] * L[2];
  hipLaunchKernelGGL(k_pack_links2<R>, dim3(nblocks(V)), dim3(kBlock), 0, st, U, perm, V, L[3], Vs, antiperiodic,
                     out);
  WCMG_CHECK_LAUNCH();
}
template void launch_pack_links2<double>(const cd64*, const int*, const int*, int, cd64*, hipStream_t);
template void launch_pack_links2<float>(const cd64*, const int*, const int*, int, cf32*, hipStream_t);

int su3_defect_blocks(long n_links) { return (int)nblocks(n_links); }
void launch_su3_defect(const cd64* U, long n_links, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_su3_defect, dim3(nblocks(n_links)), dim3(kBlock), 0, st, U, n_links, part);
  WCMG_CHECK_LAUNCH();
}

int wilson_blocks(long V) { return (int)nblocks(V, 64); }

KernelTiming& kernel_timing() {
  static thread_local KernelTiming slot;
  return slot;
}

void launch_wilson_mrhs(const cf32* in, cf32* out, const cf32* U, const float* clov, const int* nbr, long V, int nrhs,
                        const int* run, int rs, cd64* dots, hipStream_t st) {
  require(12L * V * 8 < (1L << 31), WCMG_ERR_DIMS, "multi-RHS Dslash: field exceeds the 2 GiB buffer range");
  require(nrhs >= 1 && nrhs <= 64, WCMG_ERR_ARG, "multi-RHS Dslash takes 1..64 right-hand sides");
  // waves per workgroup: at most 8, as few as keep every wave's share equal
  const int per = (nrhs + 7) / 8;
  const int nw = (nrhs + per - 1) / per;
  WCMG_LAUNCH(k_wilson_mrhs, dim3(nblocks(V, 64)), dim3(64 * nw), 0, st, in, out, U, clov, nbr, V, nrhs, dots, run,
              rs);
  WCMG_CHECK_LAUNCH();
}

}  // namespace wcmg
