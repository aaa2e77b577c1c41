// Site-local pieces of the Wilson-clover operator (Sec. 2.1, "Dirac
// operator"), shared by the Dslash kernels and the Galerkin coarsening:
// spin projection and reconstruction of a hop, the hop itself, and the
// chirality blocks of (4 + m0) + C.  Chiral basis, component k = 3*spin + colour.
#pragma once

#include <type_traits>

#include "kernels.h"

namespace wcmg {

// Spin projection in the chiral basis.  For a hop in direction +mu the spinor
// (1 - gamma_mu) psi has upper half h and lower half fixed by h; for -mu,
// (1 + gamma_mu) psi.  Only h (2 spins x 3 colours) is transported by U.
template <typename R, int MU, bool FWD>
__device__ inline void project(const cplx<R> (&p)[12], cplx<R> (&h)[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cplx<R> p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
    if (MU == 0) {  // x: i sigma_1
      h[c] = FWD ? cadd(p0, ci(p3)) : csub(p0, ci(p3));
      h[3 + c] = FWD ? cadd(p1, ci(p2)) : csub(p1, ci(p2));
    } else if (MU == 1) {  // y: i sigma_2 = [[0,1],[-1,0]]
      h[c] = FWD ? cadd(p0, p3) : csub(p0, p3);
      h[3 + c] = FWD ? csub(p1, p2) : cadd(p1, p2);
    } else if (MU == 2) {  // z: i sigma_3
      h[c] = FWD ? cadd(p0, ci(p2)) : csub(p0, ci(p2));
      h[3 + c] = FWD ? csub(p1, ci(p3)) : cadd(p1, ci(p3));
    } else {  // t
      h[c] = FWD ? csub(p0, p2) : cadd(p0, p2);
      h[3 + c] = FWD ? csub(p1, p3) : cadd(p1, p3);
    }
  }
}

// acc += -1/2 * reconstruct(h)
template <typename R, int MU, bool FWD>
__device__ inline void reconstruct_add(cplx<R> (&acc)[12], const cplx<R> (&h)[6]) {
  const R m = (R)-0.5;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cplx<R> h0 = h[c], h1 = h[3 + c], l2, l3;
    if (MU == 0) {
      l2 = FWD ? cneg(ci(h1)) : ci(h1);
      l3 = FWD ? cneg(ci(h0)) : ci(h0);
    } else if (MU == 1) {
      l2 = FWD ? cneg(h1) : h1;
      l3 = FWD ? h0 : cneg(h0);
    } else if (MU == 2) {
      l2 = FWD ? cneg(ci(h0)) : ci(h0);
      l3 = FWD ? ci(h1) : cneg(ci(h1));
    } else {
      l2 = FWD ? cneg(h0) : h0;
      l3 = FWD ? cneg(h1) : h1;
    }
    acc[c] = cadd(acc[c], cscale(m, h0));
    acc[3 + c] = cadd(acc[3 + c], cscale(m, h1));
    acc[6 + c] = cadd(acc[6 + c], cscale(m, l2));
    acc[9 + c] = cadd(acc[9 + c], cscale(m, l3));
  }
}

// acc += the hop term along (MU, FWD) for neighbour spinor p and link u
// (u = U_mu(x) for +mu, U_mu(x - mu) for -mu, whose adjoint is applied).
template <typename R, int MU, bool FWD>
__device__ inline void hop_core(cplx<R> (&acc)[12], const cplx<R> (&p)[12], const cplx<R> (&u)[9]) {
  cplx<R> h[6];
  project<R, MU, FWD>(p, h);
  cplx<R> g[6];
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cplx<R> t = mkc((R)0, (R)0);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (FWD) cfma(t, u[a * 3 + b], h[sp * 3 + b]);
        else cfmac(t, u[b * 3 + a], h[sp * 3 + b]);  // (U^dag)_{ab} = conj(U_{ba})
      }
      g[sp * 3 + a] = t;
    }
  reconstruct_add<R, MU, FWD>(acc, g);
}

// The hop along (MU, FWD) from the neighbour site y of s.
template <typename R, int MU, bool FWD>
__device__ inline void hop_at(cplx<R> (&acc)[12], const cplx<R>* __restrict__ in, const cplx<R>* __restrict__ U,
                              long V, long s, long y) {
  cplx<R> p[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) p[k] = in[(long)k * V + y];
  const long ls = FWD ? s : y;
  cplx<R> u[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = U[(long)(MU * 9 + e) * V + ls];
  hop_core<R, MU, FWD>(acc, p, u);
}

// The hop from the neighbour site y of s with two-row link storage: rows 0
// and 1 of U in 16-byte chunks ([mu][6/K][V][K], K complex per chunk), row 2
// rebuilt as conj(row0 x row1) (U in SU(3)) times sg, the sign that the
// packing folded into rows 0 and 1 (the antiperiodic t boundary).
template <typename R, int MU, bool FWD>
__device__ inline void hop_at2(cplx<R> (&acc)[12], const cplx<R>* __restrict__ in, const cplx<R>* __restrict__ U2,
                               long V, long s, long y, R sg) {
  cplx<R> p[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) p[k] = in[(long)k * V + y];
  const long ls = FWD ? s : y;
  cplx<R> u[9];
  if constexpr (sizeof(R) == 4) {
    const float4* q = (const float4*)U2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float4 f = q[(long)(MU * 3 + c) * V + ls];
      u[2 * c] = mkc(f.x, f.y);
      u[2 * c + 1] = mkc(f.z, f.w);
    }
  } else {
#pragma unroll
    for (int e = 0; e < 6; ++e) u[e] = U2[(long)(MU * 6 + e) * V + ls];
  }
  u[6] = cscale(sg, cconj(csub(cmul(u[1], u[5]), cmul(u[2], u[4]))));
  u[7] = cscale(sg, cconj(csub(cmul(u[2], u[3]), cmul(u[0], u[5]))));
  u[8] = cscale(sg, cconj(csub(cmul(u[0], u[4]), cmul(u[1], u[3]))));
  hop_core<R, MU, FWD>(acc, p, u);
}

template <typename R, int MU, bool FWD>
__device__ inline void hop(cplx<R> (&acc)[12], const cplx<R>* __restrict__ in, const cplx<R>* __restrict__ U,
                           const int* __restrict__ nbr, long V, long s) {
  hop_at<R, MU, FWD>(acc, in, U, V, s, nbr[(long)(2 * MU + (FWD ? 0 : 1)) * V + s]);
}

// acc[chi*6 .. chi*6+5] += (block chi of (4 + m0) + C) p, block given by its
// 36 packed reals e (6 diagonal entries, then the 15 entries below the diagonal).
template <typename R, int chi>
__device__ inline void clover_block_apply(cplx<R> (&acc)[12], const R (&e)[36], const cplx<R> (&p)[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) acc[chi * 6 + i] = cadd(acc[chi * 6 + i], cscale(e[i], p[i]));
  int idx = 0;
#pragma unroll
  for (int i = 1; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < i; ++j, ++idx) {
      const cplx<R> a = mkc(e[6 + 2 * idx], e[7 + 2 * idx]);
      cfma(acc[chi * 6 + i], a, p[j]);
      cfmac(acc[chi * 6 + j], a, p[i]);
    }
}

// Clover block of chirality chi applied to p (the six components of that
// chirality at site s, already loaded).
template <typename R, int chi>
__device__ inline void clover_chirality_p(cplx<R> (&acc)[12], const cplx<R> (&p)[6], const R* __restrict__ clov,
                                          long V, long s) {
  constexpr int RC = 16 / sizeof(R);
  typedef typename std::conditional<sizeof(R) == 4, float4, double2>::type V16;
  R e[36];
  const V16* cb = (const V16*)(clov + (long)chi * 36 * V);
#pragma unroll
  for (int q = 0; q < 36 / RC; ++q) {
    V16 c = cb[(long)q * V + s];
    if constexpr (RC == 4) {
      e[q * 4 + 0] = c.x;
      e[q * 4 + 1] = c.y;
      e[q * 4 + 2] = c.z;
      e[q * 4 + 3] = c.w;
    } else {
      e[q * 2 + 0] = c.x;
      e[q * 2 + 1] = c.y;
    }
  }
  clover_block_apply<R, chi>(acc, e, p);
}

template <typename R, int chi>
__device__ inline void clover_chirality(cplx<R> (&acc)[12], const cplx<R>* __restrict__ in,
                                        const R* __restrict__ clov, long V, long s) {
  constexpr int RC = 16 / sizeof(R);
  typedef typename std::conditional<sizeof(R) == 4, float4, double2>::type V16;
  R e[36];
  const V16* cb = (const V16*)(clov + (long)chi * 36 * V);
#pragma unroll
  for (int q = 0; q < 36 / RC; ++q) {
    V16 c = cb[(long)q * V + s];
    if constexpr (RC == 4) {
      e[q * 4 + 0] = c.x;
      e[q * 4 + 1] = c.y;
      e[q * 4 + 2] = c.z;
      e[q * 4 + 3] = c.w;
    } else {
      e[q * 2 + 0] = c.x;
      e[q * 2 + 1] = c.y;
    }
  }
  cplx<R> p[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) p[k] = in[(long)(chi * 6 + k) * V + s];
  clover_block_apply<R, chi>(acc, e, p);
}

}  // namespace wcmg
