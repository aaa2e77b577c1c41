// Learned near-null proposal: kernels of the gauge-covariant network of
// parallel-transport convolutions, its least-squares loss against near-null
// vectors, the backward pass and the Adam update.
//
// Layer:  z_o(x) = sum_{h, i} W[h][o][i] (T_h a_i)(x),  h = 0 the site itself,
// h = 2 mu + 1 the hop from x + mu through U_mu(x), h = 2 mu + 2 the hop from
// x - mu through U_mu(x - mu)^dag (the packed links carry the fermion boundary
// sign, so the hops see the same boundary as the Dslash).  Weights act on
// channels only, so the map commutes with gauge transformations.  Hidden
// layers squash each channel site by site: a = z / sqrt(1 + |z(x)|^2).
//
// Fields are [channel][12][V] in the device site order of level 0.  Hidden
// activations are stored in BF16 (or FP32), weights and all accumulation are
// FP32; the loss is reduced in FP64.
//
// The channel contraction runs on the matrix cores: for 16 sites and one
// spin-colour component, sum_{(h,i)} W[h][o][i] t_{h,i}(x) is a 16 x 16 x 4 FP32
// MFMA over K = (hop, input channel), whose B operand (one component of a
// transported input channel) each lane computes itself.  Complex arithmetic by
// the real embedding: four real MFMAs per complex product.
#include "kernels.h"

namespace wcmg {

namespace {
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline f32x4 mfma4(float a, float b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

template <typename T>
__device__ inline cf32 act_ld(const T* p, long i);
template <>
__device__ inline cf32 act_ld<cf32>(const cf32* p, long i) {
  return p[i];
}
template <>
__device__ inline cf32 act_ld<uint32_t>(const uint32_t* p, long i) {
  const uint32_t w = p[i];
  return mkc(__builtin_bit_cast(float, w << 16), __builtin_bit_cast(float, w & 0xffff0000u));
}
__device__ inline void act_st(cf32* p, long i, cf32 v) { p[i] = v; }
__device__ inline void act_st(uint32_t* p, long i, cf32 v) {
  p[i] = (uint32_t)f32_to_bf16(v.re) | ((uint32_t)f32_to_bf16(v.im) << 16);
}

// (T_h a)(s), 12 components, for channel field a = [12][V]
template <typename T>
__device__ inline void transported(const T* __restrict__ a, int h, long s, const cf32* __restrict__ U,
                                   const int* __restrict__ nbr, long V, cf32 (&t)[12]) {
  if (h == 0) {
#pragma unroll
    for (int k = 0; k < 12; ++k) t[k] = act_ld(a, (long)k * V + s);
    return;
  }
  const long y = nbr[(long)(h - 1) * V + s];
  const int mu = (h - 1) >> 1;
  const bool fwd = (h & 1) != 0;
  cf32 p[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) p[k] = act_ld(a, (long)k * V + y);
  const long ls = fwd ? s : y;
  cf32 u[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = U[(long)(mu * 9 + e) * V + ls];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cf32 acc = mkc(0.f, 0.f);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (fwd) cfma(acc, u[c * 3 + b], p[sp * 3 + b]);
        else cfmac(acc, u[b * 3 + c], p[sp * 3 + b]);  // (U^dag)_{cb} = conj(U_{bc})
      }
      t[sp * 3 + c] = acc;
    }
}
}  // namespace

// One layer (or, with the adjoint weights, the input gradient of one):
// out_o = sum_{h,i} W[h][o][i] T_h in_i; with squash, out = z / s and
// scale_o(x) = s = sqrt(1 + |z_o(x)|^2).  Cin % 4 == 0.  Wave = 16 sites.
template <typename TI, typename TO>
__global__ void __launch_bounds__(256) k_nn_layer(const TI* __restrict__ in, int Cin, const cf32* __restrict__ W,
                                                   int Cout, TO* __restrict__ out, float* __restrict__ scale,
                                                   int squash, const cf32* __restrict__ U,
                                                   const int* __restrict__ nbr, long V) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, k = lane >> 4;
  const long s0 = ((long)blockIdx.x * 4 + wave) * 16;
  if (s0 >= V) return;
  const bool valid = s0 + j < V;
  const long s = valid ? s0 + j : V - 1;  // in-bounds stand-in for tail lanes
  const int nsteps = 9 * Cin / 4;
  for (int mb = 0; mb * 16 < Cout; ++mb) {
    f32x4 acc[12][2];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c][0] = acc[c][1] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int oa = 16 * mb + j;  // A-operand row of this lane
    for (int q = 0; q < nsteps; ++q) {
      const int kk = 4 * q + k;
      const int h = kk / Cin, i = kk - h * Cin;
      cf32 t[12];
      transported<TI>(in + (long)i * 12 * V, h, s, U, nbr, V, t);
      const cf32 w = oa < Cout ? W[((long)h * Cout + oa) * Cin + i] : mkc(0.f, 0.f);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        acc[c][0] = mfma4(w.re, t[c].re, acc[c][0]);
        acc[c][0] = mfma4(-w.im, t[c].im, acc[c][0]);
        acc[c][1] = mfma4(w.im, t[c].re, acc[c][1]);
        acc[c][1] = mfma4(w.re, t[c].im, acc[c][1]);
      }
    }
    // this lane holds z[o = 16 mb + 4 k + r][site s0 + j], r < 4
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = 16 * mb + 4 * k + r;
      float n2 = 0.f;
#pragma unroll
      for (int c = 0; c < 12; ++c) n2 += acc[c][0][r] * acc[c][0][r] + acc[c][1][r] * acc[c][1][r];
      const float sc = squash ? sqrtf(1.f + n2) : 1.f;
      const float inv = 1.f / sc;
      if (valid && o < Cout) {
#pragma unroll
        for (int c = 0; c < 12; ++c) act_st(out, ((long)o * 12 + c) * V + s, mkc(acc[c][0][r] * inv, acc[c][1][r] * inv));
        if (squash && scale) scale[(long)o * V + s] = sc;
      }
    }
  }
}

// Weight gradient partials for hop h = blockIdx.y:
//   part[h][blk][o][i] = sum over the block's sites x and components c of
//                        g_o(x, c) conj((T_h a_i)(x, c)).
// M = o, N = i, K = (site, component); 4 sites per MFMA step, one component
// per instruction.  Block partials are combined in LDS in a fixed wave order.
template <typename TI>
__global__ void __launch_bounds__(256) k_nn_wgrad(const cf32* __restrict__ g, int Cout, const TI* __restrict__ a,
                                                   int Cin, const cf32* __restrict__ U, const int* __restrict__ nbr,
                                                   long V, long chunk, cd64* __restrict__ part) {
  __shared__ cf32 red[4][32][32];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 15, k = lane >> 4;
  const int h = blockIdx.y;
  const long lo = blockIdx.x * chunk, hi = min(V, lo + chunk);
  const int nmb = (Cout + 15) / 16, nnb = (Cin + 15) / 16;
  f32x4 acc[2][2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y][0] = acc[x][y][1] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (long base = lo + 4 * wave; base < hi; base += 16) {
    const long x = base + k;
    const bool vx = x < hi;
    const long xs = vx ? x : lo;
    cf32 t[2][12], gv[2][12];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      const int i = 16 * nb + n;
      if (nb < nnb && i < Cin && vx) {
        transported<TI>(a + (long)i * 12 * V, h, xs, U, nbr, V, t[nb]);
      } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) t[nb][c] = mkc(0.f, 0.f);
      }
    }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      const int o = 16 * mb + n;
#pragma unroll
      for (int c = 0; c < 12; ++c)
        gv[mb][c] = (mb < nmb && o < Cout && vx) ? g[((long)o * 12 + c) * V + xs] : mkc(0.f, 0.f);
    }
#pragma unroll
    for (int c = 0; c < 12; ++c)
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          if (mb >= nmb || nb >= nnb) continue;
          acc[mb][nb][0] = mfma4(gv[mb][c].re, t[nb][c].re, acc[mb][nb][0]);
          acc[mb][nb][0] = mfma4(gv[mb][c].im, t[nb][c].im, acc[mb][nb][0]);
          acc[mb][nb][1] = mfma4(gv[mb][c].im, t[nb][c].re, acc[mb][nb][1]);
          acc[mb][nb][1] = mfma4(-gv[mb][c].re, t[nb][c].im, acc[mb][nb][1]);
        }
  }
  // D[o][i]: o = 16 mb + 4 k + r, i = 16 nb + n
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave][16 * mb + 4 * k + r][16 * nb + n] = mkc(acc[mb][nb][0][r], acc[mb][nb][1][r]);
  __syncthreads();
  for (int e = threadIdx.x; e < Cout * Cin; e += blockDim.x) {
    const int o = e / Cin, i = e - o * Cin;
    cd64 sum = mkc(0.0, 0.0);
#pragma unroll
    for (int w = 0; w < 4; ++w) sum = cadd(sum, mkc((double)red[w][o][i].re, (double)red[w][o][i].im));
    part[(((long)h * gridDim.x + blockIdx.x) * Cout + o) * Cin + i] = sum;
  }
}

// gW[h][o][i] = sum_b part[h][b][o][i] (fixed order, FP64) as FP32
__global__ void k_nn_wgrad_reduce(const cd64* __restrict__ part, int G, int n_oi, cf32* __restrict__ gW) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;  // over 9 * n_oi
  if (e >= 9L * n_oi) return;
  const long h = e / n_oi, oi = e - h * n_oi;
  cd64 s = mkc(0.0, 0.0);
  for (int b = 0; b < G; ++b) s = cadd(s, part[(h * G + b) * n_oi + oi]);
  gW[e] = mkc((float)s.re, (float)s.im);
}

// dL/dz* = (dL/da* - a Re<dL/da*, a>) / s, in place on g; one thread per (channel, site)
template <typename TI>
__global__ void k_nn_squash_bwd(cf32* __restrict__ g, const TI* __restrict__ a, const float* __restrict__ scale,
                                int C, long V) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)C * V) return;
  const long o = e / V, s = e - o * V;
  cf32 gv[12], av[12];
  float re = 0.f;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    gv[c] = g[(o * 12 + c) * V + s];
    av[c] = act_ld(a, (o * 12 + c) * V + s);
    re += gv[c].re * av[c].re + gv[c].im * av[c].im;
  }
  const float inv = 1.f / scale[o * V + s];
#pragma unroll
  for (int c = 0; c < 12; ++c)
    g[(o * 12 + c) * V + s] = mkc((gv[c].re - av[c].re * re) * inv, (gv[c].im - av[c].im * re) * inv);
}

// Loss and dL/dY* block by block: workgroup b = (aggregate b / 2, chirality b % 2).
// Rows of the block: (site of the aggregate, the two spins of the chirality,
// colour).  G = Y^dag Y and B = Y^dag T are formed over row tiles staged in LDS
// (FP64 sums), c = G^-1 B by Cholesky in FP64, then per row r = T - Y c,
// loss += |r|^2 and gY = -(r c^dag) / norm.
constexpr int kNnMaxV = 16;
__global__ void __launch_bounds__(256) k_nn_loss(const cf32* __restrict__ Y, const cf32* __restrict__ T, int nv,
                                                  const int* __restrict__ agg_sites, int A, long V, double norm,
                                                  cf32* __restrict__ gY, double* __restrict__ loss_part) {
  __shared__ cf32 ty[64][kNnMaxV], tt[64][kNnMaxV];
  __shared__ cd64 Gm[kNnMaxV][kNnMaxV], Bm[kNnMaxV][kNnMaxV], cm[kNnMaxV][kNnMaxV];
  __shared__ double red[4];
  __shared__ int bad;
  const int agg = blockIdx.x >> 1, chi = blockIdx.x & 1;
  const int rows = 6 * A;
  const int tid = threadIdx.x;
  auto row_elem = [&](int r, long* site, int* comp) {
    const int o = r / 6, w = r - 6 * o;
    *site = agg_sites[(long)agg * A + o];
    *comp = (2 * chi + w / 3) * 3 + w % 3;
  };
  // entries e < 2 nv^2: (which, a, b)
  cd64 accs[2] = {mkc(0.0, 0.0), mkc(0.0, 0.0)};
  const int ne = 2 * nv * nv;
  for (int r0 = 0; r0 < rows; r0 += 64) {
    const int nr = min(64, rows - r0);
    __syncthreads();
    for (int q = tid; q < nr * nv; q += blockDim.x) {
      const int rr = q / nv, jj = q - rr * nv;
      long site;
      int comp;
      row_elem(r0 + rr, &site, &comp);
      ty[rr][jj] = Y[((long)jj * 12 + comp) * V + site];
      tt[rr][jj] = T[((long)jj * 12 + comp) * V + site];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = tid + u * blockDim.x;
      if (e >= ne) continue;
      const int which = e / (nv * nv), ab = e - which * nv * nv, a = ab / nv, b = ab - a * nv;
      double sr = 0.0, si = 0.0;
      for (int rr = 0; rr < nr; ++rr) {
        const cf32 x = ty[rr][a];
        const cf32 y = which ? tt[rr][b] : ty[rr][b];
        sr += (double)x.re * y.re + (double)x.im * y.im;
        si += (double)x.re * y.im - (double)x.im * y.re;
      }
      accs[u] = cadd(accs[u], mkc(sr, si));
    }
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = tid + u * blockDim.x;
    if (e >= ne) continue;
    const int which = e / (nv * nv), ab = e - which * nv * nv, a = ab / nv, b = ab - a * nv;
    if (which) Bm[a][b] = accs[u];
    else Gm[a][b] = accs[u];
  }
  __syncthreads();
  if (tid == 0) {
    // Cholesky G = L L^dag in place (lower triangle), then c = G^-1 B
    bad = 0;
    for (int p = 0; p < nv; ++p) {
      double d = Gm[p][p].re;
      for (int q = 0; q < p; ++q) d -= Gm[p][q].re * Gm[p][q].re + Gm[p][q].im * Gm[p][q].im;
      if (!(d > 0.0)) {
        bad = 1;
        break;
      }
      d = sqrt(d);
      Gm[p][p] = mkc(d, 0.0);
      for (int r = p + 1; r < nv; ++r) {
        cd64 v = Gm[r][p];
        for (int q = 0; q < p; ++q) v = csub(v, cmul(Gm[r][q], cconj(Gm[p][q])));
        Gm[r][p] = mkc(v.re / d, v.im / d);
      }
    }
    if (!bad)
      for (int b = 0; b < nv; ++b) {
        cd64 z[kNnMaxV];
        for (int p = 0; p < nv; ++p) {  // L z = B_b
          cd64 v = Bm[p][b];
          for (int q = 0; q < p; ++q) v = csub(v, cmul(Gm[p][q], z[q]));
          z[p] = mkc(v.re / Gm[p][p].re, v.im / Gm[p][p].re);
        }
        for (int p = nv - 1; p >= 0; --p) {  // L^dag c = z
          cd64 v = z[p];
          for (int q = p + 1; q < nv; ++q) v = csub(v, cmul(cconj(Gm[q][p]), cm[q][b]));
          cm[p][b] = mkc(v.re / Gm[p][p].re, v.im / Gm[p][p].re);
        }
      }
  }
  __syncthreads();
  double lsum = 0.0;
  if (!bad) {
    for (int r = tid; r < rows; r += blockDim.x) {
      long site;
      int comp;
      row_elem(r, &site, &comp);
      cf32 y[kNnMaxV];
      cd64 res[kNnMaxV];
      for (int a = 0; a < nv; ++a) y[a] = Y[((long)a * 12 + comp) * V + site];
      for (int jj = 0; jj < nv; ++jj) {
        const cf32 t = T[((long)jj * 12 + comp) * V + site];
        cd64 v = mkc((double)t.re, (double)t.im);
        for (int a = 0; a < nv; ++a) v = csub(v, cmul(mkc((double)y[a].re, (double)y[a].im), cm[a][jj]));
        res[jj] = v;
        lsum += v.re * v.re + v.im * v.im;
      }
      for (int a = 0; a < nv; ++a) {
        cd64 gsum = mkc(0.0, 0.0);
        for (int jj = 0; jj < nv; ++jj) gsum = cadd(gsum, cmul(res[jj], cconj(cm[a][jj])));
        gY[((long)a * 12 + comp) * V + site] = mkc((float)(-gsum.re / norm), (float)(-gsum.im / norm));
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = lsum;
  __syncthreads();
  if (tid == 0) loss_part[blockIdx.x] = bad ? __builtin_nan("") : (red[0] + red[1] + red[2] + red[3]);
}

// Adam on the real parameters (re, im of every weight); grad = 2 * dL/dW*.
__global__ void k_nn_adam(float* __restrict__ w, const cf32* __restrict__ gW, float* __restrict__ m,
                          float* __restrict__ v, long n_complex, float lr, float b1, float b2, float eps, float c1,
                          float c2) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= 2 * n_complex) return;
  const cf32 gc = gW[e >> 1];
  const float g = 2.f * ((e & 1) ? gc.im : gc.re);
  const float mm = b1 * m[e] + (1.f - b1) * g;
  const float vv = b2 * v[e] + (1.f - b2) * g * g;
  m[e] = mm;
  v[e] = vv;
  w[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// Wadj[h][i][o] = conj(W[adj(h)][o][i]) (adjoint hop: +mu <-> -mu)
__global__ void k_nn_adjoint_weights(const cf32* __restrict__ W, int Cout, int Cin, cf32* __restrict__ Wadj) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= 9L * Cout * Cin) return;
  const int h = (int)(e / ((long)Cin * Cout));
  const long r = e - (long)h * Cin * Cout;
  const int i = (int)(r / Cout), o = (int)(r - (long)i * Cout);
  const int ha = h == 0 ? 0 : ((h & 1) ? h + 1 : h - 1);
  Wadj[e] = cconj(W[((long)ha * Cout + o) * Cin + i]);
}

// FP64 fields -> activation storage, and FP32 fields -> FP64
template <typename TO>
__global__ void k_nn_from64(const cd64* __restrict__ x, TO* __restrict__ y, long n) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e < n) act_st(y, e, mkc((float)x[e].re, (float)x[e].im));
}
__global__ void k_nn_to64(const cf32* __restrict__ x, cd64* __restrict__ y, long n) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e < n) y[e] = mkc((double)x[e].re, (double)x[e].im);
}

// ---------------------------------------------------------------- launchers
void launch_nn_layer(int act_bits_in, const void* in, int Cin, const cf32* W, int Cout, int act_bits_out, void* out,
                     float* scale, int squash, const cf32* U, const int* nbr, long V, hipStream_t st) {
  require(Cin % 4 == 0 && Cin >= 4 && Cout >= 1 && Cout <= 32, WCMG_ERR_ARG,
          "network layer: input channels a multiple of 4, at most 32 output channels");
  const dim3 g((unsigned)((V + 63) / 64)), b(kBlock);
  if (act_bits_in == 16 && act_bits_out == 16)
    hipLaunchKernelGGL((k_nn_layer<uint32_t, uint32_t>), g, b, 0, st, (const uint32_t*)in, Cin, W, Cout,
                       (uint32_t*)out, scale, squash, U, nbr, V);
  else if (act_bits_in == 16)
    hipLaunchKernelGGL((k_nn_layer<uint32_t, cf32>), g, b, 0, st, (const uint32_t*)in, Cin, W, Cout, (cf32*)out,
                       scale, squash, U, nbr, V);
  else
    hipLaunchKernelGGL((k_nn_layer<cf32, cf32>), g, b, 0, st, (const cf32*)in, Cin, W, Cout, (cf32*)out, scale,
                       squash, U, nbr, V);
  WCMG_CHECK_LAUNCH();
}

int nn_wgrad_blocks(long V) { return (int)std::min<long>(1024, std::max<long>(1, (V + 255) / 256)); }

void launch_nn_wgrad(const cf32* g, int Cout, int act_bits, const void* a, int Cin, const cf32* U, const int* nbr,
                     long V, cd64* part, cf32* gW, hipStream_t st) {
  require(Cout <= 32 && Cin <= 32, WCMG_ERR_ARG, "network layer: at most 32 channels");
  const int G = nn_wgrad_blocks(V);
  const long chunk = ((V + G - 1) / G + 15) / 16 * 16;
  if (act_bits == 16)
    hipLaunchKernelGGL(k_nn_wgrad<uint32_t>, dim3(G, 9), dim3(kBlock), 0, st, g, Cout, (const uint32_t*)a, Cin, U,
                       nbr, V, chunk, part);
  else
    hipLaunchKernelGGL(k_nn_wgrad<cf32>, dim3(G, 9), dim3(kBlock), 0, st, g, Cout, (const cf32*)a, Cin, U, nbr, V,
                       chunk, part);
  WCMG_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_nn_wgrad_reduce, dim3(nblocks(9L * Cout * Cin)), dim3(kBlock), 0, st, part, G, Cout * Cin, gW);
  WCMG_CHECK_LAUNCH();
}

void launch_nn_squash_bwd(cf32* g, int act_bits, const void* a, const float* scale, int C, long V, hipStream_t st) {
  if (act_bits == 16)
    hipLaunchKernelGGL(k_nn_squash_bwd<uint32_t>, dim3(nblocks((long)C * V)), dim3(kBlock), 0, st, g,
                       (const uint32_t*)a, scale, C, V);
  else
    hipLaunchKernelGGL(k_nn_squash_bwd<cf32>, dim3(nblocks((long)C * V)), dim3(kBlock), 0, st, g, (const cf32*)a,
                       scale, C, V);
  WCMG_CHECK_LAUNCH();
}

void launch_nn_loss(const cf32* Y, const cf32* T, int nv, const int* agg_sites, int A, long Vc, long V, double norm,
                    cf32* gY, double* loss_part, hipStream_t st) {
  require(nv >= 1 && nv <= kNnMaxV && 6 * A >= nv, WCMG_ERR_ARG, "network loss: 1..16 vectors, aggregates of 6 A >= nv rows");
  hipLaunchKernelGGL(k_nn_loss, dim3((unsigned)(2 * Vc)), dim3(kBlock), 0, st, Y, T, nv, agg_sites, A, V, norm, gY,
                     loss_part);
  WCMG_CHECK_LAUNCH();
}

void launch_nn_adam(float* w, const cf32* gW, float* m, float* v, long n_complex, float lr, int step, hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_nn_adam, dim3(nblocks(2 * n_complex)), dim3(kBlock), 0, st, w, gW, m, v, n_complex, lr, b1, b2,
                     1e-8f, c1, c2);
  WCMG_CHECK_LAUNCH();
}

void launch_nn_adjoint_weights(const cf32* W, int Cout, int Cin, cf32* Wadj, hipStream_t st) {
  hipLaunchKernelGGL(k_nn_adjoint_weights, dim3(nblocks(9L * Cout * Cin)), dim3(kBlock), 0, st, W, Cout, Cin, Wadj);
  WCMG_CHECK_LAUNCH();
}

void launch_nn_from64(const cd64* x, int act_bits, void* y, long n, hipStream_t st) {
  if (act_bits == 16)
    hipLaunchKernelGGL(k_nn_from64<uint32_t>, dim3(nblocks(n)), dim3(kBlock), 0, st, x, (uint32_t*)y, n);
  else
    hipLaunchKernelGGL(k_nn_from64<cf32>, dim3(nblocks(n)), dim3(kBlock), 0, st, x, (cf32*)y, n);
  WCMG_CHECK_LAUNCH();
}

void launch_nn_to64(const cf32* x, cd64* y, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_nn_to64, dim3(nblocks(n)), dim3(kBlock), 0, st, x, y, n);
  WCMG_CHECK_LAUNCH();
}

}  // namespace wcmg
