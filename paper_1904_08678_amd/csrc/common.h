// Shared device helpers of the wcmg HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "wcmg.h"

namespace wcmg {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define WCMG_HIP(call)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::wcmg::Error(e_ == hipErrorOutOfMemory ? WCMG_ERR_NOMEM : WCMG_ERR_HIP,   \
                          std::string(#call) + ": " + hipGetErrorString(e_));           \
  } while (0)

#define WCMG_CHECK_LAUNCH() WCMG_HIP(hipGetLastError())

inline void require(bool ok, int code, const std::string& msg) {
  if (!ok) throw Error(code, msg);
}

// ---------------------------------------------------------------- complex
template <typename R>
struct alignas(2 * sizeof(R)) cplx {
  R re, im;
};
typedef cplx<double> cd64;
typedef cplx<float> cf32;

template <typename R>
__host__ __device__ inline cplx<R> mkc(R a, R b) {
  cplx<R> c;
  c.re = a;
  c.im = b;
  return c;
}

// sum of f(g) over g = t, t + step, ... < G, added in that order, with U
// terms' loads in flight at once (indices past the end clamped, not added)
template <int U, typename F>
__device__ inline cplx<double> strided_sum(int t, int step, int G, F f) {
  cplx<double> s = mkc(0.0, 0.0);
  for (int g0 = t; g0 < G; g0 += U * step) {
    cplx<double> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = f(min(g0 + u * step, G - 1));
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (g0 + u * step < G) s = mkc(s.re + v[u].re, s.im + v[u].im);
  }
  return s;
}
template <typename R>
__host__ __device__ inline cplx<R> cadd(cplx<R> a, cplx<R> b) { return mkc(a.re + b.re, a.im + b.im); }
template <typename R>
__host__ __device__ inline cplx<R> csub(cplx<R> a, cplx<R> b) { return mkc(a.re - b.re, a.im - b.im); }
template <typename R>
__host__ __device__ inline cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return mkc(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// acc += a * b
template <typename R>
__host__ __device__ inline void cfma(cplx<R>& acc, cplx<R> a, cplx<R> b) {
  acc.re += a.re * b.re - a.im * b.im;
  acc.im += a.re * b.im + a.im * b.re;
}
// acc += conj(a) * b
template <typename R>
__host__ __device__ inline void cfmac(cplx<R>& acc, cplx<R> a, cplx<R> b) {
  acc.re += a.re * b.re + a.im * b.im;
  acc.im += a.re * b.im - a.im * b.re;
}
template <typename R>
__host__ __device__ inline cplx<R> cscale(R s, cplx<R> a) { return mkc(s * a.re, s * a.im); }
// i * a
template <typename R>
__host__ __device__ inline cplx<R> ci(cplx<R> a) { return mkc(-a.im, a.re); }
template <typename R>
__host__ __device__ inline cplx<R> cneg(cplx<R> a) { return mkc(-a.re, -a.im); }
template <typename R>
__host__ __device__ inline cplx<R> cconj(cplx<R> a) { return mkc(a.re, -a.im); }

template <typename R, typename S>
__host__ __device__ inline cplx<R> ccast(cplx<S> a) { return mkc((R)a.re, (R)a.im); }

// ---------------------------------------------------------------- bf16 (round to nearest even)
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

// ---------------------------------------------------------------- device buffers
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() {}
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t n) {
    if (n == bytes && p) return;
    release();
    if (n == 0) return;
    WCMG_HIP(hipMalloc(&p, n));
    bytes = n;
  }
  template <typename T>
  T* as() const { return (T*)p; }
};

// precision helpers
inline size_t cbytes(int prec) { return prec == WCMG_F64 ? 16 : 8; }

// ---------------------------------------------------------------- launch helpers
constexpr int kBlock = 256;
inline unsigned nblocks(long n, int bs = kBlock) { return (unsigned)((n + bs - 1) / bs); }

// Workgroup -> (item, right-hand side) for launches over items x fields, with
// the field varying fastest inside each XCD's contiguous share of the grid
// (padded to a multiple of the 8 XCDs, which receive workgroups round-robin):
// the workgroups that read the same item's operator data (links, clover, P)
// run together on one XCD, so that data crosses HBM about once per launch and
// is served from that XCD's L2 to the other fields.  Returns false for
// padding workgroups.
__device__ inline bool item_rhs(long n_items, int nrhs, long* item, long* rhs) {
  const long G = gridDim.x;
  const long h = blockIdx.x;
  const long L = (h % 8) * (G / 8) + h / 8;
  if (L >= n_items * nrhs) return false;
  *item = L / nrhs;
  *rhs = L % nrhs;
  return true;
}
inline unsigned item_rhs_grid(long n_items, int nrhs) { return (unsigned)((n_items * nrhs + 7) / 8 * 8); }

// Division of 32-bit unsigned n < 2^31 by an invariant d >= 1 with a
// multiply-high and a shift (Granlund and Montgomery, "Division by invariant
// integers using multiplication", 1994): l = ceil(log2 d),
// m = floor(2^(32+l) / d) - 2^32 + 1, q = (mulhi(n, m) + n) >> l.
struct FastDiv {
  uint32_t d = 1, m = 1, l = 0;
  FastDiv() = default;
  explicit FastDiv(uint32_t dv) : d(dv) {
    l = 0;
    while ((1ull << l) < dv) ++l;
    m = (uint32_t)((((uint64_t)1 << (32 + l)) / dv) - ((uint64_t)1 << 32) + 1);
  }
  __host__ __device__ uint32_t div(uint32_t n) const {
    const uint32_t hi = (uint32_t)(((uint64_t)n * m) >> 32);  // a multiply-high on the GPU
    return (uint32_t)(((uint64_t)hi + n) >> l);
  }
  __host__ __device__ uint32_t mod(uint32_t n) const { return n - div(n) * d; }
};

// Device site order of level 0 as arithmetic: s = c * A + o, c the aggregate
// (lexicographic over the coarse extents Lc) and o the offset inside it
// (lexicographic over the block b), x fastest in both.  Neighbours follow from
// the coordinates without a table: a hop stays inside the aggregate unless it
// leaves through a face, then it enters the neighbouring aggregate (periodic
// over the coarse lattice) on the opposite face.
struct SiteGeom {
  FastDiv divA, div_so[4], mod_b[4], div_sc[4], mod_Lc[4];
  uint32_t A = 1, so[4] = {1, 1, 1, 1}, sc[4] = {1, 1, 1, 1}, b[4] = {1, 1, 1, 1}, Lc[4] = {1, 1, 1, 1};
  int anti = 0;  // antiperiodic fermion boundary in t (the sign on t-hops crossing it)
  SiteGeom() = default;
  SiteGeom(const int L[4], const int blk[4], int antiperiodic_t = 0) {
    anti = antiperiodic_t;
    A = 1;
    uint32_t cs = 1;
    for (int m = 0; m < 4; ++m) {
      b[m] = (uint32_t)blk[m];
      Lc[m] = (uint32_t)(L[m] / blk[m]);
      so[m] = A;
      sc[m] = cs;
      A *= b[m];
      cs *= Lc[m];
    }
    divA = FastDiv(A);
    for (int m = 0; m < 4; ++m) {
      div_so[m] = FastDiv(so[m]);
      mod_b[m] = FastDiv(b[m]);
      div_sc[m] = FastDiv(sc[m]);
      mod_Lc[m] = FastDiv(Lc[m]);
    }
  }
  // the neighbours of site s in directions +mu and -mu
  template <int MU>
  __host__ __device__ void hop_sites(uint32_t s, uint32_t& fwd, uint32_t& bwd) const {
    const uint32_t c = divA.div(s), o = s - c * A;
    const uint32_t om = mod_b[MU].mod(div_so[MU].div(o)), cm = mod_Lc[MU].mod(div_sc[MU].div(c));
    const uint32_t cstep = sc[MU] * A, cwrap = (Lc[MU] - 1) * cstep, owrap = (b[MU] - 1) * so[MU];
    fwd = om + 1 < b[MU] ? s + so[MU] : (cm + 1 < Lc[MU] ? s + cstep : s - cwrap) - owrap;
    bwd = om > 0 ? s - so[MU] : (cm > 0 ? s - cstep : s + cwrap) + owrap;
  }
  // as hop_sites, and whether s lies on the last (first) slice along MU
  template <int MU>
  __host__ __device__ void hop_sites_edge(uint32_t s, uint32_t& fwd, uint32_t& bwd, bool& last, bool& first) const {
    const uint32_t c = divA.div(s), o = s - c * A;
    const uint32_t om = mod_b[MU].mod(div_so[MU].div(o)), cm = mod_Lc[MU].mod(div_sc[MU].div(c));
    const uint32_t cstep = sc[MU] * A, cwrap = (Lc[MU] - 1) * cstep, owrap = (b[MU] - 1) * so[MU];
    fwd = om + 1 < b[MU] ? s + so[MU] : (cm + 1 < Lc[MU] ? s + cstep : s - cwrap) - owrap;
    bwd = om > 0 ? s - so[MU] : (cm > 0 ? s - cstep : s + cwrap) + owrap;
    last = om + 1 == b[MU] && cm + 1 == Lc[MU];
    first = om == 0 && cm == 0;
  }
};

// Site geometry of one level as the kernels see it.
//   layout SoA (level 0): element (site s, component k) at k * V + s
//   layout AoS (levels >= 1): element at s * ns + k
struct FieldLayout {
  long V;
  int ns;
  bool soa;
  __host__ __device__ long at(long s, int k) const { return soa ? (long)k * V + s : s * ns + k; }
  __host__ __device__ long size() const { return V * ns; }
};

}  // namespace wcmg
