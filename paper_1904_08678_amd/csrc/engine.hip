// Multigrid engine: geometry, operators, setup (initial and iterative),
// MR smoother, (flexible) GMRES, V- and K-cycles (Sec. 2.1 of the paper).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>

#include "engine.h"

namespace wcmg {

// ---------------------------------------------------------------- profiler
Profiler::~Profiler() {
  for (auto& kv : fam)
    for (auto& e : kv.second.ev) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
}
void Profiler::enable(const std::string& f, bool on) { fam[f].on = on; }
void Profiler::begin(const char* f, hipStream_t st) {
  auto it = fam.find(f);
  if (it == fam.end() || !it->second.on) return;
  Family& F = it->second;
  if (F.used == F.ev.size()) {
    hipEvent_t a, b;
    WCMG_HIP(hipEventCreate(&a));
    WCMG_HIP(hipEventCreate(&b));
    F.ev.push_back({a, b});
  }
  WCMG_HIP(hipEventRecord(F.ev[F.used].first, st));
}
void Profiler::begin_kernel(const char* f) {
  auto it = fam.find(f);
  if (it == fam.end() || !it->second.on) return;
  Family& F = it->second;
  if (F.used == F.ev.size()) {
    hipEvent_t a, b;
    WCMG_HIP(hipEventCreate(&a));
    WCMG_HIP(hipEventCreate(&b));
    F.ev.push_back({a, b});
  }
  kernel_timing() = KernelTiming{F.ev[F.used].first, F.ev[F.used].second};
  F.armed = true;
}
void Profiler::end(const char* f, hipStream_t st) {
  auto it = fam.find(f);
  if (it == fam.end() || !it->second.on) return;
  Family& F = it->second;
  if (F.armed) {
    F.armed = false;
    const bool consumed = kernel_timing().start == nullptr;
    kernel_timing() = KernelTiming();
    if (consumed) F.used++;  // else no launch took the events: no sample
    return;
  }
  WCMG_HIP(hipEventRecord(F.ev[F.used].second, st));
  F.used++;
}
void Profiler::stats(const std::string& f, int64_t* launches, double* ms) {
  auto it = fam.find(f);
  *launches = 0;
  *ms = 0.0;
  if (it == fam.end()) return;
  Family& F = it->second;
  for (size_t i = 0; i < F.used; ++i) {
    WCMG_HIP(hipEventSynchronize(F.ev[i].second));
    float t = 0.f;
    WCMG_HIP(hipEventElapsedTime(&t, F.ev[i].first, F.ev[i].second));
    *ms += t;
  }
  *launches = (int64_t)F.used;
  F.used = 0;
}

// ---------------------------------------------------------------- geometry helpers
namespace {
long vol4(const int L[4]) { return (long)L[0] * L[1] * L[2] * L[3]; }
void lex_coords(long i, const int L[4], int x[4]) {
  for (int m = 0; m < 4; ++m) {
    x[m] = (int)(i % L[m]);
    i /= L[m];
  }
}
long lex_index(const int x[4], const int L[4]) { return x[0] + (long)L[0] * (x[1] + (long)L[1] * (x[2] + (long)L[2] * x[3])); }
long lex_neighbour(long i, const int L[4], int d) {
  int x[4];
  lex_coords(i, L, x);
  int mu = (d - 1) / 2, step = ((d - 1) % 2 == 0) ? 1 : -1;
  x[mu] = (x[mu] + step + L[mu]) % L[mu];
  return lex_index(x, L);
}
void upload(DevBuf& b, const std::vector<int>& v) {
  b.alloc(v.size() * sizeof(int));
  WCMG_HIP(hipMemcpy(b.p, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice));
}
}  // namespace

void CoarseOp::init_geometry(const int Lc[4], int nb_, hipStream_t) {
  for (int m = 0; m < 4; ++m) L[m] = Lc[m];
  V = vol4(L);
  nb = nb_;
  std::vector<int> nb_host(8 * V);
  for (int d = 1; d <= 8; ++d)
    for (long s = 0; s < V; ++s) nb_host[(d - 1) * V + s] = (int)lex_neighbour(s, L, d);
  upload(nbr, nb_host);
  M64.alloc((size_t)V * 9 * nb * nb * sizeof(cd64));
}

void CoarseOp::refresh(int prec, hipStream_t st) {
  if (!uses_five()) {
    refresh9(prec, st);
    return;
  }
  if (fresh5[prec]) return;
  dev5[prec].alloc(device_block5_bytes(V, nb, prec));
  launch_blocks_to_device5(M64.as<cd64>(), V, nb, prec, dev5[prec].p, st);
  fresh5[prec] = true;
}

void CoarseOp::refresh9(int prec, hipStream_t st) {
  if (fresh[prec]) return;
  dev[prec].alloc(device_block_bytes(V, nb, prec));
  launch_blocks_to_device(M64.as<cd64>(), V, nb, prec, dev[prec].p, st);
  fresh[prec] = true;
}

void CoarseOp::refresh_mfma(int prec, hipStream_t st) {
  if (mfma_fresh[prec]) return;
  mfma[prec].alloc(mfma_block_bytes(V, nb, prec));
  launch_blocks_to_mfma(M64.as<cd64>(), V, nb, prec, mfma[prec].p, st);
  mfma_fresh[prec] = true;
}

// Matrix-core tile candidates, in the order of the tuner's variant index:
// one wave per site; 4, 8, 16 sites per workgroup with neighbours and outputs
// staged in LDS; 4 or 8 sites with staged neighbours and per-wave stores.
static const int kMfmaTiles[6] = {0, 4, 8, 16, 5, 9};
constexpr int kNumMfmaTiles = 6;

int CoarseOp::choose_tile(int prec, const void* in, void* out, int k, const int* run, int run_stride,
                          hipStream_t st) {
  auto ok = [&](int tile) { return mfma_tile_ok(tile, nb, V, L[0], k); };
  if (mfma_tile >= 0) {
    require(ok(mfma_tile), WCMG_ERR_ARG,
            "matrix-core tile " + std::to_string(mfma_tile) + " does not fit this lattice or batch");
    return mfma_tile;
  }
  const int dflt = ok(4) ? 1 : 0;  // variant index of the untuned default
  if (!tuner) return kMfmaTiles[dflt];
  const std::string key = device_arch() + " coarse_mfma_tile prec=" + std::to_string(prec) +
                          " Vc=" + std::to_string(V) + " Lx=" + std::to_string(L[0]) + " nb=" + std::to_string(nb) +
                          " nrhs=" + std::to_string(k);
  auto it = tuner->choice.find(key);
  if (it != tuner->choice.end()) {
    const int v = it->second;
    return (v >= 0 && v < kNumMfmaTiles && ok(kMfmaTiles[v])) ? kMfmaTiles[v] : kMfmaTiles[dflt];
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  WCMG_HIP(hipStreamIsCapturing(st, &cs));
  if (cs != hipStreamCaptureStatusNone || !tuner->enabled) return kMfmaTiles[dflt];
  const int v = tuner->pick(
      key, kNumMfmaTiles,
      [&](int v) {
        launch_coarse_apply_mfma(prec, nb, mfma[prec].p, (const cf32*)in, (cf32*)out, nbr.as<int>(), V, k, run,
                                 run_stride, st, kMfmaTiles[v], L[0]);
      },
      st, dflt, [&](int v) { return ok(kMfmaTiles[v]); });
  return kMfmaTiles[v];
}

void CoarseOp::apply_batch(int prec, const void* in, void* out, int nrhs, int kernel, const int* run, int run_stride,
                           hipStream_t st) {
  const bool can_mfma = prec != WCMG_F64 && mfma_supported_nb(nb);
  const bool use_mfma = can_mfma && (kernel == 2 || (kernel == 0 && nrhs >= 4));
  require(kernel != 2 || can_mfma, WCMG_ERR_ARG, "matrix-core kernel needs FP32/BF16 storage and Nb in {8,16,24,32,40}");
  if (use_mfma) {
    require(mfma_fresh[prec], WCMG_ERR_STATE, "matrix-core block layout not built");
    for (int r0 = 0; r0 < nrhs; r0 += 16) {
      const int k = std::min(16, nrhs - r0);
      const long off = (long)r0 * V * nb;
      const cf32* i0 = (const cf32*)in + off;
      cf32* o0 = (cf32*)out + off;
      const int* run0 = run ? run + (long)r0 * run_stride : nullptr;
      const int tile = choose_tile(prec, i0, o0, k, run0, run_stride, st);
      launch_coarse_apply_mfma(prec, nb, mfma[prec].p, i0, o0, nbr.as<int>(), V, k, run0, run_stride, st, tile, L[0]);
    }
  } else {
    apply(prec, in, out, 0x1ff, 0, nrhs, run, st, run_stride);
  }
}

void CoarseOp::apply_batch_scratch(int prec, const void* in, void* out, int nrhs, int kernel, void* scratch,
                                   size_t scratch_bytes, hipStream_t st) {
  const bool can_mfma = prec != WCMG_F64 && mfma_supported_nb(nb);
  const bool use_mfma = can_mfma && (kernel == 2 || (kernel == 0 && nrhs >= 4));
  if (!use_mfma && fresh5[prec]) {
    void* tmp = nullptr;
    if (coarse5_uses_owner(V, nb, nrhs)) {
      const size_t need = 4 * (size_t)nrhs * V * nb * cbytes(prec);
      require(need <= scratch_bytes, WCMG_ERR_ARG,
              "five-point apply of " + std::to_string(nrhs) + " fields needs " + std::to_string(need) +
                  " bytes of scratch; the no-allocation buffer holds " + std::to_string(scratch_bytes));
      tmp = scratch;
    }
    launch_coarse_apply5(prec, dev5[prec].p, in, out, tmp, nbr.as<int>(), V, nb, 0, nrhs, nullptr, st, 0);
    return;
  }
  // the other kernels use no scratch; with their layout built they allocate nothing
  require(use_mfma ? mfma_fresh[prec] : fresh[prec], WCMG_ERR_STATE,
          "coarse operator not built in the requested precision");
  apply_batch(prec, in, out, nrhs, kernel, nullptr, 0, st);
}

void CoarseOp::apply(int prec, const void* in, void* out, int dmask, int accumulate, int nrhs, const int* run,
                     hipStream_t st, int run_stride) {
  require(built(prec), WCMG_ERR_STATE, "coarse operator not built in the requested precision");
  if (fresh5[prec] && dmask == 0x1ff) {
    void* tmp = nullptr;
    if (coarse5_uses_owner(V, nb, nrhs)) {
      // grown only (a captured apply reuses what its eager warm-up allocated)
      const size_t need = 4 * (size_t)nrhs * V * nb * cbytes(prec);
      if (tmp5.bytes < need) tmp5.alloc(need);
      tmp = tmp5.p;
    }
    launch_coarse_apply5(prec, dev5[prec].p, in, out, tmp, nbr.as<int>(), V, nb, accumulate, nrhs, run, st,
                         run_stride);
    return;
  }
  refresh9(prec, st);
  launch_coarse_apply(prec, dev[prec].p, in, out, nbr.as<int>(), V, nb, dmask, accumulate, nrhs, run, st,
                      run_stride);
}

// ---------------------------------------------------------------- context
Context::Context(const wcmg_params& prm, hipStream_t s) : p(prm), stream(s) {
  nlev = p.n_levels;
  require(nlev >= 1 && nlev <= 3, WCMG_ERR_ARG, "n_levels must be 1, 2 or 3");
  for (int m = 0; m < 4; ++m) require(p.dims[m] >= 2, WCMG_ERR_DIMS, "lattice extents must be >= 2");
  require(p.cycle_prec == WCMG_F64 || p.cycle_prec == WCMG_F32, WCMG_ERR_ARG, "cycle_prec must be F64 or F32");
  require(p.setup_prec == WCMG_F64 || p.setup_prec == WCMG_F32, WCMG_ERR_ARG, "setup_prec must be F64 or F32");
  require(p.coarse_store_prec >= 0 && p.coarse_store_prec <= 2, WCMG_ERR_ARG, "bad coarse_store_prec");
  require(p.coarse_points == 0 || p.coarse_points == 5 || p.coarse_points == 9, WCMG_ERR_ARG,
          "coarse_points must be 5 or 9");
  require(p.smoother == 0 || p.smoother == 1, WCMG_ERR_ARG, "smoother must be 0 (MR) or 1 (SAP)");
  require(p.even_odd == 0 || p.even_odd == 1, WCMG_ERR_ARG, "even_odd must be 0 or 1");
  require(p.smoother == 0 || p.sap_block_iters >= 1, WCMG_ERR_ARG, "sap_block_iters must be >= 1");
  require(p.outer_restart >= 1 && p.outer_restart <= 40 && p.coarse_restart >= 1 && p.coarse_restart <= 40 &&
              p.kcycle_maxit >= 1 && p.kcycle_maxit <= 40,
          WCMG_ERR_ARG, "restart lengths must lie in 1..40");
  geo.resize(nlev);
  tr.resize(nlev - 1);
  // level extents
  int L[3][4];
  for (int m = 0; m < 4; ++m) L[0][m] = p.dims[m];
  for (int l = 0; l + 1 < nlev; ++l) {
    for (int m = 0; m < 4; ++m) {
      require(p.block[l][m] >= 1 && L[l][m] % p.block[l][m] == 0, WCMG_ERR_DIMS,
              "block does not divide the lattice at level " + std::to_string(l));
      L[l + 1][m] = L[l][m] / p.block[l][m];
      require(L[l + 1][m] >= 2, WCMG_ERR_DIMS, "coarse lattice extent below 2 at level " + std::to_string(l + 1));
    }
    require(p.n_vec[l] >= 1 && supported_nb(2 * p.n_vec[l]), WCMG_ERR_ARG,
            "unsupported number of near-null vectors at level " + std::to_string(l));
  }
  for (int l = 0; l < nlev; ++l) {
    LevelGeom& G = geo[l];
    for (int m = 0; m < 4; ++m) G.L[m] = L[l][m];
    G.V = vol4(G.L);
    G.ns = l == 0 ? 12 : 2 * p.n_vec[l - 1];
    G.lay.V = G.V;
    G.lay.ns = G.ns;
    G.lay.soa = (l == 0);
  }
  // device order of level 0: aggregate-major under block[0] (Sec. 3: the fine
  // lattice linearised per aggregate); lexicographic without multigrid.
  {
    LevelGeom& G = geo[0];
    int b[4] = {1, 1, 1, 1};
    if (nlev > 1)
      for (int m = 0; m < 4; ++m) b[m] = p.block[0][m];
    int Lc[4];
    for (int m = 0; m < 4; ++m) Lc[m] = G.L[m] / b[m];
    const int A = b[0] * b[1] * b[2] * b[3];
    G.perm.assign(G.V, 0);
    std::vector<int> iperm(G.V);
    for (long i = 0; i < G.V; ++i) {
      int x[4], cx[4], ox[4];
      lex_coords(i, G.L, x);
      for (int m = 0; m < 4; ++m) {
        cx[m] = x[m] / b[m];
        ox[m] = x[m] % b[m];
      }
      long c = lex_index(cx, Lc);
      long o = ox[0] + (long)b[0] * (ox[1] + (long)b[1] * (ox[2] + (long)b[2] * ox[3]));
      long s = c * A + o;
      G.perm[s] = (int)i;
      iperm[i] = (int)s;
    }
    std::vector<int> nb_host(8 * G.V);
    for (int d = 1; d <= 8; ++d)
      for (long s = 0; s < G.V; ++s) nb_host[(d - 1) * G.V + s] = iperm[lex_neighbour(G.perm[s], G.L, d)];
    upload(G.nbr, nb_host);
    upload(perm0, G.perm);
    sgeo = SiteGeom(G.L, b, p.antiperiodic_t);
  }
  for (int l = 1; l < nlev; ++l) {
    LevelGeom& G = geo[l];
    G.perm.resize(G.V);
    for (long s = 0; s < G.V; ++s) G.perm[s] = (int)s;
    cop.emplace_back(new CoarseOp());
    cop.back()->init_geometry(G.L, G.ns, stream);
    cop.back()->five = p.coarse_points == 5;
    cop.back()->tuner = &tuner;
    // coarse level vectors and operator share the lexicographic neighbour table
  }
  // transfers
  for (int l = 0; l + 1 < nlev; ++l) {
    Transfer& T = tr[l];
    LevelGeom& G = geo[l];
    for (int m = 0; m < 4; ++m) T.block[m] = p.block[l][m];
    T.A = T.block[0] * T.block[1] * T.block[2] * T.block[3];
    T.Vc = geo[l + 1].V;
    T.nv = p.n_vec[l];
    T.nb = 2 * T.nv;
    std::vector<int> agg_sites(T.Vc * T.A), coarse_of(G.V);
    T.agg_host.assign(G.V, 0);
    T.off_host.assign(G.V, 0);
    std::vector<int> iperm(G.V);
    for (long s = 0; s < G.V; ++s) iperm[G.perm[s]] = (int)s;
    for (long i = 0; i < G.V; ++i) {
      int x[4], cx[4], ox[4];
      lex_coords(i, G.L, x);
      for (int m = 0; m < 4; ++m) {
        cx[m] = x[m] / T.block[m];
        ox[m] = x[m] % T.block[m];
      }
      long c = lex_index(cx, geo[l + 1].L);
      long o = ox[0] + (long)T.block[0] * (ox[1] + (long)T.block[1] * (ox[2] + (long)T.block[2] * ox[3]));
      T.agg_host[i] = (int)c;
      T.off_host[i] = (int)o;
      agg_sites[c * T.A + o] = iperm[i];
      coarse_of[iperm[i]] = (int)c;
    }
    upload(T.agg_sites, agg_sites);
    upload(T.coarse_of, coarse_of);
    const size_t nbytes = (size_t)T.nv * G.n() * sizeof(cd64);
    T.start64.alloc(nbytes);
    T.vecs64.alloc(nbytes);
    T.P64.alloc(nbytes);
    T.P32.alloc(nbytes / 2);
  }
  for (int l = 1; l < nlev; ++l) {
    // coarse-level geometry for the level operators (neighbour table equals cop's)
    geo[l].nbr.alloc(8 * geo[l].V * sizeof(int));
    WCMG_HIP(hipMemcpy(geo[l].nbr.p, cop[l - 1]->nbr.p, 8 * geo[l].V * sizeof(int), hipMemcpyDeviceToDevice));
  }
  partial.alloc(kPartialSlots * sizeof(cd64));
  bpart.alloc((size_t)16 * kPartialSlots * sizeof(cd64));
  scratch64.alloc(64 * sizeof(cd64));
  WCMG_HIP(hipHostMalloc((void**)&pinned, 256 * sizeof(int), hipHostMallocDefault));
  WCMG_HIP(hipHostMalloc((void**)&mailbox, kCgpMailboxInts * sizeof(int), hipHostMallocCoherent | hipHostMallocMapped));
  for (int q = 0; q < kCgpMailboxInts; ++q) mailbox[q] = 0;
  WCMG_HIP(hipHostGetDevicePointer((void**)&mailbox_dev, mailbox, 0));
  const long V0 = geo[0].V;
  U_lex.alloc(V0 * 36 * sizeof(cd64));
  clover_lex.alloc(V0 * 72 * sizeof(cd64));
  U64.alloc(V0 * 36 * sizeof(cd64));
  U32.alloc(V0 * 36 * sizeof(cf32));
  clov64.alloc(V0 * 72 * sizeof(double));
  clov32.alloc(V0 * 72 * sizeof(float));
}

Context::~Context() {
  // kernels still queued may write the host-mapped mailboxes freed below
  (void)hipStreamSynchronize(stream);
  drop_graph();
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  if (pinned) (void)hipHostFree(pinned);
  if (mailbox) (void)hipHostFree(mailbox);
  for (auto& kv : state_mb)
    if (kv.second.h) (void)hipHostFree(kv.second.h);
}

template <typename T>
T* Context::buf(const std::string& tag, long count) {
  auto& b = ws[tag];
  if (!b) b.reset(new DevBuf());
  size_t need = (size_t)count * sizeof(T);
  if (b->bytes < need) b->alloc(need);
  return b->as<T>();
}

GmresState& Context::gmres_state(const std::string& tag, int m, long n, int prec, bool flex) {
  auto& g = gm[tag];
  if (!g) g.reset(new GmresState());
  GmresState& G = *g;
  if (G.m != m || G.n != n || G.prec != prec || G.flex != flex) {
    const size_t cb = prec == 0 ? sizeof(cd64) : sizeof(cf32);
    G.m = m;
    G.n = n;
    G.prec = prec;
    G.flex = flex;
    G.V.alloc((size_t)(m + 1) * n * cb);
    if (flex) G.Z.alloc((size_t)m * n * cb);
    G.w.alloc((size_t)n * cb);
    G.S.alloc((size_t)((m + 1) * m + 2 * m + (m + 1) + m + 8 + 2 * (m + 1)) * sizeof(cd64));
    G.st.alloc(8 * sizeof(int));
  }
  return G;
}

void Context::sync() {
  WCMG_HIP(hipStreamSynchronize(stream));
  settle_coarse();
}

int Context::publish_state(const int* st, int n) {
  int* slot = nullptr;
  const int seq = reserve_state(st, n, &slot);
  launch_publish_state(st, n, slot, seq, stream);
  return seq;
}

int Context::reserve_state(const int* st, int n, int** slot) {
  StateMailbox& M = state_mb[st];
  if (M.cap < n) {
    // a larger buffer: earlier publications must have landed before the copy
    WCMG_HIP(hipStreamSynchronize(stream));
    const int cap = std::max(n, 16);
    int* h = nullptr;
    WCMG_HIP(hipHostMalloc((void**)&h, 2 * (cap + 1) * sizeof(int), hipHostMallocCoherent | hipHostMallocMapped));
    for (int q = 0; q < 2 * (cap + 1); ++q) h[q] = 0;
    if (M.h) {
      for (int k = 0; k < 2; ++k)
        for (int q = 0; q <= M.cap; ++q) h[k * (cap + 1) + q] = M.h[k * (M.cap + 1) + q];
      (void)hipHostFree(M.h);
    }
    M.h = h;
    WCMG_HIP(hipHostGetDevicePointer((void**)&M.d, h, 0));
    M.cap = cap;
  }
  const int seq = ++M.seq;
  M.cgp[seq & 1] = cgp_seq;
  *slot = M.d + (seq & 1) * (M.cap + 1);
  if ((int)M.words.size() < n) M.words.resize(n);
  return seq;
}

const int* Context::wait_state(const int* st, int seq) {
  StateMailbox& M = state_mb[st];
  require(M.h && seq > 0 && seq <= M.seq && seq + 1 >= M.seq, WCMG_ERR_STATE, "state publication out of range");
  volatile int* slot = M.h + (seq & 1) * (M.cap + 1);
  for (long spins = 1; slot[0] != seq; ++spins) {
#if defined(__x86_64__)
    __builtin_ia32_pause();
#endif
    if (spins % 1024 == 0) {
      // the stream is checked now and then, so an error or a lost
      // publication ends the wait
      const hipError_t e = hipStreamQuery(stream);
      if (e == hipSuccess) {
        std::atomic_thread_fence(std::memory_order_acquire);
        require(slot[0] == seq, WCMG_ERR_HIP, "solver state publication did not arrive");
        break;
      }
      if (e != hipErrorNotReady) WCMG_HIP(e);
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  const int n = (int)M.words.size();
  for (int q = 0; q < n && q < M.cap; ++q) M.words[q] = slot[1 + q];
  settle_coarse(M.cgp[seq & 1]);
  return M.words.data();
}

void Context::settle_coarse(int upto) {
  if (cgp_pending.empty()) return;
  std::atomic_thread_fence(std::memory_order_acquire);
  volatile int* mb = mailbox;
  std::vector<CgpLaunch> keep, failed;
  for (const CgpLaunch& L : cgp_pending) {
    if (L.seq > upto) {
      keep.push_back(L);
      continue;
    }
    volatile int* slot = mb + kCgpSlot0 + 2 * (L.seq & (kCgpSlots - 1));
    if (slot[0] == L.seq) {
      coarse_iters += slot[1];
    } else {
      cgp_fallbacks++;
      bool seen = false;
      for (const CgpLaunch& F : failed) seen = seen || F.bar == L.bar;
      if (!seen) failed.push_back(L);
    }
  }
  cgp_pending.swap(keep);
  for (const CgpLaunch& F : failed) {
    // a wait timed out: keep the report, clear the flags, phase and error word
    WCMG_HIP(hipStreamSynchronize(stream));
    unsigned rep[8];
    WCMG_HIP(hipMemcpy(rep, F.bar, sizeof(rep), hipMemcpyDeviceToHost));
    if (rep[2] != 0)
      cgp_last_report = "workgroup " + std::to_string(rep[3]) + " of " + std::to_string((F.V + 1) / 2) +
                        " timed out at phase " + std::to_string(rep[4]) + " waiting for workgroup " +
                        std::to_string(rep[5]) + " (its flag: " + std::to_string(rep[6]) + ")";
    WCMG_HIP(hipMemsetAsync(F.bar, 0, F.nbar * sizeof(unsigned), stream));
    WCMG_HIP(hipStreamSynchronize(stream));
  }
}

int Context::store_prec_for(int l, bool single) const {
  (void)l;
  if (!single) return WCMG_F64;
  return p.coarse_store_prec == WCMG_BF16 ? WCMG_BF16 : WCMG_F32;
}

template <typename R>
void Context::apply_op(int l, const cplx<R>* in, cplx<R>* out, int nrhs, const int* run, int terms, cd64* dots) {
  const bool single = sizeof(R) == 4;
  if (l == 0) {
    const char* fam = terms != 0x1ff ? "wilson_term" : single ? "dslash_f32" : "dslash_f64";
    prof.begin_kernel(fam);
    if (single)
      launch_wilson<float>((const cf32*)in, (cf32*)out, U32.as<cf32>(), clov32.as<float>(), geo[0].nbr.as<int>(),
                           geo[0].V, terms, nrhs, run, stream, dots, 0, nullptr, dslash_geo(), dslash_links2<float>());
    else
      launch_wilson<double>((const cd64*)in, (cd64*)out, U64.as<cd64>(), clov64.as<double>(), geo[0].nbr.as<int>(),
                            geo[0].V, terms, nrhs, run, stream, dots, 0, nullptr, dslash_geo(), dslash_links2<double>());
    prof.end(fam, stream);
  } else {
    const int prec = store_prec_for(l, single);
    const char* fam = terms != 0x1ff ? "coarse_term" : prec == WCMG_F64 ? "coarse_apply_f64"
                                                      : prec == WCMG_F32 ? "coarse_apply_f32" : "coarse_apply_bf16";
    prof.begin_kernel(fam);
    cop[l - 1]->apply(prec, in, out, terms, 0, nrhs, run, stream);
    prof.end(fam, stream);
  }
}

template <typename R>
void Context::residual0(const cplx<R>* b, const cplx<R>* x, cplx<R>* r, const int* run) {
  const bool single = sizeof(R) == 4;
  const char* fam = single ? "dslash_f32" : "dslash_f64";
  prof.begin_kernel(fam);
  if (single)
    launch_wilson<float>((const cf32*)x, (cf32*)r, U32.as<cf32>(), clov32.as<float>(), geo[0].nbr.as<int>(), geo[0].V,
                         0x1ff, 1, run, stream, nullptr, 0, (const cf32*)b, dslash_geo(), dslash_links2<float>());
  else
    launch_wilson<double>((const cd64*)x, (cd64*)r, U64.as<cd64>(), clov64.as<double>(), geo[0].nbr.as<int>(),
                          geo[0].V, 0x1ff, 1, run, stream, nullptr, 0, (const cd64*)b, dslash_geo(), dslash_links2<double>());
  prof.end(fam, stream);
}

template <typename R>
double Context::norm2_host(const cplx<R>* v, long n) {
  cd64* s = scratch64.as<cd64>() + 8;
  launch_dot<R>(v, 0, 1, nullptr, v, n, partial.as<cd64>(), 1, s, 1, 0, nullptr, stream);
  cd64 h;
  WCMG_HIP(hipMemcpyAsync(&h, s, sizeof(cd64), hipMemcpyDeviceToHost, stream));
  sync();
  return h.re;
}

// ---------------------------------------------------------------- gauge and clover
void Context::set_gauge(const cd64* U) {
  const long V0 = geo[0].V;
  WCMG_HIP(hipMemcpyAsync(U_lex.p, U, V0 * 36 * sizeof(cd64), hipMemcpyDeviceToDevice, stream));
  launch_clover_build(U_lex.as<cd64>(), geo[0].L, p.c_sw, clover_lex.as<cd64>(), stream);
  launch_pack_links<double>(U_lex.as<cd64>(), perm0.as<int>(), geo[0].L, p.antiperiodic_t, U64.as<cd64>(), stream);
  launch_pack_links<float>(U_lex.as<cd64>(), perm0.as<int>(), geo[0].L, p.antiperiodic_t, U32.as<cf32>(), stream);
  // two-row links for the Dslash when every link is SU(3) (third row = conj(row0 x row1))
  {
    const long nl = V0 * 4;
    const int G = su3_defect_blocks(nl);
    double* part = buf<double>("su3_defect", G);
    launch_su3_defect(U_lex.as<cd64>(), nl, part, stream);
    std::vector<double> h(G);
    WCMG_HIP(hipMemcpyAsync(h.data(), part, G * sizeof(double), hipMemcpyDeviceToHost, stream));
    sync();
    double m = 0.0;
    for (double d : h) m = d > m ? d : m;
    links_su3 = m <= 1e-12;
    if (links_su3) {
      U64c.alloc(V0 * 24 * sizeof(cd64));
      U32c.alloc(V0 * 24 * sizeof(cf32));
      launch_pack_links2<double>(U_lex.as<cd64>(), perm0.as<int>(), geo[0].L, p.antiperiodic_t, U64c.as<cd64>(),
                                 stream);
      launch_pack_links2<float>(U_lex.as<cd64>(), perm0.as<int>(), geo[0].L, p.antiperiodic_t, U32c.as<cf32>(),
                                stream);
    }
  }
  pack_clover();
  gauge_set = true;
  setup_done = false;
}

void Context::set_clover(const cd64* blocks) {
  WCMG_HIP(hipMemcpyAsync(clover_lex.p, blocks, geo[0].V * 72 * sizeof(cd64), hipMemcpyDeviceToDevice, stream));
  pack_clover();
  setup_done = false;
}

void Context::pack_clover() {
  eo_ready = false;  // A^{-1} follows the clover term
  launch_pack_clover<double>(clover_lex.as<cd64>(), perm0.as<int>(), geo[0].V, p.m0, clov64.as<double>(), stream);
  launch_pack_clover<float>(clover_lex.as<cd64>(), perm0.as<int>(), geo[0].V, p.m0, clov32.as<float>(), stream);
}

// ---------------------------------------------------------------- transfers
template <typename R>
void Context::restrict_(int l, const cplx<R>* fine, cplx<R>* coarse, int nrhs, const int* run) {
  Transfer& T = tr[l];
  const cplx<R>* P = sizeof(R) == 8 ? (const cplx<R>*)T.P64.p : (const cplx<R>*)T.P32.p;
  const char* fam = sizeof(R) == 8 ? "restrict_f64" : "restrict_f32";
  prof.begin_kernel(fam);
  launch_restrict<R>(fine, coarse, P, geo[l].lay, T.agg_sites.as<int>(), T.A, T.Vc, T.nb, nrhs, run, stream);
  prof.end(fam, stream);
}

template <typename R>
void Context::prolong_(int l, const cplx<R>* coarse, cplx<R>* fine, int accumulate, int nrhs, const int* run) {
  Transfer& T = tr[l];
  const cplx<R>* P = sizeof(R) == 8 ? (const cplx<R>*)T.P64.p : (const cplx<R>*)T.P32.p;
  const char* fam = sizeof(R) == 8 ? "prolong_f64" : "prolong_f32";
  prof.begin_kernel(fam);
  launch_prolong<R>(coarse, fine, P, geo[l].lay, T.coarse_of.as<int>(), T.Vc, T.nb, accumulate, nrhs, run, stream, 0,
                    T.agg_sites.as<int>(), T.A);
  prof.end(fam, stream);
}

// ---------------------------------------------------------------- smoother
// MinimalResidual (Sec. 2.1): from x and r = b - D x, `steps` times
//   p = D r; alpha = <p,r>/<p,p>; x += alpha r; r -= alpha p.
// b == nullptr means b = 0 (relaxation on D x = 0).
template <typename R>
void Context::mr(int l, const cplx<R>* b, cplx<R>* x, bool x0_zero, int steps, const int* run, cd64* x64) {
  const long nn = n(l);
  const std::string t = std::to_string(l) + (sizeof(R) == 8 ? "d" : "f");
  cplx<R>* r = buf<cplx<R>>("mr_r" + t, nn);
  cplx<R>* pp = buf<cplx<R>>("mr_p" + t, nn);
  cd64* dots = buf<cd64>("mr_dots" + t, 2);
  if (x0_zero) {
    launch_zero<R>(x, nn, run, stream);
    if (b) launch_convert<R, R>(b, r, nn, run, stream);
    else launch_zero<R>(r, nn, run, stream);
  } else if (l == 0 && b) {
    residual0<R>(b, x, r, run);
  } else {
    apply_op<R>(l, x, pp, 1, run);
    if (b) launch_sub<R>(r, b, pp, nn, run, stream);
    else launch_axpby<R>(r, pp, -1.0, 0.0, nn, run, stream);
  }
  if (l == 0) {
    // the inner products <p, r> and <p, p> come out of the operator's epilogue
    const int G = wilson_blocks(geo[0].V);
    cd64* part = buf<cd64>("mr_part" + t, 2L * G);
    for (int k = 0; k < steps; ++k) {
      apply_op<R>(l, r, pp, 1, run, 0x1ff, part);
      launch_mr_update_part<R>(x, r, pp, part, G, nn, run, stream, k + 1 == steps ? x64 : nullptr);
    }
    if (x64 && steps == 0) launch_convert<R, double>(x, x64, nn, run, stream);
    return;
  }
  require(!x64, WCMG_ERR_ARG, "MR: the FP64 output form is for the fine level");
  for (int k = 0; k < steps; ++k) {
    apply_op<R>(l, r, pp, 1, run);
    launch_mr_dots_update<R>(x, r, pp, nn, partial.as<cd64>(), dots, run, stream);
  }
}

// ---------------------------------------------------------------- GMRES / FGMRES
// Restarted GMRES with classical Gram-Schmidt applied twice (CGS2) and Givens
// rotations kept on the device.  With a preconditioner M the flexible variant
// stores z_j = M v_j and updates x with Z y (Sec. 2.1 FGMRES).
// Returns the iteration count when the host checks progress, else -1.
template <typename R>
int Context::gmres(GmresState& G, const std::function<void(const cplx<R>*, cplx<R>*, const int*)>& A,
                   const std::function<void(const cplx<R>*, cplx<R>*, const int*)>* M, const cplx<R>* b, cplx<R>* x,
                   bool x0_zero, int restart, int maxit, double tol, int fixed, bool stop_on_est, const int* parent,
                   int check_every, bool single_reduction) {
  const long nn = G.n;
  const int m = restart;
  cplx<R>* V = G.V.as<cplx<R>>();
  cplx<R>* Z = M ? G.Z.as<cplx<R>>() : nullptr;
  cplx<R>* w = G.w.as<cplx<R>>();
  cd64* S = G.S.as<cd64>();
  cd64* H = S;
  cd64* g = S + (m + 1) * m + 2 * m;
  cd64* y = g + (m + 1);
  cd64* misc = y + m;
  cd64* tmp = misc + 8;
  cd64* tmp2 = tmp + (m + 1);
  int* st = G.st.as<int>();
  int* run = st;
  int* live = st + 1;
  cd64* part = partial.as<cd64>();
  const int Gb = reduction_blocks(nn);
  launch_gmres_init(st, parent, stream);
  if (x0_zero) launch_zero<R>(x, nn, live, stream);
  launch_dot<R>(b, 0, 1, nullptr, b, nn, part, 1, misc + 0, 1, 0, live, stream);
  const int limit = fixed > 0 ? fixed : maxit;
  const int max_cycles = check_every > 0 ? limit : (limit + m - 1) / m;
  // Progress checks: within a cycle the host reads the state published at
  // the previous check while the steps since are already queued (a stopped
  // solve makes them no-ops through the run flag); at a cycle's end it waits
  // for the current state.
  StateChecks chk{*this, st, 5};
  const int* last = nullptr;
  for (int cyc = 0; cyc < max_cycles; ++cyc) {
    if (cyc == 0 && x0_zero) {
      launch_convert<R, R>(b, V, nn, live, stream);
    } else {
      A(x, w, live);
      launch_sub<R>(V, b, w, nn, live, stream);
    }
    launch_dot<R>(V, 0, 1, nullptr, V, nn, part, 1, misc + 1, 1, 0, live, stream);
    launch_gmres_cycle_start(st, S, m, tol, limit, fixed, stream);
    launch_scale_inv_norm<R>(V, V, misc + 1, nn, run, stream);
    for (int j = 0; j < m; ++j) {
      cplx<R>* vj = V + (long)j * nn;
      cplx<R>* zj = M ? Z + (long)j * nn : vj;
      if (M) (*M)(vj, zj, run);
      if (single_reduction) {
        // One sweep gives the dots of w' = A z_j - s v_j (formed in place in
        // the slot of v_{j+1}; s = Re h_00 of the cycle, none at j = 0) with
        // the basis and |w'|^2; |w1|^2 = |w'|^2 - |h|^2 (V orthonormal), and
        // the projection is repeated only when it removed more than 3/4 of
        // |w'|^2 (st[5]); the last sweep subtracts and normalises.  A z_j is
        // mostly along v_j when the preconditioner is good, so projecting w'
        // instead of A z_j avoids that cancellation; the Hessenberg column of
        // A Z is h + s e_j.
        cplx<R>* wj = V + (long)(j + 1) * nn;
        A(zj, wj, run);
        launch_arnoldi_dots<R>(V, nn, j, j > 0 ? misc + 4 : nullptr, part, j + 2, run, stream);
        launch_dot_finish_sr(part, Gb, j, tmp, st, S, m, stream);
        launch_multi_axpy<R>(wj, V, nn, j + 1, nullptr, tmp, 1, -1.0, nn, st + 5, stream, 1024);
        // the second projection is rare: a small grid, so that skipping it is cheap
        const int G2 = std::min(Gb, 256);
        launch_arnoldi_dots<R>(V, nn, j, nullptr, part, j + 2, st + 5, stream, G2);
        // a progress check after this step: the finishing kernel publishes the state
        const bool check = check_every > 0 && (j + 1) % check_every == 0 && j + 1 < m;
        int* slot = nullptr;
        const int seq = check ? reserve_state(st, 5, &slot) : 0;
        launch_gmres_sr_finish(st, S, m, j, tmp, tmp2, part, G2, tol, limit, fixed, stop_on_est ? 1 : 0, stream,
                               slot, seq, 5);
        if (j + 1 < m) launch_update_scale<R>(wj, V, nn, j + 1, tmp, misc + 3, nn, run, stream);
        if (check) {
          const int* sv = chk.ahead_issued(seq);
          if (sv && !sv[0]) break;
        }
        continue;
      }
      A(zj, w, run);
      // classical Gram-Schmidt applied twice; |w|^2 comes out of the last update
      launch_dot<R>(V, nn, j + 1, nullptr, w, nn, part, j + 1, H + j, m, 0, run, stream);
      // the partials of the second projection: from the fused sweep (the
      // batched kernels' block count) or from a separate dot pass
      const int Gp = j + 1 <= kFusedMaxM ? bred_blocks(nn) : Gb;
      if (j + 1 <= kFusedMaxM) {
        // first update and second projection in one sweep over the basis
        launch_bmulti_axpy_dot<R>(w, 0, V, nn, 0, j + 1, H + j, m, 0, nn, 1, part, run, 0, stream);
        launch_dot_finish(part, Gp, j + 1, j + 1, tmp, 1, 0, run, stream);
      } else {
        launch_multi_axpy<R>(w, V, nn, j + 1, nullptr, H + j, m, -1.0, nn, run, stream);
        launch_dot<R>(V, nn, j + 1, nullptr, w, nn, part, j + 1, tmp, 1, 0, run, stream);
      }
      launch_dot_finish(part, Gp, j + 1, j + 1, H + j, m, 1, run, stream);
      launch_multi_axpy_norm<R>(w, V, nn, j + 1, tmp, 1, -1.0, nn, part, run, stream);
      launch_dot_finish(part, Gb, 1, 1, misc + 3, 1, 0, run, stream);
      launch_gmres_givens(st, S, m, j, tol, limit, fixed, stop_on_est ? 1 : 0, stream);
      if (j + 1 < m) launch_scale_inv_norm<R>(V + (long)(j + 1) * nn, w, misc + 3, nn, run, stream);
      if (check_every > 0 && (j + 1) % check_every == 0 && j + 1 < m) {
        const int* sv = chk.ahead();
        if (sv && !sv[0]) break;
      }
    }
    launch_gmres_solve_y(st, S, m, stream);
    launch_multi_axpy<R>(x, M ? Z : V, nn, m, st + 2, y, 1, 1.0, nn, nullptr, stream);
    launch_gmres_cycle_end(st, stream);
    if (check_every > 0) {
      last = chk.now();
      if (!last[1]) break;
    }
  }
  if (check_every > 0) return (last ? last : chk.now())[3];
  return -1;
}

// ---------------------------------------------------------------- fused coarsest GMRES
// Same semantics as gmres() with restart = coarse_restart, x0 = 0 and the
// estimate ending the solve, but each Arnoldi step is four kernels
// (coarse_gmres.hip).
template <typename R>
int Context::coarse_gmres(int lc, const cplx<R>* b, cplx<R>* x, const int* parent, int check_every) {
  CoarseOp& C = *cop[lc - 1];
  const bool single = sizeof(R) == 4;
  const int prec = store_prec_for(lc, single);
  const int nb = C.nb;
  const long nn = C.V * nb;
  const int m = p.coarse_restart, m1 = m + 1;
  const std::string t = std::to_string(lc) + (single ? "f" : "d");
  GmresState& G = gmres_state("cgf" + t, m, nn, single ? 1 : 0, false);
  cplx<R>* V = G.V.as<cplx<R>>();
  cplx<R>* wb[2] = {G.w.as<cplx<R>>(), buf<cplx<R>>("cgf_w1" + t, nn)};
  cplx<R>* r = buf<cplx<R>>("cgf_r" + t, nn);
  const long G1max = (long)nblocks(nn * 8), G2 = nblocks(nn);
  cd64* partA = buf<cd64>("cgf_pa" + t, G1max * m1);
  cd64* partB = buf<cd64>("cgf_pb" + t, G2 * m1);
  cd64* partC = buf<cd64>("cgf_pc" + t, G2 * m1);
  cd64* S = G.S.as<cd64>();
  cd64* misc = S + (m + 1) * m + 2 * m + (m + 1) + m;
  cd64* y = misc - m;
  int* st = G.st.as<int>();
  int* run = st;
  int* live = st + 1;
  require(C.built(prec), WCMG_ERR_STATE, "coarse operator not built in the requested precision");
  const bool five = C.fresh5[prec];
  const void* blk = five ? C.dev5[prec].p : C.dev[prec].p;
  const int fixed = p.coarse_fixed_iters;
  const int limit = fixed > 0 ? fixed : p.coarse_maxit;
  const int max_cycles = check_every > 0 ? limit : (limit + m - 1) / m;
  StateChecks chk{*this, st, 5};  // as in gmres()
  const int* last = nullptr;
  const char* fam = prec == WCMG_F64 ? "coarse_gmres_step_f64" : prec == WCMG_F32 ? "coarse_gmres_step_f32"
                                                                                     : "coarse_gmres_step_bf16";
  // one persistent launch for the whole solve when the blocks fit the LDS
  // (reserved[0] flag 4 turns it off); only where the host checks progress,
  // since its report is checked by the host (not under stream capture)
  if (!five && check_every > 0 && !(p.reserved[0] & 4) && cg_persistent_fits(prec, nb, C.V)) {
    cd64* partP = buf<cd64>("cgp_part" + t, (long)cg_persistent_part_elems(C.V));
    const long nbar = (long)cg_persistent_bar_words(C.V);
    unsigned* bar = buf<unsigned>("cgp_bar" + t, nbar);
    cplx<R>* zP = buf<cplx<R>>("cgp_z" + t, 2 * nn);
    // a new buffer starts with cleared flags and phase (launches on the old
    // one are checked first)
    if (cgp_bar_at[t] != (void*)bar) {
      sync();
      WCMG_HIP(hipMemsetAsync(bar, 0, nbar * sizeof(unsigned), stream));
      cgp_bar_at[t] = (void*)bar;
    }
    // reserved[0] flag 16: waits that give up at once; each launch is then
    // checked at once and a timed-out solve redone by the multi-kernel form.
    // Flag 128: the first launch's waits give up at once, checked later.
    const bool give_up = (p.reserved[0] & 16) != 0;
    const bool force_late = (p.reserved[0] & 128) && !cgp_forced;
    cgp_forced = cgp_forced || force_late;
    const int seq = ++cgp_seq;
    prof.begin("coarse_gmres_persistent", stream);
    const bool launched = launch_cg_persistent(prec, nb, blk, C.nbr.as<int>(), C.V, b, x, zP, r, partP, misc, st,
                                               parent, m, p.coarse_tol, limit, fixed, bar, seq, mailbox_dev,
                                               give_up || force_late ? 0.0 : 5.0, (p.reserved[0] & 256) != 0,
                                               stream);
    prof.end("coarse_gmres_persistent", stream);
    if (launched) {
      cgp_pending.push_back(CgpLaunch{seq, bar, nbar, C.V});
      // checked (and counted) when the host next waits for the stream; the
      // report slots bound how many launches may stay unchecked
      if (!give_up && (int)cgp_pending.size() < kCgpSlots / 2) return -1;
      const long before = cgp_fallbacks;
      sync();
      if (cgp_fallbacks == before) return -1;
      // this launch timed out: redo the solve below
    }
  }
  launch_gmres_init(st, parent, stream);
  launch_zero<R>(x, nn, live, stream);
  for (int cyc = 0; cyc < max_cycles; ++cyc) {
    const cplx<R>* u0 = b;
    if (cyc > 0) {
      C.apply(prec, x, wb[0], 0x1ff, 0, 1, live, stream);
      launch_sub<R>(r, b, wb[0], nn, live, stream);
      u0 = r;
    }
    launch_cg_norm_partial<R>(u0, nn, partC, m1, live, stream);
    launch_cg_cycle_start(st, S, m, partC, (int)G2, cyc == 0 ? 1 : 0, p.coarse_tol, limit, fixed, stream);
    for (int j = 0; j < m; ++j) {
      const cplx<R>* u = j == 0 ? u0 : wb[j & 1];
      const cd64* unrm2 = j == 0 ? misc + 1 : misc + 3;
      cplx<R>* w = wb[(j + 1) & 1];
      prof.begin_kernel(fam);
      const int G1 =
          launch_cg_apply(prec, nb, blk, C.nbr.as<int>(), C.V, u, unrm2, V, j, w, partA, m1, run, stream, five);
      prof.end(fam, stream);
      launch_cg_orth<R>(V, j, w, nn, partA, G1, S, m, 0, partB, run, stream);
      launch_cg_orth<R>(V, j, w, nn, partB, (int)G2, S, m, 1, partC, run, stream);
      launch_cg_givens(st, S, m, j, partC, (int)G2, p.coarse_tol, limit, fixed, stream);
      if (check_every > 0 && (j + 1) % check_every == 0 && j + 1 < m) {
        const int* sv = chk.ahead();
        if (sv && !sv[0]) break;
      }
    }
    launch_gmres_solve_y(st, S, m, stream);
    launch_multi_axpy<R>(x, V, nn, m, st + 2, y, 1, 1.0, nn, nullptr, stream);
    launch_gmres_cycle_end(st, stream);
    if (check_every > 0) {
      last = chk.now();
      if (!last[1]) break;
    }
  }
  if (check_every > 0) return (last ? last : chk.now())[3];
  return -1;
}

// ---------------------------------------------------------------- cycle
// One application of the preconditioner rooted at level l: restrict, coarse
// correction (GMRES on the coarsest level, FGMRES preconditioned by the next
// cycle for a K-cycle, or the next V-cycle), prolong, post-smooth with MR.
template <typename R>
void Context::cycle(int l, const cplx<R>* r, cplx<R>* x, const int* run, cd64* x64) {
  const int lc = l + 1;
  const std::string t = std::to_string(lc) + (sizeof(R) == 8 ? "d" : "f");
  const long nc = n(lc);
  cplx<R>* rc = buf<cplx<R>>("cyc_rc" + t, nc);
  cplx<R>* ec = buf<cplx<R>>("cyc_ec" + t, nc);
  restrict_<R>(l, r, rc, 1, run);
  std::function<void(const cplx<R>*, cplx<R>*, const int*)> A = [this, lc](const cplx<R>* i, cplx<R>* o,
                                                                              const int* rn) {
    apply_op<R>(lc, i, o, 1, rn);
  };
  const int check = (p.reserved[0] & 1) ? 0 : 4;  // reserved[0] bit 0: no host checks inside cycles
  if (lc + 1 >= nlev && cg_fused_supported(geo[lc].ns) && !(p.reserved[0] & 2)) {
    int it = coarse_gmres<R>(lc, rc, ec, run, check);
    if (it > 0) coarse_iters += it;
  } else if (lc + 1 >= nlev) {
    GmresState& G = gmres_state("cg" + t, p.coarse_restart, nc, sizeof(R) == 8 ? 0 : 1, false);
    int it = gmres<R>(G, A, nullptr, rc, ec, true, p.coarse_restart, p.coarse_maxit, p.coarse_tol,
                      p.coarse_fixed_iters, true, run, check);
    if (it > 0) coarse_iters += it;
  } else if (p.kcycle) {
    std::function<void(const cplx<R>*, cplx<R>*, const int*)> Mc = [this, lc](const cplx<R>* i, cplx<R>* o,
                                                                               const int* rn) { cycle<R>(lc, i, o, rn); };
    GmresState& G = gmres_state("kc" + t, p.kcycle_maxit, nc, sizeof(R) == 8 ? 0 : 1, true);
    gmres<R>(G, A, &Mc, rc, ec, true, p.kcycle_maxit, p.kcycle_maxit, p.kcycle_tol, 0, true, run, 0);
  } else {
    cycle<R>(lc, rc, ec, run);
  }
  prolong_<R>(l, ec, x, 0, 1, run);
  if (l == 0 && p.smoother == 1) {
    sap<R>(r, x, p.post_smooth, 1, run, 0);
    if (x64) launch_convert<R, double>(x, x64, n(l), run, stream);
  } else if (l == 0) {
    mr<R>(l, r, x, false, p.post_smooth, run, x64);
  } else {
    mr<R>(l, r, x, false, p.post_smooth, run);
    if (x64) launch_convert<R, double>(x, x64, n(l), run, stream);
  }
  cycles++;
}

// Even-odd preconditioning (Sec. 2.1, Sec. 4: red-black preconditioning):
// the site parity table in device order and A^{-1} per site.
void Context::eo_prepare() {
  if (eo_ready) return;
  require(gauge_set, WCMG_ERR_STATE, "gauge field not set");
  const LevelGeom& G = geo[0];
  std::vector<unsigned char> par(G.V);
  for (long s = 0; s < G.V; ++s) {
    int x[4];
    lex_coords(G.perm[s], G.L, x);
    par[s] = (unsigned char)((x[0] + x[1] + x[2] + x[3]) & 1);
  }
  par0.alloc(G.V);
  WCMG_HIP(hipMemcpy(par0.p, par.data(), G.V, hipMemcpyHostToDevice));
  std::vector<int> odd, even, pos(G.V, 0);
  for (long s = 0; s < G.V; ++s) {
    std::vector<int>& list = par[s] ? odd : even;
    pos[s] = (int)list.size();
    list.push_back((int)s);
  }
  require(2 * (long)odd.size() == G.V, WCMG_ERR_DIMS, "even-odd preconditioning needs as many odd as even sites");
  upload(eo_odd, odd);
  upload(eo_even, even);
  upload(eo_pos, pos);
  eo_half = (long)odd.size();
  clovinv64.alloc(clov64.bytes);
  clovinv32.alloc(clov32.bytes);
  int* bad = (int*)(scratch64.as<cd64>() + 32);
  WCMG_HIP(hipMemsetAsync(bad, 0, sizeof(int), stream));
  launch_clover_invert(clov64.as<double>(), G.V, clovinv64.as<double>(), clovinv32.as<float>(), bad, stream);
  WCMG_HIP(hipMemcpyAsync(pinned + 8, bad, sizeof(int), hipMemcpyDeviceToHost, stream));
  sync();
  require(pinned[8] == 0, WCMG_ERR_BREAKDOWN, "singular clover block: (4 + m0) + C has no inverse");
  eo_ready = true;
}

// y_o = A_oo x_o - H_oe A_ee^{-1} H_eo x_o on parity-compact fields: two
// launches, each the hops into one parity's sites with the site-local block
// in its epilogue (A^{-1} on the even sites, then A on the odd ones).
void Context::schur64c(const cd64* xo, cd64* yo, const int* run) {
  const long V = geo[0].V, Vh = eo_half;
  cd64* ue = buf<cd64>("eo_ue", 12 * Vh);
  const int* nbr = geo[0].nbr.as<int>();
  launch_schur_hop<double>(xo, ue, nullptr, U64.as<cd64>(), clovinv64.as<double>(), nbr, eo_even.as<int>(),
                           eo_pos.as<int>(), V, Vh, 0, run, stream);
  launch_schur_hop<double>(ue, yo, xo, U64.as<cd64>(), clov64.as<double>(), nbr, eo_odd.as<int>(), eo_pos.as<int>(),
                           V, Vh, 1, run, stream);
}

// The same on full-length fields (the even part of x is ignored, that of y
// is zero): gather the odd sites, apply, scatter.
void Context::schur64(const cd64* x, cd64* y, const int* run) {
  const long V = geo[0].V, Vh = eo_half;
  cd64* xo = buf<cd64>("eo_xo", 12 * Vh);
  cd64* yo = buf<cd64>("eo_yo", 12 * Vh);
  launch_eo_gather<double>(x, xo, eo_odd.as<int>(), V, Vh, stream);
  schur64c(xo, yo, run);
  launch_eo_scatter<double>(yo, y, eo_pos.as<int>(), (const unsigned char*)par0.p, V, Vh, stream);
}

// SAP domains: the level-0 aggregates, coloured by the parity of their coarse
// coordinates (two colours need every coarse extent even; a domain is one
// aggregate of at most 256 sites, contiguous in the device site order).
void Context::sap_prepare() {
  if (sap_ndoms > 0) return;
  require(nlev >= 2, WCMG_ERR_ARG, "SAP uses the level-0 aggregates as domains: n_levels >= 2");
  const LevelGeom& Gc = geo[1];
  for (int m = 0; m < 4; ++m)
    require(Gc.L[m] % 2 == 0, WCMG_ERR_DIMS, "SAP needs an even number of aggregates in every direction");
  require(tr[0].A <= 256, WCMG_ERR_ARG, "SAP domains (aggregates) hold at most 256 sites");
  std::vector<int> lists[2];
  for (long c = 0; c < Gc.V; ++c) {
    int x[4];
    lex_coords(c, Gc.L, x);
    lists[(x[0] + x[1] + x[2] + x[3]) & 1].push_back((int)c);
  }
  std::vector<int> both(lists[0]);
  both.insert(both.end(), lists[1].begin(), lists[1].end());
  upload(sap_doms, both);
  sap_ndoms = (long)lists[0].size();
}

template <typename R>
void Context::sap(const cplx<R>* b, cplx<R>* x, int cycles, int nrhs, const int* run, int rs) {
  sap_prepare();
  const bool single = sizeof(R) == 4;
  const cplx<R>* U = single ? (const cplx<R>*)U32.as<cf32>() : (const cplx<R>*)U64.as<cd64>();
  const R* clov = single ? (const R*)clov32.as<float>() : (const R*)clov64.as<double>();
  const char* fam = single ? "sap_f32" : "sap_f64";
  for (int c = 0; c < cycles; ++c)
    for (int colour = 0; colour < 2; ++colour) {
      prof.begin_kernel(fam);
      launch_sap<R>(x, b, U, clov, geo[0].nbr.as<int>(), geo[0].V, tr[0].A, sap_doms.as<int>() + colour * sap_ndoms,
                    (int)sap_ndoms, p.sap_block_iters, nrhs, run, rs, stream);
      prof.end(fam, stream);
    }
}
template void Context::sap<double>(const cd64*, cd64*, int, int, const int*, int);
template void Context::sap<float>(const cf32*, cf32*, int, int, const int*, int);

void Context::precondition64(int l, const cd64* r, cd64* x, const int* run) {
  if (p.cycle_prec == WCMG_F64) {
    cycle<double>(l, r, x, run);
    return;
  }
  const long nn = n(l);
  const std::string t = std::to_string(l);
  cf32* r32 = buf<cf32>("pc_r32" + t, nn);
  cf32* x32 = buf<cf32>("pc_x32" + t, nn);
  launch_convert<double, float>(r, r32, nn, run, stream);
  cycle<float>(l, r32, x32, run, x);
}

// ---------------------------------------------------------------- setup
void Context::rebuild(int l) {
  Transfer& T = tr[l];
  const LevelGeom& G = geo[l];
  const long nn = G.n();
  auto t0 = std::chrono::steady_clock::now();
  WCMG_HIP(hipMemcpyAsync(T.P64.p, T.vecs64.p, T.nv * nn * sizeof(cd64), hipMemcpyDeviceToDevice, stream));
  int* flag = (int*)(scratch64.as<cd64>() + 32);
  WCMG_HIP(hipMemsetAsync(flag, 0, sizeof(int), stream));
  launch_block_orthonormalise(T.P64.as<cd64>(), G.lay, T.agg_sites.as<int>(), T.A, T.Vc, T.nv, flag, stream);
  launch_convert<double, float>(T.P64.as<cd64>(), T.P32.as<cf32>(), T.nv * nn, nullptr, stream);
  WCMG_HIP(hipMemcpyAsync(pinned + 8, flag, sizeof(int), hipMemcpyDeviceToHost, stream));
  sync();
  timers[2] += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  require(pinned[8] == 0, WCMG_ERR_BREAKDOWN, "Gram-Schmidt breakdown at level " + std::to_string(l));
  galerkin(l);
  T.built = true;
}

// Galerkin coarse operator (Sec. 2.1 CoarsenOperator): Mdiag and the four
// forward terms Mdir_{+mu} of the level operator are applied to every column
// of P and projected on P aggregate by aggregate; the four backward terms
// follow from gamma5-hermiticity (Sec. 4: five of the nine stencil points are
// independent), which halves the hop work.
void Context::galerkin(int l) {
  auto t0 = std::chrono::steady_clock::now();
  Transfer& T = tr[l];
  const LevelGeom& G = geo[l];
  CoarseOp& C = *cop[l];
  const long nn = G.n();
  WCMG_HIP(hipMemsetAsync(C.M64.p, 0, C.M64.bytes, stream));
  if (l == 0) {
    // fine level: the images of P's columns under each term are formed inside
    // the projection (no intermediate fields)
    for (int d = 0; d <= 7; d += d == 0 ? 1 : 2)
      launch_galerkin_fused(T.P64.as<cd64>(), U64.as<cd64>(), clov64.as<double>(), G.nbr.as<int>(), G.V,
                            T.agg_sites.as<int>(), T.coarse_of.as<int>(), T.A, T.Vc, T.nb, d, d == 0 ? 0 : d + 1,
                            C.M64.as<cd64>(), stream);
  } else {
    cd64* cols = buf<cd64>("gal_cols" + std::to_string(l), (long)T.nb * nn);
    cd64* W = buf<cd64>("gal_W" + std::to_string(l), (long)T.nb * nn);
    launch_prolongator_columns(T.P64.as<cd64>(), G.lay, T.nv, cols, stream);
    for (int d = 0; d <= 7; d += d == 0 ? 1 : 2) {
      apply_op<double>(l, cols, W, T.nb, nullptr, 1 << d);
      const int* nbr_d = d == 0 ? nullptr : G.nbr.as<int>() + (long)(d - 1) * G.V;
      launch_galerkin_project(W, T.P64.as<cd64>(), G.lay, T.agg_sites.as<int>(), T.coarse_of.as<int>(), nbr_d, T.A,
                              T.Vc, T.nb, d, d == 0 ? 0 : d + 1, C.M64.as<cd64>(), stream);
    }
  }
  launch_galerkin_mirror(C.M64.as<cd64>(), C.nbr.as<int>(), T.Vc, T.nb, stream);
  C.invalidate();
  C.refresh(WCMG_F64, stream);
  if (p.cycle_prec == WCMG_F32 || p.setup_prec == WCMG_F32) C.refresh(store_prec_for(l + 1, true), stream);
  sync();
  timers[3] += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

void Context::regalerkin_below(int l) {
  // down to the first level whose prolongator has not been built yet
  for (int k = l + 1; k + 1 < nlev && tr[k].built; ++k) galerkin(k);
}

// Initial setup (Sec. 2.1): iterate the smoother on random vectors.  Reading:
// relax_sweeps MR steps on D x = 0 from each start vector, then normalise.
void Context::initial_setup(int l) {
  Transfer& T = tr[l];
  require(T.has_start, WCMG_ERR_STATE, "start vectors of level " + std::to_string(l) + " not set");
  WCMG_HIP(hipMemcpyAsync(T.vecs64.p, T.start64.p, T.nv * n(l) * sizeof(cd64), hipMemcpyDeviceToDevice, stream));
  relax_vectors(l, p.relax_sweeps);
  rebuild(l);
}

// `sweeps` MR steps on D x = 0 from each of the level's current vectors (all
// vectors advance together through the batched smoother), then normalise.
void Context::relax_vectors(int l, int sweeps) {
  Transfer& T = tr[l];
  const long nn = n(l);
  auto t0 = std::chrono::steady_clock::now();
  cd64* v = T.vecs64.as<cd64>();
  if (sweeps > 0) {
    if (p.setup_prec == WCMG_F64) {
      mrB<double>(l, nullptr, v, T.nv, sweeps, nullptr, 0);
    } else {
      cf32* x32 = buf<cf32>("relax32_" + std::to_string(l), T.nv * nn);
      launch_convert<double, float>(v, x32, T.nv * nn, nullptr, stream);
      mrB<float>(l, nullptr, x32, T.nv, sweeps, nullptr, 0);
      launch_convert<float, double>(x32, v, T.nv * nn, nullptr, stream);
    }
  }
  cd64* nrm = scratch64.as<cd64>() + 16;
  for (int i = 0; i < T.nv; ++i) {
    cd64* x = v + (long)i * nn;
    launch_dot<double>(x, 0, 1, nullptr, x, nn, partial.as<cd64>(), 1, nrm, 1, 0, nullptr, stream);
    launch_scale_inv_norm<double>(x, x, nrm, nn, nullptr, stream);
  }
  sync();
  timers[1] += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Iterative setup (Sec. 2.1, DDalphaAMG-style).  One iteration at level l:
// each vector is replaced by the preconditioner rooted at l applied to it
// (zero initial guess) and normalised; then P_l and D_{l+1} are rebuilt, the
// Galerkin products below are re-taken and the next level is refined.
void Context::refine_iteration(int l) {
  Transfer& T = tr[l];
  const long nn = n(l);
  cd64* y = buf<cd64>("ref_y" + std::to_string(l), nn);
  cd64* nrm = scratch64.as<cd64>() + 20;
  for (int i = 0; i < T.nv; ++i) {
    cd64* v = T.vecs64.as<cd64>() + (long)i * nn;
    precondition64(l, v, y, nullptr);
    launch_dot<double>(y, 0, 1, nullptr, y, nn, partial.as<cd64>(), 1, nrm, 1, 0, nullptr, stream);
    launch_scale_inv_norm<double>(v, y, nrm, nn, nullptr, stream);
  }
  rebuild(l);
  regalerkin_below(l);
  if (l + 2 < nlev) refine_iteration(l + 1);
}

void Context::setup_all() {
  require(gauge_set, WCMG_ERR_STATE, "gauge field not set");
  auto t0 = std::chrono::steady_clock::now();
  for (int q = 0; q < 5; ++q) timers[q] = 0.0;
  for (int l = 0; l + 1 < nlev; ++l) initial_setup(l);
  auto t1 = std::chrono::steady_clock::now();
  for (int it = 0; it < p.refine_iters; ++it) refine_iteration(0);
  sync();
  auto t2 = std::chrono::steady_clock::now();
  timers[4] = std::chrono::duration<double>(t2 - t1).count();
  timers[0] = std::chrono::duration<double>(t2 - t0).count();
  setup_done = true;
}

// ---------------------------------------------------------------- instantiations
template void Context::apply_op<double>(int, const cd64*, cd64*, int, const int*, int, cd64*);
template void Context::apply_op<float>(int, const cf32*, cf32*, int, const int*, int, cd64*);
template void Context::restrict_<double>(int, const cd64*, cd64*, int, const int*);
template void Context::restrict_<float>(int, const cf32*, cf32*, int, const int*);
template void Context::prolong_<double>(int, const cd64*, cd64*, int, int, const int*);
template void Context::prolong_<float>(int, const cf32*, cf32*, int, int, const int*);
template void Context::mr<double>(int, const cd64*, cd64*, bool, int, const int*, cd64*);
template void Context::mr<float>(int, const cf32*, cf32*, bool, int, const int*, cd64*);
template void Context::cycle<double>(int, const cd64*, cd64*, const int*, cd64*);
template int Context::coarse_gmres<double>(int, const cd64*, cd64*, const int*, int);
template int Context::coarse_gmres<float>(int, const cf32*, cf32*, const int*, int);
template void Context::cycle<float>(int, const cf32*, cf32*, const int*, cd64*);
template int Context::gmres<double>(GmresState&, const std::function<void(const cd64*, cd64*, const int*)>&,
                                    const std::function<void(const cd64*, cd64*, const int*)>*, const cd64*, cd64*,
                                    bool, int, int, double, int, bool, const int*, int, bool);
template int Context::gmres<float>(GmresState&, const std::function<void(const cf32*, cf32*, const int*)>&,
                                   const std::function<void(const cf32*, cf32*, const int*)>*, const cf32*, cf32*,
                                   bool, int, int, double, int, bool, const int*, int, bool);
template double Context::norm2_host<double>(const cd64*, long);
template double Context::norm2_host<float>(const cf32*, long);
template cd64* Context::buf<cd64>(const std::string&, long);
template cf32* Context::buf<cf32>(const std::string&, long);

}  // namespace wcmg
