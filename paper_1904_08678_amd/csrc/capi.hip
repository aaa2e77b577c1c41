// extern "C" boundary of the wcmg library (declared in include/wcmg.h).
// Every entry point converts internal exceptions into a wcmg_status and keeps
// the message for wcmg_last_error.
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>

#include "engine.h"

using namespace wcmg;

struct wcmg_ctx {
  std::unique_ptr<Context> c;
  std::string err;
};

static thread_local std::string g_create_error;

namespace {

template <typename F>
int guarded(wcmg_ctx* h, F&& f) {
  if (!h || !h->c) return WCMG_ERR_ARG;
  try {
    f(*h->c);
    h->err.clear();
    return WCMG_OK;
  } catch (const Error& e) {
    h->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    h->err = e.what();
    return WCMG_ERR_HIP;
  }
}

void check_level(const Context& c, int level, bool need_coarse) {
  require(level >= 0 && level < c.nlev, WCMG_ERR_ARG, "level out of range");
  if (need_coarse) require(level + 1 < c.nlev, WCMG_ERR_ARG, "level has no coarser level");
}

void check_prec(int prec, bool allow_bf16) {
  require(prec == WCMG_F64 || prec == WCMG_F32 || (allow_bf16 && prec == WCMG_BF16), WCMG_ERR_ARG,
          "unsupported precision");
}

// ||b - D x|| / ||b|| from the squared norms; 0 for b = 0, NaN when either
// norm is not finite (so that a NaN in b or x is reported, never taken for
// convergence).
double true_rel_res(double rr, double bb) {
  if (!std::isfinite(rr) || !std::isfinite(bb)) return std::numeric_limits<double>::quiet_NaN();
  return bb > 0 ? std::sqrt(rr / bb) : 0.0;
}

}  // namespace

extern "C" {

void wcmg_default_params(wcmg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->dims[0] = p->dims[1] = p->dims[2] = p->dims[3] = 8;
  p->m0 = -0.05;
  p->c_sw = 1.0;
  p->antiperiodic_t = 1;
  p->n_levels = 2;
  for (int l = 0; l < 3; ++l)
    for (int m = 0; m < 4; ++m) p->block[l][m] = 4;
  p->n_vec[0] = p->n_vec[1] = p->n_vec[2] = 12;
  p->relax_sweeps = 20;
  p->refine_iters = 0;
  p->post_smooth = 4;
  p->coarse_restart = 20;
  p->coarse_maxit = 100;
  p->coarse_fixed_iters = 0;
  p->coarse_tol = 0.05;
  p->kcycle = 0;
  p->kcycle_maxit = 5;
  p->kcycle_tol = 0.1;
  p->outer_restart = 20;
  p->outer_maxit = 1000;
  p->outer_tol = 1e-10;
  p->sap_block_iters = 4;
  p->cycle_prec = WCMG_F64;
  p->coarse_store_prec = WCMG_F64;
  p->setup_prec = WCMG_F64;
}

int wcmg_create(const wcmg_params* p, void* stream, wcmg_ctx** out) {
  if (!p || !out) return WCMG_ERR_ARG;
  *out = nullptr;
  wcmg_ctx* h = new wcmg_ctx();
  try {
    h->c.reset(new Context(*p, (hipStream_t)stream));
  } catch (const Error& e) {
    g_create_error = e.what();
    delete h;
    return e.code;
  }
  *out = h;
  return WCMG_OK;
}

int wcmg_destroy(wcmg_ctx* ctx) {
  if (!ctx) return WCMG_ERR_ARG;
  if (ctx->c) (void)hipStreamSynchronize(ctx->c->stream);
  delete ctx;
  return WCMG_OK;
}

const char* wcmg_last_error(const wcmg_ctx* ctx) {
  if (!ctx) return g_create_error.c_str();
  if (ctx->err.empty() && ctx->c && !ctx->c->cgp_last_report.empty()) return ctx->c->cgp_last_report.c_str();
  return ctx->err.c_str();
}

int wcmg_set_gauge(wcmg_ctx* ctx, const void* U) {
  return guarded(ctx, [&](Context& c) {
    require(U != nullptr, WCMG_ERR_ARG, "null gauge field");
    c.set_gauge((const cd64*)U);
  });
}

int wcmg_set_clover(wcmg_ctx* ctx, const void* blocks) {
  return guarded(ctx, [&](Context& c) {
    require(c.gauge_set, WCMG_ERR_STATE, "set the gauge field first");
    if (blocks) c.set_clover((const cd64*)blocks);
    else c.set_gauge(c.U_lex.as<cd64>());
  });
}

int wcmg_get_clover(wcmg_ctx* ctx, void* blocks) {
  return guarded(ctx, [&](Context& c) {
    require(c.gauge_set && blocks, WCMG_ERR_STATE, "no clover term");
    WCMG_HIP(hipMemcpyAsync(blocks, c.clover_lex.p, c.geo[0].V * 72 * sizeof(cd64), hipMemcpyDeviceToDevice,
                            c.stream));
    c.sync();
  });
}

static void level_vectors_in(Context& c, int level, const cd64* src, cd64* dst, int nv) {
  const LevelGeom& G = c.geo[level];
  if (level == 0) launch_pack_fermion<double, double>(src, c.perm0.as<int>(), G.V, nv, dst, c.stream);
  else WCMG_HIP(hipMemcpyAsync(dst, src, (size_t)nv * G.n() * sizeof(cd64), hipMemcpyDeviceToDevice, c.stream));
}
static void level_vectors_out(Context& c, int level, const cd64* src, cd64* dst, int nv) {
  const LevelGeom& G = c.geo[level];
  if (level == 0) launch_unpack_fermion<double, double>(src, c.perm0.as<int>(), G.V, nv, dst, c.stream);
  else WCMG_HIP(hipMemcpyAsync(dst, src, (size_t)nv * G.n() * sizeof(cd64), hipMemcpyDeviceToDevice, c.stream));
}

int wcmg_set_null_vectors(wcmg_ctx* ctx, int level, const void* v, int nv) {
  return guarded(ctx, [&](Context& c) {
    check_level(c, level, true);
    require(v && nv == c.tr[level].nv, WCMG_ERR_ARG, "expected n_vec start vectors");
    level_vectors_in(c, level, (const cd64*)v, c.tr[level].start64.as<cd64>(), nv);
    c.tr[level].has_start = true;
    c.sync();
  });
}

int wcmg_get_null_vectors(wcmg_ctx* ctx, int level, void* v) {
  return guarded(ctx, [&](Context& c) {
    check_level(c, level, true);
    require(c.tr[level].built && v, WCMG_ERR_STATE, "near-null vectors not built");
    level_vectors_out(c, level, c.tr[level].vecs64.as<cd64>(), (cd64*)v, c.tr[level].nv);
    c.sync();
  });
}

int wcmg_get_prolongator(wcmg_ctx* ctx, int level, void* v) {
  return guarded(ctx, [&](Context& c) {
    check_level(c, level, true);
    require(c.tr[level].built && v, WCMG_ERR_STATE, "prolongator not built");
    level_vectors_out(c, level, c.tr[level].P64.as<cd64>(), (cd64*)v, c.tr[level].nv);
    c.sync();
  });
}

int wcmg_setup(wcmg_ctx* ctx) {
  return guarded(ctx, [&](Context& c) { c.setup_all(); });
}

int wcmg_refine(wcmg_ctx* ctx, int iterations) {
  return guarded(ctx, [&](Context& c) {
    require(c.setup_done, WCMG_ERR_STATE, "run wcmg_setup first");
    require(iterations >= 0, WCMG_ERR_ARG, "negative iteration count");
    auto t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < iterations; ++i) c.refine_iteration(0);
    c.sync();
    c.timers[4] += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  });
}

int wcmg_rebuild_from_vectors(wcmg_ctx* ctx, int level, const void* v) {
  return guarded(ctx, [&](Context& c) {
    check_level(c, level, true);
    require(c.gauge_set && v, WCMG_ERR_STATE, "gauge field not set");
    for (int l = 0; l < level; ++l) require(c.tr[l].built, WCMG_ERR_STATE, "finer levels not built");
    level_vectors_in(c, level, (const cd64*)v, c.tr[level].vecs64.as<cd64>(), c.tr[level].nv);
    c.rebuild(level);
    c.regalerkin_below(level);
    // a hierarchy whose every level has been built from given vectors is ready to cycle and solve
    bool all = true;
    for (int l = 0; l + 1 < c.nlev; ++l) all = all && c.tr[l].built;
    if (all) c.setup_done = true;
  });
}

namespace {
constexpr size_t kCkptHeader = 128;
const char kCkptMagic[8] = {'W', 'C', 'M', 'G', 'S', 'E', 'T', '1'};

uint64_t ckpt_hash(const unsigned char* p, size_t n) {  // 64-bit FNV-1a over 8-byte words
  uint64_t h = 1469598103934665603ull;
  size_t i = 0;
  for (; i + 8 <= n; i += 8) {
    uint64_t w;
    std::memcpy(&w, p + i, 8);
    h = (h ^ w) * 1099511628211ull;
  }
  for (; i < n; ++i) h = (h ^ p[i]) * 1099511628211ull;
  return h;
}

size_t ckpt_payload(const Context& c) {
  size_t b = 0;
  for (int l = 0; l + 1 < c.nlev; ++l) b += (size_t)c.tr[l].nv * c.geo[l].n() * sizeof(cd64);
  return b;
}

void ckpt_header(const Context& c, unsigned char* h, uint64_t payload, uint64_t hash) {
  std::memset(h, 0, kCkptHeader);
  std::memcpy(h, kCkptMagic, 8);
  const uint32_t ver = 1, nl = (uint32_t)c.nlev;
  std::memcpy(h + 8, &ver, 4);
  std::memcpy(h + 12, &nl, 4);
  std::memcpy(h + 16, c.p.dims, 16);
  for (int l = 0; l + 1 < c.nlev; ++l) {
    std::memcpy(h + 32 + 16 * l, c.p.block[l], 16);
    std::memcpy(h + 80 + 4 * l, &c.p.n_vec[l], 4);
  }
  std::memcpy(h + 92, &c.p.antiperiodic_t, 4);
  std::memcpy(h + 96, &c.p.m0, 8);
  std::memcpy(h + 104, &c.p.c_sw, 8);
  std::memcpy(h + 112, &payload, 8);
  std::memcpy(h + 120, &hash, 8);
}
}  // namespace

int wcmg_setup_export(wcmg_ctx* ctx, void* buf, size_t capacity, size_t* bytes) {
  return guarded(ctx, [&](Context& c) {
    require(bytes != nullptr, WCMG_ERR_ARG, "null size output");
    require(c.nlev >= 2, WCMG_ERR_STATE, "no multigrid hierarchy to export");
    require(c.setup_done, WCMG_ERR_STATE, "run wcmg_setup first");
    const size_t payload = ckpt_payload(c);
    *bytes = kCkptHeader + payload;
    if (!buf) return;
    require(capacity >= kCkptHeader + payload, WCMG_ERR_ARG, "export buffer too small");
    unsigned char* out = (unsigned char*)buf;
    size_t off = kCkptHeader;
    for (int l = 0; l + 1 < c.nlev; ++l) {
      const int nv = c.tr[l].nv;
      const size_t nb = (size_t)nv * c.geo[l].n() * sizeof(cd64);
      cd64* tmp = c.buf<cd64>("ckpt", (long)nv * c.geo[l].n());
      level_vectors_out(c, l, c.tr[l].vecs64.as<cd64>(), tmp, nv);
      WCMG_HIP(hipMemcpyAsync(out + off, tmp, nb, hipMemcpyDeviceToHost, c.stream));
      c.sync();
      off += nb;
    }
    ckpt_header(c, out, payload, ckpt_hash(out + kCkptHeader, payload));
  });
}

int wcmg_setup_import(wcmg_ctx* ctx, const void* buf, size_t bytes) {
  return guarded(ctx, [&](Context& c) {
    require(buf != nullptr, WCMG_ERR_ARG, "null checkpoint");
    require(c.nlev >= 2, WCMG_ERR_STATE, "no multigrid hierarchy to import");
    require(c.gauge_set, WCMG_ERR_STATE, "set the gauge field first");
    require(bytes >= kCkptHeader, WCMG_ERR_ARG, "checkpoint truncated");
    const unsigned char* in = (const unsigned char*)buf;
    require(std::memcmp(in, kCkptMagic, 8) == 0, WCMG_ERR_ARG, "not a setup checkpoint");
    const size_t payload = ckpt_payload(c);
    unsigned char want[kCkptHeader];
    uint64_t have_payload = 0, have_hash = 0;
    std::memcpy(&have_payload, in + 112, 8);
    std::memcpy(&have_hash, in + 120, 8);
    ckpt_header(c, want, payload, have_hash);
    require(std::memcmp(in, want, 112) == 0, WCMG_ERR_ARG,
            "checkpoint was written for another lattice, hierarchy or operator");
    require(have_payload == payload && bytes == kCkptHeader + payload, WCMG_ERR_ARG, "checkpoint size mismatch");
    require(ckpt_hash(in + kCkptHeader, payload) == have_hash, WCMG_ERR_ARG, "checkpoint checksum mismatch");
    auto t0 = std::chrono::steady_clock::now();
    c.setup_done = false;
    for (int q = 0; q < 5; ++q) c.timers[q] = 0.0;
    size_t off = kCkptHeader;
    for (int l = 0; l + 1 < c.nlev; ++l) {
      const int nv = c.tr[l].nv;
      const size_t nb = (size_t)nv * c.geo[l].n() * sizeof(cd64);
      cd64* tmp = c.buf<cd64>("ckpt", (long)nv * c.geo[l].n());
      WCMG_HIP(hipMemcpyAsync(tmp, in + off, nb, hipMemcpyHostToDevice, c.stream));
      level_vectors_in(c, l, tmp, c.tr[l].vecs64.as<cd64>(), nv);
      c.rebuild(l);
      off += nb;
    }
    c.sync();
    c.timers[0] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    c.setup_done = true;
  });
}

int wcmg_get_aggregate_map(wcmg_ctx* ctx, int level, int32_t* coarse_host, int32_t* offset_host) {
  return guarded(ctx, [&](Context& c) {
    check_level(c, level, true);
    require(coarse_host && offset_host, WCMG_ERR_ARG, "null output");
    const Transfer& T = c.tr[level];
    std::memcpy(coarse_host, T.agg_host.data(), T.agg_host.size() * sizeof(int32_t));
    std::memcpy(offset_host, T.off_host.data(), T.off_host.size() * sizeof(int32_t));
  });
}

int wcmg_get_coarse_op(wcmg_ctx* ctx, int level, void* blocks, int prec) {
  return guarded(ctx, [&](Context& c) {
    require(level >= 1 && level < c.nlev && blocks, WCMG_ERR_ARG, "level must name a coarse level");
    require(prec == WCMG_F64 || prec == WCMG_F32 || prec == WCMG_BF16, WCMG_ERR_ARG, "bad precision");
    CoarseOp& C = *c.cop[level - 1];
    require(prec != WCMG_BF16 || C.nb % 4 == 0, WCMG_ERR_ARG, "BF16 storage needs Nb divisible by 4");
    if (prec == WCMG_F64)
      WCMG_HIP(hipMemcpyAsync(blocks, C.M64.p, C.M64.bytes, hipMemcpyDeviceToDevice, c.stream));
    else
      launch_c128_to_c64(C.M64.as<cd64>(), (cf32*)blocks, (long)(C.M64.bytes / sizeof(cd64)), prec == WCMG_BF16,
                         c.stream);
    c.sync();
  });
}

int wcmg_set_coarse_op(wcmg_ctx* ctx, int level, const void* blocks, int prec) {
  return guarded(ctx, [&](Context& c) {
    require(level >= 1 && level < c.nlev && blocks, WCMG_ERR_ARG, "level must name a coarse level");
    require(prec == WCMG_F64 || prec == WCMG_F32, WCMG_ERR_ARG,
            "blocks are given in FP64 or FP32 (BF16 is a storage format of the cycle)");
    CoarseOp& C = *c.cop[level - 1];
    if (prec == WCMG_F64)
      WCMG_HIP(hipMemcpyAsync(C.M64.p, blocks, C.M64.bytes, hipMemcpyDeviceToDevice, c.stream));
    else
      launch_c64_to_c128((const cf32*)blocks, C.M64.as<cd64>(), (long)(C.M64.bytes / sizeof(cd64)), c.stream);
    C.invalidate();
    C.refresh(WCMG_F64, c.stream);
    C.refresh(WCMG_F32, c.stream);
    if (C.nb % 4 == 0) C.refresh(WCMG_BF16, c.stream);
    c.sync();
  });
}

int wcmg_apply_schur(wcmg_ctx* ctx, const void* in, void* out, int nrhs) {
  return guarded(ctx, [&](Context& c) {
    require(in && out && nrhs >= 1, WCMG_ERR_ARG, "bad fields");
    c.eo_prepare();
    const long V = c.geo[0].V, nn = c.n(0);
    cd64* a = c.buf<cd64>("abi_a64", nn);
    cd64* bb = c.buf<cd64>("abi_b64", nn);
    const unsigned char* par = (const unsigned char*)c.par0.p;
    for (int k = 0; k < nrhs; ++k) {
      launch_pack_fermion<double, double>((const cd64*)in + k * nn, c.perm0.as<int>(), V, 1, a, c.stream);
      launch_eo_local<double>(a, nullptr, a, nullptr, par, 1, 2, V, c.stream);  // even part dropped
      c.schur64(a, bb, nullptr);
      launch_unpack_fermion<double, double>(bb, c.perm0.as<int>(), V, 1, (cd64*)out + k * nn, c.stream);
    }
    WCMG_HIP(hipStreamSynchronize(c.stream));
  });
}

int wcmg_sap(wcmg_ctx* ctx, const void* b, void* x, int nrhs, int cycles, int prec) {
  return guarded(ctx, [&](Context& c) {
    check_prec(prec, false);
    require(b && x && nrhs >= 1 && cycles >= 0, WCMG_ERR_ARG, "bad fields or cycle count");
    require(c.gauge_set, WCMG_ERR_STATE, "gauge field not set");
    c.sap_prepare();
    const long V = c.geo[0].V, nn = c.n(0);
    if (prec == WCMG_F64) {
      cd64* bb = c.buf<cd64>("abi_a64", nn * nrhs);
      cd64* xx = c.buf<cd64>("abi_b64", nn * nrhs);
      launch_pack_fermion<double, double>((const cd64*)b, c.perm0.as<int>(), V, nrhs, bb, c.stream);
      launch_pack_fermion<double, double>((const cd64*)x, c.perm0.as<int>(), V, nrhs, xx, c.stream);
      c.sap<double>(bb, xx, cycles, nrhs, nullptr, 0);
      launch_unpack_fermion<double, double>(xx, c.perm0.as<int>(), V, nrhs, (cd64*)x, c.stream);
    } else {
      cf32* bb = c.buf<cf32>("abi_a32", nn * nrhs);
      cf32* xx = c.buf<cf32>("abi_b32", nn * nrhs);
      launch_pack_fermion<float, float>((const cf32*)b, c.perm0.as<int>(), V, nrhs, bb, c.stream);
      launch_pack_fermion<float, float>((const cf32*)x, c.perm0.as<int>(), V, nrhs, xx, c.stream);
      c.sap<float>(bb, xx, cycles, nrhs, nullptr, 0);
      launch_unpack_fermion<float, float>(xx, c.perm0.as<int>(), V, nrhs, (cf32*)x, c.stream);
    }
    WCMG_HIP(hipStreamSynchronize(c.stream));
  });
}

int wcmg_apply_D(wcmg_ctx* ctx, int level, const void* in, void* out, int nrhs, int prec) {
  return guarded(ctx, [&](Context& c) {
    check_level(c, level, false);
    check_prec(prec, level > 0);
    require(in && out && nrhs >= 1, WCMG_ERR_ARG, "bad fields");
    if (level == 0) {
      require(c.gauge_set, WCMG_ERR_STATE, "gauge field not set");
      const long V = c.geo[0].V, nn = c.n(0);
      if (prec == WCMG_F64) {
        cd64* a = c.buf<cd64>("abi_a64", nn * nrhs);
        cd64* b = c.buf<cd64>("abi_b64", nn * nrhs);
        launch_pack_fermion<double, double>((const cd64*)in, c.perm0.as<int>(), V, nrhs, a, c.stream);
        c.apply_op<double>(0, a, b, nrhs, nullptr);
        launch_unpack_fermion<double, double>(b, c.perm0.as<int>(), V, nrhs, (cd64*)out, c.stream);
      } else {
        cf32* a = c.buf<cf32>("abi_a32", nn * nrhs);
        cf32* b = c.buf<cf32>("abi_b32", nn * nrhs);
        launch_pack_fermion<float, float>((const cf32*)in, c.perm0.as<int>(), V, nrhs, a, c.stream);
        if (nrhs >= 2) c.apply_opB<float>(0, a, b, nrhs, nullptr, 0);  // links and clover shared by the batch
        else c.apply_op<float>(0, a, b, nrhs, nullptr);
        launch_unpack_fermion<float, float>(b, c.perm0.as<int>(), V, nrhs, (cf32*)out, c.stream);
      }
    } else {
      CoarseOp& C = *c.cop[level - 1];
      require(C.built(WCMG_F64), WCMG_ERR_STATE, "coarse operator not built");
      if (prec != WCMG_F64) C.refresh(prec, c.stream);
      C.apply(prec, in, out, 0x1ff, 0, nrhs, nullptr, c.stream);
    }
    WCMG_HIP(hipStreamSynchronize(c.stream));
  });
}

int wcmg_restrict(wcmg_ctx* ctx, int level, const void* fine, void* coarse, int nrhs, int prec) {
  return guarded(ctx, [&](Context& c) {
    check_level(c, level, true);
    check_prec(prec, false);
    require(fine && coarse && nrhs >= 1, WCMG_ERR_ARG, "bad fields");
    require(c.tr[level].built, WCMG_ERR_STATE, "prolongator not built");
    const long V = c.geo[level].V, nn = c.n(level);
    if (prec == WCMG_F64) {
      const cd64* f = (const cd64*)fine;
      if (level == 0) {
        cd64* a = c.buf<cd64>("abi_a64", nn * nrhs);
        launch_pack_fermion<double, double>(f, c.perm0.as<int>(), V, nrhs, a, c.stream);
        f = a;
      }
      c.restrict_<double>(level, f, (cd64*)coarse, nrhs, nullptr);
    } else {
      const cf32* f = (const cf32*)fine;
      if (level == 0) {
        cf32* a = c.buf<cf32>("abi_a32", nn * nrhs);
        launch_pack_fermion<float, float>(f, c.perm0.as<int>(), V, nrhs, a, c.stream);
        f = a;
      }
      c.restrict_<float>(level, f, (cf32*)coarse, nrhs, nullptr);
    }
    WCMG_HIP(hipStreamSynchronize(c.stream));
  });
}

int wcmg_prolong(wcmg_ctx* ctx, int level, const void* coarse, void* fine, int nrhs, int prec) {
  return guarded(ctx, [&](Context& c) {
    check_level(c, level, true);
    check_prec(prec, false);
    require(fine && coarse && nrhs >= 1, WCMG_ERR_ARG, "bad fields");
    require(c.tr[level].built, WCMG_ERR_STATE, "prolongator not built");
    const long V = c.geo[level].V, nn = c.n(level);
    if (prec == WCMG_F64) {
      cd64* f = (cd64*)fine;
      if (level == 0) f = c.buf<cd64>("abi_b64", nn * nrhs);
      c.prolong_<double>(level, (const cd64*)coarse, f, 0, nrhs, nullptr);
      if (level == 0) launch_unpack_fermion<double, double>(f, c.perm0.as<int>(), V, nrhs, (cd64*)fine, c.stream);
    } else {
      cf32* f = (cf32*)fine;
      if (level == 0) f = c.buf<cf32>("abi_b32", nn * nrhs);
      c.prolong_<float>(level, (const cf32*)coarse, f, 0, nrhs, nullptr);
      if (level == 0) launch_unpack_fermion<float, float>(f, c.perm0.as<int>(), V, nrhs, (cf32*)fine, c.stream);
    }
    WCMG_HIP(hipStreamSynchronize(c.stream));
  });
}

int wcmg_cycle(wcmg_ctx* ctx, const void* r, void* x) {
  return guarded(ctx, [&](Context& c) {
    require(c.setup_done, WCMG_ERR_STATE, "run wcmg_setup first");
    require(c.nlev >= 2, WCMG_ERR_STATE, "no coarse level");
    require(r && x, WCMG_ERR_ARG, "bad fields");
    const long V = c.geo[0].V, nn = c.n(0);
    cd64* a = c.buf<cd64>("cyc_in", nn);
    cd64* b = c.buf<cd64>("cyc_out", nn);
    launch_pack_fermion<double, double>((const cd64*)r, c.perm0.as<int>(), V, 1, a, c.stream);
    c.precondition64(0, a, b, nullptr);
    launch_unpack_fermion<double, double>(b, c.perm0.as<int>(), V, 1, (cd64*)x, c.stream);
    c.sync();
  });
}

int wcmg_solve(wcmg_ctx* ctx, const void* b, void* x, int nrhs, wcmg_solve_info* info) {
  int status = WCMG_OK;
  int rc = guarded(ctx, [&](Context& c) {
    require(c.gauge_set, WCMG_ERR_STATE, "gauge field not set");
    require(c.nlev == 1 || c.setup_done, WCMG_ERR_STATE, "run wcmg_setup first");
    require(b && x && nrhs >= 1, WCMG_ERR_ARG, "bad fields");
    const long V = c.geo[0].V, nn = c.n(0);
    cd64* b64 = c.buf<cd64>("solve_b", nn);
    cd64* x64 = c.buf<cd64>("solve_x", nn);
    cd64* r64 = c.buf<cd64>("solve_r", nn);
    std::function<void(const cd64*, cd64*, const int*)> A = [&c](const cd64* i, cd64* o, const int* rn) {
      c.apply_op<double>(0, i, o, 1, rn);
    };
    std::function<void(const cd64*, cd64*, const int*)> M = [&c](const cd64* i, cd64* o, const int* rn) {
      if (c.nlev >= 2) c.precondition64(0, i, o, rn);
      else launch_convert<double, double>(i, o, c.n(0), rn, c.stream);
    };
    const bool sr = !(c.p.reserved[0] & 8);  // single-reduction Arnoldi step in the outer solve
    for (int k = 0; k < nrhs; ++k) {
      auto t0 = std::chrono::steady_clock::now();
      c.coarse_iters = 0;
      c.cycles = 0;
      launch_pack_fermion<double, double>((const cd64*)b + k * nn, c.perm0.as<int>(), V, 1, b64, c.stream);
      launch_pack_fermion<double, double>((const cd64*)x + k * nn, c.perm0.as<int>(), V, 1, x64, c.stream);
      int its = 0;
      if (c.p.even_odd) {
        // Schur complement on the odd sites: bhat = b_o - H_oe A_ee^{-1} b_e,
        // FGMRES on Dhat over the odd sites only (compact vectors, half the
        // outer vector traffic; the operator and the preconditioner scatter to
        // and gather from full-length fields), tolerance scaled so that the
        // residual is measured against |b|, then x_e = A_ee^{-1} (b_e - H_eo x_o)
        c.eo_prepare();
        const unsigned char* par = (const unsigned char*)c.par0.p;
        const long Vh = c.eo_half, nh = 12 * Vh;
        const int* odd = c.eo_odd.as<int>();
        const int* pos = c.eo_pos.as<int>();
        cd64* bh = c.buf<cd64>("eo_bhat", nn);
        cd64* t = c.buf<cd64>("eo_s", nn);
        cd64* fi = c.buf<cd64>("eo_fin", nn);
        cd64* fo = c.buf<cd64>("eo_fout", nn);
        cd64* bc = c.buf<cd64>("eo_bc", nh);
        cd64* xc = c.buf<cd64>("eo_xc", nh);
        launch_eo_local<double>(b64, nullptr, t, c.clovinv64.as<double>(), par, 0, 0, V, c.stream);
        c.apply_op<double>(0, t, r64, 1, nullptr, 0x1fe);
        launch_eo_local<double>(b64, r64, bh, nullptr, par, 1, 4, V, c.stream);
        launch_eo_gather<double>(bh, bc, odd, V, Vh, c.stream);
        launch_eo_gather<double>(x64, xc, odd, V, Vh, c.stream);
        std::function<void(const cd64*, cd64*, const int*)> Ah = [&c](const cd64* i, cd64* o, const int* rn) {
          c.schur64c(i, o, rn);
        };
        std::function<void(const cd64*, cd64*, const int*)> Mh = [&c, &M, fi, fo, odd, pos, par, V, Vh](
                                                                      const cd64* i, cd64* o, const int* rn) {
          launch_eo_scatter<double>(i, fi, pos, par, V, Vh, c.stream);
          M(fi, fo, rn);
          launch_eo_gather<double>(fo, o, odd, V, Vh, c.stream);
        };
        const double bn = std::sqrt(c.norm2_host<double>(b64, nn)), bhn = std::sqrt(c.norm2_host<double>(bc, nh));
        const double tol = bhn > 0 ? c.p.outer_tol * bn / bhn : c.p.outer_tol;
        GmresState& G = c.gmres_state("outer_eo", c.p.outer_restart, nh, 0, true);
        its = c.gmres<double>(G, Ah, &Mh, bc, xc, false, c.p.outer_restart, c.p.outer_maxit, tol, 0, false, nullptr,
                              1, sr);
        launch_eo_scatter<double>(xc, x64, pos, par, V, Vh, c.stream);
        c.apply_op<double>(0, x64, t, 1, nullptr, 0x1fe);
        launch_eo_local<double>(b64, t, x64, c.clovinv64.as<double>(), par, 0, 3, V, c.stream);
      } else {
        GmresState& G = c.gmres_state("outer", c.p.outer_restart, nn, 0, true);
        its = c.gmres<double>(G, A, &M, b64, x64, false, c.p.outer_restart, c.p.outer_maxit, c.p.outer_tol, 0,
                              false, nullptr, 1, sr);
      }
      // true residual in FP64
      c.apply_op<double>(0, x64, r64, 1, nullptr);
      launch_sub<double>(r64, b64, r64, nn, nullptr, c.stream);
      double rr = c.norm2_host<double>(r64, nn);
      double bb = c.norm2_host<double>(b64, nn);
      launch_unpack_fermion<double, double>(x64, c.perm0.as<int>(), V, 1, (cd64*)x + k * nn, c.stream);
      c.sync();
      double rel = true_rel_res(rr, bb);
      double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      c.timers[5] = dt;
      bool conv = rel <= c.p.outer_tol;
      if (!(rel == rel)) status = WCMG_ERR_NAN;
      else if (!conv && status == WCMG_OK) status = WCMG_ERR_NOCONV;
      if (info) {
        info[k].outer_iters = its;
        info[k].converged = conv ? 1 : 0;
        info[k].true_rel_res = rel;
        info[k].t_solve_s = dt;
        info[k].coarse_iters = c.coarse_iters;
        info[k].cycles = c.cycles;
      }
    }
  });
  if (rc != WCMG_OK) return rc;
  if (status != WCMG_OK) ctx->err = status == WCMG_ERR_NAN ? "NaN in residual" : "solver did not converge";
  return status;
}

int wcmg_solve_batched(wcmg_ctx* ctx, const void* b, void* x, int nrhs, int flags, wcmg_solve_info* info) {
  int status = WCMG_OK;
  int rc = guarded(ctx, [&](Context& c) {
    require(c.gauge_set, WCMG_ERR_STATE, "gauge field not set");
    require(c.nlev == 1 || c.setup_done, WCMG_ERR_STATE, "run wcmg_setup first");
    require(b && x && nrhs >= 1, WCMG_ERR_ARG, "bad fields");
    require((flags & ~15) == 0 && ((flags >> 1) & 3) != 3, WCMG_ERR_ARG, "bad flags");
    const bool graph = flags & WCMG_BATCH_GRAPH;
    require(!graph || c.p.cycle_prec == WCMG_F32, WCMG_ERR_ARG, "graph capture needs an FP32 cycle");
    const long V = c.geo[0].V, nn = c.n(0);
    c.coarse_kernel = (flags >> 1) & 3;
    c.dslash_per_rhs = flags & WCMG_BATCH_DSLASH_PER_RHS;
    c.use_graph = graph;
    struct Reset {
      Context& c;
      ~Reset() {
        c.coarse_kernel = 0;
        c.dslash_per_rhs = false;
        c.use_graph = false;
        c.drop_graph();
      }
    } reset{c};
    for (int k0 = 0; k0 < nrhs; k0 += 16) {
      const int B = std::min(16, nrhs - k0);
      auto t0 = std::chrono::steady_clock::now();
      c.coarse_iters = 0;
      c.cycles = 0;
      cd64* b64 = c.buf<cd64>("bsolve_b", B * nn);
      cd64* x64 = c.buf<cd64>("bsolve_x", B * nn);
      cd64* r64 = c.buf<cd64>("bsolve_r", B * nn);
      cd64* nrm = c.buf<cd64>("bsolve_n", 2L * B);
      launch_pack_fermion<double, double>((const cd64*)b + k0 * nn, c.perm0.as<int>(), V, B, b64, c.stream);
      launch_pack_fermion<double, double>((const cd64*)x + k0 * nn, c.perm0.as<int>(), V, B, x64, c.stream);
      int its[16] = {0};
      c.solve_batched(b64, x64, B, its);
      // true residuals in FP64
      c.apply_opB<double>(0, x64, r64, B, nullptr, 0);
      launch_belem<cd64, cd64>(r64, nn, b64, nn, r64, nn, nullptr, 0, nn, B, 2, nullptr, 0, c.stream);
      launch_bdot<double>(r64, 0, nn, 1, r64, nn, nn, B, c.bpart.as<cd64>(), nrm, 1, 2, 0, nullptr, 0, c.stream);
      launch_bdot<double>(b64, 0, nn, 1, b64, nn, nn, B, c.bpart.as<cd64>(), nrm + 1, 1, 2, 0, nullptr, 0, c.stream);
      cd64 hn[32];
      WCMG_HIP(hipMemcpyAsync(hn, nrm, 2 * B * sizeof(cd64), hipMemcpyDeviceToHost, c.stream));
      launch_unpack_fermion<double, double>(x64, c.perm0.as<int>(), V, B, (cd64*)x + k0 * nn, c.stream);
      c.sync();
      const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      c.timers[5] = dt;
      for (int r = 0; r < B; ++r) {
        const double rr = hn[2 * r].re, bb = hn[2 * r + 1].re;
        const double rel = true_rel_res(rr, bb);
        const bool conv = rel <= c.p.outer_tol;
        if (!(rel == rel)) status = WCMG_ERR_NAN;
        else if (!conv && status == WCMG_OK) status = WCMG_ERR_NOCONV;
        if (info) {
          wcmg_solve_info& I = info[k0 + r];
          I.outer_iters = its[r];
          I.converged = conv ? 1 : 0;
          I.true_rel_res = rel;
          I.t_solve_s = dt;
          I.coarse_iters = c.coarse_iters;
          I.cycles = c.cycles;
        }
      }
    }
  });
  if (rc != WCMG_OK) return rc;
  if (status != WCMG_OK) ctx->err = status == WCMG_ERR_NAN ? "NaN in residual" : "solver did not converge";
  return status;
}

int wcmg_solve_ragged(wcmg_ctx* const* ctxs, int nprob, const void* const* b, void* const* x, const int* nrhs,
                      wcmg_solve_info* info) {
  if (!ctxs || nprob < 1 || !ctxs[0] || !ctxs[0]->c) return WCMG_ERR_ARG;
  int status = WCMG_OK;
  int rc = guarded(ctxs[0], [&](Context& c0) {
    require(nprob <= kRaggedMax, WCMG_ERR_ARG, "ragged solve: 1..8 problems");
    require(b && x && nrhs, WCMG_ERR_ARG, "ragged solve: null argument");
    std::vector<Context*> cs(nprob);
    for (int k = 0; k < nprob; ++k) {
      require(ctxs[k] && ctxs[k]->c, WCMG_ERR_ARG, "ragged solve: null context");
      Context& c = *ctxs[k]->c;
      cs[k] = &c;
      require(b[k] && x[k] && nrhs[k] >= 1 && nrhs[k] <= 16, WCMG_ERR_ARG,
              "ragged solve: every problem needs fields and 1..16 right-hand sides");
      require(c.gauge_set && c.setup_done, WCMG_ERR_STATE, "ragged solve: run wcmg_setup on every context first");
      require(c.nlev == 2 && c.p.cycle_prec == WCMG_F32, WCMG_ERR_ARG,
              "ragged solve: two-level hierarchies with an FP32 cycle");
      require(c.p.even_odd == 0, WCMG_ERR_ARG, "ragged solve: no even-odd outer solve");
      const int prec = c.store_prec_for(1, true);
      require(mfma_supported_nb(c.cop[0]->nb), WCMG_ERR_ARG, "ragged solve: Nb in {8,16,24,32,40}");
      require(c.cop[0]->nb == c0.cop[0]->nb && prec == c0.store_prec_for(1, true), WCMG_ERR_ARG,
              "ragged solve: every problem needs the same Nb and coarse storage precision");
      require(c.p.outer_restart == c0.p.outer_restart && c.p.coarse_restart == c0.p.coarse_restart, WCMG_ERR_ARG,
              "ragged solve: every problem needs the same outer and coarse restart lengths");
      require(c.stream == c0.stream, WCMG_ERR_ARG, "ragged solve: every context must use the same stream");
      for (int j = 0; j < k; ++j) require(cs[j] != &c, WCMG_ERR_ARG, "ragged solve: a context appears twice");
    }
    auto t0 = std::chrono::steady_clock::now();
    std::vector<const cd64*> b64(nprob);
    std::vector<cd64*> x64(nprob);
    std::vector<int> Bs(nprob);
    for (int k = 0; k < nprob; ++k) {
      Context& c = *cs[k];
      const long V = c.geo[0].V, nn = c.n(0);
      Bs[k] = nrhs[k];
      cd64* bb = c.buf<cd64>("rsolve_b", Bs[k] * nn);
      x64[k] = c.buf<cd64>("rsolve_x", Bs[k] * nn);
      launch_pack_fermion<double, double>((const cd64*)b[k], c.perm0.as<int>(), V, Bs[k], bb, c.stream);
      launch_pack_fermion<double, double>((const cd64*)x[k], c.perm0.as<int>(), V, Bs[k], x64[k], c.stream);
      b64[k] = bb;
    }
    std::vector<std::vector<int>> its(nprob);
    for (int k = 0; k < nprob; ++k) its[k].assign(Bs[k], 0);
    int64_t launches = 0;
    solve_ragged(cs, b64, x64, Bs, its, &launches);
    // true residuals in FP64, per problem
    std::vector<std::vector<cd64>> hn(nprob);
    for (int k = 0; k < nprob; ++k) {
      Context& c = *cs[k];
      const long V = c.geo[0].V, nn = c.n(0);
      const int B = Bs[k];
      cd64* r64 = c.buf<cd64>("rsolve_r", B * nn);
      cd64* nrm = c.buf<cd64>("rsolve_n", 2L * B);
      c.apply_opB<double>(0, x64[k], r64, B, nullptr, 0);
      launch_belem<cd64, cd64>(r64, nn, b64[k], nn, r64, nn, nullptr, 0, nn, B, 2, nullptr, 0, c.stream);
      launch_bdot<double>(r64, 0, nn, 1, r64, nn, nn, B, c.bpart.as<cd64>(), nrm, 1, 2, 0, nullptr, 0, c.stream);
      launch_bdot<double>(b64[k], 0, nn, 1, b64[k], nn, nn, B, c.bpart.as<cd64>(), nrm + 1, 1, 2, 0, nullptr, 0,
                          c.stream);
      hn[k].resize(2 * B);
      WCMG_HIP(hipMemcpyAsync(hn[k].data(), nrm, 2 * B * sizeof(cd64), hipMemcpyDeviceToHost, c.stream));
      launch_unpack_fermion<double, double>(x64[k], c.perm0.as<int>(), V, B, (cd64*)x[k], c.stream);
    }
    c0.sync();
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int slot = 0;
    for (int k = 0; k < nprob; ++k) {
      Context& c = *cs[k];
      c.timers[5] = dt;
      for (int r = 0; r < Bs[k]; ++r, ++slot) {
        const double rr = hn[k][2 * r].re, bb = hn[k][2 * r + 1].re;
        const double rel = true_rel_res(rr, bb);
        const bool conv = rel <= c.p.outer_tol;
        if (!(rel == rel)) status = WCMG_ERR_NAN;
        else if (!conv && status == WCMG_OK) status = WCMG_ERR_NOCONV;
        if (info) {
          wcmg_solve_info& I = info[slot];
          I.outer_iters = its[k][r];
          I.converged = conv ? 1 : 0;
          I.true_rel_res = rel;
          I.t_solve_s = dt;
          I.coarse_iters = c.coarse_iters;
          I.cycles = launches;  // shared coarse-operator launches of the whole ragged solve
        }
      }
    }
  });
  if (rc != WCMG_OK) return rc;
  if (status != WCMG_OK) ctxs[0]->err = status == WCMG_ERR_NAN ? "NaN in residual" : "solver did not converge";
  return status;
}

}  // extern "C"

struct wcmg_nn {
  std::unique_ptr<Net> n;
};

namespace {
template <typename F>
int nn_guarded(wcmg_nn* h, F&& f) {
  if (!h || !h->n) return WCMG_ERR_ARG;
  try {
    f(*h->n);
    h->n->err.clear();
    return WCMG_OK;
  } catch (const Error& e) {
    h->n->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    h->n->err = e.what();
    return WCMG_ERR_HIP;
  }
}
}  // namespace

extern "C" {

int wcmg_nn_create(int n_vec, int channels, int act_prec, uint64_t seed, void* stream, wcmg_nn** out) {
  if (!out) return WCMG_ERR_ARG;
  *out = nullptr;
  try {
    require(act_prec == WCMG_BF16 || act_prec == WCMG_F32, WCMG_ERR_ARG, "network activations: WCMG_BF16 or WCMG_F32");
    auto h = new wcmg_nn();
    h->n.reset(new Net(n_vec, channels, act_prec == WCMG_BF16 ? 16 : 32, seed, (hipStream_t)stream));
    *out = h;
    return WCMG_OK;
  } catch (const Error& e) {
    g_create_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    return WCMG_ERR_HIP;
  }
}

int wcmg_nn_destroy(wcmg_nn* nn) {
  if (!nn) return WCMG_ERR_ARG;
  if (nn->n) (void)hipStreamSynchronize(nn->n->stream);
  delete nn;
  return WCMG_OK;
}

const char* wcmg_nn_last_error(const wcmg_nn* nn) {
  if (!nn || !nn->n) return g_create_error.c_str();
  return nn->n->err.c_str();
}

int wcmg_nn_num_weights(const wcmg_nn* nn, int64_t* n_floats) {
  if (!nn || !nn->n || !n_floats) return WCMG_ERR_ARG;
  *n_floats = nn->n->n_floats();
  return WCMG_OK;
}

int wcmg_nn_get_weights(wcmg_nn* nn, float* host, int64_t n) {
  return nn_guarded(nn, [&](Net& N) {
    require(host && n == N.n_floats(), WCMG_ERR_ARG, "weight buffer size differs from wcmg_nn_num_weights");
    N.get_weights(host);
  });
}

int wcmg_nn_set_weights(wcmg_nn* nn, const float* host, int64_t n) {
  return nn_guarded(nn, [&](Net& N) {
    require(host && n == N.n_floats(), WCMG_ERR_ARG, "weight buffer size differs from wcmg_nn_num_weights");
    N.set_weights(host);
  });
}

int wcmg_nn_forward(wcmg_nn* nn, wcmg_ctx* ctx, void* out_dev) {
  if (!ctx || !ctx->c) return WCMG_ERR_ARG;
  return nn_guarded(nn, [&](Net& N) {
    Context& c = *ctx->c;
    require(out_dev != nullptr, WCMG_ERR_ARG, "null output");
    N.forward(c);
    const long n = (long)N.nv * c.n(0);
    cd64* y = c.buf<cd64>("nn_out64", n);
    launch_nn_to64(N.act[3].as<cf32>(), y, n, c.stream);
    launch_unpack_fermion<double, double>(y, c.perm0.as<int>(), c.geo[0].V, N.nv, (cd64*)out_dev, c.stream);
    c.sync();
  });
}

int wcmg_nn_loss_grad(wcmg_nn* nn, wcmg_ctx* ctx, double* loss, float* grad_host, int64_t n) {
  if (!ctx || !ctx->c) return WCMG_ERR_ARG;
  return nn_guarded(nn, [&](Net& N) {
    require(loss != nullptr, WCMG_ERR_ARG, "null loss");
    require(!grad_host || n == N.n_floats(), WCMG_ERR_ARG, "gradient buffer size differs from wcmg_nn_num_weights");
    *loss = N.loss_grad(*ctx->c);
    if (grad_host) N.get_grads(grad_host);
  });
}

int wcmg_nn_train_step(wcmg_nn* nn, wcmg_ctx* ctx, float lr, double* loss) {
  if (!ctx || !ctx->c) return WCMG_ERR_ARG;
  return nn_guarded(nn, [&](Net& N) {
    require(lr > 0.f, WCMG_ERR_ARG, "learning rate must be positive");
    const double l = N.loss_grad(*ctx->c);
    require(l == l, WCMG_ERR_NAN, "network loss is NaN");
    N.adam(lr, ctx->c->stream);
    ctx->c->sync();
    if (loss) *loss = l;
  });
}

int wcmg_setup_learned(wcmg_ctx* ctx, wcmg_nn* nn, double threshold, int relax_sweeps, int* fell_back,
                       double* quality) {
  if (!nn || !nn->n) return WCMG_ERR_ARG;
  return guarded(ctx, [&](Context& c) {
    require(relax_sweeps >= 0, WCMG_ERR_ARG, "negative relaxation sweep count");
    int fb = 0;
    double q = 0.0;
    c.setup_learned(*nn->n, threshold, relax_sweeps, &fb, &q);
    if (fell_back) *fell_back = fb;
    if (quality) *quality = q;
  });
}

int wcmg_tune_enable(wcmg_ctx* ctx, int enable) {
  return guarded(ctx, [&](Context& c) { c.tuner.enabled = enable != 0; });
}

int wcmg_tune_table(wcmg_ctx* ctx, char* buf, int len, int* needed) {
  return guarded(ctx, [&](Context& c) {
    const std::string j = c.tuner.to_json();
    if (needed) *needed = (int)j.size() + 1;
    require(buf != nullptr && len >= (int)j.size() + 1, WCMG_ERR_ARG, "tuning table does not fit the buffer");
    std::memcpy(buf, j.c_str(), j.size() + 1);
  });
}

int wcmg_tune_load(wcmg_ctx* ctx, const char* json) {
  return guarded(ctx, [&](Context& c) {
    require(json != nullptr, WCMG_ERR_ARG, "null tuning table");
    c.tuner.from_json(json);
  });
}

int wcmg_timers(wcmg_ctx* ctx, double* out_host, int n) {
  return guarded(ctx, [&](Context& c) {
    require(out_host != nullptr && n >= 0, WCMG_ERR_ARG, "bad output");
    for (int i = 0; i < n && i < 8; ++i)
      out_host[i] = i == 6 ? (double)c.cgp_fallbacks : i == 7 ? (c.use_links2() ? 2.0 : 3.0) : c.timers[i];
  });
}

int wcmg_profile_enable(wcmg_ctx* ctx, const char* family, int enable) {
  return guarded(ctx, [&](Context& c) {
    require(family != nullptr, WCMG_ERR_ARG, "null family");
    c.prof.enable(family, enable != 0);
  });
}

int wcmg_profile_stats(wcmg_ctx* ctx, const char* family, int64_t* launches, double* total_ms) {
  return guarded(ctx, [&](Context& c) {
    require(family && launches && total_ms, WCMG_ERR_ARG, "null argument");
    c.prof.stats(family, launches, total_ms);
  });
}

}  // extern "C"

// ---------------------------------------------------------------- standalone coarse operator
namespace {
// Scratch of wcmg_coarse_apply_noalloc: the five-point scatter buffer in a
// file-scope device array, one copy per GPU, held until the process ends.  In
// host code `scratch` is only a stand-in for the symbol; its device address
// comes from hipGetSymbolAddress, looked up once per device.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device ordinal -> address of that device's `scratch`

void* scratch_address() {
  int dev = 0;
  WCMG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  WCMG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  require(ptr != nullptr, WCMG_ERR_HIP, "no device address for the no-allocation scratch");
  g_scratch_ptr[dev] = ptr;
  return ptr;
}
}  // namespace

struct wcmg_coarse {
  CoarseOp op;
  Tuner tuner;  // matrix-core tile choices of this operator
  int store = WCMG_F32;
  int kernel = 0;
  hipStream_t stream = nullptr;
  std::string err;
};

template <typename F>
static int guarded_c(wcmg_coarse* h, F&& f) {
  if (!h) return WCMG_ERR_ARG;
  try {
    f(*h);
    h->err.clear();
    return WCMG_OK;
  } catch (const Error& e) {
    h->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    h->err = e.what();
    return WCMG_ERR_HIP;
  }
}

extern "C" {

int wcmg_coarse_create(const int32_t dims[4], int nb, int store_prec, void* stream, wcmg_coarse** out) {
  if (!dims || !out) return WCMG_ERR_ARG;
  *out = nullptr;
  for (int m = 0; m < 4; ++m)
    if (dims[m] < 2) return WCMG_ERR_DIMS;
  if (nb < 2 || nb % 2 || (store_prec == WCMG_BF16 && nb % 4)) return WCMG_ERR_ARG;
  if (store_prec < 0 || store_prec > 2) return WCMG_ERR_ARG;
  wcmg_coarse* h = new wcmg_coarse();
  try {
    int L[4] = {dims[0], dims[1], dims[2], dims[3]};
    h->op.init_geometry(L, nb, (hipStream_t)stream);
    h->op.tuner = &h->tuner;
    h->store = store_prec;
    h->stream = (hipStream_t)stream;
  } catch (const Error& e) {
    delete h;
    return e.code;
  }
  *out = h;
  return WCMG_OK;
}

int wcmg_coarse_destroy(wcmg_coarse* op) {
  if (!op) return WCMG_ERR_ARG;
  (void)hipStreamSynchronize(op->stream);
  delete op;
  return WCMG_OK;
}

int wcmg_coarse_set(wcmg_coarse* h, const void* blocks, int src_prec) {
  return guarded_c(h, [&](wcmg_coarse& o) {
    require(blocks && (src_prec == WCMG_F64 || src_prec == WCMG_F32), WCMG_ERR_ARG, "bad blocks");
    const long n = o.op.V * 9L * o.op.nb * o.op.nb;
    o.op.M64.alloc(n * sizeof(cd64));
    if (src_prec == WCMG_F64)
      WCMG_HIP(hipMemcpyAsync(o.op.M64.p, blocks, n * sizeof(cd64), hipMemcpyDeviceToDevice, o.stream));
    else
      launch_c64_to_c128((const cf32*)blocks, o.op.M64.as<cd64>(), n, o.stream);
    o.op.invalidate();
    o.op.five = o.kernel == 3;
    o.op.refresh(o.store, o.stream);
    if (o.store != WCMG_F64 && mfma_supported_nb(o.op.nb) && o.kernel != 3) o.op.refresh_mfma(o.store, o.stream);
    WCMG_HIP(hipStreamSynchronize(o.stream));
    // the canonical master is only needed to build the device layout
    o.op.M64.release();
    o.op.M64.alloc(16);
  });
}

int wcmg_coarse_apply(wcmg_coarse* h, const void* in, void* out, int nrhs) {
  return guarded_c(h, [&](wcmg_coarse& o) {
    require(in && out && nrhs >= 1, WCMG_ERR_ARG, "bad fields");
    o.op.apply_batch(o.store, in, out, nrhs, o.kernel, nullptr, 0, o.stream);
  });
}

int wcmg_coarse_apply_noalloc(wcmg_coarse* h, const void* in, void* out, int nrhs) {
  return guarded_c(h, [&](wcmg_coarse& o) {
    require(in && out && nrhs >= 1, WCMG_ERR_ARG, "bad fields");
    o.op.apply_batch_scratch(o.store, in, out, nrhs, o.kernel, scratch_address(), kNoAllocScratchBytes, o.stream);
  });
}

int wcmg_coarse_set_tile(wcmg_coarse* h, int tile) {
  return guarded_c(h, [&](wcmg_coarse& o) {
    require(tile == -1 || tile == 0 || tile == 4 || tile == 8 || tile == 16 || tile == 5 || tile == 9, WCMG_ERR_ARG,
            "tile must be -1 (tuned), 0, 4, 5, 8, 9 or 16");
    require(tile <= 0 || o.op.L[0] % (tile & ~1) == 0, WCMG_ERR_ARG, "the tile must divide the lattice's x extent");
    o.op.mfma_tile = tile;
  });
}

int wcmg_coarse_tune_table(wcmg_coarse* h, char* buf, int len, int* needed) {
  return guarded_c(h, [&](wcmg_coarse& o) {
    const std::string j = o.tuner.to_json();
    if (needed) *needed = (int)j.size() + 1;
    require(buf && len >= (int)j.size() + 1, WCMG_ERR_ARG, "tuning table does not fit the buffer");
    std::memcpy(buf, j.c_str(), j.size() + 1);
  });
}

int wcmg_coarse_set_kernel(wcmg_coarse* h, int kernel) {
  return guarded_c(h, [&](wcmg_coarse& o) {
    require(kernel >= 0 && kernel <= 3, WCMG_ERR_ARG,
            "kernel must be 0 (auto), 1 (vector), 2 (matrix cores) or 3 (five-point vector)");
    require(kernel != 2 || (o.store != WCMG_F64 && mfma_supported_nb(o.op.nb)), WCMG_ERR_ARG,
            "matrix-core kernel needs FP32/BF16 storage and Nb in {8,16,24,32,40}");
    require(kernel != 3 || five_point_supported(o.op.nb), WCMG_ERR_ARG,
            "five-point kernel needs Nb in {8,12,16,24,32}");
    require((kernel == 3) == (o.kernel == 3) || !o.op.built(o.store), WCMG_ERR_STATE,
            "switch to or from the five-point kernel before wcmg_coarse_set");
    o.kernel = kernel;
  });
}

}  // extern "C"

static RaggedTable ragged_table(wcmg_coarse* const* ops, int nprob, const void* const* in, void* const* out,
                                const int* nrhs) {
  require(ops && in && out && nrhs && nprob >= 1 && nprob <= kRaggedMax, WCMG_ERR_ARG,
          "ragged batch: 1..8 operators with fields");
  RaggedTable t{};
  t.n = nprob;
  t.nb = ops[0]->op.nb;
  for (int p = 0; p < nprob; ++p) {
    wcmg_coarse& o = *ops[p];
    require(o.op.nb == t.nb && o.store == ops[0]->store, WCMG_ERR_ARG,
            "ragged batch: operators must share Nb and storage precision");
    require(in[p] && out[p], WCMG_ERR_ARG, "ragged batch: null field");
    require(o.op.mfma_fresh[o.store], WCMG_ERR_STATE, "ragged batch: operator blocks not set");
    t.p[p] = RaggedProblem{o.op.mfma[o.store].p, (const cf32*)in[p], (cf32*)out[p], o.op.nbr.as<int>(), o.op.V,
                           nrhs[p], nullptr, 0};
  }
  return t;
}

extern "C" {

int wcmg_coarse_apply_ragged(wcmg_coarse* const* ops, int nprob, const void* const* in, void* const* out,
                             const int* nrhs) {
  if (!ops || nprob < 1) return WCMG_ERR_ARG;
  return guarded_c(ops[0], [&](wcmg_coarse& o) {
    launch_coarse_apply_mfma_ragged(o.store, ragged_table(ops, nprob, in, out, nrhs), o.stream);
  });
}

int wcmg_coarse_time_ragged(wcmg_coarse* const* ops, int nprob, const void* const* in, void* const* out,
                            const int* nrhs, int reps, double* avg_ms) {
  if (!ops || nprob < 1) return WCMG_ERR_ARG;
  return guarded_c(ops[0], [&](wcmg_coarse& o) {
    require(reps >= 1 && avg_ms, WCMG_ERR_ARG, "bad arguments");
    const RaggedTable t = ragged_table(ops, nprob, in, out, nrhs);
    hipEvent_t a, b;
    WCMG_HIP(hipEventCreate(&a));
    WCMG_HIP(hipEventCreate(&b));
    WCMG_HIP(hipEventRecord(a, o.stream));
    for (int i = 0; i < reps; ++i) launch_coarse_apply_mfma_ragged(o.store, t, o.stream);
    WCMG_HIP(hipEventRecord(b, o.stream));
    WCMG_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    WCMG_HIP(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *avg_ms = ms / reps;
  });
}

int wcmg_coarse_time(wcmg_coarse* h, const void* in, void* out, int nrhs, int reps, double* avg_ms) {
  return guarded_c(h, [&](wcmg_coarse& o) {
    require(in && out && nrhs >= 1 && reps >= 1 && avg_ms, WCMG_ERR_ARG, "bad arguments");
    hipEvent_t a, b;
    WCMG_HIP(hipEventCreate(&a));
    WCMG_HIP(hipEventCreate(&b));
    WCMG_HIP(hipEventRecord(a, o.stream));
    for (int i = 0; i < reps; ++i) o.op.apply_batch(o.store, in, out, nrhs, o.kernel, nullptr, 0, o.stream);
    WCMG_HIP(hipEventRecord(b, o.stream));
    WCMG_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    WCMG_HIP(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *avg_ms = ms / reps;
  });
}

const char* wcmg_coarse_last_error(const wcmg_coarse* op) { return op ? op->err.c_str() : "null operator"; }

}  // extern "C"
