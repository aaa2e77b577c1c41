// Batched multigrid solve: B right-hand sides, each with its own FP64 FGMRES
// (Sec. 2.1 FGMRES preconditioned by the cycle), advancing together.  Every
// field is right-hand-side major (field r at base + r * n), so one launch of
// the Dslash, restrict, prolong or coarse apply covers the whole batch; on the
// coarse levels the batch turns the block stencil into a complex GEMM per site
// and direction that runs on the matrix cores.  A right-hand side whose solve
// has converged (or whose coarse solve has) is masked by its run flag and
// drops out of every launch.
//
// The preconditioner application can be captured once in a HIP graph and
// replayed; the captured cycle then runs without host checks (inner solves run
// their full iteration limits, predicated off once converged).
#include <chrono>
#include <map>
#include <mutex>
#include <cmath>

#include "engine.h"

namespace wcmg {

namespace {
long scalars_per_rhs(int m) { return (long)(m + 1) * m + 2 * m + (m + 1) + m + 8 + 2 * (m + 1); }
constexpr int kMaxBatch = 16;
}  // namespace

Tuner::~Tuner() {
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
}

const std::string& device_arch() {
  static std::mutex mu;
  static std::map<int, std::string> names;
  int dev = 0;
  WCMG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  auto it = names.find(dev);
  if (it == names.end()) {
    hipDeviceProp_t prop;
    WCMG_HIP(hipGetDeviceProperties(&prop, dev));
    std::string a = prop.gcnArchName;
    a = a.substr(0, a.find(':'));  // drop feature suffixes (":sramecc+:xnack-")
    it = names.emplace(dev, a).first;
  }
  return it->second;
}

int Tuner::pick(const std::string& key, int nvar, const std::function<void(int)>& run, hipStream_t st,
                int fallback, const std::function<bool(int)>& ok) {
  auto it = choice.find(key);
  if (it != choice.end()) return it->second;
  if (!enabled || nvar <= 1) return fallback;
  // the candidates' launches must not take a profiled launch's event pair
  const KernelTiming armed = kernel_timing();
  kernel_timing() = KernelTiming();
  if (!ev[0]) {
    WCMG_HIP(hipEventCreate(&ev[0]));
    WCMG_HIP(hipEventCreate(&ev[1]));
  }
  constexpr int reps = 3;
  std::vector<double> t(nvar, -1.0);
  for (int v = 0; v < nvar; ++v) {
    if (ok && !ok(v)) continue;
    run(v);  // warm: first-touch, caches, code load
    WCMG_HIP(hipEventRecord(ev[0], st));
    for (int q = 0; q < reps; ++q) run(v);
    WCMG_HIP(hipEventRecord(ev[1], st));
    WCMG_HIP(hipEventSynchronize(ev[1]));
    float e = 0.f;
    WCMG_HIP(hipEventElapsedTime(&e, ev[0], ev[1]));
    t[v] = e / reps;
  }
  int best = -1;
  for (int v = 0; v < nvar; ++v)
    if (t[v] >= 0.0 && (best < 0 || t[v] < t[best])) best = v;
  if (best < 0) best = fallback;
  choice[key] = best;
  ms[key] = t;
  kernel_timing() = armed;
  return best;
}

std::string Tuner::to_json() const {
  std::string o = "{";
  bool first = true;
  for (auto& kv : choice) {
    o += first ? "\"" : ", \"";
    first = false;
    o += kv.first + "\": {\"choice\": " + std::to_string(kv.second) + ", \"ms\": [";
    auto m = ms.find(kv.first);
    if (m != ms.end())
      for (size_t i = 0; i < m->second.size(); ++i) {
        char b[32];
        snprintf(b, sizeof b, "%s%.5f", i ? ", " : "", m->second[i]);
        o += b;
      }
    o += "]}";
  }
  return o + "}";
}

// Reads back what to_json wrote: "key": {"choice": n, ...} entries.
void Tuner::from_json(const std::string& text) {
  size_t pos = 0;
  while (true) {
    const size_t k0 = text.find('"', pos);
    if (k0 == std::string::npos) break;
    const size_t k1 = text.find('"', k0 + 1);
    require(k1 != std::string::npos, WCMG_ERR_ARG, "tuning table: unterminated key");
    const std::string key = text.substr(k0 + 1, k1 - k0 - 1);
    const size_t c = text.find("\"choice\":", k1);
    require(c != std::string::npos, WCMG_ERR_ARG, "tuning table: entry without a choice");
    choice[key] = std::atoi(text.c_str() + c + 9);
    pos = text.find('}', c);
    if (pos == std::string::npos) break;
  }
}

BatchGmres& Context::bgmres_state(const std::string& tag, int m, long n_, int B, int prec, bool flex) {
  auto& g = bgm[tag];
  if (!g) g.reset(new BatchGmres());
  BatchGmres& G = *g;
  if (G.m != m || G.n != n_ || G.B != B || G.prec != prec || G.flex != flex) {
    const size_t cb = prec == 0 ? sizeof(cd64) : sizeof(cf32);
    G.m = m;
    G.n = n_;
    G.B = B;
    G.prec = prec;
    G.flex = flex;
    G.ss = scalars_per_rhs(m);
    G.V.alloc((size_t)(m + 1) * B * n_ * cb);
    if (flex) G.Z.alloc((size_t)m * B * n_ * cb);
    G.w.alloc((size_t)B * n_ * cb);
    G.S.alloc((size_t)B * G.ss * sizeof(cd64));
    G.st.alloc((size_t)8 * B * sizeof(int));
    drop_graph();  // captured launches may refer to the old buffers
  }
  return G;
}

void Context::drop_graph() {
  if (cgraph.exec) (void)hipGraphExecDestroy(cgraph.exec);
  cgraph = CycleGraph();
}

// FP32 Dslash on a batch: variant 0 launches the per-field kernel (fields of
// one site block grouped on one XCD), variant 1 the multi-RHS kernel that
// stages the gauge data in LDS.
void Context::dslash32_batch(const cf32* in, cf32* out, int B, const int* run, int rs, cd64* dots) {
  auto launch = [&](int v) {
    if (v == 1)
      launch_wilson_mrhs(in, out, U32.as<cf32>(), clov32.as<float>(), geo[0].nbr.as<int>(), geo[0].V, B, run, rs,
                         dots, stream);
    else
      launch_wilson<float>(in, out, U32.as<cf32>(), clov32.as<float>(), geo[0].nbr.as<int>(), geo[0].V, 0x1ff, B,
                           run, stream, dots, rs, nullptr, dslash_geo(), dslash_links2<float>());
  };
  int v = 0;
  if (dslash_per_rhs || B < 2) v = 0;
  else if (capturing) v = tuner.choice.count(dslash_key(B)) ? tuner.choice[dslash_key(B)] : 1;
  else v = tuner.pick(dslash_key(B), 2, launch, stream, 1);
  launch(v);
}

std::string Context::dslash_key(int B) const {
  return device_arch() + " dslash_f32 V=" + std::to_string(geo[0].V) + " nrhs=" + std::to_string(B);
}

template <typename R>
void Context::apply_opB(int l, const cplx<R>* in, cplx<R>* out, int B, const int* run, int rs) {
  const bool single = sizeof(R) == 4;
  if (l == 0) {
    const char* fam = single ? "dslash_f32" : "dslash_f64";
    if (!capturing) prof.begin_kernel(fam);
    if (single)
      dslash32_batch((const cf32*)in, (cf32*)out, B, run, rs, nullptr);
    else
      launch_wilson<double>((const cd64*)in, (cd64*)out, U64.as<cd64>(), clov64.as<double>(), geo[0].nbr.as<int>(),
                            geo[0].V, 0x1ff, B, run, stream, nullptr, rs, nullptr, dslash_geo(), dslash_links2<double>());
    if (!capturing) prof.end(fam, stream);
    return;
  }
  const int prec = store_prec_for(l, single);
  CoarseOp& C = *cop[l - 1];
  const bool can_mfma = prec != WCMG_F64 && mfma_supported_nb(C.nb);
  bool mfma = false;
  if (can_mfma && coarse_kernel == 2) mfma = true;
  else if (can_mfma && coarse_kernel == 0) {
    C.refresh_mfma(prec, stream);
    const std::string key = device_arch() + " coarse_apply prec=" + std::to_string(prec) +
                            " Vc=" + std::to_string(C.V) + " nb=" + std::to_string(C.nb) + " nrhs=" + std::to_string(B);
    if (capturing) mfma = tuner.choice.count(key) ? tuner.choice[key] == 1 : B >= 4;
    else
      mfma = tuner.pick(key, 2, [&](int v) { C.apply_batch(prec, in, out, B, v == 1 ? 2 : 1, run, rs, stream); },
                        stream, B >= 4 ? 1 : 0) == 1;
  }
  if (mfma) C.refresh_mfma(prec, stream);
  const char* fam = mfma ? (prec == WCMG_F32 ? "coarse_mfma_f32" : "coarse_mfma_bf16")
                         : prec == WCMG_F64 ? "coarse_apply_f64"
                         : prec == WCMG_F32 ? "coarse_apply_f32" : "coarse_apply_bf16";
  if (!capturing) prof.begin_kernel(fam);
  C.apply_batch(prec, in, out, B, mfma ? 2 : 1, run, rs, stream);
  if (!capturing) prof.end(fam, stream);
}

// MinimalResidual on each right-hand side (Sec. 2.1), as Context::mr; b ==
// nullptr means b = 0 (relaxation on D x = 0).
template <typename R>
void Context::mrB(int l, const cplx<R>* b, cplx<R>* x, int B, int steps, const int* run, int rs) {
  const long nn = n(l);
  const std::string t = std::to_string(l) + (sizeof(R) == 8 ? "d" : "f");
  cplx<R>* r = buf<cplx<R>>("bmr_r" + t, B * nn);
  cplx<R>* pp = buf<cplx<R>>("bmr_p" + t, B * nn);
  cd64* dots = buf<cd64>("bmr_dots" + t, 2L * B);
  apply_opB<R>(l, x, pp, B, run, rs);
  if (b) launch_belem<cplx<R>, cplx<R>>(r, nn, b, nn, pp, nn, nullptr, 0, nn, B, 2, run, rs, stream);
  else launch_belem<cplx<R>, cplx<R>>(r, nn, pp, nn, nullptr, 0, nullptr, 0, nn, B, 4, run, rs, stream);  // b = 0
  if (l == 0) {
    // <p, r> and <p, p> per right-hand side from the Dslash epilogue
    const int G = wilson_blocks(geo[0].V);
    cd64* part = buf<cd64>("bmr_part" + t, 2L * G * B);
    for (int k = 0; k < steps; ++k) {
      if (sizeof(R) == 4)
        dslash32_batch((const cf32*)r, (cf32*)pp, B, run, rs, part);
      else
        launch_wilson<double>((const cd64*)r, (cd64*)pp, U64.as<cd64>(), clov64.as<double>(), geo[0].nbr.as<int>(),
                              geo[0].V, 0x1ff, B, run, stream, part, rs, nullptr, dslash_geo(),
                              dslash_links2<double>());
      launch_bdot_finish(part, G, 2, 2, B, dots, 1, 2, 0, run, rs, stream);
      launch_bmr_update<R>(x, r, pp, nn, dots, nn, B, run, rs, stream);
    }
    return;
  }
  cd64* part = bpart.as<cd64>();
  for (int k = 0; k < steps; ++k) {
    apply_opB<R>(l, r, pp, B, run, rs);
    launch_bdot<R>(pp, 0, nn, 1, r, nn, nn, B, part, dots, 1, 2, 0, run, rs, stream);
    launch_bdot<R>(pp, 0, nn, 1, pp, nn, nn, B, part, dots + 1, 1, 2, 0, run, rs, stream);
    launch_bmr_update<R>(x, r, pp, nn, dots, nn, B, run, rs, stream);
  }
}

// B restarted (F)GMRES solves, CGS2 + Givens on the device, as Context::gmres.
// iters (host, B entries, may be null) receives the per-solve iteration counts
// when the host checks progress.
template <typename R>
void Context::gmresB(BatchGmres& G, const BatchOp<R>& A, const BatchOp<R>* M, const cplx<R>* b, cplx<R>* x,
                     bool x0_zero, int restart, int maxit, double tol, int fixed, bool stop_on_est,
                     const int* parent, int prs, int check_every, int* iters, bool single_reduction) {
  const long nn = G.n;
  const int m = restart, B = G.B;
  const long ss = G.ss, bn = (long)B * nn;
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
  cd64* part = bpart.as<cd64>();
  const int Gb = bred_blocks(nn);
  launch_bgmres_init(st, B, parent, prs, stream);
  if (x0_zero) launch_belem<cplx<R>, cplx<R>>(x, nn, x, nn, nullptr, 0, nullptr, 0, nn, B, 0, live, 8, stream);
  launch_bdot<R>(b, 0, nn, 1, b, nn, nn, B, part, misc + 0, 1, ss, 0, live, 8, stream);
  const int limit = fixed > 0 ? fixed : maxit;
  const int max_cycles = check_every > 0 ? limit : (limit + m - 1) / m;
  // progress checks as in Context::gmres: 8 state words per right-hand side
  StateChecks chk{*this, st, 8 * B};
  const int* last = nullptr;
  auto any = [&](const int* sv, int word) {
    for (int r = 0; r < B; ++r)
      if (sv[8 * r + word]) return true;
    return false;
  };
  for (int cyc = 0; cyc < max_cycles; ++cyc) {
    if (cyc == 0 && x0_zero) {
      launch_belem<cplx<R>, cplx<R>>(V, nn, b, nn, nullptr, 0, nullptr, 0, nn, B, 1, live, 8, stream);
    } else {
      A(x, w, live, 8);
      launch_belem<cplx<R>, cplx<R>>(V, nn, b, nn, w, nn, nullptr, 0, nn, B, 2, live, 8, stream);
    }
    launch_bdot<R>(V, 0, nn, 1, V, nn, nn, B, part, misc + 1, 1, ss, 0, live, 8, stream);
    launch_bgmres_cycle_start(st, S, ss, B, m, tol, limit, fixed, stream);
    launch_belem<cplx<R>, cplx<R>>(V, nn, V, nn, nullptr, 0, misc + 1, ss, nn, B, 3, run, 8, stream);
    for (int j = 0; j < m; ++j) {
      cplx<R>* vj = V + j * bn;
      cplx<R>* zj = M ? Z + j * bn : vj;
      if (M) (*M)(vj, zj, run, 8);
      if (single_reduction) {
        // the single-reduction step of Context::gmres, per right-hand side:
        // w' = A z_j - s v_j formed in the slot of v_{j+1}, one sweep for its
        // dots and norm, the projection repeated only where it removed more
        // than 3/4 of |w'|^2 (st[5] of that right-hand side), one sweep to
        // subtract and normalise
        cplx<R>* wj = V + (j + 1) * bn;
        A(zj, wj, run, 8);
        launch_barnoldi_dots<R>(V, bn, nn, j, nn, j > 0 ? misc + 4 : nullptr, ss, part, B, run, 8, stream);
        launch_bdot_finish(part, Gb, j + 2, j + 2, B, tmp, 1, ss, 0, run, 8, stream);
        launch_bgmres_sr(st, S, ss, B, m, j, tmp, tmp2, 0, stream);
        launch_bmulti_axpy<R>(wj, nn, V, bn, nn, j + 1, nullptr, 0, tmp, 1, ss, -1.0, nn, B, nullptr, st + 5, 8,
                              stream);
        launch_barnoldi_dots<R>(V, bn, nn, j, nn, nullptr, ss, part, B, st + 5, 8, stream);
        launch_bdot_finish(part, Gb, j + 2, j + 2, B, tmp2, 1, ss, 0, st + 5, 8, stream);
        launch_bgmres_sr(st, S, ss, B, m, j, tmp, tmp2, 1, stream);
        launch_bgmres_givens(st, S, ss, B, m, j, tol, limit, fixed, stop_on_est ? 1 : 0, stream);
        if (j + 1 < m) launch_bupdate_scale<R>(wj, nn, V, bn, nn, j + 1, tmp, ss, misc + 3, ss, nn, B, run, 8, stream);
        if (check_every > 0 && (j + 1) % check_every == 0 && j + 1 < m) {
          const int* sv = chk.ahead();
          if (sv && !any(sv, 0)) break;
        }
        continue;
      }
      A(zj, w, run, 8);
      // classical Gram-Schmidt applied twice; |w|^2 from the last update
      launch_bdot<R>(V, bn, nn, j + 1, w, nn, nn, B, part, H + j, m, ss, 0, run, 8, stream);
      if (j + 1 <= kFusedMaxM) {
        // first update and second projection in one sweep over the basis
        launch_bmulti_axpy_dot<R>(w, nn, V, bn, nn, j + 1, H + j, m, ss, nn, B, part, run, 8, stream);
        launch_bdot_finish(part, Gb, j + 1, j + 1, B, tmp, 1, ss, 0, run, 8, stream);
      } else {
        launch_bmulti_axpy<R>(w, nn, V, bn, nn, j + 1, nullptr, 0, H + j, m, ss, -1.0, nn, B, nullptr, run, 8,
                              stream);
        launch_bdot<R>(V, bn, nn, j + 1, w, nn, nn, B, part, tmp, 1, ss, 0, run, 8, stream);
      }
      launch_bdot_finish(part, Gb, j + 1, j + 1, B, H + j, m, ss, 1, run, 8, stream);
      launch_bmulti_axpy<R>(w, nn, V, bn, nn, j + 1, nullptr, 0, tmp, 1, ss, -1.0, nn, B, part, run, 8, stream);
      launch_bdot_finish(part, Gb, 1, 1, B, misc + 3, 1, ss, 0, run, 8, stream);
      launch_bgmres_givens(st, S, ss, B, m, j, tol, limit, fixed, stop_on_est ? 1 : 0, stream);
      if (j + 1 < m)
        launch_belem<cplx<R>, cplx<R>>(V + (j + 1) * bn, nn, w, nn, nullptr, 0, misc + 3, ss, nn, B, 3, run, 8,
                                       stream);
      if (check_every > 0 && (j + 1) % check_every == 0 && j + 1 < m) {
        const int* sv = chk.ahead();
        if (sv && !any(sv, 0)) break;
      }
    }
    launch_bgmres_solve_y(st, S, ss, B, m, stream);
    launch_bmulti_axpy<R>(x, nn, M ? Z : V, bn, nn, m, st + 2, 8, y, 1, ss, 1.0, nn, B, nullptr, nullptr, 0, stream);
    launch_bgmres_cycle_end(st, B, stream);
    if (check_every > 0) {
      last = chk.now();
      if (!any(last, 1)) break;
    }
  }
  if (check_every > 0) {
    if (!last) last = chk.now();
    if (iters)
      for (int r = 0; r < B; ++r) iters[r] = last[8 * r + 3];
  }
}

// One batched preconditioner application rooted at level l (as Context::cycle).
template <typename R>
void Context::cycleB(int l, const cplx<R>* r, cplx<R>* x, int B, const int* run, int rs) {
  const int lc = l + 1;
  const std::string t = std::to_string(lc) + (sizeof(R) == 8 ? "d" : "f");
  const long nc = n(lc);
  cplx<R>* rc = buf<cplx<R>>("bcyc_rc" + t, B * nc);
  cplx<R>* ec = buf<cplx<R>>("bcyc_ec" + t, B * nc);
  {
    const char* fam = sizeof(R) == 8 ? "restrict_f64" : "restrict_f32";
    if (!capturing) prof.begin_kernel(fam);
    const Transfer& T = tr[l];
    const cplx<R>* P = sizeof(R) == 8 ? (const cplx<R>*)T.P64.p : (const cplx<R>*)T.P32.p;
    launch_restrict<R>(r, rc, P, geo[l].lay, T.agg_sites.as<int>(), T.A, T.Vc, T.nb, B, run, stream, rs);
    if (!capturing) prof.end(fam, stream);
  }
  const int check = (no_checks || (p.reserved[0] & 1)) ? 0 : 4;
  const int prec = sizeof(R) == 8 ? 0 : 1;
  BatchOp<R> Ab = [this, lc, B](const cplx<R>* i, cplx<R>* o, const int* rn, int s) {
    apply_opB<R>(lc, i, o, B, rn, s);
  };
  std::vector<int> its(B, 0);
  if (lc + 1 >= nlev) {
    BatchGmres& G = bgmres_state("bcg" + t, p.coarse_restart, nc, B, prec, false);
    // without host checks every enqueued iteration costs launches even once
    // predicated off, so the graph form runs at most one restart cycle
    const int maxit = no_checks ? std::min(p.coarse_maxit, p.coarse_restart) : p.coarse_maxit;
    gmresB<R>(G, Ab, nullptr, rc, ec, true, p.coarse_restart, maxit, p.coarse_tol, p.coarse_fixed_iters, true, run, rs,
              check, check > 0 ? its.data() : nullptr);
  } else if (p.kcycle) {
    BatchOp<R> Mc = [this, lc, B](const cplx<R>* i, cplx<R>* o, const int* rn, int s) {
      cycleB<R>(lc, i, o, B, rn, s);
    };
    BatchGmres& G = bgmres_state("bkc" + t, p.kcycle_maxit, nc, B, prec, true);
    gmresB<R>(G, Ab, &Mc, rc, ec, true, p.kcycle_maxit, p.kcycle_maxit, p.kcycle_tol, 0, true, run, rs, 0, nullptr);
  } else {
    cycleB<R>(lc, rc, ec, B, run, rs);
  }
  for (int q = 0; q < B; ++q) coarse_iters += its[q];
  {
    const char* fam = sizeof(R) == 8 ? "prolong_f64" : "prolong_f32";
    if (!capturing) prof.begin_kernel(fam);
    const Transfer& T = tr[l];
    const cplx<R>* P = sizeof(R) == 8 ? (const cplx<R>*)T.P64.p : (const cplx<R>*)T.P32.p;
    launch_prolong<R>(ec, x, P, geo[l].lay, T.coarse_of.as<int>(), T.Vc, T.nb, 0, B, run, stream, rs,
                      T.agg_sites.as<int>(), T.A);
    if (!capturing) prof.end(fam, stream);
  }
  if (l == 0 && p.smoother == 1) sap<R>(r, x, p.post_smooth, B, run, rs);
  else mrB<R>(l, r, x, B, p.post_smooth, run, rs);
  cycles += B;
}

// FP64 in, FP64 out; the cycle itself in the cycle precision.  With graphs on,
// the FP32 cycle is captured on its first repeat with the same buffers and
// flags and replayed from then on.
void Context::precondition64B(int l, const cd64* r, cd64* x, int B, const int* run, int rs) {
  if (p.cycle_prec == WCMG_F64) {
    cycleB<double>(l, r, x, B, run, rs);
    return;
  }
  const long nn = n(l);
  const std::string t = std::to_string(l);
  cf32* r32 = buf<cf32>("bpc_r32" + t, B * nn);
  cf32* x32 = buf<cf32>("bpc_x32" + t, B * nn);
  launch_belem<cd64, cf32>(r32, nn, r, nn, nullptr, 0, nullptr, 0, nn, B, 1, run, rs, stream);
  const bool same = cgraph.l == l && cgraph.B == B && cgraph.rs == rs && cgraph.in == r32 && cgraph.out == x32 &&
                    cgraph.run == run;
  if (!use_graph) {
    cycleB<float>(l, r32, x32, B, run, rs);
  } else if (same && cgraph.exec) {
    WCMG_HIP(hipGraphLaunch(cgraph.exec, stream));
    graph_launches++;
  } else if (!same || !cgraph.warm) {
    // first use with these buffers: run eagerly (allocates every workspace)
    drop_graph();
    no_checks = true;  // same launch sequence as the captured one: no host checks
    cycleB<float>(l, r32, x32, B, run, rs);
    no_checks = false;
    cgraph.l = l;
    cgraph.B = B;
    cgraph.rs = rs;
    cgraph.in = r32;
    cgraph.out = x32;
    cgraph.run = run;
    cgraph.warm = true;
  } else {
    if (!cap_stream) WCMG_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
    hipStream_t saved = stream;
    stream = cap_stream;
    capturing = no_checks = true;
    hipGraph_t graph = nullptr;
    WCMG_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
    try {
      cycleB<float>(l, r32, x32, B, run, rs);
    } catch (...) {
      (void)hipStreamEndCapture(cap_stream, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      stream = saved;
      capturing = no_checks = false;
      throw;
    }
    WCMG_HIP(hipStreamEndCapture(cap_stream, &graph));
    stream = saved;
    capturing = no_checks = false;
    hipGraphExec_t exec = nullptr;
    WCMG_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    (void)hipGraphDestroy(graph);
    cgraph.exec = exec;
    WCMG_HIP(hipGraphLaunch(cgraph.exec, stream));
    graph_launches++;
  }
  launch_belem<cf32, cd64>(x, nn, x32, nn, nullptr, 0, nullptr, 0, nn, B, 1, run, rs, stream);
}

// Outer FP64 FGMRES for B right-hand sides at once (fields in device order).
void Context::solve_batched(const cd64* b, cd64* x, int B, int* iters) {
  require(B >= 1 && B <= kMaxBatch, WCMG_ERR_ARG, "batched solve takes 1..16 right-hand sides");
  const long nn = n(0);
  const int m = p.outer_restart;
  const long need = (long)kMaxBatch * kPartialSlots;
  if (bpart.bytes < (size_t)need * sizeof(cd64)) bpart.alloc((size_t)need * sizeof(cd64));
  BatchGmres& G = bgmres_state("outer", m, nn, B, 0, true);
  BatchOp<double> A = [this, B](const cd64* i, cd64* o, const int* rn, int s) { apply_opB<double>(0, i, o, B, rn, s); };
  BatchOp<double> M = [this, B, nn](const cd64* i, cd64* o, const int* rn, int s) {
    if (nlev >= 2) precondition64B(0, i, o, B, rn, s);
    else launch_belem<cd64, cd64>(o, nn, i, nn, nullptr, 0, nullptr, 0, nn, B, 1, rn, s, stream);
  };
  gmresB<double>(G, A, &M, b, x, false, m, p.outer_maxit, p.outer_tol, 0, false, nullptr, 0, 1, iters,
                 !(p.reserved[0] & 8));
}

template void Context::apply_opB<double>(int, const cd64*, cd64*, int, const int*, int);
template void Context::apply_opB<float>(int, const cf32*, cf32*, int, const int*, int);
template void Context::mrB<double>(int, const cd64*, cd64*, int, int, const int*, int);
template void Context::mrB<float>(int, const cf32*, cf32*, int, int, const int*, int);
template void Context::cycleB<double>(int, const cd64*, cd64*, int, const int*, int);
template void Context::cycleB<float>(int, const cf32*, cf32*, int, const int*, int);

}  // namespace wcmg
