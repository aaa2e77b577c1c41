// Host-side multigrid engine: levels, operators, setup, solvers.
#pragma once

#include <array>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "kernels.h"

namespace wcmg {

// HIP-event timing of kernel families on the context stream.  A family of
// one kernel launch is timed by the dispatch itself (begin_kernel arms the
// launch's event pair); a family of several launches by events recorded on
// the stream around them (begin).
struct Profiler {
  struct Family {
    bool on = false;
    bool armed = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
  };
  std::map<std::string, Family> fam;
  ~Profiler();
  void enable(const std::string& f, bool on);
  void begin(const char* f, hipStream_t st);
  void begin_kernel(const char* f);
  void end(const char* f, hipStream_t st);
  void stats(const std::string& f, int64_t* launches, double* ms);
  size_t pending_ = 0;
};

// Geometry of one level as laid out on the device.
struct LevelGeom {
  int L[4] = {0, 0, 0, 0};
  long V = 0;
  int ns = 0;
  FieldLayout lay{};
  DevBuf nbr;                  // int32 [8][V] in device site order
  std::vector<int> perm;       // device site -> lexicographic site (identity for coarse levels)
  long n() const { return V * ns; }
};

// Intergrid transfer from level l to l+1 (Sec. 2.1 Aggregation).
struct Transfer {
  int block[4] = {1, 1, 1, 1};
  int A = 1;
  long Vc = 0;
  int nv = 0;
  int nb = 0;
  DevBuf agg_sites;  // int32 [Vc][A]: device site of level l for (c, o)
  DevBuf coarse_of;  // int32 [V_l]
  std::vector<int> agg_host, off_host;  // per lexicographic site of level l
  DevBuf start64, vecs64, P64, P32;     // [nv][n_l]
  bool has_start = false, built = false;
};

// Coarse operator of one level: canonical FP64 master plus device layouts.
struct CoarseOp {
  int L[4] = {0, 0, 0, 0};
  long V = 0;
  int nb = 0;
  DevBuf nbr;   // int32 [8][V]
  DevBuf M64;   // canonical [V][9][nb][nb]
  DevBuf dev[3];
  bool fresh[3] = {false, false, false};
  DevBuf mfma[3];  // fragment-ordered blocks for the matrix-core kernel (F32, BF16)
  bool mfma_fresh[3] = {false, false, false};
  // five-point storage (Mdiag and the forward blocks): full applies read it,
  // the nine-block layout is then built only for single-term applies
  bool five = false;
  DevBuf dev5[3];
  bool fresh5[3] = {false, false, false};
  DevBuf tmp5;  // backward contributions of the owner-computes five-point apply
  void init_geometry(const int Lc[4], int nb_, hipStream_t st);
  void refresh(int prec, hipStream_t st);  // canonical -> device layout of prec
  void refresh9(int prec, hipStream_t st);
  void refresh_mfma(int prec, hipStream_t st);
  bool built(int prec) const { return fresh[prec] || fresh5[prec]; }
  bool uses_five() const { return five && five_point_supported(nb); }
  void invalidate() {
    for (int q = 0; q < 3; ++q) fresh[q] = mfma_fresh[q] = fresh5[q] = false;
  }
  // matrix-core tile: -1 tuned (or the default when no tuner is attached), 0
  // one wave per site, 4/8/16 sites per workgroup with LDS-staged neighbours
  int mfma_tile = -1;
  struct Tuner* tuner = nullptr;
  int choose_tile(int prec, const void* in, void* out, int nrhs, const int* run, int run_stride, hipStream_t st);
  // nrhs right-hand sides (RHS-major); kernel: 0 auto, 1 per-row vector kernel, 2 matrix cores
  void apply_batch(int prec, const void* in, void* out, int nrhs, int kernel, const int* run, int run_stride,
                   hipStream_t st);
  void apply(int prec, const void* in, void* out, int dmask, int accumulate, int nrhs, const int* run, hipStream_t st,
             int run_stride = 0);
  // apply_batch without any device allocation: the five-point scatter buffer is
  // the caller's `scratch` (scratch_bytes long); every layout must already be built
  void apply_batch_scratch(int prec, const void* in, void* out, int nrhs, int kernel, void* scratch,
                           size_t scratch_bytes, hipStream_t st);
};

// B independent (F)GMRES solves advancing through shared launches.  Basis
// vectors are stored [k][r][n] so that v_k of all right-hand sides is one
// RHS-major batch; scalars and state words are per right-hand side.
struct BatchGmres {
  int m = 0, B = 0, prec = 0;
  long n = 0;
  bool flex = false;
  long ss = 0;  // cd64 scalars per right-hand side
  DevBuf V, Z, w, S, st;
};

// Operator or preconditioner on a batch: (in, out, run flags, flag stride).
template <typename R>
using BatchOp = std::function<void(const cplx<R>*, cplx<R>*, const int*, int)>;

// Autotuner: for each launch configuration (operator, shape, batch size) it
// times every applicable kernel variant once on the live operands, keeps the
// fastest, and reuses that choice for the rest of the context's life.  The
// table can be saved to and loaded from a small JSON file.
// Architecture name of the current device (e.g. "gfx950"), the first part of
// every tuning key.
const std::string& device_arch();

struct Tuner {
  bool enabled = true;
  std::map<std::string, int> choice;
  std::map<std::string, std::vector<double>> ms;  // measured mean ms per variant
  hipEvent_t ev[2] = {nullptr, nullptr};
  ~Tuner();
  // variant for key: looked up, or measured with run(v) for v < nvar (each
  // candidate is launched reps + 1 times on stream st; its output is that of
  // a normal launch, so the caller's result is unaffected)
  // (variants with ok(v) false are not run; their time is recorded as -1)
  int pick(const std::string& key, int nvar, const std::function<void(int)>& run, hipStream_t st, int fallback,
           const std::function<bool(int)>& ok = nullptr);
  std::string to_json() const;
  void from_json(const std::string& text);
};

// A captured preconditioner application (one batched cycle) and the buffers
// and flags it was captured with.
struct CycleGraph {
  hipGraphExec_t exec = nullptr;
  int l = -1, B = 0, rs = 0;
  const void* in = nullptr;
  void* out = nullptr;
  const int* run = nullptr;
  bool warm = false;
};

struct Context;

// The learned near-null proposal network (three parallel-transport
// convolution layers nv -> ch -> ch -> nv) with its training state and the
// activations of its last forward pass over a context's lattice.
struct Net {
  int nv, ch, act_bits;  // act_bits: 16 = BF16 activations, 32 = FP32
  int cin[3], cout[3];
  DevBuf W[3], Wadj[3], gW[3], m[3], v[3];  // weights [9][cout][cin], their adjoint, gradients, Adam moments
  int step = 0;
  double last_loss = 0.0;
  hipStream_t stream;
  long V = 0;
  DevBuf act[4], scale[2], g0, g1, tgt, part;
  std::string err;
  Net(int nv_, int ch_, int act_bits_, uint64_t seed, hipStream_t st);
  long n_complex(int l) const;
  long n_floats() const;
  void set_weights(const float* host);
  void get_weights(float* host);
  void get_grads(float* host);
  void ensure(long V_);
  void forward(Context& c);
  double loss_grad(Context& c);
  void adam(float lr, hipStream_t st);
};

struct GmresState {
  int m = 0;
  long n = 0;
  int prec = 0;  // 0: double, 1: float
  bool flex = false;
  DevBuf V, Z, w, r, S, st;
};

struct Context {
  wcmg_params p{};
  hipStream_t stream = nullptr;
  std::string err;
  int nlev = 1;
  std::vector<LevelGeom> geo;
  std::vector<Transfer> tr;
  std::vector<std::unique_ptr<CoarseOp>> cop;  // cop[l-1] is the operator of level l
  // fine operator
  DevBuf perm0;                 // int32 device site -> lexicographic
  DevBuf U_lex, clover_lex;     // canonical copies (FP64)
  DevBuf U64, U32, clov64, clov32;
  SiteGeom sgeo;  // the level-0 device site order as arithmetic (Dslash neighbours)
  // neighbours of the fine Dslash: site arithmetic, or the table (reserved[0] flag 32, the reference form)
  const SiteGeom* dslash_geo() const { return (p.reserved[0] & 32) ? nullptr : &sgeo; }
  // two-row links of the fine Dslash (third row rebuilt), used when every link
  // is SU(3) to 1e-12 and the site arithmetic is on; reserved[0] flag 64 keeps
  // the full links (the reference form)
  DevBuf U64c, U32c;
  bool links_su3 = false;
  bool use_links2() const { return links_su3 && !(p.reserved[0] & 96); }
  template <typename R>
  const cplx<R>* dslash_links2() const {
    if (!use_links2()) return nullptr;
    return sizeof(R) == 8 ? (const cplx<R>*)U64c.p : (const cplx<R>*)U32c.p;
  }
  bool gauge_set = false, setup_done = false;
  // even-odd preconditioning: site parity (device order) and A^{-1} (packed)
  DevBuf par0, clovinv64, clovinv32;
  DevBuf eo_odd, eo_even, eo_pos;  // odd and even sites in device order; each site's compact position
  long eo_half = 0;       // number of odd sites
  bool eo_ready = false;
  // SAP domains (level-0 aggregates) of each colour: sap_doms [2][Vc/2]
  DevBuf sap_doms;
  long sap_ndoms = 0;
  // cooperative coarsest GMRES: launches that did not report a normal end (a
  // grid-barrier wait timed out, or the launch started after a time-out and
  // returned x = 0), and the last timeout's report
  long cgp_fallbacks = 0;
  std::string cgp_last_report;
  // the cooperative coarsest GMRES: its barrier flags count phases across
  // launches (the buffer keeps the phase reached), and it reports completion
  // in report slots of a coherent host-mapped mailbox, checked when the host
  // next waits for the stream (settle_coarse) instead of after every launch
  struct CgpLaunch {
    int seq;
    unsigned* bar;
    long nbar, V;
  };
  std::vector<CgpLaunch> cgp_pending;
  int cgp_seq = 0;
  bool cgp_forced = false;  // reserved[0] flag 128 has made its one launch time out
  std::map<std::string, void*> cgp_bar_at;
  int* mailbox = nullptr;  // kCgpMailboxInts words
  int* mailbox_dev = nullptr;
  // checks the cooperative coarsest solves launched up to sequence number
  // `upto` (all of them must have completed): adds their iteration counts,
  // and after a time-out clears the barrier buffer
  void settle_coarse(int upto = 0x7fffffff);
  // Solver state words published to host-mapped memory by a small kernel, so
  // the host can read a step's state while later steps are already queued.
  // One pair of slots per state buffer (a solver nested in another's
  // preconditioner has its own), each [publication number, words...].
  struct StateMailbox {
    int* h = nullptr;
    int* d = nullptr;
    int cap = 0;      // words per slot
    int seq = 0;      // last publication number
    int cgp[2] = {0, 0};  // coarsest-solve launches issued before each slot's publication
    std::vector<int> words;
  };
  std::map<const int*, StateMailbox> state_mb;
  // queues the publication of st[0..n); returns its number
  int publish_state(const int* st, int n);
  // the next publication of st[0..n) without the copy: its number, and in
  // *slot the device address a kernel writes it to (as publish_state's copy)
  int reserve_state(const int* st, int n, int** slot);
  // waits for publication `seq` of st (the last or the one before it) and
  // returns a copy of its words; the coarsest solves issued before it are
  // then checked
  const int* wait_state(const int* st, int seq);
  // A solver's progress checks: ahead() publishes the state and returns the
  // one published at the previous check (nullptr at the first), so the host
  // never waits for the steps it has just queued; now() publishes and waits.
  struct StateChecks {
    Context& c;
    const int* st;
    int n;
    int pend = 0;
    const int* ahead() { return ahead_issued(c.publish_state(st, n)); }
    // as ahead(), for a publication s that a kernel of the step has made
    const int* ahead_issued(int s) {
      const int* sv = pend ? c.wait_state(st, pend) : nullptr;
      pend = s;
      return sv;
    }
    const int* now() {
      pend = 0;
      return c.wait_state(st, c.publish_state(st, n));
    }
  };
  // workspaces
  std::map<std::string, std::unique_ptr<DevBuf>> ws;
  std::map<std::string, std::unique_ptr<GmresState>> gm;
  DevBuf partial, scratch64;
  // batched solves
  std::map<std::string, std::unique_ptr<BatchGmres>> bgm;
  DevBuf bpart;               // reduction partials [B][blocks][m]
  int coarse_kernel = 0;      // 0 auto, 1 per-row vector kernel, 2 matrix cores
  bool dslash_per_rhs = false;  // batched FP32 Dslash without shared links/clover
  bool use_graph = false;     // capture the batched cycle in a HIP graph
  bool no_checks = false;     // batched cycle without host checks (graph semantics)
  bool capturing = false;     // inside stream capture: no events, no tuning
  Tuner tuner;
  hipStream_t cap_stream = nullptr;
  CycleGraph cgraph;
  int64_t graph_launches = 0;
  int* pinned = nullptr;  // host-pinned status words
  double timers[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t coarse_iters = 0, cycles = 0;
  Profiler prof;

  Context(const wcmg_params& prm, hipStream_t s);
  ~Context();

  template <typename T>
  T* buf(const std::string& tag, long count);
  GmresState& gmres_state(const std::string& tag, int m, long n, int prec, bool flex);

  long n(int l) const { return geo[l].n(); }

  // operators
  template <typename R>
  void apply_op(int l, const cplx<R>* in, cplx<R>* out, int nrhs, const int* run, int terms = 0x1ff,
                cd64* dots = nullptr);
  // r = b - D x at the fine level, one launch
  template <typename R>
  void residual0(const cplx<R>* b, const cplx<R>* x, cplx<R>* r, const int* run);
  int store_prec_for(int l, bool single) const;

  // building blocks
  void set_gauge(const cd64* U);
  void set_clover(const cd64* blocks);
  void pack_clover();
  void initial_setup(int l);
  void relax_vectors(int l, int sweeps);
  void rebuild(int l);
  void galerkin(int l);
  void regalerkin_below(int l);
  void refine_iteration(int l);
  void setup_all();
  void setup_learned(Net& net, double threshold, int relax_sweeps, int* fell_back, double* quality);

  template <typename R>
  // x64 != nullptr (fine level): the final x goes to x64 in FP64 instead of x
  void mr(int l, const cplx<R>* b, cplx<R>* x, bool x0_zero, int steps, const int* run, cd64* x64 = nullptr);
  // `cycles` SAP cycles on D x = b at level 0 for nrhs fields (run flags with
  // stride rs; run may be null)
  void sap_prepare();
  // even-odd: parity table and A^{-1}; y = Dhat x on the odd sites (FP64,
  // x's even part must be zero, y's even part is set to zero)
  void eo_prepare();
  void schur64(const cd64* x, cd64* y, const int* run);
  void schur64c(const cd64* xo, cd64* yo, const int* run);
  template <typename R>
  void sap(const cplx<R>* b, cplx<R>* x, int cycles, int nrhs, const int* run, int rs);
  template <typename R>
  // x64 != nullptr: the result goes to x64 in FP64 (x is then scratch)
  void cycle(int l, const cplx<R>* r, cplx<R>* x, const int* run, cd64* x64 = nullptr);
  void precondition64(int l, const cd64* r, cd64* x, const int* run);
  template <typename R>
  int coarse_gmres(int lc, const cplx<R>* b, cplx<R>* x, const int* parent, int check_every);
  template <typename R>
  int gmres(GmresState& G, const std::function<void(const cplx<R>*, cplx<R>*, const int*)>& A,
            const std::function<void(const cplx<R>*, cplx<R>*, const int*)>* M, const cplx<R>* b, cplx<R>* x,
            bool x0_zero, int restart, int maxit, double tol, int fixed, bool stop_on_est, const int* parent,
            int check_every, bool single_reduction = false);
  template <typename R>
  void restrict_(int l, const cplx<R>* fine, cplx<R>* coarse, int nrhs, const int* run);
  template <typename R>
  void prolong_(int l, const cplx<R>* coarse, cplx<R>* fine, int accumulate, int nrhs, const int* run);
  template <typename R>
  double norm2_host(const cplx<R>* v, long n);
  void sync();

  // batched path (engine_batch.hip): B right-hand sides, RHS-major fields
  BatchGmres& bgmres_state(const std::string& tag, int m, long n, int B, int prec, bool flex);
  template <typename R>
  void apply_opB(int l, const cplx<R>* in, cplx<R>* out, int B, const int* run, int rs);
  template <typename R>
  void mrB(int l, const cplx<R>* b, cplx<R>* x, int B, int steps, const int* run, int rs);
  template <typename R>
  void cycleB(int l, const cplx<R>* r, cplx<R>* x, int B, const int* run, int rs);
  void precondition64B(int l, const cd64* r, cd64* x, int B, const int* run, int rs);
  template <typename R>
  void gmresB(BatchGmres& G, const BatchOp<R>& A, const BatchOp<R>* M, const cplx<R>* b, cplx<R>* x, bool x0_zero,
              int restart, int maxit, double tol, int fixed, bool stop_on_est, const int* parent, int prs,
              int check_every, int* iters, bool single_reduction = false);
  void drop_graph();
  void dslash32_batch(const cf32* in, cf32* out, int B, const int* run, int rs, cd64* dots);
  std::string dslash_key(int B) const;
  // solve D x_r = b_r, r < B (device-order FP64 fields); per-RHS outer iterations
  void solve_batched(const cd64* b, cd64* x, int B, int* iters);
};

// Ragged batched solve (engine_ragged.hip): problem k solves B[k] right-hand
// sides b[k] -> x[k] (device-order FP64 fields) on context cs[k]; the coarse
// solves of all problems share one coarse-operator launch per Arnoldi step.
// iters[k][r]: outer iterations; coarse_launches (may be null) counts those
// shared launches.  The caller validates the contexts (two levels, FP32
// cycle, equal Nb, storage, restarts and stream).
void solve_ragged(const std::vector<Context*>& cs, const std::vector<const cd64*>& b, const std::vector<cd64*>& x,
                  const std::vector<int>& B, std::vector<std::vector<int>>& iters, int64_t* coarse_launches);

}  // namespace wcmg
