// Ragged batched solve: several two-level problems, each with its own
// context (lattice, gauge field, hierarchy, tolerances) and its own batch of
// right-hand sides, solved together.  Every problem runs the method of the
// batched solve (one FP64 FGMRES per right-hand side, Sec. 2.1, preconditioned
// by the FP32 two-level cycle); the problems advance in lock-step so that the
// coarse-grid solves of all of them form one batch whose operator applies are
// ONE matrix-core launch over the sum of their coarse sites per Arnoldi step
// (the ragged form of the batched coarse apply).  The fine-level work and the
// Krylov vector operations stay per problem: their fields differ in size.
#include <chrono>
#include <cmath>

#include "engine.h"

namespace wcmg {

namespace {

// one problem of a ragged batch at one level
struct Slot {
  Context* c;
  BatchGmres* G;
  int B;
};

template <typename R>
using JointOp = std::function<void(const std::vector<const cplx<R>*>&, const std::vector<cplx<R>*>&,
                                   const std::vector<const int*>&, int)>;

// The restarted (F)GMRES of Context::gmresB for every problem of the batch at
// once: the same launches per problem, in the same order, with the operator A
// and the preconditioner M applied jointly to all problems at each step.
// Restart length m is shared; iteration limits and tolerances are per problem.
template <typename R>
void gmres_multi(std::vector<Slot>& q, const JointOp<R>& A, const JointOp<R>* M,
                 const std::vector<const cplx<R>*>& b, const std::vector<cplx<R>*>& x, bool x0_zero, int m,
                 const std::vector<int>& maxit, const std::vector<double>& tol, const std::vector<int>& fixed,
                 bool stop_on_est, const std::vector<const int*>& parent, int prs, int check_every,
                 std::vector<std::vector<int>>* iters, bool single_reduction) {
  const size_t K = q.size();
  hipStream_t stream = q[0].c->stream;
  std::vector<cplx<R>*> V(K), Z(K), w(K);
  std::vector<cd64*> S(K), H(K), g(K), y(K), misc(K), tmp(K), tmp2(K);
  std::vector<int*> st(K);
  std::vector<const int*> run(K), live(K), sr(K);
  std::vector<long> nn(K), bn(K), ss(K);
  std::vector<int> Gb(K), limit(K);
  int max_cycles = 0;
  for (size_t k = 0; k < K; ++k) {
    BatchGmres& G = *q[k].G;
    nn[k] = G.n;
    bn[k] = (long)G.B * G.n;
    ss[k] = G.ss;
    V[k] = G.V.as<cplx<R>>();
    Z[k] = M ? G.Z.as<cplx<R>>() : nullptr;
    w[k] = G.w.as<cplx<R>>();
    S[k] = G.S.as<cd64>();
    H[k] = S[k];
    g[k] = S[k] + (m + 1) * m + 2 * m;
    y[k] = g[k] + (m + 1);
    misc[k] = y[k] + m;
    tmp[k] = misc[k] + 8;
    tmp2[k] = tmp[k] + (m + 1);
    st[k] = G.st.as<int>();
    run[k] = st[k];
    live[k] = st[k] + 1;
    sr[k] = st[k] + 5;
    Gb[k] = bred_blocks(nn[k]);
    limit[k] = fixed[k] > 0 ? fixed[k] : maxit[k];
    max_cycles = std::max(max_cycles, check_every > 0 ? limit[k] : (limit[k] + m - 1) / m);
  }
  auto part = [&](size_t k) { return q[k].c->bpart.as<cd64>(); };
  for (size_t k = 0; k < K; ++k) {
    const int B = q[k].B;
    launch_bgmres_init(st[k], B, parent[k], prs, stream);
    if (x0_zero)
      launch_belem<cplx<R>, cplx<R>>(x[k], nn[k], x[k], nn[k], nullptr, 0, nullptr, 0, nn[k], B, 0, live[k], 8,
                                     stream);
    launch_bdot<R>(b[k], 0, nn[k], 1, b[k], nn[k], nn[k], B, part(k), misc[k] + 0, 1, ss[k], 0, live[k], 8, stream);
  }
  // progress checks as in Context::gmres, every problem's state published on
  // the shared stream (through the first context)
  std::vector<Context::StateChecks> chk;
  for (size_t k = 0; k < K; ++k) chk.push_back(Context::StateChecks{*q[0].c, st[k], 8 * q[k].B});
  std::vector<const int*> sv(K, nullptr);
  auto any = [&](int word) {
    for (size_t k = 0; k < K; ++k)
      for (int r = 0; r < q[k].B; ++r)
        if (sv[k][8 * r + word]) return true;
    return false;
  };
  auto check_ahead = [&]() {  // false while the previous check's state is not known
    bool known = true;
    for (size_t k = 0; k < K; ++k) known = (sv[k] = chk[k].ahead()) != nullptr && known;
    return known;
  };
  auto check_now = [&]() {
    for (size_t k = 0; k < K; ++k) sv[k] = chk[k].now();
  };
  bool have_last = false;
  std::vector<const cplx<R>*> cin(K);
  std::vector<cplx<R>*> cout(K);
  for (int cyc = 0; cyc < max_cycles; ++cyc) {
    if (!(cyc == 0 && x0_zero)) {
      for (size_t k = 0; k < K; ++k) {
        cin[k] = x[k];
        cout[k] = w[k];
      }
      A(cin, cout, live, 8);
    }
    for (size_t k = 0; k < K; ++k) {
      const int B = q[k].B;
      if (cyc == 0 && x0_zero)
        launch_belem<cplx<R>, cplx<R>>(V[k], nn[k], b[k], nn[k], nullptr, 0, nullptr, 0, nn[k], B, 1, live[k], 8,
                                       stream);
      else
        launch_belem<cplx<R>, cplx<R>>(V[k], nn[k], b[k], nn[k], w[k], nn[k], nullptr, 0, nn[k], B, 2, live[k], 8,
                                       stream);
      launch_bdot<R>(V[k], 0, nn[k], 1, V[k], nn[k], nn[k], B, part(k), misc[k] + 1, 1, ss[k], 0, live[k], 8, stream);
      launch_bgmres_cycle_start(st[k], S[k], ss[k], B, m, tol[k], limit[k], fixed[k], stream);
      launch_belem<cplx<R>, cplx<R>>(V[k], nn[k], V[k], nn[k], nullptr, 0, misc[k] + 1, ss[k], nn[k], B, 3, run[k],
                                     8, stream);
    }
    for (int j = 0; j < m; ++j) {
      if (M) {
        for (size_t k = 0; k < K; ++k) {
          cin[k] = V[k] + j * bn[k];
          cout[k] = Z[k] + j * bn[k];
        }
        (*M)(cin, cout, run, 8);
      }
      if (single_reduction) {
        for (size_t k = 0; k < K; ++k) {
          cin[k] = M ? Z[k] + j * bn[k] : V[k] + j * bn[k];
          cout[k] = V[k] + (j + 1) * bn[k];
        }
        A(cin, cout, run, 8);
        for (size_t k = 0; k < K; ++k) {
          const int B = q[k].B;
          cplx<R>* wj = V[k] + (j + 1) * bn[k];
          launch_barnoldi_dots<R>(V[k], bn[k], nn[k], j, nn[k], j > 0 ? misc[k] + 4 : nullptr, ss[k], part(k), B,
                                  run[k], 8, stream);
          launch_bdot_finish(part(k), Gb[k], j + 2, j + 2, B, tmp[k], 1, ss[k], 0, run[k], 8, stream);
          launch_bgmres_sr(st[k], S[k], ss[k], B, m, j, tmp[k], tmp2[k], 0, stream);
          launch_bmulti_axpy<R>(wj, nn[k], V[k], bn[k], nn[k], j + 1, nullptr, 0, tmp[k], 1, ss[k], -1.0, nn[k], B,
                                nullptr, sr[k], 8, stream);
          launch_barnoldi_dots<R>(V[k], bn[k], nn[k], j, nn[k], nullptr, ss[k], part(k), B, sr[k], 8, stream);
          launch_bdot_finish(part(k), Gb[k], j + 2, j + 2, B, tmp2[k], 1, ss[k], 0, sr[k], 8, stream);
          launch_bgmres_sr(st[k], S[k], ss[k], B, m, j, tmp[k], tmp2[k], 1, stream);
          launch_bgmres_givens(st[k], S[k], ss[k], B, m, j, tol[k], limit[k], fixed[k], stop_on_est ? 1 : 0, stream);
          if (j + 1 < m)
            launch_bupdate_scale<R>(wj, nn[k], V[k], bn[k], nn[k], j + 1, tmp[k], ss[k], misc[k] + 3, ss[k], nn[k], B,
                                    run[k], 8, stream);
        }
      } else {
        for (size_t k = 0; k < K; ++k) {
          cin[k] = M ? Z[k] + j * bn[k] : V[k] + j * bn[k];
          cout[k] = w[k];
        }
        A(cin, cout, run, 8);
        for (size_t k = 0; k < K; ++k) {
          const int B = q[k].B;
          // classical Gram-Schmidt applied twice; |w|^2 from the last update
          launch_bdot<R>(V[k], bn[k], nn[k], j + 1, w[k], nn[k], nn[k], B, part(k), H[k] + j, m, ss[k], 0, run[k], 8,
                         stream);
          if (j + 1 <= kFusedMaxM) {
            launch_bmulti_axpy_dot<R>(w[k], nn[k], V[k], bn[k], nn[k], j + 1, H[k] + j, m, ss[k], nn[k], B, part(k),
                                      run[k], 8, stream);
            launch_bdot_finish(part(k), Gb[k], j + 1, j + 1, B, tmp[k], 1, ss[k], 0, run[k], 8, stream);
          } else {
            launch_bmulti_axpy<R>(w[k], nn[k], V[k], bn[k], nn[k], j + 1, nullptr, 0, H[k] + j, m, ss[k], -1.0, nn[k],
                                  B, nullptr, run[k], 8, stream);
            launch_bdot<R>(V[k], bn[k], nn[k], j + 1, w[k], nn[k], nn[k], B, part(k), tmp[k], 1, ss[k], 0, run[k], 8,
                           stream);
          }
          launch_bdot_finish(part(k), Gb[k], j + 1, j + 1, B, H[k] + j, m, ss[k], 1, run[k], 8, stream);
          launch_bmulti_axpy<R>(w[k], nn[k], V[k], bn[k], nn[k], j + 1, nullptr, 0, tmp[k], 1, ss[k], -1.0, nn[k], B,
                                part(k), run[k], 8, stream);
          launch_bdot_finish(part(k), Gb[k], 1, 1, B, misc[k] + 3, 1, ss[k], 0, run[k], 8, stream);
          launch_bgmres_givens(st[k], S[k], ss[k], B, m, j, tol[k], limit[k], fixed[k], stop_on_est ? 1 : 0, stream);
          if (j + 1 < m)
            launch_belem<cplx<R>, cplx<R>>(V[k] + (j + 1) * bn[k], nn[k], w[k], nn[k], nullptr, 0, misc[k] + 3, ss[k],
                                           nn[k], B, 3, run[k], 8, stream);
        }
      }
      if (check_every > 0 && (j + 1) % check_every == 0 && j + 1 < m) {
        if (check_ahead() && !any(0)) break;
      }
    }
    for (size_t k = 0; k < K; ++k) {
      const int B = q[k].B;
      launch_bgmres_solve_y(st[k], S[k], ss[k], B, m, stream);
      launch_bmulti_axpy<R>(x[k], nn[k], M ? Z[k] : V[k], bn[k], nn[k], m, st[k] + 2, 8, y[k], 1, ss[k], 1.0, nn[k], B,
                            nullptr, nullptr, 0, stream);
      launch_bgmres_cycle_end(st[k], B, stream);
    }
    if (check_every > 0) {
      check_now();
      have_last = true;
      if (!any(1)) break;
    }
  }
  if (check_every > 0) {
    if (!have_last) check_now();
    if (iters)
      for (size_t k = 0; k < K; ++k)
        for (int r = 0; r < q[k].B; ++r) (*iters)[k][r] = sv[k][8 * r + 3];
  }
}

}  // namespace

void solve_ragged(const std::vector<Context*>& cs, const std::vector<const cd64*>& b, const std::vector<cd64*>& x,
                  const std::vector<int>& Bs, std::vector<std::vector<int>>& iters, int64_t* coarse_launches) {
  const size_t K = cs.size();
  Context& c0 = *cs[0];
  hipStream_t stream = c0.stream;
  const int prec = c0.store_prec_for(1, true);
  const int m_out = c0.p.outer_restart, m_c = c0.p.coarse_restart;
  for (Context* c : cs) {
    const long need = (long)16 * kPartialSlots;
    if (c->bpart.bytes < (size_t)need * sizeof(cd64)) c->bpart.alloc((size_t)need * sizeof(cd64));
    c->cop[0]->refresh_mfma(prec, stream);
    c->coarse_iters = 0;
    c->cycles = 0;
  }
  std::vector<Slot> outer(K), coarse(K);
  std::vector<int> maxit_o(K), maxit_c(K), fixed_o(K, 0), fixed_c(K);
  std::vector<double> tol_o(K), tol_c(K);
  for (size_t k = 0; k < K; ++k) {
    Context& c = *cs[k];
    outer[k] = Slot{&c, &c.bgmres_state("rg_outer", m_out, c.n(0), Bs[k], 0, true), Bs[k]};
    coarse[k] = Slot{&c, &c.bgmres_state("rg_coarse", m_c, c.n(1), Bs[k], 1, false), Bs[k]};
    maxit_o[k] = c.p.outer_maxit;
    tol_o[k] = c.p.outer_tol;
    maxit_c[k] = c.p.coarse_maxit;
    tol_c[k] = c.p.coarse_tol;
    fixed_c[k] = c.p.coarse_fixed_iters;
  }
  // the joint coarse operator: every problem's D_c on its batch, one launch
  JointOp<float> Ac = [&](const std::vector<const cf32*>& in, const std::vector<cf32*>& out,
                          const std::vector<const int*>& run, int rs) {
    RaggedTable t{};
    t.n = (int)K;
    t.nb = cs[0]->cop[0]->nb;
    for (size_t k = 0; k < K; ++k) {
      CoarseOp& C = *cs[k]->cop[0];
      t.p[k] = RaggedProblem{C.mfma[prec].p, in[k], out[k], C.nbr.as<int>(), C.V, Bs[k], run[k], rs};
    }
    c0.prof.begin_kernel(prec == WCMG_F32 ? "coarse_mfma_ragged_f32" : "coarse_mfma_ragged_bf16");
    launch_coarse_apply_mfma_ragged(prec, t, stream);
    c0.prof.end(prec == WCMG_F32 ? "coarse_mfma_ragged_f32" : "coarse_mfma_ragged_bf16", stream);
    if (coarse_launches) ++*coarse_launches;
  };
  // the joint preconditioner: FP64 in, the two-level cycle in FP32 per problem
  // around the joint coarse solve, FP64 out
  JointOp<double> M = [&](const std::vector<const cd64*>& in, const std::vector<cd64*>& out,
                          const std::vector<const int*>& run, int rs) {
    std::vector<const cf32*> rc(K);
    std::vector<cf32*> rcw(K), ec(K), r32(K), x32(K);
    for (size_t k = 0; k < K; ++k) {
      Context& c = *cs[k];
      const int B = Bs[k];
      const long nn = c.n(0), nc = c.n(1);
      r32[k] = c.buf<cf32>("rg_r32", B * nn);
      x32[k] = c.buf<cf32>("rg_x32", B * nn);
      rcw[k] = c.buf<cf32>("rg_rc", B * nc);
      ec[k] = c.buf<cf32>("rg_ec", B * nc);
      rc[k] = rcw[k];
      launch_belem<cd64, cf32>(r32[k], nn, in[k], nn, nullptr, 0, nullptr, 0, nn, B, 1, run[k], rs, stream);
      const Transfer& T = c.tr[0];
      launch_restrict<float>(r32[k], rcw[k], T.P32.as<cf32>(), c.geo[0].lay, T.agg_sites.as<int>(), T.A, T.Vc, T.nb, B,
                             run[k], stream, rs);
    }
    std::vector<std::vector<int>> its(K);
    for (size_t k = 0; k < K; ++k) its[k].assign(Bs[k], 0);
    gmres_multi<float>(coarse, Ac, nullptr, rc, ec, true, m_c, maxit_c, tol_c, fixed_c, true, run, rs, 4, &its, false);
    for (size_t k = 0; k < K; ++k) {
      Context& c = *cs[k];
      const int B = Bs[k];
      const long nn = c.n(0);
      for (int r = 0; r < B; ++r) c.coarse_iters += its[k][r];
      const Transfer& T = c.tr[0];
      launch_prolong<float>(ec[k], x32[k], T.P32.as<cf32>(), c.geo[0].lay, T.coarse_of.as<int>(), T.Vc, T.nb, 0, B,
                            run[k], stream, rs, T.agg_sites.as<int>(), T.A);
      if (c.p.smoother == 1) c.sap<float>(r32[k], x32[k], c.p.post_smooth, B, run[k], rs);
      else c.mrB<float>(0, r32[k], x32[k], B, c.p.post_smooth, run[k], rs);
      launch_belem<cf32, cd64>(out[k], nn, x32[k], nn, nullptr, 0, nullptr, 0, nn, B, 1, run[k], rs, stream);
      c.cycles += B;
    }
  };
  JointOp<double> A = [&](const std::vector<const cd64*>& in, const std::vector<cd64*>& out,
                          const std::vector<const int*>& run, int rs) {
    for (size_t k = 0; k < K; ++k) cs[k]->apply_opB<double>(0, in[k], out[k], Bs[k], run[k], rs);
  };
  std::vector<const int*> none(K, nullptr);
  gmres_multi<double>(outer, A, &M, b, x, false, m_out, maxit_o, tol_o, fixed_o, false, none, 0, 1, &iters,
                      !(c0.p.reserved[0] & 8));
}

}  // namespace wcmg
