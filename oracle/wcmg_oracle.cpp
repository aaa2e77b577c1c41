// Plain FP64 CPU oracle for the Wilson-clover multigrid hot path of
// D. Richtmann, P. A. Boyle, T. Wettig, "Multigrid for Wilson Clover Fermions
// in Grid" (LATTICE2018, arXiv:1904.08678).
//
// TEST INFRASTRUCTURE ONLY.  It is slow and straightforward on purpose: it is
// the independent check of the GPU library.  Only the tests, the smoke check
// and the CPU-baseline leg of the benchmark may load it; the GPU library never
// does, and the two share no code, headers or tables.
//
// The paper names its pieces (Sec. 2.1: Aggregation, CoarsenedMatrix with
// Mdiag/Mdir, the recursive solver class, initial and iterative setup, MR,
// GMRES, FGMRES, mixed precision; Sec. 2.2: the chirality-preserving
// prolongator) but writes no formula for the Dirac operator, the clover term,
// the smoother or the setup.  Every such formula below is a reading, stated
// where it is used:
//   * gamma matrices in the chiral Euclidean basis,
//       gamma_k = [[0, -i s_k], [i s_k, 0]] (k = x, y, z),  gamma_t = [[0,1],[1,0]],
//     so gamma_5 = gamma_x gamma_y gamma_z gamma_t = diag(1, 1, -1, -1);
//   * D psi(x) = (4 + m0) psi(x) + C(x) psi(x)
//              - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
//                           + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ],
//     with a factor -1 on every t-hop that crosses the t boundary when the
//     fermion boundary condition is antiperiodic;
//   * C(x) = c_sw (i/4) sum_{mu,nu} sigma_{mu nu} F_{mu nu}(x),
//     sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu], F = (Q - Q^dag)/8, Q the sum
//     of the four plaquette leaves around x in the mu-nu plane.
// Fermion component index k = 3*spin + colour; the first half of the
// components (spins 0,1) has gamma_5 = +1.  On coarse levels the first half of
// the Nb components carries sigma_3 = +1 (Sec. 2.2).
//
// Parity unpinned: nothing.  Every routine is pinned by the CPU tests against
// closed forms, invariants or brute force (see the test files).

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef std::complex<double> cd;
typedef std::vector<cd> cvec;

namespace {

const cd kI(0.0, 1.0);

// ----------------------------------------------------------------------------
// Dirac algebra (chiral Euclidean basis; the paper leaves the basis open).
// ----------------------------------------------------------------------------
struct Gammas {
  cd g[4][4][4];   // g[mu][row][col]
  cd g5[4][4];
  cd sigma[4][4][4][4];  // sigma[mu][nu][row][col] = (i/2)[g_mu, g_nu]
};

void pauli(int k, cd s[2][2]) {
  s[0][0] = s[0][1] = s[1][0] = s[1][1] = 0.0;
  if (k == 0) { s[0][1] = 1.0; s[1][0] = 1.0; }
  if (k == 1) { s[0][1] = -kI; s[1][0] = kI; }
  if (k == 2) { s[0][0] = 1.0; s[1][1] = -1.0; }
}

void matmul4(const cd a[4][4], const cd b[4][4], cd c[4][4]) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cd s = 0.0;
      for (int k = 0; k < 4; ++k) s += a[i][k] * b[k][j];
      c[i][j] = s;
    }
}

Gammas make_gammas() {
  Gammas G;
  std::memset(&G, 0, sizeof(G));
  for (int k = 0; k < 3; ++k) {
    cd s[2][2];
    pauli(k, s);
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        G.g[k][a][2 + b] = -kI * s[a][b];
        G.g[k][2 + a][b] = kI * s[a][b];
      }
  }
  for (int a = 0; a < 2; ++a) {
    G.g[3][a][2 + a] = 1.0;
    G.g[3][2 + a][a] = 1.0;
  }
  cd t1[4][4], t2[4][4];
  matmul4(G.g[0], G.g[1], t1);
  matmul4(t1, G.g[2], t2);
  matmul4(t2, G.g[3], G.g5);
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = 0; nu < 4; ++nu) {
      cd ab[4][4], ba[4][4];
      matmul4(G.g[mu], G.g[nu], ab);
      matmul4(G.g[nu], G.g[mu], ba);
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) G.sigma[mu][nu][i][j] = 0.5 * kI * (ab[i][j] - ba[i][j]);
    }
  return G;
}

const Gammas& gammas() {
  static Gammas G = make_gammas();
  return G;
}

// ----------------------------------------------------------------------------
// Lattice geometry: lexicographic sites, x fastest; directions d = 1..8 are
// +x, -x, +y, -y, +z, -z, +t, -t; d = 0 is the site itself.
// ----------------------------------------------------------------------------
struct Lattice {
  int L[4] = {0, 0, 0, 0};
  long V = 0;
  Lattice() {}
  explicit Lattice(const int* l) {
    V = 1;
    for (int mu = 0; mu < 4; ++mu) { L[mu] = l[mu]; V *= l[mu]; }
  }
  void coords(long i, int x[4]) const {
    for (int mu = 0; mu < 4; ++mu) { x[mu] = (int)(i % L[mu]); i /= L[mu]; }
  }
  long index(const int x[4]) const {
    return x[0] + (long)L[0] * (x[1] + (long)L[1] * (x[2] + (long)L[2] * x[3]));
  }
  long shift(long i, int mu, int step) const {
    int x[4];
    coords(i, x);
    x[mu] = ((x[mu] + step) % L[mu] + L[mu]) % L[mu];
    return index(x);
  }
  long neighbour(long i, int d) const {  // d in 1..8
    int mu = (d - 1) / 2;
    return shift(i, mu, ((d - 1) % 2 == 0) ? 1 : -1);
  }
};

// ----------------------------------------------------------------------------
// Level operators expose the coarsening interface of Sec. 2.1: Mdiag (the
// site-diagonal part) and Mdir (the hopping term of one direction).  D itself
// is Mdiag plus the eight Mdir terms.
// ----------------------------------------------------------------------------
struct LevelOp {
  Lattice lat;
  int ns = 0;  // complex components per site
  virtual ~LevelOp() {}
  long size() const { return lat.V * ns; }
  virtual void mdiag(const cd* in, cd* out) const = 0;          // out  = Mdiag in
  virtual void mdir_add(int d, const cd* in, cd* out) const = 0;  // out += Mdir_d in
  void mdir(int d, const cd* in, cd* out) const {
    std::fill(out, out + size(), cd(0.0));
    mdir_add(d, in, out);
  }
  void apply(const cd* in, cd* out) const {
    mdiag(in, out);
    for (int d = 1; d <= 8; ++d) mdir_add(d, in, out);
  }
};

// Wilson-clover operator on the fine lattice.
struct WilsonClover : LevelOp {
  cvec U;      // [V][4][3][3]
  cvec C;      // [V][12][12], the clover term alone
  double m0 = 0.0;
  bool antiperiodic = true;

  const cd* link(long x, int mu) const { return &U[(x * 4 + mu) * 9]; }

  void mdiag(const cd* in, cd* out) const override {
#pragma omp parallel for
    for (long x = 0; x < lat.V; ++x) {
      const cd* c = &C[x * 144];
      for (int i = 0; i < 12; ++i) {
        cd s = (4.0 + m0) * in[x * 12 + i];
        for (int j = 0; j < 12; ++j) s += c[i * 12 + j] * in[x * 12 + j];
        out[x * 12 + i] = s;
      }
    }
  }

  void mdir_add(int d, const cd* in, cd* out) const override {
#pragma omp parallel for
    for (long x = 0; x < lat.V; ++x) hop_add(x, d, &in[lat.neighbour(x, d) * 12], &out[x * 12]);
  }

  // out (12 components at site x) += Mdir_d at x applied to psi, the spinor at
  // the neighbour of x in direction d.
  void hop_add(long x, int d, const cd* psi, cd* out) const {
    const Gammas& G = gammas();
    const int mu = (d - 1) / 2;
    const bool fwd = ((d - 1) % 2 == 0);
    {
      long y = lat.neighbour(x, d);
      int xc[4];
      lat.coords(x, xc);
      double sign = 1.0;
      if (antiperiodic && mu == 3) {
        if (fwd && xc[3] == lat.L[3] - 1) sign = -1.0;
        if (!fwd && xc[3] == 0) sign = -1.0;
      }
      // colour transport
      cd u[3][3];
      const cd* l = fwd ? link(x, mu) : link(y, mu);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) u[a][b] = fwd ? l[a * 3 + b] : std::conj(l[b * 3 + a]);
      cd chi[4][3];
      for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
          cd t = 0.0;
          for (int b = 0; b < 3; ++b) t += u[a][b] * psi[s * 3 + b];
          chi[s][a] = t;
        }
      // spin structure -(1/2)(1 -+ gamma_mu)
      for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
          cd t = 0.0;
          for (int r = 0; r < 4; ++r) {
            cd p = (s == r ? cd(1.0) : cd(0.0)) + (fwd ? -G.g[mu][s][r] : G.g[mu][s][r]);
            t += p * chi[r][a];
          }
          out[s * 3 + a] += -0.5 * sign * t;
        }
    }
  }
};

// Coarse operator: nine dense Nb x Nb blocks per site (Mdiag = block 0, Mdir_d
// = block d, acting on the neighbour in direction d).
struct CoarseOp : LevelOp {
  cvec M;  // [V][9][ns][ns]
  const cd* block(long x, int d) const { return &M[((x * 9 + d) * ns) * ns]; }

  void mdiag(const cd* in, cd* out) const override {
#pragma omp parallel for
    for (long x = 0; x < lat.V; ++x) {
      const cd* m = block(x, 0);
      for (int a = 0; a < ns; ++a) {
        cd s = 0.0;
        for (int b = 0; b < ns; ++b) s += m[a * ns + b] * in[x * ns + b];
        out[x * ns + a] = s;
      }
    }
  }
  void mdir_add(int d, const cd* in, cd* out) const override {
#pragma omp parallel for
    for (long x = 0; x < lat.V; ++x) {
      long y = lat.neighbour(x, d);
      const cd* m = block(x, d);
      for (int a = 0; a < ns; ++a) {
        cd s = 0.0;
        for (int b = 0; b < ns; ++b) s += m[a * ns + b] * in[y * ns + b];
        out[x * ns + a] += s;
      }
    }
  }
};

// ----------------------------------------------------------------------------
// Clover term (Sheikholeslami-Wohlert; normalisation is a reading).
// ----------------------------------------------------------------------------
void su3_mul(const cd* a, const cd* b, cd* c) {
  cd t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cd s = 0.0;
      for (int k = 0; k < 3; ++k) s += a[i * 3 + k] * b[k * 3 + j];
      t[i * 3 + j] = s;
    }
  std::memcpy(c, t, sizeof(t));
}
void su3_dag(const cd* a, cd* c) {
  cd t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) t[i * 3 + j] = std::conj(a[j * 3 + i]);
  std::memcpy(c, t, sizeof(t));
}

// Sum of the four plaquette leaves in the mu-nu plane that start and end at x.
void clover_leaves(const Lattice& lat, const cd* U, long x, int mu, int nu, cd* Q) {
  auto lk = [&](long s, int m) { return U + (s * 4 + m) * 9; };
  long xpm = lat.shift(x, mu, 1), xpn = lat.shift(x, nu, 1);
  long xmm = lat.shift(x, mu, -1), xmn = lat.shift(x, nu, -1);
  long xmm_pn = lat.shift(xmm, nu, 1), xmm_mn = lat.shift(xmm, nu, -1);
  long xmn_pm = lat.shift(xmn, mu, 1);
  cd a[9], b[9], leaf[9];
  for (int i = 0; i < 9; ++i) Q[i] = 0.0;
  // leaf 1: x -> x+mu -> x+mu+nu -> x+nu -> x
  su3_mul(lk(x, mu), lk(xpm, nu), leaf);
  su3_dag(lk(xpn, mu), a); su3_mul(leaf, a, leaf);
  su3_dag(lk(x, nu), a); su3_mul(leaf, a, leaf);
  for (int i = 0; i < 9; ++i) Q[i] += leaf[i];
  // leaf 2: x -> x+nu -> x+nu-mu -> x-mu -> x
  su3_dag(lk(xmm_pn, mu), a); su3_mul(lk(x, nu), a, leaf);
  su3_dag(lk(xmm, nu), a); su3_mul(leaf, a, leaf);
  su3_mul(leaf, lk(xmm, mu), leaf);
  for (int i = 0; i < 9; ++i) Q[i] += leaf[i];
  // leaf 3: x -> x-mu -> x-mu-nu -> x-nu -> x
  su3_dag(lk(xmm, mu), a); su3_dag(lk(xmm_mn, nu), b); su3_mul(a, b, leaf);
  su3_mul(leaf, lk(xmm_mn, mu), leaf);
  su3_mul(leaf, lk(xmn, nu), leaf);
  for (int i = 0; i < 9; ++i) Q[i] += leaf[i];
  // leaf 4: x -> x-nu -> x-nu+mu -> x+mu -> x
  su3_dag(lk(xmn, nu), a); su3_mul(a, lk(xmn, mu), leaf);
  su3_mul(leaf, lk(xmn_pm, nu), leaf);
  su3_dag(lk(x, mu), a); su3_mul(leaf, a, leaf);
  for (int i = 0; i < 9; ++i) Q[i] += leaf[i];
}

void build_clover(const Lattice& lat, const cd* U, double csw, cd* C) {
  const Gammas& G = gammas();
#pragma omp parallel for
  for (long x = 0; x < lat.V; ++x) {
    cd* c = C + x * 144;
    for (int i = 0; i < 144; ++i) c[i] = 0.0;
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = 0; nu < 4; ++nu) {
        if (mu == nu) continue;
        cd Q[9], F[9];
        clover_leaves(lat, U, x, mu, nu, Q);
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) F[a * 3 + b] = (Q[a * 3 + b] - std::conj(Q[b * 3 + a])) / 8.0;
        for (int s = 0; s < 4; ++s)
          for (int r = 0; r < 4; ++r)
            for (int a = 0; a < 3; ++a)
              for (int b = 0; b < 3; ++b)
                c[(s * 3 + a) * 12 + r * 3 + b] += csw * 0.25 * kI * G.sigma[mu][nu][s][r] * F[a * 3 + b];
      }
  }
}

// ----------------------------------------------------------------------------
// Vector algebra.  <a, b> = sum conj(a) b.
// ----------------------------------------------------------------------------
cd dot(long n, const cd* a, const cd* b) {
  cd s = 0.0;
  for (long i = 0; i < n; ++i) s += std::conj(a[i]) * b[i];
  return s;
}
double norm(long n, const cd* a) { return std::sqrt(std::real(dot(n, a, a))); }
void axpy(long n, cd a, const cd* x, cd* y) {
  for (long i = 0; i < n; ++i) y[i] += a * x[i];
}

// ----------------------------------------------------------------------------
// Aggregation (Sec. 3: the coarse-to-fine lookup table of blockProject).
// Aggregates are origin-aligned hypercubes of b[0]x..xb[3] sites; coarse index
// and in-block offset are both lexicographic with x fastest.
// ----------------------------------------------------------------------------
struct Aggregation {
  Lattice fine, coarse;
  int b[4] = {1, 1, 1, 1};
  long A = 1;
  std::vector<long> agg, off;   // per fine site
  std::vector<long> site_of;    // [Vc][A]: the lookup table, coarse site -> fine sites
};

int make_aggregation(const Lattice& fine, const int* block, Aggregation& ag) {
  int lc[4];
  ag.fine = fine;
  ag.A = 1;
  for (int mu = 0; mu < 4; ++mu) {
    if (block[mu] <= 0 || fine.L[mu] % block[mu] != 0) return 2;
    ag.b[mu] = block[mu];
    lc[mu] = fine.L[mu] / block[mu];
    ag.A *= block[mu];
  }
  ag.coarse = Lattice(lc);
  ag.agg.assign(fine.V, 0);
  ag.off.assign(fine.V, 0);
  ag.site_of.assign(ag.coarse.V * ag.A, 0);
  for (long i = 0; i < fine.V; ++i) {
    int x[4], cx[4], ox[4];
    fine.coords(i, x);
    for (int mu = 0; mu < 4; ++mu) { cx[mu] = x[mu] / ag.b[mu]; ox[mu] = x[mu] % ag.b[mu]; }
    long c = ag.coarse.index(cx);
    long o = ox[0] + (long)ag.b[0] * (ox[1] + (long)ag.b[1] * (ox[2] + (long)ag.b[2] * ox[3]));
    ag.agg[i] = c;
    ag.off[i] = o;
    ag.site_of[c * ag.A + o] = i;
  }
  return 0;
}

// ----------------------------------------------------------------------------
// Prolongator (Sec. 2.2): P = [ (1+g5)/2 psi_i , (1-g5)/2 psi_i ], each
// chirality half of each vector orthonormalised aggregate by aggregate.
// Pv[i] holds the orthonormalised halves of vector i; column b of P is vector
// b mod nv restricted to chirality b / nv (first half of components for b < nv).
// The orthonormalisation is a reading: modified Gram-Schmidt in index order,
// each vector projected twice against the earlier ones, in FP64.
// ----------------------------------------------------------------------------
int build_prolongator(const Aggregation& ag, int ns, int nv, const cvec& vecs, cvec& Pv) {
  const long V = ag.fine.V;
  const int h = ns / 2;
  Pv = vecs;
  int status = 0;
#pragma omp parallel for
  for (long c = 0; c < ag.coarse.V; ++c) {
    for (int chi = 0; chi < 2; ++chi) {
      auto elem = [&](int i, long o, int k) -> cd& {
        long x = ag.site_of[c * ag.A + o];
        return Pv[((long)i * V + x) * ns + chi * h + k];
      };
      for (int i = 0; i < nv; ++i) {
        double pre = 0.0;
        for (long o = 0; o < ag.A; ++o)
          for (int k = 0; k < h; ++k) pre += std::norm(elem(i, o, k));
        pre = std::sqrt(pre);
        for (int pass = 0; pass < 2; ++pass)
          for (int j = 0; j < i; ++j) {
            cd p = 0.0;
            for (long o = 0; o < ag.A; ++o)
              for (int k = 0; k < h; ++k) p += std::conj(elem(j, o, k)) * elem(i, o, k);
            for (long o = 0; o < ag.A; ++o)
              for (int k = 0; k < h; ++k) elem(i, o, k) -= p * elem(j, o, k);
          }
        double post = 0.0;
        for (long o = 0; o < ag.A; ++o)
          for (int k = 0; k < h; ++k) post += std::norm(elem(i, o, k));
        post = std::sqrt(post);
        if (!(post > 1e-10 * pre) || pre == 0.0) {
#pragma omp critical
          status = 6;
          post = (post > 0.0) ? post : 1.0;
        }
        for (long o = 0; o < ag.A; ++o)
          for (int k = 0; k < h; ++k) elem(i, o, k) /= post;
      }
    }
  }
  return status;
}

// R = P^dag, restriction onto the coarse lattice (blockProject).
void restrict_vec(const Aggregation& ag, int ns, int nv, const cvec& Pv, const cd* fine, cd* coarse) {
  const long V = ag.fine.V;
  const int h = ns / 2, nb = 2 * nv;
#pragma omp parallel for
  for (long c = 0; c < ag.coarse.V; ++c) {
    for (int b = 0; b < nb; ++b) {
      int i = b % nv, chi = b / nv;
      cd s = 0.0;
      for (long o = 0; o < ag.A; ++o) {
        long x = ag.site_of[c * ag.A + o];
        for (int k = chi * h; k < chi * h + h; ++k) s += std::conj(Pv[((long)i * V + x) * ns + k]) * fine[x * ns + k];
      }
      coarse[c * nb + b] = s;
    }
  }
}

// P, prolongation onto the fine lattice (promote).
void prolong_vec(const Aggregation& ag, int ns, int nv, const cvec& Pv, const cd* coarse, cd* fine) {
  const long V = ag.fine.V;
  const int h = ns / 2, nb = 2 * nv;
#pragma omp parallel for
  for (long x = 0; x < V; ++x) {
    long c = ag.agg[x];
    for (int k = 0; k < ns; ++k) {
      int chi = k / h;
      cd s = 0.0;
      for (int i = 0; i < nv; ++i) s += Pv[((long)i * V + x) * ns + k] * coarse[c * nb + chi * nv + i];
      fine[x * ns + k] = s;
    }
  }
}

// Galerkin coarse operator D_c = P^dag D P, assembled through the coarsening
// interface (Sec. 2.1): block 0 collects Mdiag and every hop whose two ends lie
// in the same aggregate, block d collects the hops in direction d that leave it.
int galerkin(const LevelOp& D, const Aggregation& ag, int nv, const cvec& Pv, CoarseOp& Dc) {
  const long V = ag.fine.V, Vc = ag.coarse.V;
  const int ns = D.ns, h = ns / 2, nb = 2 * nv;
  for (int mu = 0; mu < 4; ++mu)
    if (ag.coarse.L[mu] < 2) return 2;
  Dc.lat = ag.coarse;
  Dc.ns = nb;
  Dc.M.assign(Vc * 9 * nb * nb, cd(0.0));
  cvec v(V * ns), w(V * ns);
  for (int b = 0; b < nb; ++b) {
    int ib = b % nv, chib = b / nv;
    std::fill(v.begin(), v.end(), cd(0.0));
    for (long x = 0; x < V; ++x)
      for (int k = chib * h; k < chib * h + h; ++k) v[x * ns + k] = Pv[((long)ib * V + x) * ns + k];
    for (int d = 0; d <= 8; ++d) {
      if (d == 0) D.mdiag(v.data(), w.data());
      else D.mdir(d, v.data(), w.data());
#pragma omp parallel for
      for (long c = 0; c < Vc; ++c) {
        for (long o = 0; o < ag.A; ++o) {
          long x = ag.site_of[c * ag.A + o];
          int dd = d;
          if (d == 0 || ag.agg[ag.fine.neighbour(x, d)] == c) dd = 0;
          cd* m = &Dc.M[((c * 9 + dd) * nb) * nb];
          for (int a = 0; a < nb; ++a) {
            int ia = a % nv, chia = a / nv;
            cd s = 0.0;
            for (int k = chia * h; k < chia * h + h; ++k) s += std::conj(Pv[((long)ia * V + x) * ns + k]) * w[x * ns + k];
            m[a * nb + b] += s;
          }
        }
      }
    }
  }
  return 0;
}

// ----------------------------------------------------------------------------
// Krylov solvers (Sec. 2.1: MR, GMRES and flexible GMRES).
// ----------------------------------------------------------------------------
typedef std::function<void(const cd*, cd*)> LinOp;

// MinimalResidual: from x (initial guess) and r = b - A x, nu times
//   p = A r; alpha = <p,r>/<p,p>; x += alpha r; r -= alpha p.
void mr(const LinOp& A, long n, const cd* b, cd* x, int steps) {
  cvec r(n), p(n);
  A(x, p.data());
  for (long i = 0; i < n; ++i) r[i] = b[i] - p[i];
  for (int k = 0; k < steps; ++k) {
    A(r.data(), p.data());
    double pp = std::real(dot(n, p.data(), p.data()));
    if (pp == 0.0) break;
    cd alpha = dot(n, p.data(), r.data()) / pp;
    axpy(n, alpha, r.data(), x);
    axpy(n, -alpha, p.data(), r.data());
  }
}

// ----------------------------------------------------------------------------
// Even-odd (red-black) preconditioning.  The paper names red-black
// preconditioning as a feature the Grid implementation lacks and DDalphaAMG
// uses (Sec. 2.1, Sec. 4) without writing it down.  Reading: sites are even or
// odd by the parity of x+y+z+t; with A = (4 + m0) + C (site-diagonal) and the
// hopping terms H_eo, H_oe connecting the two parities,
//   D = [[A_ee, H_eo], [H_oe, A_oo]],   Dhat = A_oo - H_oe A_ee^{-1} H_eo,
// and D x = b becomes Dhat x_o = b_o - H_oe A_ee^{-1} b_e,
// x_e = A_ee^{-1} (b_e - H_eo x_o).  Fields keep their full length with the
// even part zero.
// ----------------------------------------------------------------------------
int site_parity(const Lattice& lat, long x) {
  int c[4];
  lat.coords(x, c);
  return (c[0] + c[1] + c[2] + c[3]) & 1;
}

// Inverse of a dense n x n complex matrix by Gauss-Jordan elimination with
// partial pivoting (rows); returns 1 when singular.
int invert_dense(int n, const cd* a, cd* inv) {
  std::vector<cd> m(a, a + n * n);
  for (int i = 0; i < n * n; ++i) inv[i] = 0.0;
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::abs(m[i * n + k]) > std::abs(m[piv * n + k])) piv = i;
    if (std::abs(m[piv * n + k]) == 0.0) return 1;
    for (int j = 0; j < n; ++j) {
      std::swap(m[k * n + j], m[piv * n + j]);
      std::swap(inv[k * n + j], inv[piv * n + j]);
    }
    const cd d = 1.0 / m[k * n + k];
    for (int j = 0; j < n; ++j) {
      m[k * n + j] *= d;
      inv[k * n + j] *= d;
    }
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const cd f = m[i * n + k];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        m[i * n + j] -= f * m[k * n + j];
        inv[i * n + j] -= f * inv[k * n + j];
      }
    }
  }
  return 0;
}

// A(x)^{-1} for every site, [V][12][12]: A = (4 + m0) + C is block diagonal in
// chirality (C commutes with gamma5), so each 6 x 6 block is inverted alone.
int clover_inverse(const WilsonClover& D, cvec& Ainv) {
  const long V = D.lat.V;
  Ainv.assign(V * 144, cd(0.0));
  int bad = 0;
#pragma omp parallel for reduction(| : bad)
  for (long x = 0; x < V; ++x) {
    for (int chi = 0; chi < 2; ++chi) {
      cd blk[36], inv[36];
      for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j)
          blk[i * 6 + j] = D.C[x * 144 + (chi * 6 + i) * 12 + chi * 6 + j] + (i == j ? cd(4.0 + D.m0) : cd(0.0));
      bad |= invert_dense(6, blk, inv);
      for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) Ainv[x * 144 + (chi * 6 + i) * 12 + chi * 6 + j] = inv[i * 6 + j];
    }
  }
  return bad;
}

// out = (parity of x == keep) ? M(x) in(x) : 0 for site matrices M [V][12][12].
void site_apply_masked(const WilsonClover& D, const cvec& M, int keep, const cd* in, cd* out) {
#pragma omp parallel for
  for (long x = 0; x < D.lat.V; ++x) {
    const bool on = site_parity(D.lat, x) == keep;
    for (int i = 0; i < 12; ++i) {
      cd s = 0.0;
      if (on)
        for (int j = 0; j < 12; ++j) s += M[x * 144 + i * 12 + j] * in[x * 12 + j];
      out[x * 12 + i] = s;
    }
  }
}

// out = the hopping part of D applied to in (all eight Mdir terms).
void hopping(const WilsonClover& D, const cd* in, cd* out) {
  std::fill(out, out + D.size(), cd(0.0));
  for (int d = 1; d <= 8; ++d) D.mdir_add(d, in, out);
}

// y = Dhat x on the odd sites (x: odd part used, even part ignored), y even = 0.
void schur_apply(const WilsonClover& D, const cvec& Ainv, const cd* x, cd* y) {
  const long n = D.size();
  cvec xo(n), t(n), u(n), w(n), ax(n);
  for (long s = 0; s < D.lat.V; ++s)
    for (int k = 0; k < 12; ++k) xo[s * 12 + k] = site_parity(D.lat, s) == 1 ? x[s * 12 + k] : cd(0.0);
  hopping(D, xo.data(), t.data());               // even sites: H_eo x_o
  site_apply_masked(D, Ainv, 0, t.data(), u.data());  // A_ee^{-1} H_eo x_o
  hopping(D, u.data(), w.data());                // odd sites: H_oe A_ee^{-1} H_eo x_o
  D.mdiag(xo.data(), ax.data());                 // A x_o
  for (long s = 0; s < D.lat.V; ++s)
    for (int k = 0; k < 12; ++k)
      y[s * 12 + k] = site_parity(D.lat, s) == 1 ? ax[s * 12 + k] - w[s * 12 + k] : cd(0.0);
}

// ----------------------------------------------------------------------------
// Schwarz alternating procedure (SAP).  The paper names SAP as the smoother
// DDalphaAMG normally uses and as a feature the Grid implementation does not
// have yet (Sec. 2.1, Sec. 4); it gives no definition.  Reading, the
// multiplicative Schwarz method on a red-black colouring of domains: the
// domains are the level-0 aggregates, coloured by the parity of their coarse
// coordinates (so every coarse extent must be even).  One SAP cycle visits
// colour 0 and then colour 1; for each colour it forms r = b - D x with the
// current x, and for every domain B of that colour solves D_B e = r_B by
// block_iters MR steps from e = 0 (D_B: D with every coupling that leaves B
// dropped, a Dirichlet boundary), then sets x_B += e.  Domains of one colour
// do not couple, so they are independent of each other.
// ----------------------------------------------------------------------------

// out = D_B v on domain c; v and out are indexed by in-block offset.
void block_apply(const WilsonClover& D, const Aggregation& ag, long c, const cd* v, cd* out) {
  for (long o = 0; o < ag.A; ++o) {
    const long x = ag.site_of[c * ag.A + o];
    const cd* cl = &D.C[x * 144];
    for (int i = 0; i < 12; ++i) {
      cd s = (4.0 + D.m0) * v[o * 12 + i];
      for (int j = 0; j < 12; ++j) s += cl[i * 12 + j] * v[o * 12 + j];
      out[o * 12 + i] = s;
    }
    for (int d = 1; d <= 8; ++d) {
      const long y = D.lat.neighbour(x, d);
      if (ag.agg[y] != c) continue;  // the coupling leaves the domain
      D.hop_add(x, d, &v[ag.off[y] * 12], &out[o * 12]);
    }
  }
}

// colours = 2: full cycles; colours = 1: the colour-0 half of one cycle.
int sap(const WilsonClover& D, const Aggregation& ag, const cd* b, cd* x, int cycles, int block_iters,
        int colours = 2) {
  for (int mu = 0; mu < 4; ++mu)
    if (ag.coarse.L[mu] % 2) return 2;
  const long V = D.lat.V, A = ag.A;
  cvec Dx(V * 12);
  for (int cyc = 0; cyc < cycles; ++cyc)
    for (int colour = 0; colour < colours; ++colour) {
      D.apply(x, Dx.data());
#pragma omp parallel for
      for (long c = 0; c < ag.coarse.V; ++c) {
        int cx[4];
        ag.coarse.coords(c, cx);
        if ((cx[0] + cx[1] + cx[2] + cx[3]) % 2 != colour) continue;
        cvec r(A * 12), e(A * 12, cd(0.0)), p(A * 12);
        for (long o = 0; o < A; ++o) {
          const long xs = ag.site_of[c * A + o];
          for (int k = 0; k < 12; ++k) r[o * 12 + k] = b[xs * 12 + k] - Dx[xs * 12 + k];
        }
        for (int it = 0; it < block_iters; ++it) {
          block_apply(D, ag, c, r.data(), p.data());
          const double pp = std::real(dot(A * 12, p.data(), p.data()));
          if (pp == 0.0) break;
          const cd alpha = dot(A * 12, p.data(), r.data()) / pp;
          axpy(A * 12, alpha, r.data(), e.data());
          axpy(A * 12, -alpha, p.data(), r.data());
        }
        for (long o = 0; o < A; ++o) {
          const long xs = ag.site_of[c * A + o];
          for (int k = 0; k < 12; ++k) x[xs * 12 + k] += e[o * 12 + k];
        }
      }
    }
  return 0;
}

struct KrylovResult {
  int iters = 0;
  double est = 0.0;
};

// Restarted (flexible) GMRES with modified Gram-Schmidt Arnoldi and Givens
// rotations.  With a preconditioner M the Krylov basis is stored preconditioned
// (z_j = M v_j) and x += Z y (flexible variant); without one, x += V y.
// fixed > 0: exactly that many iterations, no early exit.
// tol is relative to ||b||.  x holds the initial guess on entry.
KrylovResult gmres_core(const LinOp& A, const LinOp* M, long n, const cd* b, cd* x, int restart, int maxit,
                        double tol, int fixed, bool x0_zero) {
  KrylovResult res;
  const double bnorm = norm(n, b);
  if (bnorm == 0.0) {
    std::fill(x, x + n, cd(0.0));
    return res;
  }
  if (x0_zero) std::fill(x, x + n, cd(0.0));
  const int limit = fixed > 0 ? fixed : maxit;
  std::vector<cvec> Vb(restart + 1, cvec(n)), Zb;
  if (M) Zb.assign(restart, cvec(n));
  std::vector<cd> H((restart + 1) * restart), cs(restart), sn(restart), g(restart + 1);
  cvec w(n);
  while (res.iters < limit) {
    A(x, w.data());
    for (long i = 0; i < n; ++i) Vb[0][i] = b[i] - w[i];
    double beta = norm(n, Vb[0].data());
    res.est = beta / bnorm;
    if (fixed <= 0 && beta <= tol * bnorm) break;
    if (beta == 0.0) break;
    for (long i = 0; i < n; ++i) Vb[0][i] /= beta;
    std::fill(g.begin(), g.end(), cd(0.0));
    g[0] = beta;
    int j = 0;
    bool stop = false;
    for (; j < restart && res.iters < limit; ++j) {
      const cd* zj = Vb[j].data();
      if (M) {
        (*M)(Vb[j].data(), Zb[j].data());
        zj = Zb[j].data();
      }
      A(zj, w.data());
      for (int i = 0; i <= j; ++i) {
        H[i * restart + j] = dot(n, Vb[i].data(), w.data());
        axpy(n, -H[i * restart + j], Vb[i].data(), w.data());
      }
      double hn = norm(n, w.data());
      H[(j + 1) * restart + j] = hn;
      for (int i = 0; i < j; ++i) {  // previous rotations
        cd t = cs[i] * H[i * restart + j] + sn[i] * H[(i + 1) * restart + j];
        H[(i + 1) * restart + j] = -std::conj(sn[i]) * H[i * restart + j] + std::conj(cs[i]) * H[(i + 1) * restart + j];
        H[i * restart + j] = t;
      }
      cd hjj = H[j * restart + j];
      double den = std::sqrt(std::norm(hjj) + hn * hn);
      if (den == 0.0) {
        // A z_j lies in the span of the earlier basis vectors and the rotated
        // column vanishes: it adds nothing to the least-squares problem, whose
        // minimiser is that of the leading j x j system; the residual stays |g_j|
        res.iters++;
        res.est = std::abs(g[j]) / bnorm;
        stop = true;
        break;
      }
      cs[j] = hjj / den;
      sn[j] = hn / den;
      // rotation [c s; -conj(s) conj(c)] with c = h/den, s = hn/den maps (h, hn) to (|.|, 0)
      cs[j] = std::conj(cs[j]);
      H[j * restart + j] = cs[j] * hjj + sn[j] * hn;
      H[(j + 1) * restart + j] = 0.0;
      g[j + 1] = -std::conj(sn[j]) * g[j];
      g[j] = cs[j] * g[j];
      res.iters++;
      res.est = std::abs(g[j + 1]) / bnorm;
      if (hn != 0.0)
        for (long i = 0; i < n; ++i) Vb[j + 1][i] = w[i] / hn;
      if (fixed <= 0 && res.est <= tol) { ++j; stop = true; break; }
      if (hn == 0.0) { ++j; stop = true; break; }
    }
    // back substitution H y = g on the leading j x j triangle
    std::vector<cd> y(j);
    for (int i = j - 1; i >= 0; --i) {
      cd s = g[i];
      for (int k = i + 1; k < j; ++k) s -= H[i * restart + k] * y[k];
      y[i] = s / H[i * restart + i];
    }
    for (int i = 0; i < j; ++i) axpy(n, y[i], M ? Zb[i].data() : Vb[i].data(), x);
    if (stop) break;
  }
  return res;
}

// ----------------------------------------------------------------------------
// Multigrid hierarchy (Sec. 2.1: recursive solver, initial and iterative setup).
// ----------------------------------------------------------------------------
struct Params {
  int L[4];
  double m0, csw;
  int antiperiodic;
  int n_levels;
  int block[3][4];
  int nv[3];
  int relax_sweeps, refine_iters;
  int post_smooth;
  int coarse_restart, coarse_maxit, coarse_fixed_iters;
  double coarse_tol;
  int kcycle, kcycle_maxit;
  double kcycle_tol;
  int outer_restart, outer_maxit;
  double outer_tol;
  int smoother;         // 0: MR, 1: SAP on level 0 (post_smooth cycles)
  int sap_block_iters;  // MR steps per domain solve
};

struct Level {
  LevelOp* op = nullptr;  // operator at this level (not owned for level 0)
  Aggregation ag;         // this level -> next coarser level
  int nv = 0;
  cvec start, vecs, Pv;   // [nv][V][ns]
  CoarseOp* coarse = nullptr;  // owned; the operator of the next level
};

struct Hierarchy {
  Params p;
  WilsonClover fine;
  std::vector<Level> lv;  // lv[l] for l = 0..n_levels-2 (levels with a coarser level)
  std::string err;
  ~Hierarchy() {
    for (auto& l : lv) delete l.coarse;
  }
  const LevelOp& op(int l) const { return l == 0 ? (const LevelOp&)fine : (const LevelOp&)*lv[l - 1].coarse; }
};

void cycle(const Hierarchy& H, int l, const cd* r, cd* x);

// Coarse-grid correction solve at level l+1 (l+1 is the coarsest level):
// GMRES on D_{l+1} (Sec. 2.1 fixes the coarse solver to GMRES).
void coarse_solve(const Hierarchy& H, int lc, const cd* b, cd* x) {
  const LevelOp& D = H.op(lc);
  LinOp A = [&](const cd* i, cd* o) { D.apply(i, o); };
  gmres_core(A, nullptr, D.size(), b, x, H.p.coarse_restart, H.p.coarse_maxit, H.p.coarse_tol,
             H.p.coarse_fixed_iters, true);
}

// One application of the MG preconditioner rooted at level l (V-cycle or
// K-cycle), zero initial guess, no pre-smoothing, post_smooth MR steps.
void cycle(const Hierarchy& H, int l, const cd* r, cd* x) {
  const Level& L = H.lv[l];
  const LevelOp& D = H.op(l);
  const LevelOp& Dc = H.op(l + 1);
  cvec rc(Dc.size()), ec(Dc.size());
  restrict_vec(L.ag, D.ns, L.nv, L.Pv, r, rc.data());
  const int nlev = H.p.n_levels;
  if (l + 2 >= nlev) {
    coarse_solve(H, l + 1, rc.data(), ec.data());
  } else if (H.p.kcycle) {
    LinOp A = [&](const cd* i, cd* o) { Dc.apply(i, o); };
    LinOp M = [&](const cd* i, cd* o) { cycle(H, l + 1, i, o); };
    gmres_core(A, &M, Dc.size(), rc.data(), ec.data(), H.p.kcycle_maxit, H.p.kcycle_maxit, H.p.kcycle_tol, 0, true);
  } else {
    cycle(H, l + 1, rc.data(), ec.data());
  }
  prolong_vec(L.ag, D.ns, L.nv, L.Pv, ec.data(), x);
  if (l == 0 && H.p.smoother == 1) {
    sap(H.fine, L.ag, r, x, H.p.post_smooth, H.p.sap_block_iters);
    return;
  }
  LinOp A = [&](const cd* i, cd* o) { D.apply(i, o); };
  mr(A, D.size(), r, x, H.p.post_smooth);
}

// Initial setup at level l (Sec. 2.1): iterate a smoother on random vectors.
// Reading: relax_sweeps MR steps on D x = 0 from each start vector, then
// normalise; build P and the coarse operator.
int initial_setup(Hierarchy& H, int l);

int rebuild(Hierarchy& H, int l) {
  Level& L = H.lv[l];
  const LevelOp& D = H.op(l);
  int st = build_prolongator(L.ag, D.ns, L.nv, L.vecs, L.Pv);
  if (st) { H.err = "Gram-Schmidt breakdown"; return st; }
  if (!L.coarse) L.coarse = new CoarseOp();
  st = galerkin(D, L.ag, L.nv, L.Pv, *L.coarse);
  if (st) { H.err = "coarse lattice extent below 2"; return st; }
  return 0;
}

int initial_setup(Hierarchy& H, int l) {
  Level& L = H.lv[l];
  const LevelOp& D = H.op(l);
  const long n = D.size();
  if ((long)L.start.size() != (long)L.nv * n) { H.err = "start vectors not set"; return 4; }
  L.vecs = L.start;
  std::vector<cd> zero(n, 0.0);
  LinOp A = [&](const cd* i, cd* o) { D.apply(i, o); };
  for (int i = 0; i < L.nv; ++i) {
    cd* x = &L.vecs[(long)i * n];
    mr(A, n, zero.data(), x, H.p.relax_sweeps);
    double nx = norm(n, x);
    for (long k = 0; k < n; ++k) x[k] /= nx;
  }
  return rebuild(H, l);
}

// Re-take the Galerkin products below level l with the existing prolongators
// (down to the first level whose prolongator has not been built yet).
int regalerkin_below(Hierarchy& H, int l) {
  for (int k = l + 1; k < (int)H.lv.size(); ++k) {
    if (!H.lv[k].coarse || H.lv[k].Pv.empty()) break;
    int st = galerkin(H.op(k), H.lv[k].ag, H.lv[k].nv, H.lv[k].Pv, *H.lv[k].coarse);
    if (st) return st;
  }
  return 0;
}

// Iterative (DDalphaAMG-style) setup (Sec. 2.1).  Reading: one iteration at
// level l replaces each vector by the current preconditioner applied to it
// (zero initial guess), normalises it, rebuilds P_l and D_{l+1}, re-takes the
// Galerkin products below, then does the same one level down.
int refine_iteration(Hierarchy& H, int l) {
  Level& L = H.lv[l];
  const LevelOp& D = H.op(l);
  const long n = D.size();
  cvec y(n);
  for (int i = 0; i < L.nv; ++i) {
    cd* v = &L.vecs[(long)i * n];
    cycle(H, l, v, y.data());
    double ny = norm(n, y.data());
    for (long k = 0; k < n; ++k) v[k] = y[k] / ny;
  }
  int st = rebuild(H, l);
  if (st) return st;
  st = regalerkin_below(H, l);
  if (st) return st;
  if (l + 1 < (int)H.lv.size()) return refine_iteration(H, l + 1);
  return 0;
}

}  // namespace

// ============================================================================
// C API (ctypes).  Complex arrays are interleaved (re, im) doubles.
// ============================================================================
extern "C" {

typedef Params or_params;

int or_abi_version() { return 1; }

int or_num_threads() {
#ifdef _OPENMP
  int n = 1;
#pragma omp parallel
  {
#pragma omp single
    n = omp_get_num_threads();
  }
  return n;
#else
  return 1;
#endif
}

void or_gamma(double* g /*[4][4][4]*/, double* g5 /*[4][4]*/) {
  const Gammas& G = gammas();
  std::memcpy(g, G.g, sizeof(G.g));
  std::memcpy(g5, G.g5, sizeof(G.g5));
}

// Clover term C(x) as full 12x12 matrices [V][12][12].
void or_clover(const int* L, const double* U, double csw, double* C) {
  Lattice lat(L);
  build_clover(lat, (const cd*)U, csw, (cd*)C);
}

// Aggregation map: coarse[i], offset[i] per fine site, site_of[c*A+o].
int or_agg_map(const int* L, const int* block, int32_t* coarse, int32_t* offset, int32_t* site_of) {
  Aggregation ag;
  Lattice lat(L);
  int st = make_aggregation(lat, block, ag);
  if (st) return st;
  for (long i = 0; i < lat.V; ++i) { coarse[i] = (int32_t)ag.agg[i]; offset[i] = (int32_t)ag.off[i]; }
  if (site_of)
    for (long k = 0; k < (long)ag.site_of.size(); ++k) site_of[k] = (int32_t)ag.site_of[k];
  return 0;
}

// Coarse apply with caller-given blocks [Vc][9][nb][nb]: out = D_c in, nrhs fields.
void or_coarse_apply(const int* Lc, int nb, const double* M, const double* in, double* out, int nrhs) {
  CoarseOp op;
  op.lat = Lattice(Lc);
  op.ns = nb;
  op.M.assign((const cd*)M, (const cd*)M + op.lat.V * 9 * nb * nb);
  for (int r = 0; r < nrhs; ++r) op.apply((const cd*)in + r * op.size(), (cd*)out + r * op.size());
}

// Wilson-clover apply with caller-given links and clover matrices [V][12][12].
void or_wilson_apply(const int* L, double m0, int antiperiodic, const double* U, const double* C, const double* in,
                     double* out, int nrhs) {
  WilsonClover D;
  D.lat = Lattice(L);
  D.ns = 12;
  D.m0 = m0;
  D.antiperiodic = antiperiodic != 0;
  D.U.assign((const cd*)U, (const cd*)U + D.lat.V * 36);
  D.C.assign((const cd*)C, (const cd*)C + D.lat.V * 144);
  for (int r = 0; r < nrhs; ++r) D.apply((const cd*)in + r * D.size(), (cd*)out + r * D.size());
}

// One Mdir (d = 1..8) or Mdiag (d = 0) of the Wilson-clover operator.
void or_wilson_term(const int* L, double m0, int antiperiodic, const double* U, const double* C, int d,
                    const double* in, double* out) {
  WilsonClover D;
  D.lat = Lattice(L);
  D.ns = 12;
  D.m0 = m0;
  D.antiperiodic = antiperiodic != 0;
  D.U.assign((const cd*)U, (const cd*)U + D.lat.V * 36);
  D.C.assign((const cd*)C, (const cd*)C + D.lat.V * 144);
  if (d == 0) D.mdiag((const cd*)in, (cd*)out);
  else D.mdir(d, (const cd*)in, (cd*)out);
}

// Per-aggregate, per-chirality orthonormalisation of nv vectors [nv][V][ns].
int or_orthonormalise(const int* L, const int* block, int ns, int nv, const double* vecs, double* Pv) {
  Aggregation ag;
  int st = make_aggregation(Lattice(L), block, ag);
  if (st) return st;
  cvec in((const cd*)vecs, (const cd*)vecs + (long)nv * ag.fine.V * ns), out;
  st = build_prolongator(ag, ns, nv, in, out);
  std::memcpy(Pv, out.data(), out.size() * sizeof(cd));
  return st;
}

void or_restrict(const int* L, const int* block, int ns, int nv, const double* Pv, const double* fine, double* coarse,
                 int nrhs) {
  Aggregation ag;
  make_aggregation(Lattice(L), block, ag);
  cvec P((const cd*)Pv, (const cd*)Pv + (long)nv * ag.fine.V * ns);
  for (int r = 0; r < nrhs; ++r)
    restrict_vec(ag, ns, nv, P, (const cd*)fine + (long)r * ag.fine.V * ns, (cd*)coarse + (long)r * ag.coarse.V * 2 * nv);
}

void or_prolong(const int* L, const int* block, int ns, int nv, const double* Pv, const double* coarse, double* fine,
                int nrhs) {
  Aggregation ag;
  make_aggregation(Lattice(L), block, ag);
  cvec P((const cd*)Pv, (const cd*)Pv + (long)nv * ag.fine.V * ns);
  for (int r = 0; r < nrhs; ++r)
    prolong_vec(ag, ns, nv, P, (const cd*)coarse + (long)r * ag.coarse.V * 2 * nv, (cd*)fine + (long)r * ag.fine.V * ns);
}

// Restarted GMRES on a caller-given coarse operator (x0 = 0).
int or_coarse_gmres(const int* Lc, int nb, const double* M, const double* b, double* x, int restart, int maxit,
                    double tol, int fixed, double* est) {
  CoarseOp op;
  op.lat = Lattice(Lc);
  op.ns = nb;
  op.M.assign((const cd*)M, (const cd*)M + op.lat.V * 9 * nb * nb);
  LinOp A = [&](const cd* i, cd* o) { op.apply(i, o); };
  KrylovResult r = gmres_core(A, nullptr, op.size(), (const cd*)b, (cd*)x, restart, maxit, tol, fixed, true);
  if (est) *est = r.est;
  return r.iters;
}

// MR steps on a caller-given coarse operator: x holds x0 on entry.
// SAP on the fine operator with the aggregates of `block` as domains; x holds
// the initial guess.  Returns 2 when a coarse extent is odd.
int or_sap(const int* L, const int* block, double m0, int antiperiodic, const double* U, const double* C,
           const double* b, double* x, int cycles, int block_iters, int colours) {
  WilsonClover D;
  D.lat = Lattice(L);
  D.ns = 12;
  D.m0 = m0;
  D.antiperiodic = antiperiodic != 0;
  D.U.assign((const cd*)U, (const cd*)U + D.lat.V * 36);
  D.C.assign((const cd*)C, (const cd*)C + D.lat.V * 144);
  Aggregation ag;
  if (make_aggregation(D.lat, block, ag)) return 2;
  return sap(D, ag, (const cd*)b, (cd*)x, cycles, block_iters, colours);
}

void or_coarse_mr(const int* Lc, int nb, const double* M, const double* b, double* x, int steps) {
  CoarseOp op;
  op.lat = Lattice(Lc);
  op.ns = nb;
  op.M.assign((const cd*)M, (const cd*)M + op.lat.V * 9 * nb * nb);
  LinOp A = [&](const cd* i, cd* o) { op.apply(i, o); };
  mr(A, op.size(), (const cd*)b, (cd*)x, steps);
}

// ---- hierarchy ----
void* or_mg_create(const or_params* p, const double* U, const double* C /* [V][12][12] or NULL */) {
  Hierarchy* H = new Hierarchy();
  H->p = *p;
  H->fine.lat = Lattice(p->L);
  H->fine.ns = 12;
  H->fine.m0 = p->m0;
  H->fine.antiperiodic = p->antiperiodic != 0;
  H->fine.U.assign((const cd*)U, (const cd*)U + H->fine.lat.V * 36);
  H->fine.C.assign(H->fine.lat.V * 144, cd(0.0));
  if (C) H->fine.C.assign((const cd*)C, (const cd*)C + H->fine.lat.V * 144);
  else build_clover(H->fine.lat, H->fine.U.data(), p->csw, H->fine.C.data());
  H->lv.resize(std::max(0, p->n_levels - 1));
  Lattice lat = H->fine.lat;
  for (int l = 0; l + 1 < p->n_levels; ++l) {
    if (make_aggregation(lat, p->block[l], H->lv[l].ag)) { delete H; return nullptr; }
    H->lv[l].nv = p->nv[l];
    lat = H->lv[l].ag.coarse;
  }
  if (p->smoother == 1 && !H->lv.empty())
    for (int mu = 0; mu < 4; ++mu)
      if (H->lv[0].ag.coarse.L[mu] % 2) { delete H; return nullptr; }  // SAP needs two colours
  return H;
}

void or_mg_destroy(void* h) { delete (Hierarchy*)h; }

const char* or_mg_error(void* h) { return ((Hierarchy*)h)->err.c_str(); }

long or_mg_size(void* h, int l) {
  Hierarchy* H = (Hierarchy*)h;
  if (l == 0) return H->fine.size();
  if (l - 1 < (int)H->lv.size()) {
    const Aggregation& ag = H->lv[l - 1].ag;
    return ag.coarse.V * 2 * H->lv[l - 1].nv;
  }
  return -1;
}

void or_mg_set_start(void* h, int l, const double* v) {
  Hierarchy* H = (Hierarchy*)h;
  long n = or_mg_size(h, l);
  H->lv[l].start.assign((const cd*)v, (const cd*)v + (long)H->lv[l].nv * n);
}

// Initial setup of every level from the start vectors.
int or_mg_setup(void* h) {
  Hierarchy* H = (Hierarchy*)h;
  for (int l = 0; l < (int)H->lv.size(); ++l) {
    int st = initial_setup(*H, l);
    if (st) return st;
  }
  return 0;
}

int or_mg_refine(void* h, int iters) {
  Hierarchy* H = (Hierarchy*)h;
  for (int it = 0; it < iters; ++it) {
    int st = refine_iteration(*H, 0);
    if (st) return st;
  }
  return 0;
}

// Replace the (un-orthonormalised) near-null vectors of level l and rebuild
// P_l and D_{l+1}; deeper Galerkin products are re-taken.
int or_mg_set_vectors(void* h, int l, const double* v) {
  Hierarchy* H = (Hierarchy*)h;
  if (l < 0 || l >= (int)H->lv.size() || (l > 0 && !H->lv[l - 1].coarse)) {
    H->err = "level operator not built";
    return 3;
  }
  long n = or_mg_size(h, l);
  H->lv[l].vecs.assign((const cd*)v, (const cd*)v + (long)H->lv[l].nv * n);
  int st = rebuild(*H, l);
  if (st) return st;
  return regalerkin_below(*H, l);
}

void or_mg_get_vectors(void* h, int l, double* v) {
  Hierarchy* H = (Hierarchy*)h;
  std::memcpy(v, H->lv[l].vecs.data(), H->lv[l].vecs.size() * sizeof(cd));
}
void or_mg_get_P(void* h, int l, double* v) {
  Hierarchy* H = (Hierarchy*)h;
  std::memcpy(v, H->lv[l].Pv.data(), H->lv[l].Pv.size() * sizeof(cd));
}
void or_mg_get_coarse(void* h, int l, double* M) {
  Hierarchy* H = (Hierarchy*)h;
  const CoarseOp& c = *H->lv[l - 1].coarse;
  std::memcpy(M, c.M.data(), c.M.size() * sizeof(cd));
}
void or_mg_get_clover(void* h, double* C) {
  Hierarchy* H = (Hierarchy*)h;
  std::memcpy(C, H->fine.C.data(), H->fine.C.size() * sizeof(cd));
}

void or_mg_apply(void* h, int l, const double* in, double* out) {
  Hierarchy* H = (Hierarchy*)h;
  H->op(l).apply((const cd*)in, (cd*)out);
}

void or_mg_cycle(void* h, int l, const double* r, double* x) {
  Hierarchy* H = (Hierarchy*)h;
  cycle(*H, l, (const cd*)r, (cd*)x);
}

// x = Dhat x_o for the fine operator of a field [V][12] (even part ignored).
int or_schur_apply(const int* L, double m0, int antiperiodic, const double* U, const double* C, const double* in,
                   double* out) {
  WilsonClover D;
  D.lat = Lattice(L);
  D.ns = 12;
  D.m0 = m0;
  D.antiperiodic = antiperiodic != 0;
  D.U.assign((const cd*)U, (const cd*)U + D.lat.V * 36);
  D.C.assign((const cd*)C, (const cd*)C + D.lat.V * 144);
  cvec Ainv;
  if (clover_inverse(D, Ainv)) return 1;
  schur_apply(D, Ainv, (const cd*)in, (cd*)out);
  return 0;
}

// A(x)^{-1} per site, [V][12][12].
int or_clover_inverse(const int* L, double m0, const double* C, double* out) {
  WilsonClover D;
  D.lat = Lattice(L);
  D.ns = 12;
  D.m0 = m0;
  D.C.assign((const cd*)C, (const cd*)C + D.lat.V * 144);
  cvec Ainv;
  const int st = clover_inverse(D, Ainv);
  std::copy(Ainv.begin(), Ainv.end(), (cd*)out);
  return st;
}

// Even-odd preconditioned outer solve: FGMRES(outer_restart) on Dhat with the
// MG cycle embedded as its preconditioner (Mhat r_o = odd part of
// M (0_e, r_o), since the odd part of D^{-1} (0_e, r_o) is Dhat^{-1} r_o),
// converged when |bhat - Dhat x_o| <= outer_tol |b|, which is the full true
// residual once x_e is reconstructed.  x holds the initial guess (its odd part
// is used).
int or_mg_solve_eo(void* h, const double* b, double* x, int* iters, double* relres) {
  Hierarchy* H = (Hierarchy*)h;
  const WilsonClover& D = H->fine;
  const long n = D.size(), V = D.lat.V;
  cvec Ainv;
  if (clover_inverse(D, Ainv)) return 1;
  const cd* bb = (const cd*)b;
  cd* xx = (cd*)x;
  auto mask_odd = [&](cd* v) {
    for (long s = 0; s < V; ++s)
      if (site_parity(D.lat, s) == 0)
        for (int k = 0; k < 12; ++k) v[s * 12 + k] = 0.0;
  };
  // bhat = b_o - H_oe A_ee^{-1} b_e
  cvec t(n), w(n), bh(n), xo(xx, xx + n);
  site_apply_masked(D, Ainv, 0, bb, t.data());
  hopping(D, t.data(), w.data());
  for (long i = 0; i < n; ++i) bh[i] = bb[i] - w[i];
  mask_odd(bh.data());
  mask_odd(xo.data());
  LinOp A = [&](const cd* i, cd* o) { schur_apply(D, Ainv, i, o); };
  LinOp M = [&](const cd* i, cd* o) {
    cvec in(i, i + n);
    mask_odd(in.data());
    if (H->lv.empty()) std::copy(in.begin(), in.end(), o);
    else cycle(*H, 0, in.data(), o);
    mask_odd(o);
  };
  const double bn = norm(n, bb), bhn = norm(n, bh.data());
  int total = 0;
  double rel = 0.0;
  cvec r(n);
  for (;;) {
    schur_apply(D, Ainv, xo.data(), r.data());
    for (long i = 0; i < n; ++i) r[i] = bh[i] - r[i];
    rel = bn > 0 ? norm(n, r.data()) / bn : 0.0;
    if (rel <= H->p.outer_tol || total >= H->p.outer_maxit) break;
    const int budget = H->p.outer_maxit - total;
    KrylovResult kr = gmres_core(A, &M, n, bh.data(), xo.data(), H->p.outer_restart,
                                 std::min(budget, H->p.outer_restart), H->p.outer_tol * bn / bhn, 0, false);
    total += kr.iters;
    if (kr.iters == 0) break;
  }
  // x_e = A_ee^{-1} (b_e - H_eo x_o)
  hopping(D, xo.data(), t.data());
  for (long i = 0; i < n; ++i) w[i] = bb[i] - t[i];
  site_apply_masked(D, Ainv, 0, w.data(), t.data());
  for (long i = 0; i < n; ++i) xx[i] = xo[i] + t[i];
  // the full true residual
  D.apply(xx, r.data());
  for (long i = 0; i < n; ++i) r[i] = bb[i] - r[i];
  rel = bn > 0 ? norm(n, r.data()) / bn : 0.0;
  if (iters) *iters = total;
  if (relres) *relres = rel;
  return rel <= H->p.outer_tol ? 0 : 7;
}

// Outer solve (Sec. 2.1): flexible GMRES(outer_restart) on D, preconditioned by
// the MG cycle.  Convergence is declared on the true residual b - D x,
// recomputed at each restart and at exit.  x holds the initial guess.
int or_mg_solve(void* h, const double* b, double* x, int* iters, double* relres) {
  Hierarchy* H = (Hierarchy*)h;
  const LevelOp& D = H->op(0);
  const long n = D.size();
  LinOp A = [&](const cd* i, cd* o) { D.apply(i, o); };
  LinOp M = [&](const cd* i, cd* o) {
    if (H->lv.empty()) std::memcpy(o, i, n * sizeof(cd));
    else cycle(*H, 0, i, o);
  };
  const cd* bb = (const cd*)b;
  cd* xx = (cd*)x;
  const double bn = norm(n, bb);
  int total = 0;
  double rel = 0.0;
  cvec r(n);
  for (;;) {
    D.apply(xx, r.data());
    for (long i = 0; i < n; ++i) r[i] = bb[i] - r[i];
    rel = norm(n, r.data()) / bn;
    if (rel <= H->p.outer_tol || total >= H->p.outer_maxit) break;
    int budget = H->p.outer_maxit - total;
    // one restart cycle; tolerance relative to ||b||, expressed for this residual
    KrylovResult kr = gmres_core(A, &M, n, bb, xx, H->p.outer_restart, std::min(budget, H->p.outer_restart),
                                 H->p.outer_tol, 0, false);
    total += kr.iters;
    if (kr.iters == 0) break;
  }
  if (iters) *iters = total;
  if (relres) *relres = rel;
  return rel <= H->p.outer_tol ? 0 : 7;
}

}  // extern "C"
