// Host side of the learned near-null proposal: network state (weights, Adam
// moments, activations), forward, loss and backward passes over a context's
// lattice, training step, and the learned setup with its fallback to the
// plain setup.
#include <chrono>
#include <cmath>

#include "engine.h"

namespace wcmg {

namespace {
// splitmix64 (Steele, Lea, Flood 2014) and Box-Muller for the initial weights
struct SplitMix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {
    const double u = uniform(), v = uniform();
    return std::sqrt(-2.0 * std::log(u)) * std::cos(6.283185307179586 * v);
  }
};
}  // namespace

Net::Net(int nv_, int ch_, int act_bits_, uint64_t seed, hipStream_t st) : nv(nv_), ch(ch_), act_bits(act_bits_), stream(st) {
  require(nv >= 4 && nv <= 16 && nv % 4 == 0, WCMG_ERR_ARG, "network: n_vec must be 4, 8, 12 or 16");
  require(ch >= 4 && ch <= 32 && ch % 4 == 0, WCMG_ERR_ARG, "network: channels must be a multiple of 4 up to 32");
  require(act_bits == 16 || act_bits == 32, WCMG_ERR_ARG, "network: activations BF16 or FP32");
  cin[0] = nv;
  cout[0] = ch;
  cin[1] = ch;
  cout[1] = ch;
  cin[2] = ch;
  cout[2] = nv;
  SplitMix rng{seed};
  std::vector<float> host;
  for (int l = 0; l < 3; ++l) {
    const long n = 9L * cout[l] * cin[l];
    const double sc = 0.1 / std::sqrt((double)cin[l]);
    for (long e = 0; e < n; ++e) {
      const long r = e % ((long)cout[l] * cin[l]);
      const int o = (int)(r / cin[l]), i = (int)(r % cin[l]);
      double re = sc * rng.normal(), im = sc * rng.normal();
      if (e < (long)cout[l] * cin[l] && o == i) re += 1.0;  // self hop starts near the identity
      host.push_back((float)re);
      host.push_back((float)im);
    }
    W[l].alloc(n * sizeof(cf32));
    Wadj[l].alloc(n * sizeof(cf32));
    gW[l].alloc(n * sizeof(cf32));
    m[l].alloc(2 * n * sizeof(float));
    v[l].alloc(2 * n * sizeof(float));
    WCMG_HIP(hipMemsetAsync(m[l].p, 0, m[l].bytes, stream));
    WCMG_HIP(hipMemsetAsync(v[l].p, 0, v[l].bytes, stream));
  }
  set_weights(host.data());
}

long Net::n_complex(int l) const { return 9L * cout[l] * cin[l]; }
long Net::n_floats() const { return 2 * (n_complex(0) + n_complex(1) + n_complex(2)); }

void Net::set_weights(const float* host) {
  long off = 0;
  for (int l = 0; l < 3; ++l) {
    WCMG_HIP(hipMemcpyAsync(W[l].p, host + off, n_complex(l) * sizeof(cf32), hipMemcpyHostToDevice, stream));
    launch_nn_adjoint_weights(W[l].as<cf32>(), cout[l], cin[l], Wadj[l].as<cf32>(), stream);
    off += 2 * n_complex(l);
  }
  WCMG_HIP(hipStreamSynchronize(stream));
}

void Net::get_weights(float* host) {
  long off = 0;
  for (int l = 0; l < 3; ++l) {
    WCMG_HIP(hipMemcpyAsync(host + off, W[l].p, n_complex(l) * sizeof(cf32), hipMemcpyDeviceToHost, stream));
    off += 2 * n_complex(l);
  }
  WCMG_HIP(hipStreamSynchronize(stream));
}

void Net::get_grads(float* host) {
  long off = 0;
  std::vector<cf32> tmp;
  for (int l = 0; l < 3; ++l) {
    tmp.resize(n_complex(l));
    WCMG_HIP(hipMemcpyAsync(tmp.data(), gW[l].p, n_complex(l) * sizeof(cf32), hipMemcpyDeviceToHost, stream));
    WCMG_HIP(hipStreamSynchronize(stream));
    for (long e = 0; e < n_complex(l); ++e) {  // real-parameter gradient: dL/dRe = 2 Re g, dL/dIm = 2 Im g
      host[off + 2 * e] = 2.f * tmp[e].re;
      host[off + 2 * e + 1] = 2.f * tmp[e].im;
    }
    off += 2 * n_complex(l);
  }
}

void Net::ensure(long V_) {
  if (V == V_) return;
  V = V_;
  const size_t ab = act_bits == 16 ? 4 : 8;
  act[0].alloc((size_t)nv * 12 * V * ab);
  act[1].alloc((size_t)ch * 12 * V * ab);
  act[2].alloc((size_t)ch * 12 * V * ab);
  act[3].alloc((size_t)nv * 12 * V * sizeof(cf32));
  scale[0].alloc((size_t)ch * V * sizeof(float));
  scale[1].alloc((size_t)ch * V * sizeof(float));
  const int cmax = std::max(nv, ch);
  g0.alloc((size_t)cmax * 12 * V * sizeof(cf32));
  g1.alloc((size_t)cmax * 12 * V * sizeof(cf32));
  tgt.alloc((size_t)nv * 12 * V * sizeof(cf32));
  part.alloc((size_t)9 * nn_wgrad_blocks(V) * 32 * 32 * sizeof(cd64));
}

void Net::forward(Context& c) {
  require(c.nlev >= 2 && c.tr[0].has_start, WCMG_ERR_STATE, "network: context needs start vectors of level 0");
  require(c.tr[0].nv == nv, WCMG_ERR_ARG, "network: n_vec differs from the context's");
  require(c.gauge_set, WCMG_ERR_STATE, "network: gauge field not set");
  const long Vn = c.geo[0].V;
  ensure(Vn);
  const cf32* U = c.U32.as<cf32>();
  const int* nbr = c.geo[0].nbr.as<int>();
  launch_nn_from64(c.tr[0].start64.as<cd64>(), act_bits, act[0].p, (long)nv * 12 * V, c.stream);
  c.prof.begin("nn_forward", c.stream);
  launch_nn_layer(act_bits, act[0].p, nv, W[0].as<cf32>(), ch, act_bits, act[1].p, scale[0].as<float>(), 1, U, nbr, V,
                  c.stream);
  launch_nn_layer(act_bits, act[1].p, ch, W[1].as<cf32>(), ch, act_bits, act[2].p, scale[1].as<float>(), 1, U, nbr, V,
                  c.stream);
  launch_nn_layer(act_bits, act[2].p, ch, W[2].as<cf32>(), nv, 32, act[3].p, nullptr, 0, U, nbr, V, c.stream);
  c.prof.end("nn_forward", c.stream);
}

double Net::loss_grad(Context& c) {
  require(c.tr[0].built, WCMG_ERR_STATE, "network: context has no near-null vectors (run the setup)");
  forward(c);
  const long n = (long)nv * 12 * V;
  const cd64* vt = c.tr[0].vecs64.as<cd64>();
  launch_nn_from64(vt, 32, tgt.p, n, c.stream);
  const double norm = c.norm2_host<double>(vt, n);
  const Transfer& T = c.tr[0];
  std::vector<double> lp(2 * T.Vc);
  DevBuf lpart;
  lpart.alloc(lp.size() * sizeof(double));
  const cf32* U = c.U32.as<cf32>();
  const int* nbr = c.geo[0].nbr.as<int>();
  cf32* ga = g0.as<cf32>();
  cf32* gb = g1.as<cf32>();
  launch_nn_loss(act[3].as<cf32>(), tgt.as<cf32>(), nv, T.agg_sites.as<int>(), T.A, T.Vc, V, norm, ga,
                 lpart.as<double>(), c.stream);
  c.prof.begin("nn_backward", c.stream);
  // layer 2 (linear): weight gradient, then the gradient of its input
  launch_nn_wgrad(ga, nv, act_bits, act[2].p, ch, U, nbr, V, part.as<cd64>(), gW[2].as<cf32>(), c.stream);
  launch_nn_layer(32, ga, nv, Wadj[2].as<cf32>(), ch, 32, gb, nullptr, 0, U, nbr, V, c.stream);
  launch_nn_squash_bwd(gb, act_bits, act[2].p, scale[1].as<float>(), ch, V, c.stream);
  // layer 1
  launch_nn_wgrad(gb, ch, act_bits, act[1].p, ch, U, nbr, V, part.as<cd64>(), gW[1].as<cf32>(), c.stream);
  launch_nn_layer(32, gb, ch, Wadj[1].as<cf32>(), ch, 32, ga, nullptr, 0, U, nbr, V, c.stream);
  launch_nn_squash_bwd(ga, act_bits, act[1].p, scale[0].as<float>(), ch, V, c.stream);
  // layer 0
  launch_nn_wgrad(ga, ch, act_bits, act[0].p, nv, U, nbr, V, part.as<cd64>(), gW[0].as<cf32>(), c.stream);
  c.prof.end("nn_backward", c.stream);
  WCMG_HIP(hipMemcpyAsync(lp.data(), lpart.p, lp.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
  WCMG_HIP(hipStreamSynchronize(c.stream));
  double loss = 0.0;
  for (double x : lp) loss += x;
  last_loss = loss / norm;
  return last_loss;
}

void Net::adam(float lr, hipStream_t st) {
  ++step;
  for (int l = 0; l < 3; ++l) {
    launch_nn_adam((float*)W[l].p, gW[l].as<cf32>(), m[l].as<float>(), v[l].as<float>(), n_complex(l), lr, step, st);
    launch_nn_adjoint_weights(W[l].as<cf32>(), cout[l], cin[l], Wadj[l].as<cf32>(), st);
  }
}

// Learned setup: the network maps the start vectors of level 0 to proposed
// near-null vectors, which relax_sweeps MR steps on D x = 0 then smooth (0:
// used as proposed); P and the coarse operator are built from them, deeper
// levels are set up as usual, then refine_iters refinement iterations run.
// Quality check: q = max_i |D y_i| / |y_i| over the proposals; when q is not
// finite or exceeds the threshold (or Gram-Schmidt breaks down) the plain
// setup runs instead.
void Context::setup_learned(Net& net, double threshold, int relax_sweeps, int* fell_back, double* quality) {
  require(gauge_set, WCMG_ERR_STATE, "gauge field not set");
  require(nlev >= 2, WCMG_ERR_STATE, "learned setup needs at least two levels");
  auto t0 = std::chrono::steady_clock::now();
  for (int q = 0; q < 5; ++q) timers[q] = 0.0;
  Transfer& T = tr[0];
  const long nn = n(0);
  net.forward(*this);
  launch_nn_to64(net.act[3].as<cf32>(), T.vecs64.as<cd64>(), T.nv * nn, stream);
  cd64* tmp = buf<cd64>("learn_tmp", nn);
  double q = 0.0;
  for (int i = 0; i < T.nv; ++i) {
    cd64* y = T.vecs64.as<cd64>() + (long)i * nn;
    const double yy = norm2_host<double>(y, nn);
    apply_op<double>(0, y, tmp, 1, nullptr);
    const double dd = norm2_host<double>(tmp, nn);
    const double r = (yy > 0.0) ? std::sqrt(dd / yy) : INFINITY;
    q = (r == r) ? std::max(q, r) : INFINITY;
    if (yy > 0.0 && yy == yy) {
      cd64* nrm = scratch64.as<cd64>() + 24;
      launch_dot<double>(y, 0, 1, nullptr, y, nn, partial.as<cd64>(), 1, nrm, 1, 0, nullptr, stream);
      launch_scale_inv_norm<double>(y, y, nrm, nn, nullptr, stream);
    }
  }
  *quality = q;
  *fell_back = 0;
  bool ok = q <= threshold;
  if (ok) {
    try {
      relax_vectors(0, relax_sweeps);
      rebuild(0);
    } catch (const Error& e) {
      if (e.code != WCMG_ERR_BREAKDOWN) throw;
      ok = false;
    }
  }
  if (!ok) {
    *fell_back = 1;
    setup_all();
    return;
  }
  for (int l = 1; l + 1 < nlev; ++l) initial_setup(l);
  auto t1 = std::chrono::steady_clock::now();
  for (int it = 0; it < p.refine_iters; ++it) refine_iteration(0);
  sync();
  auto t2 = std::chrono::steady_clock::now();
  timers[4] = std::chrono::duration<double>(t2 - t1).count();
  timers[0] = std::chrono::duration<double>(t2 - t0).count();
  setup_done = true;
}

}  // namespace wcmg
