// Launcher declarations of the wcmg HIP kernels.
#pragma once

#include <hip/hip_ext.h>

#include "common.h"

namespace wcmg {

template <int P>
struct BlkTraits;

// ---- fine level (wilson.hip)
void launch_clover_build(const cd64* U, const int L[4], double csw, cd64* out, hipStream_t st);
template <typename R>
void launch_pack_clover(const cd64* blocks, const int* perm, long V, double m0, R* out, hipStream_t st);
template <typename R>
void launch_pack_links(const cd64* U, const int* perm, const int L[4], int antiperiodic, cplx<R>* out, hipStream_t st);
template <typename Ti, typename To>
void launch_pack_fermion(const cplx<Ti>* in, const int* perm, long V, int nrhs, cplx<To>* out, hipStream_t st);
template <typename Ti, typename To>
void launch_unpack_fermion(const cplx<Ti>* in, const int* perm, long V, int nrhs, cplx<To>* out, hipStream_t st);
template <typename R>
// bsub != nullptr (whole operator, no dots): out = bsub - D in.  geo != nullptr:
// neighbours from the site arithmetic of the level-0 device order instead of nbr.
void launch_wilson(const cplx<R>* in, cplx<R>* out, const cplx<R>* U, const R* clov, const int* nbr, long V,
                   int terms, int nrhs, const int* run, hipStream_t st, cd64* dots = nullptr, int rs = 0,
                   const cplx<R>* bsub = nullptr, const SiteGeom* geo = nullptr, const cplx<R>* U2 = nullptr);
// two-row links of the Dslash (U2 of launch_wilson, with geo) and the SU(3)
// check that allows them: per-block maxima of |row2 - conj(row0 x row1)|
template <typename R>
void launch_pack_links2(const cd64* U, const int* perm, const int L[4], int antiperiodic, cplx<R>* out,
                        hipStream_t st);
int su3_defect_blocks(long n_links);
void launch_su3_defect(const cd64* U, long n_links, double* part, hipStream_t st);
int wilson_blocks(long V);
// FP32 D on nrhs fields with the links and clover read once per launch; MR
// partials (optional) at dots[2 * (r * wilson_blocks(V) + blk)]
void launch_wilson_mrhs(const cf32* in, cf32* out, const cf32* U, const float* clov, const int* nbr, long V, int nrhs,
                        const int* run, int rs, cd64* dots, hipStream_t st);

// ---- even-odd preconditioning (evenodd.hip): A^{-1} per site (packed like A,
// FP64 and FP32 copies; bad set on a vanishing pivot) and parity-masked
// site-local operations (modes in evenodd.hip)
// the halves of the Schur complement on parity-compact fields (evenodd.hip):
// mode 0 out = B h, mode 1 out = B aux - h, h the hops from the other parity
template <typename R>
void launch_schur_hop(const cplx<R>* in, cplx<R>* out, const cplx<R>* aux, const cplx<R>* U, const R* B,
                      const int* nbr, const int* tgt, const int* pos, long V, long Vh, int mode, const int* run,
                      hipStream_t st);
void launch_clover_invert(const double* A, long V, double* inv64, float* inv32, int* bad, hipStream_t st);
template <typename R>
void launch_eo_local(const cplx<R>* in, const cplx<R>* aux, cplx<R>* out, const R* B, const unsigned char* par,
                     int keep, int mode, long V, hipStream_t st);
// odd-site compaction ([12][Vh] with Vh = V/2; odd: device index of the j-th
// odd site; pos: the inverse on odd sites)
template <typename R>
void launch_eo_gather(const cplx<R>* full, cplx<R>* compact, const int* odd, long V, long Vh, hipStream_t st);
template <typename R>
void launch_eo_scatter(const cplx<R>* compact, cplx<R>* full, const int* pos, const unsigned char* par, long V,
                       long Vh, hipStream_t st);

// ---- SAP smoother (sap.hip): one colour of domains; x, b [nrhs][12][V];
// doms: aggregate indices of the colour; A: sites per domain (<= 256)
template <typename R>
void launch_sap(cplx<R>* x, const cplx<R>* b, const cplx<R>* U, const R* clov, const int* nbr, long V, int A,
                const int* doms, int ndoms, int iters, int nrhs, const int* run, int rs, hipStream_t st);

// ---- coarse operator (coarse.hip)
size_t device_block_bytes(long Vc, int nb, int prec);
void launch_blocks_to_device(const cd64* src, long Vc, int nb, int prec, void* dst, hipStream_t st);
void launch_c64_to_c128(const cf32* in, cd64* out, long n, hipStream_t st);
// bf16 != 0: the complex64 output holds the BF16-rounded values
void launch_c128_to_c64(const cd64* in, cf32* out, long n, int bf16, hipStream_t st);
void launch_coarse_apply(int prec, const void* blk, const void* in, void* out, const int* nbr, long Vc, int nb,
                         int dmask, int accumulate, int nrhs, const int* run, hipStream_t st, int rs = 0);

// ---- coarse operator from five-point storage (coarse5.hip): Mdiag and the
// forward blocks only, the backward hops from sigma3-hermiticity
bool five_point_supported(int nb);
size_t device_block5_bytes(long Vc, int nb, int prec);
void launch_blocks_to_device5(const cd64* src, long Vc, int nb, int prec, void* dst, hipStream_t st);
// tmp: 4 * nrhs * Vc * Nb complex of the vector precision, used when
// coarse5_uses_owner(Vc, nb, nrhs) (may be null otherwise)
bool coarse5_uses_owner(long Vc, int nb, int nrhs);
void launch_coarse_apply5(int prec, const void* blk, const void* in, void* out, void* tmp, const int* nbr, long Vc,
                          int nb, int accumulate, int nrhs, const int* run, hipStream_t st, int rs = 0);

// ---- batched coarse apply on the matrix cores (coarse_mfma.hip)
bool mfma_supported_nb(int nb);
size_t mfma_block_bytes(long Vc, int nb, int prec);
void launch_blocks_to_mfma(const cd64* src, long Vc, int nb, int prec, void* dst, hipStream_t st);
// tile 0: one wave per site, neighbour vectors read straight from memory;
// tile 4, 8, 16: workgroups of that many consecutive sites of one x-row with the
// neighbour vectors and the outputs staged in LDS; tile 5, 9: 4 or 8 sites with
// staged neighbour vectors and per-wave output stores (nbr must be the
// lexicographic table of a lattice of x extent Lx, which the site count divides)
void launch_coarse_apply_mfma(int prec, int nb, const void* blk, const cf32* in, cf32* out, const int* nbr, long Vc,
                              int nrhs, const int* run, int run_stride, hipStream_t st, int tile = 0, int Lx = 0);
bool mfma_tile_ok(int tile, int nb, long Vc, int Lx, int nrhs);

// ---- transfer and coarsening (transfer.hip)
bool supported_nb(int nb);
template <typename R>
void launch_restrict(const cplx<R>* fine, cplx<R>* coarse, const cplx<R>* P, FieldLayout lay, const int* agg_sites,
                     int A, long Vc, int nb, int nrhs, const int* run, hipStream_t st, int rs = 0);
template <typename R>
// agg_sites (optional, [Vc][A] device sites of each aggregate): lets several
// right-hand sides of an FP32 level-0 field take the per-aggregate form
void launch_prolong(const cplx<R>* coarse, cplx<R>* fine, const cplx<R>* P, FieldLayout lay, const int* coarse_of,
                    long Vc, int nb, int accumulate, int nrhs, const int* run, hipStream_t st, int rs = 0,
                    const int* agg_sites = nullptr, int A = 0);
void launch_block_orthonormalise(cd64* vecs, FieldLayout lay, const int* agg_sites, int A, long Vc, int nv,
                                 int* breakdown, hipStream_t st);
void launch_prolongator_columns(const cd64* P, FieldLayout lay, int nv, cd64* out, hipStream_t st);
// level 0 Galerkin term d with the images of P's columns formed on the fly
// (U, clov: packed FP64 links and (4 + m0) + C; nbr [8][V])
// (dint: the block slot that contributions of hops inside an aggregate go to;
// 0 = Mdiag)
void launch_galerkin_fused(const cd64* P, const cd64* U, const double* clov, const int* nbr, long V,
                           const int* agg_sites, const int* coarse_of, int A, long Vc, int nb, int d, int dint,
                           cd64* M, hipStream_t st);
void launch_galerkin_project(const cd64* W, const cd64* P, FieldLayout lay, const int* agg_sites,
                             const int* coarse_of, const int* nbr_d, int A, long Vc, int nb, int d, int dint,
                             cd64* M, hipStream_t st);
// backward terms from the forward ones (and the -mu slots' inside-aggregate
// parts folded into Mdiag); nbr_c: coarse neighbour table [8][Vc]
void launch_galerkin_mirror(cd64* M, const int* nbr_c, long Vc, int nb, hipStream_t st);

// ---- vector algebra and solver control (blas.hip)
template <typename R>
void launch_dot(const cplx<R>* a, long astride, int m, const int* m_dev, const cplx<R>* b, long n, cd64* partial,
                int mstride, cd64* out, int ostride, int mode, const int* run, hipStream_t st);
int reduction_blocks(long n);
template <typename R>
void launch_multi_axpy_norm(cplx<R>* y, const cplx<R>* V, long vstride, int m, const cd64* coef, int cstride,
                            double sign, long n, cd64* partial, const int* run, hipStream_t st);

void launch_dot_finish(const cd64* partial, int G, int m, int mstride, cd64* out, int ostride, int mode,
                       const int* run, hipStream_t st);
template <typename R>
void launch_multi_axpy(cplx<R>* y, const cplx<R>* V, long vstride, int m, const int* m_dev, const cd64* coef,
                       int cstride, double sign, long n, const int* run, hipStream_t st, int grid = 0);
template <typename R>
void launch_axpby(cplx<R>* y, const cplx<R>* x, double a, double b, long n, const int* run, hipStream_t st);
template <typename R>
void launch_scale_inv_norm(cplx<R>* y, const cplx<R>* x, const cd64* nrm2, long n, const int* run, hipStream_t st);
template <typename R>
void launch_zero(cplx<R>* y, long n, const int* run, hipStream_t st);
template <typename R>
void launch_sub(cplx<R>* y, const cplx<R>* a, const cplx<R>* b, long n, const int* run, hipStream_t st);
template <typename Ti, typename To>
void launch_convert(const cplx<Ti>* x, cplx<To>* y, long n, const int* run, hipStream_t st);
template <typename R>
void launch_mr_update(cplx<R>* x, cplx<R>* r, const cplx<R>* p, const cd64* dots, long n, const int* run,
                      hipStream_t st);
// MR update whose step length <p, r> / <p, p> is summed from G per-workgroup
// partial pairs part[2g], part[2g+1] inside the update kernel (same order and
// result as launch_dot_finish).  xout != nullptr: the new x goes there in
// FP64 instead of to x.
template <typename R>
void launch_mr_update_part(cplx<R>* x, cplx<R>* r, const cplx<R>* p, const cd64* part, int G, long n, const int* run,
                           hipStream_t st, cd64* xout = nullptr);
template <typename R>
void launch_mr_dots_update(cplx<R>* x, cplx<R>* r, const cplx<R>* p, long n, cd64* partial, cd64* dots,
                           const int* run, hipStream_t st);
void launch_gmres_init(int* st_, const int* parent, hipStream_t st);
void launch_gmres_cycle_start(int* st_, cd64* S, int m, double tol, int limit, int fixed, hipStream_t st);
void launch_gmres_givens(int* st_, cd64* S, int m, int j, double tol, int limit, int fixed, int stop_on_est,
                         hipStream_t st);
void launch_gmres_solve_y(const int* st_, cd64* S, int m, hipStream_t st);
// single-reduction Arnoldi step (blas.hip): first sweep (shifted vector, its
// dots with V_0..V_j and its norm), bookkeeping, last sweep (update + scale)
void launch_gmres_sr(int* st_, cd64* S, int m, int j, cd64* d, const cd64* d2, int stage, hipStream_t st);
// launch_dot_finish of the j + 2 first-projection sums (partials with stride
// j + 2, into d) and launch_gmres_sr stage 0 in one launch (st: the solver's
// state words, st[6] an arrival count that k_gmres_init zeroes)
void launch_dot_finish_sr(const cd64* partial, int G, int j, cd64* d, int* st_, cd64* S, int m, hipStream_t st);
// Stage 1 of launch_gmres_sr (its second-projection products summed from G2
// partials part2[g * (j + 2) + k] inside, into d2) followed by
// launch_gmres_givens, in one single-workgroup launch.
// pub != nullptr: st[0..pub_n) is then published to pub as launch_publish_state
// would (number pub_seq), in the same launch.
void launch_gmres_sr_finish(int* st_, cd64* S, int m, int j, cd64* d, cd64* d2, const cd64* part2, int G2,
                            double tol, int limit, int fixed, int stop_on_est, hipStream_t st, int* pub = nullptr,
                            int pub_seq = 0, int pub_n = 0);
template <typename R>
// grid: workgroups (partials) to use, 0 = reduction_blocks(n)
void launch_arnoldi_dots(cplx<R>* V, long n, int j, const cd64* shift, cd64* partial, int mstride, const int* run,
                         hipStream_t st, int grid = 0);
template <typename R>
void launch_update_scale(cplx<R>* y, const cplx<R>* V, long vstride, int m, const cd64* coef, const cd64* nrm2,
                         long n, const int* run, hipStream_t st);
void launch_gmres_cycle_end(int* st_, hipStream_t st);
// copies st[0..n) to out[1..n] (host-mapped memory), then out[0] = seq
void launch_publish_state(const int* st_, int n, int* out, int seq, hipStream_t st);

// ---- the coarsest GMRES in one persistent launch (coarse_persist.hip; coop_api:
// through the cooperative-launch API, else an ordinary launch of at most one
// workgroup per CU):
// false (nothing launched) when the operator's blocks, basis and image do not
// fit the LDS of co-resident workgroups; part: cd64 [cg_persistent_part_elems];
// bar: cg_persistent_bar_words words, zeroed with the buffer (bar[2] is set
// when a barrier wait timed out, bar[3..6] then hold the first timed-out
// workgroup, the phase, the workgroup it waited for and the flag value it
// saw; bar[8] holds the phase the flags have reached, which the next launch
// on the buffer continues from; a launch that starts with bar[2] set writes
// x = 0 and reports nothing); mailbox (host-mapped, coherent, kCgpMailboxInts
// ints): at a normal end workgroup 0 writes the report slot of `seq`
// (mailbox[kCgpSlot0 + 2 (seq mod kCgpSlots)] = seq, the next word the
// iteration count), [1] live flag, [3] iterations, then [0] = seq; misc: the
// solve's residual words, as the multi-kernel form writes them; z: 2 Vc Nb
// vector elements; r: Vc Nb
bool cg_persistent_fits(int prec, int nb, long Vc);
size_t cg_persistent_part_elems(long Vc);
size_t cg_persistent_bar_words(long Vc);
bool launch_cg_persistent(int prec, int nb, const void* blk, const int* nbr, long Vc, const void* b, void* x,
                          void* z, void* r, cd64* part, cd64* misc, int* st, const int* parent, int m, double tol,
                          int limit, int fixed, unsigned* bar, int seq, int* mailbox, double timeout_s,
                          bool coop_api, hipStream_t stream);
constexpr int kCgpSlot0 = 16;       // first report slot in the mailbox
constexpr int kCgpSlots = 64;       // report slots (a power of two)
constexpr int kCgpMailboxInts = kCgpSlot0 + 2 * kCgpSlots;

// ---- fused coarse GMRES (coarse_gmres.hip)
bool cg_fused_supported(int nb);
template <typename R>
void launch_cg_norm_partial(const cplx<R>* r, long n, cd64* part, int m1, const int* run, hipStream_t st);
void launch_cg_cycle_start(int* stw, cd64* S, int m, const cd64* part, int G, int first, double tol, int limit,
                           int fixed, hipStream_t st);
// five: blk holds five-point storage
int launch_cg_apply(int prec, int nb, const void* blk, const int* nbr, long Vc, const void* u, const cd64* unrm2,
                    void* V, int j, void* wout, cd64* part, int m1, const int* run, hipStream_t st, bool five = false);
template <typename R>
void launch_cg_orth(cplx<R>* V, int j, cplx<R>* w, long n, const cd64* part_in, int G_in, cd64* S, int m, int pass,
                    cd64* part_out, const int* run, hipStream_t st);
void launch_cg_givens(int* stw, cd64* S, int m, int j, const cd64* part, int G, double tol, int limit, int fixed,
                      hipStream_t st);

// ---- batched vector kernels (blas_batch.hip)
int bred_blocks(long n);
// batched single-reduction Arnoldi step (blas_batch.hip; the forms of
// launch_arnoldi_dots, launch_gmres_sr and launch_update_scale with a
// right-hand-side index)
template <typename R>
void launch_barnoldi_dots(cplx<R>* V, long vvs, long vrs, int j, long n, const cd64* shift, long shs,
                          cd64* partial, int B, const int* run, int rs, hipStream_t st);
template <typename R>
void launch_bupdate_scale(cplx<R>* y, long yrs, const cplx<R>* V, long vvs, long vrs, int m, const cd64* coef,
                          long crs, const cd64* nrm2, long nrs, long n, int B, const int* run, int rs,
                          hipStream_t st);
void launch_bgmres_sr(int* st_, cd64* S, long ss, int B, int m, int j, cd64* d, cd64* d2, int stage, hipStream_t st);
template <typename R>
void launch_bdot(const cplx<R>* a, long avs, long ars, int m, const cplx<R>* b, long brs, long n, int B,
                 cd64* partial, cd64* out, int ostride, long ors, int mode, const int* run, int rs, hipStream_t st);
void launch_bdot_finish(const cd64* partial, int G, int m, int mstride, int B, cd64* out, int ostride, long ors,
                        int mode, const int* run, int rs, hipStream_t st);
// y_r -= V_r coef_r and partials of V_r^dag y_r in one sweep (m <= kFusedMaxM);
// partial layout [r][bred_blocks(n)][m]
constexpr int kFusedMaxM = 20;
template <typename R>
void launch_bmulti_axpy_dot(cplx<R>* y, long yrs, const cplx<R>* V, long vvs, long vrs, int m, const cd64* coef,
                            int cks, long crs, long n, int B, cd64* partial, const int* run, int rs, hipStream_t st);
template <typename R>
void launch_bmulti_axpy(cplx<R>* y, long yrs, const cplx<R>* V, long vvs, long vrs, int m, const int* m_dev, int ms,
                        const cd64* coef, int cks, long crs, double sign, long n, int B, cd64* norm_part,
                        const int* run, int rs, hipStream_t st);
template <typename Ti, typename To>
void launch_belem(To* y, long yrs, const Ti* x, long xrs, const Ti* z, long zrs, const cd64* nrm2, long nrs, long n,
                  int B, int op, const int* run, int rs, hipStream_t st);
template <typename R>
void launch_bmr_update(cplx<R>* x, cplx<R>* r, const cplx<R>* p, long rsf, const cd64* dots, long n, int B,
                       const int* run, int rs, hipStream_t st);
void launch_bgmres_init(int* st_, int B, const int* parent, int prs, hipStream_t st);
void launch_bgmres_cycle_start(int* st_, cd64* S, long ss, int B, int m, double tol, int limit, int fixed,
                               hipStream_t st);
void launch_bgmres_givens(int* st_, cd64* S, long ss, int B, int m, int j, double tol, int limit, int fixed,
                          int stop_on_est, hipStream_t st);
void launch_bgmres_solve_y(const int* st_, cd64* S, long ss, int B, int m, hipStream_t st);
void launch_bgmres_cycle_end(int* st_, int B, hipStream_t st);

// ---- per-launch kernel timing
// A profiled single-kernel launch takes its event pair from this thread-local
// slot and records it in the dispatch itself (hipExtLaunchKernelGGL), so the
// measured interval is the kernel's own execution; the slot is then cleared.
struct KernelTiming {
  hipEvent_t start = nullptr, stop = nullptr;
};
KernelTiming& kernel_timing();
#define WCMG_LAUNCH(K, G, B, S, ST, ...)                                                    \
  do {                                                                                     \
    ::wcmg::KernelTiming& kt_ = ::wcmg::kernel_timing();                                   \
    if (kt_.start) {                                                                       \
      hipExtLaunchKernelGGL(K, G, B, S, ST, kt_.start, kt_.stop, 0, __VA_ARGS__);          \
      kt_ = ::wcmg::KernelTiming();                                                        \
    } else {                                                                               \
      hipLaunchKernelGGL(K, G, B, S, ST, __VA_ARGS__);                                     \
    }                                                                                      \
  } while (0)

// ---- learned near-null proposal (nn.hip); activations: 16 = BF16, 32 = FP32
void launch_nn_layer(int act_bits_in, const void* in, int Cin, const cf32* W, int Cout, int act_bits_out, void* out,
                     float* scale, int squash, const cf32* U, const int* nbr, long V, hipStream_t st);
int nn_wgrad_blocks(long V);
void launch_nn_wgrad(const cf32* g, int Cout, int act_bits, const void* a, int Cin, const cf32* U, const int* nbr,
                     long V, cd64* part, cf32* gW, hipStream_t st);
void launch_nn_squash_bwd(cf32* g, int act_bits, const void* a, const float* scale, int C, long V, hipStream_t st);
void launch_nn_loss(const cf32* Y, const cf32* T, int nv, const int* agg_sites, int A, long Vc, long V, double norm,
                    cf32* gY, double* loss_part, hipStream_t st);
void launch_nn_adam(float* w, const cf32* gW, float* m, float* v, long n_complex, float lr, int step, hipStream_t st);
void launch_nn_adjoint_weights(const cf32* W, int Cout, int Cin, cf32* Wadj, hipStream_t st);
void launch_nn_from64(const cd64* x, int act_bits, void* y, long n, hipStream_t st);
void launch_nn_to64(const cf32* x, cd64* y, long n, hipStream_t st);

// ragged batch of matrix-core coarse applies (coarse_mfma.hip)
constexpr int kRaggedMax = 8;
struct RaggedProblem {
  const void* blk;  // fragment-ordered blocks
  const cf32* in;   // [nrhs][Vc][Nb]
  cf32* out;
  const int* nbr;   // [8][Vc]
  long Vc;
  int nrhs;
  const int* run = nullptr;  // per-RHS run flags (stride rs), or none
  int rs = 0;
};
struct RaggedTable {
  RaggedProblem p[kRaggedMax];
  long site0[kRaggedMax + 1];  // prefix sums of Vc (filled by the launcher)
  int n, nb;
};
void launch_coarse_apply_mfma_ragged(int prec, RaggedTable t, hipStream_t st);

constexpr int kPartialSlots = 2048 * 48;  // partial buffer entries (blocks x max dots)

}  // namespace wcmg
