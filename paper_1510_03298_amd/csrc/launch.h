// launch.h -- host-side launchers of the gfx950 kernels (internal to the library).
//
// The rho chain of Sec. 6.1 is evaluated with mode 3 as the "slab" mode: the
// mode-3 products are GEMMs (kernels slab_fwd and slab_adj), and the mode-1 and
// mode-2 products of one i3 slab run inside one workgroup with all
// intermediates in registers (kernel slab_chain).  Modes 1 and 2 are padded to
// 16-row tiles.
//
// Internal layouts (all zero padded):
//  * k-blocked operand of a GEMM with contraction length K and free length C:
//      elem(k, c) at ((k / 16) * C + c) * 16 + kpos<T>(k % 16)
//    so that one lane's MFMA fragment is 4 contiguous elements;
//    S2 (K = n3, C = P12), the increment / Theta (K = p3, C = P12), and the two
//    copies of X_3 (K = p3, C = n3 for slab_fwd; K = n3, C = p3 for slab_adj).
//  * T1 slab-major: [i3][m], m = i1 + p1 * i2 (one contiguous p1 x p2 block per slab)
//  * tiled n-arrays (eta, V, Y, a): slab i3, mode-2 tile jb, mode-1 tile ut,
//    a 16 x 16 column-major tile (i1 fastest):
//      ((i3 * NJB + jb) * N1T + ut) * 256 + (i2 % 16) * 16 + (i1 % 16)
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include <string>
#include <vector>

namespace glam {

struct Geom {
  int n1, n2, n3, p1, p2, p3;
  int P12;          // p1 * p2
  int N1T, NJB;     // ceil(n1 / 16), ceil(n2 / 16)
  int PT;           // ceil(max(p1, p2) / 16), 1 or 2
  int KB3, KBN3;    // ceil(p3 / 16), ceil(n3 / 16)
  long long nint;   // length of a tiled n-array
  long long n;      // n1 * n2 * n3
  long long p;      // p1 * p2 * p3
  long long t1_len; // n3 * P12
  long long s2_len; // KBN3 * 16 * P12
  long long inc_len;// KB3 * 16 * P12
  long long x3f_len;// KB3 * 16 * n3
  long long x3a_len;// KBN3 * 16 * p3
};

Geom make_geom(const int64_t* n, const int64_t* p);

enum Dt { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2 };

inline size_t dt_size(int dt) { return dt == DT_F64 ? 8 : (dt == DT_F32 ? 4 : 2); }

enum SlabMode {
  SM_FWD_STD = 0,   // eta (standard layout, FP64 for F64 else FP32)
  SM_FWD_INT = 1,   // eta (tiled layout, accumulation type)
  SM_ADJ_STD = 2,   // R read from a standard-layout n-array of the chain type
  SM_FUSED = 3,     // R = eta (.* V tiled) -> S2  (inner-loop gradient)
  SM_FAMILY = 4,    // FP64: eta -> (eta, V, u, -l partial sums) -> R = u -> S2
  SM_NLL_FWD = 5,   // eta -> partial sums of exp(eta) - y eta
  SM_NLL_BWD = 6    // eta -> R = exp(eta) - y -> S2
};

struct SlabParams {
  Geom G;
  const void* img;    // LDS image of X1 and X2 in the chain type (launch_pack_chain_image)
  const void* T1;     // chain type, slab-major [n3][P12]
  void* S2;           // chain type, k-blocked (K = n3, C = P12)
  void* eta_out;      // FWD_STD / FWD_INT output
  const void* u_in;   // ADJ_STD input (chain type, standard layout)
  const void* v_int;  // FUSED weights (tiled, accumulation type) or NULL = 1
  // FAMILY (FP64 chain)
  const double* y_int;
  const double* a_int;    // prior weights (tiled), or NULL: 1
  double* eta_int;        // eta written out (tiled), or NULL: not kept
  void* v_out;        // tiled weights written for the inner loop (FP32 or FP64), may be NULL
  int v_out_f32;      // 1: v_out is float, 0: double
  int family;         // glam_family: 0 Gaussian, 1 Poisson, 2 Binomial, 3 Gamma
  // NLL (standard-layout FP64 counts)
  const double* y_std;
  const float* y_tiled;   // NLL, one-wave-per-slab kernel: the counts tiled like v_int (FP32), used instead of y_std
  double* partials;   // per-workgroup partial sums [grid][2]
  const int* stop;    // optional: the kernel does nothing when *stop != 0 (the inner loop has ended)
};

enum AdjEpi { EPI_STORE = 0, EPI_GRAD = 1, EPI_PROX = 2, EPI_PROX_BT = 3 };
constexpr int ADJ_NSUM = 6;   // partial values per slab_adj workgroup

struct AdjParams {
  Geom G;
  const void* S2;     // chain type, k-blocked (K = n3, C = P12)
  const void* X3a;    // chain type, k-blocked (K = n3, C = p3)
  void* out;          // EPI_STORE: p-array (FP64 for F64 chains, FP32 otherwise)
  double scale;       // EPI_STORE: out = scale * acc ; EPI_GRAD: g = scale * acc
  const double* gscale_dev;  // EPI_STORE: optional device scalar multiplier
  // EPI_GRAD: g = scale * acc written to gout; KKT / lambda_max partial maxima
  double* gout;
  const double* theta;   // FP64 p-array (KKT at theta) or NULL
  const double* pen_w;   // FP64 p-array or NULL
  double lambda;
  double* partials;      // per-workgroup [nblk][ADJ_NSUM]
  // EPI_PROX (inner PG iteration, FP64 state)
  const double* gref;    // gradient at the anchor
  const double* theta_ref;
  double* x;             // x^l   (updated to x^{l+1})
  double* xp;            // x^{l-1} (updated to x^l)
  double* gp;            // grad h(x^{l-1}) (updated to grad h(x^l))
  void* inc;             // chain type, k-blocked (K = p3, C = P12): x^{l+1} - theta_ref
  const int* iter;       // device iteration counter l
  double delta;          // step size
  const double* dparams; // optional device {lambda, delta[, l]} (overrides the scalars; lets a
                         // captured graph be replayed across lambdas and outer iterations)
  // EPI_PROX_BT (backtracking): previous extrapolation point and its gradient, and the
  // double-buffered next state (x^{l+1}, x^l, grad h(x^l), y_l, grad h(y_l))
  const double* yprev;
  const double* gyprev;
  double *x_out, *xp_out, *gp_out, *y_out, *gy_out;
  int s2_kb4;            // S2 in 4-deep k-blocks: elem (i3, m) at ((i3 / 4) P12 + m) 4 + i3 % 4
  double alpha;          // elastic-net weight (Sec. 6.3): J = sum w (|theta| + alpha theta^2); 0 = lasso
  int no_l1;             // 1: no l1 term (the ridge penalty, J = sum w alpha theta^2)
};

// The inner PG step of the BF16 / FP32 chains on FP32 increment state (step control nu = 1).
// The iterate x^l = theta_ref + d^l is held as FP32 increments d in the adjoint's tile layout
// (16 x 16 output tile (bm, bn) contiguous at (bn * NBM + bm) * 256, element (m % 16) * 16 +
// k3 % 16, NBM = ceil(P12 / 16)), with theta_ref and grad h(theta_ref) as FP64 copies in the same
// layout.  A coordinate whose x is exactly zero (the soft threshold's zero) is stored as a NaN
// increment, so that exact zeros survive the FP32 rounding of theta_ref.  The extrapolation
// keeps q = grad h(x^{l-1}) - grad h(theta_ref) (FP32) instead of the FP64 gradient.
struct AdjIncParams {
  Geom G;
  const void* S2;        // chain type, k-blocked (K = n3, C = P12) or in 4-deep k-blocks (s2_kb4)
  const void* X3a;       // chain type, k-blocked (K = n3, C = p3)
  int s2_kb4;
  const double* gT;      // grad h(theta_ref), tiled
  const double* tT;      // theta_ref, tiled
  const double* penT;    // penalty weights, tiled, or NULL (all 1)
  const float* dcur;     // d^l
  const float* dprev;    // d^{l-1}
  float* dout;           // d^{l+1} (in the fit: the buffer of dprev, each element read before written)
  const float* q_in;     // q of x^{l-1}
  float* q_out;          // q of x^l (in the fit: the buffer of q_in)
  void* inc;             // chain type, k-blocked (K = p3, C = P12): x^{l+1} - theta_ref
  const int* iter;       // device iteration counter l
  const double* dparams; // device {lambda, delta}
  double scale;          // 1 / n
  double alpha;          // elastic-net weight
  int no_l1;             // 1: the ridge penalty (no l1 term)
  double* partials;      // per-workgroup [nblk][ADJ_NSUM], slab_adj's layout
  int xmap;              // tile order: 0 row blocks fastest; 1 XCD-aware (each XCD a range of row blocks)
  const int* stop;       // optional: the kernel does nothing when *stop != 0 (the inner loop has ended)
};
inline long long adj_tiled_len(const Geom& G) { return (long long)((G.P12 + 15) / 16) * ((G.p3 + 15) / 16) * 256; }
hipError_t launch_slab_adj_inc(int dt, const AdjIncParams& P, int* nblk_out, hipStream_t s);
int slab_adj_inc_blocks(const Geom& G, int xmap);
// partial-sum rows a launch writes (the reduction's block count)
int slab_adj_inc_partials(const Geom& G, int xmap);
// the tile order the fits use: 16 x 16 tiles, split-K over the 4 waves, in the XCD-aware order
// (each XCD a run of row blocks, so its L2 fetches only its part of S2).  n = (100, 100, 1000),
// p = (30, 30, 200), BF16: back to back 7.7 us in either order (7.3 us for 32 x 32 tiles, 10.4 us
// for whole-contraction waves; 9.45 us for the FP64-state step), but the XCD order fetches 10.3
// instead of 22.0 MB per launch and the whole path runs 5% faster with it.
constexpr int kAdjIncForm = 1;
// per outer step: tT, gT (and penT when pen_w != NULL) from theta, gref, pen_w; d0 = d1 = q = 0,
// inc = 0 (k-blocked, chain dtype), *iter = 0
hipError_t launch_inner_init_inc(int dt, const Geom& G, const double* theta, const double* gref, const double* pen_w,
                                 double* tT, double* gT, double* penT, float* d0, float* d1, float* q, void* inc,
                                 int* iter, hipStream_t s);
// out = x (diff == 0) or x - theta_ref (diff == 1) in the standard layout, x from the tiled
// increments d and theta (theta_ref, standard layout); out may alias theta
hipError_t launch_inc_state_out(const Geom& G, const float* d, const double* theta, int diff, double* out,
                                hipStream_t s);

struct FwdParams {
  Geom G;
  const void* theta;  // chain type, k-blocked (K = p3, C = P12)
  const void* X3f;    // chain type, k-blocked (K = p3, C = n3)
  void* T1;           // chain type, slab-major [n3][P12]
  int* iter;          // optional: incremented once by the first thread
  const int* stop;    // optional: the kernel does nothing when *stop != 0 (the inner loop has ended)
};

// batched proximal step (many independent problems per launch, three launches per step)
struct BatchDesc {
  FwdParams fw;       // theta = increment (k-blocked), X3f, T1
  SlabParams sp;      // img, T1, S2, v_int
  AdjParams ap;       // EPI_PROX fields; iter -> the batch step counter
  int fwd_gx;         // slab_fwd workgroup grid x
  int adj_gx;         // slab_adj workgroup grid x
};
// The compact work list of the active problems lives in device memory, so that a captured graph
// of batched steps stays valid when the host rewrites the list (the kernels grid-stride over
// whatever the list holds).  The register-kernel slab phase orders the list by shape class
// (class c = P16 (p1, p2 <= 16) + 2 N1B4 (n1 <= 64)): class c holds entries cls_k[c] ..
// cls_k[c+1] - 1, in runs of run[c] consecutive slabs of one problem.
struct BatchWork {
  int nact;
  int cls_k[5];
  int run[4];           // slabs per run, per class (the LDS slab kernel uses run[0])
};
struct BatchParams {
  const BatchDesc* desc;
  int nprob;
  const int* off_adj;   // prefix sums of slab_adj tiles over all problems (the partials index)
  const BatchWork* work;
  const int* act;       // active problem indices (nact)
  const int* aoff_fwd;  // prefix sums of slab_fwd tiles (nact + 1)
  const int* aoff_run;  // prefix sums of slab runs, ceil(n3 / run) per problem (nact + 1)
  const int* aoff_adj;  // prefix sums of slab_adj tiles (nact + 1)
  int cls;              // the class of one slab-phase launch
  int* step;            // inner step counter (read by the prox epilogue)
  int wave;             // slabs with the register kernel (S2 in 4-deep k-blocks; batched_wave)
};
// Launch shape of one batched step: workgroups of the forward phase, of each class's slab launch
// (0: no launch; the list of a later block may hold fewer entries, never more of a class that
// had none) and of the adjoint phase; wide[c] = 1 runs class c on the kernel of the next wider
// shape (the full 32-deep p contraction, or eight X1 row tiles), the same values
struct BatchGrid {
  int fwd, adj, slab;   // slab: the LDS slab kernel (not wave)
  int cls[4];
  int wide[4];
};
// true when every problem of the batch fits the one-wave-per-slab kernel of this dtype
bool batched_wave(int dt, const Geom* Gs, int nprob);
size_t batched_lds_bytes(int dt, const Geom* Gs, int nprob);
// grid sizes for the given totals {forward tiles, slab runs, adjoint tiles} and class runs
BatchGrid batched_grid(const int* tot, const int* cls_runs);
hipError_t launch_batched_step(int dt, const BatchParams& B, const BatchGrid& g, size_t lds, hipStream_t s);
// one class's slab launch alone (the tuner's timing unit)
hipError_t launch_batched_class(int dt, const BatchParams& B, int c, int wide, int grid, hipStream_t s);
hipError_t launch_segment_max(const double* partials, const int* off, int nprob, double* out, hipStream_t s);

// Gram inner gradient (Gaussian, identity weights): Z_k3 = S_1 D_k3 S_2 for every slice k3
// of the k-blocked increment D (K = p3, C = P12) into Z (same layout); S_j FP64 p_j x p_j;
// increments *iter once when iter != NULL
hipError_t launch_gram12(int dt, const Geom& G, const void* inc, const double* S1, const double* S2, void* Z, int* iter,
                         hipStream_t s);
// One inner PG iteration of the Gram form (Sec. 6.2) in one launch; see gram.hip.
constexpr int GRAM_MAX_P3 = 2048;   // contraction length p3 (padded to 16) the fused kernel takes
struct GramIterParams {
  Geom G;
  const void* inc_in;       // increment x - theta_ref (chain dtype, k-blocked), read
  void* inc_out;            // next increment, written (must not alias inc_in)
  const double *S1, *S2, *S3;   // FP64 Gram factors X_j^T X_j (p_j x p_j, symmetric)
  const double *gref, *theta_ref, *pen_w;
  double *x, *xp, *gp;      // FISTA state, updated on each workgroup's own slice
  const double* dparams;    // device {lambda, delta}
  const int* iter_in;       // iteration counter l - 1, read
  int* iter_out;            // l, written (must not alias iter_in)
  double alpha;             // elastic-net weight
  int no_l1;                // 1: the ridge penalty (no l1 term)
  double scale;             // 1 / n
  double* partials;         // [nblk][ADJ_NSUM], slab_adj's layout
  int per_xcd;              // set by the launcher
};
int gram_iter_blocks(int dt, const Geom& G);
bool gram_iter_fits(const Geom& G);
// the fused iteration is used for BF16 and FP32 increments: in FP64 each workgroup's read of
// the whole increment (8 bytes an element) costs more than the two-kernel form
bool gram_iter_pays(int dt, const Geom& G);
// Tensor-product weights (Sec. 6.2) from the tiled eta of a family step: the weighted Gram
// factors S_j = X_j^T diag(v_j) X_j (S_3 times Vbar) and stats = {max v_1, max v_2, max v_3,
// Vbar} (device).  work: kron_work_doubles(G) doubles.  X_j: FP64 column-major factors.
size_t kron_work_doubles(const Geom& G);
hipError_t launch_kron_weights(const Geom& G, int family, const double* eta_int, const double* X1, const double* X2,
                               const double* X3, double* work, double* stats, double* S1, double* S2, double* S3,
                               hipStream_t s);
hipError_t launch_gram_iter(int dt, const GramIterParams& P, int* nblk_out, hipStream_t s);
// spectral radii of S1, S2, S3 (FP64 p_j x p_j, symmetric PSD) by the power method from the vectors
// kept in work (first: from ones): stats[4 + j] = an upper bound of rho(S_j) once converged,
// stats[7] = 1 if all three converged (else 0)
hipError_t launch_gram_radii(const Geom& G, const double* S1, const double* S2, const double* S3, double* work,
                             int first, double* stats, hipStream_t s);

// rho kernels
hipError_t launch_slab_fwd(int dt, const FwdParams& P, hipStream_t s);
hipError_t launch_slab_chain(int dt, int mode, const SlabParams& P, int* nblk_out, hipStream_t s);
// true when launch_slab_chain writes S2 in 4-deep k-blocks (AdjParams::s2_kb4) for this mode
bool chain_s2_kb4(int dt, int mode, const Geom& G);
hipError_t launch_slab_adj(int dt, int epi, const AdjParams& P, int* nblk_out, hipStream_t s);
size_t slab_chain_lds_bytes(int dt, const Geom& G);
// LDS image of the mode-1 / mode-2 factors (X1, X2: n_j x p_j column-major, FP64 or chain dtype)
size_t chain_image_bytes(int dt, const Geom& G);
// need: PACK_LDS (the workgroup-per-slab kernel's LDS image) and / or PACK_WAVE (the
// register fragments of the one-wave-per-slab BF16 kernel); chain_image_need(dt, mode, G)
// gives the part that launch_slab_chain reads for a mode
enum { PACK_LDS = 1, PACK_WAVE = 2 };
int chain_image_need(int dt, int mode, const Geom& G);
hipError_t launch_pack_chain_image(int dt, int src_dt, const Geom& G, const void* X1, const void* X2, void* img,
                                   hipStream_t s, int need);
int slab_adj_blocks(const Geom& G);
int slab_chain_blocks(int dt, const Geom& G);

// layout conversion: dst (k-blocked, dtype dt) elem(k, c) = src[k * sk + c * sc] for k < K, 0 beyond;
// src is FP64 (src_dt = DT_F64) or of dtype dt.
hipError_t launch_pack(int dt, int src_dt, const void* src, long long K, long long C, long long sk, long long sc,
                       void* dst, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

// small kernels
// out[v] = scale * sum_b partials[b][v]  (ops[v] == 0)  or  max_b partials[b][v]  (ops[v] == 1);
// summation order is fixed, so results are reproducible run to run.
hipError_t launch_reduce(const double* partials, int nblk, int nval, const int* ops, double scale, double* out,
                         hipStream_t s);
// the same, also published to mapped host memory, slot s % 2 of hout (8 doubles per slot:
// the nval values, then the "skipped" flag) followed by the sequence number *hseq = s = ++*seq_dev
// (device counter), for a host wait without a copy (nval < 8; two blocks may be in flight);
// restart_iter != NULL: *restart_iter = 0 when value restart_slot is > 0 (the restarted
// extrapolation sequence of the inner loop).  stop != NULL: the inner loop's convergence test on
// the device, crit = {lambda scale, tol_in, 4 eps}: *stop = 1 when value 0 / crit[0] is not finite or
// is <= max(crit[1], crit[2] value 1 / crit[0]) (the host's own test, in the same arithmetic); a
// launch that finds *stop already set publishes only the "skipped" flag 1 and the sequence number
hipError_t launch_reduce_publish(const double* partials, int nblk, int nval, const int* ops, double scale, double* out,
                                 double* hout, unsigned* seq_dev, unsigned* hseq, hipStream_t s, int restart_slot = -1,
                                 int* restart_iter = nullptr, int* stop = nullptr, const double* crit = nullptr);
// same with partials[b * stride + v], v < nval <= stride
hipError_t launch_reduce_strided(const double* partials, int nblk, int stride, int nval, const int* ops, double scale,
                                 double* out, hipStream_t s);
hipError_t launch_convert(int dt, const double* src, void* dst, long long count, hipStream_t s);
// the same tiling into FP32 (zeros outside the model)
hipError_t launch_to_tiled_f32(const Geom& G, const double* src_std, float* dst_tiled, hipStream_t s);
hipError_t launch_to_tiled(const Geom& G, const double* src_std, double fill_valid, double* dst_tiled,
                           hipStream_t s);
hipError_t launch_inner_init(const Geom& G, const double* theta, const double* gref, double* x, double* xp,
                             double* gp, int dt, void* inc, int* iter, hipStream_t s);
hipError_t launch_sub(long long p, const double* a, const double* b, double* out, hipStream_t s);
hipError_t launch_axpy(long long p, double alpha, const double* d, double* theta, hipStream_t s);
hipError_t launch_armijo(const Geom& G, int family, const double* eta_int, const double* xd_int,
                         const double* y_int, const double* a_int, int j0, double* partials, int* nblk_out,
                         hipStream_t s);
hipError_t launch_fill(double* p, long long count, double v, hipStream_t s);
// p[0] = 1 in dtype dt (the 1 x 1 middle factor of a lifted d = 2 model)
hipError_t launch_set_one(int dt, void* p, hipStream_t s);

// A d = 2 model X_2 (x) X_1 is the d = 3 model X_2 (x) [1] (x) X_1 (a 1 x 1 middle factor):
// the same vec layout of every array; mode 2 becomes the slab mode.  Sizes of the lift:
inline void lift_sizes(int d, const int64_t* n, const int64_t* p, int64_t* n3, int64_t* p3) {
  if (d == 2) {
    n3[0] = n[0]; n3[1] = 1; n3[2] = n[1];
    p3[0] = p[0]; p3[1] = 1; p3[2] = p[1];
  } else {
    for (int j = 0; j < 3; ++j) { n3[j] = n[j]; p3[j] = p[j]; }
  }
}
// backtracking redo of a rejected step: x = S(y - delta gy, delta lambda w), inc = x - theta_ref (k-blocked)
hipError_t launch_bt_redo(int dt, const Geom& G, const double* y, const double* gy, const double* pen_w,
                          const double* theta_ref, double lambda, double delta, double alpha, int no_l1, double* x,
                          void* inc, hipStream_t s);
// sum_m w_m (|theta_m + t_j d_m| - |theta_m|) for t = 1 (slot 0) and the Armijo trial steps (slots 1..)
hipError_t launch_pen_trials(long long p, const double* theta, const double* d, const double* pen_w, double alpha,
                             int no_l1, int j0, double* partials, int* nblk_out, hipStream_t s);
// data checks, per-block maxima of 4 indicators: non-finite y, negative y (Poisson),
// negative or non-finite a, non-positive or non-finite pen_w
// out (dims d[q0], d[q1], d[q2]) = in (dims d) with its axes permuted: out[i'] = in[i], i[q_k] = i'_k
hipError_t launch_permute3(const double* in, double* out, const int64_t* dims, const int* q, hipStream_t s);
// modes 1 and 2 of a d = 3 problem fit the slab kernels in this order (why: the reason if not)
bool rho_order_fits(const int64_t* n, const int64_t* p, int dtype, std::string* why);
// the same for elements of es bytes (8, 4 or 2), moved as raw bits
hipError_t launch_permute3_es(int es, const void* in, void* out, const int64_t* dims, const int* q, hipStream_t s);
hipError_t launch_scad_weights(long long p, const double* theta, const double* base, double lambda, double a, double* w,
                               hipStream_t s);
hipError_t launch_check(long long n, const double* y, const double* a, long long p, const double* pen_w, int family,
                        double* partials, int* nblk_out, hipStream_t s);

// ---- generic rho GEMMs and the elementwise steps on standard layouts (general.hip) ----
// C[m + ldc n] (+)= sum_k A[k + lda m] B[k + ldb n] (m < M, n < N, k < K) on the matrix cores,
// operands in dtype dt; out_kind 0: C in dt, 1: C in the accumulation type (FP32 for BF16/F32,
// FP64 for F64); acc: add into C.
hipError_t launch_rho_gemm(int dt, int out_kind, bool acc, long long M, long long N, long long K, const void* A,
                           long long lda, const void* B, long long ldb, void* C, long long ldc, hipStream_t s);
// the same with optional epilogue terms: C = (product + Cadd) .* Vmul, Cadd and Vmul in the accumulation
// type (either may be NULL; Cadd may equal C); out_kind 0 then writes dtype dt
hipError_t launch_rho_gemm_ex(int dt, int out_kind, long long M, long long N, long long K, const void* A,
                              long long lda, const void* B, long long ldb, void* C, long long ldc, const void* Cadd,
                              const void* Vmul, hipStream_t s);
// R = V .* (H(X, Theta) + Cadd) in dt (Cadd, V in the accumulation type, optional)
hipError_t general_forward_weighted(int dt, const int64_t* n, const int64_t* p, const void* const* XT,
                                    const void* theta, void* t1, void* t2, const void* Cadd, const void* V, void* R,
                                    hipStream_t s);
// eta (+)= H(X, Theta) by three GEMMs in the cyclic mode order; XT[j] = X_j^T (p_j x n_j, k-contiguous)
// in dt; t1, t2: >= general_tmp_elems elements of dt; eta in the accumulation type
hipError_t general_forward(int dt, const int64_t* n, const int64_t* p, const void* const* XT, const void* theta,
                           void* t1, void* t2, void* eta, bool acc, hipStream_t s);
// out = G(X, U); X[j] n_j x p_j in dt; out in the accumulation type
hipError_t general_adjoint(int dt, const int64_t* n, const int64_t* p, const void* const* X, const void* u, void* t1,
                           void* t2, void* out, hipStream_t s);
long long general_tmp_elems(const int64_t* n, const int64_t* p);
// dst = src (FP64) in dt; out = X^T (n x p FP64 -> p x n in dt)
hipError_t launch_gen_pack(int dt, long long count, const double* src, void* dst, hipStream_t s);
hipError_t launch_gen_transpose(int dt, long long nr, long long pc, const double* X, void* out, hipStream_t s);
// the same for X already in dt
hipError_t launch_gen_transpose_same(int dt, long long nr, long long pc, const void* X, void* out, hipStream_t s);
// family step on FP64 eta: u (adj_dt), weights (v_dt, optional), partials {sum -l, max w}
hipError_t launch_gen_family(int adj_dt, int v_dt, long long n, int family, const double* eta, const double* y,
                             const double* a, void* u_out, void* v_out, double* part, int* nblk, hipStream_t s);
// workgroups of the generic elementwise kernels for n elements (their partial-row count)
int gen_grid_blocks(long long n);
// g = scale gin (FP64); partials {max KKT residual, max |g|/w, sum w (l1 |theta| + alpha theta^2)}
hipError_t launch_gen_grad_stats(long long p, const double* gin, double scale, const double* theta, const double* w,
                                 double lambda, double alpha, int no_l1, double* gout, double* part, int* nblk,
                                 hipStream_t s);
// one inner step in place (x^{l-1} <- x^l, x^l <- x^{l+1}, gp <- grad h(x^l)), inc = x^{l+1} - theta_ref in dt;
// partials {max KKT at x^l, max |scale gi|, restart test sum, max |x^{l+1} - theta_ref|}
hipError_t launch_gen_prox(int dt, long long p, const void* gi, double scale, const double* gref,
                           const double* theta_ref, const double* w, double* x, double* xp, double* gp, void* inc,
                           double lambda, double delta, double om, double alpha, int no_l1, double* part, int* nblk,
                           hipStream_t s);
// One FP32 increment-state step of the generic path (BF16 / FP32 chains, nu = 1), applied by the last
// product of a component's adjoint chain to its output tile (general_adjoint_step).  Arrays in the
// standard coefficient layout, offset to the component's block: x^l = theta_ref + d^l (d FP32, an
// exact zero kept as a NaN code), grad h(x^{l-1}) = gref + q; writes d^{l+1}, q (in place) and
// inc = x^{l+1} - theta_ref in the chain dtype; partial rows {max KKT residual at x^l, max
// |scale gi|, restart test sum, max |x^{l+1} - theta_ref|}.
struct GenStepParams {
  double scale;                // gi -> increment gradient (1 / n)
  const double* gref;          // grad h(theta_ref)
  const double* theta_ref;
  const double* w;             // penalty weights or NULL (all 1)
  const float* dcur;           // d^l
  const float* dprev;          // d^{l-1}
  float* q;
  float* dout;                 // d^{l+1}
  void* inc;
  double lambda, delta, om, alpha;
  int no_l1;
  double* part;                // partial rows, 4 doubles each
};
// the adjoint chain of one component with the step fused into its last product (or, when that
// product has too few workgroups, written to gi, FP32, and followed by a standalone step); *nblk:
// partial rows
hipError_t general_adjoint_step(int dt, const int64_t* n, const int64_t* p, const void* const* X, const void* u,
                                void* t1, void* t2, void* gi, const GenStepParams& S, int* nblk, hipStream_t s);
// partial rows general_adjoint_step writes for a component with these sizes
long long general_step_rows(const int64_t* p);
// whether general_adjoint_step fuses the step into the last product for these sizes
bool general_step_fused(const int64_t* p);
// the standalone step over pc coefficients from gi (FP32); *nblk: partial rows
hipError_t launch_gen_step(int dt, long long pc, const void* gi, const GenStepParams& S, int* nblk, hipStream_t s);
// out = theta_ref + d (sub = 0) or that minus theta_ref (sub = 1), FP64
hipError_t launch_gen_inc_out(long long p, const float* d, const double* theta_ref, int sub, double* out,
                              hipStream_t s);
struct GenBtState {
  double* x;    // x^l
  double* xp;   // x^{l-1}
  double* gp;   // grad h(x^{l-1})
  double* y;    // y_{l-1}, the point the step into x^l started from
  double* gy;   // grad h(y_{l-1})
};
hipError_t launch_gen_prox_bt(int dt, long long p, const void* gi, double scale, const double* gref,
                              const double* theta_ref, const double* w, const GenBtState& cur, const GenBtState& nxt,
                              void* inc, double lambda, double delta, double om, double alpha, int no_l1, double* part,
                              int* nblk, hipStream_t s);
hipError_t launch_gen_bt_redo(int dt, long long p, const double* y, const double* gy, const double* w,
                              const double* theta_ref, double lambda, double delta, double alpha, int no_l1, double* x,
                              void* inc, hipStream_t s);
constexpr int kGenMaxBlocks = 4096;   // workgroups of the generic elementwise kernels (rows of partials)

// Gram matrix X^T X of a host n x p column-major matrix, and the largest eigenvalue of a
// symmetric p x p matrix (Proposition 1's spectral radii), both on the host (fit.cpp)
std::vector<double> gram_matrix(const double* X, int n, int p);
double gram_spectral_radius(std::vector<double> A, int p);

constexpr int kArmijoMaxBlocks = 2048;     // workgroups of k_armijo (rows of trial partials)
constexpr int kPenTrialsMaxBlocks = 256;   // workgroups of k_pen_trials
constexpr int ARMIJO_TRIALS = 16;   // step sizes 2^-j0 .. 2^-(j0+15) evaluated in one pass

}  // namespace glam
