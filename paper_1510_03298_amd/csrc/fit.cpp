// fit.cpp -- glam_fit_path: the GD-PG lambda path (Sec. 3, Algorithm 1; Sec. 6.4)
// on one gfx950 GPU.
//
// Per lambda, the outer loop of Algorithm 1 runs with FP64 anchors:
//   step 2 : FP64 chain at theta^k -> eta^k, weights V (eq. nine), score u
//            (eq. four), -l/n, and the FP64 gradient g^k = -G(U)/n, whose KKT
//            residual is the convergence criterion;
//   step 3 : delta = 1 / (nu Lhat), Lhat of Proposition 1;
//   step 4 : inner PG loop (Sec. 3.2) in the chosen dtype on the increment:
//            grad h(x) = g^k + G(V .* H(x - theta^k)) / n  (exact because h is
//            quadratic and grad h(theta^k) = g^k), with FISTA extrapolation;
//   step 5 : Armijo rule on FP64 reductions (F differences along t d); for the exact
//            Gaussian model (no prior weights) the inner solution is taken as is.
// The low-precision chain only ever sees the increment x - theta^k, and every
// outer iteration re-anchors at an FP64 gradient: this is the residual
// correction that lets FP32/BF16 rho products reach an FP64-certified KKT.
// Around it: the inner forms of Sec. 6.2 (Gram factors, tensor-product weights),
// the elastic net and SCAD (MSA steps) penalties, precision escalation
// (BF16 -> FP32 -> FP64) and the choice of mode order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "general.h"
#include "glam.h"
#include "launch.h"

namespace glam {

// Gram matrix X^T X (X host, n x p column-major), p x p.
std::vector<double> gram_matrix(const double* X, int n, int p) {
  std::vector<double> A((size_t)p * p, 0.0);
  for (int a = 0; a < p; ++a)
    for (int b = a; b < p; ++b) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += X[(size_t)a * n + i] * X[(size_t)b * n + i];
      A[(size_t)a * p + b] = s;
      A[(size_t)b * p + a] = s;
    }
  return A;
}

// Largest eigenvalue of a symmetric p x p matrix by cyclic Jacobi rotations
// (Proposition 1 needs rho(X_j^T X_j)).
double gram_spectral_radius(std::vector<double> A, int p) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int a = 0; a < p; ++a) {
      diag += A[(size_t)a * p + a] * A[(size_t)a * p + a];
      for (int b = a + 1; b < p; ++b) off += A[(size_t)a * p + b] * A[(size_t)a * p + b];
    }
    if (off <= 1e-30 * diag) break;
    for (int a = 0; a < p; ++a)
      for (int b = a + 1; b < p; ++b) {
        const double apq = A[(size_t)a * p + b];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = A[(size_t)a * p + a], aqq = A[(size_t)b * p + b];
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < p; ++k) {
          const double akp = A[(size_t)k * p + a], akq = A[(size_t)k * p + b];
          A[(size_t)k * p + a] = c * akp - s * akq;
          A[(size_t)k * p + b] = s * akp + c * akq;
        }
        for (int k = 0; k < p; ++k) {
          const double apk = A[(size_t)a * p + k], aqk = A[(size_t)b * p + k];
          A[(size_t)a * p + k] = c * apk - s * aqk;
          A[(size_t)b * p + k] = s * apk + c * aqk;
        }
      }
  }
  double m = 0.0;
  for (int a = 0; a < p; ++a) m = std::max(m, A[(size_t)a * p + a]);
  return m;
}


// Families whose IRLS weight (eq. nine) varies with eta: the inner chain then reads V.
static bool family_has_weights(int family) { return family == GLAM_POISSON || family == GLAM_BINOMIAL; }

// A low-precision inner loop whose best KKT residual has not halved over this many checks
// leaves for an FP64 re-anchor.  Where the model is the objective (the Gaussian model without
// prior weights: its inner solution is the step, no line search) a re-anchor costs one FP64
// family step and restarts the extrapolation: 10 checks measured 23% faster than 20 on the
// Gaussian n = (100, 100, 1000) path (and 50% slower on an ill-conditioned design whose slow
// but steady passes it cuts short).  Elsewhere each re-anchor also runs the Armijo rule, and
// 20 checks measured faster (Poisson n = (64, 64, 365) path: 1.02 s against 1.22 s).  The
// batched solver uses 10.
constexpr int kStallChecks = 10;
constexpr int kStallChecksLineSearch = 20;

static const double kEps[3] = {1.1102230246251565e-16, 5.960464477539063e-08, 3.90625e-03};

// Device memory and pinned host memory carved from a few large allocations.  A fit holds
// some thirty buffers; with one allocation call each, the set-up of a batch of small fits
// was dominated by the calls.  Shared by the fits of a batch; freed when the last owner
// goes (after the fits have synchronised their streams).
struct Arena {
  static constexpr size_t kDevChunk = (size_t)32 << 20, kHostChunk = (size_t)256 << 10;
  std::vector<void*> dev, host;
  std::mutex mu;   // the fits of a batch are set up from several host threads
  char* dcur = nullptr;
  size_t dleft = 0;
  char *hcur = nullptr, *hdcur = nullptr;   // host chunk and its device-side address
  size_t hleft = 0;
  Arena() = default;
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  ~Arena() {
    for (void* p : dev) (void)hipFree(p);
    for (void* p : host) (void)hipHostFree(p);
  }
  static size_t round_up(size_t b) { return (std::max<size_t>(b, 256) + 255) & ~(size_t)255; }
  // 256-byte aligned device buffer, or NULL
  void* dev_alloc(size_t bytes) {
    std::lock_guard<std::mutex> lock(mu);
    bytes = round_up(bytes);
    if (bytes > dleft) {
      void* p = nullptr;
      const bool own = bytes >= kDevChunk / 2;   // a large buffer takes an allocation of its own
      if (hipMalloc(&p, own ? bytes : kDevChunk) != hipSuccess) return nullptr;
      dev.push_back(p);
      if (own) return p;
      dcur = (char*)p;
      dleft = kDevChunk;
    }
    void* r = dcur;
    dcur += bytes;
    dleft -= bytes;
    return r;
  }
  // 256-byte aligned pinned host buffer (mapped, coherent) and its device address, or NULL
  void* host_alloc(size_t bytes, void** dev_addr) {
    std::lock_guard<std::mutex> lock(mu);
    bytes = round_up(bytes);
    if (bytes > hleft) {
      const size_t sz = std::max(bytes, kHostChunk);
      void *p = nullptr, *d = nullptr;
      if (hipHostMalloc(&p, sz, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) return nullptr;
      host.push_back(p);
      if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) return nullptr;
      hcur = (char*)p;
      hdcur = (char*)d;
      hleft = sz;
    }
    void* r = hcur;
    if (dev_addr) *dev_addr = hdcur;
    hcur += bytes;
    hdcur += bytes;
    hleft -= bytes;
    return r;
  }
};

struct Fit {
  Geom G;
  int dt;
  hipStream_t s;
  int family;
  const glam_problem* prob;
  // device and pinned host buffers (from the arena, which may be shared with other fits)
  std::shared_ptr<Arena> arena;
  void* imgc;              // LDS image of X1, X2 in the chain dtype
  void* imgd;              // LDS image of X1, X2 in FP64
  void *X3fc, *X3ac;       // chain-dtype packed mode-3 factor (slab_fwd / slab_adj operands)
  double *X3fd, *X3ad;     // FP64 packed mode-3 factor
  double* thpk;            // FP64 k-blocked copy of theta (or of a direction)
  double *y_int, *a_int, *eta_int, *xd_int;
  void* v_int;             // tiled weights (acc type of the chain) or NULL (Gaussian)
  void *T1c, *S2c;         // chain dtype intermediates
  bool gram = false;       // inner gradient by the Kronecker Gram factors (Sec. 6.2)
  double enet = 0.0;       // elastic-net weight alpha (Sec. 6.3): J = sum w (|theta| + alpha theta^2)
  int no_l1 = 0;           // the ridge penalty (Sec. 6.3): J = sum w theta^2 (enet = 1, no l1 term)
  const double* pen = nullptr;   // penalty weights the kernels read (the caller's, or the SCAD steps' own)
  double *S1g = nullptr, *S2g = nullptr;   // X_1^T X_1, X_2^T X_2 (FP64)
  void* S3c = nullptr;     // X_3^T X_3, k-blocked (K = C = p3), chain dtype
  void* Zc = nullptr;      // S_1 D S_2 per slice, k-blocked like the increment
  double* S3g = nullptr;   // X_3^T X_3 (FP64)
  bool kron = false;       // Gram factors reweighted each outer step with tensor-product weights (Sec. 6.2)
  bool unit_w = false;     // unit IRLS weights in the model of every family (the Gram form with W = I)
  double* kron_work = nullptr;    // log-weight margins and the factors v_j
  bool kron_first = true;         // the power method of the Gram factors starts from ones
  double* kron_stats = nullptr;   // {max v_1, max v_2, max v_3, Vbar} (device)
  bool gram_fused = false; // Gram iteration as one launch (k_gram_iter): increment and counter double-buffered
  void* inc2 = nullptr;    // the second increment buffer
  int gpar = 0;            // which of (inc, inc2) / (iter[0], iter[1]) holds the current increment / counter
  Geom Gg{};               // geometry of the mode-3 Gram product (contraction length p3)
  double *T1d, *S2d;       // FP64 intermediates
  double *theta, *gref, *x, *xp, *gp, *dvec;
  double *yb = nullptr, *gyb = nullptr;                     // backtracking: y_{l-1}, grad h(y_{l-1})
  double *x2 = nullptr, *xp2 = nullptr, *gp2 = nullptr, *yb2 = nullptr, *gyb2 = nullptr;   // next state
  void* inc;
  int* iter;
  double* part;            // partial sums
  double* red;             // reduced values (device)
  double* hred = nullptr;  // reduced values (pinned host); [32..35] input-check flags, [40..42] kkt_at_lambda
  double* hred_dev = nullptr;   // its device address: the reductions of steps 2 and 5 write there directly
  size_t npart = 0;             // doubles in part
  double* hx[3] = {nullptr, nullptr, nullptr};   // pinned host copies of the factors (set-up)
  double* hpub = nullptr;  // published check values (fine-grained pinned host, mapped)
  double* hpub_dev = nullptr;
  unsigned* hseq = nullptr;       // published sequence number (host view) ...
  unsigned* hseq_dev = nullptr;   // ... and its device address
  unsigned* seq_dev = nullptr;    // device-side counter of published checks
  unsigned seq_expect = 0;
  double sprod;            // prod_j rho(X_j^T X_j)
  std::string err;
  hipEvent_t ev[8] = {};   // sampled kernel timing
  hipStream_t us = nullptr;        // caller's stream
  bool own_stream = false;
  bool batched = false;            // set up for glam_fit_batched (its batched step uses the LDS image)
  hipEvent_t sync_ev = nullptr;
  double* dparams = nullptr;       // device {lambda, delta, -, -, lambda scale, tol_in, 4 eps} (8 slots)
  double* hparams = nullptr;       // pinned host staging of dparams
  // run-ahead inner loop (the increment-state chain loop): the next block of iterations is queued
  // before the host has read the current block's check; the reduction of each block tests
  // convergence on the device and sets *stop, after which the queued kernels do nothing
  bool runahead = false;
  int* stop = nullptr;
  // eta of the outer steps is written out only where it is read: the Armijo passes (every model
  // but the exact Gaussian one) and the tensor-product weights
  bool keep_eta = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_m = 0;                 // inner iterations per graph replay
  // the BF16 / FP32 chain loop (nu = 1) keeps its iterate as FP32 increments (AdjIncParams);
  // its two increment buffers alternate, so a block replayed from the second buffer has a
  // graph of its own
  bool incst = false;
  // restarted extrapolation sequence (the chain loop with nu = 1): at each check, a positive
  // (y - x^{l+1})^T (x^{l+1} - x^l) sets the step counter back (omega = 0 next)
  bool restart = false;
  double *tT = nullptr, *gT = nullptr, *penT = nullptr;
  float* dst[2] = {nullptr, nullptr};
  float* qst = nullptr;
  hipGraph_t graph1 = nullptr;
  hipGraphExec_t gexec1 = nullptr;
  int graph1_m = 0;
  // sampled re-runs of the step kernel write here (the fit's own state is left untouched)
  float *dS = nullptr, *qS = nullptr;
  void* incS = nullptr;
  double* partS = nullptr;
  double adj_ms = 0.0, fwd_ms = 0.0;
  bool pending = false;
  double chain_ms = 0.0, iter_ms = 0.0;
  int samples = 0;

  void* alloc(size_t bytes) {
    if (!arena) arena = std::make_shared<Arena>();
    return arena->dev_alloc(bytes);
  }
  double* host_alloc(size_t count, double** dev_addr = nullptr) {
    if (!arena) arena = std::make_shared<Arena>();
    return (double*)arena->host_alloc(count * sizeof(double), (void**)dev_addr);
  }
  Fit() = default;
  Fit(const Fit&) = delete;
  Fit& operator=(const Fit&) = delete;
  ~Fit() {
    if (s) (void)hipStreamSynchronize(s);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (gexec1) (void)hipGraphExecDestroy(gexec1);
    if (graph1) (void)hipGraphDestroy(graph1);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (sync_ev) (void)hipEventDestroy(sync_ev);
    if (own_stream && s) (void)hipStreamDestroy(s);
    arena.reset();   // the buffers go with the last owner of the arena
  }
};

struct StepStats {
  double nll;       // -l/n at theta^k
  double vmax;      // max weight
  double kkt_raw;   // max KKT residual (absolute)
  double lmax_raw;  // max |g|/w
  double pen;       // sum w |theta|
};

#define FCHK(expr)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) {                                                                \
      F.err = std::string(#expr) + ": " + hipGetErrorString(e_);                           \
      return GLAM_EDEVICE;                                                                 \
    }                                                                                      \
  } while (0)

// Step 2 of Algorithm 1 at theta (FP64): eta, V, -l/n, g = -G(U)/n, KKT.
// Enqueue step 2 of Algorithm 1 at theta (values land in F.hred, written by the reductions
// themselves through its mapped address, after the stream
// completes); family_collect reads them.
static int family_enqueue(Fit& F, const double* theta_dev, double lambda) {
  const Geom& G = F.G;
  FCHK(launch_pack(DT_F64, DT_F64, theta_dev, G.p3, G.P12, G.P12, 1, F.thpk, F.s));
  FwdParams fw{};
  fw.G = G; fw.theta = F.thpk; fw.X3f = F.X3fd; fw.T1 = F.T1d;
  FCHK(launch_slab_fwd(DT_F64, fw, F.s));
  SlabParams sp{};
  sp.G = G; sp.img = F.imgd; sp.T1 = F.T1d; sp.S2 = F.S2d;
  sp.y_int = F.y_int; sp.a_int = F.prob->obs_w ? F.a_int : nullptr; sp.eta_int = F.keep_eta ? F.eta_int : nullptr;
  sp.v_out = F.v_int; sp.v_out_f32 = F.dt != DT_F64; sp.family = F.family; sp.partials = F.part;
  int nbc = 0;
  FCHK(launch_slab_chain(DT_F64, SM_FAMILY, sp, &nbc, F.s));
  const int ops2[2] = {0, 1};
  FCHK(launch_reduce(F.part, nbc, 2, ops2, 1.0 / (double)G.n, F.hred_dev, F.s));
  AdjParams ap{};
  ap.G = G; ap.S2 = F.S2d; ap.X3a = F.X3ad; ap.scale = -1.0 / (double)G.n; ap.gout = F.gref;
  ap.theta = theta_dev; ap.pen_w = F.pen; ap.lambda = lambda; ap.alpha = F.enet; ap.no_l1 = F.no_l1;
  double* part2 = F.part + (size_t)2 * nbc;
  ap.partials = part2;
  int nb = 0;
  FCHK(launch_slab_adj(DT_F64, EPI_GRAD, ap, &nb, F.s));
  const int ops4[4] = {1, 1, 0, 0};
  FCHK(launch_reduce_strided(part2, nb, ADJ_NSUM, 4, ops4, 1.0, F.hred_dev + 2, F.s));
  return GLAM_OK;
}

static void family_collect(const Fit& F, StepStats* st) {
  st->nll = F.hred[0];
  st->vmax = F.hred[1];
  st->kkt_raw = F.hred[2];
  st->lmax_raw = F.hred[3];
  st->pen = F.hred[4];
}

static int family_step(Fit& F, const double* theta_dev, double lambda, StepStats* st) {
  const int r = family_enqueue(F, theta_dev, lambda);
  if (r) return r;
  FCHK(hipStreamSynchronize(F.s));
  family_collect(F, st);
  return GLAM_OK;
}

// Step 2 of Algorithm 1 at the theta of the last family step, for a new lambda with the same
// penalty weights (the first outer step of the next model on the path): eta, V, -l/n, the
// gradient and the penalty sum are those of that step, so only the KKT residual is evaluated
// again, from the stored gradient (the same expression as the gradient epilogue, hence the same
// value).  Returns false when the partials buffer is too small (the caller takes the full step).
static int kkt_at_lambda(Fit& F, double lambda, const StepStats& last, StepStats* st, bool* done) {
  const Geom& G = F.G;
  *done = false;
  if ((size_t)3 * gen_grid_blocks(G.p) > F.npart) return GLAM_OK;
  int nb = 0;
  FCHK(launch_gen_grad_stats(G.p, F.gref, 1.0, F.theta, F.pen, lambda, F.enet, F.no_l1, nullptr, F.part, &nb, F.s));
  const int ops[3] = {1, 1, 0};
  FCHK(launch_reduce(F.part, nb, 3, ops, 1.0, F.hred_dev + 40, F.s));   // hred[40..42]
  FCHK(hipStreamSynchronize(F.s));
  *st = last;
  st->kkt_raw = F.hred[40];
  *done = true;
  return GLAM_OK;
}

constexpr int kSampleReps = 8;   // back-to-back launches of the fused slab kernel per timing sample

// One inner PG iteration (Sec. 3.2) in the chain dtype.
static int inner_iteration(Fit& F, double lambda, double delta, int* nblk, bool sample) {
  const Geom& G = F.G;
  if (sample) FCHK(hipEventRecord(F.ev[0], F.s));
  if (F.gram && F.gram_fused) {
    // grad h(x) = g_ref + (S_3 (x) S_2 (x) S_1) vec(x - theta_ref) / n (Sec. 6.2, W = I) and the
    // proximal step, one launch; reads the current increment / counter, writes the other pair
    GramIterParams gp{};
    gp.G = G; gp.S1 = F.S1g; gp.S2 = F.S2g; gp.S3 = F.S3g;
    gp.inc_in = F.gpar ? F.inc2 : F.inc; gp.inc_out = F.gpar ? F.inc : F.inc2;
    gp.iter_in = F.iter + F.gpar; gp.iter_out = F.iter + (1 - F.gpar);
    gp.gref = F.gref; gp.theta_ref = F.theta; gp.pen_w = F.pen; gp.x = F.x; gp.xp = F.xp; gp.gp = F.gp;
    gp.dparams = F.dparams; gp.alpha = F.enet; gp.no_l1 = F.no_l1; gp.scale = 1.0 / (double)G.n; gp.partials = F.part;
    FCHK(launch_gram_iter(F.dt, gp, nblk, F.s));
    F.gpar ^= 1;
    if (sample) {   // iteration time only
      FCHK(hipEventRecord(F.ev[1], F.s));
      FCHK(hipEventRecord(F.ev[2], F.s));
      FCHK(hipEventRecord(F.ev[3], F.s));
      F.pending = true;
    }
    return GLAM_OK;
  }
  if (F.gram) {
    // grad h(x) = g_ref + (S_3 (x) S_2 (x) S_1) vec(x - theta_ref) / n (Sec. 6.2, W = I)
    FCHK(launch_gram12(F.dt, G, F.inc, F.S1g, F.S2g, F.Zc, F.iter, F.s));
    AdjParams ap{};
    ap.G = F.Gg; ap.S2 = F.Zc; ap.X3a = F.S3c; ap.scale = 1.0 / (double)G.n; ap.pen_w = F.pen; ap.alpha = F.enet; ap.no_l1 = F.no_l1;
    ap.lambda = lambda; ap.partials = F.part; ap.gref = F.gref; ap.theta_ref = F.theta; ap.x = F.x; ap.xp = F.xp;
    ap.gp = F.gp; ap.inc = F.inc; ap.iter = F.iter; ap.delta = delta; ap.dparams = F.dparams;
    FCHK(launch_slab_adj(F.dt, EPI_PROX, ap, nblk, F.s));
    if (sample) {   // iteration time only (there is no rho chain in this iteration)
      FCHK(hipEventRecord(F.ev[1], F.s));
      FCHK(hipEventRecord(F.ev[2], F.s));
      FCHK(hipEventRecord(F.ev[3], F.s));
      F.pending = true;
    }
    return GLAM_OK;
  }
  const bool incst = F.incst && F.dt != DT_F64;
  const int* stop = incst && F.runahead ? F.stop : nullptr;
  FwdParams fw{};
  fw.G = G; fw.theta = F.inc; fw.X3f = F.X3fc; fw.T1 = F.T1c; fw.iter = F.iter; fw.stop = stop;
  FCHK(launch_slab_fwd(F.dt, fw, F.s));
  SlabParams sp{};
  sp.G = G; sp.img = F.imgc; sp.T1 = F.T1c; sp.S2 = F.S2c; sp.v_int = F.v_int; sp.stop = stop;
  FCHK(launch_slab_chain(F.dt, SM_FUSED, sp, nullptr, F.s));
  if (incst) {
    // x^{l+1} from x^l = theta_ref + d[gpar] and x^{l-1} = theta_ref + d[1 - gpar], written over
    // the latter (AdjIncParams)
    AdjIncParams ai{};
    ai.G = G; ai.S2 = F.S2c; ai.X3a = F.X3ac; ai.s2_kb4 = chain_s2_kb4(F.dt, SM_FUSED, G);
    ai.gT = F.gT; ai.tT = F.tT; ai.penT = F.pen ? F.penT : nullptr;
    ai.dcur = F.dst[F.gpar]; ai.dprev = F.dst[1 - F.gpar]; ai.dout = F.dst[1 - F.gpar];
    ai.q_in = F.qst; ai.q_out = F.qst; ai.inc = F.inc; ai.iter = F.iter; ai.dparams = F.dparams;
    ai.scale = 1.0 / (double)G.n; ai.alpha = F.enet; ai.no_l1 = F.no_l1; ai.partials = F.part; ai.xmap = kAdjIncForm;
    ai.stop = stop;
    FCHK(launch_slab_adj_inc(F.dt, ai, nblk, F.s));
    F.gpar ^= 1;
    if (sample) {
      // the whole iteration between ev[0] and ev[1]; then each of its three kernels re-run
      // kSampleReps times back to back on this iteration's own inputs: slab_fwd (no counter
      // step) and slab_chain rewrite identical T1 and S2, the step kernel writes its outputs
      // into scratch buffers
      FCHK(hipEventRecord(F.ev[1], F.s));
      FCHK(hipEventRecord(F.ev[2], F.s));
      for (int r = 0; r < kSampleReps; ++r) FCHK(launch_slab_chain(F.dt, SM_FUSED, sp, nullptr, F.s));
      FCHK(hipEventRecord(F.ev[3], F.s));
      ai.dout = F.dS; ai.q_out = F.qS; ai.inc = F.incS; ai.partials = F.partS;
      for (int r = 0; r < kSampleReps; ++r) FCHK(launch_slab_adj_inc(F.dt, ai, nullptr, F.s));
      FCHK(hipEventRecord(F.ev[4], F.s));
      fw.iter = nullptr;
      for (int r = 0; r < kSampleReps; ++r) FCHK(launch_slab_fwd(F.dt, fw, F.s));
      FCHK(hipEventRecord(F.ev[5], F.s));
      F.pending = true;
    }
    return GLAM_OK;
  }
  AdjParams ap{};
  ap.G = G; ap.S2 = F.S2c; ap.X3a = F.X3ac; ap.scale = 1.0 / (double)G.n; ap.pen_w = F.pen;
  ap.alpha = F.enet; ap.no_l1 = F.no_l1; ap.lambda = lambda; ap.partials = F.part; ap.gref = F.gref; ap.theta_ref = F.theta; ap.x = F.x; ap.xp = F.xp;
  ap.gp = F.gp; ap.inc = F.inc; ap.iter = F.iter; ap.delta = delta; ap.dparams = F.dparams;
  ap.s2_kb4 = chain_s2_kb4(F.dt, SM_FUSED, G);
  FCHK(launch_slab_adj(F.dt, EPI_PROX, ap, nblk, F.s));
  if (sample) {
    // the whole iteration between ev[0] and ev[1]; then the fused slab kernel alone,
    // re-run kSampleReps times back to back on this iteration's own T1 (it rewrites
    // the same S2, which only the next iteration's own slab kernel overwrites)
    FCHK(hipEventRecord(F.ev[1], F.s));
    FCHK(hipEventRecord(F.ev[2], F.s));
    for (int r = 0; r < kSampleReps; ++r) FCHK(launch_slab_chain(F.dt, SM_FUSED, sp, nullptr, F.s));
    FCHK(hipEventRecord(F.ev[3], F.s));
    F.pending = true;
  }
  return GLAM_OK;
}

// Accumulate the durations of the last sampled inner iteration (events are complete
// after the stream synchronisation of the convergence check).
static int collect_sample(Fit& F) {
  if (!F.pending) return GLAM_OK;
  const bool three = F.incst && F.dt != DT_F64 && !F.gram;   // the step kernel and slab_fwd sampled too
  FCHK(hipEventSynchronize(F.ev[three ? 5 : 3]));
  float a = 0.f, b = 0.f;
  FCHK(hipEventElapsedTime(&a, F.ev[2], F.ev[3]));
  FCHK(hipEventElapsedTime(&b, F.ev[0], F.ev[1]));
  F.chain_ms += a / kSampleReps;
  F.iter_ms += b;
  if (three) {
    float c = 0.f, d = 0.f;
    FCHK(hipEventElapsedTime(&c, F.ev[3], F.ev[4]));
    FCHK(hipEventElapsedTime(&d, F.ev[4], F.ev[5]));
    F.adj_ms += c / kSampleReps;
    F.fwd_ms += d / kSampleReps;
  }
  F.samples += 1;
  F.pending = false;
  return GLAM_OK;
}

// One block of m inner iterations followed by the reduction of the last
// iteration's partial KKT / noise maxima into F.red[0..3].  Captured once per fit
// as a HIP graph (the only per-lambda / per-outer values live in F.dparams).
static int inner_block_eager(Fit& F, int m, bool sample_first, int* nblk) {
  for (int q = 0; q < m; ++q) {
    int r = inner_iteration(F, 0.0, 0.0, nblk, sample_first && q == 0);
    if (r) return r;
  }
  const int ops[ADJ_NSUM] = {1, 1, 0, 0, 1, 0};
  const bool ra = F.runahead && F.incst && F.dt != DT_F64;
  FCHK(launch_reduce_publish(F.part, *nblk, ADJ_NSUM, ops, 1.0, F.red, F.hpub_dev, F.seq_dev, F.hseq_dev, F.s, 2,
                             F.restart ? F.iter : nullptr, ra ? F.stop : nullptr, ra ? F.dparams + 4 : nullptr));
  return GLAM_OK;
}

// Wait for the check values of the block just launched: the last kernel of the block
// writes them to mapped host memory, then the next sequence number.  The host spins on
// that number (no copy, no stream synchronisation) and queries the stream for errors.
static int wait_published(Fit& F, double* vals, int nval) {
  const unsigned want = ++F.seq_expect;
  // reached: the sequence number is at or past this block's (a block queued behind it may have
  // published too; its values sit in the other slot)
  auto reached = [&]() { return (int)(__atomic_load_n(F.hseq, __ATOMIC_ACQUIRE) - want) >= 0; };
  for (long long spin = 0;; ++spin) {
    if (reached()) break;
    if ((spin & 255) == 255) {
      const hipError_t e = hipStreamQuery(F.s);
      if (e == hipSuccess) {
        if (reached()) break;
        F.err = "check values were not published";
        return GLAM_EDEVICE;
      }
      if (e != hipErrorNotReady) {
        F.err = std::string("inner block: ") + hipGetErrorString(e);
        return GLAM_EDEVICE;
      }
    }
  }
  const volatile double* slot = F.hpub + 8 * (want & 1u);
  for (int v = 0; v < nval; ++v) vals[v] = slot[v];
  return GLAM_OK;
}

static void drop_graphs(Fit& F) {
  if (F.gexec) { (void)hipGraphExecDestroy(F.gexec); F.gexec = nullptr; }
  if (F.graph) { (void)hipGraphDestroy(F.graph); F.graph = nullptr; }
  if (F.gexec1) { (void)hipGraphExecDestroy(F.gexec1); F.gexec1 = nullptr; }
  if (F.graph1) { (void)hipGraphDestroy(F.graph1); F.graph1 = nullptr; }
  F.graph_m = F.graph1_m = 0;
}

static int inner_block_graph(Fit& F, int m, int* nblk) {
  // a fused Gram block alternates its buffers: replayable only from buffer 0 with even m
  if (F.gram_fused && (F.gpar != 0 || (m & 1))) return inner_block_eager(F, m, false, nblk);
  // the increment-state loop alternates its buffers too: one graph per starting buffer
  const bool inc = F.incst && F.dt != DT_F64;
  const bool second = inc && F.gpar == 1;
  hipGraph_t& graph = second ? F.graph1 : F.graph;
  hipGraphExec_t& gexec = second ? F.gexec1 : F.gexec;
  int& graph_m = second ? F.graph1_m : F.graph_m;
  if (!gexec || graph_m != m) {
    if (gexec) { (void)hipGraphExecDestroy(gexec); gexec = nullptr; }
    if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
    FCHK(hipStreamBeginCapture(F.s, hipStreamCaptureModeRelaxed));
    int r = inner_block_eager(F, m, false, nblk);   // (flips F.gpar as the replay will)
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(F.s, &g);
    if (r) { if (g) (void)hipGraphDestroy(g); return r; }
    FCHK(e);
    graph = g;
    FCHK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    graph_m = m;
  } else {
    *nblk = F.gram_fused ? gram_iter_blocks(F.dt, F.G) : inc ? slab_adj_inc_partials(F.G, kAdjIncForm) : slab_adj_blocks(F.G);
    if (inc && (m & 1)) F.gpar ^= 1;
  }
  FCHK(hipGraphLaunch(gexec, F.s));
  return GLAM_OK;
}

// Inner PG loop with step control nu < 1 (Sec. 6.4): delta starts at
// 1/(nu Lhat); each iteration also tests the Beck-Teboulle sufficient decrease of the
// step that produced the current iterate and, if it fails, halves delta (never below
// 1/Lhat) and redoes that step.  The host checks every iteration.
static int inner_loop_bt(Fit& F, double lam, double delta0, double Lhat, double tol_in, int max_inner,
                         double lam_scale, double* kin_out, int* it_out) {
  const Geom& G = F.G;
  double delta = delta0;
  const double delta_min = 1.0 / Lhat;
  // state at l = 1: x = xp = theta^k, gp = grad h(theta^k); y_0 := x^1 (no test at l = 1)
  FCHK(hipMemcpyAsync(F.yb, F.theta, G.p * 8, hipMemcpyDeviceToDevice, F.s));
  FCHK(hipMemcpyAsync(F.gyb, F.gref, G.p * 8, hipMemcpyDeviceToDevice, F.s));
  double* cur[5] = {F.x, F.xp, F.gp, F.yb, F.gyb};
  double* nxt[5] = {F.x2, F.xp2, F.gp2, F.yb2, F.gyb2};
  int l = 1, it = 0, window_start = 0;
  double kin = INFINITY, best = INFINITY, window_best = INFINITY;
  while (it < max_inner) {
    F.hparams[0] = lam;
    F.hparams[1] = delta;
    F.hparams[2] = (double)l;
    FCHK(hipMemcpyAsync(F.dparams, F.hparams, 3 * sizeof(double), hipMemcpyHostToDevice, F.s));
    FwdParams fw{};
    fw.G = G; fw.theta = F.inc; fw.X3f = F.X3fc; fw.T1 = F.T1c;
    FCHK(launch_slab_fwd(F.dt, fw, F.s));
    SlabParams sp{};
    sp.G = G; sp.img = F.imgc; sp.T1 = F.T1c; sp.S2 = F.S2c; sp.v_int = F.v_int;
    FCHK(launch_slab_chain(F.dt, SM_FUSED, sp, nullptr, F.s));
    AdjParams ap{};
    ap.G = G; ap.S2 = F.S2c; ap.X3a = F.X3ac; ap.scale = 1.0 / (double)G.n; ap.pen_w = F.pen;
    ap.alpha = F.enet; ap.no_l1 = F.no_l1; ap.partials = F.part; ap.gref = F.gref; ap.theta_ref = F.theta; ap.inc = F.inc; ap.dparams = F.dparams;
    ap.x = cur[0]; ap.xp = cur[1]; ap.gp = cur[2]; ap.yprev = cur[3]; ap.gyprev = cur[4];
    ap.x_out = nxt[0]; ap.xp_out = nxt[1]; ap.gp_out = nxt[2]; ap.y_out = nxt[3]; ap.gy_out = nxt[4];
    ap.s2_kb4 = chain_s2_kb4(F.dt, SM_FUSED, G);
    int nb = 0;
    FCHK(launch_slab_adj(F.dt, EPI_PROX_BT, ap, &nb, F.s));
    const int ops[ADJ_NSUM] = {1, 1, 0, 0, 1, 0};
    FCHK(launch_reduce(F.part, nb, ADJ_NSUM, ops, 1.0, F.red, F.s));
    FCHK(hipMemcpyAsync(F.hred, F.red, ADJ_NSUM * sizeof(double), hipMemcpyDeviceToHost, F.s));
    FCHK(hipStreamSynchronize(F.s));
    ++it;
    const double sdg = F.hred[2], sdd = F.hred[3];
    if (l >= 2 && sdg > (sdd / delta) * (1.0 + 1e-12) && delta > delta_min * (1.0 + 1e-12)) {
      // divergence of the step into x^l detected: halve delta and redo that step from y_{l-1}
      delta = std::max(0.5 * delta, delta_min);
      FCHK(launch_bt_redo(F.dt, G, cur[3], cur[4], F.pen, F.theta, lam, delta, F.enet, F.no_l1, cur[0], F.inc, F.s));
      continue;
    }
    kin = F.hred[0] / lam_scale;
    for (int q = 0; q < 5; ++q) std::swap(cur[q], nxt[q]);
    ++l;
    if (!std::isfinite(kin)) break;
    const double noise = 4.0 * kEps[F.dt] * F.hred[1] / lam_scale;
    if (kin <= std::max(tol_in, noise)) break;
    best = std::min(best, kin);
    if (it - window_start >= 200) {
      if (!(best < 0.5 * window_best) && F.dt != DT_F64) break;   // stalled at the rounding floor
      window_best = best;
      window_start = it;
    }
  }
  // make the accepted x^l (now in cur[1]) available where the caller expects it (F.xp)
  if (cur[1] != F.xp) FCHK(hipMemcpyAsync(F.xp, cur[1], G.p * 8, hipMemcpyDeviceToDevice, F.s));
  *kin_out = kin;
  *it_out = it;
  return GLAM_OK;
}

// Continue a fit with the FP64 inner chain: the FP64 intermediates, factor copies and LDS
// image of the outer steps serve the inner loop from now on; the captured graph (built for
// the old dtype) is dropped.  V and the increment already have 8-byte elements.
static void escalate_f64(Fit& F) {
  F.dt = DT_F64;
  F.T1c = F.T1d; F.S2c = F.S2d; F.X3fc = F.X3fd; F.X3ac = F.X3ad; F.imgc = F.imgd;
  drop_graphs(F);
}

// Continue a BF16 fit with the FP32 inner chain (the intermediate rung before FP64): its
// intermediates, mode-3 factor copies and factor image are allocated and packed here, once.
static int escalate_f32(Fit& F) {
  const Geom& G = F.G;
  void* t1 = F.alloc(G.t1_len * 4);
  void* s2 = F.alloc(G.s2_len * 4);
  void* x3f = F.alloc(G.x3f_len * 4);
  void* x3a = F.alloc(G.x3a_len * 4);
  void* img = F.alloc(chain_image_bytes(DT_F32, G));
  if (!t1 || !s2 || !x3f || !x3a || !img) { F.err = "device allocation failed"; return GLAM_ENOMEM; }
  FCHK(launch_pack(DT_F32, DT_F64, F.prob->X[2], G.p3, G.n3, G.n3, 1, x3f, F.s));
  FCHK(launch_pack(DT_F32, DT_F64, F.prob->X[2], G.n3, G.p3, 1, G.n3, x3a, F.s));
  FCHK(launch_zero(s2, G.s2_len * 4, F.s));   // rows beyond n3 stay zero
  FCHK(launch_pack_chain_image(DT_F32, DT_F64, G, F.prob->X[0], F.prob->X[1], img, F.s,
                               chain_image_need(DT_F32, SM_FUSED, G)));
  F.dt = DT_F32;
  F.T1c = t1; F.S2c = s2; F.X3fc = x3f; F.X3ac = x3a; F.imgc = img;
  drop_graphs(F);
  return GLAM_OK;
}

// Armijo rule (Sec. 5): d = theta~ - theta^k (in F.dvec).  Returns alpha.
// Enqueue one pass of the Armijo rule (step sizes 2^-j0 .. 2^-(j0+15)) along d =
// F.dvec; j0 == 0 also computes H(d) in FP64 (the trials use eta + t H(d)).  The sums
// land in F.hred (written through its mapped address) after the stream completes;
// armijo_decide reads them.
static int armijo_enqueue(Fit& F, int j0) {
  const Geom& G = F.G;
  if (j0 == 0) {
    FCHK(launch_pack(DT_F64, DT_F64, F.dvec, G.p3, G.P12, G.P12, 1, F.thpk, F.s));
    FwdParams fw{};
    fw.G = G; fw.theta = F.thpk; fw.X3f = F.X3fd; fw.T1 = F.T1d;
    FCHK(launch_slab_fwd(DT_F64, fw, F.s));
    SlabParams sp{};
    sp.G = G; sp.img = F.imgd; sp.T1 = F.T1d; sp.eta_out = F.xd_int;
    FCHK(launch_slab_chain(DT_F64, SM_FWD_INT, sp, nullptr, F.s));
  }
  constexpr int NV = ARMIJO_TRIALS + 1;
  const int ops[NV] = {0};
  int nb1 = 0, nb2 = 0;
  FCHK(launch_armijo(G, F.family, F.eta_int, F.xd_int, F.y_int, F.a_int, j0, F.part, &nb1, F.s));
  FCHK(launch_reduce(F.part, nb1, NV, ops, 1.0 / (double)G.n, F.hred_dev, F.s));
  double* part2 = F.part + (size_t)nb1 * NV;
  FCHK(launch_pen_trials(G.p, F.theta, F.dvec, F.pen, F.enet, F.no_l1, j0, part2, &nb2, F.s));
  FCHK(launch_reduce(part2, nb2, NV, ops, 1.0, F.hred_dev + NV, F.s));
  return GLAM_OK;
}

// The first accepted trial of a pass: true with *alpha_out set, or false (try the next
// pass).  *delta_out = Delta of the rule (set on the first pass).
static bool armijo_decide(const Fit& F, int j0, double lambda, double v, double* alpha_out, double* delta_out) {
  constexpr int NV = ARMIJO_TRIALS + 1;
  const double* sm = F.hred;         // [0] = sum u xd / n ; [1+j] = smooth change / n
  const double* pj = F.hred + NV;    // [0] = J(theta~) - J(theta) ; [1+j] = J change at t_j
  if (j0 == 0) *delta_out = -sm[0] + lambda * pj[0];
  // The rule presumes a descent direction (Delta < 0; Sec. 5, the search direction of
  // Theorem 2).  A low-precision inner loop that ended on its rounding floor or stall rule
  // can return a point with Delta >= 0: no step is taken (alpha = 0), and the outer loop
  // counts it as a step that ended on the chain's floor (precision escalation).
  if (!(*delta_out < 0.0)) {
    *alpha_out = 0.0;
    return true;
  }
  for (int j = 0; j < ARMIJO_TRIALS; ++j) {
    const double t = std::ldexp(1.0, -(j0 + j));
    const double dF = sm[1 + j] + lambda * pj[1 + j];
    if (std::isfinite(dF) && dF <= t * v * *delta_out) {
      *alpha_out = t;
      return true;
    }
  }
  return false;
}

// Armijo rule from pass first_j0 on (the pass at first_j0 already enqueued when queued);
// alpha = 0 when no step size down to 2^-63 is accepted.
static int armijo_finish(Fit& F, double lambda, double v, bool queued, double* alpha_out, double* delta_out) {
  for (int j0 = 0; j0 < 64; j0 += ARMIJO_TRIALS) {
    if (!(queued && j0 == 0)) {
      const int r = armijo_enqueue(F, j0);
      if (r) return r;
    }
    FCHK(hipStreamSynchronize(F.s));
    if (armijo_decide(F, j0, lambda, v, alpha_out, delta_out)) return GLAM_OK;
  }
  *alpha_out = 0.0;
  return GLAM_OK;
}

static int armijo(Fit& F, double lambda, double v, double* alpha_out, double* delta_out) {
  *delta_out = 0.0;
  return armijo_finish(F, lambda, v, false, alpha_out, delta_out);
}

// Allocate the per-problem device state and enqueue the one-time setup kernels: input
// checks, tiled Y and a, packed factors (FP64 and chain dtype), LDS images, and host
// copies of the factors.  No host synchronisation: fit_setup_finish completes the set-up
// once the stream has run.  F.s, F.G and F.dt must be set.
static int fit_setup_enqueue(Fit& F, const glam_problem* prob, bool bt, bool events) {
  F.family = prob->family;
  F.prob = prob;
  F.pen = prob->pen_w;
  const Geom& G = F.G;
  const size_t es = dt_size(F.dt);
  const size_t accs = F.dt == DT_F64 ? 8 : 4;
  const size_t nadj = (size_t)slab_adj_blocks(G);
  const size_t npart = std::max<size_t>({(size_t)G.n3 * 2 + nadj * ADJ_NSUM, (size_t)(kArmijoMaxBlocks + kPenTrialsMaxBlocks) * (ARMIJO_TRIALS + 1),
                                         (size_t)gram_iter_blocks(F.dt, G) * ADJ_NSUM});

  bool ok = true;
  auto A = [&](size_t b) { void* p = F.alloc(b); if (!p) ok = false; return p; };
  F.y_int = (double*)A(G.nint * 8);
  F.a_int = (double*)A(G.nint * 8);
  F.eta_int = (double*)A(G.nint * 8);
  F.xd_int = (double*)A(G.nint * 8);
  // V and the increment get 8-byte elements whatever the chain dtype, so that a fit can
  // continue in FP64 (escalate_f64) without reallocating
  F.v_int = family_has_weights(F.family) ? A(G.nint * 8) : nullptr;
  F.T1d = (double*)A(G.t1_len * 8);
  F.S2d = (double*)A(G.s2_len * 8);
  F.X3fd = (double*)A(G.x3f_len * 8);
  F.X3ad = (double*)A(G.x3a_len * 8);
  F.thpk = (double*)A(G.inc_len * 8);
  F.imgd = A(chain_image_bytes(DT_F64, G));
  if (F.dt == DT_F64) {
    F.T1c = F.T1d; F.S2c = F.S2d; F.X3fc = F.X3fd; F.X3ac = F.X3ad; F.imgc = F.imgd;
  } else {
    F.T1c = A(G.t1_len * es);
    F.S2c = A(G.s2_len * es);
    F.X3fc = A(G.x3f_len * es);
    F.X3ac = A(G.x3a_len * es);
    F.imgc = A(chain_image_bytes(F.dt, G));
  }
  F.theta = (double*)A(G.p * 8);
  F.gref = (double*)A(G.p * 8);
  F.x = (double*)A(G.p * 8);
  F.xp = (double*)A(G.p * 8);
  F.gp = (double*)A(G.p * 8);
  F.dvec = (double*)A(G.p * 8);
  if (bt) {
    F.yb = (double*)A(G.p * 8); F.gyb = (double*)A(G.p * 8);
    F.x2 = (double*)A(G.p * 8); F.xp2 = (double*)A(G.p * 8); F.gp2 = (double*)A(G.p * 8);
    F.yb2 = (double*)A(G.p * 8); F.gyb2 = (double*)A(G.p * 8);
  }
  F.inc = A(G.inc_len * 8);
  if (F.incst) {
    const size_t tl = (size_t)adj_tiled_len(G);
    F.tT = (double*)A(tl * 8);
    F.gT = (double*)A(tl * 8);
    F.penT = (double*)A(tl * 8);
    F.dst[0] = (float*)A(tl * 4);
    F.dst[1] = (float*)A(tl * 4);
    F.qst = (float*)A(tl * 4);
    if (events) {
      F.dS = (float*)A(tl * 4);
      F.qS = (float*)A(tl * 4);
      F.incS = A(G.inc_len * 8);
      F.partS = (double*)A(nadj * ADJ_NSUM * 8);
    }
  }
  F.iter = (int*)A(2 * sizeof(int));
  F.part = (double*)A(npart * 8);
  F.npart = npart;
  F.red = (double*)A(64 * 8);
  F.dparams = (double*)A(8 * 8);
  F.stop = (int*)A(256);
  if (!ok) { F.err = "device allocation failed"; return GLAM_ENOMEM; }
  if (events)
    for (auto& e : F.ev)
      if (hipEventCreate(&e) != hipSuccess) { F.err = "hipEventCreate failed"; return GLAM_EDEVICE; }
  F.hred = F.host_alloc(64, &F.hred_dev);
  F.hparams = F.host_alloc(8);
  F.hpub = F.host_alloc(32, &F.hpub_dev);   // two slots of 8 published values, the sequence number at [24]
  for (int j = 0; j < 3; ++j) F.hx[j] = F.host_alloc((size_t)prob->n[j] * prob->p[j]);
  if (!F.hred || !F.hparams || !F.hpub || !F.hx[0] || !F.hx[1] || !F.hx[2]) {
    F.err = "pinned host allocation failed";
    return GLAM_ENOMEM;
  }
  F.hseq = (unsigned*)(F.hpub + 24);
  *F.hseq = 0u;
  F.hseq_dev = (unsigned*)(F.hpub_dev + 24);
  F.seq_dev = (unsigned*)A(256);
  if (!F.seq_dev || hipMemsetAsync(F.seq_dev, 0, 256, F.s) != hipSuccess) {
    F.err = "device allocation failed";
    return GLAM_ENOMEM;
  }
  F.seq_expect = 0;

  // ---- input checks (device; flags read by fit_setup_finish) ----
  {
    int nb = 0;
    FCHK(launch_check(G.n, prob->Y, prob->obs_w, G.p, prob->pen_w, prob->family, F.part, &nb, F.s));
    const int ops[4] = {1, 1, 1, 1};
    FCHK(launch_reduce(F.part, nb, 4, ops, 1.0, F.hred_dev + 32, F.s));
  }
  // ---- setup: tiled data, chain copies of the factors, spectral radii ----
  FCHK(launch_to_tiled(G, prob->Y, 0.0, F.y_int, F.s));
  FCHK(launch_to_tiled(G, prob->obs_w, 1.0, F.a_int, F.s));
  FCHK(launch_pack_chain_image(DT_F64, DT_F64, G, prob->X[0], prob->X[1], F.imgd, F.s, PACK_LDS));
  // the inner-loop chain (and, in a batched fit, the batched step's per-slab chain)
  if (F.dt != DT_F64)
    FCHK(launch_pack_chain_image(F.dt, DT_F64, G, prob->X[0], prob->X[1], F.imgc, F.s,
                                 chain_image_need(F.dt, SM_FUSED, G) | (F.batched ? PACK_LDS : 0)));
  // packed mode-3 factor (FP64 and chain dtype); zero the padded intermediates once
  FCHK(launch_pack(DT_F64, DT_F64, prob->X[2], G.p3, G.n3, G.n3, 1, F.X3fd, F.s));
  FCHK(launch_pack(DT_F64, DT_F64, prob->X[2], G.n3, G.p3, 1, G.n3, F.X3ad, F.s));
  FCHK(launch_zero(F.S2d, G.s2_len * 8, F.s));   // rows beyond n3 stay zero
  if (F.dt != DT_F64) {
    FCHK(launch_pack(F.dt, DT_F64, prob->X[2], G.p3, G.n3, G.n3, 1, F.X3fc, F.s));
    FCHK(launch_pack(F.dt, DT_F64, prob->X[2], G.n3, G.p3, 1, G.n3, F.X3ac, F.s));
    FCHK(launch_zero(F.S2c, G.s2_len * es, F.s));
  }
  for (int j = 0; j < 3; ++j)
    FCHK(hipMemcpyAsync(F.hx[j], prob->X[j], (size_t)prob->n[j] * prob->p[j] * 8, hipMemcpyDeviceToHost, F.s));
  return GLAM_OK;
}

// The rest of the set-up, after the stream has completed what fit_setup_enqueue queued:
// the input-check verdicts, the spectral radii of Proposition 1 from the host copies of
// the factors, and (Gram and Kron forms) the Gram factors.
static int fit_setup_finish(Fit& F) {
  const glam_problem* prob = F.prob;
  const Geom& G = F.G;
  const size_t es = dt_size(F.dt);
  if (F.hred[32] != 0.0) { F.err = "Y has non-finite entries"; return GLAM_EINVAL; }
  if (F.hred[33] != 0.0) {
    F.err = prob->family == GLAM_POISSON    ? "Poisson Y must be >= 0"
            : prob->family == GLAM_BINOMIAL ? "Binomial Y must be a proportion in [0, 1]"
                                            : "Gamma Y must be > 0";
    return GLAM_EINVAL;
  }
  if (F.hred[34] != 0.0) { F.err = "obs_w must be finite and >= 0"; return GLAM_EINVAL; }
  if (F.hred[35] != 0.0) { F.err = "pen_w must be finite and > 0"; return GLAM_EINVAL; }
  F.sprod = 1.0;
  std::vector<double> gm[3];
  for (int j = 0; j < 3; ++j) {
    gm[j] = gram_matrix(F.hx[j], (int)prob->n[j], (int)prob->p[j]);
    F.sprod *= gram_spectral_radius(gm[j], (int)prob->p[j]);
  }
  if (F.gram) {
    F.S1g = (double*)F.alloc(gm[0].size() * 8);
    F.S2g = (double*)F.alloc(gm[1].size() * 8);
    double* s3 = (double*)F.alloc(gm[2].size() * 8);
    F.S3c = F.alloc((size_t)G.KB3 * 16 * G.p3 * es);
    F.Zc = F.alloc((size_t)G.inc_len * es);
    if (!F.S1g || !F.S2g || !s3 || !F.S3c || !F.Zc) { F.err = "device allocation failed"; return GLAM_ENOMEM; }
    FCHK(hipMemcpyAsync(F.S1g, gm[0].data(), gm[0].size() * 8, hipMemcpyHostToDevice, F.s));
    FCHK(hipMemcpyAsync(F.S2g, gm[1].data(), gm[1].size() * 8, hipMemcpyHostToDevice, F.s));
    FCHK(hipMemcpyAsync(s3, gm[2].data(), gm[2].size() * 8, hipMemcpyHostToDevice, F.s));
    FCHK(launch_pack(F.dt, DT_F64, s3, G.p3, G.p3, 1, G.p3, F.S3c, F.s));
    FCHK(launch_zero(F.Zc, (size_t)G.inc_len * es, F.s));   // contraction padding stays zero
    FCHK(hipStreamSynchronize(F.s));                        // host Gram matrices go out of scope
    F.Gg = G;   // out = Z^T S_3: the adjoint GEMM with contraction length p3
    F.Gg.n3 = G.p3;
    F.Gg.KBN3 = G.KB3;
    F.Gg.s2_len = G.inc_len;
    F.Gg.x3a_len = (long long)G.KB3 * 16 * G.p3;
    F.S3g = s3;
    F.gram_fused = gram_iter_pays(F.dt, G);
    if (F.kron) {
      F.kron_work = (double*)F.alloc(kron_work_doubles(G) * 8);
      F.kron_stats = (double*)F.alloc(8 * 8);
      if (!F.kron_work || !F.kron_stats) { F.err = "device allocation failed"; return GLAM_ENOMEM; }
    }
    if (F.gram_fused) {
      F.inc2 = F.alloc(G.inc_len * 8);
      if (!F.inc2) { F.err = "device allocation failed"; return GLAM_ENOMEM; }
      FCHK(launch_zero(F.inc2, G.inc_len * 8, F.s));   // padding of the k-blocks stays zero
    }
  }
  return GLAM_OK;
}

static int fit_setup(Fit& F, const glam_problem* prob, bool bt, bool events) {
  const int r = fit_setup_enqueue(F, prob, bt, events);
  if (r) return r;
  FCHK(hipStreamSynchronize(F.s));
  return fit_setup_finish(F);
}

}  // namespace glam

using namespace glam;

static int fit_fail(int code, const std::string& msg);

// A d = 2 problem X_2 (x) X_1 as the d = 3 problem X_2 (x) [1] (x) X_1 (every array keeps its
// vec layout; mode 2 becomes the slab mode); unit holds the device FP64 1 of the middle factor.
struct UnitFactor {
  double* p = nullptr;
  ~UnitFactor() { if (p) (void)hipFree(p); }
};
static int lift_problem(const glam_problem* in, glam_problem* out, UnitFactor* unit, std::string* why) {
  if (in->d != 2 && in->d != 3) { *why = "d must be 2 or 3"; return GLAM_EINVAL; }
  for (int j = 0; j < in->d; ++j) {
    if (in->n[j] < 1 || in->p[j] < 1) { *why = "mode sizes must be >= 1"; return GLAM_EINVAL; }
    if (!in->X[j]) { *why = "NULL factor"; return GLAM_EINVAL; }
  }
  *out = *in;
  if (in->d == 2) {
    if (!unit->p) {
      const double one = 1.0;
      if (hipMalloc((void**)&unit->p, 256) != hipSuccess) { *why = "device allocation failed"; return GLAM_ENOMEM; }
      if (hipMemcpy(unit->p, &one, sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        *why = "hipMemcpy failed";
        return GLAM_EDEVICE;
      }
    }
    lift_sizes(2, in->n, in->p, out->n, out->p);
    out->d = 3;
    out->X[0] = in->X[0];
    out->X[1] = unit->p;
    out->X[2] = in->X[1];
  }
  return GLAM_OK;
}

// The slab kernels take modes 1 and 2 within the limits of the rho entry points and of the FP64
// outer steps' LDS image.
static bool inner_modes_fit(const int64_t* n, const int64_t* p, int dtype) {
  if (!rho_order_fits(n, p, dtype, nullptr)) return false;
  return slab_chain_lds_bytes(DT_F64, make_geom(n, p)) <= 159 * 1024;
}

// Device copies of a problem with its modes reordered (Y, obs_w: n-arrays; pen_w, theta0:
// p-arrays), freed when the fit returns.
struct PermutedProblem {
  int q[3] = {0, 1, 2};      // position k holds the caller's mode q[k]
  bool active = false;
  std::vector<void*> bufs;
  PermutedProblem() = default;
  PermutedProblem(const PermutedProblem&) = delete;
  PermutedProblem& operator=(const PermutedProblem&) = delete;
  ~PermutedProblem() { for (void* b : bufs) (void)hipFree(b); }
  double* alloc(size_t count) {
    void* b = nullptr;
    if (hipMalloc(&b, std::max<size_t>(count * 8, 256)) != hipSuccess) return nullptr;
    bufs.push_back(b);
    return (double*)b;
  }
};

// If the caller's mode order does not fit the slab kernels, pick an order that does (the largest
// remaining mode last), and permute the problem's arrays on the caller's stream.
static int permute_problem(glam_problem* prob, int dtype, const double** theta0, PermutedProblem* pp, hipStream_t us,
                           std::string* why) {
  if (inner_modes_fit(prob->n, prob->p, dtype)) return GLAM_OK;
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 2, 0}, {1, 0, 2}, {2, 0, 1}, {2, 1, 0}};
  int best = -1;
  for (int c = 1; c < 6; ++c) {
    int64_t n[3], p[3];
    for (int k = 0; k < 3; ++k) { n[k] = prob->n[perms[c][k]]; p[k] = prob->p[perms[c][k]]; }
    if (!inner_modes_fit(n, p, dtype)) continue;
    if (best < 0 || n[2] > prob->n[perms[best][2]]) best = c;
  }
  if (best < 0) {
    *why = "no order of the modes fits the slab kernels (two modes need p <= 32 and n <= 256, FP64 LDS image)";
    return GLAM_EINVAL;
  }
  pp->active = true;
  for (int k = 0; k < 3; ++k) pp->q[k] = perms[best][k];
  glam_problem out = *prob;
  for (int k = 0; k < 3; ++k) { out.n[k] = prob->n[pp->q[k]]; out.p[k] = prob->p[pp->q[k]]; out.X[k] = prob->X[pp->q[k]]; }
  const long long n = prob->n[0] * prob->n[1] * prob->n[2], p = prob->p[0] * prob->p[1] * prob->p[2];
  auto copy = [&](const double* src, long long count, const int64_t* dims, const double** dst) -> int {
    if (!src) return GLAM_OK;
    double* b = pp->alloc((size_t)count);
    if (!b) { *why = "device allocation failed"; return GLAM_ENOMEM; }
    if (launch_permute3(src, b, dims, pp->q, us) != hipSuccess) { *why = "permutation kernel failed"; return GLAM_EDEVICE; }
    *dst = b;
    return GLAM_OK;
  };
  int r;
  if ((r = copy(prob->Y, n, prob->n, &out.Y))) return r;
  if ((r = copy(prob->obs_w, n, prob->n, &out.obs_w))) return r;
  if ((r = copy(prob->pen_w, p, prob->p, &out.pen_w))) return r;
  if (theta0 && (r = copy(*theta0, p, prob->p, theta0))) return r;
  *prob = out;
  return GLAM_OK;
}

// The checks of glam_fit_path on its options and result arrays (shared with the generic solver).
int glam::check_fit_options(const glam_options* opt, const glam_result* res, int family, bool has_obs_w, std::string* why) {
  auto bad = [&](const char* m) {
    *why = m;
    return GLAM_EINVAL;
  };
  if (opt->dtype < 0 || opt->dtype > 2) return bad("bad dtype");
  if (opt->nlambda < 1) return bad("nlambda must be >= 1");
  if (!opt->lambda && !(opt->lambda_min_ratio > 0.0 && opt->lambda_min_ratio <= 1.0))
    return bad("lambda_min_ratio must be in (0, 1]");
  if (!(opt->kkt_tol > 0.0)) return bad("kkt_tol must be > 0");
  if (!(opt->nu >= 0.0 && opt->nu <= 1.0)) return bad("nu must be in [0, 1]");
  if (!(opt->alpha >= 0.0) || !std::isfinite(opt->alpha)) return bad("alpha must be finite and >= 0");
  if (opt->penalty != GLAM_PENALTY_LASSO && opt->penalty != GLAM_PENALTY_SCAD && opt->penalty != GLAM_PENALTY_RIDGE)
    return bad("bad penalty");
  if (opt->penalty == GLAM_PENALTY_RIDGE && opt->alpha != 0.0)
    return bad("the ridge penalty takes no elastic-net weight (alpha = 0)");
  if (opt->penalty == GLAM_PENALTY_SCAD) {
    if (opt->msa_steps < 1) return bad("msa_steps must be >= 1");
    if (!(opt->scad_a == 0.0 || (opt->scad_a > 2.0 && std::isfinite(opt->scad_a))))
      return bad("scad_a must be > 2 (or 0 for 3.7)");
    if (opt->alpha != 0.0) return bad("SCAD and the elastic net do not combine");
  }
  if (opt->inner_mode != GLAM_INNER_CHAIN && opt->inner_mode != GLAM_INNER_GRAM && opt->inner_mode != GLAM_INNER_KRON &&
      opt->inner_mode != GLAM_INNER_ONE)
    return bad("bad inner_mode");
  if (opt->inner_mode == GLAM_INNER_ONE && (has_obs_w || opt->nu < 1.0))
    return bad("the unit-weight inner loop takes no prior weights and runs without backtracking (nu = 1)");
  if (opt->inner_mode == GLAM_INNER_KRON && opt->nu < 1.0)
    return bad("the tensor-product-weight inner loop runs without backtracking (nu = 1)");
  if (opt->inner_mode == GLAM_INNER_GRAM && (family_has_weights(family) || has_obs_w || opt->nu < 1.0))
    return bad("the Gram inner loop is exact only for unit IRLS weights (Gaussian, Gamma-log) "
               "without prior weights (Sec. 6.2) and runs without backtracking (nu = 1)");
  if (opt->max_outer < 1 || opt->max_inner < 1 || opt->check_every < 1)
    return bad("max_outer, max_inner and check_every must be >= 1");
  if (opt->extrapolation != 0 && opt->extrapolation != 1) return bad("bad extrapolation");
  if (opt->kron_step != 0 && opt->kron_step != 1) return bad("bad kron_step");
  if (!res->theta || !res->lambda_out || !res->kkt || !res->objective || !res->iters_outer || !res->iters_inner ||
      !res->status)
    return bad("NULL result array");
  if (opt->lambda) {
    for (int l = 0; l < opt->nlambda; ++l) {
      if (!(opt->lambda[l] >= 0.0) || !std::isfinite(opt->lambda[l]))
        return bad("lambda values must be finite and >= 0");
      if (l > 0 && !(opt->lambda[l] < opt->lambda[l - 1]))
        return bad("lambda sequence must be strictly decreasing");
    }
  }
  return GLAM_OK;
}

// some order of the modes fits the slab kernels
static bool any_order_fits(const int64_t* n, const int64_t* p, int dtype) {
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 2, 0}, {1, 0, 2}, {2, 0, 1}, {2, 1, 0}};
  for (const auto& q : perms) {
    const int64_t nq[3] = {n[q[0]], n[q[1]], n[q[2]]}, pq[3] = {p[q[0]], p[q[1]], p[q[2]]};
    if (inner_modes_fit(nq, pq, dtype)) return true;
  }
  return false;
}

extern "C" int glam_fit_path(const glam_problem* prob_in, const glam_options* opt_in, glam_result* res) {
  auto t_start = std::chrono::steady_clock::now();
  if (!prob_in || !opt_in || !res) return fit_fail(GLAM_EINVAL, "NULL argument");
  glam_problem lifted;
  UnitFactor unit;
  glam_options opt_local = *opt_in;
  const glam_options* opt = &opt_local;
  PermutedProblem perm;   // declared before the Fit: its buffers outlive the fit's stream work
  {
    std::string why;
    const int r = lift_problem(prob_in, &lifted, &unit, &why);
    if (r) return fit_fail(r, why);
  }
  const glam_problem* prob = &lifted;
  if (!prob->Y) return fit_fail(GLAM_EINVAL, "NULL Y");
  if (prob->family < GLAM_GAUSSIAN || prob->family > GLAM_GAMMA) return fit_fail(GLAM_EINVAL, "bad family");
  {
    std::string why;
    const int r = check_fit_options(opt, res, prob->family, prob->obs_w != nullptr, &why);
    if (r) return fit_fail(r, why);
  }
  // modes that fit no order of the slab kernels (p_j > n_j designs, large p_j): the generic-GEMM
  // solver, which takes the rho-chain and unit-weight inner loops
  if (!any_order_fits(prob->n, prob->p, opt->dtype)) {
    if (opt->inner_mode == GLAM_INNER_GRAM || opt->inner_mode == GLAM_INNER_KRON)
      return fit_fail(GLAM_EINVAL, "no order of the modes fits the slab kernels (two modes need p <= 32 and n <= 256, "
                                   "FP64 LDS image), and the generic solver takes only the rho-chain and unit-weight "
                                   "inner loops");
    GenProblem gp;
    for (int j = 0; j < 3; ++j) gp.n[j] = prob->n[j];
    GenComponent c;
    for (int j = 0; j < 3; ++j) { c.p[j] = prob->p[j]; c.X[j] = prob->X[j]; }
    gp.comps.push_back(c);
    gp.Y = prob->Y;
    gp.obs_w = prob->obs_w;
    gp.family = prob->family;
    gp.pen_w = prob->pen_w;
    std::string why;
    const int r = general_fit_path(gp, opt, res, &why);
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (r) return fit_fail(r, why);
    return GLAM_OK;
  }
  {
    // modes reordered, when needed, so that two of them fit the slab kernels
    std::string why;
    const int r = permute_problem(&lifted, opt_local.dtype, &opt_local.theta0, &perm, (hipStream_t)opt_in->stream, &why);
    if (r) return fit_fail(r, why);
  }

  Fit F;
  F.G = make_geom(prob->n, prob->p);
  F.dt = opt->dtype;
  F.us = (hipStream_t)opt->stream;
  // work on an internal non-blocking stream (capturable), ordered after the caller's stream
  if (hipStreamCreateWithFlags(&F.s, hipStreamNonBlocking) != hipSuccess)
    return fit_fail(GLAM_EDEVICE, "hipStreamCreateWithFlags failed");
  F.own_stream = true;
  if (hipEventCreateWithFlags(&F.sync_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(F.sync_ev, F.us) != hipSuccess || hipStreamWaitEvent(F.s, F.sync_ev, 0) != hipSuccess)
    return fit_fail(GLAM_EDEVICE, "stream ordering failed");
  F.gram = opt->inner_mode == GLAM_INNER_GRAM || opt->inner_mode == GLAM_INNER_KRON || opt->inner_mode == GLAM_INNER_ONE;
  F.kron = opt->inner_mode == GLAM_INNER_KRON && family_has_weights(prob->family);
  F.unit_w = opt->inner_mode == GLAM_INNER_ONE && family_has_weights(prob->family);
  F.enet = opt->alpha;
  if (opt->penalty == GLAM_PENALTY_RIDGE) {   // Sec. 6.3: J = sum_m w_m theta_m^2
    F.enet = 1.0;
    F.no_l1 = 1;
  }
  F.incst = F.dt != DT_F64 && !F.gram && opt->nu >= 1.0;
  F.runahead = F.incst;
  F.keep_eta = !(prob->family == GLAM_GAUSSIAN && prob->obs_w == nullptr) || F.kron;
  F.restart = opt->extrapolation == 0 && !F.gram && opt->nu >= 1.0;
  {
    const int r = fit_setup(F, prob, opt->nu < 1.0, opt->profile_every > 0);
    if (r) return fit_fail(r, F.err);
  }
  const Geom& G = F.G;

#define PCHK(expr)                                                                               \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) return fit_fail(GLAM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define RCHK(expr)                                \
  do {                                            \
    int r_ = (expr);                              \
    if (r_ != GLAM_OK) return fit_fail(r_, F.err); \
  } while (0)

  // SCAD (Sec. 6.4): the MSA steps reweight a buffer of penalty weights of their own; it
  // holds the caller's weights (or ones) for step 1, which also defines lambda_max
  const bool scad = opt->penalty == GLAM_PENALTY_SCAD;
  const int msa_steps = scad ? opt->msa_steps : 1;
  const double scad_a = opt->scad_a == 0.0 ? 3.7 : opt->scad_a;
  double* pen_buf = nullptr;
  if (scad) {
    pen_buf = (double*)F.alloc(G.p * 8);
    if (!pen_buf) return fit_fail(GLAM_ENOMEM, "device allocation failed");
    F.pen = pen_buf;
  }
  auto base_weights = [&]() -> hipError_t {
    return prob->pen_w ? hipMemcpyAsync(pen_buf, prob->pen_w, G.p * 8, hipMemcpyDeviceToDevice, F.s)
                       : launch_fill(pen_buf, G.p, 1.0, F.s);
  };
  if (scad) PCHK(base_weights());

  // ---- lambda_max: the zero solution's gradient (Sec. 6.4) ----
  PCHK(launch_fill(F.theta, G.p, 0.0, F.s));
  StepStats st0;
  RCHK(family_step(F, F.theta, 0.0, &st0));
  const double lam_max = st0.lmax_raw;
  res->lambda_max = lam_max;
  if (!std::isfinite(lam_max)) return fit_fail(GLAM_ENONFINITE, "non-finite lambda_max");
  const double lam_scale = lam_max > 0.0 ? lam_max : 1.0;
  std::vector<double> lams(opt->nlambda);
  for (int l = 0; l < opt->nlambda; ++l) {
    if (opt->lambda) lams[l] = opt->lambda[l];
    else lams[l] = opt->nlambda == 1 ? lam_max
                                     : lam_max * std::pow(opt->lambda_min_ratio, (double)l / (opt->nlambda - 1));
  }
  if (opt->theta0) PCHK(hipMemcpyAsync(F.theta, opt->theta0, G.p * 8, hipMemcpyDeviceToDevice, F.s));

  const bool exact_model = F.family == GLAM_GAUSSIAN && prob->obs_w == nullptr;
  const double tol = opt->kkt_tol;
  // The inner stopping rule is checked every check_every iterations, except where the model's
  // curvature can be far from the objective's: the Gamma-log model (Fisher scoring with unit
  // weights, a non-canonical link) and the tensor-product weights of Sec. 6.2.  There,
  // iterating past the first point that meets the rule makes the outer steps short (the
  // Armijo rule cuts them), so the rule is checked every iteration.
  // an approximate model (Gamma's unit Fisher weights, tensor-product or unit weights) is
  // checked every iteration: a coarser check over-solves it past what its outer step can use
  const int check_every = (F.family == GLAM_GAMMA || F.kron || F.unit_w) ? 1 : opt->check_every;
  const int log_level = getenv("GLAM_LOG") ? atoi(getenv("GLAM_LOG")) : 0;
  const bool verbose = log_level > 0;
  int path_status = GLAM_OK;
  long long path_inner = 0;
  res->n_done = 0;
  res->escalated_at = -1;
  res->chain_ms = 0.0;
  res->adj_ms = 0.0;
  res->fwd_ms = 0.0;
  res->iter_ms = 0.0;
  res->chain_samples = 0;
  res->inner_total = 0;

  StepStats st_last{};   // the last family step's values (theta unchanged since)
  for (int l = 0; l < opt->nlambda; ++l) {
    const double lam = lams[l];
    res->lambda_out[l] = lam;
    int status = GLAM_ENOCONV;
    int outer = 0;
    long long inner_total = 0;
    StepStats st{};
    double kkt = INFINITY, Fobj = NAN;
    int outer_base = 0;
    // precision escalation: a BF16/FP32 inner loop that ends on its rounding floor (stall or
    // noise rule, not tol_in) three outer steps in a row while the FP64 KKT improves by less
    // than 10% cannot refine this problem further (its conditioning times the chain's epsilon
    // is too large); the fit then continues one rung up, BF16 -> FP32 -> FP64, for the rest
    // of the path
    int lowprec_stalls = 0;
    bool last_limited = false;
    double kkt_prev = INFINITY;
    for (int step = 0; step < msa_steps; ++step) {
    if (scad) {   // MSA-lasso: the lasso first, then weights from the previous step's estimate
      if (step == 0) PCHK(base_weights());
      else PCHK(launch_scad_weights(G.p, F.theta, prob->pen_w, lam, scad_a, pen_buf, F.s));
    }
    status = GLAM_ENOCONV;
    for (int k = 0; k <= opt->max_outer; ++k) {
      bool reused = false;
      if (k == 0 && l > 0 && !scad) RCHK(kkt_at_lambda(F, lam, st_last, &st, &reused));
      if (!reused) RCHK(family_step(F, F.theta, lam, &st));
      st_last = st;
      kkt = st.kkt_raw / lam_scale;
      Fobj = st.nll + lam * st.pen;
      outer = outer_base + k;
      if (!std::isfinite(kkt) || !std::isfinite(Fobj)) { status = GLAM_ENONFINITE; break; }
      if (kkt <= tol) { status = GLAM_OK; break; }
      if (k == opt->max_outer) break;
      if (F.dt != DT_F64 && !F.gram) {
        lowprec_stalls = (k > 0 && last_limited && kkt > 0.9 * kkt_prev) ? lowprec_stalls + 1 : 0;
        if (lowprec_stalls >= 3) {
          if (F.dt == DT_BF16) {
            RCHK(escalate_f32(F));
          } else {
            escalate_f64(F);
            // the weights V of this step were written for the FP32 chain (4-byte entries); the FP64
            // chain reads 8-byte ones: step 2 again at the same theta writes them in that format
            // (the other values are the same)
            if (F.v_int) RCHK(family_step(F, F.theta, lam, &st));
          }
          lowprec_stalls = 0;
          if (res->escalated_at < 0) res->escalated_at = l;
          if (verbose)
            fprintf(stderr, "[glam] lambda %d k %d: inner chain continues in %s\n", l, k, F.dt == DT_F32 ? "FP32" : "FP64");
        }
      }
      kkt_prev = kkt;
      double wmax = family_has_weights(F.family) && !F.unit_w ? st.vmax : 1.0;
      if (F.kron) {
        // W^(k) = V-hat (Sec. 6.2): reweighted Gram factors from this step's eta; Proposition 1
        // with max V-hat = Vbar prod_j max v_j
        PCHK(launch_kron_weights(G, F.family, F.eta_int, prob->X[0], prob->X[1], prob->X[2], F.kron_work,
                                 F.kron_stats, F.S1g, F.S2g, F.S3g, F.s));
        if (!F.gram_fused) PCHK(launch_pack(F.dt, DT_F64, F.S3g, G.p3, G.p3, 1, G.p3, F.S3c, F.s));
        // Sec. 5: with tensor-product weights the Lipschitz constant is exact,
        // L = (1/n) prod_j rho(X_j^T W_j X_j) (Vbar folded into S_3); the power method's bounds
        // replace Proposition 1 whenever all three factors converged
        if (opt->kron_step == 1) {
          PCHK(launch_gram_radii(G, F.S1g, F.S2g, F.S3g, F.kron_work, F.kron_first ? 1 : 0, F.kron_stats, F.s));
          F.kron_first = false;
        }
        PCHK(hipMemcpyAsync(F.hred, F.kron_stats, 8 * sizeof(double), hipMemcpyDeviceToHost, F.s));
        PCHK(hipStreamSynchronize(F.s));
        wmax = F.hred[3] * F.hred[0] * F.hred[1] * F.hred[2];
        if (opt->kron_step == 1 && F.hred[7] == 1.0) {
          const double lex = F.hred[4] * F.hred[5] * F.hred[6] / F.sprod;   // so that Lhat = lex sprod / n
          if (lex > 0.0 && std::isfinite(lex) && lex <= wmax) wmax = lex;
        }
      }
      const double Lhat = wmax * F.sprod / (double)G.n;
      if (!(Lhat > 0.0) || !std::isfinite(Lhat)) { status = GLAM_ENONFINITE; break; }
      // Sec. 6.4: nu in (0, 1] scales 1/Lhat; nu = 0 starts at delta = 1 and backtracks every
      // iteration (R22)
      const double delta = opt->nu > 0.0 ? 1.0 / (opt->nu * Lhat) : 1.0;
      double tol_in = exact_model ? 0.5 * tol : std::max(0.1 * tol, 0.1 * kkt);
      // A BF16 chain perturbs grad h by roughly eps_bf16 * kappa relative to the
      // increment, so one outer pass cannot gain more than that factor: each pass asks for
      // at most a ~33x reduction and re-anchors in FP64 (iterative refinement); a pass that
      // cannot get there ends on the noise floor or the stall rule below. On the Gaussian
      // 100x100x1000 path the total time is lowest at this factor: asking for 100x or 300x
      // per pass gave one same, slightly slower path; 17x and 10x took longer.
      if (F.dt == DT_BF16) tol_in = std::max(tol_in, 0.03 * kkt);
      // ---- inner PG loop ----
      const bool incst = F.incst && F.dt != DT_F64;
      if (incst)
        PCHK(launch_inner_init_inc(F.dt, G, F.theta, F.gref, F.pen, F.tT, F.gT, F.penT, F.dst[0], F.dst[1], F.qst,
                                   F.inc, F.iter, F.s));
      else
        PCHK(launch_inner_init(G, F.theta, F.gref, F.x, F.xp, F.gp, F.dt, F.inc, F.iter, F.s));
      F.gpar = 0;   // the increment and the counter start in buffer 0
      int it = 0;
      double kin = INFINITY, noise = 0.0;
      if (opt->nu < 1.0) {
        RCHK(inner_loop_bt(F, lam, delta, Lhat, tol_in, opt->max_inner, lam_scale, &kin, &it));
      } else {
      F.hparams[0] = lam;
      F.hparams[1] = delta;
      F.hparams[4] = lam_scale;            // the device's copy of the convergence test below
      F.hparams[5] = tol_in;
      F.hparams[6] = 4.0 * kEps[F.dt];
      PCHK(hipMemcpyAsync(F.dparams, F.hparams, 7 * sizeof(double), hipMemcpyHostToDevice, F.s));
      // run ahead (the increment-state chain loop): one block of iterations is queued beyond the
      // one whose check the host reads next; the reduction ending each block applies the
      // convergence test on the device and, once it holds, the queued kernels do nothing
      const bool ra = F.runahead && incst;
      if (ra) PCHK(hipMemsetAsync(F.stop, 0, sizeof(int), F.s));
      double best = INFINITY, window_best = INFINITY;
      int window_start = 0;
      int it_q = 0;              // inner iterations queued
      int inflight[2] = {0, 0};  // sizes of the queued blocks whose checks are not read yet
      bool inflight_sample[2] = {false, false};   // ... and whether they carry a timing sample
      int nq = 0;
      bool stopping = false;     // the loop has ended: nothing more is queued
      int nb = 0;
      auto queue_block = [&]() -> int {
        const int m = std::min(check_every, opt->max_inner - it_q);
        if (m <= 0) return GLAM_OK;
        const long long gi = path_inner + inner_total + it_q;
        // a sampled block (events around its kernels) that the device skips is dropped from the
        // timing when its check is read; two sampled blocks are never in flight together (one set
        // of events)
        const bool sample = opt->profile_every > 0 && !(nq > 0 && inflight_sample[nq - 1]) &&
                            (gi / check_every) % std::max(1, opt->profile_every / check_every) == 0;
        const int r = opt->graph_mode == 0 && m == check_every && !sample ? inner_block_graph(F, m, &nb)
                                                                          : inner_block_eager(F, m, sample, &nb);
        if (r) return r;
        inflight_sample[nq] = sample;
        inflight[nq++] = m;
        it_q += m;
        return GLAM_OK;
      };
      RCHK(queue_block());
      while (nq > 0) {
        if (ra && !stopping && nq < 2) RCHK(queue_block());
        const int m = inflight[0];
        const bool sampled = inflight_sample[0];
        inflight[0] = inflight[1];
        inflight_sample[0] = inflight_sample[1];
        --nq;
        double chk[ADJ_NSUM + 1];
        RCHK(wait_published(F, chk, ADJ_NSUM + 1));
        if (chk[ADJ_NSUM] != 0.0) {
          // skipped on the device (the loop ended at an earlier block): undo the parity flips
          // of its increment buffers that were booked when it was queued, and drop its timing
          if (m & 1) F.gpar ^= 1;
          if (sampled) F.pending = false;
          continue;
        }
        it += m;
        RCHK(collect_sample(F));
        kin = chk[0] / lam_scale;
        // rounding floor of the low-precision chain output (a lower bound of its error)
        noise = 4.0 * kEps[F.dt] * chk[1] / lam_scale;
        // a block that was in flight when the host ended the loop ran in full: its check values
        // are the loop's last ones (its last iterate is theta~)
        if (stopping) continue;
        best = std::min(best, kin);
        // the window counts inner iterations: 10 or 20 times max(requested check_every, 10), also
        // where every iteration is checked (Gamma-log, tensor-product and unit weights); a shorter
        // check interval (more frequent restart tests) does not shorten it (at check_every = 8 a
        // window of 80 iterations sent the Sec. 6.5 Gaussian r = 3 path to FP64 at model 82
        // instead of 91: 4.98 against 3.95 s)
        if (it - window_start >= (exact_model ? kStallChecks : kStallChecksLineSearch) * std::max(opt->check_every, 10)) {
          // stalled: no 2x progress over the window -> leave for an FP64 re-anchor (which
          // also restarts the extrapolation)
          if (!(best < 0.5 * window_best) && F.dt != DT_F64) {
            stopping = true;
            continue;
          }
          window_best = best;
          window_start = it;
        }
        if (log_level >= 2)
          fprintf(stderr, "[glam]   lambda %d k %d it %d kin %.3e noise %.3e\n", l, k, it, kin, noise);
        // (the device applies the same test to the same values when it runs ahead)
        if (!std::isfinite(kin) || kin <= std::max(tol_in, noise)) {
          stopping = true;
          continue;
        }
        if (!ra) RCHK(queue_block());
      }
      }
      inner_total += it;
      if (!std::isfinite(kin)) { status = GLAM_ENONFINITE; break; }
      last_limited = kin > tol_in && it < opt->max_inner;   // ended on the rounding floor
      // theta~ = x^l of the last checked iteration (held in xp; in the increment-state loop,
      // theta_ref + the buffer the last iteration read as d^l)
      double alpha = 0.0, Delta = 0.0;
      if (exact_model) {
        // the model is the objective itself (Sec. 6.5: no outer loop is needed), so the inner
        // solution is the new estimate (alpha = 1); further passes only re-anchor a BF16/FP32
        // inner loop in FP64, and the FP64 KKT test at the next anchor decides convergence
        alpha = 1.0;
        if (incst) PCHK(launch_inc_state_out(G, F.dst[1 - F.gpar], F.theta, 0, F.theta, F.s));
        else PCHK(hipMemcpyAsync(F.theta, F.xp, G.p * 8, hipMemcpyDeviceToDevice, F.s));
      } else {
        if (incst) PCHK(launch_inc_state_out(G, F.dst[1 - F.gpar], F.theta, 1, F.dvec, F.s));
        else PCHK(launch_sub(G.p, F.xp, F.theta, F.dvec, F.s));
        RCHK(armijo(F, lam, 0.1, &alpha, &Delta));
        if (alpha > 0.0) PCHK(launch_axpy(G.p, alpha, F.dvec, F.theta, F.s));
        else if (F.dt != DT_F64) last_limited = true;   // no descent from this low-precision pass
      }
      if (verbose)
        fprintf(stderr, "[glam] lambda %d k %d kkt %.3e F %.12e inner %d kin %.2e noise %.2e alpha %g Delta %.3e\n", l,
                k, kkt, Fobj, it, kin, noise, alpha, Delta);
    }
    outer_base = outer;
    if (status != GLAM_OK) break;
    }   // MSA steps
    if (perm.active) {   // back to the caller's mode order
      int qi[3];
      for (int k = 0; k < 3; ++k) qi[perm.q[k]] = k;
      PCHK(launch_permute3(F.theta, res->theta + (size_t)l * G.p, prob->p, qi, F.s));
    } else {
      PCHK(hipMemcpyAsync(res->theta + (size_t)l * G.p, F.theta, G.p * 8, hipMemcpyDeviceToDevice, F.s));
    }
    res->kkt[l] = kkt;
    res->objective[l] = Fobj;
    res->iters_outer[l] = outer;
    res->iters_inner[l] = (int)std::min<long long>(inner_total, 2000000000LL);
    res->status[l] = status;
    path_inner += inner_total;
    if (verbose)
      fprintf(stderr, "[glam] lambda %d = %.6e status %d kkt %.3e outer %d inner %lld\n", l, lam, status, kkt, outer,
              inner_total);
    if (status != GLAM_OK) {
      path_status = status;
      break;
    }
    res->n_done = l + 1;
  }
  PCHK(hipStreamSynchronize(F.s));
  RCHK(collect_sample(F));
  PCHK(hipEventRecord(F.sync_ev, F.s));
  PCHK(hipStreamWaitEvent(F.us, F.sync_ev, 0));
  res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  res->chain_ms = F.chain_ms;
  res->adj_ms = F.adj_ms;
  res->fwd_ms = F.fwd_ms;
  res->iter_ms = F.iter_ms;
  res->chain_samples = F.samples;
  res->inner_total = path_inner;
  if (path_status != GLAM_OK) return fit_fail(path_status, "path stopped early (see status array)");
  return GLAM_OK;
}


// ============================================================================
// glam_fit_batched
// ============================================================================
// Choices of the batched slab-phase tuner per shape-class signature: kept for the process, and
// in the text file named by GLAM_TUNE_FILE when that is set (one "key run wide" line per entry,
// read on first use and appended to).
static std::mutex g_tune_mu;
static std::map<std::string, std::pair<int, int>> g_tune;
static bool g_tune_loaded = false;

static std::string tune_key(int dt, int cls, int nprob_cls, long long slabs) {
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return "batched_slabs/cu" + std::to_string(cus) + "/dt" + std::to_string(dt) + "/class" + std::to_string(cls) + "/p" +
         std::to_string(nprob_cls) + "/s" + std::to_string(slabs);
}

static void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = getenv("GLAM_TUNE_FILE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char key[256];
  int run = 0, wide = 0;
  while (fscanf(f, "%255s %d %d", key, &run, &wide) == 3)
    if (run >= 1 && run <= 8 && (wide == 0 || wide == 1)) g_tune[key] = {run, wide};
  fclose(f);
}

static bool tune_lookup(const std::string& key, int* run, int* wide) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  *run = it->second.first;
  *wide = it->second.second;
  return true;
}

static void tune_store(const std::string& key, int run, int wide) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  g_tune[key] = {run, wide};
  const char* path = getenv("GLAM_TUNE_FILE");
  if (!path || !*path) return;
  if (FILE* f = fopen(path, "a")) {
    fprintf(f, "%s %d %d\n", key.c_str(), run, wide);
    fclose(f);
  }
}

static int validate_problem(const glam_problem* prob, int dtype, std::string* why) {
  if (prob->d != 3) { *why = "d must be 2 or 3"; return GLAM_EINVAL; }
  for (int j = 0; j < 3; ++j) {
    if (prob->n[j] < 1 || prob->p[j] < 1) { *why = "mode sizes must be >= 1"; return GLAM_EINVAL; }
    if (!prob->X[j]) { *why = "NULL factor"; return GLAM_EINVAL; }
  }
  if (!prob->Y) { *why = "NULL Y"; return GLAM_EINVAL; }
  if (prob->family < GLAM_GAUSSIAN || prob->family > GLAM_GAMMA) { *why = "bad family"; return GLAM_EINVAL; }
  if (!rho_order_fits(prob->n, prob->p, dtype, why)) return GLAM_EINVAL;
  if (slab_chain_lds_bytes(DT_F64, make_geom(prob->n, prob->p)) > 159 * 1024) {
    *why = "modes 1-2 too large for the FP64 slab kernel";
    return GLAM_EINVAL;
  }
  return GLAM_OK;
}

extern "C" int glam_fit_batched(const glam_problem* probs_in, int nprob, const glam_batch_options* opt,
                                glam_batch_result* res) {
  auto t_start = std::chrono::steady_clock::now();
  if (!probs_in || !opt || !res || nprob < 1) return fit_fail(GLAM_EINVAL, "NULL argument or nprob < 1");
  std::vector<glam_problem> lifted(nprob);
  UnitFactor unit;
  for (int i = 0; i < nprob; ++i) {
    std::string why;
    const int r = lift_problem(&probs_in[i], &lifted[i], &unit, &why);
    if (r) return fit_fail(r, "problem " + std::to_string(i) + ": " + why);
  }
  const glam_problem* probs = lifted.data();
  if (opt->dtype < 0 || opt->dtype > 2) return fit_fail(GLAM_EINVAL, "bad dtype");
  // a problem whose modes 1-2 do not fit the slab kernels is solved in another mode order
  // (its arrays permuted on the caller's stream, theta returned in the caller's order)
  std::vector<PermutedProblem> perms(nprob);
  for (int i = 0; i < nprob; ++i) {
    std::string why;
    const int r = permute_problem(&lifted[i], opt->dtype, nullptr, &perms[i], (hipStream_t)opt->stream, &why);
    if (r) return fit_fail(r, "problem " + std::to_string(i) + ": " + why);
  }
  if (!(opt->kkt_tol > 0.0)) return fit_fail(GLAM_EINVAL, "kkt_tol must be > 0");
  if (!(opt->alpha >= 0.0) || !std::isfinite(opt->alpha)) return fit_fail(GLAM_EINVAL, "alpha must be finite and >= 0");
  if (opt->max_outer < 1 || opt->max_inner < 1 || opt->check_every < 1)
    return fit_fail(GLAM_EINVAL, "max_outer, max_inner and check_every must be >= 1");
  if (opt->tuning != 0 && opt->tuning != 1) return fit_fail(GLAM_EINVAL, "bad tuning");
  if (opt->graph_mode != 0 && opt->graph_mode != 1) return fit_fail(GLAM_EINVAL, "bad graph_mode");
  if (!opt->lambda && !(opt->lambda_ratio > 0.0 && opt->lambda_ratio <= 1.0))
    return fit_fail(GLAM_EINVAL, "lambda_ratio must be in (0, 1]");
  if (!res->theta || !res->lambda_out || !res->lambda_max || !res->kkt || !res->objective || !res->iters_outer ||
      !res->status)
    return fit_fail(GLAM_EINVAL, "NULL result array");
  for (int i = 0; i < nprob; ++i) {
    std::string why;
    if (validate_problem(&probs[i], opt->dtype, &why)) return fit_fail(GLAM_EINVAL, "problem " + std::to_string(i) + ": " + why);
    if (!res->theta[i]) return fit_fail(GLAM_EINVAL, "NULL theta output");
    if (opt->lambda && !(opt->lambda[i] >= 0.0 && std::isfinite(opt->lambda[i])))
      return fit_fail(GLAM_EINVAL, "lambda values must be finite and >= 0");
  }
  const int dt = opt->dtype;
  // shared stream, ordered after the caller's stream
  hipStream_t us = (hipStream_t)opt->stream, s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return fit_fail(GLAM_EDEVICE, "stream");
  struct StreamGuard { hipStream_t s; ~StreamGuard() { if (s) { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); } } } sg{s};
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return fit_fail(GLAM_EDEVICE, "event");
  struct EvGuard { hipEvent_t e; ~EvGuard() { if (e) (void)hipEventDestroy(e); } } eg{ev};
  if (hipEventRecord(ev, us) != hipSuccess || hipStreamWaitEvent(s, ev, 0) != hipSuccess)
    return fit_fail(GLAM_EDEVICE, "stream ordering failed");
  // Each problem's own work (set-up, FP64 steps 2 and 5 of Algorithm 1) goes to one of a few
  // streams, so that the small per-problem kernels of different problems overlap; the batched
  // inner steps run on s.  The host synchronises every stream between the phases.
  constexpr int kPoolStreams = 8;
  struct PoolGuard {
    hipStream_t p[kPoolStreams] = {};
    ~PoolGuard() { for (hipStream_t q : p) if (q) { (void)hipStreamSynchronize(q); (void)hipStreamDestroy(q); } }
  } pool;
  const int npool = std::min(kPoolStreams, nprob);
  for (int k = 0; k < npool; ++k)
    if (hipStreamCreateWithFlags(&pool.p[k], hipStreamNonBlocking) != hipSuccess || hipStreamWaitEvent(pool.p[k], ev, 0) != hipSuccess)
      return fit_fail(GLAM_EDEVICE, "stream");
  auto sync_all = [&]() -> hipError_t {
    hipError_t e = hipStreamSynchronize(s);
    for (int k = 0; k < npool; ++k) {
      const hipError_t ek = hipStreamSynchronize(pool.p[k]);
      if (e == hipSuccess) e = ek;
    }
    return e;
  };

  // one arena for the whole batch; every set-up is queued before one synchronisation
  std::shared_ptr<Arena> arena = std::make_shared<Arena>();
  std::vector<std::unique_ptr<Fit>>* fits_ref = nullptr;
  // fn(i) for every problem i, the problems of pool stream k enqueued by host thread k: the
  // per-problem outer steps are thousands of small launches, and submitting them from one
  // thread left the GPU idle most of the time.  fn returns a status (message in the fit's err);
  // the failure of the lowest problem index is reported.
  auto for_each_problem = [&](const std::function<int(int)>& fn) -> int {
    std::vector<int> bad(npool, -1), code(npool, GLAM_OK);
    auto work = [&](int k) {
      for (int i = k; i < nprob; i += npool) {
        const int r = fn(i);
        if (r) { bad[k] = i; code[k] = r; return; }
      }
    };
    std::vector<std::thread> th;
    int k = 1;
    try {
      for (; k < npool; ++k) th.emplace_back(work, k);
    } catch (...) {   // no more threads: the rest on this one
      for (; k < npool; ++k) work(k);
    }
    work(0);
    for (auto& t : th) t.join();
    int first = -1, c = GLAM_OK;
    for (int q = 0; q < npool; ++q)
      if (bad[q] >= 0 && (first < 0 || bad[q] < first)) { first = bad[q]; c = code[q]; }
    if (first >= 0) return fit_fail(c, "problem " + std::to_string(first) + ": " + (*fits_ref)[first]->err);
    return GLAM_OK;
  };
  struct SyncGuard {   // every stream idle before the arena goes (on early returns too)
    std::function<hipError_t()> f;
    ~SyncGuard() { (void)f(); }
  } syncg{sync_all};
  std::vector<std::unique_ptr<Fit>> fits(nprob);
  fits_ref = &fits;
  std::vector<Geom> Gs(nprob);
  for (int i = 0; i < nprob; ++i) {
    fits[i].reset(new Fit());
    Fit& F = *fits[i];
    F.arena = arena;
    F.G = Gs[i] = make_geom(probs[i].n, probs[i].p);
    F.dt = dt;
    F.s = pool.p[i % npool];
    F.own_stream = false;
    F.batched = true;
    F.enet = opt->alpha;
  }
  {
    int r = for_each_problem([&](int i) { return fit_setup_enqueue(*fits[i], &probs[i], false, false); });
    if (r) return r;
    if (sync_all() != hipSuccess) return fit_fail(GLAM_EDEVICE, "set-up failed");
    r = for_each_problem([&](int i) { return fit_setup_finish(*fits[i]); });
    if (r) return r;
  }
  // batch bookkeeping
  std::vector<int> nfwd(nprob), nadj(nprob), off_adj(nprob + 1, 0);
  std::vector<BatchDesc> desc(nprob);
  for (int i = 0; i < nprob; ++i) {
    const Geom& G = Gs[i];
    const int fgx = (G.P12 + 31) / 32, fgy = (G.n3 + 31) / 32;
    const int agx = (G.P12 + 15) / 16, agy = (G.p3 + 15) / 16;
    nfwd[i] = fgx * fgy;
    nadj[i] = agx * agy;
    off_adj[i + 1] = off_adj[i] + nadj[i];
    desc[i].fwd_gx = fgx;
    desc[i].adj_gx = agx;
  }
  void* dmem = nullptr;
  const size_t nparts = (size_t)off_adj[nprob] * ADJ_NSUM;
  // act, aoff_fwd, aoff_run, aoff_adj, then the BatchWork header
  const size_t nwork_lists = (size_t)4 * (nprob + 1);
  const size_t nwork = nwork_lists + (sizeof(BatchWork) + sizeof(int) - 1) / sizeof(int);
  auto r256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t piece[6] = {sizeof(BatchDesc) * nprob, sizeof(int) * (nprob + 1), sizeof(int) * nwork,
                           sizeof(double) * nparts, sizeof(double) * 2 * nprob, 64};
  size_t bytes = 0;
  for (size_t b : piece) bytes += r256(b);
  if (hipMalloc(&dmem, bytes) != hipSuccess) return fit_fail(GLAM_ENOMEM, "device allocation failed");
  struct MemGuard { void* p; ~MemGuard() { if (p) (void)hipFree(p); } } mg{dmem};
  char* q = (char*)dmem;
  auto take = [&](size_t b) { char* r = q; q += r256(b); return (void*)r; };   // same order as piece[]
  BatchDesc* d_desc = (BatchDesc*)take(sizeof(BatchDesc) * nprob);
  int* d_off_adj = (int*)take(sizeof(int) * (nprob + 1));
  int* d_work = (int*)take(sizeof(int) * nwork);
  double* d_part = (double*)take(sizeof(double) * nparts);
  double* d_seg = (double*)take(sizeof(double) * 2 * nprob);
  int* d_misc = (int*)take(64);   // [0] step counter of the batched inner loop
  double* h_seg_dev = nullptr;   // per-problem check maxima, written by the device into mapped host memory
  double* h_seg = (double*)arena->host_alloc(sizeof(double) * 2 * nprob, (void**)&h_seg_dev);
  int* h_work = (int*)arena->host_alloc(sizeof(int) * nwork, nullptr);
  if (!h_seg || !h_seg_dev || !h_work) return fit_fail(GLAM_ENOMEM, "pinned host allocation failed");
  std::vector<int> h_active(nprob, 0);
  for (int i = 0; i < nprob; ++i) {
    Fit& F = *fits[i];
    const Geom& G = Gs[i];
    BatchDesc& D = desc[i];
    D.fw = FwdParams{};
    D.fw.G = G; D.fw.theta = F.inc; D.fw.X3f = F.X3fc; D.fw.T1 = F.T1c; D.fw.iter = nullptr;
    D.sp = SlabParams{};
    D.sp.G = G; D.sp.img = F.imgc; D.sp.T1 = F.T1c; D.sp.S2 = F.S2c; D.sp.v_int = F.v_int;
    D.ap = AdjParams{};
    D.ap.G = G; D.ap.S2 = F.S2c; D.ap.X3a = F.X3ac; D.ap.scale = 1.0 / (double)G.n; D.ap.pen_w = probs[i].pen_w;
    D.ap.alpha = opt->alpha;
    D.ap.partials = d_part; D.ap.gref = F.gref; D.ap.theta_ref = F.theta; D.ap.x = F.x; D.ap.xp = F.xp;
    D.ap.gp = F.gp; D.ap.inc = F.inc; D.ap.iter = d_misc; D.ap.dparams = F.dparams;
  }
#define BCHK(expr)                                                                                 \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) return fit_fail(GLAM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
  BCHK(hipMemcpyAsync(d_desc, desc.data(), sizeof(BatchDesc) * nprob, hipMemcpyHostToDevice, s));
  BCHK(hipMemcpyAsync(d_off_adj, off_adj.data(), sizeof(int) * (nprob + 1), hipMemcpyHostToDevice, s));
  BCHK(launch_zero(d_misc, 64, s));
  BCHK(hipStreamSynchronize(s));   // host vectors above must outlive the copies
  BatchParams B{};
  B.desc = d_desc; B.nprob = nprob; B.off_adj = d_off_adj; B.step = d_misc;
  B.work = (const BatchWork*)(d_work + nwork_lists);
  B.act = d_work;
  B.aoff_fwd = d_work + (nprob + 1);
  B.aoff_run = d_work + 2 * (nprob + 1);
  B.aoff_adj = d_work + 3 * (nprob + 1);
  B.wave = batched_wave(dt, Gs.data(), nprob);
  if (B.wave) {
    for (int i = 0; i < nprob; ++i) desc[i].ap.s2_kb4 = 1;
    BCHK(hipMemcpyAsync(d_desc, desc.data(), sizeof(BatchDesc) * nprob, hipMemcpyHostToDevice, s));
    BCHK(hipStreamSynchronize(s));
  }
  const size_t lds = batched_lds_bytes(dt, Gs.data(), nprob);
  int tot[3] = {0, 0, 0};
  int cls_runs[4] = {0, 0, 0, 0};
  // slab-phase launch choices per shape class: the run length (0: the heuristic below) and
  // whether the class runs on the wider kernel (set by the tuner, or left at the defaults)
  int tuned_run[4] = {0, 0, 0, 0}, tuned_wide[4] = {0, 0, 0, 0};
  // Compact work lists of the active problems, uploaded from pinned memory (the host rewrites
  // it only after a stream synchronisation, so the previous upload has completed).  Runs of
  // several slabs share one load of the factor operands; by default they are as long as still
  // leaves about 2048 runs (8 at most), so that a nearly finished batch keeps the CUs busy.
  auto upload_work = [&]() -> hipError_t {
    int* act = h_work;
    int* afwd = h_work + (nprob + 1);
    int* arun = h_work + 2 * (nprob + 1);
    int* aadj = h_work + 3 * (nprob + 1);
    BatchWork* hw = (BatchWork*)(h_work + nwork_lists);
    long long slabs = 0;
    for (int i = 0; i < nprob; ++i)
      if (h_active[i]) slabs += Gs[i].n3;
    const int run0 = B.wave ? (int)std::max(1LL, std::min(8LL, slabs / 2048)) : 1;
    int k = 0;
    afwd[0] = arun[0] = aadj[0] = 0;
    // grouped by the register kernel's shape class (one slab-phase launch per class)
    for (int c = 0; c < 4; ++c) {
      const int run = B.wave && tuned_run[c] > 0 ? tuned_run[c] : run0;
      hw->run[c] = run;
      hw->cls_k[c] = k;
      for (int i = 0; i < nprob; ++i) {
        if (!h_active[i]) continue;
        const int ci = B.wave ? (Gs[i].PT == 1 ? 1 : 0) + (Gs[i].N1T <= 4 ? 2 : 0) : 0;
        if (ci != c) continue;
        act[k] = i;
        afwd[k + 1] = afwd[k] + nfwd[i];
        arun[k + 1] = arun[k] + (Gs[i].n3 + run - 1) / run;
        aadj[k + 1] = aadj[k] + nadj[i];
        ++k;
      }
      cls_runs[c] = arun[k] - arun[hw->cls_k[c]];
    }
    hw->cls_k[4] = k;
    hw->nact = k;
    tot[0] = afwd[k];
    tot[1] = arun[k];
    tot[2] = aadj[k];
    return hipMemcpyAsync(d_work, h_work, sizeof(int) * nwork, hipMemcpyHostToDevice, s);
  };
  // A block of check_every batched steps and the per-problem check maxima (into mapped host
  // memory) is replayed as one captured HIP graph.  The kernels read the work list from device
  // memory, so the graph stays valid while problems drop out; it is captured again when a grid
  // would grow (a class the list holds has no launch in it, or more runs than workgroups) or
  // could shrink to a quarter or less (the grid-stride kernels' idle workgroups exit at once,
  // and every capture costs a few hundred microseconds).
  hipGraph_t bgraph = nullptr;
  hipGraphExec_t bexec = nullptr;
  struct BGraphGuard {
    hipGraph_t* g; hipGraphExec_t* e;
    ~BGraphGuard() { if (*e) (void)hipGraphExecDestroy(*e); if (*g) (void)hipGraphDestroy(*g); }
  } bgg{&bgraph, &bexec};
  BatchGrid bgrid{};
  int bgraph_m = 0;
  long long graph_replays = 0;
  int graph_captures = 0;
  auto block_grid = [&]() {
    BatchGrid g = batched_grid(tot, cls_runs);
    for (int c = 0; c < 4; ++c) g.wide[c] = tuned_wide[c];
    return g;
  };
  auto graph_fits = [&](const BatchGrid& want, int m) {
    if (!bexec || bgraph_m != m) return false;
    for (int c = 0; c < 4; ++c) {
      if (want.cls[c] > bgrid.cls[c]) return false;   // a class without a launch, or more runs
      if (want.cls[c] > 0 && 4 * want.cls[c] <= bgrid.cls[c]) return false;
      if (want.wide[c] != bgrid.wide[c]) return false;
    }
    if (want.fwd > bgrid.fwd || want.adj > bgrid.adj || want.slab > bgrid.slab) return false;
    return !(4 * want.fwd <= bgrid.fwd || 4 * want.adj <= bgrid.adj || 4 * want.slab <= bgrid.slab);
  };
  auto run_block = [&](int m, bool use_graph) -> int {
    const BatchGrid want = block_grid();
    if (!use_graph) {
      for (int qq = 0; qq < m; ++qq) BCHK(launch_batched_step(dt, B, want, lds, s));
      BCHK(launch_segment_max(d_part, d_off_adj, nprob, h_seg_dev, s));
      return GLAM_OK;
    }
    if (!graph_fits(want, m)) {
      if (bexec) { (void)hipGraphExecDestroy(bexec); bexec = nullptr; }
      if (bgraph) { (void)hipGraphDestroy(bgraph); bgraph = nullptr; }
      BCHK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
      hipError_t e = hipSuccess;
      for (int qq = 0; qq < m && e == hipSuccess; ++qq) e = launch_batched_step(dt, B, want, lds, s);
      if (e == hipSuccess) e = launch_segment_max(d_part, d_off_adj, nprob, h_seg_dev, s);
      hipGraph_t g = nullptr;
      const hipError_t e2 = hipStreamEndCapture(s, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fit_fail(GLAM_EDEVICE, std::string("batched step capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
      }
      bgraph = g;
      BCHK(hipGraphInstantiate(&bexec, bgraph, nullptr, nullptr, 0));
      ++graph_captures;
      bgrid = want;
      bgraph_m = m;
    }
    BCHK(hipGraphLaunch(bexec, s));
    ++graph_replays;
    return GLAM_OK;
  };

  // lambda_max_i and lambda_i (every problem's step 2 at theta = 0 before one synchronisation)
  std::vector<double> lam(nprob), lmax(nprob), scale(nprob);
  {
    const int r = for_each_problem([&](int i) -> int {
      Fit& F = *fits[i];
      if (launch_fill(F.theta, Gs[i].p, 0.0, F.s) != hipSuccess) { F.err = "fill kernel failed"; return GLAM_EDEVICE; }
      return family_enqueue(F, F.theta, 0.0);
    });
    if (r) return r;
  }
  BCHK(sync_all());
  for (int i = 0; i < nprob; ++i) {
    StepStats st0;
    family_collect(*fits[i], &st0);
    lmax[i] = st0.lmax_raw;
    scale[i] = lmax[i] > 0.0 ? lmax[i] : 1.0;
    lam[i] = opt->lambda ? opt->lambda[i] : opt->lambda_ratio * lmax[i];
    res->lambda_out[i] = lam[i];
    res->lambda_max[i] = lmax[i];
    res->status[i] = GLAM_ENOCONV;
    res->iters_outer[i] = 0;
    res->kkt[i] = INFINITY;
    res->objective[i] = NAN;
  }
  // ---- the tuner: the slab-phase variants of each shape class timed on the batch itself ----
  auto now_seconds = []() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
  };
  bool tune_pending = opt->tuning == 0 && B.wave;
  double tune_seconds = 0.0;
  auto tune_classes = [&](bool* timed) -> int {
    *timed = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      if (e0) (void)hipEventDestroy(e0);
      return fit_fail(GLAM_EDEVICE, "hipEventCreate failed");
    }
    struct EvPair { hipEvent_t a, b; ~EvPair() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } evp{e0, e1};
    for (int c = 0; c < 4; ++c) {
      if (cls_runs[c] == 0) continue;
      int np = 0;
      long long slabs = 0;
      for (int i = 0; i < nprob; ++i)
        if (h_active[i] && (Gs[i].PT == 1 ? 1 : 0) + (Gs[i].N1T <= 4 ? 2 : 0) == c) { ++np; slabs += Gs[i].n3; }
      const std::string key = tune_key(dt, c, np, slabs);
      int run = 0, wide = 0;
      if (tune_lookup(key, &run, &wide)) {
        tuned_run[c] = run;
        tuned_wide[c] = wide;
        continue;
      }
      double best_us = INFINITY;
      int brun = 1, bwide = 0;
      *timed = true;
      for (int w = 0; w < (c == 0 ? 1 : 2); ++w) {
        for (int rl : {1, 2, 4, 8}) {
          tuned_run[c] = rl;
          tuned_wide[c] = w;
          BCHK(upload_work());
          const int grid = batched_grid(tot, cls_runs).cls[c];
          BCHK(launch_batched_class(dt, B, c, w, grid, s));   // warm
          BCHK(hipEventRecord(e0, s));
          constexpr int kReps = 3;
          for (int q = 0; q < kReps; ++q) BCHK(launch_batched_class(dt, B, c, w, grid, s));
          BCHK(hipEventRecord(e1, s));
          BCHK(hipEventSynchronize(e1));
          float ms = 0.f;
          BCHK(hipEventElapsedTime(&ms, e0, e1));
          const double us = ms * 1e3 / kReps;
          if (us < best_us) { best_us = us; brun = rl; bwide = w; }
        }
      }
      tuned_run[c] = brun;
      tuned_wide[c] = bwide;
      tune_store(key, brun, bwide);
    }
    return GLAM_OK;
  };

  std::vector<char> done(nprob, 0);
  std::vector<double> tol_in(nprob), best(nprob), wbest(nprob);
  std::vector<char> exact(nprob, 0);   // the model is the objective: the inner solution is the step
  const double tol = opt->kkt_tol;
  long long launches = 0, pstep = 0;
  // checked every step when a Gamma-log problem is in the batch (as in glam_fit_path)
  int check_every = opt->check_every;
  for (int i = 0; i < nprob; ++i)
    if (probs[i].family == GLAM_GAMMA) check_every = 1;
  for (int round = 0; round <= opt->max_outer; ++round) {
    int nact = 0;
    // step 2 of Algorithm 1 for every unfinished problem, one stream synchronisation
    {
      const int r = for_each_problem([&](int i) { return done[i] ? GLAM_OK : family_enqueue(*fits[i], fits[i]->theta, lam[i]); });
      if (r) return r;
    }
    BCHK(sync_all());
    for (int i = 0; i < nprob; ++i) {
      h_active[i] = 0;
      if (done[i]) continue;
      Fit& F = *fits[i];
      StepStats st;
      family_collect(F, &st);
      const double kkt = st.kkt_raw / scale[i];
      res->kkt[i] = kkt;
      res->objective[i] = st.nll + lam[i] * st.pen;
      res->iters_outer[i] = round;
      if (!std::isfinite(kkt)) { res->status[i] = GLAM_ENONFINITE; done[i] = 1; continue; }
      if (kkt <= tol) { res->status[i] = GLAM_OK; done[i] = 1; continue; }
      if (round == opt->max_outer) { done[i] = 1; continue; }
      const double wmax = family_has_weights(F.family) ? st.vmax : 1.0;
      const double Lhat = wmax * F.sprod / (double)Gs[i].n;
      if (!(Lhat > 0.0) || !std::isfinite(Lhat)) { res->status[i] = GLAM_ENONFINITE; done[i] = 1; continue; }
      const bool exact_model = F.family == GLAM_GAUSSIAN && probs[i].obs_w == nullptr;
      exact[i] = exact_model;
      tol_in[i] = exact_model ? 0.5 * tol : std::max(0.1 * tol, 0.1 * kkt);
      if (dt == DT_BF16) tol_in[i] = std::max(tol_in[i], 0.1 * kkt);
      best[i] = wbest[i] = INFINITY;
      BCHK(launch_inner_init(Gs[i], F.theta, F.gref, F.x, F.xp, F.gp, dt, F.inc, F.iter, s));
      F.hparams[0] = lam[i];
      F.hparams[1] = 1.0 / Lhat;
      BCHK(hipMemcpyAsync(F.dparams, F.hparams, 2 * sizeof(double), hipMemcpyHostToDevice, s));
      h_active[i] = 1;
      ++nact;
    }
    if (nact == 0) break;
    std::vector<char> in_round(nprob);
    for (int i = 0; i < nprob; ++i) in_round[i] = (char)h_active[i];
    BCHK(launch_zero(d_misc, 4, s));   // step counter l = 0
    BCHK(upload_work());
    int it = 0, window_start = 0;
    while (nact > 0 && it < opt->max_inner) {
      const int m = std::min(check_every, opt->max_inner - it);
      {
        const int r = run_block(m, opt->graph_mode == 0);
        if (r) return r;
      }
      launches += m;
      pstep += (long long)m * nact;
      it += m;
      BCHK(hipStreamSynchronize(s));
      if (tune_pending) {
        // the slab-phase variants of every class, timed once on this batch's own first block
        // (T1 holds that block's last values; S2 is rewritten by the next step)
        const double t0 = now_seconds();
        bool timed = false;
        const int r = tune_classes(&timed);
        if (r) return r;
        if (timed) tune_seconds += now_seconds() - t0;
        tune_pending = false;
        BCHK(upload_work());
      }
      bool changed = false;
      const bool window = it - window_start >= kStallChecks * opt->check_every;
      for (int i = 0; i < nprob; ++i) {
        if (!h_active[i]) continue;
        const double kin = h_seg[2 * i] / scale[i];
        const double noise = 4.0 * kEps[dt] * h_seg[2 * i + 1] / scale[i];
        best[i] = std::min(best[i], kin);
        bool stop = !std::isfinite(kin) || kin <= std::max(tol_in[i], noise);
        if (window && dt != DT_F64) {
          if (!(best[i] < 0.5 * wbest[i])) stop = true;
          wbest[i] = best[i];
        }
        if (stop) { h_active[i] = 0; --nact; changed = true; }
      }
      if (window) window_start = it;
      if (changed && nact > 0) BCHK(upload_work());
    }
    // step 5 of Algorithm 1 per problem: Armijo along theta~ - theta^k (theta~ = x^l of the
    // last check); the first pass of every problem is enqueued before one synchronisation
    {
      const int r = for_each_problem([&](int i) -> int {
        if (!in_round[i]) return GLAM_OK;
        Fit& F = *fits[i];
        if (exact[i]) {   // Sec. 6.5: no outer loop for the exact model (alpha = 1)
          FCHK(hipMemcpyAsync(F.theta, F.xp, Gs[i].p * 8, hipMemcpyDeviceToDevice, F.s));
          return GLAM_OK;
        }
        FCHK(launch_sub(Gs[i].p, F.xp, F.theta, F.dvec, F.s));
        return armijo_enqueue(F, 0);
      });
      if (r) return r;
    }
    BCHK(sync_all());
    {
      const int r = for_each_problem([&](int i) -> int {
        if (!in_round[i] || exact[i]) return GLAM_OK;
        Fit& F = *fits[i];
        double alpha = 0.0, Delta = 0.0;
        if (!armijo_decide(F, 0, lam[i], 0.1, &alpha, &Delta)) {
          const int r2 = armijo_finish(F, lam[i], 0.1, true, &alpha, &Delta);
          if (r2) return r2;
        }
        if (alpha > 0.0) FCHK(launch_axpy(Gs[i].p, alpha, F.dvec, F.theta, F.s));
        return GLAM_OK;
      });
      if (r) return r;
    }
  }
  int worst = GLAM_OK;
  for (int i = 0; i < nprob; ++i) {
    if (perms[i].active) {   // back to the caller's mode order
      int qi[3];
      for (int k = 0; k < 3; ++k) qi[perms[i].q[k]] = k;
      BCHK(launch_permute3(fits[i]->theta, res->theta[i], probs[i].p, qi, fits[i]->s));
    } else {
      BCHK(hipMemcpyAsync(res->theta[i], fits[i]->theta, Gs[i].p * 8, hipMemcpyDeviceToDevice, fits[i]->s));
    }
    if (res->status[i] != GLAM_OK && worst == GLAM_OK) worst = res->status[i];
  }
  BCHK(sync_all());
  BCHK(hipEventRecord(ev, s));
  BCHK(hipStreamWaitEvent(us, ev, 0));
  res->steps = launches;
  res->problem_steps = pstep;
  res->graph_replays = graph_replays;
  if (getenv("GLAM_LOG")) fprintf(stderr, "[glam] batched: %d graph captures, %lld replays\n", graph_captures, graph_replays);
  res->tune_seconds = tune_seconds;
  res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  if (worst != GLAM_OK) return fit_fail(worst, "some problems did not converge (see status)");
  return GLAM_OK;
}

namespace glam {
void set_last_error(const std::string& msg);   // api.cpp
}
static int fit_fail(int code, const std::string& msg) {
  glam::set_last_error(msg);
  return code;
}
