// general.cpp -- the lambda path of Algorithm 1 (GD-PG) for models of c >= 1 tensor components
// (Sec. 2: X = [X_1 | ... | X_c], each X_r a tensor product, eq. fivenew) on the generic rho GEMMs:
//   eta = H(<X_rj>, <Theta_r>) = sum_r rho(X_r3, rho(X_r2, rho(X_r1, Theta_r)))   (eq. eighteen),
//   G(<X_rj>, U) = the tuple of rho(X_r3^T, rho(X_r2^T, rho(X_r1^T, U)))          (eq. nineteen),
//   Lhat = max(w)/n sum_r prod_j rho(X_rj^T X_rj)                                   (Proposition 1),
// theta the concatenation of vec(Theta_r).  It is also the solver of single-component models
// whose modes fit no order of the slab kernels (p_j > n_j designs of Sec. 6.5).
//
// The outer loop keeps the structure of the slab-kernel path: FP64 anchors (eta, the score, the
// FP64 gradient and its KKT residual, the Armijo sums), an inner PG loop on the increment
// x - theta^k in the chain dtype, grad h(x) = g^k + G(V .* H(x - theta^k)) / n, with FISTA
// extrapolation (restarted or plain), backtracking for nu < 1, precision escalation and the
// MSA steps of SCAD.  Every product is a launch of the generic GEMM; the host drives the loop
// with plain stream launches and reads the convergence checks back every check_every iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "general.h"
#include "glam.h"
#include "launch.h"

namespace glam {

namespace {

const double kEpsG[3] = {1.1102230246251565e-16, 5.960464477539063e-08, 3.90625e-03};
constexpr int kStallChecksG = 10;        // as the slab-kernel path: exact model
constexpr int kStallChecksLsG = 20;      // with the Armijo rule

bool has_weights(int family) { return family == GLAM_POISSON || family == GLAM_BINOMIAL; }

struct Comp {
  int64_t p[3] = {1, 1, 1};
  long long pr = 0, off = 0;
  const double* X[3] = {nullptr, nullptr, nullptr};   // FP64 factors (caller's)
  void* XT64[3] = {nullptr, nullptr, nullptr};        // X_j^T in FP64
  const void* Xc[3] = {nullptr, nullptr, nullptr};    // chain dtype copies (FP64: the above)
  const void* XTc[3] = {nullptr, nullptr, nullptr};
  void* Xbuf[3] = {nullptr, nullptr, nullptr};        // storage of the low-precision copies
  void* XTbuf[3] = {nullptr, nullptr, nullptr};
  double srad = 1.0;                                  // prod_j rho(X_rj^T X_rj)
};

struct GFit {
  int dt = DT_F64, family = 0;
  int64_t n[3] = {1, 1, 1};
  long long N = 0, P = 0;
  std::vector<Comp> comp;
  hipStream_t s = nullptr, us = nullptr;
  hipEvent_t sync_ev = nullptr;
  std::vector<void*> bufs;
  double* hred = nullptr;
  std::string err;
  // FP64 state
  double *theta = nullptr, *eta = nullptr, *u = nullptr, *graw = nullptr, *gref = nullptr, *x = nullptr,
         *xp = nullptr, *gp = nullptr, *dvec = nullptr, *xd = nullptr, *ones = nullptr, *part = nullptr,
         *red = nullptr;
  double* bt[10] = {};
  const double* y = nullptr;
  const double* a = nullptr;     // obs_w, or NULL (a_i = 1)
  const double* a_arm = nullptr; // obs_w, or the ones array (the Armijo kernel reads a_i)
  const double* pen = nullptr;
  void *t1d = nullptr, *t2d = nullptr, *t1 = nullptr, *t2 = nullptr;   // GEMM intermediates
  void *etai = nullptr, *R = nullptr, *V = nullptr, *gi = nullptr, *inc = nullptr;
  float* dst[3] = {nullptr, nullptr, nullptr};   // FP32 increment state (BF16/FP32 chains, nu = 1)
  float* qst = nullptr;
  bool use_v = false;
  double enet = 0.0;
  int no_l1 = 0;

  void* alloc(size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) return nullptr;
    bufs.push_back(p);
    return p;
  }
  ~GFit() {
    if (s) (void)hipStreamSynchronize(s);
    for (void* b : bufs) (void)hipFree(b);
    if (hred) (void)hipHostFree(hred);
    if (sync_ev) (void)hipEventDestroy(sync_ev);
    if (s) (void)hipStreamDestroy(s);
  }
};

#define GCHK(expr)                                                                                 \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) {                                                                        \
      F.err = std::string(#expr) + ": " + hipGetErrorString(e_);                                   \
      return GLAM_EDEVICE;                                                                         \
    }                                                                                              \
  } while (0)

size_t acc_size(int dt) { return dt == DT_F64 ? 8 : 4; }

// the chain dtype copies of every factor (FP64: the FP64 arrays themselves)
int set_chain_dtype(GFit& F, int dt) {
  F.dt = dt;
  for (Comp& c : F.comp)
    for (int j = 0; j < 3; ++j) {
      if (dt == DT_F64) {
        c.Xc[j] = c.X[j];
        c.XTc[j] = c.XT64[j];
        continue;
      }
      const long long cnt = F.n[j] * c.p[j];
      if (!c.Xbuf[j]) {
        c.Xbuf[j] = F.alloc((size_t)cnt * 4);
        c.XTbuf[j] = F.alloc((size_t)cnt * 4);
        if (!c.Xbuf[j] || !c.XTbuf[j]) { F.err = "device allocation failed"; return GLAM_ENOMEM; }
      }
      GCHK(launch_gen_pack(dt, cnt, c.X[j], c.Xbuf[j], F.s));
      GCHK(launch_gen_transpose(dt, F.n[j], c.p[j], c.X[j], c.XTbuf[j], F.s));
      c.Xc[j] = c.Xbuf[j];
      c.XTc[j] = c.XTbuf[j];
    }
  return GLAM_OK;
}

struct Stats {
  double nll, vmax, kkt_raw, lmax_raw, pen;
};

// Step 2 of Algorithm 1 at theta (FP64): eta, the score u and the weights V, -l/n, the FP64
// gradient g = -G(U)/n (into gref) and its KKT residual, lambda_max's max |g|/w, J(theta).
int family_step(GFit& F, const double* theta, double lambda, Stats* st) {
  for (size_t r = 0; r < F.comp.size(); ++r) {
    const Comp& c = F.comp[r];
    GCHK(general_forward(DT_F64, F.n, c.p, (const void* const*)c.XT64, theta + c.off, F.t1d, F.t2d, F.eta, r > 0, F.s));
  }
  int nb = 0;
  GCHK(launch_gen_family(DT_F64, F.dt == DT_F64 ? DT_F64 : DT_F32, F.N, F.family, F.eta, F.y, F.a, F.u,
                         F.use_v ? F.V : nullptr, F.part, &nb, F.s));
  const int ops2[2] = {0, 1};
  GCHK(launch_reduce(F.part, nb, 2, ops2, 1.0 / (double)F.N, F.red, F.s));
  for (const Comp& c : F.comp)
    GCHK(general_adjoint(DT_F64, F.n, c.p, (const void* const*)c.X, F.u, F.t1d, F.t2d, F.graw + c.off, F.s));
  GCHK(launch_gen_grad_stats(F.P, F.graw, -1.0 / (double)F.N, theta, F.pen, lambda, F.enet, F.no_l1, F.gref, F.part,
                             &nb, F.s));
  const int ops3[3] = {1, 1, 0};
  GCHK(launch_reduce(F.part, nb, 3, ops3, 1.0, F.red + 2, F.s));
  GCHK(hipMemcpyAsync(F.hred, F.red, 5 * sizeof(double), hipMemcpyDeviceToHost, F.s));
  GCHK(hipStreamSynchronize(F.s));
  st->nll = F.hred[0];
  st->vmax = F.hred[1];
  st->kkt_raw = F.hred[2];
  st->lmax_raw = F.hred[3];
  st->pen = F.hred[4];
  return GLAM_OK;
}

// Step 2 at the theta of the last family step for a new lambda with the same penalty weights (the
// first outer step of the next model on the path): only the KKT residual changes; it is evaluated
// from the stored gradient by the same kernel (the same value); the rest is the last step's.
int kkt_at_lambda(GFit& F, double lambda, const Stats& last, Stats* st) {
  int nb = 0;
  GCHK(launch_gen_grad_stats(F.P, F.gref, 1.0, F.theta, F.pen, lambda, F.enet, F.no_l1, nullptr, F.part, &nb, F.s));
  const int ops3[3] = {1, 1, 0};
  GCHK(launch_reduce(F.part, nb, 3, ops3, 1.0, F.red + 2, F.s));
  GCHK(hipMemcpyAsync(F.hred + 2, F.red + 2, sizeof(double), hipMemcpyDeviceToHost, F.s));
  GCHK(hipStreamSynchronize(F.s));
  *st = last;
  st->kkt_raw = F.hred[2];
  return GLAM_OK;
}

// gi = G(V .* H(inc)) in the chain dtype (accumulation-type output); the last component's forward
// chain writes R = V .* (its product + the other components' sum) directly in the chain dtype
int inner_gradient(GFit& F) {
  const size_t es = dt_size(F.dt), as = acc_size(F.dt);
  const size_t c = F.comp.size();
  for (size_t r = 0; r + 1 < c; ++r) {
    const Comp& cr = F.comp[r];
    GCHK(general_forward(F.dt, F.n, cr.p, cr.XTc, (const char*)F.inc + cr.off * es, F.t1, F.t2, F.etai, r > 0, F.s));
  }
  const Comp& cl = F.comp[c - 1];
  GCHK(general_forward_weighted(F.dt, F.n, cl.p, cl.XTc, (const char*)F.inc + cl.off * es, F.t1, F.t2,
                                c > 1 ? F.etai : nullptr, F.use_v ? F.V : nullptr, F.R, F.s));
  for (const Comp& c : F.comp)
    GCHK(general_adjoint(F.dt, F.n, c.p, c.Xc, F.R, F.t1, F.t2, (char*)F.gi + c.off * as, F.s));
  return GLAM_OK;
}

// the increment-state inner iteration (BF16 / FP32 chains): the forward chains as in inner_gradient,
// then each component's adjoint chain with the step fused into its last product; *nb: partial rows
int inner_step(GFit& F, float* const d[3], double lam, double delta, double om, int* nb) {
  const size_t es = dt_size(F.dt);
  const size_t c = F.comp.size();
  for (size_t r = 0; r + 1 < c; ++r) {
    const Comp& cr = F.comp[r];
    GCHK(general_forward(F.dt, F.n, cr.p, cr.XTc, (const char*)F.inc + cr.off * es, F.t1, F.t2, F.etai, r > 0, F.s));
  }
  const Comp& cl = F.comp[c - 1];
  GCHK(general_forward_weighted(F.dt, F.n, cl.p, cl.XTc, (const char*)F.inc + cl.off * es, F.t1, F.t2,
                                c > 1 ? F.etai : nullptr, F.use_v ? F.V : nullptr, F.R, F.s));
  auto params = [&](const Comp& cm, int rows) {
    GenStepParams S{};
    S.scale = 1.0 / (double)F.N;
    S.gref = F.gref + cm.off;
    S.theta_ref = F.theta + cm.off;
    S.w = F.pen ? F.pen + cm.off : nullptr;
    S.dcur = d[0] + cm.off;
    S.dprev = d[1] + cm.off;
    S.q = F.qst + cm.off;
    S.dout = d[2] + cm.off;
    S.inc = (char*)F.inc + cm.off * es;
    S.lambda = lam;
    S.delta = delta;
    S.om = om;
    S.alpha = F.enet;
    S.no_l1 = F.no_l1;
    S.part = F.part + (size_t)rows * 4;
    return S;
  };
  bool any_fused = false;
  for (const Comp& cm : F.comp) any_fused = any_fused || general_step_fused(cm.p);
  if (!any_fused) {
    // every component's last product is small: the adjoint chains into gi, then one step over all
    // coefficients (one launch)
    for (const Comp& cm : F.comp)
      GCHK(general_adjoint(F.dt, F.n, cm.p, cm.Xc, F.R, F.t1, F.t2, (char*)F.gi + cm.off * acc_size(F.dt), F.s));
    Comp all;
    all.off = 0;
    GCHK(launch_gen_step(F.dt, F.P, F.gi, params(all, 0), nb, F.s));
    return GLAM_OK;
  }
  int rows = 0;
  for (const Comp& cm : F.comp) {
    const GenStepParams S = params(cm, rows);
    int r = 0;
    GCHK(general_adjoint_step(F.dt, F.n, cm.p, cm.Xc, F.R, F.t1, F.t2, (char*)F.gi + cm.off * acc_size(F.dt), S, &r,
                              F.s));
    rows += r;
  }
  *nb = rows;
  return GLAM_OK;
}

int read_red(GFit& F, int nb, int nval, const int* ops, double* out) {
  GCHK(launch_reduce(F.part, nb, nval, ops, 1.0, F.red, F.s));
  GCHK(hipMemcpyAsync(F.hred, F.red, nval * sizeof(double), hipMemcpyDeviceToHost, F.s));
  GCHK(hipStreamSynchronize(F.s));
  for (int v = 0; v < nval; ++v) out[v] = F.hred[v];
  return GLAM_OK;
}

// Inner PG loop with nu = 1 (delta = 1/Lhat fixed).  Leaves theta~ = x^l of the last checked
// iteration in F.xp.  BF16/FP32 chains keep the state as FP32 increments (the step fused into the
// last adjoint product, general_adjoint_step), FP64
// chains in FP64 (k_gen_prox).
int inner_loop(GFit& F, double lam, double delta, double tol_in, double lam_scale, int max_inner, int check_every,
               bool restart, bool exact_model, int* it_out, double* kin_out) {
  const bool incst = F.dt != DT_F64;
  float* d[3] = {F.dst[0], F.dst[1], F.dst[2]};   // d^l, d^{l-1}, the next
  if (incst) {
    GCHK(hipMemsetAsync(d[0], 0, F.P * 4, F.s));
    GCHK(hipMemsetAsync(d[1], 0, F.P * 4, F.s));
    GCHK(hipMemsetAsync(F.qst, 0, F.P * 4, F.s));
  } else {
    GCHK(hipMemcpyAsync(F.x, F.theta, F.P * 8, hipMemcpyDeviceToDevice, F.s));
    GCHK(hipMemcpyAsync(F.xp, F.theta, F.P * 8, hipMemcpyDeviceToDevice, F.s));
    GCHK(hipMemcpyAsync(F.gp, F.gref, F.P * 8, hipMemcpyDeviceToDevice, F.s));
  }
  GCHK(hipMemsetAsync(F.inc, 0, F.P * dt_size(F.dt), F.s));
  int it = 0, l = 0, window_start = 0;
  double kin = INFINITY, best = INFINITY, window_best = INFINITY;
  const int stall = (exact_model ? kStallChecksG : kStallChecksLsG) * std::max(check_every, 10);   // as the slab path's window
  while (it < max_inner) {
    ++l;
    const double om = (l - 1.0) / (l + 2.0);
    int nb = 0;
    if (incst) {
      const int r = inner_step(F, d, lam, delta, om, &nb);
      if (r) return r;
      float* t = d[1];
      d[1] = d[0];
      d[0] = d[2];
      d[2] = t;
    } else {
      const int r = inner_gradient(F);
      if (r) return r;
      GCHK(launch_gen_prox(F.dt, F.P, F.gi, 1.0 / (double)F.N, F.gref, F.theta, F.pen, F.x, F.xp, F.gp, F.inc, lam,
                           delta, om, F.enet, F.no_l1, F.part, &nb, F.s));
    }
    ++it;
    if (it % check_every != 0 && it < max_inner) continue;
    double v[4];
    const int ops[4] = {1, 1, 0, 1};
    {
      const int r = read_red(F, nb, 4, ops, v);
      if (r) return r;
    }
    kin = v[0] / lam_scale;
    const double noise = 4.0 * kEpsG[F.dt] * v[1] / lam_scale;
    if (restart && v[2] > 0.0) l = 0;   // gradient restart test: omega = 0 next
    best = std::min(best, kin);
    if (it - window_start >= stall) {
      if (!(best < 0.5 * window_best) && F.dt != DT_F64) break;
      window_best = best;
      window_start = it;
    }
    if (!std::isfinite(kin)) break;
    if (kin <= std::max(tol_in, noise)) break;
  }
  if (incst) GCHK(launch_gen_inc_out(F.P, d[1], F.theta, 0, F.xp, F.s));   // theta~ = x^l
  *it_out = it;
  *kin_out = kin;
  return GLAM_OK;
}

// Inner PG loop with nu < 1: delta starts at delta0 and is halved (never below 1/Lhat) whenever
// the sufficient-decrease test of the step into the current iterate fails; that step is then
// redone from its starting point.  Checked every iteration.  theta~ ends in F.xp.
int inner_loop_bt(GFit& F, double lam, double delta0, double Lhat, double tol_in, double lam_scale, int max_inner,
                  int* it_out, double* kin_out) {
  const size_t pb = F.P * 8;
  GenBtState cur{F.bt[0], F.bt[1], F.bt[2], F.bt[3], F.bt[4]};
  GenBtState nxt{F.bt[5], F.bt[6], F.bt[7], F.bt[8], F.bt[9]};
  GCHK(hipMemcpyAsync(cur.x, F.theta, pb, hipMemcpyDeviceToDevice, F.s));
  GCHK(hipMemcpyAsync(cur.xp, F.theta, pb, hipMemcpyDeviceToDevice, F.s));
  GCHK(hipMemcpyAsync(cur.y, F.theta, pb, hipMemcpyDeviceToDevice, F.s));
  GCHK(hipMemcpyAsync(cur.gp, F.gref, pb, hipMemcpyDeviceToDevice, F.s));
  GCHK(hipMemcpyAsync(cur.gy, F.gref, pb, hipMemcpyDeviceToDevice, F.s));
  GCHK(hipMemsetAsync(F.inc, 0, F.P * dt_size(F.dt), F.s));
  double delta = delta0;
  const double delta_min = 1.0 / Lhat;
  int l = 1, it = 0, window_start = 0;
  double kin = INFINITY, best = INFINITY, window_best = INFINITY;
  while (it < max_inner) {
    int r = inner_gradient(F);
    if (r) return r;
    const double om = (l - 1.0) / (l + 2.0);
    int nb = 0;
    GCHK(launch_gen_prox_bt(F.dt, F.P, F.gi, 1.0 / (double)F.N, F.gref, F.theta, F.pen, cur, nxt, F.inc, lam, delta, om,
                            F.enet, F.no_l1, F.part, &nb, F.s));
    double v[4];
    const int ops[4] = {1, 1, 0, 0};
    r = read_red(F, nb, 4, ops, v);
    if (r) return r;
    ++it;
    if (l >= 2 && v[2] > (v[3] / delta) * (1.0 + 1e-12) && delta > delta_min * (1.0 + 1e-12)) {
      delta = std::max(0.5 * delta, delta_min);
      GCHK(launch_gen_bt_redo(F.dt, F.P, cur.y, cur.gy, F.pen, F.theta, lam, delta, F.enet, F.no_l1, cur.x, F.inc, F.s));
      continue;
    }
    kin = v[0] / lam_scale;
    std::swap(cur, nxt);
    ++l;
    if (!std::isfinite(kin)) break;
    const double noise = 4.0 * kEpsG[F.dt] * v[1] / lam_scale;
    if (kin <= std::max(tol_in, noise)) break;
    best = std::min(best, kin);
    if (it - window_start >= 200) {
      if (!(best < 0.5 * window_best) && F.dt != DT_F64) break;
      window_best = best;
      window_start = it;
    }
  }
  // the accepted x^l is the current state's x^{l-1}
  GCHK(hipMemcpyAsync(F.xp, cur.xp, pb, hipMemcpyDeviceToDevice, F.s));
  *it_out = it;
  *kin_out = kin;
  return GLAM_OK;
}

// Armijo rule (Sec. 5) along d = F.dvec from theta: H(d) in FP64, then passes of 16 trial steps
// 2^-j0 .. 2^-(j0+15) on FP64 sums of the changes of -l/n and J.  alpha = 0 when Delta >= 0 or
// no trial down to 2^-63 is accepted.
int armijo(GFit& F, double lam, double v, double* alpha_out, double* Delta_out) {
  for (size_t r = 0; r < F.comp.size(); ++r) {
    const Comp& c = F.comp[r];
    GCHK(general_forward(DT_F64, F.n, c.p, (const void* const*)c.XT64, F.dvec + c.off, F.t1d, F.t2d, F.xd, r > 0, F.s));
  }
  constexpr int NV = ARMIJO_TRIALS + 1;
  const int ops[NV] = {0};
  Geom G{};
  G.nint = F.N;
  G.n = F.N;
  G.p = F.P;
  double Delta = 0.0;
  for (int j0 = 0; j0 < 64; j0 += ARMIJO_TRIALS) {
    int nb1 = 0, nb2 = 0;
    GCHK(launch_armijo(G, F.family, F.eta, F.xd, F.y, F.a_arm, j0, F.part, &nb1, F.s));
    GCHK(launch_reduce(F.part, nb1, NV, ops, 1.0 / (double)F.N, F.red, F.s));
    double* part2 = F.part + (size_t)nb1 * NV;
    GCHK(launch_pen_trials(F.P, F.theta, F.dvec, F.pen, F.enet, F.no_l1, j0, part2, &nb2, F.s));
    GCHK(launch_reduce(part2, nb2, NV, ops, 1.0, F.red + NV, F.s));
    GCHK(hipMemcpyAsync(F.hred, F.red, 2 * NV * sizeof(double), hipMemcpyDeviceToHost, F.s));
    GCHK(hipStreamSynchronize(F.s));
    const double* sm = F.hred;
    const double* pj = F.hred + NV;
    if (j0 == 0) {
      Delta = -sm[0] + lam * pj[0];
      *Delta_out = Delta;
      // the rule presumes a descent direction (Sec. 5, Theorem 2's search direction)
      if (!(Delta < 0.0)) {
        *alpha_out = 0.0;
        return GLAM_OK;
      }
    }
    for (int j = 0; j < ARMIJO_TRIALS; ++j) {
      const double t = std::ldexp(1.0, -(j0 + j));
      const double dF = sm[1 + j] + lam * pj[1 + j];
      if (std::isfinite(dF) && dF <= t * v * Delta) {
        *alpha_out = t;
        return GLAM_OK;
      }
    }
  }
  *alpha_out = 0.0;
  return GLAM_OK;
}

int setup(GFit& F, const GenProblem& prob, int dtype, bool bt) {
  F.family = prob.family;
  for (int j = 0; j < 3; ++j) F.n[j] = prob.n[j];
  F.N = F.n[0] * F.n[1] * F.n[2];
  F.comp.resize(prob.comps.size());
  long long off = 0, tmp = 1;
  for (size_t r = 0; r < prob.comps.size(); ++r) {
    Comp& c = F.comp[r];
    for (int j = 0; j < 3; ++j) {
      c.p[j] = prob.comps[r].p[j];
      c.X[j] = prob.comps[r].X[j];
    }
    c.pr = c.p[0] * c.p[1] * c.p[2];
    c.off = off;
    off += c.pr;
    tmp = std::max(tmp, general_tmp_elems(F.n, c.p));
  }
  F.P = off;
  F.y = prob.Y;
  F.a = prob.obs_w;
  bool ok = true;
  auto A = [&](size_t b) { void* p = F.alloc(b); if (!p) ok = false; return p; };
  const size_t nb8 = (size_t)F.N * 8, pb8 = (size_t)F.P * 8;
  size_t step_rows = 0;   // partial rows of the fused increment-state step (all components)
  for (const GenComponent& gc : prob.comps) step_rows += (size_t)general_step_rows(gc.p);
  const size_t npart = std::max<size_t>({(size_t)kGenMaxBlocks * 4, step_rows * 4,
                                         (size_t)(kArmijoMaxBlocks + kPenTrialsMaxBlocks) * (ARMIJO_TRIALS + 1)});
  F.theta = (double*)A(pb8);
  F.eta = (double*)A(nb8);
  F.u = (double*)A(nb8);
  F.xd = (double*)A(nb8);
  F.graw = (double*)A(pb8);
  F.gref = (double*)A(pb8);
  F.x = (double*)A(pb8);
  F.xp = (double*)A(pb8);
  F.gp = (double*)A(pb8);
  F.dvec = (double*)A(pb8);
  F.part = (double*)A(npart * 8);
  F.red = (double*)A(64 * 8);
  // chain buffers get 8-byte elements whatever the dtype, so an escalation reuses them
  F.t1d = A((size_t)tmp * 8);
  F.t2d = A((size_t)tmp * 8);
  F.t1 = A((size_t)tmp * 8);
  F.t2 = A((size_t)tmp * 8);
  F.etai = A(nb8);
  F.R = A(nb8);
  F.gi = A(pb8);
  F.inc = A(pb8);
  F.use_v = has_weights(F.family);
  if (F.use_v) F.V = A(nb8);
  if (bt)
    for (double*& b : F.bt) b = (double*)A(pb8);
  else
    for (int q = 0; q < 4; ++q) (q < 3 ? F.dst[q] : F.qst) = (float*)A((size_t)F.P * 4);
  if (!F.a) F.ones = (double*)A(nb8);
  if (!ok) { F.err = "device allocation failed"; return GLAM_ENOMEM; }
  if (hipHostMalloc((void**)&F.hred, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    F.hred = nullptr;
    F.err = "pinned host allocation failed";
    return GLAM_ENOMEM;
  }
  if (!F.a) GCHK(launch_fill(F.ones, F.N, 1.0, F.s));
  F.a_arm = F.a ? F.a : F.ones;
  // input checks
  {
    int nb = 0;
    GCHK(launch_check(F.N, prob.Y, prob.obs_w, F.P, prob.pen_w, prob.family, F.part, &nb, F.s));
    const int ops[4] = {1, 1, 1, 1};
    double v[4];
    int r = read_red(F, nb, 4, ops, v);
    if (r) return r;
    if (v[0] != 0.0) { F.err = "Y has non-finite entries"; return GLAM_EINVAL; }
    if (v[1] != 0.0) {
      F.err = prob.family == GLAM_POISSON    ? "Poisson Y must be >= 0"
              : prob.family == GLAM_BINOMIAL ? "Binomial Y must be a proportion in [0, 1]"
                                             : "Gamma Y must be > 0";
      return GLAM_EINVAL;
    }
    if (v[2] != 0.0) { F.err = "obs_w must be finite and >= 0"; return GLAM_EINVAL; }
    if (v[3] != 0.0) { F.err = "pen_w must be finite and > 0"; return GLAM_EINVAL; }
  }
  // X_j^T in FP64 for the forward products, the chain copies, Proposition 1's radii
  for (Comp& c : F.comp)
    for (int j = 0; j < 3; ++j) {
      c.XT64[j] = A((size_t)F.n[j] * c.p[j] * 8);
      if (!ok) { F.err = "device allocation failed"; return GLAM_ENOMEM; }
      GCHK(launch_gen_transpose(DT_F64, F.n[j], c.p[j], c.X[j], c.XT64[j], F.s));
    }
  int r = set_chain_dtype(F, dtype);
  if (r) return r;
  for (Comp& c : F.comp) {
    c.srad = 1.0;
    for (int j = 0; j < 3; ++j) {
      std::vector<double> h((size_t)F.n[j] * c.p[j]);
      GCHK(hipMemcpyAsync(h.data(), c.X[j], h.size() * 8, hipMemcpyDeviceToHost, F.s));
      GCHK(hipStreamSynchronize(F.s));
      c.srad *= gram_spectral_radius(gram_matrix(h.data(), (int)F.n[j], (int)c.p[j]), (int)c.p[j]);
    }
  }
  return GLAM_OK;
}

}  // namespace

int general_fit_path(const GenProblem& prob, const glam_options* opt, glam_result* res, std::string* why) {
  GFit F;
  F.us = (hipStream_t)opt->stream;
  if (hipStreamCreateWithFlags(&F.s, hipStreamNonBlocking) != hipSuccess) {
    *why = "hipStreamCreateWithFlags failed";
    return GLAM_EDEVICE;
  }
  if (hipEventCreateWithFlags(&F.sync_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(F.sync_ev, F.us) != hipSuccess || hipStreamWaitEvent(F.s, F.sync_ev, 0) != hipSuccess) {
    *why = "stream ordering failed";
    return GLAM_EDEVICE;
  }
  const bool bt = opt->nu < 1.0;
  F.pen = prob.pen_w;
  if (opt->penalty == GLAM_PENALTY_RIDGE) {   // Sec. 6.3: J = sum_m w_m theta_m^2
    F.enet = 1.0;
    F.no_l1 = 1;
  } else {
    F.enet = opt->alpha;
  }
  auto fail = [&](int code) {
    *why = F.err;
    return code;
  };
  {
    const int r = setup(F, prob, opt->dtype, bt);
    if (r) return fail(r);
  }
  if (opt->inner_mode == GLAM_INNER_ONE) F.use_v = false;   // unit IRLS weights in the model
#define RG(expr)                      \
  do {                                \
    const int r_ = (expr);            \
    if (r_ != GLAM_OK) return fail(r_); \
  } while (0)
#define PG(expr)                                                                       \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      F.err = std::string(#expr) + ": " + hipGetErrorString(e_);                       \
      return fail(GLAM_EDEVICE);                                                       \
    }                                                                                  \
  } while (0)

  const long long P = F.P;
  const bool scad = opt->penalty == GLAM_PENALTY_SCAD;
  const int msa_steps = scad ? opt->msa_steps : 1;
  const double scad_a = opt->scad_a == 0.0 ? 3.7 : opt->scad_a;
  double* pen_buf = nullptr;
  if (scad) {
    pen_buf = (double*)F.alloc(P * 8);
    if (!pen_buf) { F.err = "device allocation failed"; return fail(GLAM_ENOMEM); }
    F.pen = pen_buf;
  }
  auto base_weights = [&]() -> hipError_t {
    return prob.pen_w ? hipMemcpyAsync(pen_buf, prob.pen_w, P * 8, hipMemcpyDeviceToDevice, F.s)
                      : launch_fill(pen_buf, P, 1.0, F.s);
  };
  if (scad) PG(base_weights());

  // lambda_max: the zero solution's gradient (Sec. 6.4)
  PG(launch_fill(F.theta, P, 0.0, F.s));
  Stats st0{};
  RG(family_step(F, F.theta, 0.0, &st0));
  const double lam_max = st0.lmax_raw;
  res->lambda_max = lam_max;
  if (!std::isfinite(lam_max)) { F.err = "non-finite lambda_max"; return fail(GLAM_ENONFINITE); }
  const double lam_scale = lam_max > 0.0 ? lam_max : 1.0;
  std::vector<double> lams(opt->nlambda);
  for (int l = 0; l < opt->nlambda; ++l) {
    if (opt->lambda) lams[l] = opt->lambda[l];
    else lams[l] = opt->nlambda == 1 ? lam_max
                                     : lam_max * std::pow(opt->lambda_min_ratio, (double)l / (opt->nlambda - 1));
  }
  if (opt->theta0) PG(hipMemcpyAsync(F.theta, opt->theta0, P * 8, hipMemcpyDeviceToDevice, F.s));

  double srad_sum = 0.0;
  for (const Comp& c : F.comp) srad_sum += c.srad;
  const bool exact_model = F.family == GLAM_GAUSSIAN && prob.obs_w == nullptr;
  const double tol = opt->kkt_tol;
  const bool unit_w = opt->inner_mode == GLAM_INNER_ONE && has_weights(F.family);
  const int check_every = (F.family == GLAM_GAMMA || unit_w) ? 1 : opt->check_every;
  const bool restart = opt->extrapolation == 0;
  const bool verbose = getenv("GLAM_LOG") && atoi(getenv("GLAM_LOG")) > 0;
  int path_status = GLAM_OK;
  long long path_inner = 0;
  res->n_done = 0;
  res->escalated_at = -1;
  res->chain_ms = res->adj_ms = res->fwd_ms = res->iter_ms = 0.0;
  res->chain_samples = 0;
  res->inner_total = 0;

  Stats st_last{};   // the last family step's values (theta unchanged since)
  for (int l = 0; l < opt->nlambda; ++l) {
    const double lam = lams[l];
    res->lambda_out[l] = lam;
    int status = GLAM_ENOCONV, outer = 0, outer_base = 0;
    long long inner_total = 0;
    double kkt = INFINITY, Fobj = NAN, kkt_prev = INFINITY;
    int lowprec_stalls = 0;
    bool last_limited = false;
    for (int step = 0; step < msa_steps; ++step) {
      if (scad) {
        if (step == 0) PG(base_weights());
        else PG(launch_scad_weights(P, F.theta, prob.pen_w, lam, scad_a, pen_buf, F.s));
      }
      status = GLAM_ENOCONV;
      for (int k = 0; k <= opt->max_outer; ++k) {
        Stats st{};
        if (k == 0 && l > 0 && !scad) RG(kkt_at_lambda(F, lam, st_last, &st));
        else RG(family_step(F, F.theta, lam, &st));
        st_last = st;
        kkt = st.kkt_raw / lam_scale;
        Fobj = st.nll + lam * st.pen;
        outer = outer_base + k;
        if (!std::isfinite(kkt) || !std::isfinite(Fobj)) { status = GLAM_ENONFINITE; break; }
        if (kkt <= tol) { status = GLAM_OK; break; }
        if (k == opt->max_outer) break;
        if (F.dt != DT_F64) {
          // precision escalation, as in the slab-kernel path
          lowprec_stalls = (k > 0 && last_limited && kkt > 0.9 * kkt_prev) ? lowprec_stalls + 1 : 0;
          if (lowprec_stalls >= 3) {
            RG(set_chain_dtype(F, F.dt == DT_BF16 ? DT_F32 : DT_F64));
            if (F.use_v) RG(family_step(F, F.theta, lam, &st));   // V in the new accumulation type
            lowprec_stalls = 0;
            if (res->escalated_at < 0) res->escalated_at = l;
          }
        }
        kkt_prev = kkt;
        const double wmax = F.use_v ? st.vmax : 1.0;
        const double Lhat = wmax * srad_sum / (double)F.N;   // Proposition 1, summed over components
        if (!(Lhat > 0.0) || !std::isfinite(Lhat)) { status = GLAM_ENONFINITE; break; }
        const double delta = opt->nu > 0.0 ? 1.0 / (opt->nu * Lhat) : 1.0;
        double tol_in = exact_model ? 0.5 * tol : std::max(0.1 * tol, 0.1 * kkt);
        if (F.dt == DT_BF16) tol_in = std::max(tol_in, 0.01 * kkt);
        int it = 0;
        double kin = INFINITY;
        if (bt) RG(inner_loop_bt(F, lam, delta, Lhat, tol_in, lam_scale, opt->max_inner, &it, &kin));
        else RG(inner_loop(F, lam, delta, tol_in, lam_scale, opt->max_inner, check_every, restart, exact_model, &it, &kin));
        inner_total += it;
        if (!std::isfinite(kin)) { status = GLAM_ENONFINITE; break; }
        last_limited = kin > tol_in && it < opt->max_inner;
        double alpha = 0.0, Delta = 0.0;
        if (exact_model) {
          alpha = 1.0;
          PG(hipMemcpyAsync(F.theta, F.xp, P * 8, hipMemcpyDeviceToDevice, F.s));
        } else {
          PG(launch_sub(P, F.xp, F.theta, F.dvec, F.s));
          RG(armijo(F, lam, 0.1, &alpha, &Delta));
          if (alpha > 0.0) PG(launch_axpy(P, alpha, F.dvec, F.theta, F.s));
          else if (F.dt != DT_F64) last_limited = true;
        }
        if (verbose)
          fprintf(stderr, "[glam-gen] lambda %d k %d kkt %.3e F %.12e inner %d kin %.2e alpha %g Delta %.3e\n", l, k,
                  kkt, Fobj, it, kin, alpha, Delta);
      }
      outer_base = outer;
      if (status != GLAM_OK) break;
    }
    PG(hipMemcpyAsync(res->theta + (size_t)l * P, F.theta, P * 8, hipMemcpyDeviceToDevice, F.s));
    res->kkt[l] = kkt;
    res->objective[l] = Fobj;
    res->iters_outer[l] = outer;
    res->iters_inner[l] = (int)std::min<long long>(inner_total, 2000000000LL);
    res->status[l] = status;
    path_inner += inner_total;
    if (status != GLAM_OK) {
      path_status = status;
      break;
    }
    res->n_done = l + 1;
  }
  PG(hipStreamSynchronize(F.s));
  PG(hipEventRecord(F.sync_ev, F.s));
  PG(hipStreamWaitEvent(F.us, F.sync_ev, 0));
  res->inner_total = path_inner;
  if (path_status != GLAM_OK) {
    F.err = "path stopped early (see status array)";
    return fail(path_status);
  }
  return GLAM_OK;
#undef RG
#undef PG
}

}  // namespace glam

namespace glam {
void set_last_error(const std::string& msg);   // api.cpp
}

using namespace glam;

extern "C" int glam_fit_path_multi(const glam_multi_problem* prob, const glam_options* opt, glam_result* res) {
  const auto t_start = std::chrono::steady_clock::now();
  auto fail = [](int code, const std::string& msg) {
    set_last_error(msg);
    return code;
  };
  if (!prob || !opt || !res) return fail(GLAM_EINVAL, "NULL argument");
  if (prob->d != 2 && prob->d != 3) return fail(GLAM_EINVAL, "d must be 2 or 3");
  if (prob->c < 1) return fail(GLAM_EINVAL, "c must be >= 1");
  if (!prob->p || !prob->X) return fail(GLAM_EINVAL, "NULL p or X");
  if (!prob->Y) return fail(GLAM_EINVAL, "NULL Y");
  if (prob->family < GLAM_GAUSSIAN || prob->family > GLAM_GAMMA) return fail(GLAM_EINVAL, "bad family");
  for (int j = 0; j < prob->d; ++j)
    if (prob->n[j] < 1) return fail(GLAM_EINVAL, "mode sizes must be >= 1");
  for (int r = 0; r < prob->c; ++r)
    for (int j = 0; j < prob->d; ++j) {
      if (prob->p[3 * r + j] < 1) return fail(GLAM_EINVAL, "mode sizes must be >= 1");
      if (!prob->X[3 * r + j]) return fail(GLAM_EINVAL, "NULL factor");
    }
  {
    std::string why;
    const int r = check_fit_options(opt, res, prob->family, prob->obs_w != nullptr, &why);
    if (r) return fail(r, why);
  }
  if (opt->inner_mode == GLAM_INNER_GRAM || opt->inner_mode == GLAM_INNER_KRON)
    return fail(GLAM_EINVAL, "the multi-component solver takes the rho-chain and unit-weight inner loops");
  // a d = 2 model is the d = 3 model with a 1 x 1 middle factor [1] in every component
  double* one = nullptr;
  if (prob->d == 2) {
    const double v = 1.0;
    if (hipMalloc((void**)&one, 256) != hipSuccess) return fail(GLAM_ENOMEM, "device allocation failed");
    if (hipMemcpy(one, &v, sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(one);
      return fail(GLAM_EDEVICE, "hipMemcpy failed");
    }
  }
  GenProblem gp;
  if (prob->d == 3) {
    for (int j = 0; j < 3; ++j) gp.n[j] = prob->n[j];
  } else {
    gp.n[0] = prob->n[0];
    gp.n[1] = 1;
    gp.n[2] = prob->n[1];
  }
  for (int r = 0; r < prob->c; ++r) {
    GenComponent c;
    if (prob->d == 3) {
      for (int j = 0; j < 3; ++j) {
        c.p[j] = prob->p[3 * r + j];
        c.X[j] = prob->X[3 * r + j];
      }
    } else {
      c.p[0] = prob->p[3 * r];
      c.p[1] = 1;
      c.p[2] = prob->p[3 * r + 1];
      c.X[0] = prob->X[3 * r];
      c.X[1] = one;
      c.X[2] = prob->X[3 * r + 1];
    }
    gp.comps.push_back(c);
  }
  gp.Y = prob->Y;
  gp.obs_w = prob->obs_w;
  gp.family = prob->family;
  gp.pen_w = prob->pen_w;
  std::string why;
  const int r = general_fit_path(gp, opt, res, &why);   // synchronises its stream before returning
  if (one) (void)hipFree(one);
  res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  if (r) return fail(r, why);
  return GLAM_OK;
}
